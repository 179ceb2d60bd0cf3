// On-chip data rates that bound the modular contraction (a ceiling for its stage copies and
// fragment reads, beside the matrix-core rate of mfma_rate.hip).
//
//  * l2_lds_dma:  global_load_lds_dwordx4 (64 lanes x 16 bytes per instruction) into a 96 KB LDS
//                 ring, each block re-reading its own 48 KB window, so that after the first pass
//                 every copy hits in L2 (32 blocks x 48 KB per XCD); 8 waves per block, 6 copies
//                 per wave per step, two steps in flight, a work-group barrier per step (the
//                 contraction's stage structure).
//  * l2_lds_reg:  the same traffic through registers (global_load_dwordx4, then ds_write_b128).
//  * hbm_lds_dma: the DMA copies streaming from HBM (each block its own 64 MB window).
//  * lds_read:    ds_read_b128 of 1 KB fragments, 8 per wave per step, 8 waves.
// One work-group per CU (96 KB of LDS each), 256 work-groups.  Prints one JSON line with each rate
// in TB/s over the device and in bytes per clock per CU (the clock from s_memtime against
// s_memrealtime, which counts at 100 MHz).
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kBlocks = 256, kWaves = 8, kThreads = 64 * kWaves, kLds = 98304, kPer = 6;

template <int IN_FLIGHT>
__device__ inline void wait_copies()
{
    // vmcnt (bits 3:0 and 15:14) at most IN_FLIGHT; expcnt and lgkmcnt not waited for
    __builtin_amdgcn_s_waitcnt((IN_FLIGHT & 15) | ((IN_FLIGHT >> 4) << 14) | (0x7 << 4) | (0xf << 8));
}

__device__ inline void stamp(long long *clk, int which)
{
    if (threadIdx.x == 0) {
        clk[4 * blockIdx.x + 2 * which] = __builtin_amdgcn_s_memtime();
        clk[4 * blockIdx.x + 2 * which + 1] = __builtin_amdgcn_s_memrealtime();
    }
}

// MODE 0: DMA copies; 1: through registers
template <int MODE>
__global__ __launch_bounds__(kThreads, 1) void copy_kernel(const char *src, long long win, int steps, long long *clk,
                                                           int *out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const char *base = src + (long long)blockIdx.x * win;
    long long off = (long long)wave * kPer * 1024;
    v4i ring[2][kPer];
    stamp(clk, 0);
    if (MODE == 1) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
#pragma unroll
            for (int c = 0; c < kPer; ++c)
                ring[d][c] = *reinterpret_cast<const v4i *>(base + (off + c * 1024LL) % win + lane * 16);
            off += (long long)kWaves * kPer * 1024;
        }
    }
    for (int s = 0; s < steps; s += 2) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
#pragma unroll
            for (int c = 0; c < kPer; ++c) {
                const int lo = ((((s + d) & 1) * kWaves + wave) * kPer + c) * 1024;   // < 96 KB
                const char *g = base + (off + c * 1024LL) % win + lane * 16;
                if (MODE == 0) {
                    __builtin_amdgcn_global_load_lds((const int __attribute__((address_space(1))) *)g,
                                                     (int __attribute__((address_space(3))) *)(smem + lo), 16, 0, 0);
                } else {
                    *reinterpret_cast<v4i *>(smem + lo + lane * 16) = ring[d][c];
                    ring[d][c] = *reinterpret_cast<const v4i *>(g);
                }
            }
            off += (long long)kWaves * kPer * 1024;
            if (MODE == 0) wait_copies<kPer>();
            __syncthreads();
        }
    }
    if (MODE == 0) wait_copies<0>();
    stamp(clk, 1);
    int x = 0;
    if (MODE == 1)
        for (int d = 0; d < 2; ++d)
            for (int c = 0; c < kPer; ++c) x += ring[d][c][0];
    __syncthreads();
    out[blockIdx.x * kThreads + tid] = smem[tid] + x;
}

__global__ __launch_bounds__(kThreads, 1) void lds_read_kernel(int steps, long long *clk, int *out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < kLds / 4; i += kThreads) reinterpret_cast<int *>(smem)[i] = i * 2654435761u;
    __syncthreads();
    stamp(clk, 0);
    int x = 0;
    for (int s = 0; s < steps; ++s) {
        const int b = ((s * 8 + (tid >> 6) * 3) & 63) * 1024;
        v4i f[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) f[i] = *reinterpret_cast<const v4i *>(smem + (b + i * 1024) % kLds + lane * 16);
#pragma unroll
        for (int i = 0; i < 8; ++i) x ^= f[i][0] + f[i][3];
    }
    stamp(clk, 1);
    out[blockIdx.x * kThreads + tid] = x;
}

struct Rate {
    double tbs, bpc, ghz;
};

// bytes moved per work-group; rate over the device (event time) and per CU per clock
Rate measure(void (*launch)(long long *, int *), double bytes_per_block)
{
    long long *clk;
    int *out;
    if (hipMalloc(&clk, 4 * kBlocks * sizeof(long long)) != hipSuccess) return {-1, -1, -1};
    if (hipMalloc(&out, kBlocks * kThreads * sizeof(int)) != hipSuccess) return {-1, -1, -1};
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    launch(clk, out);                                  // warm-up (fills L2)
    (void)hipEventRecord(e0, 0);
    launch(clk, out);
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    long long h[4 * kBlocks];
    (void)hipMemcpy(h, clk, sizeof h, hipMemcpyDeviceToHost);
    double cyc = 0.0, rt = 0.0;
    for (int b = 0; b < kBlocks; ++b) {
        cyc += (double)(h[4 * b + 2] - h[4 * b]);
        rt += (double)(h[4 * b + 3] - h[4 * b + 1]);
    }
    cyc /= kBlocks;
    rt /= kBlocks;
    (void)hipFree(clk);
    (void)hipFree(out);
    return {bytes_per_block * kBlocks / (ms * 1e-3) / 1e12, bytes_per_block / cyc, cyc / (rt / 100e6) / 1e9};
}

const char *g_src = nullptr;
long long g_win = 0;
int g_steps = 0;

void launch_dma(long long *clk, int *out)
{
    hipLaunchKernelGGL(copy_kernel<0>, dim3(kBlocks), dim3(kThreads), kLds, 0, g_src, g_win, g_steps, clk, out);
}
void launch_reg(long long *clk, int *out)
{
    hipLaunchKernelGGL(copy_kernel<1>, dim3(kBlocks), dim3(kThreads), kLds, 0, g_src, g_win, g_steps, clk, out);
}
void launch_lds(long long *clk, int *out)
{
    hipLaunchKernelGGL(lds_read_kernel, dim3(kBlocks), dim3(kThreads), kLds, 0, g_steps, clk, out);
}

}  // namespace

int main()
{
    const long long big = 64LL << 20;
    char *src;
    if (hipMalloc(&src, kBlocks * big) != hipSuccess) {
        std::printf("{\"error\": \"allocation failed\"}\n");
        return 1;
    }
    (void)hipMemset(src, 1, kBlocks * big);
    (void)hipFuncSetAttribute((const void *)copy_kernel<0>, hipFuncAttributeMaxDynamicSharedMemorySize, kLds);
    (void)hipFuncSetAttribute((const void *)copy_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, kLds);
    (void)hipFuncSetAttribute((const void *)lds_read_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLds);
    const double step = (double)kWaves * kPer * 1024;
    g_src = src;
    g_win = 49152;
    g_steps = 20000;
    const Rate dma = measure(launch_dma, step * g_steps);
    const Rate reg = measure(launch_reg, step * g_steps);
    g_win = big;
    g_steps = 2000;
    const Rate hbm = measure(launch_dma, step * g_steps);
    g_steps = 200000;
    const Rate lds = measure(launch_lds, (double)kWaves * 8 * 1024 * g_steps);
    (void)hipFree(src);
    std::printf("{\"l2_lds_dma_tbs\": %.2f, \"l2_lds_dma_bpc\": %.1f, \"l2_lds_dma_ghz\": %.2f, \"l2_lds_reg_tbs\": %.2f, "
                "\"l2_lds_reg_bpc\": %.1f, \"hbm_lds_dma_tbs\": %.2f, \"hbm_lds_dma_bpc\": %.1f, \"lds_read_tbs\": %.2f, "
                "\"lds_read_bpc\": %.1f, \"lds_read_ghz\": %.2f}\n",
                dma.tbs, dma.bpc, dma.ghz, reg.tbs, reg.bpc, hbm.tbs, hbm.bpc, lds.tbs, lds.bpc, lds.ghz);
    return 0;
}
