// Block shapes of the modular contraction against the power limit of the int8 matrix cores.
//
// Runs the library's contraction kernel (hs_mod_i8_kernel<4, 256>: 256 x 128 blocks, both
// evaluation products of a modulus in one pass) and a square-block variant (below: 256 x 256
// blocks, the two products in two passes) on the same synthetic residue planes of one k-point
// (nt 128-column tiles, kp2 rows, 11 moduli; residues uniform in [-R, R] for each R given), times
// each launch with HIP events, and checks that both write identical residue tiles.  The variant
// copies a third fewer bytes from L2 into LDS and reads a quarter fewer fragment bytes per MFMA;
// under rocprofv3 counters it needs fewer cycles at a lower clock, which is how the board's power
// limit shows.  The library keeps the 256 x 128 kernel.
//
// Usage: mod_blocks [nt [kp2 [reps [R ...]]]]   (defaults 96 123904 2 120; nt even, kp2 a
// multiple of 64); exit status 0 when the residue tiles agree, 2 when they differ.
#include "mod_contract.hip"

#include <cstdio>
#include <cstdlib>
#include <vector>

namespace flapw {
namespace {

// The square-block variant.  One block per (256 x 256 output block, modulus), eight waves of
// 128 x 64.  The two evaluation products run one after the other over all rows: the first pass
// copies only the first evaluation of each group (16 KB per 32-row group for both operands), its
// sums are reduced mod p and kept as int8 in registers (32 VGPRs), the second pass streams the
// second evaluation, and the epilogue forms Re and Im as the library's kernel does and stores them
// in the same residue-tile layout.  Per group it copies 16 KB and reads 48 KB of fragments for
// 64 MFMAs, against 24 KB and 64 KB for the library's 256 x 128 blocks.  The right fragments
// alternate between two register sets so that each half of a group's products (rows 0-63, 64-127
// of the wave) runs while the next group's fragments of the other half are read.
template <int CH>
struct SqStage {
    static constexpr int kGroups = CH / 2;               // 32-row groups per LDS stage
    static constexpr int kStageRows = 16 * CH;           // complex rows per LDS stage
    static constexpr int kRuns = 16;                     // 8 left + 8 right 32-column runs
    static constexpr int kRunBytes = kGroups * 1024;     // one evaluation of one run over one stage
    static constexpr int kStageBytes = kRuns * kRunBytes;
    static constexpr int kRing = 4;                      // 128 KB of LDS
    static constexpr int kWaves = 8;
    static constexpr int kCopies = kRuns * kGroups / kWaves;
    static constexpr int kFlushStages = 65536 / kStageRows;
    static_assert(kGroups == 2, "two groups per stage: the right fragments alternate between two register sets");
    static_assert((kRing - 1) * kCopies < 64, "vmcnt field");
};

__global__ __launch_bounds__(512, 1) void hs_mod_sq_kernel(const ModProblemDev *__restrict__ probs,
                                                           const TileDev *__restrict__ tiles, ModTable mt)
{
    using G = SqStage<4>;
    constexpr int kGroups = G::kGroups, kStageRows = G::kStageRows, kRunBytes = G::kRunBytes;
    constexpr int kStageBytes = G::kStageBytes, kRing = G::kRing, kCopies = G::kCopies;
    constexpr int kFlushStages = G::kFlushStages;
    extern __shared__ __align__(16) unsigned char smem[];
    const TileDev td = tiles[blockIdx.x];
    const ModProblemDev pb = probs[td.prob];
    const int mo = blockIdx.y, mat = td.pad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;             // rows 128 wm, columns 64 wn of the block
    const long long nch = pb.kp2 / 16;
    const long long mstride = (long long)pb.ncb * nch * 1024;
    const long long cbytes = nch * 1024;
    const int8_t *Lg = pb.L + mo * mstride + 8LL * td.ti * cbytes;
    const int8_t *Rg = (mat ? pb.RH : pb.RS) + mo * mstride + 8LL * td.tj * cbytes;
    const int nst = pb.kp2 / kStageRows;
    const int pi = mt.p[mo];
    const float ipf = 1.0f / (float)pi;

    v16i acc[4][2];
    unsigned stash[4][2][4];

    const int half = lane >> 5, col = lane & 31;
    const int la0 = (4 * wm) * kRunBytes + half * 512 + col * 16;
    const int lb0 = (8 + 2 * wn) * kRunBytes + half * 512 + col * 16;
    v4i a[4], b[2][2];

    // wave w copies segments s = w + 8 q: run (w >> 1) + 4 q (left for q < 2), group w & 1
#define SQ_COPY(st, sl, E)                                                                        \
    do {                                                                                          \
        _Pragma("unroll") for (int q_ = 0; q_ < kCopies; ++q_) {                                  \
            const int r_ = (wave >> 1) + 4 * q_, g_ = wave & 1;                                   \
            const int8_t *src_ = (r_ < 8 ? Lg + (long long)r_ * cbytes : Rg + (long long)(r_ - 8) * cbytes) + \
                                 (((long long)(st) * kGroups + g_) * 2 + (E)) * 1024 + lane * 16; \
            __builtin_amdgcn_global_load_lds((const int __attribute__((address_space(1))) *)src_,   \
                (int __attribute__((address_space(3))) *)(smem + (sl) * kStageBytes + r_ * kRunBytes + g_ * 1024), \
                16, 0, 0);                                                                        \
        }                                                                                         \
    } while (0)
#define SQ_READ_A(sl, grp, I0)                                                                    \
    do {                                                                                          \
        const unsigned char *s_ = smem + (sl) * kStageBytes + (grp) * 1024 + la0;                 \
        a[I0] = *reinterpret_cast<const v4i *>(s_ + (I0) * kRunBytes);                            \
        a[I0 + 1] = *reinterpret_cast<const v4i *>(s_ + ((I0) + 1) * kRunBytes);                  \
    } while (0)
#define SQ_READ_B(sl, grp, S)                                                                     \
    do {                                                                                          \
        const unsigned char *s_ = smem + (sl) * kStageBytes + (grp) * 1024 + lb0;                 \
        b[S][0] = *reinterpret_cast<const v4i *>(s_);                                             \
        b[S][1] = *reinterpret_cast<const v4i *>(s_ + kRunBytes);                                 \
    } while (0)

#pragma unroll 1
    for (int E = 0; E < 2; ++E) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;
#pragma unroll
        for (int s0 = 0; s0 < kRing; ++s0)
            if (s0 < nst) SQ_COPY(s0, s0, E);
        ring_wait<kCopies, kRing - 1>(min(kRing - 1, nst - 1));
        SQ_READ_A(0, 0, 0);
        SQ_READ_A(0, 0, 2);
        SQ_READ_B(0, 0, 0);

        int sl = 0;
        for (int st0 = 0; st0 < nst; st0 += kFlushStages) {
            const int st1 = min(nst, st0 + kFlushStages);
            for (int st = st0; st < st1; ++st) {
                const int sn = sl == kRing - 1 ? 0 : sl + 1;
#pragma unroll
                for (int gg = 0; gg < kGroups; ++gg) {
                    const bool last = gg + 1 == kGroups;
                    const bool more = !last || st + 1 < nst;
                    const int nslot = last ? sn : sl, ngrp = last ? 0 : gg + 1;
                    const int cs = gg, ns = gg ^ 1;             // register set of this group's and the next group's b
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[cs][j], acc[i][j], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (last && st + 1 < nst) ring_wait<kCopies, kRing - 1>(min(kRing - 2, nst - st - 2));
                    if (more) {
                        SQ_READ_A(nslot, ngrp, 0);
                        SQ_READ_B(nslot, ngrp, ns);
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int i = 2; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[cs][j], acc[i][j], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (more) SQ_READ_A(nslot, ngrp, 2);
                    if (last && st + kRing < nst) SQ_COPY(st + kRing, sl, E);
                    __builtin_amdgcn_sched_barrier(0);
                }
                sl = sn;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[i][j][r] = mod_step(acc[i][j][r], pi, ipf);
        }
        if (E == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        unsigned w = 0;
#pragma unroll
                        for (int bq = 0; bq < 4; ++bq)
                            w |= ((unsigned)mod_step(acc[i][j][4 * q + bq], pi, ipf) & 0xffu) << (8 * bq);
                        stash[i][j][q] = w;
                    }
            ring_barrier<0>();                          // every wave's reads of the ring are done
        }
    }
#undef SQ_READ_A
#undef SQ_READ_B
#undef SQ_COPY

    const int h2 = mt.h2[mo], h2j = mt.h2j[mo];
    const int slot0 = mat * pb.ntri;
    int8_t *out0 = pb.res + (long long)mo * 2 * pb.ntri * kResTileBytes;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * wm + i;
        const int ti = 2 * td.ti + (r >> 2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = 2 * wn + j;
            const int tj = 2 * td.tj + (c >> 2);
            if (ti > tj) continue;
            int8_t *out = out0 + (long long)(slot0 + tri_index(ti, tj)) * kResTileBytes;
            const int quarter = ((r >> 1) & 1) * 2 + ((c >> 1) & 1);
            unsigned wre[4], wim[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned pre = 0, pim = 0;
#pragma unroll
                for (int bq = 0; bq < 4; ++bq) {
                    const int z1 = (int)(signed char)((stash[i][j][q] >> (8 * bq)) & 0xffu);
                    const int z2 = acc[i][j][4 * q + bq];
                    const int re = mod_step(mod_step((z1 + z2) * h2, pi, ipf), pi, ipf);
                    const int im = mod_step(mod_step((z1 - z2) * h2j, pi, ipf), pi, ipf);
                    pre |= ((unsigned)re & 0xffu) << (8 * bq);
                    pim |= ((unsigned)im & 0xffu) << (8 * bq);
                }
                wre[q] = pre;
                wim[q] = pim;
            }
            const int grp = ((quarter * 2 + (r & 1)) * 2 + (c & 1)) * 2;
            *reinterpret_cast<uint4 *>(out + ((long long)grp * 64 + lane) * 16) = make_uint4(wre[0], wre[1], wre[2], wre[3]);
            *reinterpret_cast<uint4 *>(out + ((long long)(grp + 1) * 64 + lane) * 16) = make_uint4(wim[0], wim[1], wim[2], wim[3]);
        }
    }
}

__global__ void fill_kernel(int8_t *p, size_t n, unsigned seed, int R)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        unsigned h = (unsigned)i * 2654435761u ^ seed;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        p[i] = (int8_t)((int)(h % (unsigned)(2 * R + 1)) - R);
    }
}

__global__ void count_diff_kernel(const int8_t *x, const int8_t *y, size_t n, unsigned long long *cnt)
{
    unsigned long long c = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        c += x[i] != y[i];
    if (c) atomicAdd(cnt, c);
}

// blocks (bi, tj) with rt bi <= tj (rt = block rows / 128) in bands of 4 block rows, each XCD
// taking a contiguous eighth of the order (as the library lists them)
std::vector<TileDev> block_list(int nt, int rt, int ct)
{
    std::vector<TileDev> order, t;
    const int nb = nt / rt;
    for (int b0 = 0; b0 < nb; b0 += 4)
        for (int tj = rt * b0 / ct; tj < nt / ct; ++tj)
            for (int bi = b0; bi < std::min(b0 + 4, (ct * tj) / rt + 1); ++bi)
                for (int m = 0; m < 2; ++m) order.push_back(TileDev{0, bi, tj, m});
    const int n = (int)order.size(), q = n / 8, rem = n % 8;
    int start[9];
    start[0] = 0;
    for (int x = 0; x < 8; ++x) start[x + 1] = start[x] + q + (x < rem ? 1 : 0);
    t.resize(n);
    for (int b = 0; b < n; ++b) t[b] = order[start[b % 8] + b / 8];
    return t;
}

template <typename F>
float time_launches(F launch, int reps)
{
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    launch();
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(b, 0);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

}  // namespace
}  // namespace flapw

using namespace flapw;

#define CK(x)                                                                                     \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) {                                                                   \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);                 \
            return 1;                                                                             \
        }                                                                                         \
    } while (0)

static int gcd(int a, int b)
{
    while (b) {
        const int r = a % b;
        a = b;
        b = r;
    }
    return a;
}

int main(int argc, char **argv)
{
    const int nt = argc > 1 ? atoi(argv[1]) : 96;
    const long long kp2 = argc > 2 ? atoll(argv[2]) : 123904;
    const int reps = argc > 3 ? atoi(argv[3]) : 2;
    const int nm = 11;
    if (nt < 2 || nt % 2 || kp2 < 64 || kp2 % 64 || reps < 1) {
        printf("nt must be even, kp2 a positive multiple of 64\n");
        return 1;
    }
    std::vector<int> ranges;
    for (int i = 4; i < argc; ++i) ranges.push_back(atoi(argv[i]));
    if (ranges.empty()) ranges.push_back(120);
    for (int R : ranges)
        if (R < 0 || R > 127) {
            printf("R must lie in 0..127\n");
            return 1;
        }
    const long long npm = nt * 128LL, ncb = npm / 32, nch = kp2 / 16;
    const size_t plane = (size_t)ncb * nch * 1024;
    const long long ntri = (long long)nt * (nt + 1) / 2;
    const size_t rbytes = 2ULL * ntri * nm * kResTileBytes;
    printf("nt %d (N %lld), kp2 %lld, %d moduli: residue planes %.2f GB, residue tiles %.2f GB\n", nt, npm, kp2, nm,
           3.0 * plane * nm / 1e9, rbytes / 1e9);
    int8_t *L, *RS, *RH, *res1, *res2;
    CK(hipMalloc(&L, plane * nm));
    CK(hipMalloc(&RS, plane * nm));
    CK(hipMalloc(&RH, plane * nm));
    CK(hipMalloc(&res1, rbytes));
    CK(hipMalloc(&res2, rbytes));
    CK(hipMemset(res1, 0, rbytes));
    CK(hipMemset(res2, 0, rbytes));

    ModTable mt{};
    mt.nm = nm;
    for (int c = 255, k = 0; k < nm; c -= 2) {            // odd moduli with a square root of -1
        bool ok = false;
        for (int x = 1; x < c && !ok; ++x) ok = (x * x + 1) % c == 0;
        for (int j = 0; ok && j < k; ++j) ok = gcd(c, mt.p[j]) == 1;
        if (ok) mt.p[k++] = c;
    }
    for (int m = 0; m < nm; ++m) {                        // any residues do for the comparison
        mt.h2[m] = (mt.p[m] + 1) / 2;
        mt.h2j[m] = 3;
    }
    ModProblemDev pb{};
    pb.L = L;
    pb.RS = RS;
    pb.RH = RH;
    pb.ldh = npm;
    pb.n = (int)npm;
    pb.kp2 = (int)kp2;
    pb.ncb = (int)ncb;
    pb.ntri = (int)ntri;
    ModProblemDev *dpb[2];
    for (int v = 0; v < 2; ++v) {
        pb.res = v ? res2 : res1;
        CK(hipMalloc(&dpb[v], sizeof pb));
        CK(hipMemcpy(dpb[v], &pb, sizeof pb, hipMemcpyHostToDevice));
    }
    const std::vector<TileDev> t1 = block_list(nt, 2, 1), t2 = block_list(nt, 2, 2);
    for (const TileDev &t : t1)
        if (8 * t.ti + 7 >= ncb || 4 * t.tj + 3 >= ncb || 2 * t.ti > t.tj) return printf("bad block\n"), 1;
    for (const TileDev &t : t2)
        if (8 * t.ti + 7 >= ncb || 8 * t.tj + 7 >= ncb || t.ti > t.tj) return printf("bad block\n"), 1;
    TileDev *d1, *d2;
    CK(hipMalloc(&d1, t1.size() * sizeof(TileDev)));
    CK(hipMalloc(&d2, t2.size() * sizeof(TileDev)));
    CK(hipMemcpy(d1, t1.data(), t1.size() * sizeof(TileDev), hipMemcpyHostToDevice));
    CK(hipMemcpy(d2, t2.data(), t2.size() * sizeof(TileDev), hipMemcpyHostToDevice));
    using G = SqStage<4>;
    CK(init_mod_kernels());
    CK(hipFuncSetAttribute((const void *)hs_mod_sq_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                           G::kRing * G::kStageBytes));
    printf("blocks per modulus: 256 x 128 %zu, 256 x 256 %zu\n", t1.size(), t2.size());
    fflush(stdout);

    for (int R : ranges) {
        hipLaunchKernelGGL(fill_kernel, dim3(4096), dim3(256), 0, 0, L, plane * nm, 1u, R);
        hipLaunchKernelGGL(fill_kernel, dim3(4096), dim3(256), 0, 0, RS, plane * nm, 2u, R);
        hipLaunchKernelGGL(fill_kernel, dim3(4096), dim3(256), 0, 0, RH, plane * nm, 3u, R);
        CK(hipDeviceSynchronize());
        const float ms1 = time_launches([&] { (void)launch_mod_contract(dpb[0], d1, (int)t1.size(), mt, 4, 0); }, reps);
        const float ms2 = time_launches([&] {
            hipLaunchKernelGGL(hs_mod_sq_kernel, dim3((unsigned)t2.size(), nm), dim3(512), G::kRing * G::kStageBytes, 0,
                               dpb[1], d2, mt);
        }, reps);
        CK(hipDeviceSynchronize());
        printf("residues in [-%d, %d]: 256 x 128 blocks %.1f ms, 256 x 256 blocks %.1f ms per launch\n", R, R, ms1, ms2);
        fflush(stdout);
    }
    unsigned long long *cnt, h = 0;
    CK(hipMalloc(&cnt, sizeof *cnt));
    CK(hipMemset(cnt, 0, sizeof *cnt));
    hipLaunchKernelGGL(count_diff_kernel, dim3(4096), dim3(256), 0, 0, res1, res2, rbytes, cnt);
    CK(hipMemcpy(&h, cnt, sizeof h, hipMemcpyDeviceToHost));
    printf("residue tiles differing: %llu of %zu bytes\n", h, rbytes);
    return h == 0 ? 0 : 2;
}
