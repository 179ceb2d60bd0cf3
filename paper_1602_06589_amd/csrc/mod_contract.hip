// Modular split precision: the contraction modulo each modulus (the scheme, the residue slicing
// and the reconstruction are described in split_mod.hip).
//
// Residues.  r = X' mod p_m in the symmetric range [-(p-1)/2, (p-1)/2] fits int8.  Each operand is
// stored as the residues of its two evaluations at the square roots +-j of -1 mod p_m (the left one
// conjugated), so that z1 = U1^T Y1 = Re + j Im and z2 = U2^T Y2 = Re - j Im are plain real products.
// Per modulus they run on v_mfma_i32_32x32x32_i8 over 32-row groups, each evaluation of a group in a
// 1 KB fragment (lanes 0-31 rows 0-15, lanes 32-63 rows 16-31): two products per group and pair of
// 32 x 32 tiles, from two fragment reads per tile row and column.  A row adds at most 127^2 to an
// int32 accumulator; accumulators are reduced mod p every kFlushStages stages (65536 rows), so they
// stay below 2^31.  The epilogue turns z1, z2 into Re = (z1 + z2) / 2 and Im = (z1 - z2) / (2 j).
//
//   hs_mod_i8_kernel<CH> one block per (256 x 128 output block, modulus): eight waves of 64 x 64,
//                       stages of 16 CH rows copied to LDS by global_load_lds into a ring of three
//                       (CH = 4) or four (CH = 2) buffers, the younger stages in flight; fragments
//                       of the next 32-row group read ahead of the MFMAs; writes the residues of Re
//                       and Im (int8, 32 KB per 128 x 128 tile) to the problem's scratch
#include "context.hpp"

namespace flapw {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Stage geometry for CH 16-row chunks per LDS stage (CH = 4: 64-row stages, the default; CH = 2:
// 32-row stages, a choice of the autotuner).
template <int CH>
struct ModStage {
    static constexpr int kChunks = CH;                   // 16-row chunks per LDS stage
    static constexpr int kStageRows = 16 * CH;           // complex rows per LDS stage
    static constexpr int kRunBytes = CH * 1024;          // one 32-column block over one stage
    static constexpr int kStageBytes = 12 * kRunBytes;   // 8 left + 4 right column blocks
    static constexpr int kRing = CH == 4 ? 3 : 4;        // LDS stage buffers: 144 or 96 KB (s_waitcnt immediates
                                                         // use the gfx9 encoding: vmcnt bits 3:0, expcnt 6:4,
                                                         // lgkmcnt 11:8)
    static constexpr int kCopies = 12 * CH / 8;          // 1 KB copies per wave per stage
    static constexpr int kFlushStages = 65536 / kStageRows;  // 65536 rows * 127^2 < 2^31
    static_assert(CH % 2 == 0 && kRing >= 2 && kRing <= 4 && (kRing - 2) * kCopies < 16, "stage ring");
    static_assert(kRing * kStageBytes <= 163840, "LDS budget");
};

// int32 reduction mod odd p in 32-bit arithmetic.  One step leaves |r| <= 3p for any int32 x
// (the float quotient is off by at most 2); a second step on such r is exact and lands in
// [-(p-1)/2, (p-1)/2] (r/p is never a half-integer for odd p).
__device__ inline int mod_step(int x, int p, float ipf)
{
    const int q = (int)rintf((float)x * ipf);
    return x - q * p;
}

// Work-group barrier of the stage ring.  Before it, the wave waits until at most `in_flight`
// of its LDS-DMA copies are outstanding (copies complete in issue order, so the older stage has
// landed) and until all its LDS reads have returned (so the slot about to be refilled is no
// longer read).  Unlike __syncthreads it does not drain all copies.  The empty asm statements
// keep the compiler from moving memory accesses across the barrier.
template <int IN_FLIGHT>
__device__ inline void ring_barrier()
{
    static_assert(IN_FLIGHT >= 0 && IN_FLIGHT < 16, "vmcnt field");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(IN_FLIGHT | (0x7 << 4));      // vmcnt <= IN_FLIGHT, lgkmcnt 0
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ring_barrier with `later` younger stages allowed in flight (COPIES copies each per wave)
template <int COPIES>
__device__ inline void ring_wait(int later)
{
    if (later <= 0) ring_barrier<0>();
    else if (later == 1) ring_barrier<COPIES>();
    else ring_barrier<2 * COPIES>();
}

// grid (n_tiles, nm): block tile blockIdx.x of the launch's list -- rows 256 I .. 256 I + 255
// (the 128-row tiles 2I and 2I + 1), columns 128 J .. 128 J + 127 -- and modulus blockIdx.y.
// Eight waves, wave w computing rows 64 (w >> 1) and columns 64 (w & 1) of the block tile.
template <int CH>
__global__ __launch_bounds__(512, 1) void hs_mod_i8_kernel(const ModProblemDev *__restrict__ probs,
                                                           const TileDev *__restrict__ tiles, ModTable mt)
{
    constexpr int kChunks = ModStage<CH>::kChunks, kStageRows = ModStage<CH>::kStageRows;
    constexpr int kRunBytes = ModStage<CH>::kRunBytes, kStageBytes = ModStage<CH>::kStageBytes;
    constexpr int kRing = ModStage<CH>::kRing, kCopies = ModStage<CH>::kCopies;
    constexpr int kFlushStages = ModStage<CH>::kFlushStages;
    constexpr int kGroups = kChunks / 2;                 // 32-row groups per stage
    extern __shared__ __align__(16) unsigned char smem[];
    const TileDev td = tiles[blockIdx.x];
    const ModProblemDev pb = probs[td.prob];
    const int mo = blockIdx.y, mat = td.pad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const long long nch = pb.kp2 / 16;
    const long long mstride = (long long)pb.ncb * nch * 1024;
    const long long cbytes = nch * 1024;                          // one 32-column block, all rows
    const int8_t *Lg = pb.L + mo * mstride + 8LL * td.ti * cbytes;
    const int8_t *Rg = (mat ? pb.RH : pb.RS) + mo * mstride + 4LL * td.tj * cbytes;
    const int nst = pb.kp2 / kStageRows;
    const int pi = mt.p[mo];
    const float ipf = 1.0f / (float)pi;

    v16i acc[2][2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][c][r] = 0;

    // A stage is 12 runs (8 left, 4 right 32-column blocks) of kChunks 1 KB segments, 12 kChunks
    // segments in all.  Wave w copies segments g = w + 8q (run g / kChunks, chunk g % kChunks),
    // q = 0..kCopies-1, lane l's 16 bytes landing at +16 l; runs 0-7 come from the left operand
    // exactly for q < kChunks.  (The macro's own names end in '_' so that arguments cannot capture them.)  Stages go round a ring of kRing buffers, kRing - 1 stages ahead.
#define MOD_COPY(st, b)                                                                           \
    do {                                                                                          \
        _Pragma("unroll") for (int cq_ = 0; cq_ < kCopies; ++cq_) {                               \
            const int g_ = wave + 8 * cq_, r_ = g_ / kChunks, c_ = g_ % kChunks;                  \
            const int8_t *src_ = (cq_ < kChunks ? Lg + (long long)r_ * cbytes : Rg + (long long)(r_ - 8) * cbytes) + \
                                 ((long long)(st) * kChunks + c_) * 1024 + lane * 16;             \
            __builtin_amdgcn_global_load_lds((const int __attribute__((address_space(1))) *)src_,   \
                (int __attribute__((address_space(3))) *)(smem + (b) * kStageBytes + r_ * kRunBytes + c_ * 1024), \
                16, 0, 0);                                                                        \
        }                                                                                         \
    } while (0)

    // stages 0 .. kRing - 2 in flight; wait for stage 0 (later stages may stay in flight)
#pragma unroll
    for (int s0 = 0; s0 + 1 < kRing; ++s0)
        if (s0 < nst) MOD_COPY(s0, s0);
    ring_wait<kCopies>(min(kRing - 2, nst - 1));

    const int half = lane >> 5, col = lane & 31;
    int b = 0;                                    // ring slot of stage st
    for (int st0 = 0; st0 < nst; st0 += kFlushStages) {
        const int st1 = min(nst, st0 + kFlushStages);
        for (int st = st0; st < st1; ++st) {
            // slot of stage st + kRing - 1, the one read last at stage st - 1
            const int bn = b == 0 ? kRing - 1 : b - 1;
            if (st + kRing - 1 < nst) MOD_COPY(st + kRing - 1, bn);
            // fragments of 32-row group g: evaluations at j at +2048 g, at -j at +2048 g + 1024; lane
            // (half, col) holds rows 16 half .. 16 half + 15 of column col
            const unsigned char *stage = smem + b * kStageBytes;
            const unsigned char *la = stage + (2 * wm) * kRunBytes + half * 512 + col * 16;
            const unsigned char *lb = stage + (8 + 2 * wn) * kRunBytes + half * 512 + col * 16;
            v4i a1[2], a2[2], b1[2], b2[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a1[i] = *reinterpret_cast<const v4i *>(la + i * kRunBytes);
                a2[i] = *reinterpret_cast<const v4i *>(la + i * kRunBytes + 1024);
                b1[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes);
                b2[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes + 1024);
            }
#pragma unroll
            for (int gg = 0; gg < kGroups; ++gg) {
                v4i na1[2], na2[2], nb1[2], nb2[2];
                if (gg + 1 < kGroups) {          // next group's fragments, read ahead
                    const int o = (gg + 1) * 2048;
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        na1[i] = *reinterpret_cast<const v4i *>(la + i * kRunBytes + o);
                        na2[i] = *reinterpret_cast<const v4i *>(la + i * kRunBytes + o + 1024);
                        nb1[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes + o);
                        nb2[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes + o + 1024);
                    }
                }
                // keep the reads ahead of this group's products (the scheduler would sink them)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1[i], b1[j], acc[i][j][0], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2[i], b2[j], acc[i][j][1], 0, 0, 0);
                if (gg + 1 < kGroups) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        a1[i] = na1[i];
                        a2[i] = na2[i];
                        b1[i] = nb1[i];
                        b2[i] = nb2[i];
                    }
                }
            }
            // stage st + 1 must have landed before anyone reads it; later stages may still fly
            if (st + 1 < nst) ring_wait<kCopies>(min(kRing - 2, nst - st - 2));
            b = b == kRing - 1 ? 0 : b + 1;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[i][j][c][r] = mod_step(acc[i][j][c][r], pi, ipf);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][c][r] = mod_step(acc[i][j][c][r], pi, ipf);
#undef MOD_COPY
    // Re = (z1 + z2) / 2, Im = (z1 - z2) / (2 j) mod p (|z1 +- z2| <= p - 1, inverses in the
    // symmetric range: the products stay below 2^15)
    const int h2 = mt.h2[mo], h2j = mt.h2j[mo];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int z1 = acc[i][j][0][r], z2 = acc[i][j][1][r];
                acc[i][j][0][r] = mod_step(mod_step((z1 + z2) * h2, pi, ipf), pi, ipf);
                acc[i][j][1][r] = mod_step(mod_step((z1 - z2) * h2j, pi, ipf), pi, ipf);
            }

    // residues of the wave's 64 x 64 block, stored per 128 x 128 tile (2I + (wm >> 1), J) as
    // [wave in tile][i][j][re, im][lane][16 bytes]; tiles below the diagonal are skipped
    const int ti = 2 * td.ti + (wm >> 1);
    if (ti > td.tj) return;
    const int wt = (wm & 1) * 2 + wn;
    const int slot = mat * pb.ntri + tri_index(ti, td.tj);
    int8_t *out = pb.res + ((long long)mo * 2 * pb.ntri + slot) * kResTileBytes;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                unsigned w[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    unsigned packed = 0;
#pragma unroll
                    for (int bq = 0; bq < 4; ++bq) packed |= ((unsigned)acc[i][j][c][4 * q + bq] & 0xffu) << (8 * bq);
                    w[q] = packed;
                }
                const int grp = ((wt * 2 + i) * 2 + j) * 2 + c;
                *reinterpret_cast<uint4 *>(out + ((long long)grp * 64 + lane) * 16) = make_uint4(w[0], w[1], w[2], w[3]);
            }
}

}  // namespace

hipError_t init_mod_kernels()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    hipError_t e = hipFuncSetAttribute((const void *)hs_mod_i8_kernel<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       ModStage<4>::kRing * ModStage<4>::kStageBytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)hs_mod_i8_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                ModStage<2>::kRing * ModStage<2>::kStageBytes);
    done = e;
    return done;
}

hipError_t launch_mod_contract(const ModProblemDev *probs, const TileDev *tiles, int n_tiles, const ModTable &mt,
                               int chunks, hipStream_t s)
{
    hipError_t e = init_mod_kernels();
    if (e != hipSuccess) return e;
    if (chunks == 2)
        hipLaunchKernelGGL(hs_mod_i8_kernel<2>, dim3(n_tiles, mt.nm), dim3(512),
                           ModStage<2>::kRing * ModStage<2>::kStageBytes, s, probs, tiles, mt);
    else if (chunks == 4)
        hipLaunchKernelGGL(hs_mod_i8_kernel<4>, dim3(n_tiles, mt.nm), dim3(512),
                           ModStage<4>::kRing * ModStage<4>::kStageBytes, s, probs, tiles, mt);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace flapw
