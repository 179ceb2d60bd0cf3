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
//   hs_mod_i8_kernel<CH, BR> one block per (BR x 128 output block, modulus), BR = 256: eight
//                       waves of 64 x 64, stages of 16 CH rows copied to LDS by global_load_lds into
//                       a ring of three (CH = 4) or four (CH = 2) buffers, the younger stages in
//                       flight; each half of a group's products (first, second evaluation) issued
//                       while the other half's next fragments are read; writes the residues of Re
//                       and Im (int8, 32 KB per 128 x 128 tile) to the problem's scratch
#include "context.hpp"

namespace flapw {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Stage geometry for CH 16-row chunks per LDS stage (CH = 4: 64-row stages; CH = 2: 32-row
// stages) and blocks of BR x 128 (eight waves of BR/4 x 64).  The library launches BR = 256; 384
// also compiles but needs more accumulator registers than two waves per SIMD hold.  A stage is
// BR/32 left and 4 right 32-column runs of CH 1 KB segments.
template <int CH, int BR>
struct ModStage {
    static constexpr int kChunks = CH;                   // 16-row chunks per LDS stage
    static constexpr int kGroups = CH / 2;               // 32-row groups per LDS stage
    static constexpr int kStageRows = 16 * CH;           // complex rows per LDS stage
    static constexpr int kLeftRuns = BR / 32;            // 32-column runs of the left operand
    static constexpr int kRuns = kLeftRuns + 4;
    static constexpr int kRunBytes = CH * 1024;          // one 32-column run over one stage
    static constexpr int kStageBytes = kRuns * kRunBytes;
    static constexpr int kRing = 163840 / kStageBytes < 4 ? 163840 / kStageBytes : 4;  // LDS stage buffers
    static constexpr int kWaves = 8;
    static constexpr int kCopies = kRuns * CH / kWaves;  // 1 KB copies per wave per stage
    static constexpr int kWM = BR / 128;                 // 32-row tiles per wave
    static constexpr int kWN = 2;                        // 32-column tiles per wave
    static constexpr int kFlushStages = 65536 / kStageRows;  // 65536 rows * 127^2 < 2^31
    static_assert(CH % 2 == 0 && kRing >= 2 && (kRuns * CH) % kWaves == 0 && BR % 128 == 0, "stage geometry");
    static_assert((kRing - 1) * kCopies < 64, "vmcnt field");
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

// Work-group barrier of the stage ring.  Before it, the wave waits until at most IN_FLIGHT of its
// LDS-DMA copies are outstanding (copies complete in issue order, so the older stages have
// landed) and until all its LDS reads have returned (so the slot about to be refilled is no longer
// read).  Unlike __syncthreads it does not drain all copies.  s_waitcnt's immediate (gfx9
// encoding): vmcnt bits 3:0 and 15:14, expcnt 6:4 (7: no wait), lgkmcnt 11:8 (0).  The empty asm
// statements keep the compiler from moving memory accesses across the barrier.
template <int IN_FLIGHT>
__device__ inline void ring_barrier()
{
    static_assert(IN_FLIGHT >= 0 && IN_FLIGHT < 64, "vmcnt field");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((IN_FLIGHT & 15) | ((IN_FLIGHT >> 4) << 14) | (0x7 << 4));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ring_barrier with min(later, L) younger stages allowed in flight, COPIES copies each per wave
template <int COPIES, int L>
__device__ inline void ring_wait(int later)
{
    if constexpr (L == 0) {
        ring_barrier<0>();
    } else {
        if (later >= L) ring_barrier<L * COPIES>();
        else ring_wait<COPIES, L - 1>(later);
    }
}

// grid (n_tiles, nm): block tile blockIdx.x of the launch's list -- rows BR I .. BR I + BR - 1
// (the 128-row tiles (BR/128) I ..), columns 128 J .. 128 J + 127 -- and modulus blockIdx.y.
// Eight waves, wave w computing the kWM x 2 tiles of 32 x 32 at rows 32 kWM (w / 2), columns
// 64 (w % 2) of the block tile.
//
// Pipeline.  Each 32-row group issues the z1 products (first evaluations), then reads the first
// evaluations of the next group into the same registers, issues the z2 products and reads the
// second evaluations of the next group: the reads of one half run under the other half's
// products, and one group's fragments are live at a time.  At the last group of stage st, between
// its two halves, the wave waits for stage st + 1 to land (its own copies, then the barrier for
// everyone's; every read of stage st has returned by then), and after the group's products it
// refills the slot of stage st with stage st + kRing: the copies run kRing - 1 stages ahead of
// the reads.
template <int CH, int BR>
__global__ __launch_bounds__(512, 1) void hs_mod_i8_kernel(const ModProblemDev *__restrict__ probs,
                                                           const TileDev *__restrict__ tiles, ModTable mt)
{
    using G = ModStage<CH, BR>;
    constexpr int kChunks = G::kChunks, kGroups = G::kGroups, kStageRows = G::kStageRows;
    constexpr int kRunBytes = G::kRunBytes, kStageBytes = G::kStageBytes, kLeftRuns = G::kLeftRuns;
    constexpr int kRing = G::kRing, kCopies = G::kCopies, kFlushStages = G::kFlushStages;
    constexpr int WM = G::kWM, WN = G::kWN, NW = G::kWaves;
    extern __shared__ __align__(16) unsigned char smem[];
    const TileDev td = tiles[blockIdx.x];
    const ModProblemDev pb = probs[td.prob];
    const int mo = blockIdx.y, mat = td.pad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const long long nch = pb.kp2 / 16;
    const long long mstride = (long long)pb.ncb * nch * 1024;
    const long long cbytes = nch * 1024;                          // one 32-column block, all rows
    const int8_t *Lg = pb.L + mo * mstride + (long long)kLeftRuns * td.ti * cbytes;
    const int8_t *Rg = (mat ? pb.RH : pb.RS) + mo * mstride + 4LL * td.tj * cbytes;
    const int nst = pb.kp2 / kStageRows;
    const int pi = mt.p[mo];
    const float ipf = 1.0f / (float)pi;

    v16i acc[WM][WN][2];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][c][r] = 0;

    // Wave w copies segments g = w + NW q (run g / kChunks, chunk g % kChunks), q = 0..kCopies-1,
    // lane l's 16 bytes landing at +16 l; runs below kLeftRuns come from the left operand.  (The
    // macro's own names end in '_' so that arguments cannot capture them.)
#define MOD_COPY(st, b)                                                                           \
    do {                                                                                          \
        _Pragma("unroll") for (int cq_ = 0; cq_ < kCopies; ++cq_) {                               \
            const int g_ = wave + NW * cq_, r_ = g_ / kChunks, c_ = g_ % kChunks;                 \
            const int8_t *src_ = (r_ < kLeftRuns ? Lg + (long long)r_ * cbytes                    \
                                                 : Rg + (long long)(r_ - kLeftRuns) * cbytes) +   \
                                 ((long long)(st) * kChunks + c_) * 1024 + lane * 16;             \
            __builtin_amdgcn_global_load_lds((const int __attribute__((address_space(1))) *)src_,   \
                (int __attribute__((address_space(3))) *)(smem + (b) * kStageBytes + r_ * kRunBytes + c_ * 1024), \
                16, 0, 0);                                                                        \
        }                                                                                         \
    } while (0)

    // fragments of 32-row group g of a stage: evaluations at j at +2048 g, at -j at +2048 g + 1024
    // (E = 0, 1); lane (half, col) holds rows 16 half .. 16 half + 15 of column col
    const int half = lane >> 5, col = lane & 31;
    const int la0 = (WM * wm) * kRunBytes + half * 512 + col * 16;
    const int lb0 = (kLeftRuns + WN * wn) * kRunBytes + half * 512 + col * 16;
    v4i a1[WM], a2[WM], b1[WN], b2[WN];
#define MOD_READ(slot, grp, E, A, B)                                                              \
    do {                                                                                          \
        const unsigned char *st_ = smem + (slot) * kStageBytes + (grp) * 2048 + (E) * 1024;       \
        _Pragma("unroll") for (int i_ = 0; i_ < WM; ++i_)                                         \
            A[i_] = *reinterpret_cast<const v4i *>(st_ + la0 + i_ * kRunBytes);                   \
        _Pragma("unroll") for (int j_ = 0; j_ < WN; ++j_)                                         \
            B[j_] = *reinterpret_cast<const v4i *>(st_ + lb0 + j_ * kRunBytes);                   \
    } while (0)

    // all kRing slots filled; wait for stage 0 (later stages may stay in flight), read its first group
#pragma unroll
    for (int s0 = 0; s0 < kRing; ++s0)
        if (s0 < nst) MOD_COPY(s0, s0);
    ring_wait<kCopies, kRing - 1>(min(kRing - 1, nst - 1));
    MOD_READ(0, 0, 0, a1, b1);
    MOD_READ(0, 0, 1, a2, b2);

    int b = 0;                                    // ring slot of stage st
    for (int st0 = 0; st0 < nst; st0 += kFlushStages) {
        const int st1 = min(nst, st0 + kFlushStages);
        for (int st = st0; st < st1; ++st) {
            const int bn = b == kRing - 1 ? 0 : b + 1;      // slot of stage st + 1
#pragma unroll
            for (int gg = 0; gg < kGroups; ++gg) {
                const bool last = gg + 1 == kGroups;
                const bool more = !last || st + 1 < nst;
                const int nslot = last ? bn : b, ngrp = last ? 0 : gg + 1;
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        acc[i][j][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1[i], b1[j], acc[i][j][0], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                // stage st + 1 landed for everyone; stage st is no longer read
                if (last && st + 1 < nst) ring_wait<kCopies, kRing - 1>(min(kRing - 2, nst - st - 2));
                if (more) MOD_READ(nslot, ngrp, 0, a1, b1);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        acc[i][j][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2[i], b2[j], acc[i][j][1], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                if (more) MOD_READ(nslot, ngrp, 1, a2, b2);
                // refill the slot of stage st (free since the barrier) after the products are queued: a
                // copy issued before them can hold the wave while the memory queue drains
                if (last && st + kRing < nst) MOD_COPY(st + kRing, b);
                __builtin_amdgcn_sched_barrier(0);
            }
            b = bn;
        }
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[i][j][c][r] = mod_step(acc[i][j][c][r], pi, ipf);
    }
#undef MOD_READ
#undef MOD_COPY
    // Re = (z1 + z2) / 2, Im = (z1 - z2) / (2 j) mod p (|z1 +- z2| <= 6p after the flush step,
    // inverses in the symmetric range: the products stay below 2^18, exact in float)
    const int h2 = mt.h2[mo], h2j = mt.h2j[mo];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int z1 = acc[i][j][0][r], z2 = acc[i][j][1][r];
                acc[i][j][0][r] = mod_step(mod_step((z1 + z2) * h2, pi, ipf), pi, ipf);
                acc[i][j][1][r] = mod_step(mod_step((z1 - z2) * h2j, pi, ipf), pi, ipf);
            }

    // residues of each 32 x 32 tile (block row r, column c), stored per 128 x 128 tile
    // ((BR/128) I + r / 4, J) as [64 x 64 quarter (r / 2 % 2, c / 2)][r % 2][c % 2][re, im][lane]
    // [16 bytes]; tiles below the diagonal are skipped
    const int slot0 = mat * pb.ntri;
    int8_t *out0 = pb.res + (long long)mo * 2 * pb.ntri * kResTileBytes;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const int r = WM * wm + i;
        const int ti = (BR / 128) * td.ti + (r >> 2);
        if (ti > td.tj) continue;
        int8_t *out = out0 + (long long)(slot0 + tri_index(ti, td.tj)) * kResTileBytes;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int c = WN * wn + j;
            const int quarter = ((r >> 1) & 1) * 2 + (c >> 1);
#pragma unroll
            for (int cp = 0; cp < 2; ++cp) {
                unsigned w[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    unsigned packed = 0;
#pragma unroll
                    for (int bq = 0; bq < 4; ++bq) packed |= ((unsigned)acc[i][j][cp][4 * q + bq] & 0xffu) << (8 * bq);
                    w[q] = packed;
                }
                const int grp = ((quarter * 2 + (r & 1)) * 2 + (c & 1)) * 2 + cp;
                *reinterpret_cast<uint4 *>(out + ((long long)grp * 64 + lane) * 16) = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
}

template <int CH, int BR>
hipError_t set_mod_lds()
{
    using G = ModStage<CH, BR>;
    return hipFuncSetAttribute((const void *)hs_mod_i8_kernel<CH, BR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               G::kRing * G::kStageBytes);
}

template <int CH, int BR>
void launch_mod_variant(const ModProblemDev *probs, const TileDev *tiles, int n_tiles, const ModTable &mt, hipStream_t s)
{
    using G = ModStage<CH, BR>;
    hipLaunchKernelGGL((hs_mod_i8_kernel<CH, BR>), dim3(n_tiles, mt.nm), dim3(512), G::kRing * G::kStageBytes, s,
                       probs, tiles, mt);
}

}  // namespace

hipError_t init_mod_kernels()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    hipError_t e = set_mod_lds<4, 256>();
    if (e == hipSuccess) e = set_mod_lds<2, 256>();
    done = e;
    return done;
}

// chunks: 16-row chunks per LDS stage (4 or 2)
hipError_t launch_mod_contract(const ModProblemDev *probs, const TileDev *tiles, int n_tiles, const ModTable &mt,
                               int chunks, hipStream_t s)
{
    hipError_t e = init_mod_kernels();
    if (e != hipSuccess) return e;
    if (chunks == 2) launch_mod_variant<2, 256>(probs, tiles, n_tiles, mt, s);
    else if (chunks == 4) launch_mod_variant<4, 256>(probs, tiles, n_tiles, mt, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace flapw
