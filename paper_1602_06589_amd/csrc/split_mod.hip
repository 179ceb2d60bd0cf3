// Modular split precision for the S/H contraction: the FP64 operands are scaled to integers and
// the integer products are computed modulo several pairwise coprime odd moduli p_m <= 255 on the int8
// matrix cores, then rebuilt by the Chinese remainder theorem in FP64.  (The paper computes these
// updates in FP64 BLAS, sections 4.2-4.6; this is an alternative to the digit scheme of split.hip
// that needs one int8 product per modulus instead of one per kept digit pair.)
//
// Integers.  Operand column c (a basis function) is scaled by 2^e_c, e_c chosen so that the
// 2-norm of the column over all contraction rows (real and imaginary parts) is below 2^B, and
// rounded: X'_kc = rint(X_kc 2^e_c), |X'| < 2^B <= 2^50 (exact in FP64).  By Cauchy-Schwarz every
// exact integer product entry C'_ij = Re or Im of sum_k conj(X'_ki) Y'_kj has |C'| < 2^(2B) up to
// the rounding of X' and Y' (each adds at most sqrt(2K)/2 < 2^15 to a column norm below 2^B, B >= 31,
// so a factor below 1 + 2^-15 in all), and B is the largest with 2^(2B+1) <= M = prod p_m; for 8..14
// moduli log2 M exceeds 2B + 1 by at least 0.04 (a factor 1.028), so |C'| < 0.49 M and C' is the
// unique residue of C' mod M in (-M/2, M/2).
//
// Residues.  r = X' mod p_m in the symmetric range [-(p-1)/2, (p-1)/2] fits int8; the moduli are
// odd so that -128 never occurs and the packed byte negation below never carries into the next
// byte.  Per modulus the product conj(X)^T Y runs on v_mfma_i32_32x32x32_i8 with the complex
// layout of split.hip: lanes 0-31 carry real parts, lanes 32-63 imaginary parts of 16 rows,
// Re = [Xr; Xi]^T [Yr; Yi], Im = [Xr; -Xi]^T [Yi; Yr].  A 16-row step adds at most 32 * 127^2 < 2^19 to an int32
// accumulator; accumulators are reduced mod p every kFlushStages stages of 64 rows, so they stay
// below 2^31.
//
// Reconstruction.  With w_m = (M/p_m)^(-1) mod p_m, C'/M = sum_m y_m / p_m (mod 1) for the
// residues c_m and y_m = c_m w_m mod p_m; the sum is formed in double-double from 1/p_m = hi + lo,
// reduced to (-1/2, 1/2] and multiplied by M (also double-double).  Then C = C' 2^-(e_i + e_j).
//
// Kernels:
//   mod_colnorm_kernel  per column: e_c of P, of d.P (right operand of S) and of Q (right of H)
//   mod_colsum_kernel   the same e_c from column-sum shares written by the real-T panel kernel
//   mod_slice_kernel    residues of all moduli, stored as [modulus][32-column block][16-row chunk]
//                       [re, im][32 columns][16 bytes] (one 1 KB MFMA fragment per chunk)
//   hs_mod_i8_kernel    one block per (256 x 128 output block, modulus): eight waves of 64 x 64,
//                       stages of 64 rows copied to LDS by global_load_lds into a ring of three
//                       buffers (two stages in flight); fragments of the next 16-row chunk read
//                       ahead of the MFMAs; writes the residues (int8, 32 KB per 128 x 128 tile)
//                       to the problem's scratch
//   mod_crt_kernel      one block per tile: reads the residues of all moduli, rebuilds and
//                       scales the FP64 values, writes the upper triangle of S or H
#include <cmath>

#include "context.hpp"

namespace flapw {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kChunks = 4;                // 16-row chunks per LDS stage
constexpr int kStageRows = 16 * kChunks;  // complex rows per LDS stage
constexpr int kRunBytes = kChunks * 1024; // one 32-column block over one stage
constexpr int kStageBytes = 12 * kRunBytes;  // 8 left + 4 right column blocks
constexpr int kRing = 3;                  // LDS stage buffers (s_waitcnt immediates use the gfx9
                                          // encoding: vmcnt bits 3:0, expcnt 6:4, lgkmcnt 11:8)
constexpr int kCopies = 12 * kChunks / 8; // 1 KB copies per wave per stage
static_assert(kChunks % 2 == 0 && kRing >= 2 && kRing <= 4 && (kRing - 2) * kCopies < 16, "stage ring");
constexpr int kFlushStages = 32768 / kStageRows;  // 32768 rows * 2 * 127^2 < 2^31
constexpr int kResTileBytes = kModTile * kModTile * 2;  // int8 residues of Re and Im

// x mod p in [-(p-1)/2, (p-1)/2] for odd p, ip = fl(1/p) and integer-valued |x| <= 2^50 (1 + 2^-15).
// x/p lies at least 1/(2p) from the nearest half-integer (x is an integer and p is odd), and the
// two roundings in fl(x ip) move it by at most about |x|/p 2^-52 <= 1.0001/(4p), so rint returns the nearest
// quotient, the remainder from the fma is exact and already in the symmetric range.
__device__ inline int sym_mod(double x, double p, double ip)
{
    const double q = rint(x * ip);
    return (int)fma(-q, p, x);
}

// int32 reduction mod odd p in 32-bit arithmetic.  One step leaves |r| <= 3p for any int32 x
// (the float quotient is off by at most 2); a second step on such r is exact and lands in
// [-(p-1)/2, (p-1)/2] (r/p is never a half-integer for odd p).
__device__ inline int mod_step(int x, int p, float ipf)
{
    const int q = (int)rintf((float)x * ipf);
    return x - q * p;
}

__device__ inline int mod_exponent(double ss, int bits)
{
    if (!(ss > 0.0)) return 0;
    int E;
    (void)frexp(sqrt(ss), &E);                // norm < 2^E
    return bits - E;
}

__global__ __launch_bounds__(256) void mod_colnorm_kernel(const double2 *__restrict__ P, const double2 *__restrict__ Q,
                                                          const double *__restrict__ d, long long ld, int kp2, int np,
                                                          int bits, int *__restrict__ eL, int *__restrict__ eRS,
                                                          int *__restrict__ eRH)
{
    __shared__ double red[3][256];
    const long long c = blockIdx.x;
    double sp = 0.0, sd = 0.0, sq = 0.0;
    if (c < np) {
        const double2 *pc = P + c * ld, *qc = Q + c * ld;
        for (int r = threadIdx.x; r < kp2; r += 256) {
            const double2 p = pc[r], q = qc[r];
            const double a = p.x * p.x + p.y * p.y, w = d[r];
            sp += a;
            sd += a * w * w;
            sq += q.x * q.x + q.y * q.y;
        }
    }
    red[0][threadIdx.x] = sp;
    red[1][threadIdx.x] = sd;
    red[2][threadIdx.x] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        eL[c] = mod_exponent(red[0][0], bits);
        eRS[c] = mod_exponent(red[1][0], bits);
        eRH[c] = mod_exponent(red[2][0], bits);
    }
}

// The same exponents from the column-sum shares that the real-T panel kernel wrote while forming
// Q: part[(k n_slots + slot) np + c], k = 0, 1, 2 for sum |P|^2, sum |P|^2 d^2, sum |Q|^2, summed
// over the slots in order (one thread per column, reads coalesced across columns).
__global__ __launch_bounds__(256) void mod_colsum_kernel(const double *__restrict__ part, long long n_slots,
                                                         long long np, int npm, int bits, int *__restrict__ eL,
                                                         int *__restrict__ eRS, int *__restrict__ eRH)
{
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= npm) return;
    double sp = 0.0, sd = 0.0, sq = 0.0;
    if (c < np) {
        for (long long t = 0; t < n_slots; ++t) {
            sp += part[t * np + c];
            sd += part[(n_slots + t) * np + c];
            sq += part[(2 * n_slots + t) * np + c];
        }
    }
    eL[c] = mod_exponent(sp, bits);
    eRS[c] = mod_exponent(sd, bits);
    eRH[c] = mod_exponent(sq, bits);
}

// residues of 16 integer-valued doubles for every modulus, 16 bytes per modulus at out + m * mstride
__device__ inline void write_residues(const double (&v)[16], const ModTable &mt, int8_t *out, long long mstride)
{
    for (int m = 0; m < mt.nm; ++m) {
        const double p = (double)mt.p[m], ip = mt.inv_p[m];
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned packed = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) packed |= ((unsigned)sym_mod(v[4 * q + b], p, ip) & 0xffu) << (8 * b);
            w[q] = packed;
        }
        *reinterpret_cast<uint4 *>(out + m * mstride) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// grid (npm/32, kp2/128): thread (m = tid % 32, chunk = tid / 32) handles 16 rows of column
// 32 blockIdx.x + m.  MODE 0: residues of P (left) and d.P (right of S); MODE 1: of Q (right of H);
// MODE 2: of P alone (S is not contracted).  The 16 values are read once and each operand (its real
// parts, then its imaginary parts) is formed and reduced in turn, so that one operand's 16 integers
// are live beside them.
template <int MODE>
__global__ __launch_bounds__(256) void mod_slice_kernel(const double2 *__restrict__ P, const double2 *__restrict__ Q,
                                                        const double *__restrict__ d, long long ld, int kp2, int np,
                                                        ModTable mt, const int *__restrict__ eL,
                                                        const int *__restrict__ eRS, const int *__restrict__ eRH,
                                                        int8_t *__restrict__ L, int8_t *__restrict__ RS,
                                                        int8_t *__restrict__ RH)
{
    const int m = threadIdx.x & 31;
    const long long cb = blockIdx.x, col = cb * 32 + m;
    const long long ch = (long long)blockIdx.y * 8 + (threadIdx.x >> 5);
    const long long nch = kp2 / 16, ncb = gridDim.x;
    const long long mstride = ncb * nch * 1024;
    const long long off = (cb * nch + ch) * 1024 + m * 16;
    const long long r0 = ch * 16;
    double xr[16];
    if (MODE == 2) {
        const int ex = eL[col];
        double2 v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = col < np ? P[col * ld + r0 + r] : make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].x, ex));
        write_residues(xr, mt, L + off, mstride);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].y, ex));
        write_residues(xr, mt, L + off + 512, mstride);
    } else if (MODE == 0) {
        // P is read once; the four operands (Re P, Im P, Re d.P, Im d.P) are formed and reduced one
        // at a time, so only the 16 values of P and one operand are live
        const int e1 = eL[col], e2 = eRS[col];
        double2 v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = col < np ? P[col * ld + r0 + r] : make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].x, e1));
        write_residues(xr, mt, L + off, mstride);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].y, e1));
        write_residues(xr, mt, L + off + 512, mstride);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].x * d[r0 + r], e2));
        write_residues(xr, mt, RS + off, mstride);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].y * d[r0 + r], e2));
        write_residues(xr, mt, RS + off + 512, mstride);
    } else {
        const int ex = eRH[col];
        double2 v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = col < np ? Q[col * ld + r0 + r] : make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].x, ex));
        write_residues(xr, mt, RH + off, mstride);
#pragma unroll
        for (int r = 0; r < 16; ++r) xr[r] = rint(ldexp(v[r].y, ex));
        write_residues(xr, mt, RH + off + 512, mstride);
    }
}

// Two's-complement negation of the four bytes of x where the masks are set (lanes 32-63); exact
// for bytes in [-127, 127] (no carry leaves a byte).
__device__ __forceinline__ int neg_bytes(int x, unsigned m7f, unsigned m01, unsigned m80)
{
    return (int)((((unsigned)x ^ m7f) + m01) ^ m80);
}

__device__ inline int tri_index(int ti, int tj) { return tj * (tj + 1) / 2 + ti; }

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

// ring_barrier with `later` younger stages allowed in flight (kCopies copies each per wave)
__device__ inline void ring_wait(int later)
{
    if (later <= 0) ring_barrier<0>();
    else if (later == 1) ring_barrier<kCopies>();
    else ring_barrier<2 * kCopies>();
}

// grid (n_tiles, nm): block tile blockIdx.x of the launch's list -- rows 256 I .. 256 I + 255
// (the 128-row tiles 2I and 2I + 1), columns 128 J .. 128 J + 127 -- and modulus blockIdx.y.
// Eight waves, wave w computing rows 64 (w >> 1) and columns 64 (w & 1) of the block tile.
__global__ __launch_bounds__(512, 1) void hs_mod_i8_kernel(const ModProblemDev *__restrict__ probs,
                                                           const TileDev *__restrict__ tiles, ModTable mt)
{
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
    ring_wait(min(kRing - 2, nst - 1));

    const int half = lane >> 5, col = lane & 31;
    const unsigned m7f = half ? 0x7f7f7f7fu : 0u, m01 = half ? 0x01010101u : 0u, m80 = half ? 0x80808080u : 0u;
    int b = 0;                                    // ring slot of stage st
    for (int st0 = 0; st0 < nst; st0 += kFlushStages) {
        const int st1 = min(nst, st0 + kFlushStages);
        for (int st = st0; st < st1; ++st) {
            // slot of stage st + kRing - 1, the one read last at stage st - 1
            const int bn = b == 0 ? kRing - 1 : b - 1;
            if (st + kRing - 1 < nst) MOD_COPY(st + kRing - 1, bn);
            const unsigned char *stage = smem + b * kStageBytes;
            const unsigned char *la = stage + (2 * wm) * kRunBytes + col * 16;
            const unsigned char *lb = stage + (8 + 2 * wn) * kRunBytes + col * 16;
            v4i a[2], bb[2], bs[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const v4i *>(la + i * kRunBytes + half * 512);
                bb[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes + half * 512);
                bs[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes + (1 - half) * 512);
            }
#pragma unroll
            for (int kk = 0; kk < kChunks; ++kk) {
                v4i na[2], nbb[2], nbs[2];
                if (kk + 1 < kChunks) {          // next chunk's fragments, read ahead
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        na[i] = *reinterpret_cast<const v4i *>(la + i * kRunBytes + (kk + 1) * 1024 + half * 512);
                        nbb[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes + (kk + 1) * 1024 + half * 512);
                        nbs[i] = *reinterpret_cast<const v4i *>(lb + i * kRunBytes + (kk + 1) * 1024 + (1 - half) * 512);
                    }
                }
                // keep the reads ahead of this chunk's products (the scheduler would sink them)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], bb[j], acc[i][j][0], 0, 0, 0);
                v4i an[2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) an[i][q] = neg_bytes(a[i][q], m7f, m01, m80);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(an[i], bs[j], acc[i][j][1], 0, 0, 0);
                if (kk + 1 < kChunks) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        a[i] = na[i];
                        bb[i] = nbb[i];
                        bs[i] = nbs[i];
                    }
                }
            }
            // stage st + 1 must have landed before anyone reads it; later stages may still fly
            if (st + 1 < nst) ring_wait(min(kRing - 2, nst - st - 2));
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

// C'/M mod 1 from residues (double-double), times M, as one double.  y_m = c_m w_m mod p_m is
// formed exactly first, so the running sum of y_m / p_m stays below NM / 2 in magnitude.  FMA
// contraction is off here: fusing a product into the two-sum would drop its rounding error.
template <int NM>
__device__ inline double crt_value(const int (&c)[NM], const ModTable &mt)
{
#pragma clang fp contract(off)
    double fh = 0.0, fl = 0.0;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        const double p = (double)mt.p[m], ip = mt.inv_p[m];
        const double t = (double)(c[m] * mt.w[m]);        // exact, |t| < 2^15
        const double y = t - p * rint(t * ip);             // exact, |y| <= (p + 1) / 2
        const double ph = y * ip;
        double pe = fma(y, ip, -ph);
        pe = fma(y, mt.inv_p_lo[m], pe);
        const double s = fh + ph, bv = s - fh;
        const double er = (fh - (s - bv)) + (ph - bv);
        fh = s;
        fl += er + pe;
    }
    fh -= rint(fh);
    const double s = fh + fl;
    fl = fl - (s - fh);
    fh = s;
    const double ch = fh * mt.M_hi;
    double ce = fma(fh, mt.M_hi, -ch);
    ce = fma(fh, mt.M_lo, ce);
    ce = fma(fl, mt.M_hi, ce);
    return ch + ce;
}

// grid n_tiles (the contraction's list), 256 threads with the contraction's lane mapping.
template <int NM>
__global__ __launch_bounds__(256) void mod_crt_kernel(const ModProblemDev *__restrict__ probs,
                                                      const TileDev *__restrict__ tiles, ModTable mt)
{
    const TileDev td = tiles[blockIdx.x];
    const ModProblemDev pb = probs[td.prob];
    const int mat = td.pad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int slot = mat * pb.ntri + tri_index(td.ti, td.tj);
    const int *eR = mat ? pb.eRH : pb.eRS;
    double2 *outm = mat ? pb.H : pb.S;
    const long long tstride = 2LL * pb.ntri * kResTileBytes;
    const int8_t *res = pb.res + (long long)slot * kResTileBytes;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const long long cj = (long long)td.tj * kModTile + wn * 64 + j * 32 + (lane & 31);
            const long long ibase = (long long)td.ti * kModTile + wm * 64 + i * 32;
            if (ibase > cj || cj >= pb.n) continue;
            uint4 rre[NM], rim[NM];
            const int gre = ((wave * 2 + i) * 2 + j) * 2;
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                rre[m] = *reinterpret_cast<const uint4 *>(res + m * tstride + ((long long)gre * 64 + lane) * 16);
                rim[m] = *reinterpret_cast<const uint4 *>(res + m * tstride + ((long long)(gre + 1) * 64 + lane) * 16);
            }
            const int ec = eR[cj];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const long long ri = ibase + (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
                if (ri > cj) continue;
                int cre[NM], cim[NM];
                const int sh = 8 * (r & 3);
#pragma unroll
                for (int m = 0; m < NM; ++m) {
                    const unsigned wr = (r >> 2) == 0 ? rre[m].x : (r >> 2) == 1 ? rre[m].y : (r >> 2) == 2 ? rre[m].z : rre[m].w;
                    const unsigned wi = (r >> 2) == 0 ? rim[m].x : (r >> 2) == 1 ? rim[m].y : (r >> 2) == 2 ? rim[m].z : rim[m].w;
                    cre[m] = (int)(signed char)((wr >> sh) & 0xffu);
                    cim[m] = (int)(signed char)((wi >> sh) & 0xffu);
                }
                const int sc = -(pb.eL[ri] + ec);
                const double vr = ldexp(crt_value(cre, mt), sc);
                const double vi = ri == cj ? 0.0 : ldexp(crt_value(cim, mt), sc);
                outm[cj * pb.ldh + ri] = make_double2(vr, vi);
            }
        }
}

}  // namespace

hipError_t init_mod_kernels()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    done = hipFuncSetAttribute((const void *)hs_mod_i8_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kRing * kStageBytes);
    return done;
}

long long mod_digit_bytes(long long kp2, long long npm, int nm) { return 2LL * nm * kp2 * npm; }

long long mod_scratch_bytes(long long npm, int nm)
{
    const long long t = npm / kModTile;
    return 2LL * (t * (t + 1) / 2) * nm * kResTileBytes;
}

hipError_t launch_mod_slice(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                            int npm, const ModTable &mt, int *eL, int *eRS, int *eRH, int8_t *L, int8_t *RS,
                            int8_t *RH, bool with_s, const double *part, long long n_slots, hipStream_t s)
{
    if (part)
        hipLaunchKernelGGL(mod_colsum_kernel, dim3((npm + 255) / 256), dim3(256), 0, s, part, n_slots, (long long)np, npm,
                           mt.bits, eL, eRS, eRH);
    else
        hipLaunchKernelGGL(mod_colnorm_kernel, dim3(npm), dim3(256), 0, s, P, Q, d, ld, kp2, np, mt.bits, eL, eRS, eRH);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(npm / 32, kp2 / 128);
    if (with_s)
        hipLaunchKernelGGL(mod_slice_kernel<0>, grid, dim3(256), 0, s, P, Q, d, ld, kp2, np, mt, eL, eRS, eRH, L, RS, RH);
    else
        hipLaunchKernelGGL(mod_slice_kernel<2>, grid, dim3(256), 0, s, P, Q, d, ld, kp2, np, mt, eL, eRS, eRH, L, RS, RH);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mod_slice_kernel<1>, grid, dim3(256), 0, s, P, Q, d, ld, kp2, np, mt, eL, eRS, eRH, L, RS, RH);
    return hipGetLastError();
}

hipError_t launch_mod_contract(const ModProblemDev *probs, const TileDev *tiles, int n_tiles, const ModTable &mt,
                               hipStream_t s)
{
    static_assert(kRing * kStageBytes <= 163840, "LDS budget");
    hipError_t e = init_mod_kernels();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hs_mod_i8_kernel, dim3(n_tiles, mt.nm), dim3(512), kRing * kStageBytes, s, probs, tiles, mt);
    return hipGetLastError();
}

hipError_t launch_mod_crt(const ModProblemDev *probs, const TileDev *tiles, int n_tiles, const ModTable &mt,
                          hipStream_t s)
{
    switch (mt.nm) {
#define CASE(N) case N: hipLaunchKernelGGL(mod_crt_kernel<N>, dim3(n_tiles), dim3(256), 0, s, probs, tiles, mt); break;
        CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Moduli: the pairwise coprime odd integers taken greedily from 255 downwards; B from M.
ModTable make_mod_table(int nm)
{
    ModTable t{};
    t.nm = nm;
    int c = 255, k = 0;
    while (k < nm) {
        bool ok = true;
        for (int j = 0; j < k; ++j) {
            int a = c, b = t.p[j];
            while (b) { const int r = a % b; a = b; b = r; }
            if (a != 1) { ok = false; break; }
        }
        if (ok) t.p[k++] = c;
        c -= 2;
    }
    unsigned __int128 M = 1;
    double lg = 0.0;
    for (int m = 0; m < nm; ++m) {
        M *= (unsigned)t.p[m];
        lg += std::log2((double)t.p[m]);
    }
    t.bits = std::min(50, (int)std::floor((lg - 1.0) / 2.0));
    for (int m = 0; m < nm; ++m) {
        const long long p = t.p[m];
        long long q = 1;                                   // (M / p) mod p
        for (int j = 0; j < nm; ++j)
            if (j != m) q = q * t.p[j] % p;
        long long r0 = p, r1 = q, s0 = 0, s1 = 1;          // inverse of q mod p
        while (r1) {
            const long long f = r0 / r1, r2 = r0 - f * r1, s2 = s0 - f * s1;
            r0 = r1; r1 = r2; s0 = s1; s1 = s2;
        }
        t.w[m] = (int)(((s0 % p) + p) % p);
        t.inv_p[m] = 1.0 / (double)p;
        t.inv_p_lo[m] = std::fma(-t.inv_p[m], (double)p, 1.0) / (double)p;
    }
    t.M_hi = (double)M;
    const __int128 rest = (__int128)M - (__int128)t.M_hi;
    t.M_lo = (double)rest;
    return t;
}

}  // namespace flapw
