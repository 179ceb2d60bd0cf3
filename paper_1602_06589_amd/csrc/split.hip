// Split-precision S/H contraction: FP64 operands are cut into int8 digits, digit products run on
// the int8 matrix cores with exact int32 accumulation, and the digit groups are recombined and
// summed over atoms in FP64.  (The paper computes everything in FP64 BLAS; this stage replaces
// its big zherk/zher2k/zgemm updates, sections 4.2-4.6.)
//
// Digits.  Every operand column c (a basis function) gets one power-of-two scale 2^e_c over the
// whole contraction index: with a_c the largest |Re| or |Im| in the column, e_c is chosen so that
// v = x 2^(7 - e_c) lies in (-127.5, 127.5).  Then
//     d_0 = rint(v),  r_1 = v - d_0,  d_p = rint(128 r_p),  r_{p+1} = 128 r_p - d_p,
// so |d_0| <= 127, |d_p| <= 64 for p >= 1, every step is exact in FP64, and
//     x = 2^e_c sum_p d_p 2^(-7(p+1)) + O(2^(e_c - 7s)).
// A product conj(X_ki) Y_kj then splits into digit pairs (p, q) with weight 2^(eX_i + eY_j - 7(p+q+2));
// pairs with p + q <= s-1 are kept (triangular truncation, s(s+1)/2 pair products).
//
// Complex products on int8 MFMA.  v_mfma_i32_32x32x32_i8 takes 16 bytes of k per lane, k = 16 (l/32) + j.
// One k-step covers 16 complex rows: lanes 0-31 carry the real digits, lanes 32-63 the imaginary ones:
//   Re conj(X)Y = [Xr; Xi]^T [Yr; Yi],   Im conj(X)Y = [Xr; -Xi]^T [Yi; Yr],
// so each of Re and Im is a single MFMA; -Xi is formed in registers (lanes 32-63 of the A fragment).
//
// Digit storage ("fragment order"): operand digits are [col block of 32][16-row chunk][digit p]
// [half: re, im][32 columns][16 bytes], so one 512-byte half-fragment is exactly what 32 lanes
// read, global loads are contiguous, and LDS reads (lane l at 16 (l % 32)) are conflict-free.
//
// Exactness.  An int32 group accumulator receives at most 6 pairs x 2 products x 4096 rows x
// 127^2 < 2^31 between flushes; it is flushed to FP64 (times 2^(-7(g+2))) every 128 stages of
// 32 rows and at the end, so the digit products are exact and only the FP64 sums round.
#include "context.hpp"

namespace flapw {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

#if defined(__HIP_DEVICE_COMPILE__)
typedef const double2 __attribute__((address_space(1))) gdouble2;
typedef const double __attribute__((address_space(1))) gdouble;
typedef const v4i __attribute__((address_space(1))) gv4i;
#else
typedef const double2 gdouble2;
typedef const double gdouble;
typedef const v4i gv4i;
#endif

constexpr int kRowsPerChunk = 16;         // complex rows per MFMA k-step
constexpr int kChunksPerStage = 2;        // 32 complex rows per LDS stage
constexpr int kFlushStages = 128;         // int32 -> FP64 flush period (4096 rows)

// ----------------------------------------------------------------------------- slicing

// Column scale exponent: the smallest e with max|x| 2^(7-e) < 127.5 (0 for an all-zero column).
__device__ inline int digit_exponent(double a)
{
    if (!(a > 0.0)) return 0;
    int E;
    const double f = frexp(a, &E);            // a = f 2^E, f in [0.5, 1)
    return (128.0 * f >= 127.5) ? E + 1 : E;
}

// Per column: exponents of P (left operand), of d.P (right operand of S) and of Q (right of H).
__global__ __launch_bounds__(256) void colmax_kernel(const double2 *__restrict__ P, const double2 *__restrict__ Q,
                                                     const double *__restrict__ d, long long ld, int kp2,
                                                     int *__restrict__ eL, int *__restrict__ eRS,
                                                     int *__restrict__ eRH)
{
    __shared__ double red[3][256];
    const long long c = blockIdx.x;
    gdouble2 *pc = (gdouble2 *)P + c * ld;
    gdouble2 *qc = (gdouble2 *)Q + c * ld;
    gdouble *dd = (gdouble *)d;
    double mp = 0.0, md = 0.0, mq = 0.0;
    for (int r = threadIdx.x; r < kp2; r += 256) {
        const double2 p = pc[r], q = qc[r];
        const double a = fmax(fabs(p.x), fabs(p.y));
        mp = fmax(mp, a);
        md = fmax(md, a * dd[r]);
        mq = fmax(mq, fmax(fabs(q.x), fabs(q.y)));
    }
    red[0][threadIdx.x] = mp;
    red[1][threadIdx.x] = md;
    red[2][threadIdx.x] = mq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        eL[c] = digit_exponent(red[0][0]);
        eRS[c] = digit_exponent(red[1][0]);
        eRH[c] = digit_exponent(red[2][0]);
    }
}

// 16 values -> S digit records of 16 bytes, written to out[p * 2 * 512] (stride between digits).
template <int S>
__device__ inline void write_digits(double (&v)[16], int8_t *out, long long digit_stride)
{
#pragma unroll
    for (int p = 0; p < S; ++p) {
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned packed = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double &x = v[4 * q + b];
                const double dg = rint(x);
                x = (x - dg) * 128.0;
                packed |= ((unsigned)(int)dg & 0xffu) << (8 * b);
            }
            w[q] = packed;
        }
        *reinterpret_cast<uint4 *>(out + p * digit_stride) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// grid (np/32, kp2/128): thread (m = tid%32, chunk = tid/32) cuts 16 rows of column 32 cb + m.
// MODE 0: from P, write the left digits (P) and the S right digits (d.P); MODE 1: from Q.
template <int S, int MODE>
__global__ __launch_bounds__(256) void digits_kernel(const double2 *__restrict__ M, const double *__restrict__ d,
                                                     long long ld, int nkc, const int *__restrict__ e0,
                                                     const int *__restrict__ e1, int8_t *__restrict__ out0,
                                                     int8_t *__restrict__ out1)
{
    const int m = threadIdx.x & 31;
    const long long cb = blockIdx.x;
    const long long kc = (long long)blockIdx.y * 8 + (threadIdx.x >> 5);
    if (kc >= nkc) return;
    const long long col = cb * 32 + m;
    gdouble2 *src = (gdouble2 *)M + col * ld + kc * kRowsPerChunk;
    double2 x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = src[r];
    // record of (cb, kc, p, half, m): ((((cb nkc + kc) S + p) 2 + half) 32 + m) 16 bytes
    const long long rec = ((cb * nkc + kc) * S * 2 * 32 + m) * 16;
    const long long dstride = 2 * 32 * 16;            // between digits p
    const long long hstride = 32 * 16;                // between halves
    {
        const double sc = ldexp(1.0, 7 - e0[col]);
        double v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = x[r].x * sc;
        write_digits<S>(v, out0 + rec, dstride);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = x[r].y * sc;
        write_digits<S>(v, out0 + rec + hstride, dstride);
    }
    if (MODE == 0) {
        gdouble *dd = (gdouble *)d + kc * kRowsPerChunk;
        const double sc = ldexp(1.0, 7 - e1[col]);
        double v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = x[r].x * dd[r] * sc;
        write_digits<S>(v, out1 + rec, dstride);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = x[r].y * dd[r] * sc;
        write_digits<S>(v, out1 + rec + hstride, dstride);
    }
}

// ----------------------------------------------------------------------------- contraction

// Negation of the imaginary half of an A fragment (lanes 32-63), per signed byte with no byte
// equal to -128: -x = ((x ^ 0x7f) + 1) ^ 0x80.  x ^ 0x7f <= 0xfe, so the +1 never carries into
// the next byte.  With the three constants masked to zero on lanes 0-31 the same three
// instructions leave those lanes unchanged.
__device__ __forceinline__ int neg_lanes(int x, unsigned m7f, unsigned m01, unsigned m80)
{
    return (int)((((unsigned)x ^ m7f) + m01) ^ m80);
}

template <int S>
struct SplitSmem {
    static constexpr int kRunBytes = kChunksPerStage * S * 2 * 512;   // one 32-column block, one stage
    static constexpr int kStageBytes = 4 * kRunBytes;                 // 2 left + 2 right column blocks
    static constexpr int kAccBytes = 4 * 32 * 64 * 8;                 // FP64 sums: [wave][re 16, im 16][lane]
    static constexpr int kBytes = 2 * kStageBytes + kAccBytes;
};

// 64 x 64 tile of S (pad = 0) or H (pad = 1); 4 waves, each a 32 x 32 block; 32 complex rows per
// LDS stage (double-buffered); all s digit groups accumulate in int32 registers and are flushed
// to FP64 sums kept in LDS.
template <int S>
__global__ __launch_bounds__(256, 1) void hs_split_i8_kernel(const SplitProblemDev *__restrict__ probs,
                                                             const TileDev *__restrict__ tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using SM = SplitSmem<S>;
    constexpr int kRunSegs = SM::kRunBytes / 1024;                // 1 KB segments of one run (2 S)
    constexpr int kSegsPerWave = kRunSegs;                        // a stage is 4 runs, spread over 4 waves

    const TileDev td = tiles[blockIdx.x];
    const SplitProblemDev pb = probs[td.prob];
    const int mat = td.pad;                                      // 0: S, 1: H
    const int8_t *R = (const int8_t *)(mat ? pb.RQ : pb.R);
    const int *eR = mat ? pb.eRQ : pb.eR;
    double2 *out = mat ? pb.H : pb.S;
    const int8_t *Lg = (const int8_t *)pb.L;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wmb = wave >> 1, wnb = wave & 1;                   // 32 x 32 block of this wave
    const long long nkc = pb.kp2 / kRowsPerChunk;
    const int nst = (int)(nkc / kChunksPerStage);
    const long long chunk_bytes = (long long)S * 2 * 512;        // one (column block, 16-row chunk)
    const long long stage_step = kChunksPerStage * chunk_bytes;  // global advance per stage
    // run bases: left column blocks 2 ti, 2 ti + 1; right column blocks 2 tj, 2 tj + 1
    const int8_t *run_base[4] = {Lg + (2LL * td.ti) * nkc * chunk_bytes, Lg + (2LL * td.ti + 1) * nkc * chunk_bytes,
                                 R + (2LL * td.tj) * nkc * chunk_bytes, R + (2LL * td.tj + 1) * nkc * chunk_bytes};
    double *facc = reinterpret_cast<double *>(smem_raw + 2 * SM::kStageBytes) + wave * 32 * 64 + lane;

    v16i acc_re[S], acc_im[S];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
        for (int r = 0; r < 16; ++r) { acc_re[g][r] = 0; acc_im[g][r] = 0; }
#pragma unroll
    for (int r = 0; r < 32; ++r) facc[r * 64] = 0.0;

    // Stages are copied global -> LDS by the load unit itself (global_load_lds_dwordx4): one
    // instruction moves a contiguous 1 KB segment, lane l's 16 bytes landing at +16 l.  No
    // registers hold staged data; the copies of stage st + 1 are issued at the start of stage st
    // and complete by the barrier that ends it (the barrier waits for all outstanding loads).
#define SPLIT_COPY(st, b)                                                                       \
    do {                                                                                        \
        _Pragma("unroll") for (int j_ = 0; j_ < kSegsPerWave; ++j_) {                              \
            const int sg_ = wave + 4 * j_, run_ = sg_ / kRunSegs, off_ = (sg_ % kRunSegs) * 1024; \
            const int8_t *src_ = run_base[run_] + (long long)(st) * stage_step + off_ + lane * 16; \
            __builtin_amdgcn_global_load_lds((const int __attribute__((address_space(1))) *)src_, \
                (int __attribute__((address_space(3))) *)(smem_raw + (b) * SM::kStageBytes + sg_ * 1024), 16, 0, 0); \
        }                                                                                       \
    } while (0)

    SPLIT_COPY(0, 0);
    __syncthreads();

    const int half_a = lane >> 5, col = lane & 31;
    // lanes 32-63 carry Xi and negate it for the Im products
    const unsigned m7f = half_a ? 0x7f7f7f7fu : 0u, m01 = half_a ? 0x01010101u : 0u, m80 = half_a ? 0x80808080u : 0u;
    // Outer loop over flush periods, inner loop over stages: the int32 accumulators stay in the
    // matrix-core registers for a whole period and are read only by the flush.
    for (int st0 = 0; st0 < nst; st0 += kFlushStages) {
        const int st1 = min(nst, st0 + kFlushStages);
        for (int st = st0; st < st1; ++st) {
            const int b = st & 1;
            if (st + 1 < nst) SPLIT_COPY(st + 1, b ^ 1);
            const unsigned char *stage = smem_raw + b * SM::kStageBytes;
#pragma unroll 1
            for (int kk = 0; kk < kChunksPerStage; ++kk) {
                const unsigned char *lrun = stage + wmb * SM::kRunBytes + kk * S * 1024 + half_a * 512 + col * 16;
                const unsigned char *rrun = stage + (2 + wnb) * SM::kRunBytes + kk * S * 1024 + col * 16;
                // all A reads and the first B pair issued back to back
                v4i a_re[S], a_im[S];
#pragma unroll
                for (int p = 0; p < S; ++p) a_re[p] = *reinterpret_cast<const v4i *>(lrun + p * 1024);
                v4i b_re = *reinterpret_cast<const v4i *>(rrun + half_a * 512);
                v4i b_im = *reinterpret_cast<const v4i *>(rrun + (1 - half_a) * 512);
#pragma unroll
                for (int p = 0; p < S; ++p)
#pragma unroll
                    for (int i = 0; i < 4; ++i) a_im[p][i] = neg_lanes(a_re[p][i], m7f, m01, m80);
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    v4i nb_re = b_re, nb_im = b_im;
                    if (q + 1 < S) {                 // B fragments of the next q, read ahead
                        nb_re = *reinterpret_cast<const v4i *>(rrun + (q + 1) * 1024 + half_a * 512);
                        nb_im = *reinterpret_cast<const v4i *>(rrun + (q + 1) * 1024 + (1 - half_a) * 512);
                    }
                    // Re products first: they do not wait for the negated fragments
#pragma unroll
                    for (int p = 0; p + q < S; ++p)
                        acc_re[p + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_re[p], b_re, acc_re[p + q], 0, 0, 0);
#pragma unroll
                    for (int p = 0; p + q < S; ++p)
                        acc_im[p + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_im[p], b_im, acc_im[p + q], 0, 0, 0);
                    b_re = nb_re;
                    b_im = nb_im;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int g = 0; g < S; ++g) {
                const double w = ldexp(1.0, -7 * (g + 2));
                sr += w * (double)acc_re[g][r];
                si += w * (double)acc_im[g][r];
                acc_re[g][r] = 0;
                acc_im[g][r] = 0;
            }
            facc[r * 64] += sr;
            facc[(16 + r) * 64] += si;
        }
    }
#undef SPLIT_COPY

    // epilogue: scale by 2^(eL_row + eR_col); upper triangle; diagonal imaginary part zero
    const long long i0 = (long long)td.ti * 64 + wmb * 32, j0 = (long long)td.tj * 64 + wnb * 32;
    const long long cj = j0 + col;
    const int ec = eR[cj];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const long long ri = i0 + (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
        if (ri <= cj && cj < pb.n) {
            const double sc = ldexp(1.0, pb.eL[ri] + ec);
            out[cj * pb.ldh + ri] = make_double2(facc[r * 64] * sc, ri == cj ? 0.0 : facc[(16 + r) * 64] * sc);
        }
    }
}

template <int S>
hipError_t init_split_s()
{
    return hipFuncSetAttribute((const void *)hs_split_i8_kernel<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               SplitSmem<S>::kBytes);
}

template <int S>
hipError_t launch_split_s(const SplitProblemDev *probs, const TileDev *tiles, int n_tiles, hipStream_t s)
{
    constexpr int smem = SplitSmem<S>::kBytes;
    static_assert(smem <= 163840, "LDS budget");
    hipError_t e = init_split_kernels();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hs_split_i8_kernel<S>, dim3(n_tiles), dim3(256), smem, s, probs, tiles);
    return hipGetLastError();
}

template <int S>
hipError_t launch_digits_s(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                           const int *eL, const int *eRS, const int *eRH, int8_t *L, int8_t *RS, int8_t *RH,
                           hipStream_t s)
{
    const int nkc = kp2 / kRowsPerChunk;
    dim3 grid(np / 32, (nkc + 7) / 8);
    hipLaunchKernelGGL((digits_kernel<S, 0>), grid, dim3(256), 0, s, P, d, ld, nkc, eL, eRS, L, RS);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((digits_kernel<S, 1>), grid, dim3(256), 0, s, Q, d, ld, nkc, eRH, eRH, RH, RH);
    return hipGetLastError();
}

}  // namespace

long long split_digit_bytes(long long kp2, long long np, int s) { return 3LL * 2 * s * kp2 * np; }

hipError_t init_split_kernels()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    hipError_t e = init_split_s<3>();
    if (e == hipSuccess) e = init_split_s<4>();
    if (e == hipSuccess) e = init_split_s<5>();
    if (e == hipSuccess) e = init_split_s<6>();
    done = e;
    return e;
}

hipError_t launch_split_slice(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                              int slices, int *eL, int *eRS, int *eRH, int8_t *L, int8_t *RS, int8_t *RH,
                              hipStream_t s)
{
    hipLaunchKernelGGL(colmax_kernel, dim3(np), dim3(256), 0, s, P, Q, d, ld, kp2, eL, eRS, eRH);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (slices) {
        case 3: return launch_digits_s<3>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        case 4: return launch_digits_s<4>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        case 5: return launch_digits_s<5>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        case 6: return launch_digits_s<6>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_split_contract(const SplitProblemDev *probs, const TileDev *tiles, int n_tiles, int slices,
                                 hipStream_t s)
{
    switch (slices) {
        case 3: return launch_split_s<3>(probs, tiles, n_tiles, s);
        case 4: return launch_split_s<4>(probs, tiles, n_tiles, s);
        case 5: return launch_split_s<5>(probs, tiles, n_tiles, s);
        case 6: return launch_split_s<6>(probs, tiles, n_tiles, s);
        default: return hipErrorInvalidValue;
    }
}

void split_release(flapw_handle h)
{
    h->digits.release();
    h->sdesc.release();
}

long long split_bytes(flapw_handle h) { return (long long)(h->digits.n + h->sdesc.n); }

}  // namespace flapw
