// Split-precision S/H contraction with bf16 digits on the bf16 matrix cores (the int8 variant is
// in split.hip; this one keeps the same structure with 8-bit digits stored exactly in bf16).
//
// Digits.  Per operand column c one power-of-two scale 2^e_c over the contraction index: with a_c
// the largest |Re| or |Im| in the column, e_c is the smallest e with a_c 2^(8 - e) < 255.5; then
//     v = x 2^(8 - e_c),  d_0 = rint(v),  r_1 = v - d_0,  d_p = rint(256 r_p),  r_{p+1} = 256 r_p - d_p,
// so |d_0| <= 255 and |d_p| <= 128: integers of at most 8 significant bits, exact in bf16, and
//     x = 2^(e_c - 8) sum_p d_p 2^(-8p) + O(2^(e_c - 8s)).
// Pairs (p, q) with p + q <= s - 1 are kept; group g = p + q has weight 2^(eX + eY - 8(g + 2)).
//
// Products.  v_mfma_f32_32x32x16_bf16 takes 8 bf16 of k per lane, k = 8 (l/32) + j: one k-step
// covers 8 complex rows, real digits in lanes 0-31 and imaginary digits in lanes 32-63, so
//   Re conj(X)Y = [Xr; Xi]^T [Yr; Yi],   Im conj(X)Y = [Xr; -Xi]^T [Yi; Yr];
// -Xi flips the bf16 sign bits of lanes 32-63.
//
// Exactness.  Digit products are integers below 2^16 and FP32 adds them exactly while every
// partial sum stays below 2^24 in magnitude.  Per complex row a group accumulator receives at
// most 2 (2 * 255 * 128 + 4 * 128^2) = 261632 in absolute value (s <= 6), so 64 rows
// (16744448 < 2^24) are summed in FP32 and then flushed to FP64 (times 2^(-8(g+2))), whatever
// order the matrix core adds them in.
//
// Storage ("fragment order", as the int8 digits with 8-row chunks): [col block of 32][8-row chunk]
// [digit p][half: re, im][32 columns][16 bytes = 8 bf16].
#include "context.hpp"

namespace flapw {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

#if defined(__HIP_DEVICE_COMPILE__)
typedef const double2 __attribute__((address_space(1))) gdouble2;
typedef const double __attribute__((address_space(1))) gdouble;
#else
typedef const double2 gdouble2;
typedef const double gdouble;
#endif

constexpr int kRows = 8;                  // complex rows per MFMA k-step
constexpr int kChunksPerStage = 2;        // 16 complex rows per LDS stage
constexpr int kFlushStages = 4;           // FP32 -> FP64 flush period (64 rows)

// Column scale exponent: the smallest e with max|x| 2^(8-e) < 255.5 (0 for an all-zero column).
__device__ inline int digit_exponent_bf16(double a)
{
    if (!(a > 0.0)) return 0;
    int E;
    const double f = frexp(a, &E);            // a = f 2^E, f in [0.5, 1)
    return (256.0 * f >= 255.5) ? E + 1 : E;
}

__global__ __launch_bounds__(256) void colmax_bf16_kernel(const double2 *__restrict__ P, const double2 *__restrict__ Q,
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
        eL[c] = digit_exponent_bf16(red[0][0]);
        eRS[c] = digit_exponent_bf16(red[1][0]);
        eRH[c] = digit_exponent_bf16(red[2][0]);
    }
}

// 8 values -> S digit records of 16 bytes (8 bf16), written to out[p * digit_stride].
template <int S>
__device__ inline void write_digits_bf16(double (&v)[8], unsigned char *out, long long digit_stride)
{
#pragma unroll
    for (int p = 0; p < S; ++p) {
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned packed = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                double &x = v[2 * q + b];
                const double dg = rint(x);
                x = (x - dg) * 256.0;
                // |dg| <= 256 has at most 8 significant bits: the float's low 16 bits are zero
                packed |= (__float_as_uint((float)dg) >> 16) << (16 * b);
            }
            w[q] = packed;
        }
        *reinterpret_cast<uint4 *>(out + p * digit_stride) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// grid (np/32, ceil(nkc/8)): thread (m = tid%32, chunk = tid/32) cuts 8 rows of column 32 cb + m.
// MODE 0: from P, the left digits (P) and the S right digits (d.P); MODE 1: from Q.
template <int S, int MODE>
__global__ __launch_bounds__(256) void digits_bf16_kernel(const double2 *__restrict__ M, const double *__restrict__ d,
                                                          long long ld, int nkc, const int *__restrict__ e0,
                                                          const int *__restrict__ e1, unsigned char *__restrict__ out0,
                                                          unsigned char *__restrict__ out1)
{
    const int m = threadIdx.x & 31;
    const long long cb = blockIdx.x;
    const long long kc = (long long)blockIdx.y * 8 + (threadIdx.x >> 5);
    if (kc >= nkc) return;
    const long long col = cb * 32 + m;
    gdouble2 *src = (gdouble2 *)M + col * ld + kc * kRows;
    double2 x[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) x[r] = src[r];
    const long long rec = ((cb * nkc + kc) * S * 2 * 32 + m) * 16;
    const long long dstride = 2 * 32 * 16, hstride = 32 * 16;
    {
        const double sc = ldexp(1.0, 8 - e0[col]);
        double v[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) v[r] = x[r].x * sc;
        write_digits_bf16<S>(v, out0 + rec, dstride);
#pragma unroll
        for (int r = 0; r < kRows; ++r) v[r] = x[r].y * sc;
        write_digits_bf16<S>(v, out0 + rec + hstride, dstride);
    }
    if (MODE == 0) {
        gdouble *dd = (gdouble *)d + kc * kRows;
        const double sc = ldexp(1.0, 8 - e1[col]);
        double v[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) v[r] = x[r].x * dd[r] * sc;
        write_digits_bf16<S>(v, out1 + rec, dstride);
#pragma unroll
        for (int r = 0; r < kRows; ++r) v[r] = x[r].y * dd[r] * sc;
        write_digits_bf16<S>(v, out1 + rec + hstride, dstride);
    }
}

template <int S>
struct SplitBf16Smem {
    static constexpr int kRunBytes = kChunksPerStage * S * 2 * 512;   // one 32-column block, one stage
    static constexpr int kStageBytes = 4 * kRunBytes;                 // 2 left + 2 right column blocks
    static constexpr int kAccBytes = 4 * 32 * 64 * 8;                 // FP64 sums: [wave][re 16, im 16][lane]
    static constexpr int kBytes = 2 * kStageBytes + kAccBytes;
};

__device__ __forceinline__ v16f mfma_bf16(v4i a, v4i b, v16f c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0,
                                                   0);
}

// 64 x 64 tile of S (pad = 0) or H (pad = 1); 4 waves, each a 32 x 32 block; 16 complex rows per
// LDS stage (double-buffered, copied global -> LDS by global_load_lds_dwordx4); the s digit groups
// accumulate in FP32 registers for 64 rows, then in FP64 sums kept in LDS.
template <int S>
__global__ __launch_bounds__(256, 1) void hs_split_bf16_kernel(const SplitProblemDev *__restrict__ probs,
                                                               const TileDev *__restrict__ tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using SM = SplitBf16Smem<S>;
    constexpr int kRunSegs = SM::kRunBytes / 1024;

    const TileDev td = tiles[blockIdx.x];
    const SplitProblemDev pb = probs[td.prob];
    const int mat = td.pad;                                      // 0: S, 1: H
    const unsigned char *R = (const unsigned char *)(mat ? pb.RQ : pb.R);
    const int *eR = mat ? pb.eRQ : pb.eR;
    double2 *out = mat ? pb.H : pb.S;
    const unsigned char *Lg = (const unsigned char *)pb.L;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wmb = wave >> 1, wnb = wave & 1;
    const long long nkc = pb.kp2 / kRows;
    const int nst = (int)(nkc / kChunksPerStage);
    const long long chunk_bytes = (long long)S * 2 * 512;
    const long long stage_step = kChunksPerStage * chunk_bytes;
    const unsigned char *run_base[4] = {Lg + (2LL * td.ti) * nkc * chunk_bytes, Lg + (2LL * td.ti + 1) * nkc * chunk_bytes,
                                        R + (2LL * td.tj) * nkc * chunk_bytes, R + (2LL * td.tj + 1) * nkc * chunk_bytes};
    double *facc = reinterpret_cast<double *>(smem_raw + 2 * SM::kStageBytes) + wave * 32 * 64 + lane;

    v16f acc_re[S], acc_im[S];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
        for (int r = 0; r < 16; ++r) { acc_re[g][r] = 0.0f; acc_im[g][r] = 0.0f; }
#pragma unroll
    for (int r = 0; r < 32; ++r) facc[r * 64] = 0.0;

#define BF_COPY(st, b)                                                                          \
    do {                                                                                        \
        _Pragma("unroll") for (int j_ = 0; j_ < kRunSegs; ++j_) {                                  \
            const int sg_ = wave + 4 * j_, run_ = sg_ / kRunSegs, off_ = (sg_ % kRunSegs) * 1024; \
            const unsigned char *src_ = run_base[run_] + (long long)(st) * stage_step + off_ + lane * 16; \
            __builtin_amdgcn_global_load_lds((const int __attribute__((address_space(1))) *)src_, \
                (int __attribute__((address_space(3))) *)(smem_raw + (b) * SM::kStageBytes + sg_ * 1024), 16, 0, 0); \
        }                                                                                       \
    } while (0)

    BF_COPY(0, 0);
    __syncthreads();

    const int half_a = lane >> 5, col = lane & 31;
    const unsigned sgn = half_a ? 0x80008000u : 0u;              // flips the sign of Xi (lanes 32-63)
    for (int st0 = 0; st0 < nst; st0 += kFlushStages) {
        const int st1 = min(nst, st0 + kFlushStages);
        for (int st = st0; st < st1; ++st) {
            const int b = st & 1;
            if (st + 1 < nst) BF_COPY(st + 1, b ^ 1);
            const unsigned char *stage = smem_raw + b * SM::kStageBytes;
#pragma unroll 1
            for (int kk = 0; kk < kChunksPerStage; ++kk) {
                const unsigned char *lrun = stage + wmb * SM::kRunBytes + kk * S * 1024 + half_a * 512 + col * 16;
                const unsigned char *rrun = stage + (2 + wnb) * SM::kRunBytes + kk * S * 1024 + col * 16;
                v4i a_re[S], a_im[S];
#pragma unroll
                for (int p = 0; p < S; ++p) a_re[p] = *reinterpret_cast<const v4i *>(lrun + p * 1024);
                v4i b_re = *reinterpret_cast<const v4i *>(rrun + half_a * 512);
                v4i b_im = *reinterpret_cast<const v4i *>(rrun + (1 - half_a) * 512);
#pragma unroll
                for (int p = 0; p < S; ++p)
#pragma unroll
                    for (int i = 0; i < 4; ++i) a_im[p][i] = (int)((unsigned)a_re[p][i] ^ sgn);
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    v4i nb_re = b_re, nb_im = b_im;
                    if (q + 1 < S) {
                        nb_re = *reinterpret_cast<const v4i *>(rrun + (q + 1) * 1024 + half_a * 512);
                        nb_im = *reinterpret_cast<const v4i *>(rrun + (q + 1) * 1024 + (1 - half_a) * 512);
                    }
#pragma unroll
                    for (int p = 0; p + q < S; ++p) acc_re[p + q] = mfma_bf16(a_re[p], b_re, acc_re[p + q]);
#pragma unroll
                    for (int p = 0; p + q < S; ++p) acc_im[p + q] = mfma_bf16(a_im[p], b_im, acc_im[p + q]);
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
                const double w = ldexp(1.0, -8 * (g + 2));
                sr += w * (double)acc_re[g][r];
                si += w * (double)acc_im[g][r];
                acc_re[g][r] = 0.0f;
                acc_im[g][r] = 0.0f;
            }
            facc[r * 64] += sr;
            facc[(16 + r) * 64] += si;
        }
    }
#undef BF_COPY

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
hipError_t init_bf16_s()
{
    static_assert(SplitBf16Smem<S>::kBytes <= 163840, "LDS budget");
    return hipFuncSetAttribute((const void *)hs_split_bf16_kernel<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               SplitBf16Smem<S>::kBytes);
}

template <int S>
hipError_t launch_bf16_s(const SplitProblemDev *probs, const TileDev *tiles, int n_tiles, hipStream_t s)
{
    hipError_t e = init_split_bf16_kernels();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hs_split_bf16_kernel<S>, dim3(n_tiles), dim3(256), SplitBf16Smem<S>::kBytes, s, probs, tiles);
    return hipGetLastError();
}

template <int S>
hipError_t launch_digits_bf16_s(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                                const int *eL, const int *eRS, const int *eRH, void *L, void *RS, void *RH,
                                hipStream_t s)
{
    const int nkc = kp2 / kRows;
    dim3 grid(np / 32, (nkc + 7) / 8);
    hipLaunchKernelGGL((digits_bf16_kernel<S, 0>), grid, dim3(256), 0, s, P, d, ld, nkc, eL, eRS,
                       (unsigned char *)L, (unsigned char *)RS);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((digits_bf16_kernel<S, 1>), grid, dim3(256), 0, s, Q, d, ld, nkc, eRH, eRH,
                       (unsigned char *)RH, (unsigned char *)RH);
    return hipGetLastError();
}

}  // namespace

hipError_t init_split_bf16_kernels()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    hipError_t e = init_bf16_s<3>();
    if (e == hipSuccess) e = init_bf16_s<4>();
    if (e == hipSuccess) e = init_bf16_s<5>();
    if (e == hipSuccess) e = init_bf16_s<6>();
    done = e;
    return e;
}

hipError_t launch_split_bf16_slice(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                                   int slices, int *eL, int *eRS, int *eRH, void *L, void *RS, void *RH, hipStream_t s)
{
    hipLaunchKernelGGL(colmax_bf16_kernel, dim3(np), dim3(256), 0, s, P, Q, d, ld, kp2, eL, eRS, eRH);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (slices) {
        case 3: return launch_digits_bf16_s<3>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        case 4: return launch_digits_bf16_s<4>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        case 5: return launch_digits_bf16_s<5>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        case 6: return launch_digits_bf16_s<6>(P, Q, d, ld, kp2, np, eL, eRS, eRH, L, RS, RH, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_split_bf16_contract(const SplitProblemDev *probs, const TileDev *tiles, int n_tiles, int slices,
                                      hipStream_t s)
{
    switch (slices) {
        case 3: return launch_bf16_s<3>(probs, tiles, n_tiles, s);
        case 4: return launch_bf16_s<4>(probs, tiles, n_tiles, s);
        case 5: return launch_bf16_s<5>(probs, tiles, n_tiles, s);
        case 6: return launch_bf16_s<6>(probs, tiles, n_tiles, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace flapw
