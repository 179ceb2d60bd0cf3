// Modular split precision for the S/H contraction: the FP64 operands are scaled to integers and
// the integer products are computed modulo several pairwise coprime odd moduli p_m <= 255 on the int8
// matrix cores, then rebuilt by the Chinese remainder theorem in FP64.  (The paper computes these
// updates in FP64 BLAS, sections 4.2-4.6; this is an alternative to the digit scheme of split.hip
// whose work grows with the number of moduli, each worth about 7.5 bits, instead of with the number
// of kept digit pairs, and whose complex products take half the matrix-core work of a digit pair's.)
//
// Integers.  Operand column c (a basis function) is scaled by s_c = 2^B / ||X_c|| (the 2-norm of the
// column over all contraction rows, real and imaginary parts; s_c rounded down to 8 significant
// bits) and rounded: X'_kc = rint(X_kc s_c), so ||X'_c|| <= 2^B up to the rounding and every
// |X'| <= 2^B <= 2^50 (exact in FP64).  B is real:
// B = min(50, (log2 M - 1)/2 - 0.001), M = prod p_m.  By Cauchy-Schwarz every exact integer
// product entry C'_ij = Re or Im of sum_k conj(X'_ki) Y'_kj has |C'| <= ||X'_i|| ||Y'_j||, and the
// rounding adds at most sqrt(2K)/2 < 2^15 to a column norm of 2^B, B > 30 (a factor below
// 1 + 2^-15), against the 2^-0.002 margin in 2^(2B) <= M/2: |C'| < M/2 and C' is the unique residue
// of C' mod M in (-M/2, M/2).  Scaling each column to the largest admissible norm (instead of a
// power of two, which leaves it anywhere in [2^(B-1), 2^B)) makes the rounding error, relative to the
// column, the smallest the range allows: about 1.47 times smaller in the mean square.
//
// Residues.  r = X' mod p_m in the symmetric range [-(p-1)/2, (p-1)/2] fits int8 (the moduli are
// odd, so -128 never occurs); the products modulo each p_m run in mod_contract.hip.
//
// Complex products as two real ones.  Every modulus has a square root j of -1 (j^2 = -1 mod p; for
// odd p this holds exactly when every prime factor of p is 1 mod 4).  Then the Gaussian integers mod
// p split into two copies of the integers mod p: x = xr + i xi goes to the pair of evaluations
// (xr + j xi, xr - j xi) mod p, and sums and products go to the pairs' componentwise sums and
// products.  conj(x) goes to (xr - j xi, xr + j xi), so z = conj(X)^T Y goes to
// z1 = (Xr - j Xi)^T (Yr + j Yi) = Re z + j Im z and z2 = (Xr + j Xi)^T (Yr - j Yi) = Re z - j Im z,
// two real products, and Re z = (z1 + z2) / 2, Im z = (z1 - z2) / (2 j) mod p.  Against the four
// real products of Re and Im this halves the matrix-core work per modulus; the price is that the
// admissible moduli are smaller (14 of them <= 255, from 241 down to 109), so a given range M takes
// about one modulus more.  Each operand is stored as the residues of its two evaluations, in the
// places of the real and the imaginary part.
//
// Reconstruction.  With w_m = (M/p_m)^(-1) mod p_m, C'/M = sum_m y_m / p_m (mod 1) for the
// residues c_m and y_m = c_m w_m mod p_m; the sum is formed in double-double from 1/p_m = hi + lo,
// reduced to (-1/2, 1/2] and multiplied by M (also double-double).  Then C = C' / (s_i s_j), with
// the scales split as s = m 2^e (m in [1/2, 1)) so that neither product nor quotient overflows.
//
// Kernels:
//   mod_colnorm_kernel  per column: s_c of P, of d.P (right operand of S) and of Q (right of H)
//   mod_colsum_kernel   the same s_c from column-sum shares written by the real-T panel kernel
//   mod_slice_kernel    residues of all moduli, stored as [modulus][32-column block][32-row group]
//                       [evaluation at j, at -j][16-row half][32 columns][16 bytes] (one 1 KB MFMA
//                       fragment per evaluation and group)
//   hs_mod_i8_kernel    (mod_contract.hip) the products modulo each p_m
//   mod_crt_kernel      one block per tile: reads the residues of all moduli, rebuilds and
//                       scales the FP64 values, writes the upper triangle of S or H
#include <cmath>

#include "context.hpp"

namespace flapw {

namespace {



// x mod p in [-(p-1)/2, (p-1)/2] for odd p, ip = fl(1/p) and integer-valued |x| <= 2^50 (1 + 2^-15).
// x/p lies at least 1/(2p) from the nearest half-integer (x is an integer and p is odd), and the
// two roundings in fl(x ip) move it by at most about |x|/p 2^-52 <= 1.0001/(4p), so rint returns the nearest
// quotient, the remainder from the fma is exact and already in the symmetric range.
__device__ inline int sym_mod(double x, double p, double ip)
{
    const double q = rint(x * ip);
    return (int)fma(-q, p, x);
}

// Column scale about 2^B / sqrt(ss) (two2b = 2^B), rounded down to an 8-bit mantissa: j 2^(E-8),
// j in [128, 255], so that the scaled norm stays <= 2^B (within 2^-7 of it) and integer-valued
// columns stay integers whenever the scale is at least 256 (products of such columns up to 2^37
// then come back exactly: C' = C s_i s_j carries at most 16 more bits).  0 for a zero column.
__device__ inline double mod_scale(double ss, double two2b)
{
    if (!(ss > 0.0)) return 0.0;
    int E;
    const double f = frexp(two2b / sqrt(ss), &E);   // f in [1/2, 1)
    return ldexp(floor(f * 256.0), E - 8);
}

__global__ __launch_bounds__(256) void mod_colnorm_kernel(const double2 *__restrict__ P, const double2 *__restrict__ Q,
                                                          const double *__restrict__ d, long long ld, int kp2, int np,
                                                          double two2b, double *__restrict__ sL,
                                                          double *__restrict__ sRS, double *__restrict__ sRH)
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
        sL[c] = mod_scale(red[0][0], two2b);
        sRS[c] = mod_scale(red[1][0], two2b);
        sRH[c] = mod_scale(red[2][0], two2b);
    }
}

// The same scales from the column-sum shares that the real-T panel kernel wrote while forming
// Q: part[(k n_slots + slot) np + c], k = 0, 1, 2 for sum |P|^2, sum |P|^2 d^2, sum |Q|^2, summed
// over the slots in order (one thread per column, reads coalesced across columns).
__global__ __launch_bounds__(256) void mod_colsum_kernel(const double *__restrict__ part, long long n_slots,
                                                         long long np, int npm, double two2b,
                                                         double *__restrict__ sL, double *__restrict__ sRS,
                                                         double *__restrict__ sRH)
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
    sL[c] = mod_scale(sp, two2b);
    sRS[c] = mod_scale(sd, two2b);
    sRH[c] = mod_scale(sq, two2b);
}

// The low bytes of four int32 values packed into one word (byte k from value k) by two byte
// permutes (v_perm_b32: selector values 0-3 take the bytes of the second source, 4-7 those of the
// first, 0x0c a zero byte) and an or, where masking and shifting each byte takes two instructions.
__device__ inline unsigned pack_low_bytes(int b0, int b1, int b2, int b3)
{
    const unsigned lo = __builtin_amdgcn_perm((unsigned)b1, (unsigned)b0, 0x0c0c0400u);
    const unsigned hi = __builtin_amdgcn_perm((unsigned)b3, (unsigned)b2, 0x04000c0cu);
    return lo | hi;
}

// Residues of 16 Gaussian integers xr + i xi (integer-valued doubles, |xr|, |xi| <= 2^50 (1 + 2^-15))
// for every modulus, as the evaluations xr + sg j xi (16 bytes at out0 + m mstride) and xr - sg j xi
// (at out1 + m mstride); sg = -1 stores the conjugate.  xi is reduced first (c = xi mod p, exact in
// FP64); xr +- sg j c then stays within 2^50 (1 + 2^-15) + 127^2 and is reduced like xr.
__device__ inline void write_residues(const double (&xr)[16], const double (&xi)[16], int sg, const ModTable &mt,
                                      int8_t *out0, int8_t *out1, long long mstride)
{
    for (int m = 0; m < mt.nm; ++m) {
        const double p = (double)mt.p[m], ip = mt.inv_p[m];
        const double js = (double)(sg * mt.jr[m]);
        unsigned w0[4], w1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int v0[4], v1[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double x = xi[4 * q + b];
                const double c = fma(-rint(x * ip), p, x);             // xi mod p, exact
                const double r = xr[4 * q + b];
                v0[b] = sym_mod(fma(js, c, r), p, ip);
                v1[b] = sym_mod(fma(-js, c, r), p, ip);
            }
            w0[q] = pack_low_bytes(v0[0], v0[1], v0[2], v0[3]);
            w1[q] = pack_low_bytes(v1[0], v1[1], v1[2], v1[3]);
        }
        *reinterpret_cast<uint4 *>(out0 + m * mstride) = make_uint4(w0[0], w0[1], w0[2], w0[3]);
        *reinterpret_cast<uint4 *>(out1 + m * mstride) = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    }
}

// grid (npm/32, kp2/128): thread (m = tid % 32, chunk = tid / 32) handles 16 rows of column
// 32 blockIdx.x + m.  MODE 0: residues of P (left, conjugated) and d.P (right of S); MODE 1: of Q
// (right of H); MODE 2: of P alone (S is not contracted).  The 16 values are read once and each
// operand is formed and reduced in turn, so that one operand's 32 integers are live beside them.
template <int MODE>
__global__ __launch_bounds__(256) void mod_slice_kernel(const double2 *__restrict__ P, const double2 *__restrict__ Q,
                                                        const double *__restrict__ d, long long ld, int kp2, int np,
                                                        ModTable mt, const double *__restrict__ sL,
                                                        const double *__restrict__ sRS, const double *__restrict__ sRH,
                                                        int8_t *__restrict__ L, int8_t *__restrict__ RS,
                                                        int8_t *__restrict__ RH)
{
    const int m = threadIdx.x & 31;
    const long long cb = blockIdx.x, col = cb * 32 + m;
    const long long ch = (long long)blockIdx.y * 8 + (threadIdx.x >> 5);
    const long long nch = kp2 / 16, ncb = gridDim.x;
    const long long mstride = ncb * nch * 1024;
    // 32-row group ch / 2: the evaluations at j in its first 1 KB fragment, at -j in the second;
    // this 16-row chunk is half ch % 2 of each
    const long long off = (cb * nch + (ch & ~1LL)) * 1024 + (ch & 1) * 512 + m * 16, offi = off + 1024;
    const long long r0 = ch * 16;
    const double2 *src = MODE == 1 ? Q : P;
    double2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = col < np ? src[col * ld + r0 + r] : make_double2(0.0, 0.0);
    double xr[16], xi[16];
    if (MODE != 1) {
        const double s1 = sL[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            xr[r] = rint(v[r].x * s1);
            xi[r] = rint(v[r].y * s1);
        }
        write_residues(xr, xi, -1, mt, L + off, L + offi, mstride);
    }
    if (MODE == 0) {
        const double s2 = sRS[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const double w = d[r0 + r];
            xr[r] = rint(v[r].x * w * s2);
            xi[r] = rint(v[r].y * w * s2);
        }
        write_residues(xr, xi, 1, mt, RS + off, RS + offi, mstride);
    }
    if (MODE == 1) {
        const double sc = sRH[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            xr[r] = rint(v[r].x * sc);
            xi[r] = rint(v[r].y * sc);
        }
        write_residues(xr, xi, 1, mt, RH + off, RH + offi, mstride);
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
    const double *sR = mat ? pb.sRH : pb.sRS;
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
            int ec;
            const double mc = frexp(sR[cj], &ec);          // s = m 2^e, m in [1/2, 1) (0 for a zero column)
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
                int er;
                const double mr = frexp(pb.sL[ri], &er);
                const double mm = mr * mc;                         // in [1/4, 1), or 0
                const int sc = -(er + ec);
                const double vr = mm > 0.0 ? ldexp(crt_value(cre, mt) / mm, sc) : 0.0;
                const double vi = (ri == cj || !(mm > 0.0)) ? 0.0 : ldexp(crt_value(cim, mt) / mm, sc);
                outm[cj * pb.ldh + ri] = make_double2(vr, vi);
            }
        }
}

}  // namespace

long long mod_digit_bytes(long long kp2, long long npm, int nm) { return 2LL * nm * kp2 * npm; }

long long mod_scratch_bytes(long long npm, int nm)
{
    const long long t = npm / kModTile;
    return 2LL * (t * (t + 1) / 2) * nm * kResTileBytes;
}

hipError_t launch_mod_slice(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                            int npm, const ModTable &mt, double *sL, double *sRS, double *sRH, int8_t *L, int8_t *RS,
                            int8_t *RH, bool with_s, const double *part, long long n_slots, hipStream_t s)
{
    if (part)
        hipLaunchKernelGGL(mod_colsum_kernel, dim3((npm + 255) / 256), dim3(256), 0, s, part, n_slots, (long long)np, npm,
                           mt.two2b, sL, sRS, sRH);
    else
        hipLaunchKernelGGL(mod_colnorm_kernel, dim3(npm), dim3(256), 0, s, P, Q, d, ld, kp2, np, mt.two2b, sL, sRS, sRH);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(npm / 32, kp2 / 128);
    if (with_s)
        hipLaunchKernelGGL(mod_slice_kernel<0>, grid, dim3(256), 0, s, P, Q, d, ld, kp2, np, mt, sL, sRS, sRH, L, RS, RH);
    else
        hipLaunchKernelGGL(mod_slice_kernel<2>, grid, dim3(256), 0, s, P, Q, d, ld, kp2, np, mt, sL, sRS, sRH, L, RS, RH);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mod_slice_kernel<1>, grid, dim3(256), 0, s, P, Q, d, ld, kp2, np, mt, sL, sRS, sRH, L, RS, RH);
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

// The smallest x > 0 with x^2 = -1 mod c, or 0 when -1 is not a square mod c.
static int sqrt_minus_one(int c)
{
    for (int x = 1; x < c; ++x)
        if ((x * x + 1) % c == 0) return x;
    return 0;
}

// a mod p in [-(p-1)/2, (p-1)/2]
static int sym_rep(long long a, int p)
{
    long long r = ((a % p) + p) % p;
    return (int)(r > p / 2 ? r - p : r);
}

// inverse of a mod p (gcd(a, p) = 1), in [0, p)
static long long inv_mod(long long a, long long p)
{
    long long r0 = p, r1 = ((a % p) + p) % p, s0 = 0, s1 = 1;
    while (r1) {
        const long long f = r0 / r1, r2 = r0 - f * r1, s2 = s0 - f * s1;
        r0 = r1; r1 = r2; s0 = s1; s1 = s2;
    }
    return ((s0 % p) + p) % p;
}

// Moduli: the pairwise coprime odd integers <= 255 in which -1 is a square, taken greedily from 255
// downwards (241, 233, 229, 221, 205, 197, 193, 181, 173, 157, 149, 137, 113, 109); B from M.
ModTable make_mod_table(int nm)
{
    ModTable t{};
    t.nm = nm;
    int c = 255, k = 0;
    while (k < nm && c > 1) {
        bool ok = sqrt_minus_one(c) != 0;
        for (int j = 0; ok && j < k; ++j) {
            int a = c, b = t.p[j];
            while (b) { const int r = a % b; a = b; b = r; }
            if (a != 1) ok = false;
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
    // the integer range B (real): 2^(2B + 1) <= M with a 2^-0.002 margin, and at most 50
    t.bits_real = std::min(50.0, (lg - 1.0) / 2.0 - 0.001);
    t.bits = (int)std::floor(t.bits_real);
    t.two2b = std::exp2(t.bits_real);
    for (int m = 0; m < nm; ++m) {
        const long long p = t.p[m];
        long long q = 1;                                   // (M / p) mod p
        for (int j = 0; j < nm; ++j)
            if (j != m) q = q * t.p[j] % p;
        t.w[m] = (int)inv_mod(q, p);
        const int jr = sqrt_minus_one((int)p);
        t.jr[m] = sym_rep(jr, (int)p);
        t.h2[m] = sym_rep(inv_mod(2, p), (int)p);
        t.h2j[m] = sym_rep(inv_mod(2LL * jr, p), (int)p);
        t.inv_p[m] = 1.0 / (double)p;
        t.inv_p_lo[m] = std::fma(-t.inv_p[m], (double)p, 1.0) / (double)p;
    }
    t.M_hi = (double)M;
    const __int128 rest = (__int128)M - (__int128)t.M_hi;
    t.M_lo = (double)rest;
    return t;
}

}  // namespace flapw
