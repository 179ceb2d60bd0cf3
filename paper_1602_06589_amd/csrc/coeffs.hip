// Matching coefficients A_{L,a,t}, B_{L,a,t} (appendix A.1, eqs. def_a_tensor, def_b_tensor).
//
//   A = 4 pi / (W sqrt(Omega)) i^l exp(i K_t.x_a) conj(Y_lm(R_a Khat_t)) [udot K j_l'(KR) - udot' j_l(KR)]
//   B = (same prefactor)                                                 [u' j_l(KR) - u K j_l'(KR)]
//
// One work-group per basis column t.  The radial factors depend on (type, l, t) only and are
// formed once per column; Y_lm(R_a Khat) and the phase depend on (atom, t) and are formed per
// atom chunk into LDS; the store loop then walks the column's rows so that consecutive lanes
// write consecutive 16-byte elements (the column is contiguous in memory).
// The kernel is bound by the HBM writes of A and B (32 bytes per (row, column)).
#include "common.hpp"

namespace flapw {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 16;                      // atoms per chunk (16 atoms x 16 m-slots = 256 threads)
constexpr int kNLCap = (FLAPW_LMAX_CAP + 1) * (FLAPW_LMAX_CAP + 1);
constexpr int kTypeCap = 32;                    // types handled per column (LDS tables)

// Spherical Bessel functions j_0..j_n at x (n = lmax + 1).
//  x < 1e-3     : three terms of the power series x^l/(2l+1)!! (1 - x^2/(2(2l+3)) + ...)
//  x > n        : upward recurrence j_{l+1} = (2l+1)/x j_l - j_{l-1} (stable while l < x)
//  otherwise    : downward (Miller) recurrence from n + 30 + x, scaled to the closed form of
//                 j_0 = sin x / x or j_1 = (sin x / x - cos x) / x, whichever is larger.
__device__ void sph_bessel(int n, double x, double *j)
{
    if (x == 0.0) {
        j[0] = 1.0;
        for (int l = 1; l <= n; ++l) j[l] = 0.0;
        return;
    }
    if (x < 1e-3) {
        double xl = 1.0, df = 1.0;
        for (int l = 0; l <= n; ++l) {
            double x2 = x * x;
            j[l] = xl / df * (1.0 - x2 / (2.0 * (2 * l + 3)) + x2 * x2 / (8.0 * (2 * l + 3) * (2 * l + 5)));
            xl *= x;
            df *= (2.0 * l + 3.0);
        }
        return;
    }
    double s, c;
    sincos(x, &s, &c);
    const double j0 = s / x, j1 = (s / x - c) / x;
    if (x > (double)n) {
        j[0] = j0;
        if (n >= 1) j[1] = j1;
        for (int l = 1; l < n; ++l) j[l + 1] = (2.0 * l + 1.0) / x * j[l] - j[l - 1];
        return;
    }
    const int top = n + 30 + (int)x;
    double fp1 = 0.0, f = 1.0;                 // f_{l+1}, f_l
    for (int l = top; l > n; --l) {
        double fm = (2.0 * l + 1.0) / x * f - fp1;
        fp1 = f;
        f = fm;
        if (fabs(f) > 1e150) { f *= 1e-150; fp1 *= 1e-150; }
    }
    j[n] = f;
    double cur = f, nxt = fp1;
    for (int l = n; l >= 1; --l) {
        double prv = (2.0 * l + 1.0) / x * cur - nxt;
        nxt = cur;
        cur = prv;
        j[l - 1] = cur;
        if (fabs(cur) > 1e150) {
            for (int q = l - 1; q <= n; ++q) j[q] *= 1e-150;
            cur *= 1e-150;
            nxt *= 1e-150;
        }
    }
    const double sc = (fabs(j0) >= fabs(j1)) ? j0 / j[0] : j1 / j[1];
    for (int l = 0; l <= n; ++l) j[l] *= sc;
}

// Recurrence tables for Ybar_l^m (built per work-group in LDS, indexed l^2 + l + m, m >= 0):
//   Ybar_m^m = (-1)^m sqrt((2m+1)/(4 pi) prod_{k<=m} (2k-1)/(2k)),  Ybar_{m+1}^m = sqrt(2m+3) z Ybar_m^m,
//   Ybar_l^m = a_lm (z Ybar_{l-1}^m - b_lm Ybar_{l-2}^m),  a_lm = sqrt((4l^2-1)/(l^2-m^2)),
//   b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
// Y_lm = Ybar_l^m (x + i y)^m and Y_{l,-m} = (-1)^m conj(Y_lm).
struct YTables {
    double a[kNLCap];
    double b[kNLCap];
    double mm[kLStride];            // Ybar_m^m
    unsigned char lof[kNLCap];      // l of L = l^2 + l + m
};

__device__ void build_ytables(YTables &yt, int tid)
{
    for (int L = tid; L < kNLCap; L += kThreads) {
        int l = 0;
        while ((l + 1) * (l + 1) <= L) ++l;
        yt.lof[L] = (unsigned char)l;
        const int m = L - l * l - l;
        double av = 0.0, bv = 0.0;
        if (m >= 0 && l >= m + 2) {
            av = sqrt((4.0 * l * l - 1.0) / (double)(l * l - m * m));
            bv = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
        }
        yt.a[L] = av;
        yt.b[L] = bv;
    }
    if (tid < kLStride) {
        const int m = tid;
        double q = 1.0;
        for (int k = 1; k <= m; ++k) q *= (2.0 * k - 1.0) / (2.0 * k);
        const double v = sqrt((2.0 * m + 1.0) / (4.0 * kPi) * q);
        yt.mm[m] = (m & 1) ? -v : v;
    }
}

// Y_{l,m} and Y_{l,-m} for one m >= 0 and l = m..lmax at the unit vector (x, y, z).
__device__ void ylm_m(const YTables &yt, int lmax, int m, double x, double y, double z, double2 *Y)
{
    double pr = 1.0, pi = 0.0;
    for (int k = 0; k < m; ++k) {
        const double t = pr * x - pi * y;
        pi = pr * y + pi * x;
        pr = t;
    }
    const double sg = (m & 1) ? -1.0 : 1.0;
    double qm2 = 0.0, qm1 = 0.0;
    for (int l = m; l <= lmax; ++l) {
        const int L = l * l + l + m;
        double ql;
        if (l == m) ql = yt.mm[m];
        else if (l == m + 1) ql = sqrt(2.0 * m + 3.0) * z * qm1;
        else ql = yt.a[L] * (z * qm1 - yt.b[L] * qm2);
        qm2 = qm1;
        qm1 = ql;
        const double2 v = make_double2(ql * pr, ql * pi);
        Y[L] = v;
        if (m > 0) Y[l * l + l - m] = make_double2(sg * v.x, -sg * v.y);
    }
}

// Dynamic LDS: radial factors of A and B, [n_types][kLStride] each, then Y of the chunk's atoms,
// [kChunk][nlmax] (nlmax = largest (lmax+1)^2 of the atom set), so the footprint follows the
// problem's l_max rather than the library cap.
__global__ __launch_bounds__(kThreads) void coeffs_kernel(double kx, double ky, double kz, int n_g, const double *g,
                                                          const AtomDev *atoms, int n_atoms, const TypeDev *types,
                                                          int n_types, int nlmax, double pref, double2 *A, double2 *B,
                                                          long long ld, long long zr0, long long zr1)
{
    extern __shared__ double2 dyn[];
    double2 *radA = dyn, *radB = dyn + n_types * kLStride, *Ybuf = dyn + 2 * n_types * kLStride;
    __shared__ double2 phase[kChunk];
    __shared__ long long rowA[kChunk], rowB[kChunk];
    __shared__ int atype[kChunk], anl[kChunk];
    __shared__ YTables yt;
    __shared__ double kvec[4];                 // K_t (x, y, z) and |K_t|

    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    double2 *colA = A + (long long)t * ld;
    double2 *colB = B + (long long)t * ld;

    if (t >= n_g) {                            // padding column of the work layout: zeros
        for (long long r = tid; r < zr1; r += kThreads) colA[r] = make_double2(0.0, 0.0);
        return;
    }
    for (long long r = zr0 + tid; r < zr1; r += kThreads) colA[r] = make_double2(0.0, 0.0);

    if (tid == 0) {
        double x = kx + g[3 * (long long)t], y = ky + g[3 * (long long)t + 1], z = kz + g[3 * (long long)t + 2];
        kvec[0] = x; kvec[1] = y; kvec[2] = z;
        kvec[3] = sqrt(x * x + y * y + z * z);
    }
    build_ytables(yt, tid);
    __syncthreads();
    const double kn = kvec[3];

    if (tid < n_types) {
        const TypeDev &ty = types[tid];
        double j[kLStride + 1];
        sph_bessel(ty.lmax + 1, kn * ty.rmt, j);
        for (int l = 0; l <= ty.lmax; ++l) {
            const RadialDev &r = ty.rad[l];
            double jl = j[l];
            double djl = (l == 0) ? -j[1] : (l * j[l - 1] - (l + 1.0) * j[l + 1]) / (2.0 * l + 1.0);
            double fa = (r.ud * kn * djl - r.dud * jl) * r.inv_w * pref;
            double fb = (r.du * jl - r.u * kn * djl) * r.inv_w * pref;
            // multiply by i^l
            double2 ca, cb;
            switch (l & 3) {
                case 0: ca = make_double2(fa, 0.0); cb = make_double2(fb, 0.0); break;
                case 1: ca = make_double2(0.0, fa); cb = make_double2(0.0, fb); break;
                case 2: ca = make_double2(-fa, 0.0); cb = make_double2(-fb, 0.0); break;
                default: ca = make_double2(0.0, -fa); cb = make_double2(0.0, -fb); break;
            }
            radA[tid * kLStride + l] = ca;
            radB[tid * kLStride + l] = cb;
        }
    }

    double khat[3] = {0.0, 0.0, 1.0};
    if (kn > 0.0) { khat[0] = kvec[0] / kn; khat[1] = kvec[1] / kn; khat[2] = kvec[2] / kn; }

    // Per chunk of 16 atoms: thread (al = tid / 16, m = tid % 16) forms Y_{l,+-m} of atom al into
    // LDS; then thread (al, j) stores rows L = j, j + 16, ... of atom al (16 consecutive rows =
    // 256 contiguous bytes per atom and store instruction).
    const int al = tid / 16, lane16 = tid % 16;
    for (int a0 = 0; a0 < n_atoms; a0 += kChunk) {
        const int na = min(kChunk, n_atoms - a0);
        __syncthreads();                       // previous chunk's stores are done with Ybuf
        if (al < na) {
            const AtomDev &at = atoms[a0 + al];
            const int lmax = yt.lof[at.nl - 1];          // l of the atom's last row (its type's l_max,
            const int m = lane16;                        // or less when the rows are cut)
            if (m <= lmax) {
                const double *R = at.rot;
                const double x = R[0] * khat[0] + R[1] * khat[1] + R[2] * khat[2];
                const double y = R[3] * khat[0] + R[4] * khat[1] + R[5] * khat[2];
                const double z = R[6] * khat[0] + R[7] * khat[1] + R[8] * khat[2];
                ylm_m(yt, lmax, m, x, y, z, Ybuf + al * nlmax);
            }
            if (m == 0) {
                double s, c;
                sincos(kvec[0] * at.pos[0] + kvec[1] * at.pos[1] + kvec[2] * at.pos[2], &s, &c);
                phase[al] = make_double2(c, s);
                rowA[al] = at.rowA;
                rowB[al] = at.rowB;
                atype[al] = at.type;
                anl[al] = at.nl;
            }
        }
        __syncthreads();
        if (al < na) {
            const double2 ph = phase[al];
            const int ty = atype[al], nl = anl[al];
            double2 *dA = colA + rowA[al], *dB = colB + rowB[al];
            for (int L = lane16; L < nl; L += 16) {
                const int l = yt.lof[L];
                const double2 y = Ybuf[al * nlmax + L];
                // phase * conj(Y)
                const double2 pc = make_double2(ph.x * y.x + ph.y * y.y, ph.y * y.x - ph.x * y.y);
                const double2 ra = radA[ty * kLStride + l], rb = radB[ty * kLStride + l];
                dA[L] = make_double2(ra.x * pc.x - ra.y * pc.y, ra.x * pc.y + ra.y * pc.x);
                dB[L] = make_double2(rb.x * pc.x - rb.y * pc.y, rb.x * pc.y + rb.y * pc.x);
            }
        }
    }
}

}  // namespace

hipError_t launch_coeffs(const double kvec[3], int n_g, int n_cols, const double *g, const AtomDev *atoms, int n_atoms,
                         const TypeDev *types, int n_types, int nlmax, double pref, double2 *A, double2 *B,
                         long long ld, long long zero_rows_from, long long zero_rows_to, hipStream_t s)
{
    if (n_types > kTypeCap || nlmax < 1 || nlmax > kNLCap) return hipErrorInvalidValue;
    const size_t lds = sizeof(double2) * (2 * (size_t)n_types * kLStride + (size_t)kChunk * nlmax);
    hipLaunchKernelGGL(coeffs_kernel, dim3(n_cols), dim3(kThreads), lds, s, kvec[0], kvec[1], kvec[2], n_g, g, atoms,
                       n_atoms, types, n_types, nlmax, pref, A, B, ld, zero_rows_from, zero_rows_to);
    return hipGetLastError();
}

}  // namespace flapw
