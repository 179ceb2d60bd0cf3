// T matrices of the atom types (appendix A.2, eqs. gaunt and t_matrices):
//   T^[XY]_{L',L} = sum_{L''} I^{(x,y)}_{l',l,L''} G_{L,L',L''} + spherical diagonal term,
//   G_{L,L',L''} = int conj(Y_{L'}) Y_L Y_{L''} dOmega.
// The Gaunt coefficients are evaluated on the device by exact quadrature: the phi integral gives
// 2 pi delta(m' = m + m''), and the remaining integrand Ybar_{l'}^{m'} Ybar_l^m Ybar_{l''}^{m''}(z)
// is a polynomial of degree <= l + l' + l'' in z = cos(theta), integrated exactly by
// Gauss-Legendre with enough nodes (nodes and weights come from the host).
// Both kernels are tiny (microseconds); they are latency bound, not HBM or MFMA bound.
#include "common.hpp"

namespace flapw {

namespace {

// theta[(l*(l+1)/2 + m) * nq + i] = orthonormal associated Legendre function with the
// Condon-Shortley phase at node z_i (so that Y_lm = theta_l^m(cos th) e^{i m phi}), m >= 0.
__global__ void legendre_table_kernel(int lt, int nq, const double *zn, double *theta)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (lt + 1) * nq) return;
    const int m = idx / nq, i = idx % nq;
    const double z = zn[i];
    const double st = sqrt(fmax(0.0, 1.0 - z * z));
    double q = 1.0;
    for (int k = 1; k <= m; ++k) q *= (2.0 * k - 1.0) / (2.0 * k) * st * st;
    double pmm = sqrt((2.0 * m + 1.0) / (4.0 * kPi) * q);
    if (m & 1) pmm = -pmm;
    double p2 = 0.0, p1 = pmm;
    for (int l = m; l <= lt; ++l) {
        double p;
        if (l == m) p = pmm;
        else if (l == m + 1) p = sqrt(2.0 * m + 3.0) * z * pmm;
        else {
            double a = sqrt((4.0 * l * l - 1.0) / (double)(l * l - m * m));
            double b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
            p = a * (z * p1 - b * p2);
        }
        if (l > m) { p2 = p1; p1 = p; }
        theta[((long long)l * (l + 1) / 2 + m) * nq + i] = p;
    }
}

__device__ inline double theta_at(const double *theta, int nq, int l, int m, int i)
{
    const int am = m < 0 ? -m : m;
    double v = theta[((long long)l * (l + 1) / 2 + am) * nq + i];
    return (m < 0 && (am & 1)) ? -v : v;        // theta_l^{-m} = (-1)^m theta_l^m
}

// one thread per (type, row, column) of the ldt x ldt matrix of a type; rows = bra.
// lmax_t: l_max of each type's row blocks.  lnonsph >= 0: structured T (section 3.1, Fig.
// Tmat_structure): the non-spherical terms l'' >= 1 only where l' and l are both <= lnonsph.
__global__ void tmat_kernel(int n_types, const int *lmax_t, int lstride, int lpot, int nq, const double *w,
                            const double *theta, const double *i_uu, const double *i_ud, const double *i_du,
                            const double *i_dd, const double *e_l, const double *ud_norm2, double2 *T,
                            long long ldt, int lnonsph)
{
    const long long per = ldt * ldt;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * n_types) return;
    const int ty = (int)(idx / per);
    const long long rem = idx % per;
    const int c = (int)(rem / ldt), r = (int)(rem % ldt);
    const int lmax = lmax_t[ty];
    const int nl = (lmax + 1) * (lmax + 1);
    double2 *out = T + (long long)ty * per + (long long)c * ldt + r;
    if (r >= 2 * nl || c >= 2 * nl) { *out = make_double2(0.0, 0.0); return; }
    const int brab = r >= nl, ketb = c >= nl;
    const int Lp = brab ? r - nl : r, L = ketb ? c - nl : c;
    const double *I = (!brab && !ketb) ? i_uu : (!brab && ketb) ? i_ud : (brab && !ketb) ? i_du : i_dd;
    int lp = 0; while ((lp + 1) * (lp + 1) <= Lp) ++lp;
    int l = 0;  while ((l + 1) * (l + 1) <= L) ++l;
    const int mp = Lp - lp * lp - lp, m = L - l * l - l;
    const int mpp = mp - m;
    const int nlp = (lpot + 1) * (lpot + 1);
    const double *Il = I + (((long long)ty * lstride + lp) * lstride + l) * nlp;
    double s = 0.0;
    int l0 = mpp < 0 ? -mpp : mpp;
    if (l0 < (lp > l ? lp - l : l - lp)) l0 = lp > l ? lp - l : l - lp;
    if ((l0 + l + lp) & 1) ++l0;
    const bool dense = lnonsph < 0 || (lp <= lnonsph && l <= lnonsph);
    const int l1 = dense ? min(lpot, l + lp) : 0;
    for (int lpp = l0; lpp <= l1; lpp += 2) {
        const double iv = Il[lpp * lpp + lpp + mpp];
        if (iv == 0.0) continue;
        double gq = 0.0;
        for (int i = 0; i < nq; ++i)
            gq += w[i] * theta_at(theta, nq, lp, mp, i) * theta_at(theta, nq, l, m, i) * theta_at(theta, nq, lpp, mpp, i);
        s += iv * 2.0 * kPi * gq;
    }
    if (Lp == L) {
        const double el = e_l[ty * lstride + l];
        if (!brab && !ketb) s += el;
        else if (brab && ketb) s += el * ud_norm2[ty * lstride + l];
        else s += 0.5;
    }
    *out = make_double2(s, 0.0);
}

// The T entries that are diagonal in L, per (type, l) for l <= l_max of the type (lmax_t: the
// full l_max, not a cut row block): out[(ty * kLStride + l) * 4 + {0, 1, 2, 3}] = {aa, ab, ba, bb},
// the spherical terms (E_l, 1/2, 1/2, E_l ||udot||^2, eq. t_matrices) plus the l'' = 0 integrals
// times G_{L,L,00} (the same quadrature as tmat_kernel; it equals Y_00 for every m).  Entries past
// l_max are zero.  The addition-theorem kernel adds these to H for the rows a structured T leaves
// out of the contraction.
__global__ void tmat_sph_kernel(int n_types, const int *lmax_t, int lstride, int lpot, int nq, const double *w,
                                const double *theta, const double *i_uu, const double *i_ud, const double *i_du,
                                const double *i_dd, const double *e_l, const double *ud_norm2, double *out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_types * kLStride) return;
    const int ty = idx / kLStride, l = idx % kLStride;
    double *o = out + (long long)idx * 4;
    if (l > lmax_t[ty]) {
        o[0] = o[1] = o[2] = o[3] = 0.0;
        return;
    }
    double gq = 0.0;
    for (int i = 0; i < nq; ++i) gq += w[i] * theta_at(theta, nq, l, 0, i) * theta_at(theta, nq, l, 0, i) * theta_at(theta, nq, 0, 0, i);
    const double g = 2.0 * kPi * gq;
    const int nlp = (lpot + 1) * (lpot + 1);
    const long long q = (long long)ty * lstride + l, ii = (q * lstride + l) * nlp;
    o[0] = e_l[q] + i_uu[ii] * g;
    o[1] = 0.5 + i_ud[ii] * g;
    o[2] = 0.5 + i_du[ii] * g;
    o[3] = e_l[q] * ud_norm2[q] + i_dd[ii] * g;
}

}  // namespace

hipError_t launch_tmat_sph(int n_types, const int *lmax_dev, int lstride, int lpot, int nq, const double *w,
                           const double *theta, const double *i_uu, const double *i_ud, const double *i_du,
                           const double *i_dd, const double *e_l, const double *ud_norm2, double *out, hipStream_t s)
{
    const int n = n_types * kLStride;
    hipLaunchKernelGGL(tmat_sph_kernel, dim3((n + 63) / 64), dim3(64), 0, s, n_types, lmax_dev, lstride, lpot, nq, w,
                       theta, i_uu, i_ud, i_du, i_dd, e_l, ud_norm2, out);
    return hipGetLastError();
}

hipError_t launch_legendre_table(int lt, int nq, const double *z, double *theta, hipStream_t s)
{
    const int n = (lt + 1) * nq;
    hipLaunchKernelGGL(legendre_table_kernel, dim3((n + 255) / 256), dim3(256), 0, s, lt, nq, z, theta);
    return hipGetLastError();
}

hipError_t launch_tmat(int n_types, const int *lmax_dev, int lstride, int lpot, int nq, const double *w,
                       const double *theta, const double *i_uu, const double *i_ud, const double *i_du,
                       const double *i_dd, const double *e_l, const double *ud_norm2, double2 *T, long long ldt,
                       int lnonsph, hipStream_t s)
{
    const long long n = ldt * ldt * n_types;
    hipLaunchKernelGGL(tmat_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_types, lmax_dev, lstride, lpot,
                       nq, w, theta, i_uu, i_ud, i_du, i_dd, e_l, ud_norm2, T, ldt, lnonsph);
    return hipGetLastError();
}

}  // namespace flapw
