// Radial functions of the spherical muffin-tin potential (section 2.2, eq. simp_Schr) and the
// radial integrals of the non-spherical potential (appendix A.2, eq. nonsph_integrals).
//
// Units are Hartree (the kinetic prefactor hbar^2/2m of eq. simp_Schr is 1/2).  With P = r u and
// Pd = dP/dE the two radial equations are
//     P''  = [l(l+1)/r^2 + 2 (V - E)] P,       Pd'' = [l(l+1)/r^2 + 2 (V - E)] Pd - 2 P,
// the second being the energy derivative of the first.  The mesh of a type is logarithmic,
// r_i = r0 e^{i h}, h = ln(R/r0)/(n_r - 1); in x = ln r the state (P, dP/dr, Pd, dPd/dr) is
// advanced by the classical fourth-order Runge-Kutta rule with step 2h, so each midpoint is a
// mesh point where V is given and the functions are produced on the even points.  The start at
// r0 is the regular small-r form P = r^{l+1} (1 - Z r/(l+1)) with Z = -r0 V(r0), Pd = 0.
// Integrals over [r0, R] use Simpson's rule in x on the even points (dr = r dx).  P is then
// normalised to unit norm and Pd made orthogonal to it.
//
// Kernels:
//   radial_solve_kernel    one thread per (type, l): the outward integration is a sequential
//                          recurrence of n_e steps; the per-type potential is shared by the
//                          lanes of a type and read through the cache.
//   radial_integral_kernel one block per (type, L''): the table F_t (n_e x 2(lmax+1), columns
//                          u_0..u_lmax, udot_0..udot_lmax) gives the four integrals at once as
//                          the symmetric product F^T diag(w r v_{L''}) F; the block stages chunks
//                          of F and of the weighted potential in LDS and each thread accumulates
//                          pairs (a <= b) of the upper triangle.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace flapw {

namespace {

constexpr int kIntThreads = 256;
constexpr int kIntChunk = 128;           // mesh points staged per LDS round
constexpr int kFCols = 2 * kLStride;     // columns of F per mesh point (u then udot)

// Simpson weight (1, 4, 2, ..., 4, 1) of even point j of n_e.
__device__ inline double simpson_w(int j, int ne)
{
    return (j == 0 || j == ne - 1) ? 1.0 : ((j & 1) ? 4.0 : 2.0);
}

// Radial right-hand side in x = ln r: y = (P, D, Pd, Dd), c = l(l+1)/r + 2 r (V - E).
__device__ inline void rhs(const double y[4], double r, double c, double k[4])
{
    k[0] = r * y[1];
    k[1] = c * y[0];
    k[2] = r * y[3];
    k[3] = c * y[2] - 2.0 * r * y[0];
}

// fun: [n_types][n_e][kFCols]; column l is P_l, column kLStride + l is Pd_l.
// bnd: [n_types][kLStride][5] = u(R), u'(R), udot(R), udot'(R), ||udot||^2.
__global__ void __launch_bounds__(64) radial_solve_kernel(int n_r, const double *__restrict__ r0s,
                                                          const double *__restrict__ rmts,
                                                          const int *__restrict__ lmaxs,
                                                          const double *__restrict__ e_l, int lstride,
                                                          const double *__restrict__ v_sph, double *fun,
                                                          double *__restrict__ bnd)
{
    const int t = blockIdx.x, l = threadIdx.x;
    if (l > lmaxs[t]) return;
    const int ne = (n_r - 1) / 2 + 1;
    const double r0 = r0s[t], R = rmts[t];
    const double lnr = log(R / r0);
    const double h = lnr / (n_r - 1), h2 = 2.0 * h;
    const double e = e_l[t * lstride + l];
    const double ll = (double)l * (l + 1);
    const double *v = v_sph + (size_t)t * n_r;
    double *f = fun + (size_t)t * ne * kFCols;
    const int cp = l, cd = kLStride + l;

    const double z = -r0 * v[0];
    double y[4];
    y[0] = pow(r0, (double)(l + 1)) * (1.0 - z * r0 / (l + 1.0));
    y[1] = (l + 1.0) * pow(r0, (double)l) - z * (l + 2.0) / (l + 1.0) * pow(r0, (double)(l + 1));
    y[2] = 0.0;
    y[3] = 0.0;
    f[cp] = y[0];
    f[cd] = y[2];
    double ra = r0;                           // r at the step's start
    for (int j = 1; j < ne; ++j) {
        const int i0 = 2 * (j - 1);
        const double rm = r0 * exp(h * (i0 + 1)), rb = r0 * exp(h * (i0 + 2));
        const double ca = ll / ra + 2.0 * ra * (v[i0] - e);
        const double cm = ll / rm + 2.0 * rm * (v[i0 + 1] - e);
        const double cb = ll / rb + 2.0 * rb * (v[i0 + 2] - e);
        double k1[4], k2[4], k3[4], k4[4], yt[4];
        rhs(y, ra, ca, k1);
        for (int q = 0; q < 4; ++q) yt[q] = y[q] + h * k1[q];
        rhs(yt, rm, cm, k2);
        for (int q = 0; q < 4; ++q) yt[q] = y[q] + h * k2[q];
        rhs(yt, rm, cm, k3);
        for (int q = 0; q < 4; ++q) yt[q] = y[q] + h2 * k3[q];
        rhs(yt, rb, cb, k4);
        for (int q = 0; q < 4; ++q) y[q] = y[q] + h2 / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
        f[(size_t)j * kFCols + cp] = y[0];
        f[(size_t)j * kFCols + cd] = y[2];
        ra = rb;
    }
    // the thread re-reads only what it wrote itself
    auto simpson = [&](int mode) {
        double s = 0.0;
        for (int j = 0; j < ne; ++j) {
            const double p = f[(size_t)j * kFCols + cp], pd = f[(size_t)j * kFCols + cd];
            const double g = mode == 0 ? p * p : (mode == 1 ? p * pd : pd * pd);
            s += simpson_w(j, ne) * g * (r0 * exp(h2 * j));
        }
        return s * h2 / 3.0;
    };
    const double nrm = 1.0 / sqrt(simpson(0));
    for (int j = 0; j < ne; ++j) {
        f[(size_t)j * kFCols + cp] *= nrm;
        f[(size_t)j * kFCols + cd] *= nrm;
    }
    double D = y[1] * nrm, Dd = y[3] * nrm;
    const double c = simpson(1);
    for (int j = 0; j < ne; ++j) f[(size_t)j * kFCols + cd] -= c * f[(size_t)j * kFCols + cp];
    Dd -= c * D;
    const double n2 = simpson(2);
    const double P = f[(size_t)(ne - 1) * kFCols + cp], Pd = f[(size_t)(ne - 1) * kFCols + cd];
    double *b = bnd + ((size_t)t * kLStride + l) * 5;
    b[0] = P / R;
    b[1] = D / R - P / (R * R);
    b[2] = Pd / R;
    b[3] = Dd / R - Pd / (R * R);
    b[4] = n2;
}

struct IntSmem {
    double F[kIntChunk][kFCols + 1];
    double wv[kIntChunk];
};

// out_*: [n_types][lstride][lstride][nlp], bra l' first; zero-filled beforehand for l > lmax.
__global__ void __launch_bounds__(kIntThreads) radial_integral_kernel(
    int n_r, int nlp, const double *__restrict__ r0s, const double *__restrict__ rmts,
    const int *__restrict__ lmaxs, int lstride, const double *__restrict__ v_lm,
    const double *__restrict__ fun, double *__restrict__ i_uu, double *__restrict__ i_ud,
    double *__restrict__ i_du, double *__restrict__ i_dd)
{
    __shared__ IntSmem sm;
    const int L = blockIdx.x, t = blockIdx.y, tid = threadIdx.x;
    const int n = lmaxs[t] + 1, n2 = 2 * n;
    const int npair = n2 * (n2 + 1) / 2;
    const int ne = (n_r - 1) / 2 + 1;
    const double r0 = r0s[t];
    const double h2 = 2.0 * log(rmts[t] / r0) / (n_r - 1);
    const double *v = v_lm + ((size_t)t * nlp + L) * n_r;
    const double *ft = fun + (size_t)t * ne * kFCols;

    // pairs p = tid and tid + kIntThreads (npair <= 351 < 2 * kIntThreads)
    int pa[2], pb[2];
    for (int s = 0; s < 2; ++s) {
        int p = tid + s * kIntThreads, a = 0;
        pa[s] = -1;
        pb[s] = -1;
        if (p < npair) {
            while (p >= n2 - a) { p -= n2 - a; ++a; }
            pa[s] = a;
            pb[s] = a + p;
        }
    }
    // column of F for row index a of the 2n x 2n product
    auto col = [&](int a) { return a < n ? a : kLStride + (a - n); };
    const int ca0 = pa[0] >= 0 ? col(pa[0]) : 0, cb0 = pb[0] >= 0 ? col(pb[0]) : 0;
    const int ca1 = pa[1] >= 0 ? col(pa[1]) : 0, cb1 = pb[1] >= 0 ? col(pb[1]) : 0;
    double acc0 = 0.0, acc1 = 0.0;

    for (int j0 = 0; j0 < ne; j0 += kIntChunk) {
        const int m = min(kIntChunk, ne - j0);
        __syncthreads();
        for (int q = tid; q < m * kFCols; q += kIntThreads) {
            const int jj = q / kFCols, cc = q % kFCols;
            sm.F[jj][cc] = ft[(size_t)(j0 + jj) * kFCols + cc];
        }
        for (int jj = tid; jj < m; jj += kIntThreads) {
            const int j = j0 + jj;
            sm.wv[jj] = simpson_w(j, ne) * (r0 * exp(h2 * j)) * v[2 * j];
        }
        __syncthreads();
        if (pa[0] >= 0)
            for (int jj = 0; jj < m; ++jj) acc0 += sm.F[jj][ca0] * sm.F[jj][cb0] * sm.wv[jj];
        if (pa[1] >= 0)
            for (int jj = 0; jj < m; ++jj) acc1 += sm.F[jj][ca1] * sm.F[jj][cb1] * sm.wv[jj];
    }
    for (int s = 0; s < 2; ++s) {
        if (pa[s] < 0) continue;
        const double val = (s == 0 ? acc0 : acc1) * h2 / 3.0;
        const int a = pa[s], b = pb[s];
        auto at = [&](double *arr, int lp, int l) { arr[(((size_t)t * lstride + lp) * lstride + l) * nlp + L] = val; };
        if (b < n) {                          // u_a, u_b
            at(i_uu, a, b);
            at(i_uu, b, a);
        } else if (a >= n) {                  // udot_{a-n}, udot_{b-n}
            at(i_dd, a - n, b - n);
            at(i_dd, b - n, a - n);
        } else {                              // u_a, udot_{b-n}
            at(i_ud, a, b - n);
            at(i_du, b - n, a);
        }
    }
}

}  // namespace

size_t radial_fun_bytes(int n_types, int n_r)
{
    return sizeof(double) * (size_t)n_types * ((n_r - 1) / 2 + 1) * kFCols;
}

hipError_t launch_radial(int n_types, int n_r, int nlp, const double *r0, const double *rmt, const int *lmax,
                         const double *e_l, int lstride, const double *v_sph, const double *v_lm, double *fun,
                         double *bnd, double *i_uu, double *i_ud, double *i_du, double *i_dd, hipStream_t s)
{
    hipLaunchKernelGGL(radial_solve_kernel, dim3(n_types), dim3(64), 0, s, n_r, r0, rmt, lmax, e_l, lstride, v_sph,
                       fun, bnd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radial_integral_kernel, dim3(nlp, n_types), dim3(kIntThreads), 0, s, n_r, nlp, r0, rmt, lmax,
                       lstride, v_lm, fun, i_uu, i_ud, i_du, i_dd);
    return hipGetLastError();
}

}  // namespace flapw
