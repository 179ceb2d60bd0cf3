/*
 * flapw_oracle.c -- the plain, slow CPU reference for FLAPW muffin-tin H and S generation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this library.  The GPU library shares no code with it.
 *
 * Everything is FP64 (complex128 where complex), written as the paper's sums with no
 * blocking or reordering beyond what is stated next to each function.
 *
 * Conventions (the paper leaves them open):
 *   - complex spherical harmonics, orthonormal, with the Condon-Shortley phase,
 *     Y_{l,-m} = (-1)^m conj(Y_{l,m});
 *   - L = l*l + l + m;
 *   - the Gaunt coefficient is G_{L,L',L''} = integral of conj(Y_{L'}) Y_L Y_{L''} over the
 *     unit sphere (appendix A.2, eq. gaunt), with L' the bra index;
 *   - T-matrix diagonal (appendix A.2, eq. t_matrices): AA gets E_l, BB gets
 *     E_l ||udot_l||^2 (the derivation of <udot|H_sph|udot>), AB and BA each get 1/2
 *     (the Hermitian part of the printed +1 / +0, which keeps T^BA = (T^AB)^H as section
 *     4.4 requires).  The printed form (+1 on AB, +0 on BA) is available with literal=1.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------------------------------
 * Spherical Bessel functions j_l(x) and their derivatives (appendix A.1: the radial part of
 * the Rayleigh expansion of a plane wave).
 *
 * j_l is the minimal solution of f_{l-1} + f_{l+1} = (2l+1)/x f_l, so it is computed by
 * Miller's downward recurrence from an index far above max(lmax, x) and normalised with the
 * sum rule  sum_{l>=0} (2l+1) j_l(x)^2 = 1.  The overall sign is fixed by the closed forms
 * j_0 = sin x / x, j_1 = sin x / x^2 - cos x / x (whichever is larger in magnitude).
 * Derivative: j_0' = -j_1 and j_l' = j_{l-1} - (l+1)/x j_l.
 * ------------------------------------------------------------------------------------- */
void or_sph_bessel(int lmax, double x, double *j, double *dj)
{
    if (x == 0.0) {
        for (int l = 0; l <= lmax; ++l) { j[l] = (l == 0) ? 1.0 : 0.0; dj[l] = (l == 1) ? 1.0 / 3.0 : 0.0; }
        return;
    }
    int top = (lmax > (int)ceil(x) ? lmax : (int)ceil(x)) + 40;
    double *f = (double *)malloc(sizeof(double) * (top + 2));
    f[top + 1] = 0.0;
    f[top] = 1.0;
    for (int l = top; l >= 1; --l) {
        f[l - 1] = (2.0 * l + 1.0) / x * f[l] - f[l + 1];
        if (fabs(f[l - 1]) > 1e120) {           /* rescale so that f^2 stays in range */
            for (int q = l - 1; q <= top + 1; ++q) f[q] *= 1e-120;
        }
    }
    double s = 0.0;
    for (int l = top; l >= 0; --l) s += (2.0 * l + 1.0) * f[l] * f[l];
    double nrm = 1.0 / sqrt(s);
    double j0 = sin(x) / x, j1 = sin(x) / (x * x) - cos(x) / x;
    double sgn = (fabs(j0) >= fabs(j1)) ? ((j0 * f[0] >= 0.0) ? 1.0 : -1.0) : ((j1 * f[1] >= 0.0) ? 1.0 : -1.0);
    double jl[top + 1];
    for (int l = 0; l <= top; ++l) jl[l] = sgn * nrm * f[l];
    for (int l = 0; l <= lmax; ++l) {
        j[l] = jl[l];
        dj[l] = (l == 0) ? -jl[1] : jl[l - 1] - (l + 1.0) / x * jl[l];
    }
    free(f);
}

/* ---------------------------------------------------------------------------------------
 * Spherical harmonics Y_lm(v/|v|) for l = 0..lmax, stored at L = l*l + l + m.
 * Y_lm(theta, phi) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta) e^{i m phi}, m >= 0,
 * with P_l^m including the Condon-Shortley factor (-1)^m, from the textbook recurrences
 *   P_m^m = (-1)^m (2m-1)!! sin^m theta,  P_{m+1}^m = (2m+1) cos theta P_m^m,
 *   (l-m) P_l^m = (2l-1) cos theta P_{l-1}^m - (l+m-1) P_{l-2}^m;
 * negative m from Y_{l,-m} = (-1)^m conj(Y_lm).  v = 0 is read as the z direction.
 * ------------------------------------------------------------------------------------- */
static double factorial(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

void or_ylm(int lmax, const double *v, zc *y)
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double ct, st, phi;
    if (r == 0.0) { ct = 1.0; st = 0.0; phi = 0.0; }
    else {
        ct = v[2] / r;
        st = sqrt(v[0] * v[0] + v[1] * v[1]) / r;
        phi = (v[0] == 0.0 && v[1] == 0.0) ? 0.0 : atan2(v[1], v[0]);
    }
    for (int m = 0; m <= lmax; ++m) {
        double pmm = 1.0;
        for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * st;
        double plm2 = 0.0, plm1 = pmm;
        for (int l = m; l <= lmax; ++l) {
            double p;
            if (l == m) p = pmm;
            else if (l == m + 1) p = (2.0 * m + 1.0) * ct * pmm;
            else p = ((2.0 * l - 1.0) * ct * plm1 - (l + m - 1.0) * plm2) / (double)(l - m);
            if (l > m) { plm2 = plm1; plm1 = p; }
            double nrm = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            zc ylm = nrm * p * cexp(I * (double)m * phi);
            y[l * l + l + m] = ylm;
            if (m > 0) y[l * l + l - m] = ((m & 1) ? -1.0 : 1.0) * conj(ylm);
        }
    }
}

/* ---------------------------------------------------------------------------------------
 * Wigner 3j symbol by Racah's closed formula, and the Gaunt coefficient
 *   G_{L,L',L''} = int conj(Y_{L'}) Y_L Y_{L''} dOmega          (appendix A.2, eq. gaunt)
 *               = (-1)^{m'} sqrt((2l'+1)(2l+1)(2l''+1)/(4 pi))
 *                 (l' l l''; 0 0 0) (l' l l''; -m' m m'')
 * using conj(Y_{l'm'}) = (-1)^{m'} Y_{l',-m'}.
 * ------------------------------------------------------------------------------------- */
double or_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3)
{
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(m3) > j3) return 0.0;
    if (m1 == 0 && m2 == 0 && ((j1 + j2 + j3) & 1)) return 0.0;   /* (j1 j2 j3; 0 0 0) = 0 for odd sum */
    double delta = factorial(j1 + j2 - j3) * factorial(j1 - j2 + j3) * factorial(-j1 + j2 + j3) / factorial(j1 + j2 + j3 + 1);
    double pre = sqrt(delta * factorial(j1 + m1) * factorial(j1 - m1) * factorial(j2 + m2) * factorial(j2 - m2) *
                      factorial(j3 + m3) * factorial(j3 - m3));
    int kmin = 0, kmax = j1 + j2 - j3;
    if (j2 - j3 - m1 > kmin) kmin = j2 - j3 - m1;
    if (j1 - j3 + m2 > kmin) kmin = j1 - j3 + m2;
    if (j1 - m1 < kmax) kmax = j1 - m1;
    if (j2 + m2 < kmax) kmax = j2 + m2;
    double sum = 0.0;
    for (int k = kmin; k <= kmax; ++k) {
        double den = factorial(k) * factorial(j3 - j2 + k + m1) * factorial(j3 - j1 + k - m2) *
                     factorial(j1 + j2 - j3 - k) * factorial(j1 - k - m1) * factorial(j2 - k + m2);
        sum += ((k & 1) ? -1.0 : 1.0) / den;
    }
    int ph = j1 - j2 - m3;
    double sgn = ((ph % 2) != 0) ? -1.0 : 1.0;
    return sgn * pre * sum;
}

double or_gaunt(int l, int m, int lp, int mp, int lpp, int mpp)
{
    double w0 = or_wigner3j(lp, l, lpp, 0, 0, 0);
    if (w0 == 0.0) return 0.0;
    double w = or_wigner3j(lp, l, lpp, -mp, m, mpp);
    double sg = (mp & 1) ? -1.0 : 1.0;
    return sg * sqrt((2.0 * lp + 1.0) * (2.0 * l + 1.0) * (2.0 * lpp + 1.0) / (4.0 * M_PI)) * w0 * w;
}

/* ---------------------------------------------------------------------------------------
 * T matrices of one atom type (appendix A.2, eq. t_matrices):
 *   T^[XY]_{L',L} = sum_{L''} I^{(x,y)}_{l',l,L''} G_{L,L',L''} + diagonal spherical term.
 * Structured T (section 3.1, Fig. Tmat_structure): with lnonsph >= 0 the non-spherical terms
 * (l'' >= 1) are kept only where both l' and l are <= lnonsph; the spherical terms (l'' = 0 and
 * the diagonal term) are kept for every l.  lnonsph < 0 keeps everything.
 * Output: T (2NL x 2NL, column-major, leading dimension ldt) = [[T^AA, T^AB], [T^BA, T^BB]],
 * rows = bra (L'), columns = ket (L), NL = (lmax+1)^2.  I arrays for this type are
 * [lstride][lstride][(lpot+1)^2] indexed [l'][l][L''].
 * ------------------------------------------------------------------------------------- */
void or_tmat(int lmax, int lstride, int lpot, const double *i_uu, const double *i_ud, const double *i_du,
             const double *i_dd, const double *e_l, const double *ud_norm2, int literal, int lnonsph, zc *T, int ldt)
{
    int nl = (lmax + 1) * (lmax + 1);
    int nlp = (lpot + 1) * (lpot + 1);
    const double *ints[4] = {i_uu, i_ud, i_du, i_dd};     /* AA, AB, BA, BB */
    for (int blk = 0; blk < 4; ++blk) {
        int r0 = (blk == 0 || blk == 1) ? 0 : nl;           /* bra block: A rows, then B rows */
        int c0 = (blk == 0 || blk == 2) ? 0 : nl;           /* ket block */
        for (int lp = 0; lp <= lmax; ++lp)
            for (int mp = -lp; mp <= lp; ++mp)
                for (int l = 0; l <= lmax; ++l)
                    for (int m = -l; m <= l; ++m) {
                        int Lp = lp * lp + lp + mp, L = l * l + l + m;
                        double s = 0.0;
                        const int dense = lnonsph < 0 || (lp <= lnonsph && l <= lnonsph);
                        for (int lpp = 0; lpp <= (dense ? lpot : 0); ++lpp)
                            for (int mpp = -lpp; mpp <= lpp; ++mpp) {
                                int Lpp = lpp * lpp + lpp + mpp;
                                double iv = ints[blk][((size_t)lp * lstride + l) * nlp + Lpp];
                                if (iv != 0.0) s += iv * or_gaunt(l, m, lp, mp, lpp, mpp);
                            }
                        if (Lp == L) {
                            if (blk == 0) s += e_l[l];
                            else if (blk == 3) s += e_l[l] * ud_norm2[l];
                            else if (literal) s += (blk == 1) ? 1.0 : 0.0;
                            else s += 0.5;
                        }
                        T[(size_t)(c0 + L) * ldt + (r0 + Lp)] = s;
                    }
    }
}

/* ---------------------------------------------------------------------------------------
 * Matching coefficients (appendix A.1, eqs. def_a_tensor and def_b_tensor):
 *   A_{L,a,t} = c [udot(R) K j_l'(K R) - udot'(R) j_l(K R)]
 *   B_{L,a,t} = c [-u(R) K j_l'(K R) + u'(R) j_l(K R)]
 *   c = 4 pi / (W sqrt(Omega)) i^l exp(i K_t . x_a) conj(Y_lm(R_a Khat_t)),
 *   W = udot(R) u'(R) - u(R) udot'(R),   K_t = k + G_t, K = |K_t|.
 * Rows are the atoms stacked in order, each with (lmax(type)+1)^2 rows ordered by L
 * (section 4.2, stacked layout); columns are the given G vectors.  Column-major, ld = K.
 * R_a is row-major; R_a Khat means (R_a Khat)_i = sum_j R_a[i][j] Khat_j.
 * ------------------------------------------------------------------------------------- */
void or_coeffs(int n_atoms, const int *type, const double *pos, const double *rot, double omega, int lstride,
               const int *lmax_t, const double *rmt, const double *u, const double *du, const double *ud,
               const double *dud, const double *kvec, int n_g, const double *g, zc *A, zc *B, long ld)
{
    long *off = (long *)malloc(sizeof(long) * (n_atoms + 1));
    off[0] = 0;
    for (int a = 0; a < n_atoms; ++a) off[a + 1] = off[a] + (long)(lmax_t[type[a]] + 1) * (lmax_t[type[a]] + 1);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < n_g; ++t) {
        double kt[3] = {kvec[0] + g[3 * t], kvec[1] + g[3 * t + 1], kvec[2] + g[3 * t + 2]};
        double kn = sqrt(kt[0] * kt[0] + kt[1] * kt[1] + kt[2] * kt[2]);
        double khat[3] = {0.0, 0.0, 1.0};
        if (kn > 0.0) { khat[0] = kt[0] / kn; khat[1] = kt[1] / kn; khat[2] = kt[2] / kn; }
        for (int a = 0; a < n_atoms; ++a) {
            int ty = type[a], lm = lmax_t[ty];
            const double *ra = rot + 9 * a;
            double rk[3];
            for (int i = 0; i < 3; ++i) rk[i] = ra[3 * i] * khat[0] + ra[3 * i + 1] * khat[1] + ra[3 * i + 2] * khat[2];
            zc y[(lm + 1) * (lm + 1)];
            or_ylm(lm, rk, y);
            double jl[lm + 1], djl[lm + 1];
            or_sph_bessel(lm, kn * rmt[ty], jl, djl);
            double kx = kt[0] * pos[3 * a] + kt[1] * pos[3 * a + 1] + kt[2] * pos[3 * a + 2];
            zc phase = cexp(I * kx);
            for (int l = 0; l <= lm; ++l) {
                int q = ty * lstride + l;
                double w = ud[q] * du[q] - u[q] * dud[q];
                double fa = ud[q] * kn * djl[l] - dud[q] * jl[l];
                double fb = -u[q] * kn * djl[l] + du[q] * jl[l];
                zc il = (l % 4 == 0) ? 1.0 : (l % 4 == 1) ? I : (l % 4 == 2) ? -1.0 : -I;
                zc pre = 4.0 * M_PI / (w * sqrt(omega)) * il * phase;
                for (int m = -l; m <= l; ++m) {
                    int L = l * l + l + m;
                    zc c = pre * conj(y[L]);
                    A[(size_t)t * ld + off[a] + L] = c * fa;
                    B[(size_t)t * ld + off[a] + L] = c * fb;
                }
            }
        }
    }
    free(off);
}

/* ---------------------------------------------------------------------------------------
 * One block of S and H (section 2.3, eqs. def_overlap and def_hamilton):
 *   S_{t',t} = sum_a sum_L conj(A_{L,a,t'}) A_{L,a,t} + ||udot_{l,a}||^2 conj(B_{L,a,t'}) B_{L,a,t}
 *   H_{t',t} = sum_a sum_{L',L} conj(A_{L'}) T^AA_{L'L} A_L + conj(A_{L'}) T^AB_{L'L} B_L
 *                               + conj(B_{L'}) T^BA_{L'L} A_L + conj(B_{L'}) T^BB_{L'L} B_L
 * for bra columns (t') given by (Al, Bl) and ket columns (t) given by (Ar, Br); the output
 * blocks H, S are nr x nc, column-major.  The only reordering: for one ket column the
 * vector v_a = T_a [A_a; B_a] is formed once per atom before the bra sum.
 * T: per type a (2 nlmax) x (2 nlmax) matrix with leading dimension ldt, type stride
 * ldt * 2 nlmax, laid out as or_tmat writes it.
 * ------------------------------------------------------------------------------------- */
void or_hs_block(int n_atoms, const int *type, const int *lmax_t, int lstride, const double *ud_norm2,
                 const zc *T, int ldt, int nlmax, long krows, int nr, const zc *Al, const zc *Bl, long ldl,
                 int nc, const zc *Ar, const zc *Br, long ldr, zc *H, zc *S)
{
    long *off = (long *)malloc(sizeof(long) * (n_atoms + 1));
    off[0] = 0;
    for (int a = 0; a < n_atoms; ++a) off[a + 1] = off[a] + (long)(lmax_t[type[a]] + 1) * (lmax_t[type[a]] + 1);
    (void)krows;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nc; ++c) {
        const zc *ar = Ar + (size_t)c * ldr, *br = Br + (size_t)c * ldr;
        zc *va = (zc *)malloc(sizeof(zc) * (size_t)off[n_atoms]);
        zc *vb = (zc *)malloc(sizeof(zc) * (size_t)off[n_atoms]);
        for (int a = 0; a < n_atoms; ++a) {
            int ty = type[a], nl = (lmax_t[ty] + 1) * (lmax_t[ty] + 1);
            const zc *Tt = T + (size_t)ty * ldt * 2 * nlmax;
            for (int lp = 0; lp < nl; ++lp) {
                zc sa = 0.0, sb = 0.0;
                for (int l = 0; l < nl; ++l) {
                    zc x = ar[off[a] + l], yv = br[off[a] + l];
                    sa += Tt[(size_t)l * ldt + lp] * x + Tt[(size_t)(nl + l) * ldt + lp] * yv;
                    sb += Tt[(size_t)l * ldt + nl + lp] * x + Tt[(size_t)(nl + l) * ldt + nl + lp] * yv;
                }
                va[off[a] + lp] = sa;
                vb[off[a] + lp] = sb;
            }
        }
        for (int r = 0; r < nr; ++r) {
            const zc *al = Al + (size_t)r * ldl, *bl = Bl + (size_t)r * ldl;
            zc s = 0.0, h = 0.0;
            for (int a = 0; a < n_atoms; ++a) {
                int ty = type[a], lm = lmax_t[ty];
                for (int l = 0; l <= lm; ++l) {
                    double n2 = ud_norm2[ty * lstride + l];
                    for (int m = -l; m <= l; ++m) {
                        long q = off[a] + l * l + l + m;
                        s += conj(al[q]) * ar[q] + n2 * conj(bl[q]) * br[q];
                        h += conj(al[q]) * va[q] + conj(bl[q]) * vb[q];
                    }
                }
            }
            S[(size_t)c * nr + r] = s;
            H[(size_t)c * nr + r] = h;
        }
        free(va);
        free(vb);
    }
    free(off);
}

/* ---------------------------------------------------------------------------------------
 * Interstitial S and H of one block (section 2.3: eq. HS_Mat over the region outside the
 * muffin-tin spheres, where eq. basis_function makes every basis function the plane wave
 * exp(i K_t . r) / sqrt(Omega)):
 *   S^I_{t',t} = (1/Omega) int_{cell minus spheres} exp(i G . r) dr,   G = K_t - K_t'
 *             = delta_{G,0} - sum_a (1/Omega) int_{|r - x_a| < R_a} exp(i G . r) dr
 *             = delta_{G,0} - sum_a exp(i G . x_a) (4 pi R_a^3 / Omega) j_1(|G| R_a) / (|G| R_a)
 * (the cell integral of a plane wave of a reciprocal lattice vector G vanishes unless G = 0, and
 * the integral over a ball is 4 pi int_0^R j_0(|G| s) s^2 ds = 4 pi R^2 j_1(|G| R) / |G|, with the
 * limit 4 pi R^3 / 3 at G = 0).  The spheres must not overlap.
 *   H^I_{t',t} = (1/2 K_t' . K_t + v_int) S^I_{t',t}
 * (kinetic energy in the symmetric form (1/2) int grad conj(phi_t') . grad phi_t, and a constant
 * interstitial potential v_int).  Bra rows gr (nr x 3), ket columns gc (nc x 3), Cartesian G;
 * K = k + G.  Output blocks H, S: nr x nc, column-major.
 * ------------------------------------------------------------------------------------- */
void or_interstitial_block(int n_atoms, const int *type, const double *rmt, const double *pos, double omega,
                           double v_int, const double *kvec, int nr, const double *gr, int nc, const double *gc,
                           zc *H, zc *S)
{
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c) {
        for (int r = 0; r < nr; ++r) {
            double G[3], kb[3], kk[3];
            for (int i = 0; i < 3; ++i) {
                G[i] = gc[3 * c + i] - gr[3 * r + i];
                kb[i] = kvec[i] + gr[3 * r + i];
                kk[i] = kvec[i] + gc[3 * c + i];
            }
            double gn = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
            zc s = (gn == 0.0) ? 1.0 : 0.0;
            for (int a = 0; a < n_atoms; ++a) {
                double R = rmt[type[a]];
                double ball;                               /* (1/Omega) int over the ball at the origin */
                if (gn == 0.0) {
                    ball = 4.0 * M_PI * R * R * R / (3.0 * omega);
                } else {
                    double j[2], dj[2];
                    or_sph_bessel(1, gn * R, j, dj);
                    ball = 4.0 * M_PI * R * R * j[1] / (gn * omega);
                }
                double gx = G[0] * pos[3 * a] + G[1] * pos[3 * a + 1] + G[2] * pos[3 * a + 2];
                s -= cexp(I * gx) * ball;
            }
            double kin = 0.5 * (kb[0] * kk[0] + kb[1] * kk[1] + kb[2] * kk[2]);
            S[(size_t)c * nr + r] = s;
            H[(size_t)c * nr + r] = (kin + v_int) * s;
        }
    }
}

/* ---------------------------------------------------------------------------------------
 * Radial functions (section 2.2, eq. simp_Schr) and the non-spherical radial integrals
 * (appendix A.2, eq. nonsph_integrals), in Hartree atomic units (hbar = m = 1, so the
 * kinetic prefactor is 1/2):
 *     -1/2 P'' + [l(l+1) / (2 r^2) + V(r) - E] P = 0,        P = r u,
 * and its energy derivative Pd = dP/dE:
 *     -1/2 Pd'' + [l(l+1) / (2 r^2) + V(r) - E] Pd = P.
 * Mesh: r_i = r0 (R / r0)^(i / (n_r - 1)), i = 0..n_r-1, with n_r - 1 a multiple of 4.
 * In x = ln r the system for (P, D = dP/dr, Pd, Dd) reads
 *     dP/dx = r D,   dD/dx = [l(l+1)/r + 2 r (V - E)] P,
 *     dPd/dx = r Dd, dDd/dx = [l(l+1)/r + 2 r (V - E)] Pd - 2 r P,
 * integrated outward by classical Runge-Kutta (4th order) with step 2h, h = ln(R/r0)/(n_r-1),
 * so that every midpoint is a mesh point where V is given; results live on the even points.
 * Start at r0 with the regular behaviour P = r^(l+1) (1 - Z r / (l+1)), Z = -r0 V(r0), and
 * Pd = Dd = 0.  Integrals over [r0, R] by Simpson's rule on the even points in x (dr = r dx);
 * the piece below r0 is of order r0^3 and is left out.
 * Then u is normalised (integral of P^2 = 1) and udot made orthogonal to it (Pd -= <P,Pd> P).
 * Outputs on the even points (n_e = (n_r - 1)/2 + 1 values each): P, Pd; boundary values
 * out5 = {u(R), u'(R), udot(R), udot'(R), ||udot||^2} with u = P/r, u' = D/r - P/r^2.
 * ------------------------------------------------------------------------------------- */
static double simpson_even(int n_r, double r0, double R, const double *f_even)
{
    const int ne = (n_r - 1) / 2 + 1;
    const double h2 = 2.0 * log(R / r0) / (n_r - 1);
    double s = 0.0;
    for (int j = 0; j < ne; ++j) {
        const double r = r0 * exp(h2 * j);
        const double w = (j == 0 || j == ne - 1) ? 1.0 : ((j & 1) ? 4.0 : 2.0);
        s += w * f_even[j] * r;
    }
    return s * h2 / 3.0;
}

void or_radial(int n_r, double r0, double R, const double *v, int l, double e, double *P, double *Pd, double *out5)
{
    const int ne = (n_r - 1) / 2 + 1;
    const double h = log(R / r0) / (n_r - 1);
    const double ll = l * (l + 1.0);
    const double z = -r0 * v[0];
    double *D = (double *)malloc(sizeof(double) * ne), *Dd = (double *)malloc(sizeof(double) * ne);
    P[0] = pow(r0, l + 1) * (1.0 - z * r0 / (l + 1.0));
    D[0] = (l + 1.0) * pow(r0, l) - z * (l + 2.0) / (l + 1.0) * pow(r0, l + 1);
    Pd[0] = 0.0;
    Dd[0] = 0.0;
    for (int j = 0; j + 1 < ne; ++j) {
        /* RK4 from mesh point i = 2j (x) over 2h; midpoint i + 1, end i + 2 */
        double y[4] = {P[j], D[j], Pd[j], Dd[j]}, k[4][4];
        for (int s = 0; s < 4; ++s) {
            const int i = 2 * j + (s == 0 ? 0 : (s == 3 ? 2 : 1));
            const double r = r0 * exp(h * i);
            const double c = ll / r + 2.0 * r * (v[i] - e);
            double yy[4];
            for (int q = 0; q < 4; ++q) yy[q] = y[q] + (s == 0 ? 0.0 : (s == 3 ? 2.0 * h : h)) * (s == 0 ? 0.0 : k[s - 1][q]);
            k[s][0] = r * yy[1];
            k[s][1] = c * yy[0];
            k[s][2] = r * yy[3];
            k[s][3] = c * yy[2] - 2.0 * r * yy[0];
        }
        P[j + 1] = y[0] + 2.0 * h / 6.0 * (k[0][0] + 2.0 * k[1][0] + 2.0 * k[2][0] + k[3][0]);
        D[j + 1] = y[1] + 2.0 * h / 6.0 * (k[0][1] + 2.0 * k[1][1] + 2.0 * k[2][1] + k[3][1]);
        Pd[j + 1] = y[2] + 2.0 * h / 6.0 * (k[0][2] + 2.0 * k[1][2] + 2.0 * k[2][2] + k[3][2]);
        Dd[j + 1] = y[3] + 2.0 * h / 6.0 * (k[0][3] + 2.0 * k[1][3] + 2.0 * k[2][3] + k[3][3]);
    }
    double *f = (double *)malloc(sizeof(double) * ne);
    for (int j = 0; j < ne; ++j) f[j] = P[j] * P[j];
    const double nrm = 1.0 / sqrt(simpson_even(n_r, r0, R, f));
    for (int j = 0; j < ne; ++j) { P[j] *= nrm; D[j] *= nrm; Pd[j] *= nrm; Dd[j] *= nrm; }
    for (int j = 0; j < ne; ++j) f[j] = P[j] * Pd[j];
    const double c = simpson_even(n_r, r0, R, f);
    for (int j = 0; j < ne; ++j) { Pd[j] -= c * P[j]; Dd[j] -= c * D[j]; }
    for (int j = 0; j < ne; ++j) f[j] = Pd[j] * Pd[j];
    out5[4] = simpson_even(n_r, r0, R, f);
    out5[0] = P[ne - 1] / R;
    out5[1] = D[ne - 1] / R - P[ne - 1] / (R * R);
    out5[2] = Pd[ne - 1] / R;
    out5[3] = Dd[ne - 1] / R - Pd[ne - 1] / (R * R);
    free(f);
    free(D);
    free(Dd);
}

/* integral over [r0, R] of fa v fb dr with all three given on the even mesh points */
double or_radial_integral(int n_r, double r0, double R, const double *fa, const double *v_even, const double *fb)
{
    const int ne = (n_r - 1) / 2 + 1;
    double *f = (double *)malloc(sizeof(double) * ne);
    for (int j = 0; j < ne; ++j) f[j] = fa[j] * v_even[j] * fb[j];
    const double s = simpson_even(n_r, r0, R, f);
    free(f);
    return s;
}
