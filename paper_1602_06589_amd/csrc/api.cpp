// Host side of the C-ABI declared in include/flapw.h: argument validation, the handle's device
// work buffers, descriptor tables and kernel launches.  No arithmetic of the method runs here
// except the Gauss-Legendre nodes handed to the Gaunt quadrature kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "common.hpp"
#include "flapw.h"
#include "context.hpp"

using namespace flapw;

namespace {

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

flapw_status check_radial(flapw_handle h, const flapw_radial *rad)
{
    if (!rad) return fail(h, FLAPW_ERR_ARG, "radial descriptor is NULL");
    if (rad->n_types < 1 || rad->n_types > 32) return fail(h, FLAPW_ERR_ARG, "n_types must be in 1..32");
    if (!rad->lmax || !rad->rmt || !rad->u || !rad->du || !rad->ud || !rad->dud || !rad->ud_norm2 || !rad->e_l)
        return fail(h, FLAPW_ERR_ARG, "radial array pointer is NULL");
    int lm = 0;
    for (int t = 0; t < rad->n_types; ++t) {
        if (rad->lmax[t] < 0 || rad->lmax[t] > FLAPW_LMAX_CAP)
            return fail(h, FLAPW_ERR_ARG, "lmax out of range 0.." + std::to_string(FLAPW_LMAX_CAP));
        if (!(rad->rmt[t] > 0.0) || !std::isfinite(rad->rmt[t])) return fail(h, FLAPW_ERR_ARG, "rmt must be > 0");
        lm = std::max(lm, rad->lmax[t]);
    }
    if (rad->lstride < lm + 1) return fail(h, FLAPW_ERR_ARG, "lstride < max lmax + 1");
    const size_t n = (size_t)rad->n_types * rad->lstride;
    for (const double *p : {rad->u, rad->du, rad->ud, rad->dud, rad->ud_norm2, rad->e_l})
        if (!finite_all(p, n)) return fail(h, FLAPW_ERR_ARG, "non-finite radial data");
    for (int t = 0; t < rad->n_types; ++t)
        for (int l = 0; l <= rad->lmax[t]; ++l) {
            const int q = t * rad->lstride + l;
            const double a = rad->ud[q] * rad->du[q], b = rad->u[q] * rad->dud[q];
            const double w = a - b;
            if (!(std::fabs(w) > 1e-12 * std::max(std::fabs(a), std::fabs(b))) || w == 0.0)
                return fail(h, FLAPW_ERR_WRONSKIAN,
                            "Wronskian vanishes for type " + std::to_string(t) + ", l " + std::to_string(l));
        }
    return FLAPW_OK;
}

flapw_status check_atoms(flapw_handle h, const flapw_atoms *at, const flapw_radial *rad, bool need_geometry)
{
    if (!at) return fail(h, FLAPW_ERR_ARG, "atoms descriptor is NULL");
    if (at->n_atoms < 1) return fail(h, FLAPW_ERR_ARG, "n_atoms must be >= 1");
    if (!at->type) return fail(h, FLAPW_ERR_ARG, "atom type array is NULL");
    for (int a = 0; a < at->n_atoms; ++a)
        if (at->type[a] < 0 || at->type[a] >= rad->n_types) return fail(h, FLAPW_ERR_ARG, "atom type out of range");
    if (!need_geometry) return FLAPW_OK;
    if (!at->pos || !at->rot) return fail(h, FLAPW_ERR_ARG, "atom position/rotation array is NULL");
    if (!(at->omega > 0.0) || !std::isfinite(at->omega)) return fail(h, FLAPW_ERR_ARG, "omega must be > 0");
    if (!finite_all(at->pos, 3 * (size_t)at->n_atoms) || !finite_all(at->rot, 9 * (size_t)at->n_atoms))
        return fail(h, FLAPW_ERR_ARG, "non-finite atom data");
    for (int a = 0; a < at->n_atoms; ++a) {
        const double *R = at->rot + 9 * a;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += R[3 * i + k] * R[3 * j + k];
                if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-10)
                    return fail(h, FLAPW_ERR_ARG, "rotation of atom " + std::to_string(a) + " is not orthogonal");
            }
    }
    return FLAPW_OK;
}

flapw_status check_potential(flapw_handle h, const flapw_potential *pot, const flapw_radial *rad)
{
    if (!pot) return fail(h, FLAPW_ERR_ARG, "potential descriptor is NULL");
    if (pot->lpot < 0 || pot->lpot > FLAPW_LPOT_CAP)
        return fail(h, FLAPW_ERR_ARG, "lpot out of range 0.." + std::to_string(FLAPW_LPOT_CAP));
    if (!pot->i_uu || !pot->i_ud || !pot->i_du || !pot->i_dd) return fail(h, FLAPW_ERR_ARG, "integral array is NULL");
    const int ls = rad->lstride, nlp = (pot->lpot + 1) * (pot->lpot + 1);
    const size_t n = (size_t)rad->n_types * ls * ls * nlp;
    double mx = 0.0;
    for (const double *p : {pot->i_uu, pot->i_ud, pot->i_du, pot->i_dd}) {
        if (!finite_all(p, n)) return fail(h, FLAPW_ERR_ARG, "non-finite integrals");
        for (size_t i = 0; i < n; ++i) mx = std::max(mx, std::fabs(p[i]));
    }
    const double tol = 1e-12 * mx;
    auto at = [&](const double *p, int t, int lp, int l, int L) { return p[(((size_t)t * ls + lp) * ls + l) * nlp + L]; };
    for (int t = 0; t < rad->n_types; ++t)
        for (int lp = 0; lp <= rad->lmax[t]; ++lp)
            for (int l = 0; l <= rad->lmax[t]; ++l)
                for (int lpp = 0; lpp <= pot->lpot; ++lpp)
                    for (int m = -lpp; m <= lpp; ++m) {
                        const int L = lpp * lpp + lpp + m, Lm = lpp * lpp + lpp - m;
                        const double sg = (m & 1) ? -1.0 : 1.0;
                        for (const double *p : {pot->i_uu, pot->i_ud, pot->i_du, pot->i_dd})
                            if (std::fabs(at(p, t, lp, l, Lm) - sg * at(p, t, lp, l, L)) > tol)
                                return fail(h, FLAPW_ERR_NOT_HERMITIAN, "integrals violate I(l'',-m) = (-1)^m I(l'',m)");
                        if (std::fabs(at(pot->i_uu, t, lp, l, L) - at(pot->i_uu, t, l, lp, L)) > tol ||
                            std::fabs(at(pot->i_dd, t, lp, l, L) - at(pot->i_dd, t, l, lp, L)) > tol)
                            return fail(h, FLAPW_ERR_NOT_HERMITIAN, "I^{uu} or I^{udot udot} not symmetric in (l', l)");
                        if (std::fabs(at(pot->i_du, t, lp, l, L) - at(pot->i_ud, t, l, lp, L)) > tol)
                            return fail(h, FLAPW_ERR_NOT_HERMITIAN, "I^{udot u}(l', l) != I^{u udot}(l, l')");
                    }
    return FLAPW_OK;
}

// The interstitial region needs muffin-tin spheres that do not overlap (section 2.2): every pair
// of atoms (and every atom with its own images) at least R_a + R_b apart over the 27 nearest
// periodic images.  The lattice (rows a_1, a_2, a_3) must hold the cell volume omega.
flapw_status check_spheres(flapw_handle h, const flapw_atoms *at, const flapw_radial *rad, const double *lat)
{
    if (!lat) return fail(h, FLAPW_ERR_ARG, "NULL lattice");
    if (!finite_all(lat, 9)) return fail(h, FLAPW_ERR_ARG, "non-finite lattice");
    const double det = lat[0] * (lat[4] * lat[8] - lat[5] * lat[7]) - lat[1] * (lat[3] * lat[8] - lat[5] * lat[6]) +
                       lat[2] * (lat[3] * lat[7] - lat[4] * lat[6]);
    if (!(std::fabs(std::fabs(det) - at->omega) <= 1e-9 * at->omega))
        return fail(h, FLAPW_ERR_ARG, "|det(lattice)| does not match omega");
    for (int a = 0; a < at->n_atoms; ++a) {
        const double ra = rad->rmt[at->type[a]];
        for (int b = a; b < at->n_atoms; ++b) {
            const double rb = rad->rmt[at->type[b]];
            for (int n1 = -1; n1 <= 1; ++n1)
                for (int n2 = -1; n2 <= 1; ++n2)
                    for (int n3 = -1; n3 <= 1; ++n3) {
                        if (a == b && n1 == 0 && n2 == 0 && n3 == 0) continue;
                        double d2 = 0.0;
                        for (int c = 0; c < 3; ++c) {
                            const double d = at->pos[3 * b + c] - at->pos[3 * a + c] + n1 * lat[c] + n2 * lat[3 + c] +
                                             n3 * lat[6 + c];
                            d2 += d * d;
                        }
                        if (d2 < (ra + rb) * (ra + rb))
                            return fail(h, FLAPW_ERR_ARG, "muffin-tin spheres of atoms " + std::to_string(a) + " and " +
                                                              std::to_string(b) + " overlap");
                    }
        }
    }
    return FLAPW_OK;
}

// Host copies of the per-atom / per-type descriptors.
struct Layout {
    std::vector<AtomDev> atoms;
    std::vector<TypeDev> types;
    std::vector<int> atom_type, atom_nl2;
    std::vector<long long> atom_row;        // first row of [A_a; B_a] in the work layout
    std::vector<double> d;                  // S row weights of the work layout
    long long k = 0;                        // sum_a NL_a
    long long kp2 = 0;                      // padded 2K
    int nlmax = 0;
    // S through the addition theorem: atom positions, the row of each atom in the phase panel
    // (atoms grouped by type, each group padded to 16 rows), and the per-type row ranges
    std::vector<double> apos;
    std::vector<int> leg_row;
    std::vector<LegTypeRange> leg_ranges;
    std::vector<double> leg_un2;            // ||udot_l||^2 per type, stride kLStride
    long long ldE = 0;
};

// lcut >= 0: the rows of each atom stop at l = min(l_max, lcut) (the dense block of a structured T
// whose L-diagonal remainder is handled through the addition theorem); the types keep their l_max.
void build_layout(const flapw_atoms *at, const flapw_radial *rad, bool work_layout, Layout &L, int lcut = -1)
{
    const int na = at->n_atoms;
    L.atoms.resize(na);
    L.types.assign(rad->n_types, TypeDev{});
    L.atom_type.resize(na);
    L.atom_nl2.resize(na);
    L.atom_row.resize(na);
    int lm = 0;
    for (int t = 0; t < rad->n_types; ++t) {
        TypeDev &T = L.types[t];
        T.rmt = rad->rmt[t];
        T.lmax = rad->lmax[t];
        lm = std::max(lm, T.lmax);
        for (int l = 0; l <= T.lmax; ++l) {
            const int q = t * rad->lstride + l;
            RadialDev &r = T.rad[l];
            r.u = rad->u[q];
            r.du = rad->du[q];
            r.ud = rad->ud[q];
            r.dud = rad->dud[q];
            r.inv_w = 1.0 / (rad->ud[q] * rad->du[q] - rad->u[q] * rad->dud[q]);
            r.ud_norm2 = rad->ud_norm2[q];
        }
    }
    auto row_lmax = [&](int t) { return lcut >= 0 ? std::min(rad->lmax[t], lcut) : rad->lmax[t]; };
    if (lcut >= 0) lm = std::min(lm, lcut);
    L.nlmax = (lm + 1) * (lm + 1);
    long long off = 0;
    for (int a = 0; a < na; ++a) {
        const int t = at->type[a];
        const int nl = (row_lmax(t) + 1) * (row_lmax(t) + 1);
        AtomDev &A = L.atoms[a];
        for (int i = 0; i < 3; ++i) A.pos[i] = at->pos ? at->pos[3 * a + i] : 0.0;
        for (int i = 0; i < 9; ++i) A.rot[i] = at->rot ? at->rot[9 * a + i] : (i % 4 == 0 ? 1.0 : 0.0);
        A.type = t;
        A.nl = nl;
        if (work_layout) {
            A.rowA = 2 * off;
            A.rowB = 2 * off + nl;
        } else {
            A.rowA = off;
            A.rowB = off;
        }
        L.atom_type[a] = t;
        L.atom_nl2[a] = 2 * nl;
        L.atom_row[a] = 2 * off;
        off += nl;
    }
    L.k = off;
    L.kp2 = round_up(2 * off, kRowAlign);
    L.apos.resize(3 * (size_t)na);
    for (int a = 0; a < na; ++a)
        for (int i = 0; i < 3; ++i) L.apos[3 * a + i] = L.atoms[a].pos[i];
    L.leg_row.assign(na, 0);
    L.leg_ranges.assign(rad->n_types, LegTypeRange{0, 0, 0, 0});
    {
        int row = 0;
        for (int t = 0; t < rad->n_types; ++t) {
            int cnt = 0;
            for (int a = 0; a < na; ++a)
                if (at->type[a] == t) L.leg_row[a] = row + cnt++;
            const int rows = (int)round_up(cnt, kKTile);
            L.leg_ranges[t] = LegTypeRange{row, rows, rad->lmax[t], 0};
            row += rows;
        }
        L.ldE = std::max(row, kKTile);
    }
    L.leg_un2.assign((size_t)rad->n_types * kLStride, 0.0);
    for (int t = 0; t < rad->n_types; ++t)
        for (int l = 0; l <= rad->lmax[t]; ++l) L.leg_un2[(size_t)t * kLStride + l] = rad->ud_norm2[t * rad->lstride + l];
    L.d.assign(L.kp2, 0.0);
    for (int a = 0; a < na; ++a) {
        const int t = at->type[a], lmx = row_lmax(t);
        const long long r0 = L.atom_row[a];
        const int nl = L.atoms[a].nl;
        for (int l = 0; l <= lmx; ++l)
            for (int m = -l; m <= l; ++m) {
                const int Lq = l * l + l + m;
                L.d[r0 + Lq] = 1.0;
                L.d[r0 + nl + Lq] = rad->ud_norm2[t * rad->lstride + l];
            }
    }
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n from the usual cosine guesses).
void gauss_legendre(int n, std::vector<double> &z, std::vector<double> &w)
{
    z.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        z[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

// Host preparation of the T build: quadrature nodes and weights, integrals, E_l, ||udot||^2,
// l_max, and room for the Legendre table, packed into one buffer for one upload.
struct GauntPlan {
    int lt = 0, nq = 0, ls = 0, lpot = 0, n_types = 0, lnonsph = -1;
    size_t oz = 0, ow = 0, o1 = 0, o2 = 0, o3 = 0, o4 = 0, oe = 0, on = 0, ol = 0, oth = 0;
    bool sph = false;            // also the L-diagonal T terms per (type, l), at osph (full l_max at olf)
    size_t osph = 0, olf = 0;
};

// lnonsph >= 0: structured T; lcut >= 0: each type's row blocks stop at min(l_max, lcut), and the
// L-diagonal T terms of every l (needed for the rows past the cut) are formed on the device too.
void prepare_T(const flapw_radial *rad, const flapw_potential *pot, std::vector<unsigned char> &hb, GauntPlan &gp,
               int lnonsph = -1, int lcut = -1)
{
    gp.sph = lcut >= 0;
    gp.lnonsph = lnonsph;
    int lm = 0;
    for (int t = 0; t < rad->n_types; ++t) lm = std::max(lm, rad->lmax[t]);
    gp.lt = std::max(lm, pot->lpot);
    gp.nq = lm + pot->lpot + 2;                  // exact for polynomial degree <= 2 lmax + lpot
    gp.ls = rad->lstride;
    gp.lpot = pot->lpot;
    gp.n_types = rad->n_types;
    std::vector<double> z, w;
    gauss_legendre(gp.nq, z, w);
    const int nlp = (pot->lpot + 1) * (pot->lpot + 1);
    const size_t ni = (size_t)rad->n_types * gp.ls * gp.ls * nlp;
    hb.clear();
    gp.oz = put(hb, z.data(), z.size());
    gp.ow = put(hb, w.data(), w.size());
    gp.o1 = put(hb, pot->i_uu, ni);
    gp.o2 = put(hb, pot->i_ud, ni);
    gp.o3 = put(hb, pot->i_du, ni);
    gp.o4 = put(hb, pot->i_dd, ni);
    gp.oe = put(hb, rad->e_l, (size_t)rad->n_types * gp.ls);
    gp.on = put(hb, rad->ud_norm2, (size_t)rad->n_types * gp.ls);
    std::vector<int> lrow(rad->lmax, rad->lmax + rad->n_types);
    if (lcut >= 0)
        for (int &x : lrow) x = std::min(x, lcut);
    gp.ol = put(hb, lrow.data(), lrow.size());
    gp.olf = put(hb, rad->lmax, (size_t)rad->n_types);
    gp.oth = round_up(hb.size(), 256);
    const size_t nth = (size_t)(gp.lt + 1) * (gp.lt + 2) / 2 * gp.nq;
    hb.resize(gp.oth + nth * sizeof(double));
    gp.osph = round_up(hb.size(), 256);
    if (gp.sph) hb.resize(gp.osph + (size_t)rad->n_types * kLStride * 4 * sizeof(double));
}

flapw_status launch_T(flapw_handle h, const unsigned char *base, const GauntPlan &gp, double2 *T, long long ldt,
                      hipStream_t s)
{
    ProfScope prof(h, "tmat", s);
    hipError_t e = launch_legendre_table(gp.lt, gp.nq, (const double *)(base + gp.oz), (double *)(base + gp.oth), s);
    if (e != hipSuccess) return dev_fail(h, e, "legendre table kernel");
    e = launch_tmat(gp.n_types, (const int *)(base + gp.ol), gp.ls, gp.lpot, gp.nq, (const double *)(base + gp.ow),
                    (const double *)(base + gp.oth), (const double *)(base + gp.o1), (const double *)(base + gp.o2),
                    (const double *)(base + gp.o3), (const double *)(base + gp.o4), (const double *)(base + gp.oe),
                    (const double *)(base + gp.on), T, ldt, gp.lnonsph, s);
    if (e != hipSuccess) return dev_fail(h, e, "T assembly kernel");
    if (gp.sph) {
        e = launch_tmat_sph(gp.n_types, (const int *)(base + gp.olf), gp.ls, gp.lpot, gp.nq,
                            (const double *)(base + gp.ow), (const double *)(base + gp.oth),
                            (const double *)(base + gp.o1), (const double *)(base + gp.o2),
                            (const double *)(base + gp.o3), (const double *)(base + gp.o4),
                            (const double *)(base + gp.oe), (const double *)(base + gp.on),
                            (double *)(const_cast<unsigned char *>(base) + gp.osph), s);
        if (e != hipSuccess) return dev_fail(h, e, "spherical T terms kernel");
    }
    return FLAPW_OK;
}

// T of all types into dev (ldt x ldt each).
flapw_status build_T_impl(flapw_handle h, const flapw_radial *rad, const flapw_potential *pot, double2 *T, long long ldt,
                          hipStream_t s)
{
    GauntPlan gp;
    prepare_T(rad, pot, h->host_gaunt, gp, h->lnonsph);
    flapw_status st = upload(h, h->gaunt, h->host_gaunt, s);
    if (st != FLAPW_OK) return st;
    return launch_T(h, (const unsigned char *)h->gaunt.p, gp, T, ldt, s);
}

// Upper-triangle tile list of several problems, ordered in bands of kBand tile rows (so that
// work-groups running together share operand panels) and remapped so that each of the eight
// XCDs (work-group b runs on XCD b % 8) receives a contiguous run of that order.  With mats = 2
// (split precision) every (ti, tj) gives an S tile and an H tile next to each other.
// Tiles (prob, ti <= tj, m) for m in [m0, m1) (split precision: 0 = S, 1 = H), in bands of kBand
// tile rows, then dealt round-robin over the 8 XCDs so that neighbours in the band order run on
// the same XCD (and share its L2).
void xcd_interleave(const std::vector<TileDev> &order, std::vector<TileDev> &out);

void build_tiles(const std::vector<int> &np_tiles, int m0, int m1, std::vector<TileDev> &out, int kBand = 4)
{
    std::vector<TileDev> order;
    for (int p = 0; p < (int)np_tiles.size(); ++p) {
        const int nt = np_tiles[p];
        for (int b0 = 0; b0 < nt; b0 += kBand)
            for (int tj = b0; tj < nt; ++tj)
                for (int ti = b0; ti < std::min(b0 + kBand, tj + 1); ++ti)
                    for (int m = m0; m < m1; ++m) order.push_back(TileDev{p, ti, tj, m});
    }
    xcd_interleave(order, out);
}

// Blocks of the modular contraction: rows 256 I .. 256 I + 255 (128-row tiles 2I, 2I + 1) by
// columns 128 J .. 128 J + 127, for the upper triangle (2I <= J); nc_tiles counts the 128-column
// tiles that hold columns, ceil(n / 128), so that a tile of padding columns only (the residue
// planes are 256-column aligned) costs no block.  Bands of kBand block rows walk the columns, as in
// build_tiles.
void build_mod_tiles(const std::vector<int> &nc_tiles, int m0, int m1, std::vector<TileDev> &out, int kBand)
{
    std::vector<TileDev> order;
    for (int p = 0; p < (int)nc_tiles.size(); ++p) {
        const int nt = nc_tiles[p], nb = (nt + 1) / 2;
        for (int b0 = 0; b0 < nb; b0 += kBand)
            for (int tj = 2 * b0; tj < nt; ++tj)
                for (int bi = b0; bi < std::min(b0 + kBand, tj / 2 + 1); ++bi)
                    for (int m = m0; m < m1; ++m) order.push_back(TileDev{p, bi, tj, m});
    }
    xcd_interleave(order, out);
}

// Consecutive work-groups go to the 8 XCDs in turn: give XCD x the x-th contiguous eighth of the
// ordered list, so neighbouring tiles (which share panels) meet in one L2.
void xcd_interleave(const std::vector<TileDev> &order, std::vector<TileDev> &out)
{
    const int n = (int)order.size();
    out.resize(n);
    const int q = n / 8, rem = n % 8;
    int start[9];
    start[0] = 0;
    for (int x = 0; x < 8; ++x) start[x + 1] = start[x] + q + (x < rem ? 1 : 0);
    for (int b = 0; b < n; ++b) out[b] = order[start[b % 8] + b / 8];
}

int default_slices(flapw_prec prec) { return prec == FLAPW_PREC_SPLIT_I8_MOD ? 11 : 6; }

// Precision and digit (modulus) count of a call: FLAPW_ERR_ARG for an unknown precision or a count
// outside 0..FLAPW_MODULI_CAP, FLAPW_ERR_UNSUPPORTED for a count the precision does not implement.
flapw_status check_prec(flapw_handle h, flapw_prec prec, int slices)
{
    if (prec == FLAPW_PREC_SPLIT_FP32)
        return fail(h, FLAPW_ERR_UNSUPPORTED,
                    "FP32 slices are not implemented: FP32 accumulation over the contraction cannot reach 1e-10");
    if (prec != FLAPW_PREC_FP64 && prec != FLAPW_PREC_SPLIT_BF16 && prec != FLAPW_PREC_SPLIT_I8 &&
        prec != FLAPW_PREC_SPLIT_I8_MOD)
        return fail(h, FLAPW_ERR_ARG, "unknown precision");
    if (prec == FLAPW_PREC_SPLIT_I8_MOD) {
        if (slices < 0 || slices > FLAPW_MODULI_CAP) return fail(h, FLAPW_ERR_ARG, "modulus count out of range");
        if (slices != 0 && slices < kModMin)
            return fail(h, FLAPW_ERR_UNSUPPORTED, "modular split precision supports 8..14 moduli");
        return FLAPW_OK;
    }
    if (slices < 0 || slices > FLAPW_SLICES_CAP) return fail(h, FLAPW_ERR_ARG, "slices out of range");
    if (prec != FLAPW_PREC_FP64 && slices != 0 && (slices < 3 || slices > 6))
        return fail(h, FLAPW_ERR_UNSUPPORTED, "split precision supports 3..6 digits");
    return FLAPW_OK;
}

// bytes per digit: int8 digits 1, bf16 digits 2
int digit_bytes(flapw_prec prec) { return prec == FLAPW_PREC_SPLIT_BF16 ? 2 : 1; }

// The tuner's choice for (prec, padded contraction rows, S method, lnonsph), or NULL.
const flapw_context::Tuned *find_tuned(flapw_handle h, flapw_prec prec, long long kp2, int s_method, int lnonsph)
{
    for (const auto &t : h->tuned)
        if (t.prec == (int)prec && t.kp2 == kp2 && t.s_method == s_method && t.lnonsph == lnonsph) return &t;
    return nullptr;
}

// The tuner accepts a digit or modulus count whose estimated whole-matrix errors are at most this
// fraction of the tolerance (room for the k-points it does not sample, whose errors grow like the
// square root of their basis size).
constexpr double kTuneMargin = 2.0 / 3.0;

// slices == 0: the tuned digit count for the key, else the library default
int effective_slices(flapw_handle h, flapw_prec prec, long long kp2, int s_method, int lnonsph, int slices)
{
    if (prec == FLAPW_PREC_FP64) return 0;
    if (slices) return slices;
    const auto *t = find_tuned(h, prec, kp2, s_method, lnonsph);
    return t && t->slices ? t->slices : default_slices(prec);
}

int effective_band(flapw_handle h, flapw_prec prec, long long kp2, int s_method, int lnonsph)
{
    const auto *t = find_tuned(h, prec, kp2, s_method, lnonsph);
    return t ? t->band : 4;
}

// 16-row chunks per LDS stage of the modular contraction: the tuned count, else 4 (64-row stages;
// the environment variable FLAPW_MOD_STAGE_ROWS = 32 selects 32-row stages instead)
int effective_chunks(flapw_handle h, flapw_prec prec, long long kp2, int s_method, int lnonsph)
{
    const auto *t = find_tuned(h, prec, kp2, s_method, lnonsph);
    if (t && t->chunks) return t->chunks;
    const char *env = std::getenv("FLAPW_MOD_STAGE_ROWS");
    return env && std::atoi(env) == 32 ? 2 : 4;
}

// Digit storage of one problem inside a digit buffer.
struct DigitArea {
    int8_t *L, *RS, *RH;
    int *eL, *eRS, *eRH;
};

long long digit_area_bytes(long long kp2, long long np, int s, int eb)
{
    const long long one = round_up(2LL * s * kp2 * np * eb, 256);
    return 3 * one + 3 * round_up(np * 4, 256);
}

DigitArea digit_area(void *base, long long kp2, long long np, int s, int eb)
{
    const long long one = round_up(2LL * s * kp2 * np * eb, 256);
    const long long ex = round_up(np * 4, 256);
    unsigned char *b = (unsigned char *)base;
    return DigitArea{(int8_t *)b, (int8_t *)(b + one), (int8_t *)(b + 2 * one), (int *)(b + 3 * one),
                     (int *)(b + 3 * one + ex), (int *)(b + 3 * one + 2 * ex)};
}

// Residue storage of one problem of the modular path: planes of P, d.P and Q (npm columns,
// np rounded up to 256 = two 128-column tiles, the row extent of a contraction block), their
// column exponents, and the residue tiles.
struct ModArea {
    int8_t *L, *RS, *RH;
    double *sL, *sRS, *sRH;
    int8_t *res;
    long long npm;
};

long long mod_area_bytes(long long kp2, long long np, int nm)
{
    const long long npm = round_up(np, 2 * kModTile);
    return 3 * round_up(mod_digit_bytes(kp2, npm, nm), 256) + 3 * round_up(npm * 8, 256) +
           round_up(mod_scratch_bytes(npm, nm), 256);
}

ModArea mod_area(void *base, long long kp2, long long np, int nm)
{
    const long long npm = round_up(np, 2 * kModTile);
    const long long one = round_up(mod_digit_bytes(kp2, npm, nm), 256), ex = round_up(npm * 8, 256);
    unsigned char *b = (unsigned char *)base;
    return ModArea{(int8_t *)b,
                   (int8_t *)(b + one),
                   (int8_t *)(b + 2 * one),
                   (double *)(b + 3 * one),
                   (double *)(b + 3 * one + ex),
                   (double *)(b + 3 * one + 2 * ex),
                   (int8_t *)(b + 3 * one + 3 * ex),
                   npm};
}

ModProblemDev mod_problem(const ModArea &ma, double2 *H, double2 *S, long long ldh, int n, long long kp2)
{
    const long long t = ma.npm / kModTile;
    return ModProblemDev{ma.L, ma.RS, ma.RH, ma.sL, ma.sRS, ma.sRH, H, S, ma.res, ldh, n, (int)kp2,
                         (int)(ma.npm / 32), (int)(t * (t + 1) / 2)};
}

flapw_status mod_slice_problem(flapw_handle h, const ProblemDev &pb, long long np, const ModArea &ma,
                               const ModTable &mt, bool with_s, const double *part, long long n_slots, hipStream_t st)
{
    ProfScope prof(h, "slice", st);
    hipError_t e = launch_mod_slice(pb.P, pb.Q, pb.d, pb.ldp, pb.kp2, (int)np, (int)ma.npm, mt, ma.sL, ma.sRS, ma.sRH,
                                    ma.L, ma.RS, ma.RH, with_s, part, n_slots, st);
    if (e != hipSuccess) return dev_fail(h, e, "residue slicing kernels");
    return FLAPW_OK;
}

// Modular contraction of a batch: residues per (256 x 128 block, modulus), then the CRT
// reconstruction per 128 x 128 tile.
hipError_t launch_mod_pair(flapw_handle h, const ModProblemDev *probs, const TileDev *blocks, int n_blocks,
                           const TileDev *tiles, int n_tiles, const ModTable &mt, int chunks, hipStream_t st)
{
    hipError_t e;
    {
        ProfScope prof(h, "hs_mod", st);
        e = launch_mod_contract(probs, blocks, n_blocks, mt, chunks, st);
    }
    if (e != hipSuccess) return e;
    ProfScope prof(h, "mod_crt", st);
    return launch_mod_crt(probs, tiles, n_tiles, mt, st);
}

flapw_status slice_problem(flapw_handle h, const ProblemDev &pb, long long np, int s, const DigitArea &da, bool bf16,
                           hipStream_t st)
{
    ProfScope prof(h, "slice", st);
    hipError_t e = bf16 ? launch_split_bf16_slice(pb.P, pb.Q, pb.d, pb.ldp, pb.kp2, (int)np, s, da.eL, da.eRS, da.eRH,
                                                  da.L, da.RS, da.RH, st)
                        : launch_split_slice(pb.P, pb.Q, pb.d, pb.ldp, pb.kp2, (int)np, s, da.eL, da.eRS, da.eRH, da.L,
                                             da.RS, da.RH, st);
    if (e != hipSuccess) return dev_fail(h, e, "digit slicing kernels");
    return FLAPW_OK;
}

hipError_t launch_split_any(bool bf16, const SplitProblemDev *probs, const TileDev *tiles, int n_tiles, int s,
                            hipStream_t st)
{
    return bf16 ? launch_split_bf16_contract(probs, tiles, n_tiles, s, st)
                : launch_split_contract(probs, tiles, n_tiles, s, st);
}

flapw_status run_split(flapw_handle h, const std::vector<SplitProblemDev> &probs, const std::vector<int> &npt, int s,
                       int band, bool bf16, hipStream_t st)
{
    std::vector<TileDev> tiles;
    build_tiles(npt, 0, 2, tiles, band);
    auto &hb = h->host_sdesc;
    hb.clear();
    const size_t op = put(hb, probs.data(), probs.size());
    const size_t ot = put(hb, tiles.data(), tiles.size());
    flapw_status r = upload(h, h->sdesc, hb, st);
    if (r != FLAPW_OK) return r;
    unsigned char *base = (unsigned char *)h->sdesc.p;
    ProfScope prof(h, "hs_split", st);
    hipError_t e = launch_split_any(bf16, (const SplitProblemDev *)(base + op), (const TileDev *)(base + ot),
                                    (int)tiles.size(), s, st);
    if (e != hipSuccess) return dev_fail(h, e, "S/H split-precision kernel");
    return FLAPW_OK;
}

// FP64 contraction stage for a batch of problems whose P and Q are in the work buffer.
flapw_status run_fp64(flapw_handle h, const std::vector<ProblemDev> &probs_in, const std::vector<int> &npt, int band,
                      hipStream_t s)
{
    std::vector<TileDev> tiles;
    build_tiles(npt, 0, 1, tiles, band);
    auto &hb = h->host_tiles;
    hb.clear();
    const size_t op = put(hb, probs_in.data(), probs_in.size());
    const size_t ot = put(hb, tiles.data(), tiles.size());
    flapw_status st = upload(h, h->tiles, hb, s);
    if (st != FLAPW_OK) return st;
    unsigned char *base = (unsigned char *)h->tiles.p;
    ProfScope prof(h, "hs_fp64", s);
    hipError_t e = launch_hs_fp64((const ProblemDev *)(base + op), (const TileDev *)(base + ot), (int)tiles.size(), true, s);
    if (e != hipSuccess) return dev_fail(h, e, "S/H FP64 kernel");
    return FLAPW_OK;
}


// ----------------------------------------------------------------------------- S/H generation plans

// Everything one S/H generation over n_k k-points launches.  prepare_generate validates nothing
// (callers do), sizes and allocates the device buffers, and uploads every descriptor;
// enqueue_generate only launches kernels, so it can also be captured into a HIP graph.
struct GenBatch {
    int i0 = 0, i1 = 0;          // k-points [i0, i1)
    size_t o_probs = 0, o_tiles = 0;
    int n_tiles = 0;
    size_t o_ctiles = 0;         // modular path: 128 x 128 tiles of the reconstruction
    int n_ctiles = 0;
};

struct GenPlan {
    Layout L;
    int n_k = 0;
    bool split = false;
    bool leg = false;            // S through the addition theorem; the contraction computes H only
    bool inter = false;          // add the interstitial terms after the muffin-tin parts
    double v_int = 0.0;
    bool bf16 = false;           // split digits in bf16 (else int8)
    bool mod = false;            // modular split precision (residues mod p_m, CRT)
    ModTable mt{};               // its moduli (mod only)
    int lnonsph = -1;            // structured T (-1: dense T)
    int lh0 = 1 << 20;           // the Legendre kernel adds to H the L-diagonal terms of l >= lh0
    double omega = 0.0;
    int sl = 0, band = 4;
    int chunks = 4;              // modular contraction: 16-row chunks per LDS stage
    long long ldt = 0;
    double pref = 0.0;
    int n_atoms = 0, n_types = 0;
    std::vector<double> kv;
    std::vector<const double *> g;
    std::vector<int> ng;
    std::vector<long long> np;
    std::vector<flapw_z *> S, H;
    std::vector<long long> ldh;
    std::vector<size_t> off;     // per k-point: byte offset of its P/Q (FP64) or digits (split)
    GauntPlan gp;
    size_t oa = 0, ot = 0, od = 0, oty = 0, onl = 0, orow = 0;
    size_t oapos = 0, olrow = 0, olrng = 0, oun2 = 0;        // Legendre tables
    std::vector<size_t> o_stiles;                            // Legendre S tiles of each k-point
    std::vector<int> n_stiles;
    std::vector<GenBatch> batches;
    double2 *T = nullptr;
    unsigned char *tables = nullptr, *gaunt = nullptr, *desc = nullptr, *work = nullptr, *digits = nullptr;
    double *part = nullptr;      // modular split: column-sum shares of the panel kernel (in work)
    long long n_slots = 0;       // their (atom, row tile) slots
    unsigned char *legbuf = nullptr;                         // khat, ab, E of one k-point
    size_t leg_ab = 0, leg_E = 0;                            // byte offsets inside `leg`
};

struct GenBuffers {
    DevBuf *tmat, *tables, *gaunt, *desc, *work, *digits, *leg;
    std::vector<unsigned char> *h_tables, *h_gaunt, *h_desc;
};

// Legendre scratch of one k-point with np columns: khat, ab, E (each 256-byte aligned).
size_t leg_bytes(const Layout &L, long long np, int n_types, size_t *o_ab, size_t *o_E)
{
    const size_t khat = round_up(np * 32, 256);
    const size_t ab = round_up((long long)n_types * kLStride * np * 16, 256);
    *o_ab = khat;
    *o_E = khat + ab;
    return khat + ab + round_up(np * L.ldE * 16, 256);
}

// Upper-triangle tile list (ti, tj) of an np x np matrix for the Legendre S kernel.
void s_tiles(long long np, std::vector<int> &out)
{
    const int nt = (int)(np / kTile);
    out.clear();
    for (int tj = 0; tj < nt; ++tj)
        for (int ti = 0; ti <= tj; ++ti) {
            out.push_back(ti);
            out.push_back(tj);
        }
}

flapw_status put_device(flapw_handle h, DevBuf &dst, const std::vector<unsigned char> &src, hipStream_t s, bool sync)
{
    hipError_t e = dst.ensure(src.size());
    if (e != hipSuccess) return dev_fail(h, e, "allocating descriptor buffer");
    e = sync ? hipMemcpy(dst.p, src.data(), src.size(), hipMemcpyHostToDevice)
             : hipMemcpyAsync(dst.p, src.data(), src.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return dev_fail(h, e, "uploading descriptors");
    return FLAPW_OK;
}

flapw_status prepare_generate(flapw_handle h, int n_k, const double *k, const int *n_g, const double *const *g,
                              const flapw_atoms *at, const flapw_radial *rad, const flapw_potential *pot,
                              flapw_z *const *H, flapw_z *const *S, const long *ldh, flapw_prec prec, int slices,
                              int band, bool leg, GenBuffers &b, GenPlan &p, hipStream_t s, bool sync_upload)
{
    Layout &L = p.L;
    p.lnonsph = h->lnonsph;
    int lmx = 0;
    for (int t = 0; t < rad->n_types; ++t) lmx = std::max(lmx, rad->lmax[t]);
    // With S from the addition theorem and a structured T, the contraction covers only the dense
    // block (rows l <= lnonsph); the L-diagonal remainder joins the Legendre kernel.
    const int lcut = (leg && p.lnonsph >= 0 && p.lnonsph < lmx) ? p.lnonsph : -1;
    p.lh0 = lcut >= 0 ? lcut + 1 : (1 << 20);
    build_layout(at, rad, true, L, lcut);
    p.n_k = n_k;
    p.leg = leg;
    p.inter = h->inter;
    p.v_int = h->v_int;
    p.omega = at->omega;
    p.n_atoms = at->n_atoms;
    p.n_types = rad->n_types;
    p.split = prec != FLAPW_PREC_FP64;
    p.bf16 = prec == FLAPW_PREC_SPLIT_BF16;
    p.mod = prec == FLAPW_PREC_SPLIT_I8_MOD;
    const int smeth = leg ? (int)FLAPW_S_LEGENDRE : (int)FLAPW_S_GEMM;
    p.sl = effective_slices(h, prec, L.kp2, smeth, p.lnonsph, slices);
    if (p.mod) p.mt = make_mod_table(p.sl);
    p.band = band ? band : effective_band(h, prec, L.kp2, smeth, p.lnonsph);
    p.chunks = effective_chunks(h, prec, L.kp2, smeth, p.lnonsph);
    p.ldt = 2LL * L.nlmax;
    p.pref = 4.0 * kPi / std::sqrt(at->omega);
    p.kv.assign(k, k + 3 * (size_t)n_k);
    p.g.assign(g, g + n_k);
    p.ng.assign(n_g, n_g + n_k);
    p.S.assign(S, S + n_k);
    p.H.assign(H, H + n_k);
    p.ldh.assign(ldh, ldh + n_k);
    p.np.resize(n_k);
    for (int i = 0; i < n_k; ++i) p.np[i] = round_up(n_g[i], kTile);

    hipError_t e = b.tmat->ensure((size_t)rad->n_types * p.ldt * p.ldt * sizeof(double2));
    if (e != hipSuccess) return dev_fail(h, e, "allocating T");
    p.T = (double2 *)b.tmat->p;
    prepare_T(rad, pot, *b.h_gaunt, p.gp, p.lnonsph, lcut);
    flapw_status st = put_device(h, *b.gaunt, *b.h_gaunt, s, sync_upload);
    if (st != FLAPW_OK) return st;
    p.gaunt = (unsigned char *)b.gaunt->p;

    auto &ht = *b.h_tables;
    ht.clear();
    p.oa = put(ht, L.atoms.data(), L.atoms.size());
    p.ot = put(ht, L.types.data(), L.types.size());
    p.od = put(ht, L.d.data(), L.d.size());
    p.oty = put(ht, L.atom_type.data(), L.atom_type.size());
    p.onl = put(ht, L.atom_nl2.data(), L.atom_nl2.size());
    p.orow = put(ht, L.atom_row.data(), L.atom_row.size());
    p.oapos = put(ht, L.apos.data(), L.apos.size());
    p.olrow = put(ht, L.leg_row.data(), L.leg_row.size());
    p.olrng = put(ht, L.leg_ranges.data(), L.leg_ranges.size());
    p.oun2 = put(ht, L.leg_un2.data(), L.leg_un2.size());
    if ((st = put_device(h, *b.tables, ht, s, sync_upload)) != FLAPW_OK) return st;
    p.tables = (unsigned char *)b.tables->p;

    // Memory batches.  FP64: P and Q of every k-point of a batch stay resident for one grouped
    // contraction launch.  Split precision: the FP64 panels of one k-point at a time are cut into
    // digits (the panels are reused), and the digits of every k-point of a batch stay resident.
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return dev_fail(h, e, "hipMemGetInfo");
    double frac = 0.55;
    if (const char *env = std::getenv("FLAPW_WORK_FRACTION")) frac = std::atof(env);
    long long np_max = 0;
    for (int i = 0; i < n_k; ++i) np_max = std::max(np_max, p.np[i]);
    // split: one k-point's P and Q; modular split also the column-sum shares after them
    const size_t panel_pq = (size_t)2 * L.kp2 * np_max * sizeof(double2);
    const size_t panel_one =
        panel_pq + (p.mod ? (size_t)round_up(qpanel_colsum_doubles(p.ldt, p.n_atoms, np_max) * 8, 256) : 0);
    size_t budget = (size_t)(frac * (double)total_b);
    // never more than the device holds now: free memory plus this call's own work and digit
    // buffers, which are freed and allocated again when they must grow (10 % held back for the
    // rest); other handles and the caller's tensors then only make the batches smaller, which
    // leaves the results unchanged
    const size_t avail = free_b + b.work->n + (p.split ? b.digits->n : 0);
    budget = std::min(budget, (size_t)(0.9 * (double)avail));
    if (p.split) budget = budget > panel_one ? budget - panel_one : 0;
    std::vector<size_t> need(n_k);
    for (int i = 0; i < n_k; ++i)
        need[i] = p.mod     ? (size_t)mod_area_bytes(L.kp2, p.np[i], p.sl)
                  : p.split ? (size_t)digit_area_bytes(L.kp2, p.np[i], p.sl, p.bf16 ? 2 : 1)
                            : (size_t)2 * L.kp2 * p.np[i] * sizeof(double2);
    p.off.assign(n_k, 0);
    size_t biggest = 0;
    for (int i0 = 0; i0 < n_k;) {
        GenBatch bt;
        bt.i0 = i0;
        int i1 = i0;
        size_t tot = 0;
        while (i1 < n_k && (i1 == i0 || tot + need[i1] <= budget)) {
            p.off[i1] = tot;
            tot += need[i1++];
        }
        bt.i1 = i1;
        biggest = std::max(biggest, tot);
        p.batches.push_back(bt);
        i0 = i1;
    }
    if (p.split) {
        if ((e = b.work->ensure(panel_one)) != hipSuccess) return dev_fail(h, e, "allocating work buffer");
        if ((e = b.digits->ensure(biggest)) != hipSuccess) return dev_fail(h, e, "allocating digit buffer");
        p.digits = (unsigned char *)b.digits->p;
    } else {
        if ((e = b.work->ensure(biggest)) != hipSuccess) return dev_fail(h, e, "allocating work buffer");
    }
    p.work = (unsigned char *)b.work->p;
    if (p.mod) {
        p.part = (double *)(p.work + panel_pq);
        p.n_slots = (long long)qpanel_row_tiles(p.ldt) * p.n_atoms;
    }
    if (p.leg || p.inter) {
        const size_t lb = leg_bytes(L, np_max, p.n_types, &p.leg_ab, &p.leg_E);
        if ((e = b.leg->ensure(lb)) != hipSuccess) return dev_fail(h, e, "allocating Legendre scratch");
        p.legbuf = (unsigned char *)b.leg->p;
    }

    // contraction descriptors of every batch
    auto &hd = *b.h_desc;
    hd.clear();
    if (p.leg || p.inter) {
        p.o_stiles.resize(n_k);
        p.n_stiles.resize(n_k);
        std::vector<int> tl;
        for (int i = 0; i < n_k; ++i) {
            s_tiles(p.np[i], tl);
            p.o_stiles[i] = put(hd, tl.data(), tl.size());
            p.n_stiles[i] = (int)tl.size() / 2;
        }
    }
    for (auto &bt : p.batches) {
        std::vector<int> npt;
        std::vector<ProblemDev> probs;
        std::vector<SplitProblemDev> sprobs;
        std::vector<ModProblemDev> mprobs;
        for (int i = bt.i0; i < bt.i1; ++i) {
            if (p.mod) {
                const ModArea ma = mod_area(p.digits + p.off[i], L.kp2, p.np[i], p.sl);
                npt.push_back((int)((n_g[i] + kModTile - 1) / kModTile));   // tiles holding columns
                mprobs.push_back(mod_problem(ma, (double2 *)H[i], (double2 *)S[i], (long long)ldh[i], n_g[i], L.kp2));
                continue;
            }
            npt.push_back((int)(p.np[i] / kTile));
            if (p.split) {
                const DigitArea da = digit_area(p.digits + p.off[i], L.kp2, p.np[i], p.sl, p.bf16 ? 2 : 1);
                sprobs.push_back(SplitProblemDev{da.L, da.RS, da.RH, da.eL, da.eRS, da.eRH, (double2 *)H[i],
                                                 (double2 *)S[i], (long long)ldh[i], n_g[i], (int)L.kp2});
            } else {
                double2 *P = (double2 *)(p.work + p.off[i]);
                probs.push_back(ProblemDev{P, P + L.kp2 * p.np[i], (const double *)(p.tables + p.od), (double2 *)H[i],
                                           (double2 *)S[i], L.kp2, (long long)ldh[i], n_g[i], (int)L.kp2});
            }
        }
        std::vector<TileDev> tiles;
        if (p.mod) {
            std::vector<TileDev> ctiles;
            build_mod_tiles(npt, p.leg ? 1 : 0, 2, tiles, p.band);
            build_tiles(npt, p.leg ? 1 : 0, 2, ctiles, p.band);
            bt.o_ctiles = put(hd, ctiles.data(), ctiles.size());
            bt.n_ctiles = (int)ctiles.size();
        } else if (p.split) {
            build_tiles(npt, p.leg ? 1 : 0, 2, tiles, p.band);
        } else {
            build_tiles(npt, 0, 1, tiles, p.band);
        }
        bt.o_probs = p.mod     ? put(hd, mprobs.data(), mprobs.size())
                     : p.split ? put(hd, sprobs.data(), sprobs.size())
                               : put(hd, probs.data(), probs.size());
        bt.o_tiles = put(hd, tiles.data(), tiles.size());
        bt.n_tiles = (int)tiles.size();
    }
    if ((st = put_device(h, *b.desc, hd, s, sync_upload)) != FLAPW_OK) return st;
    p.desc = (unsigned char *)b.desc->p;
    return FLAPW_OK;
}

// S of k-point i through the addition theorem (prep kernel, then the tile kernel).
flapw_status enqueue_s_legendre(flapw_handle h, const GenPlan &p, int i, double2 *S, long long lds, hipStream_t s)
{
    const Layout &L = p.L;
    double *khat = (double *)p.legbuf, *ab = (double *)(p.legbuf + p.leg_ab);
    double2 *E = (double2 *)(p.legbuf + p.leg_E);
    hipError_t e;
    {
        ProfScope prof(h, "leg_prep", s);
        e = launch_legendre_prep(p.kv.data() + 3 * i, p.ng[i], (int)p.np[i], p.g[i], (const TypeDev *)(p.tables + p.ot),
                                 p.n_types, (const double *)(p.tables + p.oapos), (const int *)(p.tables + p.olrow),
                                 p.n_atoms, khat, ab, E, L.ldE, s);
    }
    if (e != hipSuccess) return dev_fail(h, e, "Legendre preparation kernel");
    {
        ProfScope prof(h, "s_legendre", s);
        const bool with_h = p.lh0 < (1 << 20) && !p.H.empty();
        e = launch_s_legendre(khat, ab, E, L.ldE, (const LegTypeRange *)(p.tables + p.olrng), p.n_types,
                              (const int *)(p.desc + p.o_stiles[i]), p.n_stiles[i], (int)p.np[i], p.ng[i],
                              4.0 * kPi / p.omega, S, lds, (const double *)(p.tables + p.oun2),
                              with_h ? (const double *)(p.gaunt + p.gp.osph) : nullptr,
                              p.lh0, with_h ? (double2 *)p.H[i] : nullptr, with_h ? (long long)p.ldh[i] : 0, s);
    }
    if (e != hipSuccess) return dev_fail(h, e, "Legendre S kernel");
    return FLAPW_OK;
}

// Interstitial terms of k-point i added to its H and S; with prep the phases E are formed first
// (the addition-theorem path has formed them already).
flapw_status enqueue_interstitial(flapw_handle h, const GenPlan &p, int i, bool prep, hipStream_t s)
{
    const Layout &L = p.L;
    double *khat = (double *)p.legbuf, *ab = (double *)(p.legbuf + p.leg_ab);
    double2 *E = (double2 *)(p.legbuf + p.leg_E);
    hipError_t e = hipSuccess;
    if (prep) {
        ProfScope prof(h, "leg_prep", s);
        e = launch_legendre_prep(p.kv.data() + 3 * i, p.ng[i], (int)p.np[i], p.g[i], (const TypeDev *)(p.tables + p.ot),
                                 p.n_types, (const double *)(p.tables + p.oapos), (const int *)(p.tables + p.olrow),
                                 p.n_atoms, khat, ab, E, L.ldE, s);
        if (e != hipSuccess) return dev_fail(h, e, "phase preparation kernel");
    }
    ProfScope prof(h, "interstitial", s);
    e = launch_interstitial(p.g[i], p.kv.data() + 3 * i, E, L.ldE, (const LegTypeRange *)(p.tables + p.olrng),
                            (const TypeDev *)(p.tables + p.ot), p.n_types, (const int *)(p.desc + p.o_stiles[i]),
                            p.n_stiles[i], p.ng[i], p.omega, p.v_int, (double2 *)p.S[i], p.ldh[i],
                            (double2 *)p.H[i], p.ldh[i], s);
    if (e != hipSuccess) return dev_fail(h, e, "interstitial kernel");
    return FLAPW_OK;
}

flapw_status enqueue_generate(flapw_handle h, const GenPlan &p, hipStream_t s)
{
    flapw_status st = launch_T(h, p.gaunt, p.gp, p.T, p.ldt, s);
    if (st != FLAPW_OK) return st;
    const Layout &L = p.L;
    for (const auto &bt : p.batches) {
        for (int i = bt.i0; i < bt.i1; ++i) {
            double2 *P = (double2 *)(p.work + (p.split ? 0 : p.off[i]));
            double2 *Q = P + L.kp2 * p.np[i];
            hipError_t e;
            {
                ProfScope prof(h, "coeffs", s);
                e = launch_coeffs(p.kv.data() + 3 * i, p.ng[i], (int)p.np[i], p.g[i], (const AtomDev *)(p.tables + p.oa),
                                  p.n_atoms, (const TypeDev *)(p.tables + p.ot), p.n_types, L.nlmax, p.pref, P, P, L.kp2,
                                  2 * L.k, L.kp2, s);
            }
            if (e != hipSuccess) return dev_fail(h, e, "coefficient kernel");
            {
                ProfScope prof(h, "qpanel", s);
                e = launch_qpanel(p.T, p.ldt, p.ldt * p.ldt, (const int *)(p.tables + p.oty),
                                  (const int *)(p.tables + p.onl), (const long long *)(p.tables + p.orow), p.n_atoms, P,
                                  Q, L.kp2, (int)p.np[i], L.kp2, true,
                                  *std::min_element(L.atom_nl2.begin(), L.atom_nl2.end()),
                                  (const double *)(p.tables + p.od), p.part, s);
            }
            if (e != hipSuccess) return dev_fail(h, e, "Q panel kernel");
            if (p.split) {
                const ProblemDev pd{P, Q, (const double *)(p.tables + p.od), nullptr, nullptr, L.kp2, 0, p.ng[i],
                                    (int)L.kp2};
                if (p.mod) {
                    const ModArea ma = mod_area(p.digits + p.off[i], L.kp2, p.np[i], p.sl);
                    if ((st = mod_slice_problem(h, pd, p.np[i], ma, p.mt, !p.leg, p.part, p.n_slots, s)) !=
                        FLAPW_OK)
                        return st;
                } else {
                    const DigitArea da = digit_area(p.digits + p.off[i], L.kp2, p.np[i], p.sl, p.bf16 ? 2 : 1);
                    if ((st = slice_problem(h, pd, p.np[i], p.sl, da, p.bf16, s)) != FLAPW_OK) return st;
                }
            }
        }
        hipError_t e;
        if (p.mod) {
            e = launch_mod_pair(h, (const ModProblemDev *)(p.desc + bt.o_probs), (const TileDev *)(p.desc + bt.o_tiles),
                                bt.n_tiles, (const TileDev *)(p.desc + bt.o_ctiles), bt.n_ctiles, p.mt, p.chunks, s);
        } else if (p.split) {
            ProfScope prof(h, "hs_split", s);
            e = launch_split_any(p.bf16, (const SplitProblemDev *)(p.desc + bt.o_probs),
                                 (const TileDev *)(p.desc + bt.o_tiles), bt.n_tiles, p.sl, s);
        } else {
            ProfScope prof(h, "hs_fp64", s);
            e = launch_hs_fp64((const ProblemDev *)(p.desc + bt.o_probs), (const TileDev *)(p.desc + bt.o_tiles), bt.n_tiles,
                               !p.leg, s);
        }
        if (e != hipSuccess) return dev_fail(h, e, p.split ? "S/H split-precision kernel" : "S/H FP64 kernel");
        // S (and the L-diagonal part of H beyond the dense block) once H of the batch is written,
        // then the interstitial terms on top of the muffin-tin parts
        for (int i = bt.i0; i < bt.i1; ++i) {
            if (p.leg && (st = enqueue_s_legendre(h, p, i, (double2 *)p.S[i], p.ldh[i], s)) != FLAPW_OK) return st;
            if (p.inter && (st = enqueue_interstitial(h, p, i, !p.leg, s)) != FLAPW_OK) return st;
        }
    }
    return FLAPW_OK;
}

flapw_status check_generate(flapw_handle h, int n_k, const double *k, const int *n_g, const double *const *g,
                            const flapw_atoms *at, const flapw_radial *rad, const flapw_potential *pot,
                            flapw_z *const *H, flapw_z *const *S, const long *ldh, flapw_prec prec, int slices)
{
    if (n_k < 1) return fail(h, FLAPW_ERR_ARG, "n_k must be >= 1");
    if (!k || !n_g || !g || !H || !S || !ldh) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    flapw_status pst = check_prec(h, prec, slices);
    if (pst != FLAPW_OK) return pst;
    for (int i = 0; i < n_k; ++i) {
        if (n_g[i] < 1) return fail(h, FLAPW_ERR_ARG, "n_g must be >= 1");
        if (!g[i] || !H[i] || !S[i]) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
        if (ldh[i] < n_g[i]) return fail(h, FLAPW_ERR_ARG, "ldh < n_g");
    }
    if (!finite_all(k, 3 * (size_t)n_k)) return fail(h, FLAPW_ERR_ARG, "non-finite k");
    flapw_status st = check_radial(h, rad);
    if (st != FLAPW_OK) return st;
    if ((st = check_atoms(h, at, rad, true)) != FLAPW_OK) return st;
    if ((st = check_potential(h, pot, rad)) != FLAPW_OK) return st;
    if (h->inter && (st = check_spheres(h, at, rad, h->lattice)) != FLAPW_OK) return st;
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    return FLAPW_OK;
}


// Times the first min(n_tiles, cap) tiles of the (single) contraction batch of a prepared plan.
flapw_status time_contraction(flapw_handle h, const GenPlan &p, int cap, float *ms)
{
    const GenBatch &bt = p.batches[0];
    const int n = std::min(bt.n_tiles, cap);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {     // first launch warms caches and code
        e = hipEventRecord(e0, nullptr);
        if (e == hipSuccess)
            e = p.mod     ? launch_mod_contract((const ModProblemDev *)(p.desc + bt.o_probs),
                                                (const TileDev *)(p.desc + bt.o_tiles), n, p.mt, p.chunks, nullptr)
                : p.split ? launch_split_any(p.bf16, (const SplitProblemDev *)(p.desc + bt.o_probs),
                                             (const TileDev *)(p.desc + bt.o_tiles), n, p.sl, nullptr)
                          : launch_hs_fp64((const ProblemDev *)(p.desc + bt.o_probs),
                                           (const TileDev *)(p.desc + bt.o_tiles), n, !p.leg, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return dev_fail(h, e, "timing the contraction");
    return FLAPW_OK;
}

// Relative Frobenius error of a whole N x N Hermitian matrix estimated from its principal submatrix
// on a uniform random subset of n indices (upper triangles of two n x n column-major matrices): the
// n diagonal entries stand for the N diagonal entries (weight N/n), the n(n-1)/2 pairs t' < t for
// the N(N-1)/2 pairs (weight N(N-1)/(n(n-1)), counted twice for the Hermitian lower half), in the
// squared norms of the error and of the reference.  With n = N it is the matrix's own error.
double sampled_relfro(const std::vector<double2> &got, const std::vector<double2> &ref, int n, int N)
{
    double ed = 0.0, eo = 0.0, rd = 0.0, ro = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) {
            const double2 a = got[(size_t)j * n + i], b = ref[(size_t)j * n + i];
            const double e2 = (a.x - b.x) * (a.x - b.x) + (a.y - b.y) * (a.y - b.y), r2 = b.x * b.x + b.y * b.y;
            if (i == j) ed += e2, rd += r2;
            else eo += e2, ro += r2;
        }
    const double wd = (double)N / n, wo = n > 1 ? (double)N * (N - 1.0) / ((double)n * (n - 1.0)) : 0.0;
    const double num = wd * ed + 2.0 * wo * eo, den = wd * rd + 2.0 * wo * ro;
    return den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
}

// Device scratch of the tuner, freed on every exit path.
struct TuneScratch {
    std::vector<void *> ptrs;
    hipError_t alloc(void **p, size_t bytes)
    {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    ~TuneScratch()
    {
        (void)hipDeviceSynchronize();
        for (void *p : ptrs) (void)hipFree(p);
    }
};


// The handle's work buffers: their bytes, and releasing them (the grow-only buffers the next call
// allocates again).
long long ws_bytes(flapw_handle h)
{
    return (long long)(h->work.n + h->tmat.n + h->tables.n + h->gaunt.n + h->tiles.n + h->leg.n + h->eig.n) +
           split_bytes(h);
}

void ws_release(flapw_handle h)
{
    h->work.release();
    h->tmat.release();
    h->tables.release();
    h->gaunt.release();
    h->tiles.release();
    h->leg.release();
    h->radial.release();
    h->eig.release();
    split_release(h);
}

// After a computing call that succeeded: with a workspace limit set and the handle's buffers above
// it, wait for the call's work on its stream and free them.
flapw_status trim_workspace(flapw_handle h, hipStream_t s, flapw_status st)
{
    if (st != FLAPW_OK || h->ws_limit < 0 || ws_bytes(h) <= h->ws_limit) return st;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_fail(h, e, "waiting to release the workspace");
    ws_release(h);
    return st;
}

// ------------------------------------------------------------------------ no-allocation scratch

}  // namespace

// Work memory of flapw_hs_contract_noalloc: every device the library runs on holds one copy of this
// array from the load of the library's code until the process ends.  Host code never uses its name
// as an address: flapw_create looks up each device's copy with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[(size_t)64 << 20];

namespace {

constexpr size_t kScratchBytes = sizeof(scratch);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxDevices] = {};

// Device address of the scratch array on device `dev`, looked up once with that device current.
hipError_t record_scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (unsigned char *)p;
    return hipSuccess;
}

unsigned char *scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[dev];
}

// ------------------------------------------------------------------ S/H contraction of given A, B, T

// Where the contraction's work buffers come from: the handle's grow-only buffers, or (no_alloc)
// consecutive 256-byte aligned pieces of the per-device static scratch array.
struct ContractBufs {
    flapw_handle h;
    unsigned char *arena = nullptr;    // device address of this device's scratch array, or NULL
    size_t used = 0;
    hipError_t get(DevBuf &b, size_t bytes, void **p)
    {
        if (!arena) {
            hipError_t e = b.ensure(bytes);
            *p = b.p;
            return e;
        }
        const size_t off = (size_t)round_up((long long)used, 256);
        if (off + bytes > kScratchBytes) return hipErrorOutOfMemory;     // sized beforehand; never taken
        used = off + bytes;
        *p = arena + off;
        return hipSuccess;
    }
    flapw_status upload(DevBuf &b, const std::vector<unsigned char> &src, hipStream_t s, unsigned char **p)
    {
        void *d = nullptr;
        hipError_t e = get(b, src.size(), &d);
        if (e != hipSuccess) return dev_fail(h, e, arena ? "no-allocation scratch" : "allocating descriptor buffer");
        e = hipMemcpyAsync(d, src.data(), src.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return dev_fail(h, e, "uploading descriptors");
        *p = (unsigned char *)d;
        return FLAPW_OK;
    }
};

// Bytes of the scratch the contraction of one problem takes (the pieces ContractBufs::get hands
// out, each rounded up to 256 bytes).
size_t contract_scratch_bytes(size_t pq, size_t tables, size_t area, size_t desc)
{
    return (size_t)(round_up((long long)pq, 256) + round_up((long long)tables, 256) + round_up((long long)area, 256) +
                    round_up((long long)desc, 256));
}

flapw_status hs_contract_impl(flapw_handle h, int n_g, const flapw_atoms *at, const flapw_radial *rad,
                              const flapw_z *A, const flapw_z *B, long lda, const flapw_z *T, long ldt, flapw_z *H,
                              flapw_z *S, long ldh, flapw_prec prec, int slices, flapw_stream stream, bool no_alloc)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!A || !B || !T || !H || !S) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (n_g < 1) return fail(h, FLAPW_ERR_ARG, "n_g must be >= 1");
    flapw_status st = check_prec(h, prec, slices);
    if (st != FLAPW_OK) return st;
    st = check_radial(h, rad);
    if (st != FLAPW_OK) return st;
    if ((st = check_atoms(h, at, rad, false)) != FLAPW_OK) return st;
    Layout L;
    build_layout(at, rad, true, L);
    if (lda < L.k) return fail(h, FLAPW_ERR_ARG, "lda < K");
    if (ldt < 2LL * L.nlmax) return fail(h, FLAPW_ERR_ARG, "ldt < 2 NL_max");
    if (ldh < n_g) return fail(h, FLAPW_ERR_ARG, "ldh < n_g");
    hipStream_t s = (hipStream_t)stream;
    const long long np = round_up(n_g, kTile);
    // T is taken as given and S from the matrix cores: the key of the default handle settings
    const int band = effective_band(h, prec, L.kp2, FLAPW_S_GEMM, -1);
    const int sl = effective_slices(h, prec, L.kp2, FLAPW_S_GEMM, -1, slices);
    const bool mod = prec == FLAPW_PREC_SPLIT_I8_MOD, split = prec != FLAPW_PREC_FP64;
    const bool bf16 = prec == FLAPW_PREC_SPLIT_BF16;

    // host side first: row map and atom tables, the tile lists, and the sizes of every buffer
    // row map of the work layout: >= 0: row of A, <= -2: row -(v+2) of B, -1: zero
    auto &src = h->host_src;
    src.assign(L.kp2, -1);
    long long off = 0;
    for (int a = 0; a < at->n_atoms; ++a) {
        const int nl = L.atoms[a].nl;
        for (int q = 0; q < nl; ++q) {
            src[L.atom_row[a] + q] = off + q;
            src[L.atom_row[a] + nl + q] = -(off + q) - 2;
        }
        off += nl;
    }
    auto &hb = h->host_tables;
    hb.clear();
    const size_t osrc = put(hb, src.data(), src.size());
    const size_t od = put(hb, L.d.data(), L.d.size());
    const size_t oty = put(hb, L.atom_type.data(), L.atom_type.size());
    const size_t onl = put(hb, L.atom_nl2.data(), L.atom_nl2.size());
    const size_t orow = put(hb, L.atom_row.data(), L.atom_row.size());
    const size_t pq_bytes = (size_t)2 * L.kp2 * np * sizeof(double2);
    size_t area = 0;
    long long npm = np;
    std::vector<TileDev> blocks, tiles;
    if (mod) {
        area = (size_t)mod_area_bytes(L.kp2, np, sl);
        npm = round_up(np, 2 * kModTile);
        build_mod_tiles({(int)((n_g + kModTile - 1) / kModTile)}, 0, 2, blocks, band);
        build_tiles({(int)((n_g + kModTile - 1) / kModTile)}, 0, 2, tiles, band);
    } else if (split) {
        area = (size_t)digit_area_bytes(L.kp2, np, sl, digit_bytes(prec));
        build_tiles({(int)(np / kTile)}, 0, 2, tiles, band);
    } else {
        build_tiles({(int)(np / kTile)}, 0, 1, tiles, band);
    }
    // descriptors: the problem record (largest of the three kinds) and the tile lists
    const size_t desc_bytes = 256 + std::max(sizeof(ModProblemDev), std::max(sizeof(SplitProblemDev), sizeof(ProblemDev))) +
                              256 + blocks.size() * sizeof(TileDev) + 256 + tiles.size() * sizeof(TileDev);
    ContractBufs bufs{h};
    if (no_alloc) {
        const size_t need = contract_scratch_bytes(pq_bytes, hb.size(), area, desc_bytes);
        if (need > kScratchBytes)
            return fail(h, FLAPW_ERR_ARG, "problem needs " + std::to_string(need) + " bytes of work memory, above the " +
                                              std::to_string(kScratchBytes) + "-byte no-allocation scratch");
    }
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    if (no_alloc) {
        bufs.arena = scratch_address(h->device);
        if (!bufs.arena) return fail(h, FLAPW_ERR_DEVICE, "no-allocation scratch address unknown for this device");
    }

    void *pq = nullptr;
    hipError_t e = bufs.get(h->work, pq_bytes, &pq);
    if (e != hipSuccess) return dev_fail(h, e, "allocating work buffer");
    double2 *P = (double2 *)pq;
    double2 *Q = P + L.kp2 * np;
    unsigned char *base = nullptr;
    if ((st = bufs.upload(h->tables, hb, s, &base)) != FLAPW_OK) return st;
    void *ar = nullptr;
    if (split && (e = bufs.get(h->digits, area, &ar)) != hipSuccess)
        return dev_fail(h, e, mod ? "allocating residue buffer" : "allocating digit buffer");
    {
        ProfScope prof(h, "repack", s);
        e = launch_repack((const double2 *)A, (const double2 *)B, lda, n_g, nullptr, 0, (const long long *)(base + osrc), P,
                          L.kp2, (int)L.kp2, (int)np, s);
    }
    if (e != hipSuccess) return dev_fail(h, e, "repack kernel");
    {
        ProfScope prof(h, "qpanel", s);
        e = launch_qpanel((const double2 *)T, ldt, ldt * ldt, (const int *)(base + oty), (const int *)(base + onl),
                          (const long long *)(base + orow), at->n_atoms, P, Q, L.kp2, (int)np, L.kp2, false, 0,
                          nullptr, nullptr, s);
    }
    if (e != hipSuccess) return dev_fail(h, e, "Q panel kernel");
    ProblemDev pd{P, Q, (const double *)(base + od), (double2 *)H, (double2 *)S, L.kp2, ldh, n_g, (int)L.kp2};
    auto &hs = h->host_sdesc;
    hs.clear();
    unsigned char *db = nullptr;
    if (!split) {
        const size_t op = put(hs, &pd, 1);
        const size_t ot = put(hs, tiles.data(), tiles.size());
        if ((st = bufs.upload(h->tiles, hs, s, &db)) != FLAPW_OK) return st;
        ProfScope prof(h, "hs_fp64", s);
        e = launch_hs_fp64((const ProblemDev *)(db + op), (const TileDev *)(db + ot), (int)tiles.size(), true, s);
        if (e != hipSuccess) return dev_fail(h, e, "S/H FP64 kernel");
        return FLAPW_OK;
    }
    if (mod) {
        const ModArea ma = mod_area(ar, L.kp2, np, sl);
        const ModTable mt = make_mod_table(sl);
        if ((st = mod_slice_problem(h, pd, np, ma, mt, true, nullptr, 0, s)) != FLAPW_OK) return st;
        const ModProblemDev mp = mod_problem(ma, (double2 *)H, (double2 *)S, ldh, n_g, L.kp2);
        const size_t op = put(hs, &mp, 1);
        const size_t ob = put(hs, blocks.data(), blocks.size());
        const size_t ot = put(hs, tiles.data(), tiles.size());
        if ((st = bufs.upload(h->sdesc, hs, s, &db)) != FLAPW_OK) return st;
        e = launch_mod_pair(h, (const ModProblemDev *)(db + op), (const TileDev *)(db + ob), (int)blocks.size(),
                            (const TileDev *)(db + ot), (int)tiles.size(), mt,
                            effective_chunks(h, prec, L.kp2, FLAPW_S_GEMM, -1), s);
        if (e != hipSuccess) return dev_fail(h, e, "S/H modular split kernels");
        return FLAPW_OK;
    }
    const DigitArea da = digit_area(ar, L.kp2, np, sl, digit_bytes(prec));
    if ((st = slice_problem(h, pd, np, sl, da, bf16, s)) != FLAPW_OK) return st;
    SplitProblemDev sp{da.L, da.RS, da.RH, da.eL, da.eRS, da.eRH, (double2 *)H, (double2 *)S, ldh, n_g, (int)L.kp2};
    const size_t op = put(hs, &sp, 1);
    const size_t ot = put(hs, tiles.data(), tiles.size());
    if ((st = bufs.upload(h->sdesc, hs, s, &db)) != FLAPW_OK) return st;
    ProfScope prof(h, "hs_split", s);
    e = launch_split_any(bf16, (const SplitProblemDev *)(db + op), (const TileDev *)(db + ot), (int)tiles.size(), sl, s);
    if (e != hipSuccess) return dev_fail(h, e, "S/H split-precision kernel");
    return FLAPW_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------ C-ABI

extern "C" {

flapw_status flapw_create(flapw_handle *h)
{
    if (!h) return FLAPW_ERR_ARG;
    *h = nullptr;
    flapw_context *c = new (std::nothrow) flapw_context();
    if (!c) return FLAPW_ERR_NOMEM;
    // Without a usable device the handle still serves argument validation; computing calls
    // then fail with FLAPW_ERR_DEVICE after their checks.
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        c->device = -1;
        c->err = "no HIP device";
    } else {
        // the no-allocation scratch of this device; on failure only flapw_hs_contract_noalloc
        // is unavailable (it then returns FLAPW_ERR_DEVICE)
        hipError_t e = record_scratch_address(c->device);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            c->err = std::string("no-allocation scratch: ") + hipGetErrorString(e);
        }
    }
    *h = c;
    return FLAPW_OK;
}

flapw_status flapw_destroy(flapw_handle h)
{
    if (!h) return FLAPW_ERR_ARG;
    if (h->device >= 0) (void)hipDeviceSynchronize();
    for (auto &p : h->prof) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (auto e : h->spare_events) (void)hipEventDestroy(e);
    h->work.release();
    h->tmat.release();
    h->tables.release();
    h->gaunt.release();
    h->tiles.release();
    h->leg.release();
    h->radial.release();
    split_release(h);
    eigen_release(h);
    delete h;
    return FLAPW_OK;
}

const char *flapw_status_string(flapw_status s)
{
    switch (s) {
        case FLAPW_OK: return "success";
        case FLAPW_ERR_ARG: return "invalid argument";
        case FLAPW_ERR_WRONSKIAN: return "vanishing Wronskian";
        case FLAPW_ERR_NOT_HERMITIAN: return "T would not be Hermitian";
        case FLAPW_ERR_NOMEM: return "out of device memory";
        case FLAPW_ERR_DEVICE: return "HIP device error";
        case FLAPW_ERR_UNSUPPORTED: return "unsupported request";
        case FLAPW_ERR_NOT_POSDEF: return "S is not positive definite";
        case FLAPW_ERR_NO_CONVERGENCE: return "eigensolver did not converge";
    }
    return "unknown status";
}

const char *flapw_last_error(flapw_handle h) { return h ? h->err.c_str() : "NULL handle"; }

flapw_status flapw_tune(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                        const flapw_radial *rad, const flapw_potential *pot, flapw_prec prec, double tol, int *slices,
                        int *band, int *stage_rows, double *digit_err, double *band_ms)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!slices || !band) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(h, FLAPW_ERR_ARG, "tol must be finite and > 0");
    flapw_z *dummy = reinterpret_cast<flapw_z *>(&tol);       // stands in for H/S in the shared checks
    const long ld1 = n_g;
    flapw_status st = check_generate(h, 1, k, &n_g, &g, at, rad, pot, &dummy, &dummy, &ld1, prec, 0);
    if (st != FLAPW_OK) return st;
    for (int i = 0; digit_err && i < 4; ++i) digit_err[i] = std::nan("");
    for (int i = 0; band_ms && i < 10; ++i) band_ms[i] = std::nan("");
    const bool split = prec != FLAPW_PREC_FP64;
    // the gate and the timing cover the muffin-tin parts (the interstitial terms are FP64 either way)
    struct InterOff {
        flapw_handle h;
        bool was;
        ~InterOff() { h->inter = was; }
    } inter_off{h, h->inter};
    h->inter = false;
    TuneScratch scratch;
    hipError_t e;
    int chosen = 0;
    GenBuffers b{&h->tmat,        &h->tables,      &h->gaunt,     &h->tiles,     &h->work, &h->digits,
                 &h->leg,         &h->host_tables, &h->host_gaunt, &h->host_tiles};
    if (split) {
        // accuracy gate on a random subset of n_acc basis functions (seeded, so the choice is
        // reproducible), against the FP64 path on the same subset
        const int n_acc = std::min(n_g, 1024);
        std::vector<int> pick(n_g);
        for (int i = 0; i < n_g; ++i) pick[i] = i;
        if (n_acc < n_g) {
            std::mt19937_64 rng(0x1602065890ULL);
            for (int i = 0; i < n_acc; ++i) std::swap(pick[i], pick[i + (int)(rng() % (unsigned long long)(n_g - i))]);
            pick.resize(n_acc);
            std::sort(pick.begin(), pick.end());
        }
        std::vector<double> gall((size_t)3 * n_g), gsub((size_t)3 * n_acc);
        if ((e = hipMemcpy(gall.data(), g, gall.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
            return dev_fail(h, e, "reading the G list");
        for (int i = 0; i < n_acc; ++i)
            for (int c = 0; c < 3; ++c) gsub[3 * i + c] = gall[3 * (size_t)pick[i] + c];
        void *gs = nullptr;
        if ((e = scratch.alloc(&gs, gsub.size() * sizeof(double))) != hipSuccess ||
            (e = hipMemcpy(gs, gsub.data(), gsub.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
            return dev_fail(h, e, "uploading the sampled G list");
        const double *gsd = (const double *)gs;
        const size_t mat = (size_t)n_acc * n_acc * sizeof(double2);
        void *buf[4];
        for (int i = 0; i < 4; ++i)
            if ((e = scratch.alloc(&buf[i], mat)) != hipSuccess) return dev_fail(h, e, "allocating tuner outputs");
        std::vector<double2> Hr((size_t)n_acc * n_acc), Sr(Hr.size()), Hc(Hr.size()), Sc(Hr.size());
        const long ldn = n_acc;
        // candidate 0: the FP64 reference; then 3..6 digits, or 10..13 moduli
        const int c0 = prec == FLAPW_PREC_SPLIT_I8_MOD ? 10 : 3;
        const int cand[5] = {0, c0, c0 + 1, c0 + 2, c0 + 3};
        for (int ci = 0; ci < 5; ++ci) {
            const int s = cand[ci];
            flapw_z *Hp = (flapw_z *)buf[s ? 2 : 0], *Sp = (flapw_z *)buf[s ? 3 : 1];
            GenPlan p;
            st = prepare_generate(h, 1, k, &n_acc, &gsd, at, rad, pot, &Hp, &Sp, &ldn, s ? prec : FLAPW_PREC_FP64, s, 4,
                                  false, b, p, nullptr, false);
            if (st == FLAPW_OK) st = enqueue_generate(h, p, nullptr);
            if (st != FLAPW_OK) return st;
            e = hipMemcpy((s ? Hc : Hr).data(), Hp, mat, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy((s ? Sc : Sr).data(), Sp, mat, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return dev_fail(h, e, "reading tuner outputs");
            if (!s) continue;
            // the whole matrix's relative Frobenius error, estimated without bias from the sample
            const double err = std::max(sampled_relfro(Hc, Hr, n_acc, n_g), sampled_relfro(Sc, Sr, n_acc, n_g));
            if (digit_err) digit_err[ci - 1] = err;
            if (!chosen && err <= kTuneMargin * tol) chosen = s;
        }
        if (!chosen)
            return fail(h, FLAPW_ERR_UNSUPPORTED, prec == FLAPW_PREC_SPLIT_I8_MOD
                                                      ? "no modulus count in 10..13 meets the tolerance"
                                                      : "no digit count in 3..6 meets the tolerance");
    }
    // tile band: time a prefix of the full contraction of this k-point with every candidate band
    const size_t mat = (size_t)n_g * n_g * sizeof(double2);
    void *Hb = nullptr, *Sb = nullptr;
    if ((e = scratch.alloc(&Hb, mat)) != hipSuccess || (e = scratch.alloc(&Sb, mat)) != hipSuccess)
        return dev_fail(h, e, "allocating tuner outputs");
    static const int bands[5] = {1, 2, 4, 8, 16};
    const bool mod = prec == FLAPW_PREC_SPLIT_I8_MOD;
    int best = 4, best_chunks = 0;
    float best_ms = 0.0f;
    for (int i = 0; i < (mod ? 10 : 5); ++i) {
        flapw_z *Hp = (flapw_z *)Hb, *Sp = (flapw_z *)Sb;
        GenPlan p;
        st = prepare_generate(h, 1, k, &n_g, &g, at, rad, pot, &Hp, &Sp, &ld1, prec, chosen, bands[i % 5],
                              h->s_method == FLAPW_S_LEGENDRE, b, p, nullptr,
                              false);
        if (st == FLAPW_OK && i == 0) st = enqueue_generate(h, p, nullptr);   // panels / digits for the timing
        if (st != FLAPW_OK) return st;
        if (p.batches.size() != 1) return fail(h, FLAPW_ERR_NOMEM, "one k-point does not fit the work budget");
        p.chunks = i < 5 ? 4 : 2;                       // the modular path: 64-row, then 32-row stages
        float ms = 0.0f;
        if ((st = time_contraction(h, p, 8192, &ms)) != FLAPW_OK) return st;
        if (band_ms) band_ms[i] = ms;
        if (i == 0 || ms < best_ms) best_ms = ms, best = bands[i % 5], best_chunks = mod ? p.chunks : 0;
    }
    // keyed as prepare_generate looks it up: the row layout with the same cut, the S method, lnonsph
    Layout L;
    int lmx = 0;
    for (int t = 0; t < rad->n_types; ++t) lmx = std::max(lmx, rad->lmax[t]);
    const bool leg = h->s_method == FLAPW_S_LEGENDRE;
    build_layout(at, rad, true, L, (leg && h->lnonsph >= 0 && h->lnonsph < lmx) ? h->lnonsph : -1);
    flapw_context::Tuned t{(int)prec, L.kp2, leg ? (int)FLAPW_S_LEGENDRE : (int)FLAPW_S_GEMM, h->lnonsph, chosen, best,
                           best_chunks};
    bool found = false;
    for (auto &x : h->tuned)
        if (x.prec == t.prec && x.kp2 == t.kp2 && x.s_method == t.s_method && x.lnonsph == t.lnonsph) x = t, found = true;
    if (!found) h->tuned.push_back(t);
    *slices = chosen;
    *band = best;
    if (stage_rows) *stage_rows = 16 * best_chunks;
    return FLAPW_OK;
}

flapw_status flapw_profile_enable(flapw_handle h, int on)
{
    if (!h) return FLAPW_ERR_ARG;
    for (auto &p : h->prof) {
        (void)hipEventSynchronize(p.second.second);
        h->spare_events.push_back(p.second.first);
        h->spare_events.push_back(p.second.second);
    }
    h->prof.clear();
    h->profiling = on != 0 && h->device >= 0;
    return FLAPW_OK;
}

flapw_status flapw_profile_query(flapw_handle h, const char *family, int *launches, double *total_ms)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!family || !launches || !total_ms) return fail(h, FLAPW_ERR_ARG, "NULL argument");
    static const char *known[] = {"coeffs",   "tmat",      "qpanel",   "repack",     "hs_fp64",
                                  "slice",    "hs_split",  "hs_mod",   "mod_crt",    "graph",
                                  "leg_prep", "s_legendre", "interstitial", "eigensolve", "radial"};
    bool ok = false;
    for (const char *k : known) ok = ok || std::strcmp(k, family) == 0;
    if (!ok) return fail(h, FLAPW_ERR_ARG, std::string("unknown kernel family ") + family);
    int n = 0;
    double ms = 0.0;
    for (auto &p : h->prof) {
        if (p.first != family) continue;
        hipError_t e = hipEventSynchronize(p.second.second);
        if (e != hipSuccess) return dev_fail(h, e, "event synchronize");
        float t = 0.f;
        e = hipEventElapsedTime(&t, p.second.first, p.second.second);
        if (e != hipSuccess) return dev_fail(h, e, "event elapsed time");
        ms += t;
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    return FLAPW_OK;
}

flapw_status flapw_release_workspace(flapw_handle h)
{
    if (!h) return FLAPW_ERR_ARG;
    if (h->device >= 0) (void)hipDeviceSynchronize();
    ws_release(h);
    return FLAPW_OK;
}

flapw_status flapw_set_workspace_limit(flapw_handle h, long long bytes)
{
    if (!h) return FLAPW_ERR_ARG;
    h->ws_limit = bytes < 0 ? -1 : bytes;
    return FLAPW_OK;
}

long long flapw_workspace_bytes(flapw_handle h)
{
    if (!h) return -1;
    return ws_bytes(h);
}

flapw_status flapw_coeffs(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                          const flapw_radial *rad, flapw_z *A, flapw_z *B, long ld, flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!k || !g || !A || !B) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (n_g < 1) return fail(h, FLAPW_ERR_ARG, "n_g must be >= 1");
    if (!finite_all(k, 3)) return fail(h, FLAPW_ERR_ARG, "non-finite k");
    flapw_status st = check_radial(h, rad);
    if (st != FLAPW_OK) return st;
    if ((st = check_atoms(h, at, rad, true)) != FLAPW_OK) return st;
    Layout L;
    build_layout(at, rad, false, L);
    if (ld < L.k) return fail(h, FLAPW_ERR_ARG, "ld < K");
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    hipStream_t s = (hipStream_t)stream;
    auto &hb = h->host_tables;
    hb.clear();
    const size_t oa = put(hb, L.atoms.data(), L.atoms.size());
    const size_t ot = put(hb, L.types.data(), L.types.size());
    if ((st = upload(h, h->tables, hb, s)) != FLAPW_OK) return st;
    unsigned char *base = (unsigned char *)h->tables.p;
    const double pref = 4.0 * kPi / std::sqrt(at->omega);
    ProfScope prof(h, "coeffs", s);
    hipError_t e = launch_coeffs(k, n_g, n_g, g, (const AtomDev *)(base + oa), at->n_atoms, (const TypeDev *)(base + ot),
                                 rad->n_types, L.nlmax, pref, (double2 *)A, (double2 *)B, ld, 0, 0, s);
    if (e != hipSuccess) return dev_fail(h, e, "coefficient kernel");
    return FLAPW_OK;
}

flapw_status flapw_build_T(flapw_handle h, const flapw_radial *rad, const flapw_potential *pot, flapw_z *T, long ldt,
                           flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!T) return fail(h, FLAPW_ERR_ARG, "T is NULL");
    flapw_status st = check_radial(h, rad);
    if (st != FLAPW_OK) return st;
    if ((st = check_potential(h, pot, rad)) != FLAPW_OK) return st;
    int lm = 0;
    for (int t = 0; t < rad->n_types; ++t) lm = std::max(lm, rad->lmax[t]);
    if (ldt < 2LL * (lm + 1) * (lm + 1)) return fail(h, FLAPW_ERR_ARG, "ldt < 2 NL_max");
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    return build_T_impl(h, rad, pot, (double2 *)T, ldt, (hipStream_t)stream);
}

flapw_status flapw_hs_contract(flapw_handle h, int n_g, const flapw_atoms *at, const flapw_radial *rad,
                               const flapw_z *A, const flapw_z *B, long lda, const flapw_z *T, long ldt, flapw_z *H,
                               flapw_z *S, long ldh, flapw_prec prec, int slices, flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    return trim_workspace(h, (hipStream_t)stream,
                          hs_contract_impl(h, n_g, at, rad, A, B, lda, T, ldt, H, S, ldh, prec, slices, stream, false));
}

flapw_status flapw_hs_contract_noalloc(flapw_handle h, int n_g, const flapw_atoms *at, const flapw_radial *rad,
                                       const flapw_z *A, const flapw_z *B, long lda, const flapw_z *T, long ldt,
                                       flapw_z *H, flapw_z *S, long ldh, flapw_prec prec, int slices,
                                       flapw_stream stream)
{
    return hs_contract_impl(h, n_g, at, rad, A, B, lda, T, ldt, H, S, ldh, prec, slices, stream, true);
}

long long flapw_noalloc_scratch_bytes(void) { return (long long)kScratchBytes; }

flapw_status flapw_hs_generate(flapw_handle h, int n_k, const double *k, const int *n_g, const double *const *g,
                               const flapw_atoms *at, const flapw_radial *rad, const flapw_potential *pot,
                               flapw_z *const *H, flapw_z *const *S, const long *ldh, flapw_prec prec, int slices,
                               flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    flapw_status st = check_generate(h, n_k, k, n_g, g, at, rad, pot, H, S, ldh, prec, slices);
    if (st != FLAPW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    GenPlan p;
    GenBuffers b{&h->tmat,        &h->tables,      &h->gaunt,     &h->tiles,     &h->work, &h->digits,
                 &h->leg,         &h->host_tables, &h->host_gaunt, &h->host_tiles};
    st = prepare_generate(h, n_k, k, n_g, g, at, rad, pot, H, S, ldh, prec, slices, 0, h->s_method == FLAPW_S_LEGENDRE,
                          b, p, s, false);
    if (st != FLAPW_OK) return st;
    return trim_workspace(h, s, enqueue_generate(h, p, s));
}

flapw_status flapw_set_s_method(flapw_handle h, flapw_s_method method)
{
    if (!h) return FLAPW_ERR_ARG;
    if (method != FLAPW_S_GEMM && method != FLAPW_S_LEGENDRE) return fail(h, FLAPW_ERR_ARG, "unknown S method");
    h->s_method = (int)method;
    return FLAPW_OK;
}

flapw_status flapw_set_lnonsph(flapw_handle h, int lnonsph)
{
    if (!h) return FLAPW_ERR_ARG;
    if (lnonsph < -1 || lnonsph > FLAPW_LMAX_CAP) return fail(h, FLAPW_ERR_ARG, "lnonsph out of range");
    h->lnonsph = lnonsph;
    return FLAPW_OK;
}

flapw_status flapw_s_legendre(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                              const flapw_radial *rad, flapw_z *S, long lds, flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!k || !g || !S) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (n_g < 1) return fail(h, FLAPW_ERR_ARG, "n_g must be >= 1");
    if (lds < n_g) return fail(h, FLAPW_ERR_ARG, "lds < n_g");
    if (!finite_all(k, 3)) return fail(h, FLAPW_ERR_ARG, "non-finite k");
    flapw_status st = check_radial(h, rad);
    if (st != FLAPW_OK) return st;
    if ((st = check_atoms(h, at, rad, true)) != FLAPW_OK) return st;
    if (!(at->omega > 0.0)) return fail(h, FLAPW_ERR_ARG, "omega must be > 0");
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    hipStream_t s = (hipStream_t)stream;
    GenPlan p;
    Layout &L = p.L;
    build_layout(at, rad, true, L);
    p.leg = true;
    p.omega = at->omega;
    p.n_atoms = at->n_atoms;
    p.n_types = rad->n_types;
    p.kv.assign(k, k + 3);
    p.g.assign(1, g);
    p.ng.assign(1, n_g);
    p.np.assign(1, round_up(n_g, kTile));
    auto &ht = h->host_tables;
    ht.clear();
    p.ot = put(ht, L.types.data(), L.types.size());
    p.oapos = put(ht, L.apos.data(), L.apos.size());
    p.olrow = put(ht, L.leg_row.data(), L.leg_row.size());
    p.olrng = put(ht, L.leg_ranges.data(), L.leg_ranges.size());
    p.oun2 = put(ht, L.leg_un2.data(), L.leg_un2.size());
    if ((st = upload(h, h->tables, ht, s)) != FLAPW_OK) return st;
    p.tables = (unsigned char *)h->tables.p;
    std::vector<int> tl;
    s_tiles(p.np[0], tl);
    auto &hd = h->host_tiles;
    hd.clear();
    p.o_stiles.assign(1, put(hd, tl.data(), tl.size()));
    p.n_stiles.assign(1, (int)tl.size() / 2);
    if ((st = upload(h, h->tiles, hd, s)) != FLAPW_OK) return st;
    p.desc = (unsigned char *)h->tiles.p;
    hipError_t e = h->leg.ensure(leg_bytes(L, p.np[0], p.n_types, &p.leg_ab, &p.leg_E));
    if (e != hipSuccess) return dev_fail(h, e, "allocating Legendre scratch");
    p.legbuf = (unsigned char *)h->leg.p;
    return trim_workspace(h, s, enqueue_s_legendre(h, p, 0, (double2 *)S, lds, s));
}

flapw_status flapw_interstitial(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                                const flapw_radial *rad, const double *lattice, double v_int, flapw_z *H,
                                flapw_z *S, long ldh, flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!k || !g || !S || !H) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (n_g < 1) return fail(h, FLAPW_ERR_ARG, "n_g must be >= 1");
    if (ldh < n_g) return fail(h, FLAPW_ERR_ARG, "ldh < n_g");
    if (!finite_all(k, 3) || !std::isfinite(v_int)) return fail(h, FLAPW_ERR_ARG, "non-finite k or v_int");
    flapw_status st = check_radial(h, rad);
    if (st != FLAPW_OK) return st;
    if ((st = check_atoms(h, at, rad, true)) != FLAPW_OK) return st;
    if ((st = check_spheres(h, at, rad, lattice)) != FLAPW_OK) return st;
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    hipStream_t s = (hipStream_t)stream;
    GenPlan p;
    Layout &L = p.L;
    build_layout(at, rad, true, L);
    p.inter = true;
    p.v_int = v_int;
    p.omega = at->omega;
    p.n_atoms = at->n_atoms;
    p.n_types = rad->n_types;
    p.kv.assign(k, k + 3);
    p.g.assign(1, g);
    p.ng.assign(1, n_g);
    p.np.assign(1, round_up(n_g, kTile));
    p.S.assign(1, S);
    p.H.assign(1, H);
    p.ldh.assign(1, ldh);
    auto &ht = h->host_tables;
    ht.clear();
    p.ot = put(ht, L.types.data(), L.types.size());
    p.oapos = put(ht, L.apos.data(), L.apos.size());
    p.olrow = put(ht, L.leg_row.data(), L.leg_row.size());
    p.olrng = put(ht, L.leg_ranges.data(), L.leg_ranges.size());
    if ((st = upload(h, h->tables, ht, s)) != FLAPW_OK) return st;
    p.tables = (unsigned char *)h->tables.p;
    std::vector<int> tl;
    s_tiles(p.np[0], tl);
    auto &hd = h->host_tiles;
    hd.clear();
    p.o_stiles.assign(1, put(hd, tl.data(), tl.size()));
    p.n_stiles.assign(1, (int)tl.size() / 2);
    if ((st = upload(h, h->tiles, hd, s)) != FLAPW_OK) return st;
    p.desc = (unsigned char *)h->tiles.p;
    hipError_t e = h->leg.ensure(leg_bytes(L, p.np[0], p.n_types, &p.leg_ab, &p.leg_E));
    if (e != hipSuccess) return dev_fail(h, e, "allocating phase scratch");
    p.legbuf = (unsigned char *)h->leg.p;
    return trim_workspace(h, s, enqueue_interstitial(h, p, 0, true, s));
}

flapw_status flapw_set_interstitial(flapw_handle h, int on, const double *lattice, double v_int)
{
    if (!h) return FLAPW_ERR_ARG;
    if (on && !lattice) return fail(h, FLAPW_ERR_ARG, "NULL lattice");
    if (!std::isfinite(v_int)) return fail(h, FLAPW_ERR_ARG, "non-finite v_int");
    if (on && !finite_all(lattice, 9)) return fail(h, FLAPW_ERR_ARG, "non-finite lattice");
    h->inter = on != 0;
    h->v_int = v_int;
    if (on) std::memcpy(h->lattice, lattice, sizeof(h->lattice));
    return FLAPW_OK;
}

namespace {

flapw_status check_radial_mesh(flapw_handle h, const flapw_radial_mesh *m)
{
    if (!m) return fail(h, FLAPW_ERR_ARG, "radial mesh descriptor is NULL");
    if (m->n_types < 1 || m->n_types > 32) return fail(h, FLAPW_ERR_ARG, "n_types must be in 1..32");
    if (!m->lmax || !m->rmt || !m->r0 || !m->e_l || !m->v_sph || !m->v_lm)
        return fail(h, FLAPW_ERR_ARG, "radial mesh array pointer is NULL");
    if (m->n_r < 9 || m->n_r > FLAPW_NR_CAP || (m->n_r - 1) % 4 != 0)
        return fail(h, FLAPW_ERR_ARG, "n_r must be in 9.." + std::to_string(FLAPW_NR_CAP) + " with n_r - 1 a multiple of 4");
    if (m->lpot < 0 || m->lpot > FLAPW_LPOT_CAP)
        return fail(h, FLAPW_ERR_ARG, "lpot out of range 0.." + std::to_string(FLAPW_LPOT_CAP));
    int lm = 0;
    for (int t = 0; t < m->n_types; ++t) {
        if (m->lmax[t] < 0 || m->lmax[t] > FLAPW_LMAX_CAP)
            return fail(h, FLAPW_ERR_ARG, "lmax out of range 0.." + std::to_string(FLAPW_LMAX_CAP));
        if (!std::isfinite(m->rmt[t]) || !std::isfinite(m->r0[t]) || !(m->r0[t] >= 1e-10) || !(m->r0[t] < m->rmt[t]))
            return fail(h, FLAPW_ERR_ARG, "mesh of type " + std::to_string(t) + " needs 1e-10 <= r0 < rmt");
        lm = std::max(lm, m->lmax[t]);
    }
    if (m->lstride < lm + 1) return fail(h, FLAPW_ERR_ARG, "lstride < max lmax + 1");
    for (int t = 0; t < m->n_types; ++t)
        if (!finite_all(m->e_l + (size_t)t * m->lstride, m->lmax[t] + 1))
            return fail(h, FLAPW_ERR_ARG, "non-finite energy parameter");
    const int nlp = (m->lpot + 1) * (m->lpot + 1);
    if (!finite_all(m->v_sph, (size_t)m->n_types * m->n_r) || !finite_all(m->v_lm, (size_t)m->n_types * nlp * m->n_r))
        return fail(h, FLAPW_ERR_ARG, "non-finite potential");
    for (int t = 0; t < m->n_types; ++t) {
        const double *v = m->v_lm + (size_t)t * nlp * m->n_r;
        double mx = 0.0;
        for (size_t i = 0; i < (size_t)nlp * m->n_r; ++i) mx = std::max(mx, std::fabs(v[i]));
        for (int lpp = 1; lpp <= m->lpot; ++lpp)
            for (int mm = 1; mm <= lpp; ++mm) {
                const double *vp = v + (size_t)(lpp * lpp + lpp + mm) * m->n_r;
                const double *vm = v + (size_t)(lpp * lpp + lpp - mm) * m->n_r;
                const double sg = (mm & 1) ? -1.0 : 1.0;
                for (int i = 0; i < m->n_r; ++i)
                    if (std::fabs(vm[i] - sg * vp[i]) > 1e-12 * mx)
                        return fail(h, FLAPW_ERR_NOT_HERMITIAN, "v_lm violates v(l'',-m) = (-1)^m v(l'',m)");
            }
    }
    return FLAPW_OK;
}

}  // namespace

flapw_status flapw_radial_setup(flapw_handle h, const flapw_radial_mesh *m, double *u, double *du, double *ud,
                                double *dud, double *ud_norm2, double *i_uu, double *i_ud, double *i_du,
                                double *i_dd, flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!u || !du || !ud || !dud || !ud_norm2 || !i_uu || !i_ud || !i_du || !i_dd)
        return fail(h, FLAPW_ERR_ARG, "NULL output pointer");
    flapw_status st = check_radial_mesh(h, m);
    if (st != FLAPW_OK) return st;
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    hipStream_t s = (hipStream_t)stream;
    const int nt = m->n_types, ls = m->lstride, nr = m->n_r, nlp = (m->lpot + 1) * (m->lpot + 1);
    // device layout: small per-type inputs, v_sph, v_lm, functions, boundary values, four tables
    std::vector<unsigned char> &hb = h->host_tables;
    hb.clear();
    const size_t o_r0 = put(hb, m->r0, nt), o_rmt = put(hb, m->rmt, nt), o_lmax = put(hb, m->lmax, nt);
    const size_t o_el = put(hb, m->e_l, (size_t)nt * ls);
    const size_t n_small = hb.size();
    auto align = [](size_t x) { return (size_t)round_up((long long)x, 256); };
    const size_t o_vs = align(n_small), n_vs = sizeof(double) * nt * nr;
    const size_t o_vl = align(o_vs + n_vs), n_vl = sizeof(double) * nt * nlp * nr;
    const size_t o_fun = align(o_vl + n_vl), n_fun = radial_fun_bytes(nt, nr);
    const size_t o_bnd = align(o_fun + n_fun), n_bnd = sizeof(double) * nt * kLStride * 5;
    const size_t n_tab = sizeof(double) * nt * ls * ls * nlp;
    const size_t o_tab = align(o_bnd + n_bnd), total = o_tab + 4 * align(n_tab);
    hipError_t e = h->radial.ensure(total);
    if (e != hipSuccess) return dev_fail(h, e, "allocating radial buffers");
    unsigned char *d = (unsigned char *)h->radial.p;
    double *tab[4];
    for (int q = 0; q < 4; ++q) tab[q] = (double *)(d + o_tab + q * align(n_tab));
    if ((e = hipMemcpyAsync(d, hb.data(), n_small, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d + o_vs, m->v_sph, n_vs, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d + o_vl, m->v_lm, n_vl, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemsetAsync(d + o_tab, 0, 4 * align(n_tab), s)) != hipSuccess)
        return dev_fail(h, e, "uploading radial meshes");
    {
        ProfScope ps(h, "radial", s);
        e = launch_radial(nt, nr, nlp, (const double *)(d + o_r0), (const double *)(d + o_rmt),
                          (const int *)(d + o_lmax), (const double *)(d + o_el), ls, (const double *)(d + o_vs),
                          (const double *)(d + o_vl), (double *)(d + o_fun), (double *)(d + o_bnd), tab[0], tab[1],
                          tab[2], tab[3], s);
    }
    if (e != hipSuccess) return dev_fail(h, e, "launching radial kernels");
    std::vector<double> bnd((size_t)nt * kLStride * 5), tabs(4 * (size_t)nt * ls * ls * nlp);
    if ((e = hipMemcpyAsync(bnd.data(), d + o_bnd, n_bnd, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return dev_fail(h, e, "reading radial results");
    for (int q = 0; q < 4; ++q)
        if ((e = hipMemcpyAsync(tabs.data() + q * (n_tab / sizeof(double)), tab[q], n_tab, hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            return dev_fail(h, e, "reading radial results");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return dev_fail(h, e, "radial setup");
    for (int t = 0; t < nt; ++t)
        if (!finite_all(bnd.data() + (size_t)t * kLStride * 5, 5 * (size_t)(m->lmax[t] + 1)))
            return fail(h, FLAPW_ERR_ARG, "radial solution of type " + std::to_string(t) +
                                              " is not finite (energy parameter far below the potential?)");
    if (!finite_all(tabs.data(), tabs.size())) return fail(h, FLAPW_ERR_ARG, "radial integrals are not finite");
    for (int t = 0; t < nt; ++t)
        for (int l = 0; l < ls; ++l) {
            const size_t q = (size_t)t * ls + l;
            const double *b = bnd.data() + ((size_t)t * kLStride + l) * 5;
            const bool used = l <= m->lmax[t];
            u[q] = used ? b[0] : 0.0;
            du[q] = used ? b[1] : 0.0;
            ud[q] = used ? b[2] : 0.0;
            dud[q] = used ? b[3] : 0.0;
            ud_norm2[q] = used ? b[4] : 0.0;
        }
    const size_t nn = n_tab / sizeof(double);
    double *outs[4] = {i_uu, i_ud, i_du, i_dd};
    for (int q = 0; q < 4; ++q) std::memcpy(outs[q], tabs.data() + q * nn, n_tab);
    return FLAPW_OK;
}

flapw_status flapw_plan_create(flapw_handle h, int n_k, const double *k, const int *n_g, const double *const *g,
                               const flapw_atoms *at, const flapw_radial *rad, const flapw_potential *pot,
                               flapw_z *const *H, flapw_z *const *S, const long *ldh, flapw_prec prec, int slices,
                               flapw_plan *plan)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!plan) return fail(h, FLAPW_ERR_ARG, "plan is NULL");
    *plan = nullptr;
    flapw_status st = check_generate(h, n_k, k, n_g, g, at, rad, pot, H, S, ldh, prec, slices);
    if (st != FLAPW_OK) return st;
    hipError_t e = init_fp64_kernels();
    if (e == hipSuccess && prec == FLAPW_PREC_SPLIT_I8) e = init_split_kernels();
    if (e == hipSuccess && prec == FLAPW_PREC_SPLIT_BF16) e = init_split_bf16_kernels();
    if (e == hipSuccess && prec == FLAPW_PREC_SPLIT_I8_MOD) e = init_mod_kernels();
    if (e == hipSuccess && h->s_method == FLAPW_S_LEGENDRE) e = init_legendre_kernels();
    if (e == hipSuccess && h->inter) e = init_interstitial_kernel();
    if (e != hipSuccess) return dev_fail(h, e, "kernel attributes");
    flapw_plan_s *pl = new (std::nothrow) flapw_plan_s();
    if (!pl) return fail(h, FLAPW_ERR_NOMEM, "plan allocation");
    pl->h = h;
    GenPlan p;
    GenBuffers b{&pl->tmat, &pl->tables, &pl->gaunt, &pl->desc, &pl->work, &pl->digits, &pl->leg, &pl->h_tables,
                 &pl->h_gaunt, &pl->h_desc};
    st = prepare_generate(h, n_k, k, n_g, g, at, rad, pot, H, S, ldh, prec, slices, 0, h->s_method == FLAPW_S_LEGENDRE,
                          b, p, nullptr, true);
    hipStream_t cs = nullptr;
    if (st == FLAPW_OK) {
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) st = dev_fail(h, e, "capture stream");
    }
    if (st == FLAPW_OK) {
        const bool prof = h->profiling;
        h->profiling = false;                      // no event nodes inside the graph
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) st = dev_fail(h, e, "begin capture");
        if (st == FLAPW_OK) {
            flapw_status se = enqueue_generate(h, p, cs);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(cs, &graph);
            if (se != FLAPW_OK) st = se;
            else if (e != hipSuccess) st = dev_fail(h, e, "end capture");
            else {
                e = hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0);
                if (e != hipSuccess) st = dev_fail(h, e, "graph instantiation");
            }
            if (graph) (void)hipGraphDestroy(graph);
        }
        h->profiling = prof;
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (st != FLAPW_OK) {
        flapw_plan_destroy(pl);
        return st;
    }
    *plan = pl;
    return FLAPW_OK;
}

flapw_status flapw_plan_launch(flapw_plan plan, flapw_stream stream)
{
    if (!plan || !plan->exec) return FLAPW_ERR_ARG;
    ProfScope prof(plan->h, "graph", (hipStream_t)stream);
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(plan->h, e, "graph launch");
    return FLAPW_OK;
}

flapw_status flapw_plan_destroy(flapw_plan plan)
{
    if (!plan) return FLAPW_ERR_ARG;
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    plan->work.release();
    plan->digits.release();
    plan->tmat.release();
    plan->tables.release();
    plan->gaunt.release();
    plan->desc.release();
    plan->leg.release();
    delete plan;
    return FLAPW_OK;
}

}  // extern "C"
