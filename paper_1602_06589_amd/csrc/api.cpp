// Host side of the C-ABI declared in include/flapw.h: argument validation, the handle's device
// work buffers, descriptor tables and kernel launches.  No arithmetic of the method runs here
// except the Gauss-Legendre nodes handed to the Gaunt quadrature kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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
};

void build_layout(const flapw_atoms *at, const flapw_radial *rad, bool work_layout, Layout &L)
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
        }
    }
    L.nlmax = (lm + 1) * (lm + 1);
    long long off = 0;
    for (int a = 0; a < na; ++a) {
        const int t = at->type[a];
        const int nl = (rad->lmax[t] + 1) * (rad->lmax[t] + 1);
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
    L.d.assign(L.kp2, 0.0);
    for (int a = 0; a < na; ++a) {
        const int t = at->type[a], lmx = rad->lmax[t];
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

// T of all types into dev (ldt x ldt each).
flapw_status build_T_impl(flapw_handle h, const flapw_radial *rad, const flapw_potential *pot, double2 *T, long long ldt,
                          hipStream_t s)
{
    int lm = 0;
    for (int t = 0; t < rad->n_types; ++t) lm = std::max(lm, rad->lmax[t]);
    const int lt = std::max(lm, pot->lpot);
    const int nq = lm + pot->lpot + 2;            // exact for polynomial degree <= 2 lmax + lpot
    std::vector<double> z, w;
    gauss_legendre(nq, z, w);
    const int ls = rad->lstride, nlp = (pot->lpot + 1) * (pot->lpot + 1);
    const size_t ni = (size_t)rad->n_types * ls * ls * nlp;
    auto &hb = h->host_gaunt;
    hb.clear();
    const size_t oz = put(hb, z.data(), z.size());
    const size_t ow = put(hb, w.data(), w.size());
    const size_t o1 = put(hb, pot->i_uu, ni), o2 = put(hb, pot->i_ud, ni), o3 = put(hb, pot->i_du, ni),
                 o4 = put(hb, pot->i_dd, ni);
    const size_t oe = put(hb, rad->e_l, (size_t)rad->n_types * ls);
    const size_t on = put(hb, rad->ud_norm2, (size_t)rad->n_types * ls);
    const size_t ol = put(hb, rad->lmax, (size_t)rad->n_types);
    const size_t oth = round_up(hb.size(), 256);
    const size_t nth = (size_t)(lt + 1) * (lt + 2) / 2 * nq;
    hb.resize(oth + nth * sizeof(double));
    flapw_status st = upload(h, h->gaunt, hb, s);
    if (st != FLAPW_OK) return st;
    unsigned char *base = (unsigned char *)h->gaunt.p;
    ProfScope prof(h, "tmat", s);
    hipError_t e = launch_legendre_table(lt, nq, (const double *)(base + oz), (double *)(base + oth), s);
    if (e != hipSuccess) return dev_fail(h, e, "legendre table kernel");
    e = launch_tmat(rad->n_types, (const int *)(base + ol), ls, pot->lpot, nq, (const double *)(base + ow),
                    (const double *)(base + oth), (const double *)(base + o1), (const double *)(base + o2),
                    (const double *)(base + o3), (const double *)(base + o4), (const double *)(base + oe),
                    (const double *)(base + on), T, ldt, s);
    if (e != hipSuccess) return dev_fail(h, e, "T assembly kernel");
    return FLAPW_OK;
}

// Upper-triangle tile list of several problems, ordered in bands of kBand tile rows (so that
// work-groups running together share operand panels) and remapped so that each of the eight
// XCDs (work-group b runs on XCD b % 8) receives a contiguous run of that order.  With mats = 2
// (split precision) every (ti, tj) gives an S tile and an H tile next to each other.
void build_tiles(const std::vector<int> &np_tiles, int mats, std::vector<TileDev> &out)
{
    constexpr int kBand = 4;
    std::vector<TileDev> order;
    for (int p = 0; p < (int)np_tiles.size(); ++p) {
        const int nt = np_tiles[p];
        for (int b0 = 0; b0 < nt; b0 += kBand)
            for (int tj = b0; tj < nt; ++tj)
                for (int ti = b0; ti < std::min(b0 + kBand, tj + 1); ++ti)
                    for (int m = 0; m < mats; ++m) order.push_back(TileDev{p, ti, tj, m});
    }
    const int n = (int)order.size();
    out.resize(n);
    const int q = n / 8, rem = n % 8;
    int start[9];
    start[0] = 0;
    for (int x = 0; x < 8; ++x) start[x + 1] = start[x] + q + (x < rem ? 1 : 0);
    for (int b = 0; b < n; ++b) out[b] = order[start[b % 8] + b / 8];
}

int default_slices(flapw_prec prec) { return prec == FLAPW_PREC_SPLIT_I8 ? 6 : 5; }

// Digit storage of one problem inside a digit buffer.
struct DigitArea {
    int8_t *L, *RS, *RH;
    int *eL, *eRS, *eRH;
};

long long digit_area_bytes(long long kp2, long long np, int s)
{
    const long long one = round_up(2LL * s * kp2 * np, 256);
    return 3 * one + 3 * round_up(np * 4, 256);
}

DigitArea digit_area(void *base, long long kp2, long long np, int s)
{
    const long long one = round_up(2LL * s * kp2 * np, 256);
    const long long ex = round_up(np * 4, 256);
    unsigned char *b = (unsigned char *)base;
    return DigitArea{(int8_t *)b, (int8_t *)(b + one), (int8_t *)(b + 2 * one), (int *)(b + 3 * one),
                     (int *)(b + 3 * one + ex), (int *)(b + 3 * one + 2 * ex)};
}

flapw_status slice_problem(flapw_handle h, const ProblemDev &pb, long long np, int s, const DigitArea &da,
                           hipStream_t st)
{
    ProfScope prof(h, "slice", st);
    hipError_t e = launch_split_slice(pb.P, pb.Q, pb.d, pb.ldp, pb.kp2, (int)np, s, da.eL, da.eRS, da.eRH, da.L,
                                      da.RS, da.RH, st);
    if (e != hipSuccess) return dev_fail(h, e, "digit slicing kernels");
    return FLAPW_OK;
}

flapw_status run_split(flapw_handle h, const std::vector<SplitProblemDev> &probs, const std::vector<int> &npt, int s,
                       hipStream_t st)
{
    std::vector<TileDev> tiles;
    build_tiles(npt, 2, tiles);
    auto &hb = h->host_sdesc;
    hb.clear();
    const size_t op = put(hb, probs.data(), probs.size());
    const size_t ot = put(hb, tiles.data(), tiles.size());
    flapw_status r = upload(h, h->sdesc, hb, st);
    if (r != FLAPW_OK) return r;
    unsigned char *base = (unsigned char *)h->sdesc.p;
    ProfScope prof(h, "hs_split", st);
    hipError_t e = launch_split_contract((const SplitProblemDev *)(base + op), (const TileDev *)(base + ot),
                                         (int)tiles.size(), s, st);
    if (e != hipSuccess) return dev_fail(h, e, "S/H split-precision kernel");
    return FLAPW_OK;
}

// FP64 contraction stage for a batch of problems whose P and Q are in the work buffer.
flapw_status run_fp64(flapw_handle h, const std::vector<ProblemDev> &probs_in, const std::vector<int> &npt,
                      hipStream_t s)
{
    std::vector<TileDev> tiles;
    build_tiles(npt, 1, tiles);
    auto &hb = h->host_tiles;
    hb.clear();
    const size_t op = put(hb, probs_in.data(), probs_in.size());
    const size_t ot = put(hb, tiles.data(), tiles.size());
    flapw_status st = upload(h, h->tiles, hb, s);
    if (st != FLAPW_OK) return st;
    unsigned char *base = (unsigned char *)h->tiles.p;
    ProfScope prof(h, "hs_fp64", s);
    hipError_t e = launch_hs_fp64((const ProblemDev *)(base + op), (const TileDev *)(base + ot), (int)tiles.size(), s);
    if (e != hipSuccess) return dev_fail(h, e, "S/H FP64 kernel");
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
    split_release(h);
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
    }
    return "unknown status";
}

const char *flapw_last_error(flapw_handle h) { return h ? h->err.c_str() : "NULL handle"; }

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
    static const char *known[] = {"coeffs", "tmat", "qpanel", "repack", "hs_fp64", "slice", "hs_split"};
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

long long flapw_workspace_bytes(flapw_handle h)
{
    if (!h) return -1;
    return (long long)(h->work.n + h->tmat.n + h->tables.n + h->gaunt.n + h->tiles.n) + split_bytes(h);
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
                                 rad->n_types, pref, (double2 *)A, (double2 *)B, ld, 0, 0, s);
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
    if (!A || !B || !T || !H || !S) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (n_g < 1) return fail(h, FLAPW_ERR_ARG, "n_g must be >= 1");
    if (prec != FLAPW_PREC_FP64 && prec != FLAPW_PREC_SPLIT_BF16 && prec != FLAPW_PREC_SPLIT_I8)
        return fail(h, FLAPW_ERR_ARG, "unknown precision");
    if (slices < 0 || slices > FLAPW_SLICES_CAP) return fail(h, FLAPW_ERR_ARG, "slices out of range");
    if (prec == FLAPW_PREC_SPLIT_I8 && slices != 0 && (slices < 3 || slices > 6))
        return fail(h, FLAPW_ERR_UNSUPPORTED, "int8 split precision supports 3..6 digits");
    if (prec == FLAPW_PREC_SPLIT_BF16) return fail(h, FLAPW_ERR_UNSUPPORTED, "bf16 split precision is not built");
    flapw_status st = check_radial(h, rad);
    if (st != FLAPW_OK) return st;
    if ((st = check_atoms(h, at, rad, false)) != FLAPW_OK) return st;
    Layout L;
    build_layout(at, rad, true, L);
    if (lda < L.k) return fail(h, FLAPW_ERR_ARG, "lda < K");
    if (ldt < 2LL * L.nlmax) return fail(h, FLAPW_ERR_ARG, "ldt < 2 NL_max");
    if (ldh < n_g) return fail(h, FLAPW_ERR_ARG, "ldh < n_g");
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    hipStream_t s = (hipStream_t)stream;
    const long long np = round_up(n_g, kTile);
    hipError_t e = h->work.ensure((size_t)2 * L.kp2 * np * sizeof(double2));
    if (e != hipSuccess) return dev_fail(h, e, "allocating work buffer");
    double2 *P = (double2 *)h->work.p;
    double2 *Q = P + L.kp2 * np;
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
    if ((st = upload(h, h->tables, hb, s)) != FLAPW_OK) return st;
    unsigned char *base = (unsigned char *)h->tables.p;
    {
        ProfScope prof(h, "repack", s);
        e = launch_repack((const double2 *)A, (const double2 *)B, lda, n_g, nullptr, 0, (const long long *)(base + osrc), P,
                      L.kp2, (int)L.kp2, (int)np, s);
    }
    if (e != hipSuccess) return dev_fail(h, e, "repack kernel");
    {
        ProfScope prof(h, "qpanel", s);
        e = launch_qpanel((const double2 *)T, ldt, ldt * ldt, (const int *)(base + oty), (const int *)(base + onl),
                          (const long long *)(base + orow), at->n_atoms, P, Q, L.kp2, (int)np, s);
    }
    if (e != hipSuccess) return dev_fail(h, e, "Q panel kernel");
    ProblemDev pd{P, Q, (const double *)(base + od), (double2 *)H, (double2 *)S, L.kp2, ldh, n_g, (int)L.kp2};
    std::vector<int> npt{(int)(np / kTile)};
    if (prec == FLAPW_PREC_FP64) return run_fp64(h, {pd}, npt, s);
    const int sl = slices ? slices : default_slices(prec);
    e = h->digits.ensure((size_t)digit_area_bytes(L.kp2, np, sl));
    if (e != hipSuccess) return dev_fail(h, e, "allocating digit buffer");
    const DigitArea da = digit_area(h->digits.p, L.kp2, np, sl);
    if ((st = slice_problem(h, pd, np, sl, da, s)) != FLAPW_OK) return st;
    SplitProblemDev sp{da.L, da.RS, da.RH, da.eL, da.eRS, da.eRH, (double2 *)H, (double2 *)S, ldh, n_g, (int)L.kp2};
    return run_split(h, {sp}, npt, sl, s);
}

flapw_status flapw_hs_generate(flapw_handle h, int n_k, const double *k, const int *n_g, const double *const *g,
                               const flapw_atoms *at, const flapw_radial *rad, const flapw_potential *pot,
                               flapw_z *const *H, flapw_z *const *S, const long *ldh, flapw_prec prec, int slices,
                               flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    if (n_k < 1) return fail(h, FLAPW_ERR_ARG, "n_k must be >= 1");
    if (!k || !n_g || !g || !H || !S || !ldh) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (prec != FLAPW_PREC_FP64 && prec != FLAPW_PREC_SPLIT_BF16 && prec != FLAPW_PREC_SPLIT_I8)
        return fail(h, FLAPW_ERR_ARG, "unknown precision");
    if (slices < 0 || slices > FLAPW_SLICES_CAP) return fail(h, FLAPW_ERR_ARG, "slices out of range");
    if (prec == FLAPW_PREC_SPLIT_I8 && slices != 0 && (slices < 3 || slices > 6))
        return fail(h, FLAPW_ERR_UNSUPPORTED, "int8 split precision supports 3..6 digits");
    if (prec == FLAPW_PREC_SPLIT_BF16) return fail(h, FLAPW_ERR_UNSUPPORTED, "bf16 split precision is not built");
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
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    hipStream_t s = (hipStream_t)stream;

    Layout L;
    build_layout(at, rad, true, L);
    const long long ldt = 2LL * L.nlmax;
    hipError_t e = h->tmat.ensure((size_t)rad->n_types * ldt * ldt * sizeof(double2));
    if (e != hipSuccess) return dev_fail(h, e, "allocating T");
    if ((st = build_T_impl(h, rad, pot, (double2 *)h->tmat.p, ldt, s)) != FLAPW_OK) return st;

    auto &hb = h->host_tables;
    hb.clear();
    const size_t oa = put(hb, L.atoms.data(), L.atoms.size());
    const size_t ot = put(hb, L.types.data(), L.types.size());
    const size_t od = put(hb, L.d.data(), L.d.size());
    const size_t oty = put(hb, L.atom_type.data(), L.atom_type.size());
    const size_t onl = put(hb, L.atom_nl2.data(), L.atom_nl2.size());
    const size_t orow = put(hb, L.atom_row.data(), L.atom_row.size());
    if ((st = upload(h, h->tables, hb, s)) != FLAPW_OK) return st;
    unsigned char *base = (unsigned char *)h->tables.p;
    const double pref = 4.0 * kPi / std::sqrt(at->omega);

    // Memory batches of k-points.  FP64: the P and Q panels of every k-point of a batch stay
    // resident for one grouped contraction launch.  Split precision: P and Q of one k-point at a
    // time are cut into digits (the FP64 panels are reused), and the digits of every k-point of a
    // batch stay resident for the grouped launch.
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return dev_fail(h, e, "hipMemGetInfo");
    double frac = 0.55;
    if (const char *env = std::getenv("FLAPW_WORK_FRACTION")) frac = std::atof(env);
    const bool split = prec != FLAPW_PREC_FP64;
    const int sl = split ? (slices ? slices : default_slices(prec)) : 0;
    long long np_max = 0;
    for (int i = 0; i < n_k; ++i) np_max = std::max(np_max, round_up(n_g[i], kTile));
    const size_t panel_one = (size_t)2 * L.kp2 * np_max * sizeof(double2);
    size_t budget = (size_t)(frac * (double)total_b);
    std::vector<size_t> need(n_k);
    for (int i = 0; i < n_k; ++i) {
        const long long np = round_up(n_g[i], kTile);
        need[i] = split ? (size_t)digit_area_bytes(L.kp2, np, sl) : (size_t)2 * L.kp2 * np * sizeof(double2);
    }
    if (split) {
        e = h->work.ensure(panel_one);
        if (e != hipSuccess) return dev_fail(h, e, "allocating work buffer");
        budget = budget > panel_one ? budget - panel_one : 0;
    }
    int i0 = 0;
    while (i0 < n_k) {
        int i1 = i0;
        size_t tot = 0;
        while (i1 < n_k && (i1 == i0 || tot + need[i1] <= budget)) tot += need[i1++];
        e = (split ? h->digits : h->work).ensure(tot);
        if (e != hipSuccess) return dev_fail(h, e, split ? "allocating digit buffer" : "allocating work buffer");
        std::vector<ProblemDev> probs;
        std::vector<SplitProblemDev> sprobs;
        std::vector<int> npt;
        size_t off = 0;
        for (int i = i0; i < i1; ++i) {
            const long long np = round_up(n_g[i], kTile);
            double2 *P = (double2 *)((unsigned char *)h->work.p + (split ? 0 : off));
            double2 *Q = P + L.kp2 * np;
            {
                ProfScope prof(h, "coeffs", s);
                e = launch_coeffs(k + 3 * i, n_g[i], (int)np, g[i], (const AtomDev *)(base + oa), at->n_atoms,
                                  (const TypeDev *)(base + ot), rad->n_types, pref, P, P, L.kp2, 2 * L.k, L.kp2, s);
            }
            if (e != hipSuccess) return dev_fail(h, e, "coefficient kernel");
            {
                ProfScope prof(h, "qpanel", s);
                e = launch_qpanel((const double2 *)h->tmat.p, ldt, ldt * ldt, (const int *)(base + oty),
                                  (const int *)(base + onl), (const long long *)(base + orow), at->n_atoms, P, Q,
                                  L.kp2, (int)np, s);
            }
            if (e != hipSuccess) return dev_fail(h, e, "Q panel kernel");
            const ProblemDev pd{P, Q, (const double *)(base + od), (double2 *)H[i], (double2 *)S[i], L.kp2,
                                (long long)ldh[i], n_g[i], (int)L.kp2};
            if (split) {
                const DigitArea da = digit_area((unsigned char *)h->digits.p + off, L.kp2, np, sl);
                if ((st = slice_problem(h, pd, np, sl, da, s)) != FLAPW_OK) return st;
                sprobs.push_back(SplitProblemDev{da.L, da.RS, da.RH, da.eL, da.eRS, da.eRH, (double2 *)H[i],
                                                 (double2 *)S[i], (long long)ldh[i], n_g[i], (int)L.kp2});
            } else {
                probs.push_back(pd);
            }
            off += need[i];
            npt.push_back((int)(np / kTile));
        }
        st = split ? run_split(h, sprobs, npt, sl, s) : run_fp64(h, probs, npt, s);
        if (st != FLAPW_OK) return st;
        i0 = i1;
    }
    return FLAPW_OK;
}

}  // extern "C"
