// Internal declarations shared by the library's HIP sources (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "flapw.h"

namespace flapw {

constexpr double kPi = 3.14159265358979323846;

// Per atom, as the coefficient kernel reads it.
struct AtomDev {
    double pos[3];
    double rot[9];        // row-major R_a
    int type;
    int nl;               // (lmax(type)+1)^2
    long long rowA;       // first output row of this atom's A block
    long long rowB;       // first output row of this atom's B block
};

// Per (type, l) radial boundary data, as the coefficient kernel reads it.
struct RadialDev {
    double u, du, ud, dud;
    double inv_w;         // 1 / W, W = udot u' - u udot'
    double ud_norm2;      // ||udot_l||^2
};

constexpr int kMaxTypes = 64;
constexpr int kLStride = FLAPW_LMAX_CAP + 1;

struct TypeDev {
    double rmt;
    int lmax;
    int pad;
    RadialDev rad[kLStride];
};

// One k-point problem of the contraction stage (padded work layout).
//   P, Q : kp2 x np complex, column-major (ld = ldp).  Rows are the atoms in order, each as
//          [A_a (NL_a rows); B_a (NL_a rows)], followed by zero rows up to kp2.  Columns
//          n..np-1 are zero.
//   d    : kp2 row weights of S (1 on A rows, ||udot_l||^2 on B rows, 0 on padding).
struct ProblemDev {
    const double2 *P;
    const double2 *Q;
    const double *d;
    double2 *H;
    double2 *S;
    long long ldp;
    long long ldh;
    int n;
    int kp2;
};

// Split-precision operands of one k-point (digit layout described in split.hip).
struct SplitProblemDev {
    const void *L;        // left digits (from P)
    const void *R;        // right digits of S (from the d-weighted P)
    const void *RQ;       // right digits of H (from Q)
    const int *eL;        // per-column scale exponents, np entries each
    const int *eR;
    const int *eRQ;
    double2 *H;
    double2 *S;
    long long ldh;
    int n;
    int kp2;              // contraction rows (padded)
};

struct TileDev {
    int prob;             // problem index
    int ti;               // tile row
    int tj;               // tile column (ti <= tj)
    int pad;              // split precision: 0 = S tile, 1 = H tile
};

// kernel launchers (return hipError_t of the launch)
// nlmax: the largest (lmax+1)^2 over the atom types (sizes the kernel's LDS)
hipError_t launch_coeffs(const double kvec[3], int n_g, int n_cols, const double *g, const AtomDev *atoms, int n_atoms,
                         const TypeDev *types, int n_types, int nlmax, double pref, double2 *A, double2 *B,
                         long long ld, long long zero_rows_from, long long zero_rows_to, hipStream_t s);

hipError_t launch_legendre_table(int lt, int nq, const double *z, double *theta, hipStream_t s);
// lmax_dev: l_max of each type's row blocks; lnonsph >= 0: structured T (non-spherical terms only
// for l', l <= lnonsph)
hipError_t launch_tmat(int n_types, const int *lmax_dev, int lstride, int lpot, int nq, const double *w,
                       const double *theta, const double *i_uu, const double *i_ud, const double *i_du,
                       const double *i_dd, const double *e_l, const double *ud_norm2, double2 *T, long long ldt,
                       int lnonsph, hipStream_t s);
hipError_t launch_tmat_sph(int n_types, const int *lmax_dev, int lstride, int lpot, int nq, const double *w,
                           const double *theta, const double *i_uu, const double *i_ud, const double *i_du,
                           const double *i_dd, const double *e_l, const double *ud_norm2, double *out, hipStream_t s);

// Q_a = T_type(a) P_a for every atom; rows from the end of the last atom block up to kp2 are set
// to zero.  real_t: T is known to be real (built by the library from real integrals): half the MFMAs
// Q_a = T_a P_a for every atom.  With part (real T only; d the row weights), the real-T kernel also
// writes per (atom, row tile) shares of the column sums sum |P|^2, sum |P|^2 d^2 and sum |Q|^2:
// 3 x qpanel_row_tiles(ldt) x n_atoms x np doubles (qpanel_colsum_doubles), summed by
// launch_mod_slice.
constexpr int kQRowsPerTile = 256;
inline int qpanel_row_tiles(long long ldt) { return (int)((ldt + kQRowsPerTile - 1) / kQRowsPerTile); }
inline long long qpanel_colsum_doubles(long long ldt, int n_atoms, long long np)
{
    return 3LL * qpanel_row_tiles(ldt) * n_atoms * np;
}
hipError_t launch_qpanel(const double2 *T, long long ldt, long long tstride, const int *atom_type, const int *atom_nl2,
                         const long long *atom_row, int n_atoms, const double2 *P, double2 *Q, long long ldp, int np,
                         long long kp2, bool real_t, int min_nl2, const double *d, double *part, hipStream_t s);

// with_s = false: H alone (S tiles of the problems are not touched)
hipError_t launch_hs_fp64(const ProblemDev *probs, const TileDev *tiles, int n_tiles, bool with_s, hipStream_t s);

hipError_t launch_repack(const double2 *A, const double2 *B, long long lda, int n_g, const AtomDev *atoms,
                         int n_atoms, const long long *src_off, double2 *P, long long ldp, int kp2, int np,
                         hipStream_t s);

long long split_digit_bytes(long long kp2, long long np, int s);
// dynamic-LDS attributes of the contraction kernels (set once, before any launch or graph capture)
hipError_t init_fp64_kernels();
hipError_t init_split_kernels();
hipError_t launch_split_slice(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                              int slices, int *eL, int *eRS, int *eRH, int8_t *L, int8_t *RS, int8_t *RH,
                              hipStream_t s);
hipError_t launch_split_contract(const SplitProblemDev *probs, const TileDev *tiles, int n_tiles, int slices,
                                 hipStream_t s);
// bf16 digits (split_bf16.hip): same operands, 2 bytes per digit, 8-row chunks
hipError_t init_split_bf16_kernels();
hipError_t launch_split_bf16_slice(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                                   int slices, int *eL, int *eRS, int *eRH, void *L, void *RS, void *RH, hipStream_t s);
hipError_t launch_split_bf16_contract(const SplitProblemDev *probs, const TileDev *tiles, int n_tiles, int slices,
                                      hipStream_t s);

// Overlap matrix through the addition theorem (legendre.hip).
//   khat : np x 4 doubles (unit K_t), ab : n_types x kLStride x np x 2 doubles {alpha, beta},
//   E    : np columns of ldE complex phases exp(i K_t.x_a), rows grouped by type.
struct LegTypeRange {
    int row0;             // first row of the type's atoms in E
    int rows;             // rows of the type (multiple of 16; padding rows hold zeros)
    int lmax;
    int pad;
};
hipError_t init_legendre_kernels();
hipError_t launch_legendre_prep(const double kvec[3], int n_g, int np, const double *g, const TypeDev *types,
                                int n_types, const double *apos, const int *arow, int n_atoms, double *khat,
                                double *ab, double2 *E, long long ldE, hipStream_t s);
// tiles: n_tiles (ti, tj) pairs with ti <= tj; S written on the upper triangle, scale = 4 pi / Omega.
// H != nullptr: also adds to H (upper triangle) the L-diagonal T terms of l >= lh0, with
// hsph = n_types x kLStride x {aa, ab, ba, bb}.
// ud_norm2: n_types x kLStride values of ||udot_l||^2.
hipError_t launch_s_legendre(const double *khat, const double *ab, const double2 *E, long long ldE,
                             const LegTypeRange *ranges, int n_types, const int *tiles, int n_tiles, int np, int n,
                             double scale, double2 *S, long long lds, const double *ud_norm2, const double *hsph,
                             int lh0, double2 *H, long long ldh, hipStream_t s);

// Interstitial S and H (interstitial.hip): phases E and ranges as for launch_s_legendre; g the
// n x 3 Cartesian G list; adds to the upper triangles of S and H.
hipError_t init_interstitial_kernel();
hipError_t launch_interstitial(const double *g, const double kvec[3], const double2 *E, long long ldE,
                               const LegTypeRange *ranges, const TypeDev *types, int n_types, const int *tiles,
                               int n_tiles, int n, double omega, double v_int, double2 *S, long long lds, double2 *H,
                               long long ldh, hipStream_t s);

// Modular split precision (split_mod.hip).  Moduli p_m, 1/p_m as double-double, the CRT
// constants w_m = (M/p_m)^-1 mod p_m, M = prod p_m as double-double, and the integer range: the
// column norm 2^B the operands are scaled to (bits_real = B, bits = floor(B), two2b = 2^B).  Per
// modulus also a square root j_m of -1 and the inverses of 2 and of 2 j_m (all in the symmetric
// range), which split the complex products mod p_m into two real ones.
constexpr int kModCap = 14;
constexpr int kModMin = 8;
constexpr int kModTile = 128;   // output tile edge of the modular contraction
constexpr int kResTileBytes = kModTile * kModTile * 2;  // int8 residues of Re and Im of one tile
// slot of upper-triangle tile (ti <= tj) in the residue scratch of one matrix
__host__ __device__ inline int tri_index(int ti, int tj) { return tj * (tj + 1) / 2 + ti; }
struct ModTable {
    int nm;
    int bits;
    double bits_real;
    double two2b;
    int p[kModCap];
    int w[kModCap];
    int jr[kModCap];
    int h2[kModCap];
    int h2j[kModCap];
    double inv_p[kModCap];
    double inv_p_lo[kModCap];
    double M_hi, M_lo;
};
// One k-point of the modular contraction.  L, RS, RH: residue planes (layout in split_mod.hip),
// ncb 32-column blocks wide; res: residue tiles, 2 ntri slots per modulus (S tiles, then H).
struct ModProblemDev {
    const int8_t *L, *RS, *RH;
    const double *sL, *sRS, *sRH;     // column scales (integers = rint(value * scale))
    double2 *H, *S;
    int8_t *res;
    long long ldh;
    int n;
    int kp2;
    int ncb;
    int ntri;
};
ModTable make_mod_table(int nm);
hipError_t init_mod_kernels();    // dynamic-LDS attribute of the contraction (before launch or capture)
long long mod_digit_bytes(long long kp2, long long npm, int nm);
long long mod_scratch_bytes(long long npm, int nm);
// with_s = false: no S operand.  part: the column-sum shares of the real-T panel kernel over
// n_slots (atom, row tile) slots, or nullptr to read the column norms from P and Q.
hipError_t launch_mod_slice(const double2 *P, const double2 *Q, const double *d, long long ld, int kp2, int np,
                            int npm, const ModTable &mt, double *sL, double *sRS, double *sRH, int8_t *L, int8_t *RS,
                            int8_t *RH, bool with_s, const double *part, long long n_slots, hipStream_t s);
// chunks: 16-row chunks per LDS stage of the contraction kernel (4 or 2)
hipError_t launch_mod_contract(const ModProblemDev *probs, const TileDev *tiles, int n_tiles, const ModTable &mt,
                               int chunks, hipStream_t s);
hipError_t launch_mod_crt(const ModProblemDev *probs, const TileDev *tiles, int n_tiles, const ModTable &mt,
                          hipStream_t s);

// Radial functions and radial integrals (radial.hip).  fun: scratch of radial_fun_bytes();
// bnd: n_types x kLStride x 5 (u, u', udot, udot', ||udot||^2); i_*: the four flapw_potential
// tables, zero-filled by the caller.
size_t radial_fun_bytes(int n_types, int n_r);
hipError_t launch_radial(int n_types, int n_r, int nlp, const double *r0, const double *rmt, const int *lmax,
                         const double *e_l, int lstride, const double *v_sph, const double *v_lm, double *fun,
                         double *bnd, double *i_uu, double *i_ud, double *i_du, double *i_dd, hipStream_t s);

constexpr int kTile = 64;     // output tile edge (complex elements) of the contraction kernels
constexpr int kKTile = 16;    // contraction rows per pipeline stage (FP64 kernels)

}  // namespace flapw
