// FP64 matrix-core kernels of the contraction stage.
//
//  qpanel_real_kernel : Q_a = T_type(a) P_a for every atom (the paper's X_a, Z_a of sections
//                  4.4-4.6, here for the whole 2NL x 2NL block T at once), P_a = [A_a; B_a], for a
//                  real T (the generation path: real radial integrals and Gaunt coefficients);
//  qpanel_kernel : the same for a complex T supplied by the caller.
//  hs_fp64_kernel: upper-triangle 64 x 64 tiles of
//                    S = P^H D P   (D = 1 on A rows, ||udot_l||^2 on B rows; eq. def_overlap)
//                    H = P^H Q     (eq. def_hamilton)
//                  for one or many k-points (grouped launch over a host-built tile list).
//                  The contraction index runs over all atoms' rows, so the per-atom sum of the
//                  paper is the K-loop of the tile and is accumulated in FP64 registers.
//
// Both kernels compute C = X^H Y on 64 x 64 complex tiles with v_mfma_f64_16x16x4f64.  A complex
// product uses four real products (Re = Xr.Yr + Xi.Yi, Im = Xr.Yi - Xi.Yr).  Operands are
// column-major with the contraction index contiguous, so a 16-row stage of one column is one
// 256-byte segment; stages are double-buffered in LDS as [column][k] complex panels padded to
// 17 slots per column, so that the MFMA operand reads (lane l: row k = l/16, column l%16, one
// 16-byte {re, im} read) and the staging writes are both free of bank conflicts.
// Each wave owns a 32 x 32 quadrant (2 x 2 MFMA blocks); the accumulator of block (m, n) holds
// rows l/16 + 4r, column l%16 in register r of lane l.
#include "common.hpp"

namespace flapw {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
// Operand pointers are read from descriptors, so the compiler cannot infer that they point to
// global memory; the address-space qualifier makes it emit global (not flat) loads, whose
// completion is tracked apart from LDS traffic.  (The host compilation pass only parses.)
#if defined(__HIP_DEVICE_COMPILE__)
typedef const double2 __attribute__((address_space(1))) gdouble2;
typedef const double __attribute__((address_space(1))) gdouble;
#else
typedef const double2 gdouble2;
typedef const double gdouble;
#endif

constexpr int kThreads = 256;
constexpr int kSlot = kKTile + 1;           // complex slots per column in LDS (one pad slot)

__device__ __forceinline__ v4d mfma(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One LDS stage of C += X^H Y for a wave's 2 x 2 blocks and NY right operands sharing X.
// LDS panels are [column][k] complex; lane l reads row k = ks + l/16 of column base + l%16.
// acc[y][0] = Re, acc[y][1] = Im.  The first sweep issues Xr.Yr and Xr.Yi for every block, the
// second Xi.Yi and -Xi.Yr, so no two consecutive MFMAs use the same accumulator.
template <int NY, int KS0 = 0, int KSTEP = 4>
__device__ __forceinline__ void stage_mma(const double2 (*X)[kSlot], const double2 (*Y0)[kSlot],
                                          const double2 (*Y1)[kSlot], int wm, int wn, int lane,
                                          v4d (&acc)[NY][2][2][2])
{
    const int c = lane & 15;
#pragma unroll
    for (int ks = KS0; ks < kKTile; ks += KSTEP) {
        const int k = ks + (lane >> 4);
        double2 x[2], y[NY][2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            x[q] = X[wm + q * 16 + c][k];
            y[0][q] = Y0[wn + q * 16 + c][k];
            if constexpr (NY > 1) y[NY - 1][q] = Y1[wn + q * 16 + c][k];
        }
#pragma unroll
        for (int v = 0; v < NY; ++v)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    acc[v][0][mi][ni] = mfma(x[mi].x, y[v][ni].x, acc[v][0][mi][ni]);
                    acc[v][1][mi][ni] = mfma(x[mi].x, y[v][ni].y, acc[v][1][mi][ni]);
                }
#pragma unroll
        for (int v = 0; v < NY; ++v)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    acc[v][0][mi][ni] = mfma(x[mi].y, y[v][ni].y, acc[v][0][mi][ni]);
                    acc[v][1][mi][ni] = mfma(-x[mi].y, y[v][ni].x, acc[v][1][mi][ni]);
                }
    }
}

struct HsSmem {
    double2 v[2][3][kTile][kSlot];          // [buffer][left P, right d.P, right Q][column][k]
};

constexpr int kHsThreads = 512;             // 8 waves: two per SIMD, splitting each stage's k-steps

// Eight waves: wave w owns quadrant (w & 3) of the 64 x 64 tile (2 x 2 MFMA blocks) and the
// k-steps {0, 8} (w < 4) or {4, 12} (w >= 4) of every 16-row stage, so two waves per SIMD
// keep the FP64 matrix core busy across barriers and LDS waits.  Their partial sums are
// added through LDS at the end; with S, waves 0-3 then store S and waves 4-7 store H.
// WITH_S = false computes H alone (S comes from another method) and stages no d.P panel.
template <bool WITH_S>
__global__ __launch_bounds__(kHsThreads, 1) void hs_fp64_kernel(const ProblemDev *__restrict__ probs,
                                                                const TileDev *__restrict__ tiles)
{
    constexpr int NM = WITH_S ? 2 : 1;                 // matrices: [S,] H
    extern __shared__ __align__(16) unsigned char smem_raw[];
    HsSmem &sm = *reinterpret_cast<HsSmem *>(smem_raw);

    const TileDev td = tiles[blockIdx.x];
    const ProblemDev pb = probs[td.prob];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quad = wave & 3, khalf = wave >> 2;
    const int wm = (quad >> 1) * 32, wn = (quad & 1) * 32;
    const long long i0 = (long long)td.ti * kTile, j0 = (long long)td.tj * kTile;

    const int lc = tid >> 3, lk = (tid & 7) * 2;       // loader: column lc, rows lk, lk+1 of a stage
    gdouble2 *gL = (gdouble2 *)pb.P + (i0 + lc) * pb.ldp + lk;
    gdouble2 *gR = (gdouble2 *)pb.P + (j0 + lc) * pb.ldp + lk;
    gdouble2 *gQ = (gdouble2 *)pb.Q + (j0 + lc) * pb.ldp + lk;
    gdouble *gd = (gdouble *)pb.d + lk;

    v4d acc[NM][2][2][2];                              // [S,] H x [re, im][mi][ni]
#pragma unroll
    for (int a = 0; a < NM; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n) acc[a][b][m][n] = (v4d){0.0, 0.0, 0.0, 0.0};

    // Stage loads go through registers (issued one stage ahead) and are written to LDS after the
    // MFMAs of the current stage.  Plain scalars, not captured arrays, keep them in registers.
    double2 l0, l1, r0, r1, q0, q1;
    double d0, d1;
#define HS_LOAD(kt)                                                     \
    do {                                                                \
        const long long off_ = (long long)(kt) * kKTile;                \
        l0 = gL[off_]; l1 = gL[off_ + 1];                               \
        if (WITH_S) {                                                   \
            r0 = gR[off_]; r1 = gR[off_ + 1];                           \
            d0 = gd[off_]; d1 = gd[off_ + 1];                           \
        }                                                               \
        q0 = gQ[off_]; q1 = gQ[off_ + 1];                               \
    } while (0)
#define HS_STORE(b)                                                                              \
    do {                                                                                         \
        double2 *sl_ = &sm.v[b][0][lc][lk], *sr_ = &sm.v[b][1][lc][lk], *sq_ = &sm.v[b][2][lc][lk]; \
        sl_[0] = l0; sl_[1] = l1;                                                                \
        if (WITH_S) {                                                                            \
            sr_[0] = make_double2(r0.x * d0, r0.y * d0); sr_[1] = make_double2(r1.x * d1, r1.y * d1); \
        }                                                                                        \
        sq_[0] = q0; sq_[1] = q1;                                                                \
    } while (0)

    const int nkt = pb.kp2 / kKTile;
    HS_LOAD(0);
    HS_STORE(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        const int b = kt & 1;
        if (kt + 1 < nkt) HS_LOAD(kt + 1);
        if (WITH_S) {
            if (khalf == 0) stage_mma<NM, 0, 8>(sm.v[b][0], sm.v[b][1], sm.v[b][2], wm, wn, lane, acc);
            else            stage_mma<NM, 4, 8>(sm.v[b][0], sm.v[b][1], sm.v[b][2], wm, wn, lane, acc);
        } else {
            if (khalf == 0) stage_mma<NM, 0, 8>(sm.v[b][0], sm.v[b][2], sm.v[b][2], wm, wn, lane, acc);
            else            stage_mma<NM, 4, 8>(sm.v[b][0], sm.v[b][2], sm.v[b][2], wm, wn, lane, acc);
        }
        if (kt + 1 < nkt) HS_STORE(b ^ 1);
        __syncthreads();
    }
#undef HS_LOAD
#undef HS_STORE

    // add the two halves: S partials of waves 4-7 to waves 0-3, then H partials the other way
    // (H alone: waves 4-7 to waves 0-3)
    double *xch = reinterpret_cast<double *>(smem_raw);   // [quadrant][32 values][64 lanes]
#pragma unroll
    for (int mat = 0; mat < NM; ++mat) {
        const bool sender = (mat == 0) ? (khalf == 1) : (khalf == 0);
        if (sender) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            xch[((quad * 32) + ((c * 2 + mi) * 2 + ni) * 4 + r) * 64 + lane] = acc[mat][c][mi][ni][r];
        }
        __syncthreads();
        if (!sender) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            acc[mat][c][mi][ni][r] += xch[((quad * 32) + ((c * 2 + mi) * 2 + ni) * 4 + r) * 64 + lane];
        }
        __syncthreads();
    }

    // epilogue: upper triangle (row <= col < n); diagonal imaginary part set to zero
    const int mat = WITH_S ? khalf : 0;                     // with S: waves 0-3 store S, waves 4-7 H
    if (!WITH_S && khalf == 1) return;
    double2 *out = (WITH_S && mat == 0) ? pb.S : pb.H;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = i0 + wm + mi * 16 + (lane >> 4) + 4 * r;
                const long long col = j0 + wn + ni * 16 + (lane & 15);
                if (row <= col && col < pb.n) {
                    const double re = mat == 0 ? acc[0][0][mi][ni][r] : acc[NM - 1][0][mi][ni][r];
                    const double im = mat == 0 ? acc[0][1][mi][ni][r] : acc[NM - 1][1][mi][ni][r];
                    out[col * pb.ldh + row] = make_double2(re, row == col ? 0.0 : im);
                }
            }
}

struct QSmem {
    double2 v[2][2][kTile][kSlot];          // [buffer][X = T columns, Y = P rows of the atom][column][k]
};

// One block per (atom, 64-column tile, 64-row tile of the atom's 2NL rows); complex T.
__global__ __launch_bounds__(kThreads, 1) void qpanel_kernel(const double2 *__restrict__ T, long long ldt,
                                                             long long tstride, const int *__restrict__ atom_type,
                                                             const int *__restrict__ atom_nl2,
                                                             const long long *__restrict__ atom_row,
                                                             const double2 *__restrict__ P, double2 *__restrict__ Q,
                                                             long long ldp, int n_atoms, long long kp2, int n_ct,
                                                             int row_tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    QSmem &sm = *reinterpret_cast<QSmem *>(smem_raw);

    // Block order: the row tiles of one (atom, column tile) unit are dispatched back to back on
    // one XCD (work-group b runs on XCD b mod 8), so the unit's panel of P is read from HBM once
    // and then found in that XCD's L2.  Unit u = atom * n_ct + column tile goes to XCD u mod 8.
    const int xcd = blockIdx.x & 7, rest = blockIdx.x >> 3;
    const int rt = rest % row_tiles;
    const long long u = (long long)(rest / row_tiles) * 8 + xcd;
    if (u >= (long long)(n_atoms + 1) * n_ct) return;
    const int a = (int)(u / n_ct);
    const int ctile = (int)(u % n_ct);
    if (a == n_atoms) {                                 // the padding rows of Q are zero, like P's
        if (rt != 0) return;
        const long long c0 = (long long)ctile * kTile;
        const long long pad0 = atom_row[n_atoms - 1] + atom_nl2[n_atoms - 1];
        const long long nr = kp2 - pad0;
        for (long long i = threadIdx.x; i < nr * kTile; i += blockDim.x)
            Q[(c0 + i / nr) * ldp + pad0 + i % nr] = make_double2(0.0, 0.0);
        return;
    }
    const int m2 = atom_nl2[a];                         // 2 NL of this atom
    const int r0 = rt * kTile;
    if (r0 >= m2) return;
    const long long prow = atom_row[a];
    const long long c0 = (long long)ctile * kTile;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lc = tid >> 2, lk = (tid & 3) * 4;
    const bool xcol_ok = (r0 + lc) < m2;
    gdouble2 *gX = (gdouble2 *)T + (long long)atom_type[a] * tstride + (long long)(xcol_ok ? r0 + lc : 0) * ldt + lk;
    gdouble2 *gY = (gdouble2 *)P + (c0 + lc) * ldp + prow + lk;

    v4d acc[1][2][2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[0][q][m][n] = (v4d){0.0, 0.0, 0.0, 0.0};

    double2 x0, x1, x2, x3, y0, y1, y2, y3;
#define Q_LOAD(kt)                                                           \
    do {                                                                     \
        const int k0_ = (kt) * kKTile + lk, o_ = (kt) * kKTile;              \
        const double2 z_ = make_double2(0.0, 0.0);                           \
        x0 = z_; x1 = z_; x2 = z_; x3 = z_; y0 = z_; y1 = z_; y2 = z_; y3 = z_; \
        if (k0_ + 0 < m2) { y0 = gY[o_ + 0]; if (xcol_ok) x0 = gX[o_ + 0]; } \
        if (k0_ + 1 < m2) { y1 = gY[o_ + 1]; if (xcol_ok) x1 = gX[o_ + 1]; } \
        if (k0_ + 2 < m2) { y2 = gY[o_ + 2]; if (xcol_ok) x2 = gX[o_ + 2]; } \
        if (k0_ + 3 < m2) { y3 = gY[o_ + 3]; if (xcol_ok) x3 = gX[o_ + 3]; } \
    } while (0)
#define Q_STORE(b)                                                              \
    do {                                                                        \
        double2 *sx_ = &sm.v[b][0][lc][lk], *sy_ = &sm.v[b][1][lc][lk];         \
        sx_[0] = x0; sx_[1] = x1; sx_[2] = x2; sx_[3] = x3;                     \
        sy_[0] = y0; sy_[1] = y1; sy_[2] = y2; sy_[3] = y3;                     \
    } while (0)
    const int nkt = (m2 + kKTile - 1) / kKTile;
    Q_LOAD(0);
    Q_STORE(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        const int b = kt & 1;
        if (kt + 1 < nkt) Q_LOAD(kt + 1);
        stage_mma<1>(sm.v[b][0], sm.v[b][1], sm.v[b][1], wm, wn, lane, acc);
        if (kt + 1 < nkt) Q_STORE(b ^ 1);
        __syncthreads();
    }
#undef Q_LOAD
#undef Q_STORE
    // T is Hermitian, so X^H Y with X = T is T P.
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wm + mi * 16 + (lane >> 4) + 4 * r;
                const long long col = c0 + wn + ni * 16 + (lane & 15);
                if (row < m2) Q[col * ldp + prow + row] = make_double2(acc[0][0][mi][ni][r], acc[0][1][mi][ni][r]);
            }
}

constexpr int kQRows = 256;                 // rows of Q_a per block of the real-T kernel
constexpr int kQThreads = 512;
static_assert(kQRows == kQRowsPerTile, "row tile of the real-T panel kernel");

struct QRealSmem {
    double x[2][kQRows][kSlot];             // [buffer][row of Q_a = column of T][k], Re T
    double2 y[2][kTile][kSlot];             // [buffer][column of P_a][k]
};

// Real T: Re Q = T Re P and Im Q = T Im P, two real products per complex element.  One block per
// unit (atom, 64-column tile, 256-row tile of the atom's 2NL rows; 2NL <= 256 needs one row tile),
// so T is read once per 64 columns and P once in all.  Eight waves: wave w owns the 16-row blocks
// (w >> 1) + 4 i, i = 0..3, and columns 32 (w & 1) of the 256 x 64 tile (4 x 2 MFMA blocks); row
// blocks are dealt round-robin so that an atom with fewer rows (2NL = 162 at l_max 8) still keeps
// every wave busy, and row blocks past 2NL are skipped, as are k-steps past 2NL (rows past them
// are zero in LDS).  Units are listed atom-major and XCD x
// (work-group b runs on XCD b mod 8) takes the x-th contiguous eighth of the list, so the column
// tiles of one atom follow each other on one XCD and find T of its type in that XCD's L2.
// FULL: every atom of the launch has 2NL > 240 and one row tile, so every row block of every wave
// holds rows and the per-block tests (which cost a few per cent) compile away.
// NORMS: the block also writes its share of three column sums, sum |P|^2, sum |P|^2 d^2 (d the row
// weights) over the atom's rows and sum |Q|^2 over the tile's rows, to part[(k n_slots + slot) np
// + column] for k = 0, 1, 2 and slot = atom * row_tiles + row tile (the P sums only from row tile
// 0, zeros from the others), each reduced in a fixed order, so that the sums over slots are
// reproducible.  Those squared column norms set the integer scaling of the modular contraction.
template <bool FULL, bool NORMS>
__global__ __launch_bounds__(kQThreads, 1) void qpanel_real_kernel(
    const double2 *__restrict__ T, long long ldt, long long tstride, const int *__restrict__ atom_type,
    const int *__restrict__ atom_nl2, const long long *__restrict__ atom_row, const double2 *__restrict__ P,
    double2 *__restrict__ Q, long long ldp, int n_atoms, long long kp2, int n_ct, int row_tiles, long long per_xcd,
    const double *__restrict__ dw, double *__restrict__ part, long long np)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    QRealSmem &sm = *reinterpret_cast<QRealSmem *>(smem_raw);

    const long long idx = blockIdx.x >> 3;
    const long long u = (long long)(blockIdx.x & 7) * per_xcd + idx;
    if (idx >= per_xcd || u >= (long long)(n_atoms + 1) * n_ct * row_tiles) return;
    const int rt = (int)(u % row_tiles);
    const long long v = u / row_tiles;
    const int a = (int)(v / n_ct);
    const long long c0 = (v % n_ct) * kTile;
    if (a == n_atoms) {                                 // the padding rows of Q are zero, like P's
        if (rt != 0) return;
        const long long pad0 = atom_row[n_atoms - 1] + atom_nl2[n_atoms - 1];
        const long long nr = kp2 - pad0;
        for (long long i = threadIdx.x; i < nr * kTile; i += blockDim.x)
            Q[(c0 + i / nr) * ldp + pad0 + i % nr] = make_double2(0.0, 0.0);
        return;
    }
    const int m2 = atom_nl2[a];                         // 2 NL of this atom
    const int r0 = rt * kQRows;
    const long long n_slots = (long long)n_atoms * row_tiles, slot = (long long)a * row_tiles + rt;
    if (r0 >= m2) {                                     // no rows here: zero shares
        if (NORMS && threadIdx.x < 3 * kTile)
            part[((threadIdx.x >> 6) * n_slots + slot) * np + c0 + (threadIdx.x & 63)] = 0.0;
        return;
    }
    const long long prow = atom_row[a];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wn = (wave & 1) * 32;
    bool act[4];                                        // row block wr + 4 i holds rows of this atom
#pragma unroll
    for (int i = 0; i < 4; ++i) act[i] = FULL || r0 + (wr + 4 * i) * 16 < m2;
    const bool active = act[0];
    // loaders: lane group g = tid / 16 reads row lk = tid % 16 of a stage in T columns (tile rows)
    // g + 32 j, j = 0..7, and in P columns g + 32 j, j = 0..1: 16 lanes cover one column's 256
    // contiguous bytes.  Only the real part of T is kept.
    const int lg = tid >> 4, lk = tid & 15;
    gdouble2 *gX = (gdouble2 *)T + (long long)atom_type[a] * tstride + (long long)(r0 + lg) * ldt + lk;
    gdouble2 *gY = (gdouble2 *)P + (c0 + lg) * ldp + prow + lk;

    v4d acc[2][4][2];                                   // [re, im][mi][ni]
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[q][m][n] = (v4d){0.0, 0.0, 0.0, 0.0};

    double xv[8];
    double2 yv[2];
    double sp[2] = {0.0, 0.0}, sd[2] = {0.0, 0.0};     // NORMS: this lane's rows of columns lg + 32 j
    double wv = 0.0;                                    // NORMS: weight of the loaded row
    auto load = [&](int kt) {
        const int kb = kt * kKTile;
        const bool k_ok = kb + lk < m2;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            xv[j] = 0.0;
            if (k_ok && r0 + lg + 32 * j < m2) xv[j] = gX[32LL * j * ldt + kb].x;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            yv[j] = make_double2(0.0, 0.0);
            if (k_ok) yv[j] = gY[32LL * j * ldp + kb];
        }
        if (NORMS) wv = k_ok ? dw[prow + kb + lk] : 0.0;
    };
    // the sums use the loaded values here, after the stage's MFMAs have covered the loads
    auto store = [&](int b) {
        if (NORMS) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const double a2 = yv[j].x * yv[j].x + yv[j].y * yv[j].y;
                sp[j] += a2;
                sd[j] += a2 * wv * wv;
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) sm.x[b][lg + 32 * j][lk] = xv[j];
#pragma unroll
        for (int j = 0; j < 2; ++j) sm.y[b][lg + 32 * j][lk] = yv[j];
    };

    const int nkt = (m2 + kKTile - 1) / kKTile;
    const int c = lane & 15;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        const int b = kt & 1;
        if (kt + 1 < nkt) load(kt + 1);
        if (active) {
            const int kv = m2 - kt * kKTile;            // rows of this stage inside the atom
#pragma unroll
            for (int ks = 0; ks < kKTile; ks += 4) {
                if (ks < kv) {
                    const int k = ks + (lane >> 4);
                    double xa[4];
                    double2 yb[2];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi) xa[mi] = act[mi] ? sm.x[b][(wr + 4 * mi) * 16 + c][k] : 0.0;
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni) yb[ni] = sm.y[b][wn + ni * 16 + c][k];
#pragma unroll
                    for (int mi = 0; mi < 4; ++mi)
                        if (act[mi]) {
#pragma unroll
                            for (int ni = 0; ni < 2; ++ni) {
                                acc[0][mi][ni] = mfma(xa[mi], yb[ni].x, acc[0][mi][ni]);
                                acc[1][mi][ni] = mfma(xa[mi], yb[ni].y, acc[1][mi][ni]);
                            }
                        }
                }
            }
        }
        if (kt + 1 < nkt) store(b ^ 1);
        __syncthreads();
    }
    if (NORMS) {
        // P sums: the 16 lanes of a loader group hold the rows of the same two columns
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                sp[j] += __shfl_xor(sp[j], o);
                sd[j] += __shfl_xor(sd[j], o);
            }
        if (lk == 0) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const long long col = c0 + lg + 32 * j;
                part[slot * np + col] = rt == 0 ? sp[j] : 0.0;
                part[(n_slots + slot) * np + col] = rt == 0 ? sd[j] : 0.0;
            }
        }
        // Q sums: rows of the lane's accumulators (zero in row blocks past 2NL), then the four lane
        // groups of a column, then the four waves with the same columns, through LDS (the stage
        // buffers are free after the last barrier)
        double sq[2];
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            sq[ni] = 0.0;
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    sq[ni] += acc[0][mi][ni][r] * acc[0][mi][ni][r] + acc[1][mi][ni][r] * acc[1][mi][ni][r];
            sq[ni] += __shfl_xor(sq[ni], 16);
            sq[ni] += __shfl_xor(sq[ni], 32);
        }
        double *red = &sm.x[0][0][0];                   // [wr][64 columns]
        if (lane < 16) {
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) red[wr * kTile + wn + ni * 16 + lane] = sq[ni];
        }
        __syncthreads();
        if (tid < kTile)
            part[(2 * n_slots + slot) * np + c0 + tid] =
                ((red[tid] + red[kTile + tid]) + red[2 * kTile + tid]) + red[3 * kTile + tid];
    }
    if (!active) return;
    // T is symmetric, so the product of its columns with P is T P.
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + (wr + 4 * mi) * 16 + (lane >> 4) + 4 * r;
                const long long col = c0 + wn + ni * 16 + (lane & 15);
                if (row < m2) Q[col * ldp + prow + row] = make_double2(acc[0][mi][ni][r], acc[1][mi][ni][r]);
            }
}

// Copy caller-supplied A_*, B_* into the work layout: per atom [A_a; B_a], zero padding.
__global__ void repack_kernel(const double2 *__restrict__ A, const double2 *__restrict__ B, long long lda, int n_g,
                              const long long *__restrict__ src, double2 *__restrict__ P, long long ldp, int kp2)
{
    const long long t = blockIdx.x;
    double2 *dst = P + t * ldp;
    for (int r = threadIdx.x; r < kp2; r += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (t < n_g) {
            const long long s = src[r];
            if (s >= 0) v = A[t * lda + s];
            else if (s <= -2) v = B[t * lda + (-s - 2)];
        }
        dst[r] = v;
    }
}

}  // namespace

hipError_t init_fp64_kernels()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    hipError_t e = hipFuncSetAttribute((const void *)hs_fp64_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sizeof(HsSmem));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)hs_fp64_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sizeof(HsSmem));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)qpanel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sizeof(QSmem));
    const void *qreal[4] = {(const void *)qpanel_real_kernel<true, false>, (const void *)qpanel_real_kernel<false, false>,
                            (const void *)qpanel_real_kernel<true, true>, (const void *)qpanel_real_kernel<false, true>};
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
        e = hipFuncSetAttribute(qreal[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(QRealSmem));
    done = e;
    return e;
}

hipError_t launch_hs_fp64(const ProblemDev *probs, const TileDev *tiles, int n_tiles, bool with_s, hipStream_t s)
{
    hipError_t e = init_fp64_kernels();
    if (e != hipSuccess) return e;
    if (with_s)
        hipLaunchKernelGGL(hs_fp64_kernel<true>, dim3(n_tiles), dim3(kHsThreads), sizeof(HsSmem), s, probs, tiles);
    else
        hipLaunchKernelGGL(hs_fp64_kernel<false>, dim3(n_tiles), dim3(kHsThreads), sizeof(HsSmem), s, probs, tiles);
    return hipGetLastError();
}

hipError_t launch_qpanel(const double2 *T, long long ldt, long long tstride, const int *atom_type, const int *atom_nl2,
                         const long long *atom_row, int n_atoms, const double2 *P, double2 *Q, long long ldp, int np,
                         long long kp2, bool real_t, int min_nl2, const double *d, double *part, hipStream_t s)
{
    hipError_t e = init_fp64_kernels();
    if (e != hipSuccess) return e;
    const int n_ct = np / kTile;
    if (real_t) {
        const int row_tiles = qpanel_row_tiles(ldt);
        const long long units = (long long)(n_atoms + 1) * n_ct * row_tiles;
        const long long per_xcd = (units + 7) / 8;
        if (8 * per_xcd > 0x7fffffffLL) return hipErrorInvalidValue;
        if (part && !d) return hipErrorInvalidValue;
        const bool full = row_tiles == 1 && min_nl2 > kQRows - 16;
        const dim3 grid((unsigned)(8 * per_xcd));
#define QREAL(F, N)                                                                                                    \
    hipLaunchKernelGGL((qpanel_real_kernel<F, N>), grid, dim3(kQThreads), sizeof(QRealSmem), s, T, ldt, tstride,         \
                       atom_type, atom_nl2, atom_row, P, Q, ldp, n_atoms, kp2, n_ct, row_tiles, per_xcd, d, part,      \
                       (long long)np)
        if (part) {
            if (full) QREAL(true, true);
            else QREAL(false, true);
        } else {
            if (full) QREAL(true, false);
            else QREAL(false, false);
        }
#undef QREAL
        return hipGetLastError();
    }
    if (part) return hipErrorInvalidValue;             // column sums only from the real-T kernel
    // row tiles: enough for the largest atom block (2 NL <= ldt)
    const int row_tiles = (int)((ldt + kTile - 1) / kTile);
    // units (atom, column tile), atom n_atoms zeroing the padding rows; 8 units per group of
    // 8 * row_tiles work-groups
    const long long units = (long long)(n_atoms + 1) * n_ct;
    const long long blocks = (units + 7) / 8 * 8 * row_tiles;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(qpanel_kernel, dim3((unsigned)blocks), dim3(kThreads), sizeof(QSmem), s, T, ldt, tstride,
                       atom_type, atom_nl2, atom_row, P, Q, ldp, n_atoms, kp2, n_ct, row_tiles);
    return hipGetLastError();
}

hipError_t launch_repack(const double2 *A, const double2 *B, long long lda, int n_g, const AtomDev *atoms, int n_atoms,
                         const long long *src_off, double2 *P, long long ldp, int kp2, int np, hipStream_t s)
{
    (void)atoms;
    (void)n_atoms;
    hipLaunchKernelGGL(repack_kernel, dim3(np), dim3(256), 0, s, A, B, lda, n_g, src_off, P, ldp, kp2);
    return hipGetLastError();
}

}  // namespace flapw
