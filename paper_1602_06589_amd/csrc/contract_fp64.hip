// FP64 matrix-core kernels of the contraction stage.
//
//  qpanel_kernel : Q_a = T_type(a) P_a for every atom (the paper's X_a, Z_a of sections 4.4-4.6,
//                  here for the whole 2NL x 2NL block T at once), P_a = [A_a; B_a].
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
// 256-byte segment; stages are double-buffered in LDS as planar [k][column] arrays of doubles,
// which is the layout the MFMA operands read (lane l takes row k = l/16, column l%16).
// Four waves each own a 32 x 32 quadrant (2 x 2 MFMA blocks); the accumulator of block (m, n)
// holds rows l/16 + 4r, column l%16 in register r of lane l.
#include "common.hpp"

namespace flapw {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kLW = kTile;                  // LDS row width (doubles)

__device__ __forceinline__ v4d mfma(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C += X^H Y over one LDS stage for a wave's 2x2 blocks; acc[0] = Re, acc[1] = Im.
__device__ __forceinline__ void stage_mma(const double (*xr)[kLW], const double (*xi)[kLW], const double (*yr)[kLW],
                                          const double (*yi)[kLW], int wm, int wn, int lane, v4d (*acc)[2][2])
{
#pragma unroll
    for (int ks = 0; ks < kKTile; ks += 4) {
        const int kr = ks + (lane >> 4), cc = lane & 15;
        double ar[2], ai[2], br[2], bi[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            ar[q] = xr[kr][wm + q * 16 + cc];
            ai[q] = xi[kr][wm + q * 16 + cc];
            br[q] = yr[kr][wn + q * 16 + cc];
            bi[q] = yi[kr][wn + q * 16 + cc];
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) {
                acc[0][mi][ni] = mfma(ar[mi], br[ni], acc[0][mi][ni]);
                acc[0][mi][ni] = mfma(ai[mi], bi[ni], acc[0][mi][ni]);
                acc[1][mi][ni] = mfma(ar[mi], bi[ni], acc[1][mi][ni]);
                acc[1][mi][ni] = mfma(-ai[mi], br[ni], acc[1][mi][ni]);
            }
    }
}

struct HsSmem {
    double v[2][6][kKTile][kLW];            // [buffer][Lre, Lim, Rre, Rim, Qre, Qim][k][col]
};

__global__ __launch_bounds__(kThreads, 1) void hs_fp64_kernel(const ProblemDev *__restrict__ probs,
                                                              const TileDev *__restrict__ tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    HsSmem &sm = *reinterpret_cast<HsSmem *>(smem_raw);

    const TileDev td = tiles[blockIdx.x];
    const ProblemDev pb = probs[td.prob];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const long long i0 = (long long)td.ti * kTile, j0 = (long long)td.tj * kTile;

    const int lc = tid >> 2, lk = (tid & 3) * 4;       // loader: column lc, rows lk..lk+3 of a stage
    const double2 *gL = pb.P + (i0 + lc) * pb.ldp + lk;
    const double2 *gR = pb.P + (j0 + lc) * pb.ldp + lk;
    const double2 *gQ = pb.Q + (j0 + lc) * pb.ldp + lk;
    const double *gd = pb.d + lk;

    v4d acc[4][2][2];                                  // S re, S im, H re, H im
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[a][m][n] = (v4d){0.0, 0.0, 0.0, 0.0};

    double2 rl[4], rr[4], rq[4];
    double rd[4];
    auto gload = [&](int kt) {
        const long long off = (long long)kt * kKTile;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            rl[r] = gL[off + r];
            rr[r] = gR[off + r];
            rq[r] = gQ[off + r];
            rd[r] = gd[off + r];
        }
    };
    auto sstore = [&](int b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sm.v[b][0][lk + r][lc] = rl[r].x;
            sm.v[b][1][lk + r][lc] = rl[r].y;
            sm.v[b][2][lk + r][lc] = rr[r].x * rd[r];
            sm.v[b][3][lk + r][lc] = rr[r].y * rd[r];
            sm.v[b][4][lk + r][lc] = rq[r].x;
            sm.v[b][5][lk + r][lc] = rq[r].y;
        }
    };

    const int nkt = pb.kp2 / kKTile;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        const int b = kt & 1;
        if (kt + 1 < nkt) gload(kt + 1);
        stage_mma(sm.v[b][0], sm.v[b][1], sm.v[b][2], sm.v[b][3], wm, wn, lane, &acc[0]);
        stage_mma(sm.v[b][0], sm.v[b][1], sm.v[b][4], sm.v[b][5], wm, wn, lane, &acc[2]);
        if (kt + 1 < nkt) sstore(b ^ 1);
        __syncthreads();
    }

    // epilogue: upper triangle (row <= col < n); diagonal imaginary part set to zero
#pragma unroll
    for (int mat = 0; mat < 2; ++mat) {
        double2 *out = mat == 0 ? pb.S : pb.H;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long long row = i0 + wm + mi * 16 + (lane >> 4) + 4 * r;
                    const long long col = j0 + wn + ni * 16 + (lane & 15);
                    if (row <= col && col < pb.n) {
                        const double re = acc[2 * mat][mi][ni][r];
                        const double im = row == col ? 0.0 : acc[2 * mat + 1][mi][ni][r];
                        out[col * pb.ldh + row] = make_double2(re, im);
                    }
                }
    }
}

struct QSmem {
    double v[2][4][kKTile][kLW];            // [buffer][Xre, Xim, Yre, Yim][k][col]
};

// grid: x = column tile, y = atom, z = row tile of the atom's 2NL rows
__global__ __launch_bounds__(kThreads, 1) void qpanel_kernel(const double2 *__restrict__ T, long long ldt,
                                                             long long tstride, const int *__restrict__ atom_type,
                                                             const int *__restrict__ atom_nl2,
                                                             const long long *__restrict__ atom_row,
                                                             const double2 *__restrict__ P, double2 *__restrict__ Q,
                                                             long long ldp)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    QSmem &sm = *reinterpret_cast<QSmem *>(smem_raw);

    const int a = blockIdx.y;
    const int m2 = atom_nl2[a];                         // 2 NL of this atom
    const int r0 = blockIdx.z * kTile;
    if (r0 >= m2) return;
    const long long prow = atom_row[a];
    const double2 *Ta = T + (long long)atom_type[a] * tstride;
    const long long c0 = (long long)blockIdx.x * kTile;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lc = tid >> 2, lk = (tid & 3) * 4;
    const bool xcol_ok = (r0 + lc) < m2;
    const double2 *gX = Ta + (long long)(xcol_ok ? r0 + lc : 0) * ldt + lk;
    const double2 *gY = P + (c0 + lc) * ldp + prow + lk;

    v4d acc[2][2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[q][m][n] = (v4d){0.0, 0.0, 0.0, 0.0};

    double2 rx[4], ry[4];
    auto gload = [&](int kt) {
        const int k0 = kt * kKTile + lk;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool ok = (k0 + r) < m2;
            rx[r] = (ok && xcol_ok) ? gX[kt * kKTile + r] : make_double2(0.0, 0.0);
            ry[r] = ok ? gY[kt * kKTile + r] : make_double2(0.0, 0.0);
        }
    };
    auto sstore = [&](int b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sm.v[b][0][lk + r][lc] = rx[r].x;
            sm.v[b][1][lk + r][lc] = rx[r].y;
            sm.v[b][2][lk + r][lc] = ry[r].x;
            sm.v[b][3][lk + r][lc] = ry[r].y;
        }
    };
    const int nkt = (m2 + kKTile - 1) / kKTile;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        const int b = kt & 1;
        if (kt + 1 < nkt) gload(kt + 1);
        stage_mma(sm.v[b][0], sm.v[b][1], sm.v[b][2], sm.v[b][3], wm, wn, lane, &acc[0]);
        if (kt + 1 < nkt) sstore(b ^ 1);
        __syncthreads();
    }
    // T is Hermitian, so X^H Y with X = T is T P.
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wm + mi * 16 + (lane >> 4) + 4 * r;
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

hipError_t launch_hs_fp64(const ProblemDev *probs, const TileDev *tiles, int n_tiles, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)hs_fp64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sizeof(HsSmem));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(hs_fp64_kernel, dim3(n_tiles), dim3(kThreads), sizeof(HsSmem), s, probs, tiles);
    return hipGetLastError();
}

hipError_t launch_qpanel(const double2 *T, long long ldt, long long tstride, const int *atom_type, const int *atom_nl2,
                         const long long *atom_row, int n_atoms, const double2 *P, double2 *Q, long long ldp, int np,
                         hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)qpanel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sizeof(QSmem));
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int rt = (2 * (FLAPW_LMAX_CAP + 1) * (FLAPW_LMAX_CAP + 1) + kTile - 1) / kTile;
    (void)rt;
    int max_rows = 0;
    (void)max_rows;
    // row tiles: enough for the largest atom block, passed by the caller through tstride's matrix size
    const int row_tiles = (int)((ldt + kTile - 1) / kTile);
    hipLaunchKernelGGL(qpanel_kernel, dim3(np / kTile, n_atoms, row_tiles), dim3(kThreads), sizeof(QSmem), s, T, ldt,
                       tstride, atom_type, atom_nl2, atom_row, P, Q, ldp);
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
