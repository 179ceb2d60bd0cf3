// Interstitial parts of S and H (section 2.3: eq. HS_Mat integrated over the cell minus the
// muffin-tin spheres, where eq. basis_function makes every basis function the plane wave
// exp(i K_t.r) / sqrt(Omega)).  With G = K_t - K_t':
//     S^I_{t',t} = delta_{t't} - sum_a exp(i G.x_a) (4 pi R_a^3 / Omega) j_1(|G| R_a) / (|G| R_a)
//     H^I_{t',t} = (K_t'.K_t / 2 + v_int) S^I_{t',t}
// (the integral of a plane wave over a ball, subtracted from the cell integral, which vanishes
// unless G = 0; the kinetic energy in its symmetric form; a constant interstitial potential).
//
// exp(i G.x_a) = conj(exp(i K_t'.x_a)) exp(i K_t.x_a) and the ball factor depends on the atom
// only through its radius, so per atom type the atom sum is the phase product E_type^H E_type
// of the addition-theorem path (legendre.hip prepares E) times a per-entry function of |G|:
//     S^I = 1 - sum_types f_type(|G|) o (E_type^H E_type),   f = (4 pi R^3 / Omega) j_1(x)/x, x = |G| R.
// interstitial_kernel: one work-group per upper-triangle 64 x 64 tile, 4 waves of 32 x 32; the
// phase rows of all types stream through LDS in 16-row stages with FP64 MFMAs, and at the last
// stage of a type its f is applied.  The result is added to S and H (read, add, write), upper
// triangle only, diagonal imaginary parts set to zero.  Algorithmic work: 8 N_A flops of phase
// product per entry plus one sincos per (entry, type); bytes: S and H read and written once.
#include "common.hpp"

namespace flapw {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
#if defined(__HIP_DEVICE_COMPILE__)
typedef const double2 __attribute__((address_space(1))) gdouble2;
#else
typedef const double2 gdouble2;
#endif

constexpr int kThreads = 256;
constexpr int kSlot = kKTile + 1;

__device__ __forceinline__ v4d mfma(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// j_1(x) / x: its Taylor series below 0.3 (the closed form loses bits to cancellation there),
// (sin x - x cos x) / x^3 above.
__device__ inline double j1_over_x(double x)
{
    if (x < 0.3) {
        const double y = x * x;
        return 1.0 / 3.0 +
               y * (-1.0 / 30.0 + y * (1.0 / 840.0 + y * (-1.0 / 45360.0 + y * (1.0 / 3991680.0 - y / 518918400.0))));
    }
    double s, c;
    sincos(x, &s, &c);
    return (s - x * c) / (x * x * x);
}

struct ISmem {
    double2 e[2][2][kTile][kSlot];      // [buffer][left, right][column][k] phases
    double4 kv[2][kTile];               // [left, right][column] K_t (zero past n)
};

__global__ __launch_bounds__(kThreads, 1) void interstitial_kernel(const double *__restrict__ g, double kx, double ky,
                                                                    double kz, const double2 *__restrict__ E,
                                                                    long long ldE, const LegTypeRange *__restrict__ tr,
                                                                    const TypeDev *__restrict__ types, int n_types,
                                                                    const int2 *__restrict__ tiles, int n, double omega,
                                                                    double v_int, double2 *__restrict__ S, long long lds,
                                                                    double2 *__restrict__ H, long long ldh)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ISmem &sm = *reinterpret_cast<ISmem *>(smem_raw);
    const int2 td = tiles[blockIdx.x];
    const long long i0 = (long long)td.x * kTile, j0 = (long long)td.y * kTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int c = lane & 15, rq = lane >> 4;

    if (tid < 2 * kTile) {
        const int side = tid / kTile, q = tid % kTile;
        const long long t = (side ? j0 : i0) + q;
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
        if (t < n) v = make_double4(kx + g[3 * t], ky + g[3 * t + 1], kz + g[3 * t + 2], 0.0);
        sm.kv[side][q] = v;
    }
    auto next_type = [&](int ty) {
        int q = ty + 1;
        while (q < n_types && tr[q].rows == 0) ++q;
        return q;
    };
    int ty = next_type(-1);

    const int lc = tid >> 2, lk = (tid & 3) * 4;          // loader: column lc, rows lk..lk+3 of a stage
    gdouble2 *gX = (gdouble2 *)E + (i0 + lc) * ldE + lk;
    gdouble2 *gY = (gdouble2 *)E + (j0 + lc) * ldE + lk;
    double2 x0, x1, x2, x3, y0, y1, y2, y3;
#define IN_LOAD(st)                                                                 \
    do {                                                                            \
        const long long o_ = (long long)(st) * kKTile;                              \
        x0 = gX[o_]; x1 = gX[o_ + 1]; x2 = gX[o_ + 2]; x3 = gX[o_ + 3];             \
        y0 = gY[o_]; y1 = gY[o_ + 1]; y2 = gY[o_ + 2]; y3 = gY[o_ + 3];             \
    } while (0)
#define IN_STORE(b)                                                                 \
    do {                                                                            \
        double2 *sx_ = &sm.e[b][0][lc][lk], *sy_ = &sm.e[b][1][lc][lk];             \
        sx_[0] = x0; sx_[1] = x1; sx_[2] = x2; sx_[3] = x3;                         \
        sy_[0] = y0; sy_[1] = y1; sy_[2] = y2; sy_[3] = y3;                         \
    } while (0)
    const int first = ty < n_types ? tr[ty].row0 / kKTile : 0;
    int last = first;                                    // one past the last stage
    for (int q = 0; q < n_types; ++q)
        if (tr[q].rows) last = max(last, (tr[q].row0 + tr[q].rows) / kKTile);
    if (first < last) {
        IN_LOAD(first);
        IN_STORE(0);
    }
    __syncthreads();

    // |G| and K'.K / 2 of the 16 entries of this lane: [mi][ni][r]
    double gn[2][2][4], kin[2][2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const double4 kc = sm.kv[1][wn + ni * 16 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double4 kr = sm.kv[0][wm + mi * 16 + rq + 4 * r];
                const double gx = kc.x - kr.x, gy = kc.y - kr.y, gz = kc.z - kr.z;
                gn[mi][ni][r] = sqrt(gx * gx + gy * gy + gz * gz);
                kin[mi][ni][r] = 0.5 * (kr.x * kc.x + kr.y * kc.y + kr.z * kc.z);
            }
        }

    double sre[2][2][4], sim[2][2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) sre[mi][ni][r] = sim[mi][ni][r] = 0.0;
    v4d acc[2][2][2];                                    // phase product of the current type: [re, im][mi][ni]
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int k = 0; k < 2; ++k) acc[q][m][k] = (v4d){0.0, 0.0, 0.0, 0.0};

    int type_end = ty < n_types ? (tr[ty].row0 + tr[ty].rows) / kKTile : 0;
    for (int st = first, b = 0; st < last; ++st, b ^= 1) {
        if (st + 1 < last) IN_LOAD(st + 1);
#pragma unroll
        for (int ks = 0; ks < kKTile; ks += 4) {
            const int k = ks + rq;
            double2 xv[2], yv[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                xv[q] = sm.e[b][0][wm + q * 16 + c][k];
                yv[q] = sm.e[b][1][wn + q * 16 + c][k];
            }
            // conj(x) y: Re = xr yr + xi yi, Im = xr yi - xi yr
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    acc[0][mi][ni] = mfma(xv[mi].x, yv[ni].x, acc[0][mi][ni]);
                    acc[1][mi][ni] = mfma(xv[mi].x, yv[ni].y, acc[1][mi][ni]);
                }
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    acc[0][mi][ni] = mfma(xv[mi].y, yv[ni].y, acc[0][mi][ni]);
                    acc[1][mi][ni] = mfma(-xv[mi].y, yv[ni].x, acc[1][mi][ni]);
                }
        }
        if (st + 1 == type_end) {
            const double R = types[ty].rmt;
            const double ball = 4.0 * kPi * R * R * R / omega;
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double f = ball * j1_over_x(gn[mi][ni][r] * R);
                        sre[mi][ni][r] += f * acc[0][mi][ni][r];
                        sim[mi][ni][r] += f * acc[1][mi][ni][r];
                        acc[0][mi][ni][r] = 0.0;
                        acc[1][mi][ni][r] = 0.0;
                    }
            ty = next_type(ty);
            if (ty < n_types) type_end = (tr[ty].row0 + tr[ty].rows) / kKTile;
        }
        if (st + 1 < last) IN_STORE(b ^ 1);
        __syncthreads();
    }
#undef IN_LOAD
#undef IN_STORE

    // epilogue: S += delta - sum, H += (K'.K / 2 + v_int) (delta - sum); upper triangle (row <= col < n)
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = i0 + wm + mi * 16 + rq + 4 * r;
                const long long col = j0 + wn + ni * 16 + c;
                if (row <= col && col < n) {
                    const double tre = (row == col ? 1.0 : 0.0) - sre[mi][ni][r];
                    const double tim = row == col ? 0.0 : -sim[mi][ni][r];
                    const double hf = kin[mi][ni][r] + v_int;
                    double2 *sp = S + col * lds + row;
                    double2 *hp = H + col * ldh + row;
                    const double2 sv = *sp, hv = *hp;
                    *sp = make_double2(sv.x + tre, row == col ? 0.0 : sv.y + tim);
                    *hp = make_double2(hv.x + hf * tre, row == col ? 0.0 : hv.y + hf * tim);
                }
            }
}

}  // namespace

hipError_t init_interstitial_kernel()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    done = hipFuncSetAttribute((const void *)interstitial_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               sizeof(ISmem));
    return done;
}

hipError_t launch_interstitial(const double *g, const double kvec[3], const double2 *E, long long ldE,
                               const LegTypeRange *ranges, const TypeDev *types, int n_types, const int *tiles,
                               int n_tiles, int n, double omega, double v_int, double2 *S, long long lds, double2 *H,
                               long long ldh, hipStream_t s)
{
    hipError_t e = init_interstitial_kernel();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(interstitial_kernel, dim3(n_tiles), dim3(kThreads), sizeof(ISmem), s, g, kvec[0], kvec[1],
                       kvec[2], E, ldE, ranges, types, n_types, (const int2 *)tiles, n, omega, v_int, S, lds, H, ldh);
    return hipGetLastError();
}

}  // namespace flapw
