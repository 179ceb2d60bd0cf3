// Overlap matrix S through the addition theorem (section 3.1, eqs. sum_single_overlap and
// overlap_no_m, with the prefactor 4 pi / Omega that the identity above them implies).
//
// Summing the m of A* A over a shell gives (2l+1)/(4 pi) P_l(Khat_t . Khat_t'), so
//     S_{t',t} = (4 pi / Omega) sum_a exp(i (K_t - K_t').x_a)
//                 sum_l (2l+1)/W_l^2 [fA_l(t') fA_l(t) + ||udot_l||^2 fB_l(t') fB_l(t)] P_l(cos g)
// with fA = udot K j_l' - udot' j_l and fB = u' j_l - u K j_l' at K R_MT of the atom's type.
// The radial part depends on the atom only through its type, so
//     S_{t',t} = (4 pi / Omega) sum_types g_type(t', t) Phi_type(t', t),
//     Phi_type = E_type^H E_type,   E_type[a][t] = exp(i K_t.x_a) over the atoms of the type,
// which is an FP64 matrix-core contraction over the atoms of one type (64 at 512 atoms / 8 types)
// instead of over all 2 sum_a N_L rows, and g_type is a short Legendre sum per matrix entry.
//
//  legendre_prep_kernel : per column t: Khat_t, and per type and l the radial factors
//                         alpha = fA sqrt(2l+1)/W, beta = fB sqrt(2l+1)/W, beta_n = ||udot||^2 beta;
//                         and the phases E (atoms grouped by type, each group padded to 16 rows).
//  s_legendre_kernel    : upper-triangle 64 x 64 tiles of S.  With WITH_H it also adds to H the
//                         terms of the T matrices that are diagonal in L for l > lnonsph (the part
//                         of a structured T outside its dense block, section 3.1 Fig.
//                         Tmat_structure):  H_{t',t} += (4 pi / Omega) sum_types Phi sum_{l > lnonsph}
//                         P_l (2l+1)/W^2 [aa fA' fA + ab fA' fB + ba fB' fA + bb fB' fB], with
//                         aa = E_l + I^uu_{l,l,00} Y_00, bb = E_l ||udot||^2 + I^dd_{l,l,00} Y_00,
//                         ab = 1/2 + I^{u udot}_{l,l,00} Y_00, ba = 1/2 + I^{udot u}_{l,l,00} Y_00.
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

// Legendre recurrence coefficients (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1}, l = 0..kLStride-1
__constant__ double kRecA[kLStride] = {1.0, 3.0 / 2, 5.0 / 3, 7.0 / 4, 9.0 / 5, 11.0 / 6, 13.0 / 7,
                                       15.0 / 8, 17.0 / 9, 19.0 / 10, 21.0 / 11, 23.0 / 12, 25.0 / 13};
__constant__ double kRecB[kLStride] = {0.0, 1.0 / 2, 2.0 / 3, 3.0 / 4, 4.0 / 5, 5.0 / 6, 6.0 / 7,
                                       7.0 / 8, 8.0 / 9, 9.0 / 10, 10.0 / 11, 11.0 / 12, 12.0 / 13};

// Spherical Bessel functions j_0..j_n at x; same method as the coefficient kernel.
__device__ void bessel_all(int n, double x, double *j)
{
    if (x == 0.0) {
        j[0] = 1.0;
        for (int l = 1; l <= n; ++l) j[l] = 0.0;
        return;
    }
    if (x < 1e-3) {
        double xl = 1.0, df = 1.0;
        for (int l = 0; l <= n; ++l) {
            const double x2 = x * x;
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
    double fp1 = 0.0, f = 1.0;
    for (int l = top; l > n; --l) {
        const double fm = (2.0 * l + 1.0) / x * f - fp1;
        fp1 = f;
        f = fm;
        if (fabs(f) > 1e150) { f *= 1e-150; fp1 *= 1e-150; }
    }
    j[n] = f;
    double cur = f, nxt = fp1;
    for (int l = n; l >= 1; --l) {
        const double prv = (2.0 * l + 1.0) / x * cur - nxt;
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

// One thread per column t (np columns; t >= n_g gets zeros).
//   khat[t]           : unit vector of K_t (z axis for K_t = 0, where only l = 0 survives)
//   ab[(type kLStride + l) np + t] = {alpha, beta}
//   E[t ldE + row]    : exp(i K_t.x_a) at row = type offset + rank of the atom in its type
__global__ __launch_bounds__(kThreads) void legendre_prep_kernel(double kx, double ky, double kz, int n_g, int np,
                                                                  const double *__restrict__ g,
                                                                  const TypeDev *__restrict__ types, int n_types,
                                                                  const double *__restrict__ apos,
                                                                  const int *__restrict__ arow, int n_atoms,
                                                                  double4 *__restrict__ khat, double2 *__restrict__ ab,
                                                                  double2 *__restrict__ E, long long ldE)
{
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= np) return;
    double x = 0.0, y = 0.0, z = 0.0;
    if (t < n_g) {
        x = kx + g[3 * (long long)t];
        y = ky + g[3 * (long long)t + 1];
        z = kz + g[3 * (long long)t + 2];
    }
    const double kn = sqrt(x * x + y * y + z * z);
    khat[t] = kn > 0.0 ? make_double4(x / kn, y / kn, z / kn, 0.0) : make_double4(0.0, 0.0, 1.0, 0.0);
    for (int ty = 0; ty < n_types; ++ty) {
        const TypeDev &tp = types[ty];
        double j[kLStride + 1];
        bessel_all(tp.lmax + 1, kn * tp.rmt, j);
        for (int l = 0; l < kLStride; ++l) {
            double2 v = make_double2(0.0, 0.0);
            if (t < n_g && l <= tp.lmax) {
                const RadialDev &r = tp.rad[l];
                const double jl = j[l];
                const double djl = (l == 0) ? -j[1] : (l * j[l - 1] - (l + 1.0) * j[l + 1]) / (2.0 * l + 1.0);
                const double w = sqrt(2.0 * l + 1.0) * r.inv_w;
                const double fa = (r.ud * kn * djl - r.dud * jl) * w;
                const double fb = (r.du * jl - r.u * kn * djl) * w;
                v = make_double2(fa, fb);
            }
            ab[((long long)ty * kLStride + l) * np + t] = v;
        }
    }
    double2 *col = E + (long long)t * ldE;
    for (long long r = 0; r < ldE; ++r) col[r] = make_double2(0.0, 0.0);      // padding rows
    for (int a = 0; a < n_atoms; ++a) {
        double s = 0.0, c = 0.0;
        if (t < n_g) sincos(x * apos[3 * a] + y * apos[3 * a + 1] + z * apos[3 * a + 2], &s, &c);
        col[arow[a]] = t < n_g ? make_double2(c, s) : make_double2(0.0, 0.0);
    }
}

__device__ __forceinline__ v4d mfma(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct SLegSmem {
    double2 e[2][2][kTile][kSlot];                // [buffer][left, right][column][k] phases
    double2 ab[2][2][kLStride][kTile];            // [type parity][left, right][l][column] {alpha, beta}
    double4 khat[2][kTile];                       // [left, right][column]
};

// grid: one work-group per upper-triangle tile; 4 waves, each a 32 x 32 quadrant (2 x 2 blocks
// of 16 x 16; the accumulator of block (m, n) holds rows l/16 + 4r, column l%16 in register r).
// The phase rows of all types form one stream of 16-row stages (types are contiguous in E); at
// the last stage of a type the Legendre sum of that type is applied to its phase product.  The
// radial factors of the next type are copied global -> LDS (global_load_lds) while the current
// type streams, into the other of two buffers.
template <bool WITH_H>
__global__ __launch_bounds__(kThreads, 1) void s_legendre_kernel(const double4 *__restrict__ khat,
                                                                 const double2 *__restrict__ ab,
                                                                 const double2 *__restrict__ E, long long ldE,
                                                                 const LegTypeRange *__restrict__ tr, int n_types,
                                                                 const int2 *__restrict__ tiles, int np, int n,
                                                                 double scale, double2 *__restrict__ S, long long lds,
                                                                 const double *__restrict__ un2,
                                                                 const double4 *__restrict__ hsph, int lh0,
                                                                 double2 *__restrict__ H, long long ldh)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SLegSmem &sm = *reinterpret_cast<SLegSmem *>(smem_raw);
    const int2 td = tiles[blockIdx.x];
    const long long i0 = (long long)td.x * kTile, j0 = (long long)td.y * kTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int c = lane & 15, rq = lane >> 4;

    // radial factors of type ty into buffer par: one 1 KB segment (64 columns) per (side, l)
    auto copy_ab = [&](int ty, int par, int lmax) {
        for (int sg = wave; sg < 2 * (lmax + 1); sg += 4) {
            const int side = sg & 1, l = sg >> 1;
            const double2 *src = ab + ((long long)ty * kLStride + l) * np + (side ? j0 : i0) + lane;
            __builtin_amdgcn_global_load_lds((const int __attribute__((address_space(1))) *)src,
                                             (int __attribute__((address_space(3))) *)&sm.ab[par][side][l][0], 16, 0,
                                             0);
        }
    };
    // next type with atoms after ty (n_types if none)
    auto next_type = [&](int ty) {
        int q = ty + 1;
        while (q < n_types && tr[q].rows == 0) ++q;
        return q;
    };

    int ty = next_type(-1);
    if (tid < 2 * kTile) {
        const int side = tid / kTile, q = tid % kTile;
        sm.khat[side][q] = khat[(side ? j0 : i0) + q];
    }
    copy_ab(ty, 0, tr[ty].lmax);

    const int lc = tid >> 2, lk = (tid & 3) * 4;          // loader: column lc, rows lk..lk+3 of a stage
    gdouble2 *gX = (gdouble2 *)E + (i0 + lc) * ldE + lk;
    gdouble2 *gY = (gdouble2 *)E + (j0 + lc) * ldE + lk;
    double2 x0, x1, x2, x3, y0, y1, y2, y3;
#define SL_LOAD(st)                                                                 \
    do {                                                                            \
        const long long o_ = (long long)(st) * kKTile;                              \
        x0 = gX[o_]; x1 = gX[o_ + 1]; x2 = gX[o_ + 2]; x3 = gX[o_ + 3];             \
        y0 = gY[o_]; y1 = gY[o_ + 1]; y2 = gY[o_ + 2]; y3 = gY[o_ + 3];             \
    } while (0)
#define SL_STORE(b)                                                                 \
    do {                                                                            \
        double2 *sx_ = &sm.e[b][0][lc][lk], *sy_ = &sm.e[b][1][lc][lk];             \
        sx_[0] = x0; sx_[1] = x1; sx_[2] = x2; sx_[3] = x3;                         \
        sy_[0] = y0; sy_[1] = y1; sy_[2] = y2; sy_[3] = y3;                         \
    } while (0)
    const int first = tr[ty].row0 / kKTile;
    int last = 0;                                        // one past the last stage
    for (int q = 0; q < n_types; ++q) last = max(last, (tr[q].row0 + tr[q].rows) / kKTile);
    SL_LOAD(first);
    SL_STORE(0);
    __syncthreads();

    // cosines of the 16 entries of this lane: [mi][ni][r]
    double cg[2][2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const double4 kc = sm.khat[1][wn + ni * 16 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double4 kr = sm.khat[0][wm + mi * 16 + rq + 4 * r];
                cg[mi][ni][r] = fmin(1.0, fmax(-1.0, kr.x * kc.x + kr.y * kc.y + kr.z * kc.z));
            }
        }

    double sre[2][2][4], sim[2][2][4], hre[2][2][4], him[2][2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sre[mi][ni][r] = 0.0;
                sim[mi][ni][r] = 0.0;
                hre[mi][ni][r] = 0.0;
                him[mi][ni][r] = 0.0;
            }
    v4d acc[2][2][2];                                    // phase product of the current type: [re, im][mi][ni]
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int k = 0; k < 2; ++k) acc[q][m][k] = (v4d){0.0, 0.0, 0.0, 0.0};

    int par = 0;                                         // ab buffer of the current type
    int type_end = (tr[ty].row0 + tr[ty].rows) / kKTile;
    int nty = next_type(ty);
    if (nty < n_types) copy_ab(nty, 1, tr[nty].lmax);
    for (int st = first, b = 0; st < last; ++st, b ^= 1) {
        if (st + 1 < last) SL_LOAD(st + 1);
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
            // the Legendre sum of this type, recurrence (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1}
            const int lmax = tr[ty].lmax;
            const double *nn = un2 + ty * kLStride;
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    double pm[4], pc[4], gsum[4], hsum[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) { pm[r] = 0.0; pc[r] = 1.0; gsum[r] = 0.0; hsum[r] = 0.0; }
                    for (int l = 0; l <= lmax; ++l) {
                        const double2 bc = sm.ab[par][1][l][wn + ni * 16 + c];
                        const double nb = nn[l] * bc.y;                   // ||udot||^2 fB of the ket
                        const double ra = kRecA[l], rb = kRecB[l];
                        const bool hl = WITH_H && l >= lh0;
                        double2 hq = make_double2(0.0, 0.0);
                        if (hl) {
                            const double4 hc = hsph[ty * kLStride + l];
                            hq = make_double2(hc.x * bc.x + hc.y * bc.y, hc.z * bc.x + hc.w * bc.y);
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const double2 br = sm.ab[par][0][l][wm + mi * 16 + rq + 4 * r];
                            gsum[r] += (br.x * bc.x + br.y * nb) * pc[r];    // fA fA + ||udot||^2 fB fB
                            if (hl) hsum[r] += (br.x * hq.x + br.y * hq.y) * pc[r];
                            const double pn = ra * cg[mi][ni][r] * pc[r] - rb * pm[r];
                            pm[r] = pc[r];
                            pc[r] = pn;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        sre[mi][ni][r] += gsum[r] * acc[0][mi][ni][r];
                        sim[mi][ni][r] += gsum[r] * acc[1][mi][ni][r];
                        if (WITH_H) {
                            hre[mi][ni][r] += hsum[r] * acc[0][mi][ni][r];
                            him[mi][ni][r] += hsum[r] * acc[1][mi][ni][r];
                        }
                        acc[0][mi][ni][r] = 0.0;
                        acc[1][mi][ni][r] = 0.0;
                    }
                }
            ty = nty;
            if (ty < n_types) {
                type_end = (tr[ty].row0 + tr[ty].rows) / kKTile;
                par ^= 1;
                nty = next_type(ty);
            }
        }
        if (st + 1 < last) SL_STORE(b ^ 1);
        __syncthreads();                                 // also completes the radial-factor copies
        // the buffer the finished type used is free now: start the copy of the type after next
        if (ty < n_types && nty < n_types && st + 1 == type_end - tr[ty].rows / kKTile)
            copy_ab(nty, par ^ 1, tr[nty].lmax);
    }
#undef SL_LOAD
#undef SL_STORE

    // epilogue: upper triangle (row <= col < n); diagonal imaginary part set to zero
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = i0 + wm + mi * 16 + rq + 4 * r;
                const long long col = j0 + wn + ni * 16 + c;
                if (row <= col && col < n) {
                    S[col * lds + row] = make_double2(scale * sre[mi][ni][r], row == col ? 0.0 : scale * sim[mi][ni][r]);
                    if (WITH_H) {
                        double2 *hp = H + col * ldh + row;
                        const double2 hv = *hp;
                        *hp = make_double2(hv.x + scale * hre[mi][ni][r], row == col ? 0.0 : hv.y + scale * him[mi][ni][r]);
                    }
                }
            }
}

}  // namespace

hipError_t init_legendre_kernels()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    hipError_t e = hipFuncSetAttribute((const void *)s_legendre_kernel<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(SLegSmem));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)s_legendre_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                sizeof(SLegSmem));
    done = e;
    return done;
}

hipError_t launch_legendre_prep(const double kvec[3], int n_g, int np, const double *g, const TypeDev *types,
                                int n_types, const double *apos, const int *arow, int n_atoms, double *khat,
                                double *ab, double2 *E, long long ldE, hipStream_t s)
{
    hipLaunchKernelGGL(legendre_prep_kernel, dim3((np + kThreads - 1) / kThreads), dim3(kThreads), 0, s, kvec[0],
                       kvec[1], kvec[2], n_g, np, g, types, n_types, apos, arow, n_atoms, (double4 *)khat,
                       (double2 *)ab, E, ldE);
    return hipGetLastError();
}

hipError_t launch_s_legendre(const double *khat, const double *ab, const double2 *E, long long ldE,
                             const LegTypeRange *ranges, int n_types, const int *tiles, int n_tiles, int np, int n,
                             double scale, double2 *S, long long lds, const double *ud_norm2, const double *hsph,
                             int lh0, double2 *H, long long ldh, hipStream_t s)
{
    hipError_t e = init_legendre_kernels();
    if (e != hipSuccess) return e;
    if (H)
        hipLaunchKernelGGL(s_legendre_kernel<true>, dim3(n_tiles), dim3(kThreads), sizeof(SLegSmem), s,
                           (const double4 *)khat, (const double2 *)ab, E, ldE, ranges, n_types, (const int2 *)tiles, np,
                           n, scale, S, lds, ud_norm2, (const double4 *)hsph, lh0, H, ldh);
    else
        hipLaunchKernelGGL(s_legendre_kernel<false>, dim3(n_tiles), dim3(kThreads), sizeof(SLegSmem), s,
                           (const double4 *)khat, (const double2 *)ab, E, ldE, ranges, n_types, (const int2 *)tiles, np,
                           n, scale, S, lds, ud_norm2, (const double4 *)nullptr, 0, (double2 *)nullptr, 0LL);
    return hipGetLastError();
}

}  // namespace flapw
