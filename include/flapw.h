/*
 * flapw.h -- C-ABI of the MI355X (gfx950) library that generates the muffin-tin parts of the
 * FLAPW Hamiltonian H and overlap S (Di Napoli, Peise, Hrywniak, Bientinesi, "High-performance
 * generation of the Hamiltonian and Overlap matrices in FLAPW methods").
 *
 * What is computed (the paper's notation):
 *   A_{L,a,t}, B_{L,a,t}   matching coefficients, appendix A.1, eqs. def_a_tensor / def_b_tensor
 *   T_a                    [[T^AA, T^AB], [T^BA, T^BB]], appendix A.2, eq. t_matrices
 *   S = sum_a A_a^H A_a + B_a^H U_a^H U_a B_a       section 2.3 eq. def_overlap, section 4 eqn:S
 *   H = sum_a [A_a;B_a]^H T_a [A_a;B_a]              section 2.3 eq. def_hamilton, section 4 eqn:H
 *
 * Conventions fixed by this library where the paper is silent:
 *   - atomic units (bohr, bohr^-1); complex Y_lm orthonormal with the Condon-Shortley phase;
 *     L = l*l + l + m;
 *   - A and B rows: atoms stacked in order, each with (lmax(type)+1)^2 rows ordered by L
 *     (section 4.2 "A_*" layout, section 4.7 ragged blocks);
 *   - T diagonal: E_l on AA, E_l ||udot_l||^2 on BB, 1/2 on AB and on BA (the Hermitian part of
 *     the printed +1 / +0, so that T^BA = (T^AB)^H as section 4.4 uses);
 *   - non-spherical integrals I^{(x,y)} are indexed [type][l'][l][L''], bra function first
 *     (eq. nonsph_integrals), L'' = l''^2 + l'' + m'';
 *   - K_t = 0 uses the z direction for Khat (only l = 0 survives there);
 *   - H and S are written on the upper triangle including the diagonal only (column-major
 *     'U'; the strictly lower part is left untouched); the diagonal's imaginary parts are
 *     set to exactly zero.  (The paper's BLAS calls write the lower triangle; both hold the
 *     same Hermitian matrix.)
 *
 * Memory and ownership: arrays marked [device] live in GPU memory of the current HIP device,
 * arrays marked [host] in host memory.  The caller allocates and owns every input and output
 * buffer; the library keeps no pointer to them after a call returns.  Work buffers belong to
 * the handle and are reused across calls; a handle must not be used by two threads at once.
 * Every computing call is asynchronous with respect to the host and ordered on `stream`
 * (a hipStream_t; NULL is the default stream).  All dense matrices are column-major
 * complex128 ({re, im} pairs) with an explicit leading dimension (section 4.1 storage format).
 *
 * Errors: arguments are validated before any launch; on FLAPW_ERR_ARG, FLAPW_ERR_WRONSKIAN or
 * FLAPW_ERR_NOT_HERMITIAN no output is touched.  FLAPW_ERR_DEVICE leaves outputs undefined.
 * flapw_last_error() returns a human-readable message for the last failure on a handle.
 * No C++ exception crosses this interface.
 */
#ifndef FLAPW_H
#define FLAPW_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } flapw_z;     /* complex128 */
typedef struct flapw_context *flapw_handle;
typedef void *flapw_stream;                    /* hipStream_t */

typedef enum {
    FLAPW_OK = 0,
    FLAPW_ERR_ARG = -1,            /* invalid argument (null pointer, size, leading dimension, ...) */
    FLAPW_ERR_WRONSKIAN = -2,      /* |W_{l,type}| too small: coefficients undefined */
    FLAPW_ERR_NOT_HERMITIAN = -3,  /* non-spherical integrals would make T non-Hermitian */
    FLAPW_ERR_NOMEM = -4,          /* device work buffer allocation failed */
    FLAPW_ERR_DEVICE = -5,         /* a HIP call failed */
    FLAPW_ERR_UNSUPPORTED = -6,    /* request outside what the library implements */
    FLAPW_ERR_NOT_POSDEF = -7,     /* flapw_eigensolve: S is not positive definite */
    FLAPW_ERR_NO_CONVERGENCE = -8  /* flapw_eigensolve: the tridiagonal eigensolver did not converge */
} flapw_status;

/* Arithmetic of the S and H contractions.  Coefficients, T and the per-atom panels T_a P_a
 * are always FP64.
 *   FP64        FP64 matrix cores throughout (complex128 accumulation).
 *   SPLIT_BF16  each FP64 operand column is split, with one power-of-two scale per column,
 *               into `slices` signed digits (first in [-255, 255], later in [-128, 128]) held
 *               exactly in bfloat16; digit pairs p + q < slices run on the BF16 matrix cores
 *               and accumulate exactly in FP32 over 64 contraction rows, then are recombined
 *               and summed over atoms in FP64.  3..6 digits.
 *   SPLIT_FP32  two-term FP32 slices (hi = fl32(x), lo = fl32(x - hi)) with three slice products
 *               on the FP32 matrix cores and FP32 accumulation.  Reserved and not implemented:
 *               FP32 accumulation over the 2K contraction rows cannot reach a 1e-10 relative
 *               error, and three FP32 products per FP64 one run below the FP64 matrix-core rate,
 *               so every call with it returns FLAPW_ERR_UNSUPPORTED.
 *   SPLIT_I8    the BF16 scheme with int8 digits (first in [-127, 127], later in [-64, 64]) and
 *               exact int32 accumulation over 4096 rows.  3..6 digits.
 *   SPLIT_I8_MOD  modular split: each operand column is scaled (by 2^B over its 2-norm, to 8
 *               significant bits) and rounded to integers; the exact integer products are
 *               computed modulo `slices` pairwise coprime odd moduli <= 255 in which -1 is a
 *               square (241, 233, 229, 221, 205, 197, 193, 181, 173, 157, 149, 137, 113, 109, in
 *               this order), each complex product as two real int8 matrix-core products with
 *               int32 accumulation, and rebuilt by the Chinese remainder theorem in FP64
 *               (B = min(50, (log2 M - 1)/2 - 0.001), M the product of the moduli).  8..14
 *               moduli.  Needs, per k-point in flight, 2 `slices` bytes per element of each of
 *               three 2K x N operands plus 64 `slices` KiB per 128 x 128 output tile of S and of
 *               H.
 * `slices` (the digit or modulus count) outside the ranges above returns FLAPW_ERR_UNSUPPORTED
 * (FLAPW_ERR_ARG beyond FLAPW_SLICES_CAP digits or FLAPW_MODULI_CAP moduli, or below 0); 0
 * selects the count flapw_tune chose for the same precision and problem shape, else the default
 * (6 digits; 11 moduli). */
typedef enum {
    FLAPW_PREC_FP64 = 0,
    FLAPW_PREC_SPLIT_BF16 = 1,
    FLAPW_PREC_SPLIT_FP32 = 2,
    FLAPW_PREC_SPLIT_I8 = 3,
    FLAPW_PREC_SPLIT_I8_MOD = 4
} flapw_prec;
#define FLAPW_MODULI_CAP 14        /* largest number of moduli of FLAPW_PREC_SPLIT_I8_MOD */

#define FLAPW_LMAX_CAP 12          /* largest supported l_max per type */
#define FLAPW_LPOT_CAP 12          /* largest supported l'' of the non-spherical potential */
#define FLAPW_SLICES_CAP 8         /* largest number of digits per operand in split precision */

/* Per atom type tau = 0..n_types-1 and l = 0..lmax[tau]; per-l arrays have row stride
 * `lstride` (>= max lmax + 1) and are indexed [tau * lstride + l].  [host] */
typedef struct {
    int n_types;
    int lstride;
    const int *lmax;          /* [n_types] l_max of the type, 0..FLAPW_LMAX_CAP */
    const double *rmt;        /* [n_types] muffin-tin radius R (bohr), > 0 */
    const double *u;          /* u_l(R) */
    const double *du;         /* u_l'(R)   (radial derivative) */
    const double *ud;         /* udot_l(R) (energy derivative) */
    const double *dud;        /* udot_l'(R) */
    const double *ud_norm2;   /* ||udot_l||^2 over the sphere (eq. def_overlap) */
    const double *e_l;        /* energy parameter E_l (eq. t_matrices) */
} flapw_radial;

/* Atoms.  [host] */
typedef struct {
    int n_atoms;
    const int *type;          /* [n_atoms] type index */
    const double *pos;        /* [n_atoms][3] Cartesian position x_a (bohr) */
    const double *rot;        /* [n_atoms][3][3] row-major orthogonal R_a; Y_lm is taken at R_a Khat */
    double omega;             /* unit-cell volume (bohr^3), > 0 */
} flapw_atoms;

/* Non-spherical radial integrals (eq. nonsph_integrals), each [n_types][lstride][lstride][(lpot+1)^2]
 * indexed [tau][l'][l][L''] (bra l' first).  Hermitian T requires I^{uu} and I^{udot udot}
 * symmetric in (l', l), I^{udot u}_{l',l,L''} = I^{u udot}_{l,l',L''}, and the reality rule
 * I_{(l'',-m)} = (-1)^m I_{(l'',m)}; flapw_build_T checks this.  [host] */
typedef struct {
    int lpot;                 /* l''_max, 0..FLAPW_LPOT_CAP */
    const double *i_uu;       /* I^{(u,u)} */
    const double *i_ud;       /* I^{(u,udot)} */
    const double *i_du;       /* I^{(udot,u)} */
    const double *i_dd;       /* I^{(udot,udot)} */
} flapw_potential;

/* Handle life cycle.  flapw_create binds the handle to the current HIP device. */
flapw_status flapw_create(flapw_handle *h);
flapw_status flapw_destroy(flapw_handle h);
const char *flapw_status_string(flapw_status s);
const char *flapw_last_error(flapw_handle h);
/* Device memory held by the handle's work buffers, in bytes. */
long long flapw_workspace_bytes(flapw_handle h);
/* Frees the handle's work buffers.  They grow to the largest call made so far (about 100 GB for
 * a 512-atom k-point in the modular split precision) and are allocated again by the next call
 * that needs them; nothing in them outlives a call.  Waits for the device first, as
 * flapw_destroy does; plans keep their own buffers.  Errors: FLAPW_ERR_ARG for a NULL handle. */
flapw_status flapw_release_workspace(flapw_handle h);
/* Workspace watermark: after every flapw_hs_generate, flapw_hs_contract, flapw_s_legendre or
 * flapw_interstitial call that leaves the handle's work buffers above `bytes`, the call waits for
 * its stream and frees them (as flapw_release_workspace), so that one handle's buffers do not
 * crowd out other handles or the caller's allocations between calls.  bytes < 0 (the default):
 * no limit, buffers are kept for the next call.  Errors: FLAPW_ERR_ARG for a NULL handle. */
flapw_status flapw_set_workspace_limit(flapw_handle h, long long bytes);

/* Matching coefficients A_* and B_* of one k-point (appendix A.1, eqs. def_a_tensor,
 * def_b_tensor; Wronskian W = udot u' - u udot'; stacked layout of section 4.2).
 *   k      [host]   k-point, Cartesian (bohr^-1)
 *   g      [device] n_g x 3 doubles, Cartesian G_t (row t = basis function t); K_t = k + G_t
 *   A, B   [device] K x n_g, column-major, leading dimension ld >= K = sum_a (lmax(type_a)+1)^2
 * Errors: FLAPW_ERR_ARG (n_g < 1, ld < K, bad type/l_max, omega <= 0, R_a not orthogonal to
 * 1e-10), FLAPW_ERR_WRONSKIAN (|W| <= 1e-12 max(|udot u'|, |u udot'|) for some used (type, l)). */
flapw_status flapw_coeffs(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                          const flapw_radial *rad, flapw_z *A, flapw_z *B, long ld, flapw_stream stream);

/* T matrices of all atom types (appendix A.2, eqs. gaunt, t_matrices); the Gaunt coefficients
 * are evaluated on the device.
 *   T [device] n_types matrices of ldt x ldt complex128, type tau at T + tau * ldt * ldt, each
 *             holding its 2NL x 2NL matrix (NL = (lmax+1)^2) in the top-left corner, column-major,
 *             rows = bra (L'), columns = ket (L), blocks [[AA, AB], [BA, BB]].  ldt >= 2 NL_max.
 *             Entries outside the 2NL x 2NL corner are set to zero.
 * Errors: FLAPW_ERR_ARG, FLAPW_ERR_NOT_HERMITIAN (integral symmetries violated by more than
 * 1e-12 of the largest |I|). */
flapw_status flapw_build_T(flapw_handle h, const flapw_radial *rad, const flapw_potential *pot, flapw_z *T,
                           long ldt, flapw_stream stream);

/* S and H from given coefficients and T (the contraction stage on its own):
 *   S = sum_a A_a^H A_a + B_a^H diag(||udot||^2) B_a,   H = sum_a P_a^H T_type(a) P_a,  P_a = [A_a; B_a].
 *   A, B [device] K x n_g (lda >= K), stacked as flapw_coeffs writes them
 *   T    [device] as flapw_build_T writes it (must be Hermitian; it is not re-checked)
 *   H, S [device] n_g x n_g, ldh >= n_g; upper triangle written
 * `at` supplies n_atoms and type (positions and rotations are not read); `rad` supplies
 * n_types, lmax and ud_norm2.  slices: digits (3..6) or moduli (8..14) of the split precisions
 * (0 = tuned or library default, see flapw_prec); ignored for FP64. */
flapw_status flapw_hs_contract(flapw_handle h, int n_g, const flapw_atoms *at, const flapw_radial *rad,
                               const flapw_z *A, const flapw_z *B, long lda, const flapw_z *T, long ldt,
                               flapw_z *H, flapw_z *S, long ldh, flapw_prec prec, int slices,
                               flapw_stream stream);

/* flapw_hs_contract for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same arguments, kernels and results (bit
 * for bit), but every work buffer (the P and Q panels, digits or residues, descriptors) is carved
 * out of one static device array of flapw_noalloc_scratch_bytes() bytes (64 MiB) per device,
 * which the device holds from the load of the library until the process ends.  The call makes
 * no hipMalloc / hipFree and allocates nothing else on the device; descriptors reach the array by
 * hipMemcpyAsync from the handle's host buffers.  Every call on a device shares that device's
 * array and leaves its contents behind (the kernels write every byte they read, so nothing needs
 * clearing); calls that overlap on one device -- from two streams or two threads, through any
 * handle -- race on it and must be serialised by the caller.  Errors: as flapw_hs_contract;
 * FLAPW_ERR_ARG (nothing launched) when the problem needs more than the array holds (about
 * 2 * roundup(2K, 256) * roundup(n_g, 64) * 16 bytes of panels plus, for the split precisions,
 * their digits or residues); FLAPW_ERR_DEVICE when the array's address could not be found at
 * flapw_create. */
flapw_status flapw_hs_contract_noalloc(flapw_handle h, int n_g, const flapw_atoms *at, const flapw_radial *rad,
                                       const flapw_z *A, const flapw_z *B, long lda, const flapw_z *T, long ldt,
                                       flapw_z *H, flapw_z *S, long ldh, flapw_prec prec, int slices,
                                       flapw_stream stream);
/* Size of that per-device array in bytes. */
long long flapw_noalloc_scratch_bytes(void);

/* The whole path for n_k k-points (one H and one S per k-point, section 2.3): coefficients,
 * T, per-atom panels and the S/H contractions, all k-points of a memory batch in one grouped
 * launch of the contraction kernel.
 *   k    [host] n_k x 3 doubles, Cartesian
 *   n_g  [host] n_k basis sizes (each >= 1)
 *   g    [host] n_k pointers to [device] n_g[i] x 3 doubles (Cartesian G)
 *   H, S [host] n_k pointers to [device] n_g[i] x n_g[i] outputs with leading dimensions
 *        ldh[i] >= n_g[i] ([host] array)
 * Errors as flapw_coeffs and flapw_build_T. */
flapw_status flapw_hs_generate(flapw_handle h, int n_k, const double *k, const int *n_g, const double *const *g,
                               const flapw_atoms *at, const flapw_radial *rad, const flapw_potential *pot,
                               flapw_z *const *H, flapw_z *const *S, const long *ldh, flapw_prec prec, int slices,
                               flapw_stream stream);

/* Method for S in flapw_hs_generate / flapw_plan_create (a handle setting, FLAPW_S_GEMM by
 * default).
 *   FLAPW_S_GEMM     : S = P^H D P on the matrix cores with H (eq. def_overlap; in the chosen
 *                      precision: FP64 or split digits).
 *   FLAPW_S_LEGENDRE : S through the addition theorem (section 3.1, eq. overlap_no_m with the
 *                      prefactor 4 pi / Omega): the sum over m becomes (2l+1)/(4 pi) P_l of the
 *                      angle between K_t and K_t', and the sum over atoms becomes, per atom type,
 *                      E^H E with E the plane-wave phases of that type's atoms.  Always FP64
 *                      (any prec); the contraction then computes H alone.  Same S up to rounding.
 * Plans use the method set when they are created. */
typedef enum { FLAPW_S_GEMM = 0, FLAPW_S_LEGENDRE = 1 } flapw_s_method;
flapw_status flapw_set_s_method(flapw_handle h, flapw_s_method method);

/* Structured T (section 3.1, Fig. Tmat_structure), a handle setting: with lnonsph >= 0 the
 * non-spherical terms (l'' >= 1) of T are kept only where both l' and l are <= lnonsph; the
 * spherical terms (diagonal in L: E_l, E_l ||udot||^2, 1/2, 1/2 and the l'' = 0 integrals) are
 * kept for every l.  lnonsph = -1 (default) keeps the dense T.  Affects flapw_build_T,
 * flapw_hs_generate, flapw_plan_create and flapw_tune (flapw_hs_contract takes T as given).
 * With FLAPW_S_LEGENDRE and lnonsph < l_max the contraction runs over the rows l <= lnonsph
 * only and the L-diagonal remainder of H is added by the addition-theorem kernel (the same H).
 * Errors: FLAPW_ERR_ARG unless -1 <= lnonsph <= FLAPW_LMAX_CAP. */
flapw_status flapw_set_lnonsph(flapw_handle h, int lnonsph);

/* S of one k-point through the addition theorem (FLAPW_S_LEGENDRE above), FP64.
 *   k[3] host, g device [n_g][3] Cartesian G (K_t = k + G_t), at/rad as flapw_coeffs (positions
 *   required, omega > 0).  S device, column-major, lds >= n_g; written on the upper triangle with
 *   the diagonal imaginary part exactly 0; the strictly lower part is untouched.
 * Errors: FLAPW_ERR_ARG, FLAPW_ERR_WRONSKIAN, FLAPW_ERR_DEVICE (as flapw_coeffs). */
flapw_status flapw_s_legendre(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                              const flapw_radial *rad, flapw_z *S, long lds, flapw_stream stream);

/* Interstitial parts of S and H of one k-point (section 2.3: eq. HS_Mat over the cell minus the
 * muffin-tin spheres, where eq. basis_function makes every basis function the plane wave
 * exp(i K_t.r) / sqrt(Omega)), ADDED to the upper triangles of S and H:
 *     S^I_{t',t} = delta_{t't} - sum_a exp(i G.x_a) (4 pi R_a^3 / Omega) j_1(|G| R_a) / (|G| R_a)
 *     H^I_{t',t} = (K_t'.K_t / 2 + v_int) S^I_{t',t},        G = K_t - K_t',
 * i.e. the plane-wave overlap over the cell minus the balls, the kinetic energy in its symmetric
 * form (1/2) int grad conj(phi_t') . grad phi_t over that region, and a constant interstitial
 * potential v_int (hartree).  With the muffin-tin parts of flapw_hs_generate these make the full
 * S (positive definite) and H of eq. matrix_kohnsham.  FP64; the atom sum runs per atom type as
 * a phase product on the FP64 matrix cores.
 *   k [host] 3 doubles; g [device] n_g x 3 Cartesian G; at (positions, omega) and rad (n_types,
 *   rmt; validated as for flapw_coeffs) as elsewhere; lattice [host] 3 x 3 row-major lattice
 *   vectors (bohr), used only to check that no two spheres overlap among the nearest periodic
 *   images (|det| must match omega to 1e-9 relative).
 *   H, S [device] n_g x n_g column-major, ldh >= n_g: the terms are added on the upper triangle
 *   (diagonal imaginary parts set to 0); the strictly lower part is untouched.
 * Errors: FLAPW_ERR_ARG (also for overlapping spheres or a lattice that does not match omega),
 * FLAPW_ERR_WRONSKIAN, FLAPW_ERR_NOMEM, FLAPW_ERR_DEVICE. */
flapw_status flapw_interstitial(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                                const flapw_radial *rad, const double *lattice, double v_int, flapw_z *H,
                                flapw_z *S, long ldh, flapw_stream stream);

/* Handle setting: with on != 0, flapw_hs_generate and flapw_plan_create add the interstitial
 * terms of flapw_interstitial (same lattice check, potential v_int) to every k-point's H and S
 * after the muffin-tin parts, so that the outputs are the full matrices of eq. matrix_kohnsham.
 * lattice [host] as for flapw_interstitial (copied; may be NULL when on == 0).  Default: off.
 * Errors: FLAPW_ERR_ARG (NULL lattice with on != 0, non-finite v_int). */
flapw_status flapw_set_interstitial(flapw_handle h, int on, const double *lattice, double v_int);

/* Generalized Hermitian eigenproblem H c = eps S c of one k-point (section 2.3, eq.
 * matrix_kohnsham; the eigensolve step of the self-consistency cycle), in place and in FP64:
 * S = U^H U (Cholesky), the reduced standard problem, its eigenvalues and (vectors != 0)
 * eigenvectors, back-transformed -- the LAPACK zhegvd scheme, by rocSOLVER on `stream`.
 *   H, S [device] n x n column-major, upper triangles read (as flapw_hs_generate writes them with
 *   the interstitial terms on); on return S holds U in its upper triangle, and with vectors the
 *   columns of H hold the eigenvectors (S-orthonormal: c^H S c = 1), else H is overwritten.
 *   w [device] n doubles: the eigenvalues in ascending order.
 * The call waits for the stream before it returns (it reads the solver's status).
 * Errors: FLAPW_ERR_ARG, FLAPW_ERR_NOT_POSDEF (S not positive definite, e.g. the muffin-tin S
 * alone, which has rank <= 2K), FLAPW_ERR_NO_CONVERGENCE, FLAPW_ERR_NOMEM, FLAPW_ERR_DEVICE. */
flapw_status flapw_eigensolve(flapw_handle h, int n, flapw_z *H, long ldh, flapw_z *S, long lds, double *w,
                              int vectors, flapw_stream stream);

/* Radial functions and non-spherical radial integrals from radial meshes (section 2.2,
 * eq. simp_Schr; appendix A.2, eq. nonsph_integrals), FP64, Hartree atomic units (the kinetic
 * prefactor of eq. simp_Schr is 1/2).  Per type tau the mesh is logarithmic,
 *     r_i = r0 (R / r0)^(i / (n_r - 1)),  i = 0..n_r-1,
 * with n_r - 1 a multiple of 4.  For l = 0..lmax[tau] the library solves eq. simp_Schr for P = r u
 * at E = e_l and its energy derivative (the same equation with right-hand side P), outward from
 * the regular small-r form P = r^(l+1)(1 - Z r/(l+1)), Z = -r0 v_sph(r0), by fourth-order
 * Runge-Kutta in ln r with step 2 ln(R/r0)/(n_r - 1) (the odd mesh points are the midpoints), and
 * evaluates integrals over [r0, R] by Simpson's rule in ln r on the even points.  u is normalised
 * (integral of u^2 r^2 = 1) and udot made orthogonal to u.
 * Outputs are the inputs of the other calls: u, du, ud, dud, ud_norm2 as in flapw_radial, host
 * arrays [n_types * lstride] (E_l is m->e_l), and the four tables of flapw_potential, host
 * arrays [n_types][lstride][lstride][(lpot+1)^2], with I^{(x,y)}_{l',l,L''} = integral of
 * x_{l'}(r) v_{L''}(r) y_l(r) r^2 dr.  Entries of l > lmax[tau] are 0.  With v_lm obeying the
 * reality rule the tables obey the symmetries flapw_build_T checks, and udot u' - u udot' = 2/R^2
 * up to the discretisation error.
 * The call uploads its inputs, runs two kernels on `stream` and returns after the results are
 * on the host (it synchronises the stream).
 * Errors: FLAPW_ERR_ARG (NULL pointer, n_types not in 1..32, lmax not in 0..FLAPW_LMAX_CAP,
 * lstride < max lmax + 1, lpot not in 0..FLAPW_LPOT_CAP, n_r - 1 not a multiple of 4 or n_r not
 * in 9..FLAPW_NR_CAP, r0 not in [1e-10, R), non-finite input, or a solution that overflows);
 * FLAPW_ERR_NOT_HERMITIAN (v_lm violates v_{(l'',-m)} = (-1)^m v_{(l'',m)} by more than 1e-12
 * of the type's largest |v_lm|); FLAPW_ERR_NOMEM, FLAPW_ERR_DEVICE.  On error no output is
 * written. */
#define FLAPW_NR_CAP 16385         /* largest number of radial mesh points */
typedef struct {
    int n_types;
    int lstride;
    const int *lmax;          /* [n_types] */
    const double *rmt;        /* [n_types] muffin-tin radius R (bohr) */
    const double *r0;         /* [n_types] first mesh point (bohr) */
    int n_r;                  /* mesh points per type */
    const double *e_l;        /* [n_types * lstride] energy parameters E_l (hartree) */
    const double *v_sph;      /* [n_types][n_r] spherical potential on the mesh (hartree) */
    int lpot;                 /* l''_max of v_lm */
    const double *v_lm;       /* [n_types][(lpot+1)^2][n_r] components v_{L''}(r), L'' = l''^2+l''+m'' */
} flapw_radial_mesh;
flapw_status flapw_radial_setup(flapw_handle h, const flapw_radial_mesh *m, double *u, double *du, double *ud,
                                double *dud, double *ud_norm2, double *i_uu, double *i_ud, double *i_du,
                                double *i_dd, flapw_stream stream);

/* Captured generation.  flapw_plan_create validates like flapw_hs_generate, allocates device
 * buffers owned by the plan (not shared with the handle), uploads every descriptor, and records
 * the whole generation (T, and per k-point coefficients, panels, digit slicing, then the grouped
 * contraction launches) into a HIP graph.  flapw_plan_launch replays it on `stream`; every replay
 * recomputes H and S from the same inputs (the device G lists are read at replay time, the host
 * descriptors -- k, atoms, radial data, potential -- are those given at creation).  The plan
 * keeps the output pointers; the caller keeps the outputs and the G lists alive while the plan
 * exists.  Replays of one plan must not overlap.  A plan is used from one thread at a time.
 * Errors: as flapw_hs_generate; FLAPW_ERR_DEVICE when capture or instantiation fails. */
typedef struct flapw_plan_s *flapw_plan;
flapw_status flapw_plan_create(flapw_handle h, int n_k, const double *k, const int *n_g, const double *const *g,
                               const flapw_atoms *at, const flapw_radial *rad, const flapw_potential *pot,
                               flapw_z *const *H, flapw_z *const *S, const long *ldh, flapw_prec prec, int slices,
                               flapw_plan *plan);
flapw_status flapw_plan_launch(flapw_plan plan, flapw_stream stream);
flapw_status flapw_plan_destroy(flapw_plan plan);

/* Autotuner.  Chooses, for one k-point (k, n_g G vectors, device list g), the digit or modulus
 * count of the split path and the tile band of the contraction (the number of tile rows one band
 * of the launch order walks; neighbouring work-groups of a band share their row panel in L2).
 *   count:  a seeded uniform random subset of n = min(n_g, 1024) basis functions is generated with
 *           FP64 and with 3, 4, 5, 6 digits (SPLIT_I8, SPLIT_BF16) or 10, 11, 12, 13 moduli
 *           (SPLIT_I8_MOD).  From the n x n principal submatrices of H and S the relative
 *           Frobenius error of each whole n_g x n_g matrix is estimated without bias (the sampled
 *           diagonal entries weighted by n_g / n, the sampled pairs by n_g (n_g - 1) / (n (n - 1)),
 *           in the squared norms of the error and of the FP64 result); the smallest count whose
 *           estimates for H and S are both <= 2 tol / 3 is chosen.  FP64: 0.
 *   band and stage depth:  a prefix of at most 8192 tiles of the contraction of the whole k-point
 *           is timed with HIP events for bands 1, 2, 4, 8, 16 and, for SPLIT_I8_MOD, each with
 *           64-row and with 32-row LDS stages of the contraction kernel; the fastest is chosen.
 * The choice is stored in the handle under (prec, padded contraction rows of the atom set as the
 * generation lays them out, S method, lnonsph) and used by later flapw_hs_generate /
 * flapw_plan_create calls with slices = 0 (band: every call) under the same handle settings and
 * atom set, and by flapw_hs_contract when it was tuned with the default settings (S_GEMM, dense T).
 * Outputs: *slices, *band; *stage_rows (64 or 32 for SPLIT_I8_MOD, else 0) when not NULL;
 * digit_err[4] (the estimated errors of the four candidate counts, NaN where not evaluated) and
 * band_ms[10] (prefix times for bands 1, 2, 4, 8, 16 with 64-row stages, then with 32-row stages;
 * NaN where not timed) when not NULL.
 * Runs synchronously on the null stream and allocates temporary device memory for two n_g x n_g
 * outputs (freed before returning).  Errors: as flapw_hs_generate; FLAPW_ERR_ARG for tol <= 0;
 * FLAPW_ERR_UNSUPPORTED when no candidate count meets tol (digit_err is still filled) or for
 * FLAPW_PREC_SPLIT_FP32. */
flapw_status flapw_tune(flapw_handle h, const double *k, int n_g, const double *g, const flapw_atoms *at,
                        const flapw_radial *rad, const flapw_potential *pot, flapw_prec prec, double tol, int *slices,
                        int *band, int *stage_rows, double *digit_err, double *band_ms);

/* Kernel timing for profiling (off by default).  While enabled, the library records a pair of
 * HIP events on the launch stream around every launch of its kernels.  flapw_profile_query
 * waits for the recorded events of one kernel family and returns the number of launches and
 * their summed duration in milliseconds since the last flapw_profile_enable(h, 1).
 * Families: "coeffs", "tmat", "qpanel", "repack", "hs_fp64", "slice", "hs_split", "hs_mod",
 * "mod_crt", "leg_prep", "s_legendre", "interstitial", "eigensolve", "radial", "graph"
 * (a whole flapw_plan_launch; kernels inside a graph are not timed one by one).
 * Errors: FLAPW_ERR_ARG for an unknown family or NULL output pointer. */
flapw_status flapw_profile_enable(flapw_handle h, int on);
flapw_status flapw_profile_query(flapw_handle h, const char *family, int *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* FLAPW_H */
