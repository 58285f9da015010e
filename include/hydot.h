/*
 * hydot.h - C ABI of the MI355X hyperspectral DOT Born hot path.
 *
 * Method: Saibaba, Kilmer, Miller, Fantini, "Fast algorithms for hyperspectral
 * diffuse optical tomography".  The library computes
 *   - the fields phi = A(lambda)^-1 b for every source and detector right-hand
 *     side at every wavelength (Sec. 3, eq. multipleshifted), by Algorithm 1
 *     "Augmented GMRES for parametric systems" with the deflation space recycled
 *     across wavelengths (Sec. 3.1);
 *   - the Born operator J_lambda[s,d,k] = -h^3 phi_s(k) phi_d(k) those fields
 *     define (Sec. 2.1 integral equation with the adjoint field; rows of H in
 *     eq. measurement), applied matrix-free as J v and J^H w;
 *   - the parametric level-set shape (Sec. 5, eq. pals) and the data misfit
 *     (Sec. 5, eq. minimization) with their gradients.
 *
 * Discretisation (cell-centred finite volume on a box, voxel index
 * n = i + nx*(j + ny*k), voxel edge h):
 *   A(lambda) = D_lambda K + B/(2 A_R) + (mu_a(lambda) + i omega/nu) h^3 I
 *   (K phi)_n = h * sum_{face neighbours m}(phi_n - phi_m) + 2h phi_n per Dirichlet face,
 *   B = diag(h^2 * number of Robin faces of voxel n),
 *   D_lambda = 1/(3 mu_s'(lambda)), mu_a(lambda) = sum_l c_l eps_l(lambda)
 *   (Sec. 2.1 diffusion equation with the Robin and Dirichlet conditions and
 *   eq. perturbation; the finite-element matrices of Sec. 2.2 replaced by this
 *   finite-volume form, which keeps the affine dependence on the wavelength).
 *
 * Conventions for every call:
 *   - Device buffers are allocated and owned by the caller, scratch included (each
 *     call that needs device scratch takes a caller-owned workspace sized by its
 *     *_workspace_bytes query); the library never allocates or frees device memory
 *     in a call on the hot path and never frees caller memory.  The library owns
 *     only the opaque operator (and the device copies it keeps for
 *     hydot_set_absorption_perturbation and hydot_apply_preconditioner).
 *   - Complex data are interleaved (re, im) pairs: HYDOT_C128 = 2 x double,
 *     HYDOT_C64 = 2 x float.  All arrays are densely packed, C order.
 *   - Work is enqueued on the caller's stream (NULL = default stream).  Calls
 *     that return host values synchronise that stream before returning.
 *   - Arguments are validated before any launch: HYDOT_EINVAL leaves every
 *     output untouched.  A HIP failure returns HYDOT_EDEVICE.  The message of
 *     the last non-OK status is returned by hydot_last_error() (per thread).
 */
#ifndef HYDOT_H
#define HYDOT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HYDOT_OK = 0,
  HYDOT_ENOCONV = 1,        /* warning: some systems above tolerance; outputs written */
  HYDOT_EINVAL = -1,        /* invalid argument; nothing launched, outputs untouched */
  HYDOT_ENOMEM = -2,        /* workspace too small, or a host allocation failed */
  HYDOT_EDEVICE = -3,       /* a HIP runtime call failed */
  HYDOT_EUNSUPPORTED = -4   /* valid but not supported combination (e.g. dtype) */
} hydot_status;

typedef enum {
  HYDOT_C128 = 0,           /* complex FP64 (re, im) */
  HYDOT_C64 = 1,            /* complex FP32 (re, im) */
  HYDOT_CBF16 = 2,          /* complex BF16 (re, im): 2 x bfloat16, rounded to nearest even */
  HYDOT_F64 = 3,            /* real FP64 */
  HYDOT_F32 = 4             /* real FP32 */
} hydot_dtype;

/* Box grid. robin_faces: bit f set = Robin on face f in the order
 * (-x, +x, -y, +y, -z, +z); bit clear = zero Dirichlet (Sec. 2.1). 0x3F = all Robin. */
typedef struct {
  int32_t nx, ny, nz;       /* >= 1 each; nx*ny*nz < 2^31 */
  double h_mm;              /* voxel edge [mm], > 0 */
  double A_R;               /* Robin coefficient A (refractive-index mismatch), > 0 */
  uint32_t robin_faces;
} hydot_grid;

/* Background optics per wavelength (host arrays, copied by assemble). */
typedef struct {
  int32_t n_lambda;                 /* >= 1 */
  const double* mus_prime_per_mm;   /* [n_lambda] reduced scattering mu_s' > 0 */
  int32_t n_species;                /* >= 1, <= 8 */
  const double* extinction;         /* [n_species][n_lambda] eps_l(lambda) [1/(mm uM)] */
  const double* conc_uM;            /* [n_species] background concentrations c_l */
  double omega_over_nu_per_mm;      /* modulation frequency over speed of light in tissue */
} hydot_optics;

/* Solver flags */
#define HYDOT_FLAG_NO_RECYCLE  0x1u  /* recycle_k treated as 0 and no multi-shift initial guess */
#define HYDOT_FLAG_MEAN_SHIFT  0x2u  /* K <- K + mean(sigma') R, sigma'_j <- sigma'_j - mean (Sec. 6.1) */
#define HYDOT_FLAG_GRAPH       0x4u  /* capture each restart cycle in a hipGraph and replay it */
#define HYDOT_FLAG_PER_SYSTEM  0x8u  /* plain mode: one (rhs, lambda) system at a time, per-call launches */
#define HYDOT_FLAG_SHIFT_MIN   0x20u /* like MEAN_SHIFT with min_j sigma'_j in K_hat (Sec. 6.1 variants) */
#define HYDOT_FLAG_SHIFT_MAX   0x40u /* like MEAN_SHIFT with max_j sigma'_j in K_hat; at most one of
                                        MEAN_SHIFT, SHIFT_MIN, SHIFT_MAX */
#define HYDOT_FLAG_PRECOND_SEP 0x80u /* mixed batched path only: right preconditioner
                                        P_j = K_hat + sigma_j I, inverted exactly on the box by
                                        three 1-D eigenvector transforms per axis pass (a GPU
                                        replacement for the ILU of K_hat used in Sec. 6.1);
                                        K_hat includes the sigma*' of the shift flag in use */
#define HYDOT_FLAG_PRECOND_SEP_FIXED 0x100u /* as PRECOND_SEP with one shift for every system: the
                                        mean of sigma_j over the wavelengths; at most one of the two.
                                        Both need recycle_k <= 10, restart_m - recycle_k <= 32 and
                                        grid axes of at most 256 cells (else EUNSUPPORTED) */
#define HYDOT_FLAG_FULL_REORTH 0x10u /* mixed only: apply the second Gram-Schmidt pass at every step.
                                        Default: the FP32 inner Arnoldi skips it for a system whose
                                        second-pass projection is below 1e-4 ||w'|| (orthogonal to
                                        working precision); the FP64 path always applies it. */

#define HYDOT_PREC_FP64  0           /* Krylov basis and operator in complex FP64 */
#define HYDOT_PREC_MIXED 1           /* complex FP32 Krylov inner solves, FP64 residual refinement */

typedef struct {
  double rel_tol;           /* stop when ||b - A phi||_2/||b||_2 <= rel_tol (FP64-recomputed), > 0 */
  int32_t max_iter;         /* cap on Arnoldi steps per system, >= 1 */
  int32_t restart_m;        /* m: Arnoldi steps per cycle are m - k; m - k in [1, 128] */
  int32_t recycle_k;        /* k: deflation space dimension, 0..32, < lanczos_n */
  int32_t lanczos_n;        /* n: shift-invariant Krylov steps on K (Alg. 1 step 1), 1..128 */
  int32_t precision;        /* HYDOT_PREC_FP64 or HYDOT_PREC_MIXED */
  uint32_t flags;           /* HYDOT_FLAG_* */
  double inner_tol;         /* mixed only: relative tolerance of each FP32 inner solve (e.g. 1e-5) */
  int32_t max_batch;        /* systems solved concurrently (0 = all); ignored with PER_SYSTEM */
} hydot_solve_opts;

typedef struct hydot_operator hydot_operator;   /* opaque, library-owned */

/* Copy the grid and optics into a new operator (host memory only) and evaluate the
 * optical model: D_lambda, mu_a(lambda), the shifts sigma_j = (mu_a + i omega/nu)/D,
 * sigma'_j = 1/(2 A_R D) of eq. multipleshifted and their mean (Sec. 6.1). */
hydot_status hydot_assemble_operator(const hydot_grid* grid, const hydot_optics* optics,
                                     hydot_operator** out);
void hydot_free_operator(hydot_operator* op);

/* Host copies of the per-wavelength model: D [mm], mu_a [1/mm] (each [n_lambda], any may be NULL). */
hydot_status hydot_operator_optics(const hydot_operator* op, double* D_out, double* mua_out);

/* y_v = A(lambda_v) x_v for n_vec vectors (the matrix-free operator of Sec. 2.2 in
 * finite-volume form).  x, y: device [n_vec][N] complex of dtype C128 or C64.
 * lam_index: host [n_vec], each in [0, n_lambda). x and y must not overlap. */
hydot_status hydot_apply_operator(const hydot_operator* op, int32_t n_vec, const int32_t* lam_index,
                                  const void* x, void* y, hydot_dtype dtype, hipStream_t stream);

/* The separable preconditioner of HYDOT_FLAG_PRECOND_SEP(_FIXED) on its own (Sec. 6.1 uses an
 * ILU of the mean-shifted matrix in its place): y_v = (K_hat + sigma I)^{-1} x_v in the scaled
 * form of eq. multipleshifted, A(lambda_j) / (D_j h^3) = K / h^3 + sigma'_j B / h^3 + sigma_j I, with
 * K_hat = K / h^3 + sigma*' B / h^3, sigma*' the mean, minimum or maximum of sigma'_j per
 * the shift flag in `flags` (0 without one), sigma = sigma_{lam_index} with PRECOND_SEP or the mean
 * of sigma_j with PRECOND_SEP_FIXED (exactly one of the two in flags).  Exact on the box up to FP32
 * rounding; any absorption perturbation of the operator is not included.
 * x, y: device [count][N] complex FP32 (HYDOT_C64); y may equal x (in place), other overlaps are
 * not allowed.  1 <= count <= 65535; grid axes of at most 256 cells (else EUNSUPPORTED).  The
 * first call for a given sigma*' builds the axis eigen-decompositions (host, then one
 * synchronous copy into an operator-owned device buffer). */
hydot_status hydot_apply_preconditioner(const hydot_operator* op, uint32_t flags, int32_t lam_index,
                                        const void* x, void* y, int32_t count, hipStream_t stream);

/* Heterogeneous absorption (Sec. 2.1 diffusion equation with mu_a varying in space; eq.
 * perturbation): mu_a(k, lambda_l) = mu_a(lambda_l) + scale[l] * shape[k], so A(lambda_l) gains
 * h^3 diag(scale_l shape) -- the full forward model the Born approximation linearises.  Every
 * later hydot_apply_operator and hydot_solve_fields call on this operator includes it; the
 * recycled solver still applies (the perturbation is one more per-wavelength diagonal shift; its
 * mean over wavelengths joins K_hat with HYDOT_FLAG_MEAN_SHIFT).  The Born calls do not use it.
 * shape: host [N] (e.g. a PaLS shape), scale: host [n_lambda] in mm^-1 (ebar_l = sum over species
 * of eps(lambda_l) dconc).  shape = NULL clears the perturbation.  The operator keeps device
 * copies of the shape (FP64 and FP32), freed with the operator.  Synchronous. */
hydot_status hydot_set_absorption_perturbation(hydot_operator* op, const double* shape, const double* scale);

/* Bytes of device workspace hydot_solve_fields needs for n_rhs right-hand sides. */
hydot_status hydot_solve_workspace_bytes(const hydot_operator* op, int32_t n_rhs,
                                         const hydot_solve_opts* opts, size_t* bytes);

/* Fields for every right-hand side at every wavelength (Alg. 1, Sec. 3.1).
 * rhs_voxel: host [n_rhs] voxel indices; right-hand side r is a unit injection
 *   into that voxel (S = S0 delta(r - r_s) with S0 = 1).  Sources and detectors
 *   (adjoint fields, Sec. 2.1) are both passed here; slice the output.
 * phi: device [n_lambda][n_rhs][N], the physical fields (not D*phi), dtype C128, C64 or
 *   CBF16 (rounded from the FP64 iterate; the storage the BF16 Born products read).
 * workspace: device, >= the size from hydot_solve_workspace_bytes, 256-byte aligned.
 * iters: host [n_lambda*n_rhs] (lambda-major) Arnoldi steps per system, or NULL.
 * rel_res: host [n_lambda*n_rhs] final FP64-recomputed ||b - A phi||/||b|| of the
 *   FP64 iterate (before any conversion to C64 or CBF16), or NULL.
 * Returns HYDOT_ENOCONV (fields still written) if any system stays above rel_tol; HYDOT_ENOMEM if
 * a host allocation of the set-up fails (work may then be left queued on the stream). */
hydot_status hydot_solve_fields(hydot_operator* op, int32_t n_rhs, const int64_t* rhs_voxel,
                                const hydot_solve_opts* opts, void* phi, hydot_dtype phi_dtype,
                                void* workspace, size_t ws_bytes, int32_t* iters, double* rel_res,
                                hipStream_t stream);

/* Several independent solves of Alg. 1 (Sec. 3.1), one per operator (e.g. a main grid and smaller
 * grids at the same wavelengths), run as one batch: each problem's kernels go to a stream of
 * its own forked from `stream` (they start after the work queued on `stream` before the call)
 * and one host thread per problem drives its restart cycles, so the grids' launches run on
 * the GPU concurrently.  Every problem's fields, iters and rel_res are exactly those of a
 * hydot_solve_fields call with the same arguments (the arithmetic of each problem is unchanged).
 * problems: host [n_problems], 1 <= n_problems <= HYDOT_SOLVE_BATCH_MAX; the fields of each are
 *   as in hydot_solve_fields; the operators must be distinct (a solve updates its operator's
 *   caches) and the workspaces and outputs must not overlap.  `status` is written per problem.
 * Returns the lowest-indexed problem's error if any failed (hydot_last_error names it; the other
 * problems still ran), else HYDOT_ENOCONV if any problem returned it, else HYDOT_OK; EINVAL (nothing
 * launched) for a bad count, a null operator or a repeated operator.  All work has completed
 * when it returns.  While the profiler is enabled the problems run one after another. */
#define HYDOT_SOLVE_BATCH_MAX 16
typedef struct {
  hydot_operator* op;
  int32_t n_rhs;
  const int64_t* rhs_voxel;
  const hydot_solve_opts* opts;
  void* phi;
  hydot_dtype phi_dtype;
  void* workspace;
  size_t ws_bytes;
  int32_t* iters;
  double* rel_res;
  hydot_status status;      /* out */
} hydot_solve_problem;
hydot_status hydot_solve_fields_batch(int32_t n_problems, hydot_solve_problem* problems, hipStream_t stream);

/* Read-back of the solver's intermediates (Alg. 1) for tests and diagnosis, from the workspace
 * of the last hydot_solve_fields call made with the same operator, n_rhs and opts (the workspace
 * must not have been used since).  Synchronous host copies on `stream`.
 *   HYDOT_INSPECT_U, HYDOT_INSPECT_C: index = right-hand side of the last Lanczos batch (every
 *     right-hand side unless PER_SYSTEM); out: host [k][N] double, U and C of Alg. 1 steps 2-4
 *     (real; in the scaled form of eq. multipleshifted K_hat U = C and C^T C = I, eq. gcr, with
 *     K_hat = K/h^3 + sigma*' B/h^3 and sigma*' the shift moved into K_hat by the shift flag).
 *   HYDOT_INSPECT_CHOL: index = system of the last batch (all R*L systems in right-hand-side-major
 *     order when max_batch is 0; info->rhs and info->lam name it); out: host [k][k] complex
 *     double, column-major lower factor F of G_j = C_j'^H C_j' = F F^H, C_j' = A_j U with
 *     A_j = A(lambda_j)/(D_j h^3) (Alg. 1 steps 7-8: C_j = C_j' F^-H, U_j = U F^-H).
 *   HYDOT_INSPECT_CYCLE: index as CHOL; the system's last restart cycle of m = info->nsteps
 *     deflated Arnoldi steps (Alg. 1 step 10): out: host complex double, in order
 *     F' [k][m] (F'[i][l] = (C_j' e_i)^H A_j v_l summed over both Gram-Schmidt passes),
 *     Hbar [(m+1) x m] column-major (the Hessenberg matrix, Givens rotations undone),
 *     V [m][N] (the basis v_0..v_{m-1}), so that A_j v_l = C_j' G_j^-1 F'[:, l] + sum_i Hbar[i][l] v_i
 *     (the modified Arnoldi relation) with v_m = r / Hbar[m][m-1] for the residual r of the last
 *     column: v_m itself is never formed (the cycle's update uses only v_0..v_{m-1}), so r has
 *     norm |Hbar[m][m-1]| and is orthogonal to C_j and V.  Needs 16 (k m + (m+1) m + m N) bytes.
 * out = NULL fills only info (then out_bytes is ignored).  EINVAL for an index outside the last
 * batch or an item the options do not have; ENOMEM if out_bytes is too small. */
enum { HYDOT_INSPECT_U = 0, HYDOT_INSPECT_C = 1, HYDOT_INSPECT_CHOL = 2, HYDOT_INSPECT_CYCLE = 3 };
typedef struct {
  int32_t rhs, lam;   /* the right-hand side and wavelength the item belongs to (lam -1 for U, C) */
  int32_t k;          /* deflation dimension */
  int32_t nsteps;     /* CHOL, CYCLE: Arnoldi steps of the system's last restart cycle */
} hydot_inspect_info;
hydot_status hydot_solve_inspect(const hydot_operator* op, int32_t n_rhs, const hydot_solve_opts* opts,
                                 const void* workspace, size_t ws_bytes, int32_t what, int32_t index,
                                 void* out, size_t out_bytes, hydot_inspect_info* info, hipStream_t stream);

#define HYDOT_BORN_PAIRS_MIN_NV 12

/* Arithmetic of the J v products.  HYDOT_BORN_SPLIT_BF16 (C64 fields only): each FP32 operand
 * x is split into hi = bf16(x) and lo = bf16(x - hi) and the product accumulates
 * hi*hi + hi*lo + lo*hi on the BF16 MFMA (relative error of order 1e-5, FP32 field bytes). */
typedef enum { HYDOT_BORN_NATIVE = 0, HYDOT_BORN_SPLIT_BF16 = 1 } hydot_born_compute;

/* Born products (Sec. 2.1 integral equation with the adjoint field; the rows of H in eq.
 * measurement), never forming J:
 *   y[c][l][s][d] = -h^3 sum_k phi_src[l][s][k] * v[c][k] * phi_det[l][d][k]   (no conjugation)
 * the derivative of the detector reading of source s at wavelength l with respect to the
 * absorption in voxel k, times v_c (Sec. 2.1, Born approximation).
 * phi_src: device, source s at wavelength l at phi_src + (l*lam_stride + s)*N elements;
 * phi_det: likewise with d.  lam_stride >= max(S, D) counts N-vectors between wavelengths
 * (S for a packed source array, n_rhs for slices of the hydot_solve_fields output).
 * field_dtype C128: v is FP64, y is C128 (FP64 MFMA).
 *             C64:  v is FP32, y is C64 (FP32 MFMA, FP64 sums across 32-voxel stages and splits).
 *             CBF16: v is FP32, y is C64; both operands (phi_src v formed in FP32, and phi_det)
 *                   rounded to BF16 for the BF16 MFMA, FP32 accumulation within a stage, FP64
 *                   beyond.  Relative error of order 1e-2 (a stated-error variant).
 * Blocks of n_v >= HYDOT_BORN_PAIRS_MIN_NV probe vectors are contracted over source-detector
 * pairs instead: phi_src * phi_det formed once per pair and voxel (FP64 for C128 fields, FP32
 * otherwise) and multiplied with the probe block on MFMA.  Same accumulation; half the MFMA work
 * per probe vector.  With CBF16 fields it is the pair product and v that are rounded to BF16.
 * v: device [n_v][N] real.  y: device [n_v][n_lambda][S][D].  1 <= S, D <= 64, 1 <= n_v <= 64.
 * workspace: device scratch for the FP64 partial sums over voxel ranges, 256-byte aligned, at
 *   least the bytes hydot_born_workspace_bytes returns for the same operator (its current launch
 *   shapes), S, D, field_dtype, compute and n_v; smaller is HYDOT_ENOMEM before any launch.
 *   Its contents on entry do not matter; the call overwrites it.  Calls that overlap in time must
 *   not share a workspace. */
hydot_status hydot_born_workspace_bytes(const hydot_operator* op, int32_t S, int32_t D, hydot_dtype field_dtype,
                                        hydot_born_compute compute, int32_t n_v, size_t* bytes);
hydot_status hydot_born_apply(const hydot_operator* op, const void* phi_src, int32_t S,
                              const void* phi_det, int32_t D, int64_t lam_stride,
                              hydot_dtype field_dtype, const void* v, int32_t n_v, void* y,
                              void* workspace, size_t ws_bytes, hipStream_t stream);

hydot_status hydot_born_apply_ex(const hydot_operator* op, const void* phi_src, int32_t S,
                                 const void* phi_det, int32_t D, int64_t lam_stride,
                                 hydot_dtype field_dtype, hydot_born_compute compute, const void* v,
                                 int32_t n_v, void* y, void* workspace, size_t ws_bytes,
                                 hipStream_t stream);

/* Measurement hook: achievable peaks of the current GPU from hand-written probe kernels, for
 * stating rooflines against measured figures beside the published ones (HBM 8 TB/s, FP32 MFMA
 * 157.3 TFLOP/s, BF16 MFMA 2.5 PFLOP/s dense).  buffer: device, 256-byte aligned, at least 1 GiB
 * (caller-owned scratch; its contents are overwritten).  Streams: ten vectors read with
 * non-temporal loads (read_GBps), a copy (copy_GBps, read + write bytes), ten vectors read and
 * one written (read10_write1_GBps: the traffic mix of an Arnoldi update); MFMA: independent chains
 * of v_mfma_f32_32x32x2f32 and v_mfma_f32_16x16x32_bf16 with operands in registers.  Each figure
 * is the median of five timed launches.  Synchronises the stream. */
typedef struct {
  double read_GBps, copy_GBps, read10_write1_GBps;
  double mfma_f32_TFLOPs, mfma_bf16_TFLOPs;
  int32_t compute_units;
} hydot_peaks;
hydot_status hydot_measure_peaks(void* buffer, size_t bytes, hydot_peaks* out, hipStream_t stream);

/* Allocation-free J v, for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same products, kernels and
 * arguments as hydot_born_apply_ex, without the workspace.  The FP64 partial sums live in a
 * static device array of HYDOT_BORN_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds until the process ends; the voxel split of the current launch shapes is lowered until
 * the partials fit.  A call whose partials for a single voxel range (n_v * n_lambda * S * D
 * complex FP64 values with the pair-product kernel, n_v * n_lambda * 2S' * 2D' FP64 values
 * otherwise, S' and D' rounded up to 8) exceed the array returns HYDOT_ENOMEM before any launch.
 * Calls no hipMalloc or hipFree and allocates no host memory on success (only an error path
 * formats its message).  The first call on a device looks up that device's address of the
 * array (hipGetSymbolAddress) and keeps it.  Works on the current device.  Every call
 * on one GPU shares that GPU's array: calls that overlap in time on one GPU (other streams,
 * other host threads) race and must be serialised by the caller. */
#define HYDOT_BORN_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
hydot_status hydot_born_apply_noalloc(const hydot_operator* op, const void* phi_src, int32_t S,
                                      const void* phi_det, int32_t D, int64_t lam_stride,
                                      hydot_dtype field_dtype, hydot_born_compute compute,
                                      const void* v, int32_t n_v, void* y, hipStream_t stream);

/* Adjoint product summed over wavelengths: the product with the conjugate transpose of H that
 * the gradient of the misfit needs (Sec. 5, the gradient of eq. minimization uses H^T; the
 * Jacobian step of Alg. opt):
 *   g[k] = sum_{l,s,d} conj(J_l[s,d,k]) w[l][s][d] = -h^3 sum conj(phi_src[l][s][k] phi_det[l][d][k]) w[l][s][d]
 * w: device [n_lambda][S][D] complex and g: device [N] complex, both C128 for C128 fields and C64
 * for C64 or CBF16 fields.  CBF16 fields are widened exactly to FP32 for the FP32 MFMA, except
 * with S and D both above 32: then the BF16 MFMA multiplies the stored field words directly with
 * w split into BF16 hi + lo (w kept to about 2^-17 relative; sums in FP32 over the sources, FP64
 * over detectors and wavelengths).
 * Field layout and lam_stride as hydot_born_apply.  Needs no scratch: each block owns a range of
 * voxels and sums over every wavelength in registers, writing g once. */
hydot_status hydot_born_apply_adjoint(const hydot_operator* op, const void* phi_src, int32_t S,
                                      const void* phi_det, int32_t D, int64_t lam_stride,
                                      hydot_dtype field_dtype, const void* w, void* g,
                                      hipStream_t stream);

/* Block form of the adjoint product: g[c] = sum_l J_l^H w[c][l] for c < n_w, 1 <= n_w <= 1024
 * (the products with the transpose of H that the randomized compression of Sec. 4 and its
 * appendix need).  w: device [n_w][n_lambda][S][D], g: device [n_w][N], dtypes as
 * hydot_born_apply_adjoint. */
hydot_status hydot_born_apply_adjoint_ex(const hydot_operator* op, const void* phi_src, int32_t S,
                                         const void* phi_det, int32_t D, int64_t lam_stride,
                                         hydot_dtype field_dtype, const void* w, int32_t n_w, void* g,
                                         hipStream_t stream);

/* PaLS shape (Sec. 5, eq. pals) at the voxel centres ((i+1/2)h, (j+1/2)h, (k+1/2)h):
 *   mu(r) = H_eps(varphi(r) - tau),  varphi(r) = sum_b alpha_b psi(beta_b ||r - chi_b||_dag),
 *   ||x||_dag = sqrt(||x||^2 + nu^2), H_eps the C^1 sine-smoothed Heaviside of half-width eps,
 *   and psi chosen by basis: HYDOT_PALS_WENDLAND (the paper's compactly supported radial
 *   functions, read as Wendland's C^2 psi(t) = (1 - t)^4 (4t + 1) on t < 1 and 0 beyond, support
 *   radius 1/beta_b) or HYDOT_PALS_GAUSSIAN (psi(t) = exp(-t^2), width 1/beta_b).
 * p: host [5*n_bumps] = [alpha, beta, chi_x, chi_y, chi_z] (Sec. 5 ordering), 1 <= n_bumps <= 32.
 * mu: device [N] real of dtype F64 or F32. */
enum { HYDOT_PALS_WENDLAND = 0, HYDOT_PALS_GAUSSIAN = 1 };
typedef struct {
  double tau, eps, nu;
  int32_t basis;   /* HYDOT_PALS_WENDLAND or HYDOT_PALS_GAUSSIAN; anything else is EINVAL */
} hydot_pals_opts;

hydot_status hydot_pals_shape(const hydot_operator* op, const double* p, int32_t n_bumps,
                              const hydot_pals_opts* popts, void* mu, hydot_dtype mu_dtype,
                              hipStream_t stream);

/* Vector-Jacobian product of the shape: grad_p[i] = sum_k (d mu_k / d p_i) * Re(g_k).
 * g: device [N] of dtype F64, F32, C128 or C64 (the real part is used).
 * grad_p: host [5*n_bumps].  workspace: device, >= hydot_pals_workspace_bytes(). Synchronises. */
size_t hydot_pals_workspace_bytes(const hydot_operator* op, int32_t n_bumps);
hydot_status hydot_pals_shape_vjp(const hydot_operator* op, const double* p, int32_t n_bumps,
                                  const hydot_pals_opts* popts, const void* g, hydot_dtype g_dtype,
                                  double* grad_p, void* workspace, size_t ws_bytes,
                                  hipStream_t stream);

/* Shape Jacobian (Sec. 5, the derivative of eq. pals used by the Levenberg-Marquardt step of
 * Alg. opt): jac[i][k] = d mu_k / d p_i for the 5*n_bumps parameters in the order of p, as a
 * device [5*n_bumps][N] array of dtype F64 or F32 -- a block of probe vectors for
 * hydot_born_apply, whose product gives H d mu / d p. */
hydot_status hydot_pals_shape_jacobian(const hydot_operator* op, const double* p, int32_t n_bumps,
                                       const hydot_pals_opts* popts, void* jac, hydot_dtype jac_dtype,
                                       hipStream_t stream);

/* Data misfit of the Born model with co-located chromophores (eq. measurement, eq. minimization):
 *   ebar_l = sum_species eps(lambda_l) dconc,  yhat = ebar_l * Jmu,  r = yhat - y_obs,
 *   f = 1/2 sum weights^2 |r|^2,
 *   grad_dconc[sp] = Re sum conj(weights^2 r) eps_sp(lambda_l) Jmu,
 *   w_adj = ebar_l * weights^2 * r   (input of hydot_born_apply_adjoint for df/dmu = Re J^H w_adj).
 * Jmu, y_obs, w_adj: device [n_lambda][S][D] complex of dtype C128 or C64 (all the same).
 * weights: device [n_lambda][S][D] real of the matching real dtype, or NULL for W = I.
 * dconc: host [n_species].  f, grad_dconc: host outputs.  workspace >= hydot_misfit_workspace_bytes().
 * Synchronises the stream. */
size_t hydot_misfit_workspace_bytes(const hydot_operator* op, int32_t S, int32_t D);
hydot_status hydot_misfit(const hydot_operator* op, int32_t S, int32_t D, const double* dconc,
                          const void* Jmu, const void* y_obs, const void* weights, hydot_dtype dtype,
                          void* w_adj, double* f, double* grad_dconc, void* workspace,
                          size_t ws_bytes, hipStream_t stream);

/* Launch shapes of the hot kernels, held by the operator and used by every later call on it.
 * They change only the speed and the FP32 summation order (so results within the tolerance of
 * the precision in use), never the method.  A field set to 0 selects the library default.
 *   step_presum  Arnoldi step kernels of the complex FP32 path: number of neighbouring lanes
 *                (1, 2 or 4) whose inner-product terms are summed in registers before the LDS
 *                product tile of every 128-voxel sub-tile; 2 and 4 shrink the tile so more
 *                blocks fit a CU; 16: each thread sums the terms of its 16 voxels of the chunk
 *                in registers and the block reduces once per chunk (instances up to 16 basis
 *                vectors and x rows of at most 128 voxels; otherwise 4 is used) (default 16).
 *   step_order   1: blocks ordered so each XCD runs a contiguous range of (system, chunk) tiles;
 *                2: plain dispatch order; 3: z-slab order, each XCD runs a contiguous range of
 *                chunks (a slab of z-planes) of every system, so the stencil's z-neighbour
 *                chunks are read on the XCD that reads them as centres (falls back to 2 where
 *                the chunk count does not split over the XCDs); 4: chunk c on XCD c % 8 for
 *                every system (its z-neighbour chunks on the same XCD), with the wavelengths of
 *                one right-hand side taking each chunk in consecutive blocks there, so each
 *                chunk of the shared recycled basis is fetched once per XCD (implies the
 *                wavelength grouping when the batch holds whole right-hand sides; falls back to
 *                2 where the chunk count is not a multiple of 8) (default: 4 where nx ny is a
 *                multiple of 16384, so that a z-plane holds a multiple of 8 chunks, else 3).
 *   step_group   1: consecutive blocks walk the wavelengths of one right-hand side at one chunk
 *                (shared recycled basis in L2); 2: no grouping (default 2).
 *   born_stage   J v voxels per LDS stage: 16 or 32 (default: 32 where the stage fits 64 KB).
 *   born_blocks  J v target grid size in blocks (split over voxels), 256..65536 (default 4096).
 *   step_vx      Arnoldi step kernels, up to 16 basis vectors: voxels per thread per sub-tile,
 *                1 or 2 (2 only with step_presum 4); their terms are summed in registers before
 *                the pre-sum (default 1).
 *   step_pair    2: with step_presum 16, the Arnoldi step kernels of systems without an absorption
 *                perturbation or a preconditioner take two wavelengths of one right-hand side per
 *                block, loading the C and U they share once (batches of whole right-hand sides
 *                with an even number of wavelengths; results identical with the instances for
 *                k = 5, equal to rounding otherwise); 1: one system per block
 *                (default 2). */
typedef struct {
  int32_t step_presum, step_order, step_group;
  int32_t born_stage, born_blocks;
  int32_t step_vx;
  int32_t step_pair;
} hydot_tuning;
hydot_status hydot_get_tuning(const hydot_operator* op, hydot_tuning* out);   /* resolved values */
hydot_status hydot_set_tuning(hydot_operator* op, const hydot_tuning* t);      /* EINVAL if out of range */

/* Autotuner.  Each trial is one candidate hydot_tuning and its measured time in ms. */
typedef struct {
  hydot_tuning t;
  double ms;
} hydot_tune_trial;

/* Times every candidate ((step_presum, step_vx) in {(16,1), (4,1), (2,1), (4,2)} x step_order in
 * {the grid's default order, 2 (3 where the default is 2)} x step_group in {2, 1}) on the caller's
 * problem: each
 * trial is the hydot_solve_fields call with these arguments, timed by HIP events around the
 * Arnoldi step kernels only.  Candidates are tried with the library default first; a later one
 * replaces the best only when it is more than 1% faster (timing noise keeps the default).  The
 * chosen candidate is stored in the operator and phi holds the fields of the last trial.
 * trials: host [max_trials] or NULL; n_trials: host, number of candidates timed.
 * Synchronises the stream.  Not thread-safe (uses the process-wide instrumentation). */
hydot_status hydot_autotune_solve(hydot_operator* op, int32_t n_rhs, const int64_t* rhs_voxel,
                                  const hydot_solve_opts* opts, void* phi, hydot_dtype phi_dtype,
                                  void* workspace, size_t ws_bytes, hydot_tune_trial* trials,
                                  int32_t max_trials, int32_t* n_trials, hipStream_t stream);

/* Times every J v candidate (born_stage x born_blocks) on the given arguments (the median of
 * 5 calls of hydot_born_apply each; default first, a later candidate must be more than 2%
 * faster) and stores the chosen one in the operator; y receives the product.  Arguments as
 * hydot_born_apply; the workspace must hold the largest candidate's scratch,
 * hydot_autotune_born_workspace_bytes (else HYDOT_ENOMEM before any launch); trials and n_trials
 * as hydot_autotune_solve.  Synchronises the stream. */
hydot_status hydot_autotune_born_workspace_bytes(const hydot_operator* op, int32_t S, int32_t D,
                                                 hydot_dtype field_dtype, int32_t n_v, size_t* bytes);
hydot_status hydot_autotune_born(hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det,
                                 int32_t D, int64_t lam_stride, hydot_dtype field_dtype, const void* v,
                                 int32_t n_v, void* y, void* workspace, size_t ws_bytes,
                                 hydot_tune_trial* trials, int32_t max_trials, int32_t* n_trials,
                                 hipStream_t stream);

/* Measurement instrumentation (not part of the method).  While enabled, hydot_solve_fields
 * records HIP events on its stream around every launch of the three Arnoldi step kernels
 * (first-pass dots with the operator, CGS2 update, normalisation) and accumulates, per
 * kernel, launches, elapsed milliseconds and algorithmic HBM bytes: for step j with
 * storage b bytes per complex, k deflation vectors, A systems stepping and R' distinct
 * right-hand sides among them,
 *   dots (A*(j+2) + R'*k)*N*b, update (A*(j+3) + R'*k)*N*b, finish (A'*(j+3) + min(A', R')*k)*N*b
 * with A' the systems whose second Gram-Schmidt pass is applied at step j: each unique
 * vector is read once and the written vector counted; C and U (real, b/2 each) are
 * shared by the wavelengths of a right-hand side, so they count once per right-hand side.
 * The complex FP32 kernels for up to 16 basis vectors without a preconditioner keep the
 * work vector W = A v_j out of memory (the update recomputes it from the stencil of V_j):
 * there dots (A*(j+1) + R'*k)*N*b and update (A*(j+2) + R'*k)*N*b.  Record names: the kernel
 * of the last solve's form ("k_step_dots_t", "k_step_update_t", "k_step_finish_t"; with two
 * systems per block "k_step_pair_t<dots>", "k_step_pair_t<update>"; "k_step_dots" etc. for
 * the generic kernels).
 * Enabling resets the counters; the graph flag is ignored while enabled (launches are
 * timed one by one).  Process-wide; not thread-safe (hydot_solve_fields_batch runs its
 * problems one after another while it is enabled). */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double total_bytes;
} hydot_kernel_profile;
hydot_status hydot_profile_enable(int32_t on);
/* Writes up to max_records records; returns the number written (records available if out == NULL). */
int32_t hydot_profile_read(hydot_kernel_profile* out, int32_t max_records);

const char* hydot_last_error(void);
const char* hydot_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HYDOT_H */
