/*
 * pprpa.h -- C ABI of the MI355X (gfx950) particle-particle RPA library (libpprpa.so).
 *
 * The library solves the ppRPA generalised eigenproblem of arXiv 2512.12515,
 * section "ppRPA Equation", Eq. eigen_equation:
 *
 *     [[A, B], [B^T, C]] [X; Y] = Omega diag(I, -I) [X; Y]
 *
 * for a closed-shell reference in its spin-adapted singlet or triplet form (same section),
 * with the physicists' integrals <pq|rs> = (pr|qs) (defined beside Eq. dyson) from
 * density-fitted MO-basis three-centre integrals, (pq|rs) = sum_P L^P_pq L^P_rs
 * (section "Implementation Details"), optionally in a canonical active window.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Orbitals are in physical order: occupied 0..nocc-1 then virtual nocc..nmo-1, each block
 *    in ascending energy. Energies in Hartree.
 *  - Active window: the highest nocc_act occupied and the lowest nvir_act virtual orbitals
 *    (<= 0 means all of them). Below, no/nv are the active counts.
 *  - Packed pair vectors: z = [x; y], x over virtual pairs (a, b), y over occupied pairs
 *    (i, j), each in upper-triangle row-major order with the first index outer:
 *    singlet a <= b (n_pp = nv(nv+1)/2), triplet a < b (n_pp = nv(nv-1)/2); the same for y.
 *    n = n_pp + n_hh. Blocks of k vectors are row-major [k][n] (vector-contiguous), FP64.
 *  - Returned eigenvectors are normalised to x^T x - y^T y = +1 (Eq. xy_norm, pp roots) and
 *    signed so that their largest-magnitude component is positive.
 *  - All functions are synchronous with respect to the caller: device work is ordered on
 *    the context's stream, which is synchronised before results are returned.
 *  - No exception crosses the ABI. Every function returns a pprpa_status; on failure
 *    pprpa_last_error() gives a message for the calling thread.
 *  - "host or device" pointers: the on_device flag says which; device pointers must be
 *    memory of the context's device (e.g. a torch tensor's data_ptr()).
 *  - Environment: PPRPA_ROCTX=1 makes the library open the ROCm profiler SDK's roctx library
 *    (by dlopen, on first use) and push a named range around each entry point and each host-side
 *    Davidson phase, for rocprofv3 --marker-trace; unset, or when that library cannot be opened,
 *    nothing is traced and nothing else changes.
 */
#ifndef PPRPA_H
#define PPRPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PPRPA_OK = 0,
  PPRPA_EINVAL = 1,       /* invalid or inconsistent argument (sizes, window, NaN/Inf input) */
  PPRPA_ENOMEM = 2,       /* device allocation failed or exceeded a budget */
  PPRPA_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed */
  PPRPA_ENOCONV = 4,      /* Davidson did not converge in max_iter; outputs hold the last iterate */
  PPRPA_ENONDEF = 5,      /* (projected) pencil M - 2 mu W not positive definite */
  PPRPA_EUNSUPPORTED = 6, /* valid but unsupported combination */
  PPRPA_EBUSY = 7         /* the context is in use by another thread */
} pprpa_status;

typedef enum { PPRPA_SINGLET = 0, PPRPA_TRIPLET = 1 } pprpa_mult;

/* Arithmetic of the sigma contractions (the Davidson linear algebra is FP64 always).
 * FP64: FP64 MFMA. FP32: L and the unpacked vectors rounded to FP32, FP32 MFMA, FP32
 * accumulation. BF16X3 / BF16X6: each FP32 operand split into bf16 hi+mid+lo, products
 * hh+hm+mh (X3) or hh+hm+mh+mm+hl+lh (X6) on BF16 MFMA, FP32 accumulation. The diagonal
 * (e_a+e_b) x term is always applied in FP64. */
typedef enum { PPRPA_FP64 = 0, PPRPA_FP32 = 1, PPRPA_BF16X6 = 2, PPRPA_BF16X3 = 3 } pprpa_prec;

typedef struct pprpa_ctx pprpa_ctx; /* opaque; owns every device allocation it makes */

typedef struct {
  int32_t nmo;          /* number of MO (full space)                                        */
  int32_t nocc;         /* occupied count (full space); 0 <= nocc <= nmo                    */
  int32_t naux;         /* auxiliary (density-fitting) count, > 0                           */
  int32_t nocc_act;     /* active occupied (<= 0: all)                                      */
  int32_t nvir_act;     /* active virtual  (<= 0: all)                                      */
  const double* eps;    /* [nmo] orbital energies (host or device, see on_device), ascending
                           within the occupied and the virtual block, HOMO below LUMO         */
  const double* Lpq;    /* [naux][nmo][nmo] row-major, symmetric in (p,q); or, when
                           lpq_is_active, [naux][nact][nact] over the active orbitals in
                           physical order (nact = no + nv). FP64. Host or device.           */
  int32_t lpq_is_active;
  int32_t on_device;    /* 1: eps and Lpq are device pointers                               */
  int32_t mult;         /* pprpa_mult                                                        */
  int32_t prec;         /* pprpa_prec                                                        */
  int32_t dense;        /* 1: also build the dense matrix M on the device (small systems)   */
  int32_t max_block;    /* largest k passed to pprpa_matvec / Davidson block (<= 0: 32)     */
  void* stream;         /* hipStream_t to order work on, or NULL (library-owned stream)     */
} pprpa_build_args;

/* Stage the problem on the current device: slice the active window, reorder L into the
 * sigma kernels' padded layout in the chosen precision, tabulate pair energies, and (dense=1)
 * build M. Copies everything it needs: no caller pointer is retained after return.
 * Errors: EINVAL (sizes, window outside the spaces, non-finite eps/L, eps not ascending within
 * the occupied or the virtual block or the highest occupied energy not below the lowest virtual
 * one, nv or no = 0 with no pairs), ENOMEM, EDEVICE. On error *out is set to NULL. */
pprpa_status pprpa_build(const pprpa_build_args* args, pprpa_ctx** out);

/* Spin-unrestricted ppRPA (section "Implementation Details": the matrix is built and
 * diagonalised in three spin subspaces). The alpha-alpha and beta-beta sectors carry the triplet
 * elements of one spin's orbitals and integrals: build them with pprpa_build (mult = TRIPLET) on
 * that spin's eps, nocc and Lpq. The alpha-beta sector, pairs (a_alpha, b_beta) and
 * (i_alpha, j_beta) of every combination with the alpha index outer,
 *   A = d(e^a_a + e^b_b) + (ac|bd),  B = (ai|bj),  C = -d(e^a_i + e^b_j) + (ik|jl),
 * (pq|rs) = sum_P La^P_pq Lb^P_rs, no exchange term, is built here as an FP64 context, either
 *  - dense (density_fitted = 0): M is built on the device and sigma = M z; pprpa_dims,
 *    pprpa_matvec, pprpa_davidson (Davidson or direct, both channels), pprpa_dense_matrix and
 *    pprpa_correlation_energy apply; order n = nvir_a nvir_b + nocc_a nocc_b <= 32768; or
 *  - density fitted (density_fitted = 1): both spins' integrals are staged and sigma is
 *    Q = sum_P La^P Z Lb^P with Z = blockdiag(X, Y) the rectangular amplitude blocks (alpha rows,
 *    beta columns), sigma_x = (e^a_a + e^b_b) x + Q_vv, sigma_y = -(e^a_i + e^b_j) y + Q_oo; no
 *    matrix is formed, so the order is limited by memory only (nvir, nocc < 65536);
 *    pprpa_dims, pprpa_matvec and pprpa_davidson (Davidson, both channels) apply, the direct
 *    solve, pprpa_dense_matrix and pprpa_correlation_energy return EUNSUPPORTED.
 * The density-fitted form also takes FP32 and BF16-split sigma (prec). pprpa_nto takes both
 * forms (rectangular amplitude blocks, see there). 2 mu = (e^a_HOMO + e^b_HOMO + e^a_LUMO + e^b_LUMO) / 2. Inputs (host, or device with on_device) are read during the call only.
 * Errors: EINVAL (arguments, non-finite input, energies of a spin not ascending within its
 * occupied or virtual block or its HOMO not below its LUMO), ENOMEM, EDEVICE. */
typedef struct {
  int32_t nmo;          /* orbitals per spin                                                 */
  int32_t nocc_a;       /* occupied alpha orbitals (< nmo)                                   */
  int32_t nocc_b;       /* occupied beta orbitals (< nmo)                                    */
  int32_t naux;
  const double* eps_a;  /* [nmo] alpha orbital energies (occupied first)                     */
  const double* eps_b;  /* [nmo] beta orbital energies                                       */
  const double* Lpq_a;  /* [naux][nmo][nmo] alpha MO three-centre integrals, symmetric in pq */
  const double* Lpq_b;  /* [naux][nmo][nmo] beta                                             */
  int32_t on_device;
  int32_t max_block;    /* largest sigma block per call (<= 0: 32, at most 64)               */
  void* stream;         /* hipStream_t to run on, or NULL for a new non-blocking stream      */
  int32_t density_fitted; /* 1: density-fitted sigma (no dense matrix); 0: dense context     */
  int32_t prec;         /* pprpa_prec, the sigma precision: PPRPA_FP64; density fitted only: PPRPA_FP32
                           (integrals and amplitudes in FP32, FP32 MFMA accumulation) or
                           PPRPA_BF16X6 / PPRPA_BF16X3 (three BF16 planes each, six or three
                           plane products on the BF16 MFMA, FP32 accumulation); the epilogue
                           and every Davidson step in FP64. A dense context with any
                           precision but FP64 is EUNSUPPORTED                                */
} pprpa_build_ab_args;
pprpa_status pprpa_build_ab(const pprpa_build_ab_args* args, pprpa_ctx** out);

/* Packed dimensions of the context: n_pp (virtual pairs) and n_hh (occupied pairs). */
pprpa_status pprpa_dims(const pprpa_ctx* ctx, int64_t* n_pp, int64_t* n_hh);

/* sigma = M z for k packed vectors (the density-fitted product of the method: the A, B, B^T
 * and C blocks of Eq. eigen_equation applied without forming M).
 * z, sigma: [k][n] FP64, host or device (on_device). 1 <= k <= max_block.
 * Errors: EINVAL, EDEVICE, EBUSY. */
pprpa_status pprpa_matvec(pprpa_ctx* ctx, int32_t k, const double* z, double* sigma,
                          int32_t on_device);

/* The dense ppRPA matrix M = [[A, B], [B^T, C]] (requires dense=1 at build): [n][n] row-major
 * FP64, host or device. Errors: EUNSUPPORTED (no dense build), EINVAL, EDEVICE. */
pprpa_status pprpa_dense_matrix(pprpa_ctx* ctx, double* M, int32_t on_device);

typedef struct {
  int32_t nroot;        /* number of roots wanted (>= 1)                                    */
  int32_t block;        /* max correction vectors added per iteration (<= 0: nroot)         */
  int32_t max_iter;     /* iteration cap (<= 0: 100)                                        */
  int32_t max_subspace; /* subspace size that triggers a restart (<= 0: automatic,
                           max(8 nroot, nroot + 4 block); at most 256). A restart keeps the
                           wanted Ritz vectors only, so a cap close to nroot + block can stall
                           (reported as ENOCONV with the last iterate)                        */
  double tol;           /* converged when ||M z - Omega W z||_2 <= tol for every root       */
  const double* guess;  /* optional [nguess][n] FP64 host start vectors, or NULL             */
  int32_t nguess;
  int32_t direct;       /* 1: dense direct diagonalisation (requires dense=1 at build)     */
  void (*log)(void* user, const char* json_line); /* optional per-iteration log            */
  void* user;
  int32_t channel;      /* 0: pp, two-electron addition roots (Omega > 2 mu, X^T X - Y^T Y = +1);
                         * 1: hh, two-electron removal roots (Omega < 2 mu, X^T X - Y^T Y = -1),
                         * section "ppRPA Equation", Eq. xy_norm. Other values: EINVAL.       */
} pprpa_davidson_args;

typedef struct {
  int32_t iters;        /* Davidson iterations done                                        */
  int32_t n_sigma;      /* single-vector sigma products computed                           */
  int32_t n_conv;       /* roots with residual <= tol                                      */
  int32_t subspace;     /* final subspace size                                             */
  double max_resid;     /* largest residual norm of the returned roots                     */
  double t_sigma_s;     /* seconds in sigma launches (device events)                       */
  double t_total_s;     /* seconds for the whole call (host clock)                         */
} pprpa_report;

/* Lowest nroot two-electron-addition (pp) roots Omega of Eq. eigen_equation, ascending
 * (channel 0), or the nroot two-electron-removal (hh) roots nearest the gap, descending
 * (channel 1), by the block Davidson method (direct=0) or by dense diagonalisation (direct=1).
 * omega: [nroot] host. vecs: [nroot][n] host or NULL, normalised to z^T W z = +1 (pp) or -1
 * (hh). resid: [nroot] host or NULL. rep: host or NULL. Returns ENOCONV (outputs filled with
 * the last iterate) when max_iter is reached, ENONDEF if the projected pencil is not definite,
 * EUNSUPPORTED for direct without a dense build or above order 8192, EINVAL for nroot > n_pp
 * (pp) or > n_hh (hh). */
pprpa_status pprpa_davidson(pprpa_ctx* ctx, const pprpa_davidson_args* args, double* omega,
                            double* vecs, double* resid, pprpa_report* rep);

/* ppRPA correlation energy (section "Total Energy", Eq. correlation_energy) of the context's
 * spin block from the whole spectrum of the dense pencil (eigenvalues only, on the device):
 * ec_pp = sum of the pp roots - Tr A and, from the same spectrum, ec_hh = -(sum of the hh
 * roots) - Tr C; the two agree by the sum rule of the method, their difference measures the
 * eigenvalue accuracy. For a closed shell the total is E(singlet) + 3 E(triplet).
 * Requires dense=1 at build and n <= 8192 (else EUNSUPPORTED). ENONDEF if M - 2 mu W is not
 * positive definite or the spectrum does not split into n_pp pp and n_hh hh roots (out is
 * still filled in the latter case). The call allocates 3 n^2 doubles of device scratch. */
typedef struct {
  double ec_pp;         /* sum(Omega_pp) - Tr A                                             */
  double ec_hh;         /* -sum(Omega_hh) - Tr C                                            */
  double trace_a, trace_c;
  int32_t n_pp_roots, n_hh_roots;
} pprpa_corr_energy;
pprpa_status pprpa_correlation_energy(pprpa_ctx* ctx, pprpa_corr_energy* out);

/* pprpa_correlation_energy for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same solve and the same
 * results, bit for bit, with its workspace in a static device array of the library (3 * 512^2 + 32
 * doubles, about 6 MiB, held by each device the library runs on until the process ends) instead
 * of a hipMalloc per call. Order n <= 512 (EUNSUPPORTED beyond; pprpa_correlation_energy goes
 * to 8192).
 * Every call on one device shares that array: calls that overlap on one device race and must be
 * serialised by the caller. Errors as pprpa_correlation_energy, plus EDEVICE if the array's
 * device address cannot be obtained. */
pprpa_status pprpa_correlation_energy_noalloc(pprpa_ctx* ctx, pprpa_corr_energy* out);

/* Natural transition orbital weights (section "Natural Transition Orbital", Eqs. nto_pp and
 * nto_hh) and the two-electron part of the one-particle density matrix (section "Density
 * Matrix") of k roots z ([k][n] packed FP64, host or device per on_device, e.g. the vectors of
 * pprpa_davidson). The amplitudes of each root are placed on the upper triangle of an nv x nv
 * matrix X (pp pairs) and an no x no matrix Y (hh pairs), nv and no being the active window's;
 * lam_p [k][nv] and lam_h [k][no] (host) receive the squared singular values of X and Y,
 * descending (sum lam_p - sum lam_h = z^T W z = +1 for a pp root, -1 for an hh root);
 * d_vv [k][nv][nv] = X X^T + X^T X and d_oo [k][no][no] = -(Y Y^T + Y^T Y) (host, may be NULL;
 * trace of the pair = +-2). 1 <= k <= 64, nv, no <= 512 (else EINVAL / EUNSUPPORTED). The call
 * allocates its device scratch (about 3 k (nv^2 + no^2) doubles) and frees it before returning.
 * On an alpha-beta context (dense or density fitted) the amplitude blocks are rectangular: X is
 * nvir_a x nvir_b and Y nocc_a x nocc_b (the packed order, alpha index outer); lam_p [k][nvir_a]
 * and lam_h [k][nocc_a] receive the eigenvalues of X X^T and Y Y^T (the squared singular values,
 * then zeros where the alpha side is the longer), d_vv [k][nvir_a^2 + nvir_b^2] the alpha block
 * X X^T followed by the beta block X^T X, and d_oo [k][nocc_a^2 + nocc_b^2] = -(Y Y^T, Y^T Y)
 * (one electron of each spin: each spin's trace is x^T x, or -y^T y); every block <= 512. */
pprpa_status pprpa_nto(pprpa_ctx* ctx, int32_t k, const double* z, int32_t on_device,
                       double* lam_p, double* lam_h, double* d_vv, double* d_oo);

/* The natural transition orbitals themselves (section "Natural Transition Orbital", Eqs. nto_pp
 * and nto_hh): for each of k roots z (as pprpa_nto), the leading nvec singular-vector pairs of its
 * amplitude matrices, X = C^p1 sqrt(lam^p) C^p2^T and Y = C^h1 sqrt(lam^h) C^h2^T, in the order
 * of pprpa_nto's weights (descending). X and Y are those of pprpa_nto: the triangular nv x nv and
 * no x no matrices of a restricted context, the rectangular nvir_a x nvir_b and nocc_a x nocc_b
 * blocks of an alpha-beta one. Outputs (host, each may be NULL), one vector per row:
 * c_p1 [k][nvec][rows of X], c_p2 [k][nvec][columns of X], c_h1 [k][nvec][rows of Y],
 * c_h2 [k][nvec][columns of Y]. The right vectors are eigenvectors of X^T X (Householder
 * tridiagonal form, bisection, inverse iteration), the left ones u = X v / |X v|; each pair's
 * sign is fixed so that the largest |u_i| (lowest i among equals) is positive; rows beyond
 * min(nvec, rows, columns), and u of a null direction (|X v| <= 1e-10 of the first), are zero.
 * Vectors of equal weights are an orthonormal basis of their subspace, not unique. 1 <= k <= 64,
 * 1 <= nvec <= 64, blocks <= 512 (else EINVAL / EUNSUPPORTED). Allocates and frees its device
 * scratch. Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, EBUSY. */
pprpa_status pprpa_nto_vectors(pprpa_ctx* ctx, int32_t k, const double* z, int32_t on_device,
                               int32_t nvec, double* c_p1, double* c_p2, double* c_h1,
                               double* c_h2);

/* Timing of the sigma contraction kernel (the fused sandwich kernel only, without the unpack
 * and epilogue kernels), measured with HIP events recorded on the context's stream around
 * every launch since the last reset. flops and bytes are algorithmic counts: per vector
 * 4 naux (nv + no) (nv^2 + no^2) flops; per launch the staged integrals once plus the packed
 * input and output vectors. */
typedef struct {
  int64_t launches;
  double seconds;
  double flops;
  double bytes;
} pprpa_kernel_stats;
pprpa_status pprpa_sigma_stats(pprpa_ctx* ctx, pprpa_kernel_stats* out, int32_t reset);

/* The Davidson solve of pprpa_davidson advanced by the caller, a few iterations at a time (for
 * callers that interleave the solve with other work, time it per iteration, or stop it early).
 * An iteration is the sigma product of the pending block of trial vectors (the density-fitted
 * product of Eq. eigen_equation), the Rayleigh-Ritz step on the projected pencil, the residuals
 * and the new correction vectors; iterations run exactly as in pprpa_davidson, so a solve driven
 * to convergence here returns bitwise what pprpa_davidson returns for the same arguments.
 *
 * pprpa_solve_begin: validate args (as pprpa_davidson; direct = 1 is EUNSUPPORTED), take the
 *   workspace and form the initial subspace. The solve holds the context until
 *   pprpa_solve_end: other calls on the context return EBUSY, and the context must not be freed
 *   before the solve is ended. Errors: EINVAL, EUNSUPPORTED, EBUSY, ENOMEM, EDEVICE (nothing
 *   is held and *out is NULL).
 * pprpa_solve_iterate: run up to n_iter (>= 0) iterations; *iters_done (may be NULL) receives
 *   the number run and *done (may be NULL) 1 once the solve has finished (converged, failed,
 *   or reached max_iter). Errors: EINVAL, EDEVICE (the solve is then finished).
 * pprpa_solve_end: the outputs of pprpa_davidson (omega [nroot] host or NULL, vecs [nroot][n]
 *   host or NULL, resid [nroot] host or NULL, rep or NULL) and its status: OK when converged, ENOCONV
 *   when the solve was ended before convergence or reached max_iter (outputs from the last
 *   iterate; omega and resid are left untouched if no iteration ran), ENONDEF and the other
 *   failures as pprpa_davidson. Releases the solve and its hold on the context in every case. */
typedef struct pprpa_solve pprpa_solve; /* opaque */
pprpa_status pprpa_solve_begin(pprpa_ctx* ctx, const pprpa_davidson_args* args,
                               pprpa_solve** out);
pprpa_status pprpa_solve_iterate(pprpa_solve* solve, int32_t n_iter, int32_t* iters_done,
                                 int32_t* done);
pprpa_status pprpa_solve_end(pprpa_solve* solve, double* omega, double* vecs, double* resid,
                             pprpa_report* rep);
/* pprpa_sigma_stats of the solve's context while the solve holds it (same counters, same reset). */
pprpa_status pprpa_solve_stats(pprpa_solve* solve, pprpa_kernel_stats* out, int32_t reset);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching of many independent solves on the current device.
 *
 * The method's cost is dominated by the sigma products of the Davidson iterations (section
 * "Implementation Details"); a server keeps many solves resident and overlaps them: requests
 * are admitted in arrival order when their device footprint (staged integrals, sigma buffers,
 * Davidson workspace; computed exactly at submit) fits in the server's HBM arena and one of
 * max_inflight slots is free; every in-flight solve advances independently on its own stream,
 * and the sigma products of all solves that need one at the same time run as one grouped grid.
 * A request's arithmetic is the same as pprpa_build + pprpa_davidson with the same arguments
 * (same kernels and decomposition), so its roots do not depend on what it was served with.
 * Threads: an admission thread (builds) and a worker thread (phases, grouped launches); the
 * Davidson log callback, if any, is called from the worker thread.
 * --------------------------------------------------------------------------------------- */
typedef struct pprpa_server pprpa_server; /* opaque */

typedef struct {
  int32_t state;        /* 0 queued, 1 running (the caller's inputs are no longer read), 2 done */
  int32_t status;       /* pprpa_status of the solve (meaningful once done)                  */
  int32_t nroot;
  int32_t max_overtaken; /* the most times the grouped sigma launches of another kernel
                            variant (the sigma precision, and for FP64 the kernel chosen by the
                            size of the virtual block) went ahead of one of this request's
                            waiting sigma blocks; the variant of the longest-waiting block goes
                            first, so this is at most 4 (one per other variant)               */
  double t_submit;      /* seconds on the server's steady clock (0 = creation)               */
  double t_admit;       /* reservation taken, build started                                  */
  double t_done;        /* roots copied out, memory released                                 */
  uint64_t footprint;   /* device bytes reserved for the request                             */
  char message[256];    /* error text when status != OK                                     */
} pprpa_request_info;

typedef struct {
  int64_t submitted, completed, failed;   /* requests                                         */
  int64_t queued, inflight, peak_inflight;
  uint64_t budget;                         /* arena bytes                                      */
  uint64_t reserved, peak_reserved;        /* bytes held by admitted requests (now, highest)   */
  int64_t group_launches;                  /* grouped sigma grids launched (and timed)         */
  int64_t grouped_products;                /* block sigma products they carried                */
  double sigma_seconds;                    /* device time of those grids (HIP events)          */
  double sigma_flops;                      /* their algorithmic flops (as pprpa_kernel_stats)  */
} pprpa_serving_stats;

/* Reserve hbm_budget_bytes (>= 1 MiB) of device memory as the admission arena, max_inflight
 * (1..64) slots (a stream and a pinned status buffer each), and start the server's threads.
 * Errors: EINVAL, ENOMEM (the arena cannot be allocated), EDEVICE. */
pprpa_status pprpa_server_create(size_t hbm_budget_bytes, int32_t max_inflight,
                                 pprpa_server** out);

/* Queue one solve: the problem as for pprpa_build (any prec; dense, stream and max_block are
 * chosen by the server) and the Davidson arguments (direct = 0). The memory
 * that args point to (eps, Lpq, guess) must stay valid and unchanged until pprpa_server_poll
 * reports state >= 1; device inputs must be complete (their producer synchronised) before the
 * call. Errors (nothing queued): EINVAL, EUNSUPPORTED (direct). A request larger than
 * the whole arena is accepted and finishes with ENOMEM. */
pprpa_status pprpa_server_submit(pprpa_server* srv, const pprpa_build_args* build,
                                 const pprpa_davidson_args* dav, uint64_t* ticket);

/* State of a request. Once done (info->state == 2) the roots ([nroot] host, ascending), residual
 * norms and report are copied out as pprpa_davidson would return them (omega, resid, rep may
 * be NULL) and the ticket is retired: polling it again is EINVAL. */
pprpa_status pprpa_server_poll(pprpa_server* srv, uint64_t ticket, pprpa_request_info* info,
                               double* omega, double* resid, pprpa_report* rep);

/* Block until the request is done (timeout_s < 0: no limit). EBUSY on timeout, EINVAL for an
 * unknown ticket. */
pprpa_status pprpa_server_wait(pprpa_server* srv, uint64_t ticket, double timeout_s);

pprpa_status pprpa_server_stats(pprpa_server* srv, pprpa_serving_stats* out);

/* Finish the in-flight solves, fail the queued ones with EBUSY, release everything. NULL-safe. */
void pprpa_server_destroy(pprpa_server* srv);

/* Release the context and all its device memory. NULL-safe. */
void pprpa_free(pprpa_ctx* ctx);

const char* pprpa_strerror(pprpa_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char* pprpa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PPRPA_H */
