// Internal declarations shared by the host side (api.cpp, davidson.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pprpa.h"

namespace pprpa {

void set_error(const char* fmt, ...);

#define PPRPA_HIP(expr)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      ::pprpa::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,    \
                         __LINE__);                                                          \
      return PPRPA_EDEVICE;                                                                  \
    }                                                                                        \
  } while (0)

// Named roctx range for the lifetime of the object (host-side phase markers for rocprofv3
// --marker-trace); a no-op unless PPRPA_ROCTX=1 is set and the roctx library opens.
class TraceRange {
 public:
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;

 private:
  bool on_;
};
bool trace_enabled();

#define PPRPA_TRY(expr)                   \
  do {                                    \
    pprpa_status s_ = (expr);             \
    if (s_ != PPRPA_OK) return s_;        \
  } while (0)

// Tiles of the sigma kernels are 16 x 16 (one MFMA output tile).
constexpr int TILE = 16;
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Geometry of the padded orbital layout used by the sigma kernels: virtual block first
// (rows/cols [0, nvp)), then the occupied block ([nvp, nvp + nop)); each block padded with
// zeros to a multiple of 16.
struct Geometry {
  int nv = 0, no = 0, naux = 0;
  int nvp = 0, nop = 0, nmop = 0;
  int nvt = 0, nct = 0;  // tiles in the virtual block; tiles in total
  int mult = 0;          // 0 singlet, 1 triplet
  int64_t nvv = 0, noo = 0, n = 0;
};

// A served context's device memory: one contiguous reservation, handed out by bumping `top`
// (nothing is freed until the whole reservation is released).
struct Slab {
  char* base = nullptr;
  size_t size = 0, top = 0;
};

// Sigma precision and storage type.
enum class Store { F64, F32, BF16 };

// Arguments of one sigma launch.
struct SigmaLaunch {
  const void* L;     // staged integrals
  const void* ZT;    // unpacked transposed vectors [kcap][nmop][nmop]
  void* Sp;          // partial sums [nsplit][k][nmop][nmop]
  int k;             // vectors in the block
  int nsplit;        // aux-index splits
  int npan_v, npan_o;
  size_t plane;      // elements per bf16 plane of L (BF16 only)
  size_t zplane;     // elements per bf16 plane of ZT (BF16 only)
  int nprod;         // 3 or 6 (BF16 only)
};

// Sigma launch plan (kernel variant and its work-item table), fixed per context.
struct SigmaPlan {
  int variant = 0;
  int RT = 16;
  int nitems = 0;
  int npan_v = 0;
  int* d_items = nullptr;
};
// Work items (panel index << 16 | first row tile): panels of pw adjacent column tiles of one
// diagonal block, row ranges of RT tiles.
void make_sigma_items(const Geometry& g, int RT, std::vector<int>& items, int& npan_v, int pw = 4);
// Column tiles per panel of a sigma kernel variant.
inline int panel_width(int variant) { return variant == 7 ? 8 : 4; }
constexpr int UNITS_F64 = 16384;      // work units per launch of the pipelined FP64 kernel
constexpr int F64_PIPE_MIN_NVT = 20;  // virtual 16-tiles from which FP64 sigma uses that kernel
constexpr int BF16_WIDE_MIN_NVT = 32;  // the same for the wide-panel BF16x6 kernel
// Largest order of the dense pencil solves on the device (the direct diagonalisation and the
// whole-spectrum solve of the correlation energy), and the largest order solved by one
// workgroup (many workgroups above).
constexpr int DENSE_SOLVE_MAX = 8192;
constexpr int DENSE_ENERGY_MAX = 8192;
constexpr int DENSE_ONE_WG_MAX = 96;
int sigma_variant(const Geometry& g, Store st, int nprod, int* RT);

// --- kernel launchers (k_sigma.hip) -------------------------------------------------------
hipError_t launch_stage_L(const Geometry& g, Store st, const double* Lin, int nin, int p0, int np,
                          const int* d_src, void* Lout, size_t plane, int* d_bad,
                          hipStream_t s);
hipError_t launch_unpack(const Geometry& g, Store st, const double* z, int k, const int* d_ptab,
                         void* ZT, size_t zplane, hipStream_t s);
hipError_t launch_sigma(const Geometry& g, Store st, const SigmaPlan& plan, const SigmaLaunch& a,
                        hipStream_t s);
// Up to GROUP_MAX sigma products of the same kernel variant in one launch (serving).
constexpr int GROUP_MAX = 16;
struct GroupMember {
  const Geometry* g;
  const SigmaPlan* plan;
  SigmaLaunch la;
};
hipError_t launch_sigma_group(const GroupMember* m, int n, hipStream_t s);
hipError_t launch_epilogue(const Geometry& g, Store st, const double* z, int k, const void* Sp,
                           int nsplit, const int* d_ptab, const double* d_epair, double* sigma,
                           hipStream_t s);
hipError_t launch_check_finite(const double* x, size_t n, int* d_bad, hipStream_t s);

// Alpha-beta sector of unrestricted ppRPA, density fitted: each spin's orbitals in the padded
// [virtual; occupied] layout of the sigma kernels (alpha: rows and c; beta: d and columns).
struct AbGeometry {
  int nva = 0, noa = 0, nvb = 0, nob = 0, naux = 0;
  int nvpa = 0, nopa = 0, nmopa = 0, nvta = 0, ncta = 0;
  int nvpb = 0, nopb = 0, nmopb = 0, nvtb = 0, nctb = 0;
  int64_t nvv = 0, noo = 0, n = 0;
};
// Kernel arguments of one alpha-beta sigma launch.
struct AbParams {
  int nvta, ncta, nvtb, nctb, nvpa, nvpb, nmopa, nmopb, naux;
  int k, nsplit, nitems, nunits, per_xcd, npan_v;
  const int* items;  // [nitems]: beta panel index << 16 | first alpha row tile of the range
  int64_t la_stride, lb_stride, zt_stride, q_stride;
};
void make_sigma_items_ab(const AbGeometry& g, std::vector<int>& items, int& npan_v);
// The packed alpha-beta vectors z [k][n] (device) unpacked in the sigma precision st: Z^T[kv][d][c]
// for FP64 and FP32, Z[kv][c][d] as three BF16 planes zplane elements apart for BF16.
hipError_t launch_unpack_ab(const AbGeometry& g, Store st, const double* z, int k, void* ZT,
                            size_t zplane, hipStream_t s);
// Partial Q = sum_P La^P Z Lb^P per aux split: Qp [nsplit][k][nmopa][nmopb], in precision st (FP32
// for BF16, whose nprod = 6 or 3 products; La, Lb then three planes of naux nmop^2 each).
hipError_t launch_sigma_ab(const AbGeometry& g, Store st, int nprod, const SigmaPlan& plan,
                           const void* La, const void* Lb, const void* ZT, size_t zplane, void* Qp,
                           int k, int nsplit, hipStream_t s);
// sigma [k][n] = epair * z + the split sums of Qp (fixed order, FP64).
hipError_t launch_epilogue_ab(const AbGeometry& g, Store st, const double* z, int k,
                              const void* Qp, int nsplit, const double* epair, double* sigma,
                              hipStream_t s);

// --- dense (k_dense.hip) -------------------------------------------------------------------
hipError_t launch_dense_build(const Geometry& g, const double* L64, const int* d_ptab,
                              const double* d_epair, double* M, hipStream_t s);
// Alpha-beta sector of unrestricted ppRPA as a dense matrix (La, Lb: full [naux][nmo][nmo]
// FP64 integrals of each spin on the device), and sigma = M z for k vectors of a dense matrix.
hipError_t launch_dense_build_ab(const double* La, const double* Lb, int naux, int nmo, int nocc_a,
                                 int nocc_b, int64_t n, int64_t nvv, const int* d_ptab,
                                 const double* d_epair, double* M, hipStream_t s);
hipError_t launch_dense_sigma(const double* M, int64_t n, const double* z, int k, double* sigma,
                              hipStream_t s);
hipError_t launch_epair(const Geometry& g, const int* d_ptab, const double* d_ev,
                        const double* d_eo, double* d_epair, hipStream_t s);
hipError_t launch_set_units(double* V, int64_t ld, const int64_t* idx, int r, hipStream_t s);
hipError_t launch_metric_matrix(double* W, int64_t n, int64_t nvv, hipStream_t s);
hipError_t launch_transpose(const double* in, int ldi, int m, int r, double* out, int64_t ldo,
                            hipStream_t s);

// --- FP64 linear algebra (k_linalg.hip) ----------------------------------------------------
// C[i][j] (ldc) = sum_t A[i][t] * w(t) * B[j][t], i < ma, j < mb; w(t) = -1 for t >= nsplit_w
// when signed != 0. A: [ma][n] (lda), B: [mb][n] (ldb). Uses partial buffer `part` of
// nchunk * ma * mb doubles.
hipError_t launch_dots(const double* A, int64_t lda, int ma, const double* B, int64_t ldb, int mb,
                       int64_t n, int64_t nsign, int signed_w, double* C, int ldc, double* part,
                       int nchunk, hipStream_t s);
// Y[j][t] (ldy) = beta * Y[j][t] + alpha * sum_i Cm[i][j] X[i][t], i < m, j < r.
// Cm: [m][ldcm] device, r <= ldcm (any r: one launch per 64 rows of Y).
hipError_t launch_combine(const double* X, int64_t ldx, int m, const double* Cm, int ldcm, int r,
                          int64_t n, double alpha, double beta, double* Y, int64_t ldy,
                          hipStream_t s);
// Residual + norms + preconditioner for r roots.
hipError_t launch_residual(const double* Z, const double* SZ, int64_t ld, int r, int64_t n,
                           int64_t nvv, const double* d_omega, double* R, double* part_norm,
                           int nchunk, hipStream_t s);
hipError_t launch_reduce_norms(const double* part, int nchunk, int r, double* out, hipStream_t s);
hipError_t launch_precond(const double* R, int64_t ld, const int* h_sel, int nsel, int64_t n,
                          int64_t nvv, const double* d_diag, const double* d_omega, double* T,
                          int64_t ldt, hipStream_t s);
// Pencil solve on one workgroup: K = Ms - 2 mu Ws = R R^T, G = R^-1 Ws R^-T = U diag(theta) U^T
// (Householder tridiagonalisation, bisection, inverse iteration), Omega = 2 mu + 1/theta; returns
// the nroot wanted roots of the channel and coefficient columns Cout[m][ldc] with c^T Ws c = +1
// (pp) or -1 (hh); columns
// nroot..nret-1 hold the next Ritz vectors (kept on restart). Ms, Ws: upper triangles (ld ldm).
// m <= 512, nroot <= nret <= m. channel 0 (pp): the largest theta, roots ascending in Omega;
// channel 1 (hh): the smallest theta, the hh roots nearest 2 mu first (Omega descending).
// work: m^2 + 4 nret m doubles (m <= 96, matrices in LDS) or 3 m^2 + 4 nret m (larger m).
// info: [0] status (0 ok, 1 not definite, 2 fewer than nroot roots of the channel), [1] number
// of roots of the channel, [2] 0.
hipError_t launch_pencil(const double* Ms, const double* Ws, int ldm, int m, double mu2,
                         int nroot, int nret, int channel, double* omega, double* Cout, int ldc,
                         double* work, int* info, hipStream_t s);
// Whole spectrum of the dense pencil (M, W) for m <= DENSE_ONE_WG_MAX (eigenvalues only): out[0] =
// sum of the pp roots - Tr A, out[1] = -(sum of the hh roots) - Tr C, out[2] = Tr A, out[3] = Tr C;
// info: [0] 0 ok / 1 not definite, [1] pp roots, [2] hh roots. work: 3 m^2 doubles.
hipError_t launch_pencil_energy(const double* M, int m, int64_t nvv, double mu2, double* out,
                                double* work, int* info, hipStream_t s);
// The same outputs as launch_pencil_energy for 2 <= m <= DENSE_ENERGY_MAX on many workgroups
// (blocked Cholesky, S = L^T W L, Householder tridiagonal form, bisection; k_dense_mw.hip).
// work: pencil_energy_mw_work(m) doubles.
size_t pencil_energy_mw_work(int n);
hipError_t launch_pencil_energy_mw(const double* M, int m, int64_t nvv, double mu2, double* out,
                                   double* work, int* info, hipStream_t s);
// Direct solve of the dense pencil (M, W), W = diag(+1 for i < nvv, -1), for 3 <= m <=
// DENSE_SOLVE_MAX on many workgroups (the chain of launch_pencil_energy_mw keeping its
// reflections, multisection for the wanted eigenvalues, inverse iteration, back-transformation,
// L^T z = u): the outputs of launch_pencil (nret = nroot). work: direct_pencil_mw_work(m, nroot)
// doubles.
size_t direct_pencil_mw_work(int n, int nroot);
hipError_t launch_direct_pencil_mw(const double* M, int m, int64_t nvv, double mu2, int nroot,
                                   int channel, double* omega, double* Cout, int ldc,
                                   double* work, int* info, hipStream_t s);
// NTO weights and two-electron density blocks of k packed roots Z [k][ldz] (nv, no <= 512):
// X [k][nv][nv], Y [k][no][no] (triangular amplitude matrices), Gx, Gy (their T^T T, destroyed),
// Dv = X X^T + X^T X, Do = -(Y Y^T + Y^T Y) (may be null), lam_p [k][nv], lam_h [k][no]
// (squared singular values, descending).
hipError_t launch_nto(const double* Z, int64_t ldz, int k, const Geometry& g, const int* ptab,
                      double* X, double* Y, double* Gx, double* Gy, double* Dv, double* Do,
                      double* lam_p, double* lam_h, hipStream_t s);
// The same for k packed alpha-beta roots: X = nva x nvb and Y = noa x nob read in place from Z
// (alpha index outer); Gx = X X^T [k][nva][nva], Gy = Y Y^T (destroyed); Dv [k][nva^2 + nvb^2]
// = (X X^T, X^T X), Do [k][noa^2 + nob^2] = -(Y Y^T, Y^T Y) (may be null); lam_p [k][nva],
// lam_h [k][noa] (eigenvalues of X X^T and Y Y^T, descending, clamped at zero). All <= 512.
hipError_t launch_nto_ab(const double* Z, int64_t ldz, int k, int nva, int nvb, int noa, int nob,
                         double* Gx, double* Gy, double* Dv, double* Do, double* lam_p,
                         double* lam_h, hipStream_t s);
// The packed roots' triangular amplitude matrices X [k][nv][nv], Y [k][no][no] (zeros below).
hipError_t launch_unpack_triangular(const double* Z, int64_t ldz, int k, const Geometry& g,
                                    const int* ptab, double* X, double* Y, hipStream_t s);
// Leading singular vectors of k matrices A (rows x cols, row-major, astride apart; rows, cols
// <= 512): the nsel = min(nvec, rows, cols) right vectors from the largest eigenvalues of A^T A,
// the left ones u = A v / |A v|, signs fixed (largest |u_i| positive); U [k][nvec][rows] and
// V [k][nvec][cols] (rows beyond nsel, and u of a null direction, zero). 1 <= nvec <= 64.
// work: svd_vectors_work(k, rows, cols, nvec) doubles.
size_t svd_vectors_work(int k, int rows, int cols, int nvec);
hipError_t launch_svd_vectors(const double* A, int64_t astride, int rows, int cols, int k,
                              int nvec, double* work, double* U, double* V, hipStream_t s);
hipError_t launch_normalize_rows(double* V, int64_t ld, int r, int64_t n, hipStream_t s);
hipError_t prepare_kernels();
// Small orthonormalisation in the m-dim subspace (one workgroup): Q = orth(C) by MGS.
hipError_t launch_small_orth(const double* C, int ldc, int m, int r, double* Q, int ldq,
                             int* rank, hipStream_t s);
// Ms_new = Q^T Ms Q (r x r), one workgroup.
hipError_t launch_small_congruence(const double* Ms, int ldm, int m, const double* Q, int ldq,
                                   int r, double* out, int ldo, double* work, hipStream_t s);
// Orthonormal basis of block T (b x n) against itself (symmetric orthonormalisation from its
// Gram matrix with eigenvalue cut). Produces Tmat (b x b, rows = combos) and count kept.
hipError_t launch_gram_orth(const double* G, int ldg, int b, double cut, double* Tm, int ldt,
                            int* kept, double* work, hipStream_t s);
hipError_t launch_scale_sign(double* V, int64_t ld, int r, int64_t n, hipStream_t s);
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s);

}  // namespace pprpa
