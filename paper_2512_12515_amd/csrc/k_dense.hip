// Dense ppRPA matrix on the device (small systems; direct diagonalisation path) and the small
// device-side helpers of context set-up: pair energies, unit guess vectors, metric matrix.
//
// M = [[A, B], [B^T, C]] with the spin-adapted elements of arXiv 2512.12515, section
// "ppRPA Equation" (<pq|rs> = (pr|qs), (pq|rs) = sum_P L^P_pq L^P_rs):
//   A_ab,cd = d(e_a + e_b) + N_ab N_cd [(ac|bd) + s (ad|bc)]
//   B_ab,kl =               N_ab N_kl [(ak|bl) + s (al|bk)]
//   C_ij,kl = -d(e_i + e_j) + N_ij N_kl [(ik|jl) + s (il|jk)]
// s = +1 and N = 1/sqrt(1 + delta) for the singlet; s = -1 and N = 1 for the triplet.
#include "internal.h"

namespace pprpa {
namespace {

// One thread per matrix element; the aux sum runs over the staged FP64 integrals in the padded
// layout (virtual orbital a at padded index a, occupied i at nvp + i).
__global__ __launch_bounds__(256) void k_dense_build(const double* __restrict__ L, int naux,
                                                     int nmop, int nvp, int64_t n, int64_t nvv,
                                                     int mult, const int* __restrict__ ptab,
                                                     const double* __restrict__ epair,
                                                     double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e / n, c = e % n;
  const int pr = ptab[r], pc = ptab[c];
  const int p = (pr >> 16) + (r < nvv ? 0 : nvp), q = (pr & 0xFFFF) + (r < nvv ? 0 : nvp);
  const int u = (pc >> 16) + (c < nvv ? 0 : nvp), v = (pc & 0xFFFF) + (c < nvv ? 0 : nvp);
  const double sg = mult == 0 ? 1.0 : -1.0;
  const size_t z = (size_t)nmop * nmop;
  double direct = 0.0, exch = 0.0;
  // <pq|uv> = (pu|qv); <pq|vu> = (pv|qu)
  for (int P = 0; P < naux; ++P) {
    const double* Lp = L + P * z;
    direct += Lp[(size_t)p * nmop + u] * Lp[(size_t)q * nmop + v];
    exch += Lp[(size_t)p * nmop + v] * Lp[(size_t)q * nmop + u];
  }
  double nrm = 1.0;
  if (mult == 0) {
    if ((pr >> 16) == (pr & 0xFFFF)) nrm *= 0.70710678118654752440;
    if ((pc >> 16) == (pc & 0xFFFF)) nrm *= 0.70710678118654752440;
  }
  double val = nrm * (direct + sg * exch);
  if (r == c) val += epair[r];
  M[e] = val;
}

// Alpha-beta sector of spin-unrestricted ppRPA (section "Implementation Details": the matrix
// built and diagonalised in three spin subspaces): pair e = (p_alpha, q_beta), alpha index
// outer, virtual pairs first; M[r][c] = d_rc epair[r] + sum_P La^P[p_r][p_c] Lb^P[q_r][q_c]
// (<pq|uv> = (pu|qv); no exchange term between orbitals of different spin). La, Lb: the full
// [naux][nmo][nmo] FP64 integrals of each spin; orbital index of a virtual pair's alpha member
// nocc_a + p, of an occupied pair's p (beta likewise). One thread per element.
__global__ __launch_bounds__(256) void k_dense_build_ab(const double* __restrict__ La,
                                                        const double* __restrict__ Lb, int naux,
                                                        int nmo, int nocc_a, int nocc_b,
                                                        int64_t n, int64_t nvv,
                                                        const int* __restrict__ ptab,
                                                        const double* __restrict__ epair,
                                                        double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e / n, c = e % n;
  const int pr = ptab[r], pc = ptab[c];
  const int p = (pr >> 16) + (r < nvv ? nocc_a : 0), q = (pr & 0xFFFF) + (r < nvv ? nocc_b : 0);
  const int u = (pc >> 16) + (c < nvv ? nocc_a : 0), v = (pc & 0xFFFF) + (c < nvv ? nocc_b : 0);
  const size_t z = (size_t)nmo * nmo;
  double s = 0.0;
  for (int P = 0; P < naux; ++P)
    s += La[P * z + (size_t)p * nmo + u] * Lb[P * z + (size_t)q * nmo + v];
  if (r == c) s += epair[r];
  M[e] = s;
}

// sigma[j][t] = sum_i M[i][t] z[j][i] for j < k (M symmetric, so this is M z): one thread per t
// (column t of M read down its rows, coalesced across the threads), KB vectors per pass.
template <int KB>
__global__ __launch_bounds__(256) void k_dense_sigma(const double* __restrict__ M, int64_t n,
                                                     const double* __restrict__ z, int k,
                                                     double* __restrict__ sigma) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  for (int j0 = 0; j0 < k; j0 += KB) {
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double m = M[i * n + t];
#pragma unroll
      for (int j = 0; j < KB; ++j)
        if (j0 + j < k) acc[j] += m * z[(int64_t)(j0 + j) * n + i];
    }
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j0 + j < k) sigma[(int64_t)(j0 + j) * n + t] = acc[j];
  }
}

// epair[e] = +(e_a + e_b) for virtual pairs, -(e_i + e_j) for occupied pairs.
__global__ void k_epair(const int* __restrict__ ptab, const double* __restrict__ ev,
                        const double* __restrict__ eo, int64_t n, int64_t nvv,
                        double* __restrict__ epair) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int pq = ptab[e];
  const int p = pq >> 16, q = pq & 0xFFFF;
  epair[e] = e < nvv ? ev[p] + ev[q] : -(eo[p] + eo[q]);
}

// Rows i < r of V (ld) become unit vectors e_{idx[i]} (V zeroed beforehand).
struct IdxList {
  int64_t idx[64];
};
__global__ void k_set_units(double* __restrict__ V, int64_t ld, int r, IdxList il) {
  const int i = threadIdx.x;
  if (i < r) V[i * ld + il.idx[i]] = 1.0;
}

// W = diag(+1 (x part), -1 (y part)), n x n
__global__ void k_metric_matrix(double* __restrict__ W, int64_t n, int64_t nvv) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e / n, c = e % n;
  W[e] = r == c ? (r < nvv ? 1.0 : -1.0) : 0.0;
}

// out[j][i] = in[i][j], in: m x r (ld ldi), out: r x m (ld ldo)
__global__ void k_transpose(const double* __restrict__ in, int ldi, int m, int r,
                            double* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)m * r) return;
  const int i = (int)(e / r), j = (int)(e % r);
  out[j * ldo + i] = in[(int64_t)i * ldi + j];
}

}  // namespace

hipError_t launch_dense_build(const Geometry& g, const double* L64, const int* d_ptab,
                              const double* d_epair, double* M, hipStream_t s) {
  const int64_t e = g.n * g.n;
  hipLaunchKernelGGL(k_dense_build, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, L64,
                     g.naux, g.nmop, g.nvp, g.n, g.nvv, g.mult, d_ptab, d_epair, M);
  return hipGetLastError();
}

hipError_t launch_epair(const Geometry& g, const int* d_ptab, const double* d_ev,
                        const double* d_eo, double* d_epair, hipStream_t s) {
  hipLaunchKernelGGL(k_epair, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, d_ptab, d_ev,
                     d_eo, g.n, g.nvv, d_epair);
  return hipGetLastError();
}

hipError_t launch_set_units(double* V, int64_t ld, const int64_t* idx, int r, hipStream_t s) {
  if (r > 64) return hipErrorInvalidValue;
  IdxList il;
  for (int i = 0; i < 64; ++i) il.idx[i] = i < r ? idx[i] : 0;
  hipLaunchKernelGGL(k_set_units, dim3(1), dim3(64), 0, s, V, ld, r, il);
  return hipGetLastError();
}

hipError_t launch_metric_matrix(double* W, int64_t n, int64_t nvv, hipStream_t s) {
  hipLaunchKernelGGL(k_metric_matrix, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, W,
                     n, nvv);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* in, int ldi, int m, int r, double* out, int64_t ldo,
                            hipStream_t s) {
  const int64_t e = (int64_t)m * r;
  if (e == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, in, ldi, m,
                     r, out, ldo);
  return hipGetLastError();
}

hipError_t launch_dense_build_ab(const double* La, const double* Lb, int naux, int nmo, int nocc_a,
                                 int nocc_b, int64_t n, int64_t nvv, const int* d_ptab,
                                 const double* d_epair, double* M, hipStream_t s) {
  const int64_t nn = n * n;
  hipLaunchKernelGGL(k_dense_build_ab, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, La, Lb,
                     naux, nmo, nocc_a, nocc_b, n, nvv, d_ptab, d_epair, M);
  return hipGetLastError();
}

hipError_t launch_dense_sigma(const double* M, int64_t n, const double* z, int k, double* sigma,
                              hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_sigma<8>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, n, z,
                     k, sigma);
  return hipGetLastError();
}

}  // namespace pprpa
