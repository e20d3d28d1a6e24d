// Whole spectrum of the dense definite pencil (M, W) on many workgroups: the correlation energy of
// arXiv 2512.12515 (section "Total Energy", Eq. correlation_energy) at orders above the
// one-workgroup solver's.
//
// With 2 mu inside the gap, K = M - 2 mu W is positive definite. K z = (Omega - 2 mu) W z, so the
// eigenvalues lambda = Omega - 2 mu are those of W K = W L L^T (K = L L^T, Cholesky), which is
// similar to the symmetric S = L^T W L; lambda > 0 exactly for the pp roots (z^T K z > 0 and
// lambda z^T W z = z^T K z). The steps:
//   1. K = M - 2 mu W;
//   2. K = L L^T by the blocked right-looking Cholesky: a one-workgroup factorisation of each
//      32 x 32 diagonal block, the panel below it by forward substitution (a row per thread),
//      the trailing lower triangle updated in 32 x 32 tiles;
//   3. S = L^T W L in 32 x 32 tiles (both triangles written);
//   4. Householder reduction of S to tridiagonal form, one reflection per column: the reflection
//      vector (one workgroup), p = beta S2 v (a wave per row), then S2 -= v w^T + w v^T with
//      w = p - (beta p^T v / 2) v (every workgroup forms the dot product itself, in the same fixed
//      order);
//   5. every eigenvalue of the tridiagonal form by Sturm-count bisection (a thread per
//      eigenvalue), and the sums of the sum rule in a fixed order.
// The direct solve for the wanted roots (Eq. eigen_equation with the normalisation of Eq.
// xy_norm) runs steps 1-4 keeping the reflection vectors, then
//   5'. the wanted eigenvalues only: the Sturm count at 0 gives the number of hh roots, and
//      multisection (a workgroup per root, 256 Sturm counts per round) the j-th eigenvalue above
//      (pp) or below (hh) 0;
//   6. their eigenvectors u of the tridiagonal form by inverse iteration (a thread per root),
//      orthonormalised among nearly equal eigenvalues;
//   7. per root (a workgroup each, the vector in LDS): the reflections applied to u, then
//      L^T z = u by blocked back substitution and z scaled by sqrt|lambda|, so that
//      z^T W z = |lambda| u^T S^-1 u = sign(lambda) (S^-1 = L^-1 W L^-T).
// Every reduction runs in a fixed order: the result is bitwise repeatable.
#include "internal.h"

namespace pprpa {
namespace {

constexpr int CB = 32;  // Cholesky block and tile edge

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over the workgroup (every thread gets it); red: blockDim.x / 64 doubles of LDS
__device__ __forceinline__ double wg_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r += red[w];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double wg_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double wg_min(double v, double* red) {
  return -wg_max(-v, red);
}

// (row, col) of pair index x in the lower triangle of a t x t tile grid (row >= col)
__device__ __forceinline__ void tri_pair(int x, int* r, int* c) {
  int i = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= x) ++i;
  while (i * (i + 1) / 2 > x) --i;
  *r = i;
  *c = x - i * (i + 1) / 2;
}

__global__ void k_mw_init(int* flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

// K = M - mu2 W, mu2 = 2 mu, W = diag(+1 for i < nvv, -1)
__global__ __launch_bounds__(256) void k_mw_shift(const double* __restrict__ M, int n, int64_t nvv,
                                                  double mu2, double* __restrict__ K) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  K[e] = M[e] - (i == j ? mu2 * (i < nvv ? 1.0 : -1.0) : 0.0);
}

// Cholesky of the diagonal block at (j0, j0), b = min(CB, n - j0) rows, in place (lower); a
// non-positive pivot sets flag.
__global__ __launch_bounds__(256) void k_mw_chol_diag(double* __restrict__ K, int n, int j0,
                                                      int* __restrict__ flag) {
  __shared__ double a[CB][CB + 1];
  const int b = min(CB, n - j0);
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    a[r][c] = (r < b && c < b) ? K[(int64_t)(j0 + r) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < b; ++c) {
    if (threadIdx.x == 0) {
      const double piv = a[c][c];
      if (!(piv > 0.0)) flag[0] = 1;
      a[c][c] = sqrt(fmax(piv, 0.0));
    }
    __syncthreads();
    const double dc = a[c][c];
    for (int r = c + 1 + threadIdx.x; r < b; r += 256) a[r][c] = dc > 0.0 ? a[r][c] / dc : 0.0;
    __syncthreads();
    for (int e = threadIdx.x; e < CB * CB; e += 256) {
      const int r = e / CB, t = e % CB;
      if (r > c && r < b && t > c && t <= r) a[r][t] -= a[r][c] * a[t][c];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    if (r < b && c <= r) K[(int64_t)(j0 + r) * n + j0 + c] = a[r][c];
  }
}

// Panel below the diagonal block: row i >= j0 + CB solves x L_jj^T = K[i][j0 .. j0 + CB) by
// forward substitution (a thread per row).
__global__ __launch_bounds__(256) void k_mw_chol_trsm(double* __restrict__ K, int n, int j0) {
  __shared__ double l[CB][CB + 1];
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    l[r][c] = c <= r ? K[(int64_t)(j0 + r) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  const int i = j0 + CB + blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double x[CB];
  double* row = K + (int64_t)i * n + j0;
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = row[c];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    double s = x[c];
#pragma unroll
    for (int t = 0; t < c; ++t) s -= x[t] * l[c][t];
    x[c] = l[c][c] > 0.0 ? s / l[c][c] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) row[c] = x[c];
}

// Trailing update of the lower triangle right of the panel: K[i][k] -= sum_t L[i][j0+t] L[k][j0+t]
// for j0 + CB <= k <= i, one 32 x 32 tile (I >= J) per workgroup, four elements per thread.
__global__ __launch_bounds__(256) void k_mw_chol_update(double* __restrict__ K, int n, int j0) {
  __shared__ double pi[CB][CB + 1], pk[CB][CB + 1];
  int I, J;
  tri_pair(blockIdx.x, &I, &J);
  const int r0 = j0 + CB + I * CB, c0 = j0 + CB + J * CB;
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, t = e % CB;
    pi[r][t] = r0 + r < n ? K[(int64_t)(r0 + r) * n + j0 + t] : 0.0;
    pk[r][t] = c0 + r < n ? K[(int64_t)(c0 + r) * n + j0 + t] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    const int i = r0 + r, k = c0 + c;
    if (i < n && k < n && k <= i) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < CB; ++t) s += pi[r][t] * pk[c][t];
      K[(int64_t)i * n + k] -= s;
    }
  }
}

// S = L^T W L (L: the lower triangle of K; the entries above its diagonal are ignored), tiles
// (I, J) with I >= J, both triangles written: S[i][j] = sum over k >= max(i, j) of
// L[k][i] w_k L[k][j].
__global__ __launch_bounds__(256) void k_mw_sym(const double* __restrict__ K, int n, int64_t nvv,
                                                double* __restrict__ S) {
  __shared__ double a[CB][CB + 1], bb[CB][CB + 1];
  int I, J;
  tri_pair(blockIdx.x, &I, &J);
  const int i0 = I * CB, j0 = J * CB;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = i0; k0 < n; k0 += CB) {
    __syncthreads();
    for (int e = threadIdx.x; e < CB * CB; e += 256) {
      const int kk = e / CB, c = e % CB;
      const int k = k0 + kk;
      const double w = k < nvv ? 1.0 : -1.0;
      const int ci = i0 + c, cj = j0 + c;
      a[kk][c] = (k < n && ci < n && k >= ci) ? K[(int64_t)k * n + ci] * w : 0.0;
      bb[kk][c] = (k < n && cj < n && k >= cj) ? K[(int64_t)k * n + cj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int r = e / CB, c = e % CB;
      double s = acc[q];
#pragma unroll 8
      for (int kk = 0; kk < CB; ++kk) s += a[kk][r] * bb[kk][c];
      acc[q] = s;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int i = i0 + e / CB, j = j0 + e % CB;
    if (i < n && j < n) {
      S[(int64_t)i * n + j] = acc[q];
      S[(int64_t)j * n + i] = acc[q];
    }
  }
}

// Householder step k: x = S[k][k+1 ..] (column k below the diagonal, read as row k), alpha =
// -sign(x_0) |x|, v = x - alpha e_1, beta = 2 / v^T v (0 when x = 0); d[k] = S[k][k], e[k] = alpha.
// Launched for the first step; the update kernel of step k forms the vector of step k + 1.
__global__ __launch_bounds__(1024) void k_mw_hh_vec(const double* __restrict__ S, int n, int k,
                                                    double* __restrict__ v,
                                                    double* __restrict__ scal,
                                                    double* __restrict__ d,
                                                    double* __restrict__ e,
                                                    double* __restrict__ beta_keep) {
  __shared__ double red[16];
  const int m = n - k - 1;
  const double* x = S + (int64_t)k * n + k + 1;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 1024) s += x[i] * x[i];
  const double nrm2 = wg_sum(s, red);
  const double x0 = x[0];
  const double nrm = sqrt(nrm2);
  const double alpha = nrm > 0.0 ? (x0 > 0.0 ? -nrm : nrm) : 0.0;
  const double v0 = x0 - alpha;
  const double vtv = nrm2 - x0 * x0 + v0 * v0;
  for (int i = threadIdx.x; i < m; i += 1024) v[i] = i == 0 ? v0 : x[i];
  if (threadIdx.x == 0) {
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    scal[0] = beta;
    if (beta_keep) beta_keep[k] = beta;
    d[k] = S[(int64_t)k * n + k];
    e[k] = alpha;
  }
}

// p = beta S2 v, S2 = S[k+1 ..][k+1 ..]: a wave per row (lanes stride the row).
__global__ __launch_bounds__(256) void k_mw_hh_matvec(const double* __restrict__ S, int n, int k,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ scal,
                                                      double* __restrict__ p) {
  const int m = n - k - 1;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= m) return;
  const double* row = S + (int64_t)(k + 1 + r) * n + k + 1;
  double s = 0.0;
  for (int j = lane; j < m; j += 64) s += row[j] * v[j];
  s = wave_sum(s);
  if (lane == 0) p[r] = scal[0] * s;
}

// S2 -= v w^T + w v^T, w = p - (beta p^T v / 2) v: a wave per row; every workgroup forms p^T v
// itself in the same fixed order. keep: row k right of the diagonal becomes the reflection vector
// (only its first entry differs from x; no kernel of this step reads row k). The wave of row
// k + 1, the first row of S2, then forms the reflection of step k + 1 from the row it has just
// updated (as k_mw_hh_vec does; its norm summed over the wave's lanes in a fixed order) into the
// other buffer of v and beta: v_next, beta_next[0], d[k + 1], e[k + 1] (and beta_keep[k + 1]).
__global__ __launch_bounds__(256) void k_mw_hh_update(double* __restrict__ S, int n, int k,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ bet,
                                                      const double* __restrict__ p, int keep,
                                                      double* __restrict__ v_next,
                                                      double* __restrict__ beta_next,
                                                      double* __restrict__ d,
                                                      double* __restrict__ e,
                                                      double* __restrict__ beta_keep) {
  __shared__ double red[4];
  if (keep && blockIdx.x == 0 && threadIdx.x == 0) S[(int64_t)k * n + k + 1] = v[0];
  const int m = n - k - 1;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) s += p[i] * v[i];
  const double ptv = wg_sum(s, red);
  const double kk = 0.5 * bet[0] * ptv;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= m) return;
  const double vr = v[r], wr = p[r] - kk * vr;
  double* row = S + (int64_t)(k + 1 + r) * n + k + 1;
  const bool next = r == 0 && k + 3 < n;  // uniform over the wave
  double ss = 0.0, x0 = 0.0, dg = 0.0;
  for (int j = lane; j < m; j += 64) {
    const double vj = v[j], wj = p[j] - kk * vj;
    const double nv = row[j] - (vr * wj + wr * vj);
    row[j] = nv;
    if (j == 0) dg = nv;
    if (j == 1) x0 = nv;
    if (j >= 1) ss += nv * nv;
  }
  if (!next) return;
  const double nrm2 = wave_sum(ss);
  x0 = __shfl(x0, 1, 64);
  dg = __shfl(dg, 0, 64);
  const double nrm = sqrt(nrm2);
  const double alpha = nrm > 0.0 ? (x0 > 0.0 ? -nrm : nrm) : 0.0;
  const double v0 = x0 - alpha;
  const double vtv = nrm2 - x0 * x0 + v0 * v0;
  for (int j = lane + (lane == 0 ? 64 : 0); j < m; j += 64) v_next[j - 1] = j == 1 ? v0 : row[j];
  if (lane == 0) {
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    beta_next[0] = beta;
    if (beta_keep) beta_keep[k + 1] = beta;
    d[k + 1] = dg;
    e[k + 1] = alpha;
  }
}

__device__ __forceinline__ int mw_sturm_below(const double* __restrict__ d,
                                              const double* __restrict__ e, int n, double x,
                                              double tiny) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    if (fabs(q) < tiny) q = -tiny;
    q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// The last two diagonal and the last off-diagonal entry, then the Gershgorin interval of T:
// bnd[0] = lower, bnd[1] = upper, bnd[2] = a norm of T (one workgroup).
__global__ __launch_bounds__(1024) void k_mw_bounds(const double* __restrict__ S, int n,
                                                    double* __restrict__ d, double* __restrict__ e,
                                                    double* __restrict__ bnd) {
  __shared__ double red[16];
  if (threadIdx.x == 0) {
    if (n >= 2) {
      d[n - 2] = S[(int64_t)(n - 2) * n + n - 2];
      e[n - 2] = S[(int64_t)(n - 1) * n + n - 2];
    }
    d[n - 1] = S[(int64_t)(n - 1) * n + n - 1];
  }
  __syncthreads();
  double lo = 1e300, hi = -1e300, nr = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    nr = fmax(nr, fabs(d[i]) + r);
  }
  const double glo = wg_min(lo, red), ghi = wg_max(hi, red), gn = wg_max(nr, red);
  if (threadIdx.x == 0) {
    bnd[0] = glo;
    bnd[1] = ghi;
    bnd[2] = fmax(gn, 1e-300);
  }
}

// Eigenvalue idx (ascending) of T, 16 lanes each: per round the lanes take the Sturm count at 16
// evenly spaced interior points of the bracket, which shrinks to the two neighbouring points that
// enclose the index (reduced over the 16 lanes by shuffles), until its width is at the rounding
// level. A wave runs until its four brackets are done.
__global__ __launch_bounds__(256) void k_mw_bisect(const double* __restrict__ d,
                                                   const double* __restrict__ e, int n,
                                                   const double* __restrict__ bnd,
                                                   double* __restrict__ lam) {
  const int gid = blockIdx.x * 256 + threadIdx.x;
  const int idx = gid >> 4, g = gid & 15;
  const double tnorm = bnd[2];
  const double tiny = 1e-300 + 2.2e-16 * tnorm * 1e-8;
  double lo = bnd[0] - 1e-12 * tnorm, hi = bnd[1] + 1e-12 * tnorm;
  bool done = idx >= n;
  for (int round = 0; round < 64; ++round) {
    if (!done) done = !(hi - lo > 4.4e-16 * fmax(fabs(lo), fabs(hi)) + tiny);
    if (__all(done)) break;
    const double x = lo + (hi - lo) * ((double)(g + 1) / 17.0);
    double xl = -1e300, xh = 1e300;
    if (!done && x > lo && x < hi) {
      if (mw_sturm_below(d, e, n, x, tiny) <= idx)
        xl = x;
      else
        xh = x;
    }
    for (int off = 8; off > 0; off >>= 1) {
      xl = fmax(xl, __shfl_xor(xl, off, 64));
      xh = fmin(xh, __shfl_xor(xh, off, 64));
    }
    if (!done) {
      const double nlo = fmax(lo, xl), nhi = fmin(hi, xh);
      if (nlo > nhi || (nlo == lo && nhi == hi)) {
        done = true;
      } else {
        lo = nlo;
        hi = nhi;
      }
    }
  }
  if (idx < n && g == 0) lam[idx] = 0.5 * (lo + hi);
}

// out[0] = sum over lambda > 0 of (mu2 + lambda) - Tr A, out[1] = -(sum over lambda < 0 of
// (mu2 + lambda)) - Tr C, out[2] = Tr A, out[3] = Tr C; info: [0] 0 / 1 (K not positive definite),
// [1] pp roots, [2] hh roots. Fixed-order sums (one workgroup).
__global__ __launch_bounds__(1024) void k_mw_sums(const double* __restrict__ M, int n,
                                                  int64_t nvv, double mu2,
                                                  const double* __restrict__ lam,
                                                  const int* __restrict__ flag,
                                                  double* __restrict__ out,
                                                  int* __restrict__ info) {
  __shared__ double red[16];
  double spp = 0.0, shh = 0.0, npp = 0.0, nhh = 0.0, tra = 0.0, trc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double l = lam[i], om = mu2 + l;
    if (l > 0.0) {
      spp += om;
      npp += 1.0;
    } else {
      shh += om;
      nhh += 1.0;
    }
    if (i < nvv)
      tra += M[(int64_t)i * n + i];
    else
      trc += M[(int64_t)i * n + i];
  }
  const double SPP = wg_sum(spp, red), SHH = wg_sum(shh, red);
  const double NPP = wg_sum(npp, red), NHH = wg_sum(nhh, red);
  const double TA = wg_sum(tra, red), TC = wg_sum(trc, red);
  if (threadIdx.x == 0) {
    out[0] = SPP - TA;
    out[1] = -SHH - TC;
    out[2] = TA;
    out[3] = TC;
    info[0] = flag[0] ? 1 : 0;
    info[1] = (int)NPP;
    info[2] = (int)NHH;
  }
}

// Number of eigenvalues of T below 0 (the hh roots) -> cnt[0].
__global__ void k_mw_count(const double* __restrict__ d, const double* __restrict__ e, int n,
                           const double* __restrict__ bnd, int* __restrict__ cnt) {
  if (threadIdx.x != 0) return;
  const double tiny = 1e-300 + 2.2e-16 * bnd[2] * 1e-8;
  cnt[0] = mw_sturm_below(d, e, n, 0.0, tiny);
}

// Ascending index of wanted root j: pp (channel 0) the j-th eigenvalue above 0, hh the j-th below
// 0; -1 when the channel has no such root.
__device__ __forceinline__ int mw_wanted(int j, int nbelow, int n, int channel) {
  const int idx = channel == 0 ? nbelow + j : nbelow - 1 - j;
  return idx >= 0 && idx < n ? idx : -1;
}

// Wanted eigenvalue j of T (a workgroup each): per round the 256 threads take the Sturm count at
// 256 evenly spaced interior points of the bracket, which shrinks to the two neighbouring points
// that enclose the root's index, until its width is at the rounding level. lam[j] = 0 for a root
// the channel does not have.
__global__ __launch_bounds__(256) void k_mw_select(const double* __restrict__ d,
                                                   const double* __restrict__ e, int n,
                                                   const double* __restrict__ bnd,
                                                   const int* __restrict__ cnt, int channel,
                                                   const int* __restrict__ flag,
                                                   double* __restrict__ lam) {
  __shared__ double red[4];
  const int j = blockIdx.x, t = threadIdx.x;
  const int idx = mw_wanted(j, cnt[0], n, channel);
  if (flag[0] || idx < 0) {
    if (t == 0) lam[j] = 0.0;
    return;
  }
  const double tnorm = bnd[2];
  const double tiny = 1e-300 + 2.2e-16 * tnorm * 1e-8;
  double lo = bnd[0] - 1e-12 * tnorm, hi = bnd[1] + 1e-12 * tnorm;
  for (int round = 0; round < 64; ++round) {
    if (!(hi - lo > 4.4e-16 * fmax(fabs(lo), fabs(hi)) + tiny)) break;
    const double x = lo + (hi - lo) * ((double)(t + 1) / 257.0);
    double xl = -1e300, xh = 1e300;
    if (x > lo && x < hi) {
      if (mw_sturm_below(d, e, n, x, tiny) <= idx)
        xl = x;
      else
        xh = x;
    }
    const double nlo = fmax(lo, wg_max(xl, red));
    const double nhi = fmin(hi, wg_min(xh, red));
    if (nlo > nhi || (nlo == lo && nhi == hi)) break;
    lo = nlo;
    hi = nhi;
  }
  if (t == 0) lam[j] = 0.5 * (lo + hi);
}

// Eigenvector of T at lam[j] by inverse iteration (thread j): three solves of (T - lam I) y = b
// by Gaussian elimination with partial pivoting (the fill-in on a second superdiagonal), y
// normalised after each; the start vector a fixed pseudo-random sequence per root. Y [nsel][n]
// (zero for a root the channel does not have); U [nsel][3][n] elimination scratch.
__global__ __launch_bounds__(64) void k_mw_inviter(const double* __restrict__ d,
                                                   const double* __restrict__ e, int n,
                                                   const double* __restrict__ bnd,
                                                   const int* __restrict__ cnt, int channel,
                                                   const int* __restrict__ flag,
                                                   const double* __restrict__ lam, int nsel,
                                                   double* __restrict__ Y,
                                                   double* __restrict__ U) {
  const int j = threadIdx.x;
  if (j >= nsel) return;
  double* y = Y + (size_t)j * n;
  if (flag[0] || mw_wanted(j, cnt[0], n, channel) < 0) {
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    return;
  }
  double* U0 = U + (size_t)j * 3 * n;
  double* U1 = U0 + n;
  double* U2 = U1 + n;
  const double th = lam[j];
  const double pert = 2.2e-16 * bnd[2];
  unsigned long long h = 0xD1B54A32D192ED03ull * (unsigned long long)(j + 1);
  for (int i = 0; i < n; ++i) {
    h ^= h >> 31;
    h *= 0x9FB21C651E98DF25ull;
    h ^= h >> 29;
    y[i] = 0.5 + (double)(h >> 11) * (1.0 / 9007199254740992.0);
  }
  for (int pass = 0; pass < 3; ++pass) {
    // forward elimination: row i holds (a_d, a_u, a_u2 | rhs) after the pivots above it
    double a_d = d[0] - th, a_u = n > 1 ? e[0] : 0.0, a_u2 = 0.0, rhs = y[0];
    for (int i = 0; i + 1 < n; ++i) {
      const double b_l = e[i], b_d = d[i + 1] - th, b_u = i + 2 < n ? e[i + 1] : 0.0;
      const double rb = y[i + 1];
      if (fabs(a_d) >= fabs(b_l)) {
        const double piv = fabs(a_d) < pert ? (a_d < 0.0 ? -pert : pert) : a_d;
        const double l = b_l / piv;
        U0[i] = piv;
        U1[i] = a_u;
        U2[i] = a_u2;
        y[i] = rhs;
        a_d = b_d - l * a_u;
        a_u = b_u - l * a_u2;
        a_u2 = 0.0;
        rhs = rb - l * rhs;
      } else {  // rows i and i + 1 exchanged
        const double l = a_d / b_l;
        U0[i] = b_l;
        U1[i] = b_d;
        U2[i] = b_u;
        y[i] = rb;
        a_d = a_u - l * b_d;
        a_u = a_u2 - l * b_u;
        a_u2 = 0.0;
        rhs = rhs - l * rb;
      }
    }
    if (fabs(a_d) < pert) a_d = a_d < 0.0 ? -pert : pert;
    U0[n - 1] = a_d;
    U1[n - 1] = 0.0;
    U2[n - 1] = 0.0;
    y[n - 1] = rhs;
    double y1 = 0.0, y2 = 0.0, nrm2 = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double v = (y[i] - U1[i] * y1 - U2[i] * y2) / U0[i];
      y[i] = v;
      y2 = y1;
      y1 = v;
      nrm2 += v * v;
    }
    const double inv = 1.0 / sqrt(nrm2);
    for (int i = 0; i < n; ++i) y[i] *= inv;
  }
}

// Vectors of nearly equal eigenvalues (|lam_i - lam_j| <= 1e-7 |T|) orthonormalised in order
// (modified Gram-Schmidt; one workgroup). Only roots the channel has take part.
__global__ __launch_bounds__(1024) void k_mw_orth(int n, const double* __restrict__ bnd,
                                                  const int* __restrict__ cnt, int channel,
                                                  const int* __restrict__ flag,
                                                  const double* __restrict__ lam, int nsel,
                                                  double* __restrict__ Y) {
  __shared__ double red[16];
  if (flag[0]) return;
  const double tol = 1e-7 * bnd[2];
  for (int j = 1; j < nsel; ++j) {
    if (mw_wanted(j, cnt[0], n, channel) < 0) break;
    double* yj = Y + (size_t)j * n;
    for (int i = 0; i < j; ++i) {
      if (fabs(lam[i] - lam[j]) > tol) continue;
      const double* yi = Y + (size_t)i * n;
      double s = 0.0;
      for (int r = threadIdx.x; r < n; r += 1024) s += yi[r] * yj[r];
      const double dot = wg_sum(s, red);
      double s2 = 0.0;
      for (int r = threadIdx.x; r < n; r += 1024) {
        const double v = yj[r] - dot * yi[r];
        yj[r] = v;
        s2 += v * v;
      }
      const double inv = 1.0 / sqrt(wg_sum(s2, red));
      for (int r = threadIdx.x; r < n; r += 1024) yj[r] *= inv;
      __syncthreads();
    }
  }
}

// Root j (a workgroup each; the vector in LDS, element r owned by thread r mod 256): u = H_0 H_1
// ... H_{n-3} y (reflection k kept in row k of S right of the diagonal, beta[k]), then L^T z = u
// by back substitution in 32-row blocks (the block's triangle within one wave, the rows above it
// updated by all threads), z scaled by sqrt|lambda| into column j of Cout [n][ldc]. omega[j] =
// mu2 + lambda_j; a root the channel does not have gets omega 0 and a zero column. info (block 0):
// [0] 0 ok / 1 not definite / 2 fewer than nroot roots, [1] roots of the channel, [2] 0.
__global__ __launch_bounds__(256) void k_mw_vectors(const double* __restrict__ K,
                                                    const double* __restrict__ S,
                                                    const double* __restrict__ beta, int n,
                                                    const int* __restrict__ cnt, int channel,
                                                    const int* __restrict__ flag,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ Y, double mu2,
                                                    double* __restrict__ omega,
                                                    double* __restrict__ Cout, int ldc,
                                                    int* __restrict__ info) {
  __shared__ double y[DENSE_SOLVE_MAX];
  __shared__ double red[2][4];
  const int j = blockIdx.x, t = threadIdx.x;
  const int bad = flag[0];
  const int nb = cnt[0];
  const int npos = bad ? 0 : (channel == 0 ? n - nb : nb);
  if (j == 0 && t == 0) {
    info[0] = bad ? 1 : (npos < (int)gridDim.x ? 2 : 0);
    info[1] = npos;
    info[2] = 0;
  }
  if (bad || j >= npos) {
    if (t == 0) omega[j] = 0.0;
    for (int r = t; r < n; r += 256) Cout[(size_t)r * ldc + j] = 0.0;
    return;
  }
  const double lj = lam[j];
  if (t == 0) omega[j] = mu2 + lj;
  for (int r = t; r < n; r += 256) y[r] = Y[(size_t)j * n + r];
  // reflections, last first; each thread updates only the elements it owns (r = t + 256 q), so
  // one barrier (inside the reduction, its partials alternating between two buffers) per
  // reflection; the next reflection's entries are loaded into registers a step ahead
  constexpr int NQ = DENSE_SOLVE_MAX / 256;
  double vc[NQ], vn[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = t + 256 * q;
    vc[q] = n >= 3 && r > n - 3 && r < n ? S[(size_t)(n - 3) * n + r] : 0.0;
  }
  int ph = 0;
  for (int k = n - 3; k >= 0; --k) {
    const double b = beta[k];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = t + 256 * q;
      vn[q] = k >= 1 && r > k - 1 && r < n ? S[(size_t)(k - 1) * n + r] : 0.0;
    }
    if (b != 0.0) {  // uniform
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = t + 256 * q;
        if (r > k && r < n) s += vc[q] * y[r];
      }
      s = wave_sum(s);
      double* rb = red[ph];
      ph ^= 1;
      if ((t & 63) == 0) rb[t >> 6] = s;
      __syncthreads();
      const double bs = b * (rb[0] + rb[1] + rb[2] + rb[3]);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = t + 256 * q;
        if (r > k && r < n) y[r] -= bs * vc[q];
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) vc[q] = vn[q];
  }
  __syncthreads();
  // L^T z = u, blocks of 32 rows from the last; lane l of wave 0 holds column l of the block's
  // triangle in registers before the block's chain of shuffles
  for (int j0 = ((n - 1) / CB) * CB; j0 >= 0; j0 -= CB) {
    const int jb = min(CB, n - j0);
    if (t < 64) {
      const int l = t;
      double lc[CB];
#pragma unroll
      for (int jj = 0; jj < CB; ++jj)
        lc[jj] = jj < jb && l <= jj ? K[(size_t)(j0 + jj) * n + j0 + l] : 0.0;
      double r = l < jb ? y[j0 + l] : 0.0;
#pragma unroll
      for (int jj = CB - 1; jj >= 0; --jj) {
        if (jj < jb) {  // uniform
          const double z = l == jj ? r / lc[jj] : 0.0;
          const double zj = __shfl(z, jj, 64);
          if (l == jj) r = zj;
          if (l < jj) r -= lc[jj] * zj;
        }
      }
      if (l < jb) y[j0 + l] = r;
    }
    __syncthreads();
    for (int r = t; r < j0; r += 256) {
      double acc = 0.0;
      for (int jj = 0; jj < jb; ++jj) acc += K[(size_t)(j0 + jj) * n + r] * y[j0 + jj];
      y[r] -= acc;
    }
    __syncthreads();
  }
  const double sc = sqrt(fabs(lj));
  for (int r = t; r < n; r += 256) Cout[(size_t)r * ldc + j] = y[r] * sc;
}

}  // namespace

// Steps 1-4 (K, its Cholesky factor, S = L^T W L, the tridiagonal form (d, e) with the bounds
// of its spectrum) on stream s. v2: 2 n (the reflection vectors of two steps), bsc: 5 doubles
// ([0], [1] beta of even and odd steps, [2 .. 4] the bounds); beta_keep: n doubles or null (keep
// the reflections in the rows of S); flag: zeroed, then set when K is not positive definite.
static void mw_reduce(const double* M, int n, int64_t nvv, double mu2, double* K, double* S,
                      double* v2, double* p, double* d, double* e, double* bsc,
                      double* beta_keep, int* flag, hipStream_t s) {
  const size_t nn = (size_t)n * n;
  hipLaunchKernelGGL(k_mw_init, dim3(1), dim3(64), 0, s, flag);
  hipLaunchKernelGGL(k_mw_shift, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, M, n, nvv,
                     mu2, K);
  for (int j0 = 0; j0 < n; j0 += CB) {
    hipLaunchKernelGGL(k_mw_chol_diag, dim3(1), dim3(256), 0, s, K, n, j0, flag);
    const int rest = n - j0 - CB;
    if (rest > 0) {
      hipLaunchKernelGGL(k_mw_chol_trsm, dim3((rest + 255) / 256), dim3(256), 0, s, K, n, j0);
      const int nt = (rest + CB - 1) / CB;
      hipLaunchKernelGGL(k_mw_chol_update, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, K, n, j0);
    }
  }
  const int ntile = (n + CB - 1) / CB;
  hipLaunchKernelGGL(k_mw_sym, dim3(ntile * (ntile + 1) / 2), dim3(256), 0, s, K, n, nvv, S);
  if (n > 2)
    hipLaunchKernelGGL(k_mw_hh_vec, dim3(1), dim3(1024), 0, s, S, n, 0, v2, bsc, d, e, beta_keep);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1, c = k & 1;
    double* vk = v2 + (size_t)c * n;
    double* vn = v2 + (size_t)(1 - c) * n;
    hipLaunchKernelGGL(k_mw_hh_matvec, dim3((m + 3) / 4), dim3(256), 0, s, S, n, k, vk, bsc + c, p);
    hipLaunchKernelGGL(k_mw_hh_update, dim3((m + 3) / 4), dim3(256), 0, s, S, n, k, vk, bsc + c, p,
                       beta_keep ? 1 : 0, vn, bsc + (1 - c), d, e, beta_keep);
  }
  hipLaunchKernelGGL(k_mw_bounds, dim3(1), dim3(1024), 0, s, S, n, d, e, bsc + 2);
}

size_t pencil_energy_mw_work(int n) { return 2 * (size_t)n * n + 6 * (size_t)n + 8; }

hipError_t launch_pencil_energy_mw(const double* M, int n, int64_t nvv, double mu2, double* out,
                                   double* work, int* info, hipStream_t s) {
  if (n < 2 || n > DENSE_ENERGY_MAX) return hipErrorInvalidValue;
  const size_t nn = (size_t)n * n;
  double* K = work;
  double* S = K + nn;
  double* v2 = S + nn;
  double* p = v2 + 2 * (size_t)n;
  double* d = p + n;
  double* e = d + n;
  double* lam = e + n;
  double* bsc = lam + n;  // [0], [1] beta, [2 .. 4] Gershgorin bounds and norm
  int* flag = info;       // info[0] doubles as the not-definite flag until the last kernel
  mw_reduce(M, n, nvv, mu2, K, S, v2, p, d, e, bsc, nullptr, flag, s);
  hipLaunchKernelGGL(k_mw_bisect, dim3((unsigned)((16 * (size_t)n + 255) / 256)), dim3(256), 0, s,
                     d, e, n, bsc + 2, lam);
  hipLaunchKernelGGL(k_mw_sums, dim3(1), dim3(1024), 0, s, M, n, nvv, mu2, lam, flag, out, info);
  return hipGetLastError();
}

size_t direct_pencil_mw_work(int n, int nroot) {
  return 2 * (size_t)n * n + 6 * (size_t)n + 4 * (size_t)nroot * n + 64 + 8 + 8;
}

hipError_t launch_direct_pencil_mw(const double* M, int n, int64_t nvv, double mu2, int nroot,
                                   int channel, double* omega, double* Cout, int ldc,
                                   double* work, int* info, hipStream_t s) {
  if (n < 3 || n > DENSE_SOLVE_MAX || nroot < 1 || nroot > 64 || nroot > n || ldc < nroot ||
      (channel != 0 && channel != 1))
    return hipErrorInvalidValue;
  const size_t nn = (size_t)n * n;
  double* K = work;
  double* S = K + nn;
  double* v2 = S + nn;
  double* p = v2 + 2 * (size_t)n;
  double* d = p + n;
  double* e = d + n;
  double* beta = e + n;
  double* Y = beta + n;
  double* U = Y + (size_t)nroot * n;
  double* lam = U + 3 * (size_t)nroot * n;  // 64
  double* bsc = lam + 64;                   // [0], [1] beta, [2 .. 4] bounds
  int* cnt = (int*)(bsc + 8);               // [0] eigenvalues below 0
  int* flag = cnt + 1;                      // K not positive definite
  mw_reduce(M, n, nvv, mu2, K, S, v2, p, d, e, bsc, beta, flag, s);
  hipLaunchKernelGGL(k_mw_count, dim3(1), dim3(64), 0, s, d, e, n, bsc + 2, cnt);
  hipLaunchKernelGGL(k_mw_select, dim3(nroot), dim3(256), 0, s, d, e, n, bsc + 2, cnt, channel,
                     flag, lam);
  hipLaunchKernelGGL(k_mw_inviter, dim3(1), dim3(64), 0, s, d, e, n, bsc + 2, cnt, channel, flag,
                     lam, nroot, Y, U);
  hipLaunchKernelGGL(k_mw_orth, dim3(1), dim3(1024), 0, s, n, bsc + 2, cnt, channel, flag, lam,
                     nroot, Y);
  hipLaunchKernelGGL(k_mw_vectors, dim3(nroot), dim3(256), 0, s, K, S, beta, n, cnt, channel, flag,
                     lam, Y, mu2, omega, Cout, ldc, info);
  return hipGetLastError();
}

}  // namespace pprpa
