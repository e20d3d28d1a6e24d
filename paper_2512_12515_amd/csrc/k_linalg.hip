// FP64 linear algebra of the Davidson solver and of the direct path, on the GPU.
//
//  * tall-skinny products over the long pair dimension (HBM-bound, FP64 MFMA):
//      dots     C = A diag(w) B^T       (subspace matrices V^T M V, V^T W V, projections)
//      combine  Y = beta Y + alpha C^T X (Ritz vectors, projections, basis rotations)
//      residual r = sigma(z) - Omega W z and its 2-norm; Davidson diagonal preconditioner
//  * one-workgroup dense solvers for the small projected problems:
//      pencil   the definite generalised eigenproblem M c = Omega W c via
//               M - 2 mu W = R R^T (Cholesky), G = R^-1 W R^-T, Householder tridiagonal form of
//               G, Sturm-count bisection for the wanted eigenvalues theta and inverse iteration
//               for their vectors, Omega = 2 mu + 1/theta; pp roots have theta > 0
//               (c^T W c = +1 after scaling by 1/sqrt(theta))
//      gram_orth / small_orth / congruence for the basis bookkeeping (cyclic Jacobi on the small
//               Gram matrices).
#include "internal.h"

namespace pprpa {
namespace {

constexpr int NT = 256;  // threads per block of the streaming kernels

// ------------------------------------------------------------------------------------------
// dots: part[chunk][i][j] = sum_{t in chunk} A[i][t] w(t) B[j][t], w(t) = -1 for t >= nsign when
// signed, else 1. FP64 MFMA 16x16x4 over the long index t: workgroup = one chunk of t, wave = one
// 16-row block of A against up to four 16-row blocks of B. In MFMA s of a 16-wide step at t0,
// lane (li, lk) supplies A[.. + li][t0 + 4 lk + s] and B[.. + li][t0 + 4 lk + s] (the reduction
// index permuted alike in both operands), so each lane reads four consecutive doubles of its row.
// Fixed summation order: deterministic.
// ------------------------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int DOT_STEP = 16;
constexpr int DOT_WAVES = 8;  // at most, per workgroup

template <int NJ>
__device__ __forceinline__ void dots_unit(const double* __restrict__ A, int64_t lda, int ma,
                                          const double* __restrict__ B, int64_t ldb, int mb,
                                          int64_t t0, int64_t t1, int64_t nsign, int signed_w,
                                          int I, int J0, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int ia = I * 16 + li;
  const double* a = A + (int64_t)(ia < ma ? ia : ma - 1) * lda;
  const bool aok = ia < ma;
  const double* b[NJ];
  bool bok[NJ];
#pragma unroll
  for (int J = 0; J < NJ; ++J) {
    const int jb = (J0 + J) * 16 + li;
    b[J] = B + (int64_t)(jb < mb ? jb : mb - 1) * ldb;
    bok[J] = jb < mb;
  }
  d4 acc[NJ];
#pragma unroll
  for (int J = 0; J < NJ; ++J) acc[J] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t t = t0; t < t1; t += DOT_STEP) {
    const int64_t tl = t + 4 * lk;
    const bool full = t + DOT_STEP <= t1;
    double av[4], bv[NJ][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool ok = full || tl + s < t1;
      av[s] = (aok && ok) ? a[tl + s] : 0.0;
    }
#pragma unroll
    for (int J = 0; J < NJ; ++J)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool ok = full || tl + s < t1;
        double v = (bok[J] && ok) ? b[J][tl + s] : 0.0;
        bv[J][s] = (signed_w && tl + s >= nsign) ? -v : v;
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int J = 0; J < NJ; ++J)
        acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[J][s], acc[J], 0, 0, 0);
  }
  // accumulator register r of lane (li, lk) holds row lk + 4 r, column li of the 16 x 16 tile
#pragma unroll
  for (int J = 0; J < NJ; ++J) {
    const int col = (J0 + J) * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = I * 16 + lk + 4 * r;
      if (row < ma && col < mb) out[(int64_t)row * mb + col] = acc[J][r];
    }
  }
}

__global__ __launch_bounds__(64 * DOT_WAVES) void k_dots(const double* __restrict__ A,
                                                         int64_t lda, int ma,
                                                         const double* __restrict__ B,
                                                         int64_t ldb, int mb, int64_t n,
                                                         int64_t nsign, int signed_w,
                                                         int64_t chunk,
                                                         double* __restrict__ part) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * chunk;
  const int64_t t1 = t0 + chunk < n ? t0 + chunk : n;
  const int nI = (ma + 15) / 16, nG = (mb + 63) / 64;  // row blocks; groups of 4 column blocks
  double* out = part + (size_t)blockIdx.x * ma * mb;
  for (int u = w; u < nI * nG; u += nw) {
    const int I = u / nG, J0 = 4 * (u % nG);
    const int nj = min(4, (mb + 15) / 16 - J0);
    switch (nj) {
      case 1: dots_unit<1>(A, lda, ma, B, ldb, mb, t0, t1, nsign, signed_w, I, J0, out); break;
      case 2: dots_unit<2>(A, lda, ma, B, ldb, mb, t0, t1, nsign, signed_w, I, J0, out); break;
      case 3: dots_unit<3>(A, lda, ma, B, ldb, mb, t0, t1, nsign, signed_w, I, J0, out); break;
      default: dots_unit<4>(A, lda, ma, B, ldb, mb, t0, t1, nsign, signed_w, I, J0, out); break;
    }
  }
}

// C[i][j] = sum over chunks of part[c][i][j]: 16 elements per workgroup, sixteen threads per
// element (16 consecutive elements of one chunk are one 128-byte segment), thread q summing
// chunks q, q + 16, ... in order; the sixteen sums are added in a fixed order (deterministic).
constexpr int RED_T = 16;  // threads per element of k_dots_reduce
__global__ __launch_bounds__(256) void k_dots_reduce(const double* __restrict__ part, int nchunk,
                                                     int ma, int mb, double* __restrict__ C,
                                                     int ldc) {
  __shared__ double red[RED_T][17];
  const int e = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int nel = ma * mb;
  const int p = blockIdx.x * 16 + e;
  const size_t stride = (size_t)nel;
  const double* src = part + (p < nel ? p : nel - 1);
  double s = 0.0;
  // chunks q, q + 16, ... in order, four loads at a time (indices clamped, loads unguarded; the
  // partial sums are finite, so the steps past the end add exact zeros)
  for (int c0 = q; c0 < nchunk; c0 += 4 * RED_T) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * RED_T;
      v[u] = src[(size_t)(c < nchunk ? c : nchunk - 1) * stride] * (c < nchunk ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += v[u];
  }
  red[q][e] = s;
  __syncthreads();
  if (q == 0 && p < nel) {
    double t = red[0][e];
#pragma unroll
    for (int i = 1; i < RED_T; ++i) t += red[i][e];
    C[(p / mb) * ldc + (p % mb)] = t;
  }
}

// ------------------------------------------------------------------------------------------
// combine: Y[j][t] = beta Y[j][t] + alpha sum_i Cm[i][j] X[i][t]   (Y = beta Y + alpha Cm^T X)
// FP64 MFMA 16x16x4 with the row index i as the reduction: wave = CMB_CT tiles of 16 columns t,
// all rows j < r (NJ tiles of 16). A operand (lane li, lk) = Cm[i0 + lk][16 J + li], B operand =
// X[i0 + lk][t0 + li]: a wave-wide load reads four 128-byte row segments of X.
// ------------------------------------------------------------------------------------------
constexpr int CMB_CT = 2;     // column tiles per wave
constexpr int CMB_WAVES = 4;  // waves per workgroup

template <int NJ>
__global__ __launch_bounds__(64 * CMB_WAVES) void k_combine(const double* __restrict__ X,
                                                            int64_t ldx, int m,
                                                            const double* __restrict__ Cm,
                                                            int ldcm, int r, int64_t n,
                                                            double alpha, double beta,
                                                            double* __restrict__ Y, int64_t ldy) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t tw = ((int64_t)blockIdx.x * CMB_WAVES + w) * (16 * CMB_CT);
  if (tw >= n) return;
  int64_t tc[CMB_CT];
  bool tok[CMB_CT];
#pragma unroll
  for (int c = 0; c < CMB_CT; ++c) {
    const int64_t t = tw + 16 * c + li;
    tok[c] = t < n;
    tc[c] = t < n ? t : n - 1;
  }
  d4 acc[NJ][CMB_CT];
#pragma unroll
  for (int J = 0; J < NJ; ++J)
#pragma unroll
    for (int c = 0; c < CMB_CT; ++c) acc[J][c] = d4{0.0, 0.0, 0.0, 0.0};
  // four k steps per iteration. Every address is clamped into its row and no load is guarded
  // (so the loads of an iteration are issued together): steps past m get a zero coefficient
  // (the clamped X row is finite data), and the products landing in columns past n or rows past
  // r are never stored
  constexpr int KU = 4;
  for (int i0 = 0; i0 < m; i0 += 4 * KU) {
    double xb[KU][CMB_CT], ca[KU][NJ];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int i = i0 + 4 * u + lk;
      const bool iok = i < m;
      const double keep = iok ? 1.0 : 0.0;
      const double* xr = X + (int64_t)(iok ? i : m - 1) * ldx;
      const double* cr = Cm + (int64_t)(iok ? i : m - 1) * ldcm;
#pragma unroll
      for (int c = 0; c < CMB_CT; ++c) xb[u][c] = xr[tc[c]];
#pragma unroll
      for (int J = 0; J < NJ; ++J) {
        const int j = 16 * J + li;
        ca[u][J] = cr[j < r ? j : r - 1] * keep;
      }
    }
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int J = 0; J < NJ; ++J)
#pragma unroll
        for (int c = 0; c < CMB_CT; ++c)
          acc[J][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u][J], xb[u][c], acc[J][c], 0, 0, 0);
  }
  // accumulator register q of lane (li, lk) holds row lk + 4 q, column li of the tile
  // the old values of Y first, all at once (rows clamped below r, columns clamped into the
  // row), then the stores
  double yv[NJ][4][CMB_CT];
  if (beta != 0.0) {
#pragma unroll
    for (int J = 0; J < NJ; ++J)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = 16 * J + lk + 4 * q;
        const double* y = Y + (int64_t)(j < r ? j : r - 1) * ldy;
#pragma unroll
        for (int c = 0; c < CMB_CT; ++c) yv[J][q][c] = y[tc[c]];
      }
  }
#pragma unroll
  for (int J = 0; J < NJ; ++J)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = 16 * J + lk + 4 * q;
      if (j >= r) continue;
      double* y = Y + (int64_t)j * ldy;
#pragma unroll
      for (int c = 0; c < CMB_CT; ++c)
        if (tok[c]) {
          const double v = alpha * acc[J][c][q];
          y[tc[c]] = beta == 0.0 ? v : beta * yv[J][q][c] + v;
        }
    }
}

// ------------------------------------------------------------------------------------------
// residuals: R[j][t] = SZ[j][t] - omega_j w(t) Z[j][t]; partial squared norms per chunk
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_residual(const double* __restrict__ Z,
                                                 const double* __restrict__ SZ, int64_t ld,
                                                 int64_t n, int64_t nvv,
                                                 const double* __restrict__ omega,
                                                 double* __restrict__ R, double* __restrict__ part) {
  __shared__ double red[NT];
  const int j = blockIdx.y;
  const double om = omega[j];
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT) {
    const double w = t < nvv ? 1.0 : -1.0;
    const double r = SZ[j * ld + t] - om * w * Z[j * ld + t];
    R[j * ld + t] = r;
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_reduce_norms(const double* __restrict__ part, int nchunk, int r,
                               double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)j * nchunk + c];
  out[j] = sqrt(s);
}

struct SelList {
  int idx[64];
};

// Davidson correction t = r / (omega w - D), |den| floored at 1e-6 (D = diagonal pair energies
// with the sign of the metric block: +(e_a+e_b) for x, -(e_i+e_j) for y).
__global__ __launch_bounds__(NT) void k_precond(const double* __restrict__ R, int64_t ld,
                                                SelList sel, int64_t n, int64_t nvv,
                                                const double* __restrict__ diag,
                                                const double* __restrict__ omega,
                                                double* __restrict__ T, int64_t ldt) {
  const int jj = blockIdx.y;
  const int j = sel.idx[jj];
  const double om = omega[j];
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT) {
    const double w = t < nvv ? 1.0 : -1.0;
    double den = om * w - diag[t];
    if (fabs(den) < 1e-6) den = den < 0.0 ? -1e-6 : 1e-6;
    T[jj * ldt + t] = R[j * ld + t] / den;
  }
}

// Make the largest-magnitude component of each row positive (ties: lowest index).
__global__ __launch_bounds__(NT) void k_scale_sign(double* __restrict__ V, int64_t ld, int64_t n) {
  __shared__ double bv[NT];
  __shared__ int64_t bi[NT];
  double* v = V + blockIdx.x * ld;
  double best = -1.0;
  int64_t besti = 0;
  for (int64_t t = threadIdx.x; t < n; t += NT) {
    const double a = fabs(v[t]);
    if (a > best) {
      best = a;
      besti = t;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double o = bv[threadIdx.x + h];
      const int64_t oi = bi[threadIdx.x + h];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sgn = v[bi[0]] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  if (sgn < 0.0)
    for (int64_t t = threadIdx.x; t < n; t += NT) v[t] = -v[t];
}

// Scale each row to unit 2-norm (rows of zero norm are left as they are). One 1024-thread
// workgroup per row; four independent partial sums per thread keep four loads in flight (a
// single chain waits for each load in turn), then a butterfly per wave and the wave sums in a
// fixed order (deterministic).
constexpr int NRM_T = 1024;
__global__ __launch_bounds__(NRM_T) void k_normalize_rows(double* __restrict__ V, int64_t ld,
                                                          int64_t n) {
  __shared__ double red[NRM_T / 64];
  double* v = V + blockIdx.x * ld;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t t = threadIdx.x;
  for (; t + 3 * NRM_T < n; t += 4 * NRM_T) {
    const double a = v[t], b = v[t + NRM_T], c = v[t + 2 * NRM_T], d = v[t + 3 * NRM_T];
    s0 += a * a;
    s1 += b * b;
    s2 += c * c;
    s3 += d * d;
  }
  for (; t < n; t += NRM_T) s0 += v[t] * v[t];
  double s = (s0 + s1) + (s2 + s3);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = red[0];
  for (int w = 1; w < NRM_T / 64; ++w) tot += red[w];
  const double nrm = sqrt(tot);
  if (nrm > 0.0) {
    const double inv = 1.0 / nrm;
    for (int64_t u = threadIdx.x; u < n; u += NRM_T) v[u] *= inv;
  }
}

__global__ void k_fill(double* __restrict__ p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) p[i] = v;
}

// ------------------------------------------------------------------------------------------
// One-workgroup dense kernels (1024 threads). Matrices live in global memory (L2-resident).
// ------------------------------------------------------------------------------------------
constexpr int WG = 1024;
constexpr int JMAX = 512;   // largest matrix order of the one-workgroup Davidson-side solvers
constexpr int DMAX = DENSE_ONE_WG_MAX;  // largest order of the one-workgroup dense pencil solves

// Workgroup-wide sum / min / max (every thread calls it; every thread gets the result): a
// butterfly within each wave, then the WG / 64 wave results in a fixed order (deterministic).
// The first barrier also orders the caller's earlier LDS writes.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < WG / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// Sum over an NT-thread workgroup (every thread gets it), wave results in a fixed order.
__device__ __forceinline__ double block_sum_nt(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < NT / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// Cyclic Jacobi on the symmetric m x m matrix G (ld), accumulating eigenvectors into U (ld).
// Round-robin ordering: m (padded to even) - 1 rounds of m/2 disjoint rotations per sweep.
// On return G's diagonal holds the eigenvalues and U's columns the eigenvectors.
__device__ int jacobi_eigh(double* G, int ld, int m, double* U, double* red, double* cs,
                           double* sn, bool init_u = true) {
  const int me = m + (m & 1);
  const int half = me / 2;
  if (init_u)
    for (int e = threadIdx.x; e < m * m; e += WG) U[(e / m) * ld + (e % m)] = (e / m == e % m);
  __syncthreads();
  if (m < 2) return 0;
  __shared__ int nrot;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) nrot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < me - 1; ++rnd) {
      // rotation parameters for each pair of this round
      for (int pi = threadIdx.x; pi < half; pi += WG) {
        int p, q;
        if (pi == 0) {
          p = 0;
          q = rnd % (me - 1) + 1;
        } else {
          p = (rnd + pi) % (me - 1) + 1;
          q = (rnd - pi + me - 1) % (me - 1) + 1;
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = G[p * ld + q];
          const double app = G[p * ld + p], aqq = G[q * ld + q];
          // rotate unless |apq| is negligible against the diagonal (relative 1e-15; below that
          // the rotations only move rounding noise)
          if (fabs(apq) > 1e-15 * sqrt(fabs(app) * fabs(aqq)) && fabs(apq) > 1e-300) {
            atomicAdd(&nrot, 1);
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        cs[pi] = c;
        sn[pi] = s;
        red[2 * pi] = (double)p;
        red[2 * pi + 1] = (double)q;
      }
      __syncthreads();
      // G <- J^T G J on all 2x2 blocks (pair a, pair b)
      for (int e = threadIdx.x; e < half * half; e += WG) {
        const int pa = e / half, pb = e % half;
        const int p = (int)red[2 * pa], q = (int)red[2 * pa + 1];
        const int r = (int)red[2 * pb], s = (int)red[2 * pb + 1];
        if (q >= m || s >= m) {
          // pairs with the padding index: rotate only the real row/column
          if (q >= m && s >= m) {
          } else if (q >= m) {
            // row p only (c=1,s=0 for pair a); columns rotate by pair b
            const double c2 = cs[pb], s2 = sn[pb];
            const double x0 = G[p * ld + r], x1 = G[p * ld + s];
            G[p * ld + r] = c2 * x0 - s2 * x1;
            G[p * ld + s] = s2 * x0 + c2 * x1;
          } else {
            const double c1 = cs[pa], s1 = sn[pa];
            const double x0 = G[p * ld + r], x1 = G[q * ld + r];
            G[p * ld + r] = c1 * x0 - s1 * x1;
            G[q * ld + r] = s1 * x0 + c1 * x1;
          }
          continue;
        }
        const double c1 = cs[pa], s1 = sn[pa], c2 = cs[pb], s2 = sn[pb];
        const double apr = G[p * ld + r], aps = G[p * ld + s];
        const double aqr = G[q * ld + r], aqs = G[q * ld + s];
        const double x0r = c1 * apr - s1 * aqr, x0s = c1 * aps - s1 * aqs;
        const double x1r = s1 * apr + c1 * aqr, x1s = s1 * aps + c1 * aqs;
        G[p * ld + r] = c2 * x0r - s2 * x0s;
        G[p * ld + s] = s2 * x0r + c2 * x0s;
        G[q * ld + r] = c2 * x1r - s2 * x1s;
        G[q * ld + s] = s2 * x1r + c2 * x1s;
      }
      // U <- U J
      for (int e = threadIdx.x; e < m * half; e += WG) {
        const int i = e / half, pb = e % half;
        const int r = (int)red[2 * pb], s = (int)red[2 * pb + 1];
        if (s >= m) continue;
        const double c2 = cs[pb], s2 = sn[pb];
        const double u0 = U[i * ld + r], u1 = U[i * ld + s];
        U[i * ld + r] = c2 * u0 - s2 * u1;
        U[i * ld + s] = s2 * u0 + c2 * u1;
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  return sweep >= 60 ? -1 : sweep;
}

// Pencils of order up to PLDS keep their matrices in LDS.
constexpr int PLDS = 96;

// ------------------------------------------------------------------------------------------
// Symmetric-definite pencil solves by tridiagonalisation (one workgroup of WG threads).
// With K = R R^T (Cholesky) and G = R^-1 W R^-T, Omega = 2 mu + 1/theta over the eigenpairs of G;
// G = Q T Q^T by Householder reflections (T symmetric tridiagonal), the wanted (largest) theta by
// bisection on Sturm counts of T (the count at 0 gives the number of pp roots), their vectors by
// inverse iteration on T (vectors of nearly equal theta orthonormalised against each other),
// back-transformed by the reflections; c = R^-T u / sqrt(theta), so that c^T W c = +1.
// Two kernels use these steps: k_pencil_energy (the whole spectrum of the small dense pencils,
// W = diag(+-1), matrices in global memory, n up to DMAX; eigenvalues only) and k_pencil_tri
// (the Davidson pencils and the direct path up to order 96, matrices in LDS, W the projected
// metric).
// ------------------------------------------------------------------------------------------
// 1 / b from the hardware reciprocal estimate and two Newton-Raphson steps r <- r (2 - b r)
// (each squares the relative error): a shorter dependent chain than the IEEE division sequence,
// within an ulp or two of it. Magnitudes below 1e-300 (near the denormal range, where the
// estimate is not trusted) take the IEEE division.
__device__ __forceinline__ double recip_nr(double b) {
  if (!(fabs(b) >= 1e-300)) return 1.0 / b;
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  r = fma(r, fma(-b, r, 1.0), r);
  return r;
}

__device__ __forceinline__ int sturm_below(const double* d, const double* e2, int m, double x,
                                           double tiny) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0.0) ++cnt;
#pragma unroll 4
  for (int i = 1; i < m; ++i) {
    if (fabs(q) < tiny) q = -tiny;  // a zero pivot counts as negative (the usual convention)
    q = (d[i] - x) - e2[i - 1] * recip_nr(q);
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__device__ __forceinline__ double block_reduce(double v, double* red, bool is_max) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = is_max ? fmax(v, o) : fmin(v, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < WG / 64; ++w) r = is_max ? fmax(r, red[w]) : fmin(r, red[w]);
  __syncthreads();
  return r;
}

// Cholesky of A (m x m, row-major, ld m) in place: lower R. Returns false if A is not positive
// definite (uniform across the workgroup). col: scratch of m doubles (LDS when A is in global
// memory: the scaled column j is read from there by the trailing update, or null).
__device__ __forceinline__ bool tri_cholesky(double* A, int m, int* flag, double* col = nullptr) {
  const int t = threadIdx.x;
  if (t == 0) *flag = 0;
  __syncthreads();
  const int lane = t & 63, w = t >> 6;
  for (int j = 0; j < m; ++j) {
    const double dj = A[j * m + j];
    if (!(dj > 0.0)) {
      if (t == 0) *flag = 1;
      __syncthreads();
      break;
    }
    const double rjj = sqrt(dj);
    for (int i = j + 1 + t; i < m; i += WG) {
      const double v = A[i * m + j] / rjj;
      A[i * m + j] = v;
      if (col) col[i] = v;
    }
    __syncthreads();
    if (t == 0) A[j * m + j] = rjj;  // no thread reads it in the update below
    // trailing lower triangle: a wave per row, lanes along it
    for (int i = j + 1 + w; i < m; i += WG / 64) {
      const double li = col ? col[i] : A[i * m + j];
      for (int k = j + 1 + lane; k <= i; k += 64)
        A[i * m + k] -= li * (col ? col[k] : A[k * m + j]);
    }
    __syncthreads();
  }
  return *flag == 0;
}

// Ri = R^-1 (lower) by forward substitution, one row at a time, the row's columns in parallel;
// each element's dot product is split over tpe consecutive lanes (as many as the row's i + 1
// elements leave room for), k = c + q, c + q + tpe, ..., and the lane partials are combined by a
// fixed butterfly: dependent chains tpe times shorter. RiT: scratch of m^2 doubles (global
// matrices) that keeps the transposed copy, so that the lanes read column c of R^-1 as a
// contiguous row, or null (matrices in LDS: column c read in place).
__device__ __forceinline__ void tri_inverse(const double* A, double* Ri, int m,
                                            double* RiT = nullptr) {
  const int t = threadIdx.x;
  for (int i = 0; i < m; ++i) {
    const double rii = A[i * m + i];
    const int nc = i + 1;
    const int tpe = nc * 8 <= WG ? 8 : (nc * 4 <= WG ? 4 : (nc * 2 <= WG ? 2 : 1));
    for (int base = 0; base < nc * tpe; base += WG) {
      const int id = base + t;
      const int c = id / tpe, q = id % tpe;
      double s = 0.0;
      if (c < nc) {
        if (RiT) {
          const double* rc = RiT + (size_t)c * m;
          for (int k = c + q; k < i; k += tpe) s += A[i * m + k] * rc[k];
        } else {
          for (int k = c + q; k < i; k += tpe) s += A[i * m + k] * Ri[k * m + c];
        }
      }
      for (int off = 1; off < tpe; off <<= 1) s += __shfl_xor(s, off, 64);
      if (c < nc && q == 0) {
        const double v = ((c == i ? 1.0 : 0.0) - s) / rii;
        Ri[i * m + c] = v;
        if (RiT) RiT[(size_t)c * m + i] = v;
      }
    }
    for (int c = i + 1 + t; c < m; c += WG) Ri[i * m + c] = 0.0;
    __syncthreads();
  }
}

// Householder tridiagonalisation of the symmetric G (m x m, ld m) in place: diagonal d, off-
// diagonal e, reflection k (H = I - beta[k] v v^T acting on rows/cols k+1..) kept in column k
// below the diagonal. vv, vw, pq: LDS scratch of m (vv and vw hold the reflection vectors of
// alternate steps); red: WG doubles.
//
// Step k: p = beta G' v (eight lanes per row), K = beta p^T v / 2 from the waves' partial sums
// (fixed order), G' -= v q^T + q v^T with q = p - K v (a wave per row); the wave that updates
// row k + 1 (the first row of G') then forms the reflection of step k + 1 from that row (by
// symmetry, column k + 1 below the diagonal) while the other waves finish their rows: two
// barriers a step.
__device__ __forceinline__ void tri_reflector(const double* G, int m, int k, double* v, double* d,
                                              double* e, double* beta, int lane) {
  // one wave: x = row k right of the diagonal, |x_1..|^2 by a butterfly, alpha = -sign(x_0) |x|,
  // v = x - alpha e_1, beta = 2 / v^T v (0: already tridiagonal)
  const int s0 = k + 1, ns = m - s0;
  double part = 0.0;
  for (int i = lane; i < ns; i += 64) {
    const double x = G[k * m + s0 + i];
    v[i] = x;
    if (i > 0) part += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if (lane == 0) {
    const double x0 = v[0];
    d[k] = G[k * m + k];
    if (part == 0.0) {
      e[k] = x0;
      beta[k] = 0.0;
    } else {
      const double nrm = sqrt(x0 * x0 + part);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      v[0] = v0;
      e[k] = alpha;
      beta[k] = 2.0 / (v0 * v0 + part);  // H = I - beta v v^T
    }
  }
}

__device__ __forceinline__ void tri_householder(double* G, int m, double* d, double* e, double* beta, double* vv,
                                double* pq, double* red, double* vw) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double* vc = vv;
  double* vn = vw;
  if (m > 2 && w == 0) tri_reflector(G, m, 0, vc, d, e, beta, lane);
  __syncthreads();
  for (int k = 0; k + 2 < m; ++k) {
    const int s0 = k + 1, ns = m - s0;
    const double b = beta[k];
    if (b != 0.0) {  // uniform; else column k is already in tridiagonal form
      // p = b G' v: eight lanes per row, their partials combined by three shuffles; each wave's
      // share of p^T v into red
      double part = 0.0;
      for (int r0 = 0; r0 < ns; r0 += WG / 8) {
        const int i = r0 + (t >> 3), q = t & 7;
        double sum = 0.0;
        if (i < ns) {
          const double* gi = G + (s0 + i) * m + s0;
#pragma unroll 4
          for (int j = q; j < ns; j += 8) sum += gi[j] * vc[j];
        }
        sum += __shfl_xor(sum, 1, 64);
        sum += __shfl_xor(sum, 2, 64);
        sum += __shfl_xor(sum, 4, 64);
        if (q == 0 && i < ns) {
          const double p_ = b * sum;
          pq[i] = p_;
          part += p_ * vc[i];
        }
      }
      part += __shfl_xor(part, 8, 64);
      part += __shfl_xor(part, 16, 64);
      part += __shfl_xor(part, 32, 64);
      if (lane == 0) red[w] = part;
      __syncthreads();
      double kp = 0.0;
      for (int ww = 0; ww < WG / 64; ++ww) kp += red[ww];
      const double K = 0.5 * b * kp;
      // G' -= v q^T + q v^T: a wave per row, lanes along it
      if (ns <= 128) {
        const int j0 = lane, j1 = lane + 64;
        const double vj0 = j0 < ns ? vc[j0] : 0.0, qj0 = j0 < ns ? pq[j0] - K * vj0 : 0.0;
        const double vj1 = j1 < ns ? vc[j1] : 0.0, qj1 = j1 < ns ? pq[j1] - K * vj1 : 0.0;
#pragma unroll 2
        for (int i = w; i < ns; i += WG / 64) {
          const double vi = vc[i], qi = pq[i] - K * vi;
          double* Gi = G + (size_t)(s0 + i) * m + s0;
          if (j0 < ns) Gi[j0] -= vi * qj0 + qi * vj0;
          if (j1 < ns) Gi[j1] -= vi * qj1 + qi * vj1;
        }
      } else {
        for (int i = w; i < ns; i += WG / 64) {
          const double vi = vc[i], qi = pq[i] - K * vi;
          double* Gi = G + (size_t)(s0 + i) * m + s0;
          for (int j = lane; j < ns; j += 64) {
            const double vj = vc[j];
            Gi[j] -= vi * (pq[j] - K * vj) + qi * vj;
          }
        }
      }
      for (int i = t; i < ns; i += WG) G[(s0 + i) * m + k] = vc[i];
    }
    if (w == 0 && k + 3 < m) {
      __threadfence_block();  // row k + 1, just updated by this wave's lanes, read across lanes
      tri_reflector(G, m, k + 1, vn, d, e, beta, lane);
    }
    __syncthreads();
    double* const tmp = vc;
    vc = vn;
    vn = tmp;
  }
  if (t == 0) {
    if (m >= 2) {
      d[m - 2] = G[(m - 2) * m + (m - 2)];
      e[m - 2] = G[(m - 1) * m + (m - 2)];
      beta[m - 2] = 0.0;
    }
    d[m - 1] = G[(m - 1) * m + (m - 1)];
    beta[m - 1] = 0.0;
  }
  __syncthreads();
}

// The nsel eigenvalues of T at the wanted end (channel 0, pp: the largest, theta[0] largest;
// channel 1, hh: the smallest, theta[0] smallest), the count of roots of the channel's sign
// (*npos: positive theta for pp, negative for hh), and their eigenvectors X[j][0..m) (global
// scratch: 4 nsel m doubles from X). e2, lo_s, hi_s (nsel each): LDS scratch; xs: LDS scratch of
// 4 nsel (m | 1) doubles for the inverse iteration (X may be xs itself: the vectors then end in
// its first nsel m doubles), or null (then it works in X). nsel <= WG.
__device__ __forceinline__ void tri_eigen(const double* d, const double* e, double* e2, int m, int nsel,
                          int channel, double* theta, int* npos, double* X, double* red,
                          double* lo_s, double* hi_s, double* xs) {
  const int t = threadIdx.x;
  for (int i = t; i < m; i += WG) e2[i] = i + 1 < m ? e[i] * e[i] : 0.0;
  double lo_p = 1e300, hi_p = -1e300, nrm_p = 0.0;
  for (int i = t; i < m; i += WG) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    lo_p = fmin(lo_p, d[i] - r);
    hi_p = fmax(hi_p, d[i] + r);
    nrm_p = fmax(nrm_p, fabs(d[i]) + r);
  }
  const double gmin = block_reduce(lo_p, red, false);
  const double gmax = block_reduce(hi_p, red, true);
  const double tnorm = fmax(block_reduce(nrm_p, red, true), 1e-300);
  const double tiny = 1e-300 + 2.2e-16 * tnorm * 1e-8;
  if (t == 0) {
    const int nbelow = sturm_below(d, e2, m, 0.0, tiny);
    *npos = channel == 0 ? m - nbelow : nbelow;
  }
  // multisection: root j (the j-th from the wanted end) gets G threads, which evaluate the
  // Sturm count at G interior points of its bracket per round; the bracket shrinks to the two
  // neighbouring points that enclose the root's index, until its width is at the rounding level.
  // The counts are bound by the one CU's FP64 rate: 8 points per round measured faster than 16,
  // 32 or 51 (fewer counts in all)
  const int G = max(1, min(8, WG / max(nsel, 1)));
  for (int j = t; j < nsel; j += WG) {
    lo_s[j] = gmin - 1e-12 * tnorm;
    hi_s[j] = gmax + 1e-12 * tnorm;
  }
  __syncthreads();
  for (int round = 0; round < 200; ++round) {
    const int j = t / G, g = t % G;
    double cnt = -1.0;  // -1: not evaluated
    if (j < nsel) {
      const double lo = lo_s[j], hi = hi_s[j];
      const double x = lo + (hi - lo) * (double)(g + 1) / (double)(G + 1);
      if (hi - lo > 4.4e-16 * fmax(fabs(lo), fabs(hi)) + tiny && x > lo && x < hi)
        cnt = (double)sturm_below(d, e2, m, x, tiny);
    }
    red[t] = cnt;
    __syncthreads();
    int moved = 0;
    if (t < nsel) {
      const int idx = channel == 0 ? m - 1 - t : t;  // ascending index
      const double lo = lo_s[t], hi = hi_s[t];
      double nlo = lo, nhi = hi;
      for (int q = 0; q < G; ++q) {
        const double c = red[t * G + q];
        if (c < 0.0) continue;
        moved = 1;
        const double x = lo + (hi - lo) * (double)(q + 1) / (double)(G + 1);
        if (c <= (double)idx)
          nlo = fmax(nlo, x);
        else
          nhi = fmin(nhi, x);
      }
      if (nlo <= nhi) {
        lo_s[t] = nlo;
        hi_s[t] = nhi;
      }
    }
    if (!__syncthreads_or(moved)) break;
  }
  for (int j = t; j < nsel; j += WG) theta[j] = 0.5 * (lo_s[j] + hi_s[j]);
  __syncthreads();
  // inverse iteration (thread j): (T - theta I) y = b by Gaussian elimination with partial
  // pivoting on the tridiagonal (fill-in: a second superdiagonal), three solves
  // rows of the LDS scratch at an odd stride ms (in doubles), so that the nsel threads' accesses
  // fall in distinct banks; 4 nsel ms doubles
  const int ms = xs ? (m | 1) : m;
  if (t < nsel) {
    double* const base = xs ? xs : X;
    double* y = base + (size_t)t * ms;
    double* U0 = base + (size_t)nsel * ms + (size_t)t * 3 * ms;
    double* U1 = U0 + ms;
    double* U2 = U1 + ms;
    const double th = theta[t];
    const double pert = 2.2e-16 * tnorm;
    unsigned long long h = 0x9E3779B97F4A7C15ull * (unsigned long long)(t + 1);
    for (int i = 0; i < m; ++i) {  // start vector: a fixed pseudo-random sequence per root
      h ^= h >> 33;
      h *= 0xff51afd7ed558ccdull;
      h ^= h >> 33;
      y[i] = 0.5 + (double)(h >> 11) * (1.0 / 9007199254740992.0);
    }
    for (int pass = 0; pass < 3; ++pass) {
      double a_d = d[0] - th, a_u = m > 1 ? e[0] : 0.0, a_u2 = 0.0, rhs = y[0];
      for (int i = 0; i + 1 < m; ++i) {
        const double b_l = e[i], b_d = d[i + 1] - th, b_u = i + 2 < m ? e[i + 1] : 0.0;
        const double rb = y[i + 1];
        if (fabs(a_d) >= fabs(b_l)) {
          double piv = a_d;
          if (fabs(piv) < pert) piv = piv < 0.0 ? -pert : pert;
          const double l = b_l * recip_nr(piv);
          U0[i] = piv;
          U1[i] = a_u;
          U2[i] = a_u2;
          y[i] = rhs;
          a_d = b_d - l * a_u;
          a_u = b_u - l * a_u2;
          a_u2 = 0.0;
          rhs = rb - l * rhs;
        } else {
          const double l = a_d * recip_nr(b_l);  // rows i and i+1 swapped
          U0[i] = b_l;
          U1[i] = b_d;
          U2[i] = b_u;
          y[i] = rb;
          const double nd = a_u - l * b_d, nu = a_u2 - l * b_u;
          a_d = nd;
          a_u = nu;
          a_u2 = 0.0;
          rhs = rhs - l * rb;
        }
      }
      if (fabs(a_d) < pert) a_d = a_d < 0.0 ? -pert : pert;
      U0[m - 1] = a_d;
      U1[m - 1] = 0.0;
      U2[m - 1] = 0.0;
      y[m - 1] = rhs;
      double y1 = 0.0, y2 = 0.0, nrm2 = 0.0;
      for (int i = m - 1; i >= 0; --i) {
        const double v = (y[i] - U1[i] * y1 - U2[i] * y2) * recip_nr(U0[i]);
        y[i] = v;
        y2 = y1;
        y1 = v;
        nrm2 += v * v;
      }
      const double inv = 1.0 / sqrt(nrm2);
      for (int i = 0; i < m; ++i) y[i] *= inv;
    }
    if (xs && X != xs)  // the vector goes on to the orthonormalisation and back-transformation in X
      for (int i = 0; i < m; ++i) X[(size_t)t * m + i] = y[i];
  }
  __syncthreads();
  if (xs && X == xs) {
    // X is the scratch itself: rows of ms -> rows of m, through the free elimination rows
    double* const tmp = xs + (size_t)nsel * ms;
    for (int e_ = t; e_ < nsel * m; e_ += WG) tmp[e_] = xs[(size_t)(e_ / m) * ms + e_ % m];
    __syncthreads();
    for (int e_ = t; e_ < nsel * m; e_ += WG) X[e_] = tmp[e_];
    __syncthreads();
  }
  // vectors of nearly equal theta: orthonormalise in order (modified Gram-Schmidt)
  for (int j = 1; j < nsel; ++j) {
    for (int i = 0; i < j; ++i) {
      if (fabs(theta[i] - theta[j]) > 1e-7 * tnorm) continue;
      double part2 = 0.0;
      for (int r = t; r < m; r += WG) part2 += X[(size_t)i * m + r] * X[(size_t)j * m + r];
      const double dot = block_sum(part2, red);
      for (int r = t; r < m; r += WG) X[(size_t)j * m + r] -= dot * X[(size_t)i * m + r];
      __syncthreads();
      double part3 = 0.0;
      for (int r = t; r < m; r += WG) part3 += X[(size_t)j * m + r] * X[(size_t)j * m + r];
      const double nn = sqrt(block_sum(part3, red));
      for (int r = t; r < m; r += WG) X[(size_t)j * m + r] /= nn;
      __syncthreads();
    }
  }
}

// u = H_0 H_1 ... H_{m-3} y for the nsel vectors X (last reflection first); 16 threads a vector.
__device__ __forceinline__ void tri_back_transform(const double* G, int m, const double* beta, double* X,
                                   int nsel) {
  const int t = threadIdx.x;
  const int ln = t % 16;
  for (int k = m - 3; k >= 0; --k) {
    const double b = beta[k];
    if (b == 0.0) continue;  // uniform
    const int s0 = k + 1, ns = m - s0;
    for (int v0 = 0; v0 < nsel; v0 += WG / 16) {
      const int vj = v0 + t / 16;
      double s = 0.0;
      if (vj < nsel)
        for (int i = ln; i < ns; i += 16) s += G[(s0 + i) * m + k] * X[(size_t)vj * m + s0 + i];
      for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
      if (vj < nsel)
        for (int i = ln; i < ns; i += 16)
          X[(size_t)vj * m + s0 + i] -= b * s * G[(s0 + i) * m + k];
    }
    __syncthreads();
  }
}

// omega[j] (j < nroot) and the columns j < nsel of Cout: c = R^-T u / sqrt|theta| (c^T W c = +1
// for pp, -1 for hh); columns of roots of the other channel are zero. info: [0] 0 ok / 2 fewer
// than nroot roots of the channel, [1] roots of the channel, [2] 0.
__device__ __forceinline__ void tri_outputs(const double* Ri, const double* X, const double* theta, int m,
                            int nroot, int nsel, int npos, double mu2, double* omega,
                            double* Cout, int ldc, int* info) {
  const int t = threadIdx.x;
  for (int j = t; j < nroot; j += WG) omega[j] = j < npos ? mu2 + 1.0 / theta[j] : 0.0;
  for (int e_ = t; e_ < m * nsel; e_ += WG) {
    const int row = e_ / nsel, j = e_ % nsel;
    if (j >= npos) {
      Cout[row * ldc + j] = 0.0;
      continue;
    }
    double s = 0.0;
    for (int k = row; k < m; ++k) s += Ri[k * m + row] * X[(size_t)j * m + k];
    Cout[row * ldc + j] = s / sqrt(fabs(theta[j]));
  }
  if (t == 0) {
    info[0] = npos < nroot ? 2 : 0;
    info[1] = npos;
    info[2] = 0;
  }
}

// Dense pencil (M, W), W = diag(+1 for i < nvv, -1), brought to tridiagonal form: K = M - 2 mu W
// = R R^T (Cholesky, A), Ri = R^-1, G = R^-1 W R^-T (Householder reflections kept in G), T in
// (d, e). Returns false (uniform) if K is not positive definite. work: A, Ri, G (3 m^2).
__device__ __forceinline__ bool dense_pencil_tridiag(const double* __restrict__ M, int m,
                                                     int64_t nvv, double mu2, double* A,
                                                     double* Ri, double* G, double* d, double* e,
                                                     double* beta, double* vv, double* pq,
                                                     double* red, int* flag, double* vw) {
  const int t = threadIdx.x;
  for (int e_ = t; e_ < m * m; e_ += WG) {
    const int i = e_ / m, j = e_ % m;
    A[e_] = M[(size_t)i * m + j] - (i == j ? mu2 * (i < nvv ? 1.0 : -1.0) : 0.0);
  }
  __syncthreads();
  if (!tri_cholesky(A, m, flag, vv)) return false;
  tri_inverse(A, Ri, m, G);  // G holds the transposed copy until G itself is formed
  // G = R^-1 W R^-T with W diagonal (both triangles): element (i, j), i <= j, pair index
  // pe = j (j + 1) / 2 + i, is reduced by 8 consecutive lanes (k = q, q + 8, ... <= i, so each load
  // instruction reads 64-byte segments of rows i and j of R^-1), the lane partials combined by a
  // fixed butterfly
  const int npairs = m * (m + 1) / 2;
  for (int base = 0; base < npairs * 8; base += WG) {
    const int id = base + t, pe = id >> 3, q = id & 7;
    double s = 0.0;
    int i = 0, j = 0;
    if (pe < npairs) {
      j = (int)((sqrt(8.0 * pe + 1.0) - 1.0) * 0.5);
      while ((j + 1) * (j + 2) / 2 <= pe) ++j;  // exact integer row of the pair index
      while (j * (j + 1) / 2 > pe) --j;
      i = pe - j * (j + 1) / 2;
      const double* ri = Ri + (size_t)i * m;
      const double* rj = Ri + (size_t)j * m;
      for (int k = q; k <= i; k += 8) s += ri[k] * (k < nvv ? 1.0 : -1.0) * rj[k];
    }
    for (int off = 1; off < 8; off <<= 1) s += __shfl_xor(s, off, 64);
    if (pe < npairs && q == 0) {
      G[i * m + j] = s;
      G[j * m + i] = s;
    }
  }
  __syncthreads();
  tri_householder(G, m, d, e, beta, vv, pq, red, vw);
  return true;
}

// Correlation energy from the whole spectrum of the dense pencil (section "Total Energy", Eq.
// correlation_energy): every eigenvalue theta of T by bisection (thread t: ascending indices t,
// t + WG, ...), Omega = 2 mu + 1/theta; out[0] = sum over theta > 0 of Omega - Tr A, out[1] =
// -(sum over theta < 0 of Omega) - Tr C (the two sides of the sum rule), out[2] = Tr A,
// out[3] = Tr C. info: [0] 0 ok / 1 not definite, [1] roots with theta > 0, [2] with theta < 0.
// Sums in a fixed order (deterministic). work: 3 m^2.
__global__ __launch_bounds__(WG) void k_pencil_energy(const double* __restrict__ M, int m,
                                                      int64_t nvv, double mu2,
                                                      double* __restrict__ out,
                                                      double* __restrict__ work,
                                                      int* __restrict__ info) {
  __shared__ double red[WG];
  __shared__ double d[DMAX], e[DMAX], e2[DMAX], beta[DMAX], vv[DMAX], pq[DMAX];
  __shared__ int flag;
  const int t = threadIdx.x;
  double* A = work;
  double* Ri = work + (size_t)m * m;
  double* G = work + 2 * (size_t)m * m;
  if (!dense_pencil_tridiag(M, m, nvv, mu2, A, Ri, G, d, e, beta, vv, pq, red, &flag, e2)) {
    if (t == 0) {
      info[0] = 1;
      info[1] = 0;
      info[2] = 0;
    }
    return;
  }
  for (int i = t; i < m; i += WG) e2[i] = i + 1 < m ? e[i] * e[i] : 0.0;
  double lo_p = 1e300, hi_p = -1e300, nrm_p = 0.0;
  for (int i = t; i < m; i += WG) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    lo_p = fmin(lo_p, d[i] - r);
    hi_p = fmax(hi_p, d[i] + r);
    nrm_p = fmax(nrm_p, fabs(d[i]) + r);
  }
  const double gmin = block_reduce(lo_p, red, false);
  const double gmax = block_reduce(hi_p, red, true);
  const double tnorm = fmax(block_reduce(nrm_p, red, true), 1e-300);
  const double tiny = 1e-300 + 2.2e-16 * tnorm * 1e-8;
  double spp = 0.0, shh = 0.0, npp = 0.0, nhh = 0.0, tra = 0.0, trc = 0.0;
  for (int idx = t; idx < m; idx += WG) {
    double lo = gmin - 1e-12 * tnorm, hi = gmax + 1e-12 * tnorm;
    for (int it = 0; it < 200 && hi - lo > 4.4e-16 * fmax(fabs(lo), fabs(hi)) + tiny; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_below(d, e2, m, mid, tiny) <= idx)
        lo = mid;
      else
        hi = mid;
    }
    const double th = 0.5 * (lo + hi);
    const double om = mu2 + 1.0 / th;
    if (th > 0.0) {
      spp += om;
      npp += 1.0;
    } else {
      shh += om;
      nhh += 1.0;
    }
  }
  for (int i = t; i < m; i += WG) {
    if (i < nvv)
      tra += M[(size_t)i * m + i];
    else
      trc += M[(size_t)i * m + i];
  }
  const double SPP = block_sum(spp, red), SHH = block_sum(shh, red);
  const double NPP = block_sum(npp, red), NHH = block_sum(nhh, red);
  const double TA = block_sum(tra, red), TC = block_sum(trc, red);
  if (t == 0) {
    out[0] = SPP - TA;
    out[1] = -SHH - TC;
    out[2] = TA;
    out[3] = TC;
    info[0] = 0;
    info[1] = (int)NPP;
    info[2] = (int)NHH;
  }
}

// ------------------------------------------------------------------------------------------
// Natural transition orbitals and the two-electron density matrix of k roots
// ------------------------------------------------------------------------------------------
// Packed amplitudes onto the triangular matrices X [k][nv][nv] (pp pairs) and Y [k][no][no]
// (hh pairs), which are zero beforehand: entry (p, q) of every packed pair.
__global__ void k_unpack_triangular(const double* __restrict__ Z, int64_t ldz, int64_t n,
                                    int64_t nvv, int nv, int no, const int* __restrict__ ptab,
                                    double* __restrict__ X, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= n) return;
  const int pq = ptab[e];
  const int p = pq >> 16, q = pq & 0xFFFF;
  const double v = Z[(int64_t)r * ldz + e];
  if (e < nvv)
    X[((int64_t)r * nv + p) * nv + q] = v;
  else
    Y[((int64_t)r * no + p) * no + q] = v;
}

// Per root (blockIdx.y): Gt = T^T T and D = sgn (T T^T + T^T T) for the m x m matrices T.
__global__ void k_triangular_products(const double* __restrict__ T, int m, double sgn,
                                      double* __restrict__ Gt, double* __restrict__ D) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  const double* A = T + (int64_t)r * m * m;
  double tt = 0.0, ttt = 0.0;  // (T T^T)_ij, (T^T T)_ij
  for (int c = 0; c < m; ++c) {
    tt += A[i * m + c] * A[j * m + c];
    ttt += A[c * m + i] * A[c * m + j];
  }
  Gt[(int64_t)r * m * m + e] = ttt;
  if (D) D[(int64_t)r * m * m + e] = sgn * (tt + ttt);
}

// G = A^T A of k matrices A (rows x cols, row-major, astride doubles apart): G [k][cols][cols],
// one thread per element, sums in a fixed order.
__global__ void k_gram_ata(const double* __restrict__ Aall, int64_t astride, int rows, int cols,
                           double* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= (int64_t)cols * cols) return;
  const int i = (int)(e / cols), j = (int)(e % cols);
  const double* A = Aall + (int64_t)r * astride;
  double s = 0.0;
  for (int c = 0; c < rows; ++c) s += A[(int64_t)c * cols + i] * A[(int64_t)c * cols + j];
  G[(int64_t)r * cols * cols + e] = s;
}

// The nsel eigenvectors of the largest eigenvalues (descending) of the symmetric m x m matrices
// G (one workgroup per matrix; G overwritten by the Householder reflections): tridiagonal form,
// multisection, inverse iteration (vectors of nearly equal eigenvalues orthonormalised),
// back-transformation. X: per matrix 4 nsel m doubles; the vectors end in its first nsel m
// (row j = vector j). nsel <= 64.
__global__ __launch_bounds__(WG) void k_gram_vectors(double* __restrict__ Gall, int m, int nsel,
                                                     double* __restrict__ Xall) {
  __shared__ double red[WG];
  __shared__ double d[JMAX], e[JMAX], e2[JMAX], beta[JMAX], vv[JMAX], pq[JMAX];
  __shared__ double theta[64];
  __shared__ int npos;
  double* G = Gall + (int64_t)blockIdx.x * m * m;
  double* X = Xall + (int64_t)blockIdx.x * 4 * nsel * m;
  tri_householder(G, m, d, e, beta, vv, pq, red, e2);
  tri_eigen(d, e, e2, m, nsel, 0, theta, &npos, X, red, vv, pq, nullptr);
  tri_back_transform(G, m, beta, X, nsel);
}

// Left singular vectors from the right ones: for root r and vector j, u = A v_j / |A v_j|
// (zero when |A v_j| <= 1e-10 |A v_0|: no left vector for a null direction), the sign fixed so
// that the largest |u_i| (lowest i among equals) is positive, v flipped with it. A: rows x cols at
// astride per root; V: per root 4 nsel cols doubles, vectors in its first nsel cols; U [k][nvec]
// [rows] and Vo [k][nvec][cols], rows nsel .. nvec zero. One workgroup per root.
__global__ __launch_bounds__(NT) void k_svd_left(const double* __restrict__ Aall, int64_t astride,
                                                int rows, int cols, const double* __restrict__ Vall,
                                                int nsel, int nvec, double* __restrict__ Uall,
                                                double* __restrict__ Voall) {
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  const int r = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double* A = Aall + (int64_t)r * astride;
  const double* V = Vall + (int64_t)r * 4 * nsel * cols;
  double* U = Uall + (int64_t)r * nvec * rows;
  double* Vo = Voall + (int64_t)r * nvec * cols;
  double s0 = 0.0;
  for (int j = 0; j < nvec; ++j) {
    if (j >= nsel) {  // uniform
      for (int i = t; i < rows; i += NT) U[(int64_t)j * rows + i] = 0.0;
      for (int i = t; i < cols; i += NT) Vo[(int64_t)j * cols + i] = 0.0;
      continue;
    }
    const double* v = V + (int64_t)j * cols;
    double part = 0.0;
    for (int i = t; i < rows; i += NT) {
      double u = 0.0;
      for (int c = 0; c < cols; ++c) u += A[(int64_t)i * cols + c] * v[c];
      U[(int64_t)j * rows + i] = u;
      part += u * u;
    }
    const double nrm = sqrt(block_sum_nt(part, red));
    if (j == 0) s0 = nrm;
    const bool null_dir = !(nrm > 1e-10 * s0) || nrm == 0.0;
    // the largest |u_i|, lowest i among equals (a fixed reduction order)
    double best = -1.0;
    int bi = 0;
    for (int i = t; i < rows; i += NT) {
      const double a = fabs(U[(int64_t)j * rows + i]);
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      red[w] = best;
      redi[w] = bi;
    }
    __syncthreads();
    double gb = red[0];
    int gi = redi[0];
    for (int ww = 1; ww < NT / 64; ++ww)
      if (red[ww] > gb || (red[ww] == gb && redi[ww] < gi)) {
        gb = red[ww];
        gi = redi[ww];
      }
    const double ug = U[(int64_t)j * rows + gi];
    __syncthreads();
    const double sgn = ug < 0.0 ? -1.0 : 1.0;
    const double us = null_dir ? 0.0 : sgn / nrm;
    for (int i = t; i < rows; i += NT) U[(int64_t)j * rows + i] *= us;
    for (int i = t; i < cols; i += NT) Vo[(int64_t)j * cols + i] = (null_dir ? 1.0 : sgn) * v[i];
    __syncthreads();
  }
}

// Gram matrices of the rectangular amplitude blocks of alpha-beta roots: A = rows x cols
// (row-major, at offset off of root r's packed vector, ld ldz), element e of A A^T (rows^2,
// into G and sgn times it into D) or, for e >= rows^2, of A^T A (cols^2, sgn times it into D
// after the rows^2 block). One thread per element, sums in a fixed order.
__global__ void k_rect_products(const double* __restrict__ Z, int64_t ldz, int64_t off, int rows,
                                int cols, double sgn, double* __restrict__ G,
                                double* __restrict__ D) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int r = blockIdx.y;
  const int64_t m1 = (int64_t)rows * rows, m2 = (int64_t)cols * cols;
  if (e >= m1 + m2) return;
  const double* A = Z + (int64_t)r * ldz + off;
  double s = 0.0;
  if (e < m1) {
    const int i = (int)(e / rows), j = (int)(e % rows);
    for (int c = 0; c < cols; ++c) s += A[(int64_t)i * cols + c] * A[(int64_t)j * cols + c];
    G[(int64_t)r * m1 + e] = s;
  } else {
    const int64_t f = e - m1;
    const int i = (int)(f / cols), j = (int)(f % cols);
    for (int c = 0; c < rows; ++c) s += A[(int64_t)c * cols + i] * A[(int64_t)c * cols + j];
  }
  if (D) D[(int64_t)r * (m1 + m2) + e] = sgn * s;
}

// Eigenvalues of the symmetric m x m matrices G (one workgroup per matrix, blockIdx.x; G is
// overwritten by the Householder reflections), descending and clamped at zero (they are
// squared singular values): lam [k][m].
__global__ __launch_bounds__(WG) void k_gram_eigenvalues(double* __restrict__ Gall, int m,
                                                         double* __restrict__ lam) {
  __shared__ double red[WG];
  __shared__ double d[JMAX], e[JMAX], e2[JMAX], beta[JMAX], vv[JMAX], pq[JMAX];
  const int t = threadIdx.x;
  double* G = Gall + (int64_t)blockIdx.x * m * m;
  tri_householder(G, m, d, e, beta, vv, pq, red, e2);
  for (int i = t; i < m; i += WG) e2[i] = i + 1 < m ? e[i] * e[i] : 0.0;
  double lo_p = 1e300, hi_p = -1e300, nrm_p = 0.0;
  for (int i = t; i < m; i += WG) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    lo_p = fmin(lo_p, d[i] - r);
    hi_p = fmax(hi_p, d[i] + r);
    nrm_p = fmax(nrm_p, fabs(d[i]) + r);
  }
  const double gmin = block_reduce(lo_p, red, false);
  const double gmax = block_reduce(hi_p, red, true);
  const double tnorm = fmax(block_reduce(nrm_p, red, true), 1e-300);
  const double tiny = 1e-300 + 2.2e-16 * tnorm * 1e-8;
  for (int idx = t; idx < m; idx += WG) {
    double lo = gmin - 1e-12 * tnorm, hi = gmax + 1e-12 * tnorm;
    for (int it = 0; it < 200 && hi - lo > 4.4e-16 * fmax(fabs(lo), fabs(hi)) + tiny; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_below(d, e2, m, mid, tiny) <= idx)
        lo = mid;
      else
        hi = mid;
    }
    lam[(int64_t)blockIdx.x * m + (m - 1 - idx)] = fmax(0.5 * (lo + hi), 0.0);
  }
}

// Davidson pencil: Ms, Ws upper triangles (ld ldm). nret columns of Cout (the nroot wanted and
// the next Ritz vectors, kept on restart). A, B, G: m x m matrices (LDS or global; G may alias A:
// then Gt stages G), X: 4 nret m doubles of global scratch (vectors, inverse-iteration rows).
__device__ __forceinline__ void pencil_tri_body(const double* __restrict__ Ms,
                                                const double* __restrict__ Ws, int ldm, int m,
                                                double mu2, int nroot, int nret, int channel,
                                                double* omega, double* Cout, int ldc, double* A,
                                                double* B,
                                                double* G, double* Gt, double* X, int* info,
                                                double* red, double* d, double* e, double* e2,
                                                double* beta, double* vv, double* pq,
                                                double* theta, int* flag, int* npos_s) {
  const int t = threadIdx.x;
  for (int e_ = t; e_ < m * m; e_ += WG) {
    const int i = e_ / m, j = e_ % m;
    const int a = i < j ? i : j, b = i < j ? j : i;
    A[e_] = Ms[a * ldm + b] - mu2 * Ws[a * ldm + b];
  }
  __syncthreads();
  // matrices in global memory (no LDS staging Gt): the Cholesky column goes through LDS (vv)
  // and G's storage, free until G is formed, keeps R^-1 transposed for the substitution
  const bool global = Gt == nullptr;
  if (!tri_cholesky(A, m, flag, global ? vv : nullptr)) {
    if (t == 0) {
      info[0] = 1;
      info[1] = 0;
      info[2] = 0;
    }
    return;
  }
  tri_inverse(A, B, m, global ? G : nullptr);  // B = R^-1
  // Y = R^-1 Wsym into A (R is no longer needed), then G = Y R^-T
  for (int e_ = t; e_ < m * m; e_ += WG) {
    const int i = e_ / m, j = e_ % m;
    double s = 0.0;
    for (int k = 0; k <= i; ++k) {
      const int a = k < j ? k : j, b = k < j ? j : k;
      s += B[i * m + k] * Ws[a * ldm + b];
    }
    A[e_] = s;
  }
  __syncthreads();
  double* Gw = G == A ? Gt : G;
  for (int e_ = t; e_ < m * m; e_ += WG) {
    const int i = e_ / m, j = e_ % m;
    if (j < i) continue;
    double s = 0.0;
    for (int k = 0; k <= j; ++k) s += A[i * m + k] * B[j * m + k];
    Gw[i * m + j] = s;
    Gw[j * m + i] = s;
  }
  __syncthreads();
  if (G == A) {
    for (int e_ = t; e_ < m * m; e_ += WG) G[e_] = Gt[e_];
    __syncthreads();
  }
  tri_householder(G, m, d, e, beta, vv, pq, red, e2);
  const int nsel = nret < m ? nret : m;
  // with the matrices in LDS (Gt given): R^-1 moves to the global staging area and its LDS
  // holds the inverse-iteration rows when they fit (B spans PLDS^2 doubles)
  double* Rinv = B;
  double* xs = nullptr;
  if (Gt && (size_t)4 * nsel * (m | 1) <= (size_t)PLDS * PLDS) {
    for (int e_ = threadIdx.x; e_ < m * m; e_ += WG) Gt[e_] = B[e_];
    __syncthreads();
    Rinv = Gt;
    xs = B;
  }
  // with the inverse-iteration rows in LDS the vectors stay there (the first nsel m doubles of
  // xs) through the orthonormalisation, the back-transformation and the outputs
  double* const Xv = xs ? xs : X;
  tri_eigen(d, e, e2, m, nsel, channel, theta, npos_s, Xv, red, vv, pq, xs);
  tri_back_transform(G, m, beta, Xv, nsel);
  tri_outputs(Rinv, Xv, theta, m, nroot, nsel, *npos_s, mu2, omega, Cout, ldc, info);
}

// m <= PLDS: K, R, G in LDS (G over K); work: m^2 (G staging) + 4 nret m.
__global__ __launch_bounds__(WG) void k_pencil_tri(const double* __restrict__ Ms,
                                                   const double* __restrict__ Ws, int ldm, int m,
                                                   double mu2, int nroot, int nret, int channel,
                                                   double* __restrict__ omega,
                                                   double* __restrict__ Cout, int ldc,
                                                   double* __restrict__ work,
                                                   int* __restrict__ info) {
  __shared__ double sA[PLDS * PLDS];
  __shared__ double sB[PLDS * PLDS];
  __shared__ double red[WG];
  __shared__ double d[PLDS], e[PLDS], e2[PLDS], beta[PLDS], vv[PLDS], pq[PLDS];
  __shared__ double theta[PLDS];
  __shared__ int flag, npos_s;
  pencil_tri_body(Ms, Ws, ldm, m, mu2, nroot, nret, channel, omega, Cout, ldc, sA, sB, sA, work,
                  work + (size_t)m * m, info, red, d, e, e2, beta, vv, pq, theta, &flag, &npos_s);
}

// PLDS < m <= JMAX: matrices L2-resident in work: 3 m^2 + 4 nret m.
__global__ __launch_bounds__(WG) void k_pencil_tri_l2(const double* __restrict__ Ms,
                                                      const double* __restrict__ Ws, int ldm,
                                                      int m, double mu2, int nroot, int nret,
                                                      int channel, double* __restrict__ omega,
                                                      double* __restrict__ Cout, int ldc,
                                                      double* __restrict__ work,
                                                      int* __restrict__ info) {
  __shared__ double red[WG];
  __shared__ double d[JMAX], e[JMAX], e2[JMAX], beta[JMAX], vv[JMAX], pq[JMAX];
  __shared__ double theta[JMAX];
  __shared__ int flag, npos_s;
  const size_t mm = (size_t)m * m;
  pencil_tri_body(Ms, Ws, ldm, m, mu2, nroot, nret, channel, omega, Cout, ldc, work, work + mm,
                  work + 2 * mm, nullptr, work + 3 * mm, info, red, d, e, e2, beta, vv, pq, theta,
                  &flag, &npos_s);
}

// Q = orth(C[:, :r]) by classical Gram-Schmidt applied twice per column (CGS2): in each pass
// the projections on the kept columns come from one set of dot products, each computed by one
// wave over the rows in a fixed order, and are subtracted in column order; columns with relative
// norm below 1e-10 are dropped. Q: [m][ldq], r <= JMAX; rank written to rank[0].
__global__ __launch_bounds__(WG) void k_small_orth(const double* __restrict__ C, int ldc, int m,
                                                   int r, double* __restrict__ Q, int ldq,
                                                   int* __restrict__ rank) {
  __shared__ double red[WG];
  __shared__ double dk[JMAX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int kept = 0;
  for (int j = 0; j < r; ++j) {
    // copy column j into column kept
    for (int i = threadIdx.x; i < m; i += WG) Q[i * ldq + kept] = C[i * ldc + j];
    __syncthreads();
    double n0 = 0.0;
    for (int i = threadIdx.x; i < m; i += WG) n0 += Q[i * ldq + kept] * Q[i * ldq + kept];
    n0 = sqrt(block_sum(n0, red));
    for (int pass = 0; pass < 2 && kept > 0; ++pass) {
      for (int k = wv; k < kept; k += WG / 64) {
        double d = 0.0;
        for (int i = lane; i < m; i += 64) d += Q[i * ldq + k] * Q[i * ldq + kept];
        for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
        if (lane == 0) dk[k] = d;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += WG) {
        double p = 0.0;
        for (int k = 0; k < kept; ++k) p += dk[k] * Q[i * ldq + k];
        Q[i * ldq + kept] -= p;
      }
      __syncthreads();
    }
    double nn = 0.0;
    for (int i = threadIdx.x; i < m; i += WG) nn += Q[i * ldq + kept] * Q[i * ldq + kept];
    nn = sqrt(block_sum(nn, red));
    if (nn > 1e-10 * n0 && nn > 1e-300) {
      for (int i = threadIdx.x; i < m; i += WG) Q[i * ldq + kept] /= nn;
      __syncthreads();
      ++kept;
    }
  }
  if (threadIdx.x == 0) rank[0] = kept;
}

// out = Q^T sym(A) Q, A upper-stored (ld lda), Q [m][ldq] r columns; work m*r.
__global__ __launch_bounds__(WG) void k_congruence(const double* __restrict__ A, int lda, int m,
                                                   const double* __restrict__ Q, int ldq, int r,
                                                   double* __restrict__ out, int ldo,
                                                   double* __restrict__ work) {
  for (int e = threadIdx.x; e < m * r; e += WG) {
    const int i = e / r, j = e % r;
    double s = 0.0;
    for (int k = 0; k < m; ++k) {
      const int a = i < k ? i : k, b = i < k ? k : i;
      s += A[a * lda + b] * Q[k * ldq + j];
    }
    work[e] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * r; e += WG) {
    const int i = e / r, j = e % r;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += Q[k * ldq + i] * work[k * r + j];
    out[i * ldo + j] = s;
  }
}

// Symmetric orthonormalisation of a block from its Gram matrix G (b x b): G = U diag(l) U^T;
// keep l_j > cut * l_max (descending order); Tm[i][jj] = U[i][j] / sqrt(l_j).
__global__ __launch_bounds__(WG) void k_gram_orth(const double* __restrict__ Gin, int ldg, int b,
                                                  double cut, double* __restrict__ Tm, int ldt,
                                                  int* __restrict__ kept,
                                                  double* __restrict__ work) {
  __shared__ double red[WG];
  __shared__ double cs[JMAX / 2 + 1], sn[JMAX / 2 + 1];
  __shared__ int rank_of[JMAX];
  double* G = work;
  double* U = work + (size_t)b * b;
  for (int e = threadIdx.x; e < b * b; e += WG) {
    const int i = e / b, j = e % b;
    G[e] = 0.5 * (Gin[i * ldg + j] + Gin[j * ldg + i]);
  }
  __syncthreads();
  jacobi_eigh(G, b, b, U, red, cs, sn);
  double lmax = 0.0;
  for (int i = 0; i < b; ++i) lmax = fmax(lmax, G[i * b + i]);
  for (int i = threadIdx.x; i < b; i += WG) {
    const double li = G[i * b + i];
    int rk = -1;
    if (li > cut * lmax && li > 1e-280) {
      rk = 0;
      for (int j = 0; j < b; ++j) {
        const double lj = G[j * b + j];
        if (lj > li || (lj == li && j < i)) rk += (lj > cut * lmax && lj > 1e-280);
      }
    }
    rank_of[i] = rk;
  }
  __syncthreads();
  int nk = 0;
  for (int i = 0; i < b; ++i) nk += rank_of[i] >= 0;
  for (int e = threadIdx.x; e < b * b; e += WG) {
    const int row = e / b, i = e % b;
    const int rk = rank_of[i];
    if (rk >= 0) Tm[row * ldt + rk] = U[row * b + i] / sqrt(G[i * b + i]);
  }
  if (threadIdx.x == 0) kept[0] = nk;
}

}  // namespace

// ==========================================================================================
// Launchers
// ==========================================================================================
hipError_t launch_dots(const double* A, int64_t lda, int ma, const double* B, int64_t ldb, int mb,
                       int64_t n, int64_t nsign, int signed_w, double* C, int ldc, double* part,
                       int nchunk, hipStream_t s) {
  if (ma <= 0 || mb <= 0) return hipSuccess;
  if (n <= 0) return hipErrorInvalidValue;
  // chunks of at least 64 along t (a multiple of the 16-wide step); part holds nchunk * ma * mb
  int64_t chunk = (n + nchunk - 1) / nchunk;
  chunk = std::max<int64_t>(64, (chunk + DOT_STEP - 1) / DOT_STEP * DOT_STEP);
  const int nch = (int)((n + chunk - 1) / chunk);
  const int units = ((ma + 15) / 16) * ((mb + 63) / 64);
  const int waves = std::min(units, DOT_WAVES);
  hipLaunchKernelGGL(k_dots, dim3(nch), dim3(64 * waves), 0, s, A, lda, ma, B, ldb, mb, n, nsign,
                     signed_w, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_reduce, dim3((ma * mb + 15) / 16), dim3(256), 0, s, part, nch, ma,
                     mb, C, ldc);
  return hipGetLastError();
}

hipError_t launch_combine(const double* X, int64_t ldx, int m, const double* Cm, int ldcm, int r,
                          int64_t n, double alpha, double beta, double* Y, int64_t ldy,
                          hipStream_t s) {
  if (r <= 0 || n <= 0) return hipSuccess;
  if (r > ldcm) return hipErrorInvalidValue;
  const int64_t per_block = (int64_t)16 * CMB_CT * CMB_WAVES;
  dim3 grid((unsigned)((n + per_block - 1) / per_block)), block(64 * CMB_WAVES);
  // one launch per 64 output rows (a restart keeps up to 2 nroot = 128 vectors): rows j0.. of Y
  // from columns j0.. of Cm, each row's sum in the same order as in a single launch
  for (int j0 = 0; j0 < r; j0 += 64) {
    const int rj = r - j0 < 64 ? r - j0 : 64;
    const double* Cj = Cm + j0;
    double* Yj = Y + (int64_t)j0 * ldy;
    switch ((rj + 15) / 16) {
      case 1: hipLaunchKernelGGL(k_combine<1>, grid, block, 0, s, X, ldx, m, Cj, ldcm, rj, n, alpha, beta, Yj, ldy); break;
      case 2: hipLaunchKernelGGL(k_combine<2>, grid, block, 0, s, X, ldx, m, Cj, ldcm, rj, n, alpha, beta, Yj, ldy); break;
      case 3: hipLaunchKernelGGL(k_combine<3>, grid, block, 0, s, X, ldx, m, Cj, ldcm, rj, n, alpha, beta, Yj, ldy); break;
      default: hipLaunchKernelGGL(k_combine<4>, grid, block, 0, s, X, ldx, m, Cj, ldcm, rj, n, alpha, beta, Yj, ldy); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_residual(const double* Z, const double* SZ, int64_t ld, int r, int64_t n,
                           int64_t nvv, const double* d_omega, double* R, double* part_norm,
                           int nchunk, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(nchunk, r), dim3(NT), 0, s, Z, SZ, ld, n, nvv, d_omega, R,
                     part_norm);
  return hipGetLastError();
}

hipError_t launch_reduce_norms(const double* part, int nchunk, int r, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_norms, dim3((r + 63) / 64), dim3(64), 0, s, part, nchunk, r, out);
  return hipGetLastError();
}

hipError_t launch_precond(const double* R, int64_t ld, const int* h_sel, int nsel, int64_t n,
                          int64_t nvv, const double* d_diag, const double* d_omega, double* T,
                          int64_t ldt, hipStream_t s) {
  if (nsel <= 0) return hipSuccess;
  if (nsel > 64) return hipErrorInvalidValue;
  SelList sl;
  for (int i = 0; i < 64; ++i) sl.idx[i] = i < nsel ? h_sel[i] : 0;
  const int nb = (int)std::min<int64_t>((n + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_precond, dim3(nb, nsel), dim3(NT), 0, s, R, ld, sl, n, nvv, d_diag,
                     d_omega, T, ldt);
  return hipGetLastError();
}

hipError_t launch_pencil(const double* Ms, const double* Ws, int ldm, int m, double mu2,
                         int nroot, int nret, int channel, double* omega, double* Cout, int ldc,
                         double* work, int* info, hipStream_t s) {
  if (m > JMAX || nret > m || nroot > nret || nret > WG || (channel != 0 && channel != 1))
    return hipErrorInvalidValue;
  if (m <= PLDS)
    hipLaunchKernelGGL(k_pencil_tri, dim3(1), dim3(WG), 0, s, Ms, Ws, ldm, m, mu2, nroot, nret,
                       channel, omega, Cout, ldc, work, info);
  else
    hipLaunchKernelGGL(k_pencil_tri_l2, dim3(1), dim3(WG), 0, s, Ms, Ws, ldm, m, mu2, nroot, nret,
                       channel, omega, Cout, ldc, work, info);
  return hipGetLastError();
}

hipError_t launch_pencil_energy(const double* M, int m, int64_t nvv, double mu2, double* out,
                                double* work, int* info, hipStream_t s) {
  if (m < 1 || m > DMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pencil_energy, dim3(1), dim3(WG), 0, s, M, m, nvv, mu2, out, work, info);
  return hipGetLastError();
}

hipError_t launch_unpack_triangular(const double* Z, int64_t ldz, int k, const Geometry& g,
                                    const int* ptab, double* X, double* Y, hipStream_t s) {
  const size_t xv = (size_t)k * g.nv * g.nv, yo = (size_t)k * g.no * g.no;
  hipError_t e = launch_fill(X, xv, 0.0, s);
  if (e == hipSuccess && yo) e = launch_fill(Y, yo, 0.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpack_triangular, dim3((unsigned)((g.n + NT - 1) / NT), k), dim3(NT), 0, s,
                     Z, ldz, g.n, g.nvv, g.nv, g.no, ptab, X, Y);
  return hipGetLastError();
}

size_t svd_vectors_work(int k, int rows, int cols, int nvec) {
  const int nsel = std::min(nvec, std::min(rows, cols));
  return (size_t)k * cols * cols + (size_t)k * 4 * std::max(nsel, 1) * cols;
}

hipError_t launch_svd_vectors(const double* A, int64_t astride, int rows, int cols, int k,
                              int nvec, double* work, double* U, double* V, hipStream_t s) {
  if (k < 1 || rows < 1 || cols < 1 || rows > JMAX || cols > JMAX || nvec < 1 || nvec > 64)
    return hipErrorInvalidValue;
  const int nsel = std::min(nvec, std::min(rows, cols));
  double* G = work;
  double* X = work + (size_t)k * cols * cols;
  const int64_t ev = (int64_t)cols * cols;
  hipLaunchKernelGGL(k_gram_ata, dim3((unsigned)((ev + NT - 1) / NT), k), dim3(NT), 0, s, A,
                     astride, rows, cols, G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_vectors, dim3(k), dim3(WG), 0, s, G, cols, nsel, X);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_svd_left, dim3(k), dim3(NT), 0, s, A, astride, rows, cols, X, nsel, nvec, U,
                     V);
  return hipGetLastError();
}

hipError_t launch_nto_ab(const double* Z, int64_t ldz, int k, int nva, int nvb, int noa, int nob,
                         double* Gx, double* Gy, double* Dv, double* Do, double* lam_p,
                         double* lam_h, hipStream_t s) {
  if (k < 1 || nva > JMAX || nvb > JMAX || noa > JMAX || nob > JMAX) return hipErrorInvalidValue;
  const int64_t nvv = (int64_t)nva * nvb;
  const int64_t ev = (int64_t)nva * nva + (int64_t)nvb * nvb;
  hipLaunchKernelGGL(k_rect_products, dim3((unsigned)((ev + NT - 1) / NT), k), dim3(NT), 0, s, Z,
                     ldz, (int64_t)0, nva, nvb, 1.0, Gx, Dv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_eigenvalues, dim3(k), dim3(WG), 0, s, Gx, nva, lam_p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (noa > 0) {
    const int64_t eo = (int64_t)noa * noa + (int64_t)nob * nob;
    hipLaunchKernelGGL(k_rect_products, dim3((unsigned)((eo + NT - 1) / NT), k), dim3(NT), 0, s,
                       Z, ldz, nvv, noa, nob, -1.0, Gy, Do);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_eigenvalues, dim3(k), dim3(WG), 0, s, Gy, noa, lam_h);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_nto(const double* Z, int64_t ldz, int k, const Geometry& g, const int* ptab,
                      double* X, double* Y, double* Gx, double* Gy, double* Dv, double* Do,
                      double* lam_p, double* lam_h, hipStream_t s) {
  if (k < 1 || g.nv > JMAX || g.no > JMAX) return hipErrorInvalidValue;
  const size_t xv = (size_t)k * g.nv * g.nv, yo = (size_t)k * g.no * g.no;
  hipError_t e = launch_fill(X, xv, 0.0, s);
  if (e == hipSuccess && yo) e = launch_fill(Y, yo, 0.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpack_triangular, dim3((unsigned)((g.n + NT - 1) / NT), k), dim3(NT), 0, s,
                     Z, ldz, g.n, g.nvv, g.nv, g.no, ptab, X, Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t mv = (int64_t)g.nv * g.nv, mo = (int64_t)g.no * g.no;
  hipLaunchKernelGGL(k_triangular_products, dim3((unsigned)((mv + NT - 1) / NT), k), dim3(NT), 0, s,
                     X, g.nv, 1.0, Gx, Dv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_eigenvalues, dim3(k), dim3(WG), 0, s, Gx, g.nv, lam_p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (g.no > 0) {
    hipLaunchKernelGGL(k_triangular_products, dim3((unsigned)((mo + NT - 1) / NT), k), dim3(NT), 0,
                       s, Y, g.no, -1.0, Gy, Do);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_eigenvalues, dim3(k), dim3(WG), 0, s, Gy, g.no, lam_h);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_small_orth(const double* C, int ldc, int m, int r, double* Q, int ldq,
                             int* rank, hipStream_t s) {
  if (r > JMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_small_orth, dim3(1), dim3(WG), 0, s, C, ldc, m, r, Q, ldq, rank);
  return hipGetLastError();
}

hipError_t launch_small_congruence(const double* Ms, int ldm, int m, const double* Q, int ldq,
                                   int r, double* out, int ldo, double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_congruence, dim3(1), dim3(WG), 0, s, Ms, ldm, m, Q, ldq, r, out, ldo, work);
  return hipGetLastError();
}

hipError_t launch_gram_orth(const double* G, int ldg, int b, double cut, double* Tm, int ldt,
                            int* kept, double* work, hipStream_t s) {
  if (b > JMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gram_orth, dim3(1), dim3(WG), 0, s, G, ldg, b, cut, Tm, ldt, kept, work);
  return hipGetLastError();
}

hipError_t launch_scale_sign(double* V, int64_t ld, int r, int64_t n, hipStream_t s) {
  if (r <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_sign, dim3(r), dim3(NT), 0, s, V, ld, n);
  return hipGetLastError();
}

hipError_t launch_normalize_rows(double* V, int64_t ld, int r, int64_t n, hipStream_t s) {
  if (r <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize_rows, dim3(r), dim3(NRM_T), 0, s, V, ld, n);
  return hipGetLastError();
}

hipError_t prepare_kernels() { return hipSuccess; }

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)std::min<size_t>((n + NT - 1) / NT, 4096);
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(NT), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace pprpa
