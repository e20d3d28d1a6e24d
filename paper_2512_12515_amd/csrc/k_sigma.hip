// Density-fitted ppRPA sigma product on CDNA4 (gfx950): staging, unpack, the fused
// two-contraction "sandwich" kernel on MFMA, and the epilogue.
//
// Method (arXiv 2512.12515, section "ppRPA Equation", spin-adapted A, B, C; <pq|rs> = (pr|qs)):
// with the packed pair vector z = [x; y] unpacked into full matrices
//   Xh (nv x nv): Xh[a][b] = x_ab (a<b), Xh[b][a] = s x_ab, Xh[a][a] = sqrt2 x_aa (singlet; s=+1)
//                 or 0 (triplet; s=-1);  Yh (no x no) likewise,
// and Zh = blockdiag(Xh, Yh) over the active orbitals ordered [virtual; occupied],
//   S = sum_P L^P Zh L^P    (L^P the symmetric nact x nact slice of the three-centre tensor)
// holds in its virtual-virtual block A'x + B y and in its occupied-occupied block B^T x + C'y
// (primes: interaction parts), up to the 1/sqrt2 factor of diagonal singlet pairs:
//   sigma_x(ab) = (e_a+e_b) x_ab + N_ab S[a][b],   sigma_y(ij) = -(e_i+e_j) y_ij + N_ij S[i][j].
// The vv block alone is (ac|bd) X_cd = sum_P L^P_ac (sum_d L^P_bd X_cd); the B blocks come out
// of the occupied-virtual parts of L^P.
//
// Kernel design (one workgroup = 4 waves; MFMA 16x16x4, FP64 or FP32):
//   * the product is computed as Q = sum_P L^P U L^P with U the upper triangle of Zh (diagonal
//     halved for the singlet, zero for the triplet), so that the S block is Q + s Q^T (formed in
//     the epilogue); the triangle halves contraction 1 and every work unit does the same work;
//   * a workgroup owns one vector, a panel of up to 4 adjacent 16-column tiles of one diagonal
//     block, a range of up to RT row tiles of that block, and a contiguous range of the aux
//     index P; wave w owns column tile w of the panel (in a panel of one or two tiles the
//     waves of a column share out its c groups in contraction 1, exchange their T tiles through
//     LDS, and share out its rows in contraction 2);
//   * per P: contraction 1, T[c][cols] = sum_{d >= c} U[c][d] L^P[d][cols], accumulates in
//     registers (CT row tiles of T at a time); contraction 2, Q[r][cols] += sum_c L^P[r][c]
//     T[c][cols], takes T straight from those registers as its B operand (the reduction index c
//     is permuted to match the MFMA output layout, acc_row, and the A operand is read with the
//     same permutation), so T stays in the register file (narrow panels aside);
//   * the A operands (rows of U^T and of L^P) are shared by the 4 waves and staged in LDS by
//     direct global-to-LDS loads; L^P being symmetric, every staged tile is a contiguous row
//     segment in HBM;
//   * the aux index is split over workgroups; partial Q per split are summed in the epilogue in
//     a fixed order (deterministic);
//   * workgroup ids are remapped so the 8 XCDs each take a contiguous range of work units; the
//     vector index runs fastest within it, so the units of one (panel, P range) over all vectors
//     run at the same time on one XCD and read its L^P tiles from that XCD's L2.
#include "internal.h"
#include "sigma_common.h"
#include "sigma_bf16.h"

namespace pprpa {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

template <typename T> struct AccT;
template <> struct AccT<double> { using V = d4; };
template <> struct AccT<float> { using V = f4; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row (within the 16-row output tile) of accumulator register j in lane group lk (lane / 16),
// measured on gfx950: FP64 16x16x4 places row lk + 4 j in register j; FP32 (and BF16) 16x16x4
// place row 4 lk + j.
template <typename T> __device__ __forceinline__ int acc_row(int lk, int j);
template <> __device__ __forceinline__ int acc_row<double>(int lk, int j) { return lk + 4 * j; }
template <> __device__ __forceinline__ int acc_row<float>(int lk, int j) { return 4 * lk + j; }


// ------------------------------------------------------------------------------------------
// Staging of L into the padded [P][nmop][nmop] layout in the sigma precision.
// src[r] = row index in the input tensor for padded index r, or -1 for padding.
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_stage_L(const double* __restrict__ Lin, int nin, int p0,
                          const int* __restrict__ src, int nmop, T* __restrict__ Lout,
                          int* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nmop * nmop) return;
  const int P = blockIdx.y;
  const int r = (int)(e / nmop), c = (int)(e % nmop);
  const int sr = src[r], sc = src[c];
  double v = 0.0;
  if (sr >= 0 && sc >= 0) {
    v = Lin[((int64_t)P * nin + sr) * nin + sc];
    if (!__builtin_isfinite(v)) {
      atomicOr(bad, 1);
      v = 0.0;
    }
  }
  Lout[((int64_t)(p0 + P) * nmop + r) * nmop + c] = (T)v;
}

// BF16 planes: hi = bf16(v), mid = bf16(v - hi), lo = bf16(v - hi - mid) (round to nearest even,
// residuals formed in FP64).
__global__ void k_stage_L_bf16(const double* __restrict__ Lin, int nin, int p0,
                               const int* __restrict__ src, int nmop,
                               unsigned short* __restrict__ Lout, size_t plane,
                               int* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nmop * nmop) return;
  const int P = blockIdx.y;
  const int r = (int)(e / nmop), c = (int)(e % nmop);
  const int sr = src[r], sc = src[c];
  double v = 0.0;
  if (sr >= 0 && sc >= 0) {
    v = Lin[((int64_t)P * nin + sr) * nin + sc];
    if (!__builtin_isfinite(v)) {
      atomicOr(bad, 1);
      v = 0.0;
    }
  }
  const unsigned short h = bf16_rne((float)v);
  const double r1 = v - (double)bf16_to_f(h);
  const unsigned short m = bf16_rne((float)r1);
  const double r2 = r1 - (double)bf16_to_f(m);
  const unsigned short l = bf16_rne((float)r2);
  const size_t o = ((size_t)(p0 + P) * nmop + r) * nmop + c;
  Lout[o] = h;
  Lout[o + plane] = m;
  Lout[o + 2 * plane] = l;
}

__global__ void k_check_finite(const double* __restrict__ x, size_t n, int* __restrict__ bad) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    if (!__builtin_isfinite(x[i])) atomicOr(bad, 1);
}

// ------------------------------------------------------------------------------------------
// Unpack packed vectors into UT[k][nmop][nmop] = U^T (only the two diagonal blocks written; the
// off-diagonal blocks stay zero from allocation).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double unpacked_value(const double* __restrict__ zk, int nb, int mult,
                                                 int c, int d) {
  // U[c][d], the upper triangle of the unpacked block (Zh = U + s U^T): x_cd for c < d; on the
  // diagonal half of Zh[c][c] = sqrt2 x_cc (singlet), 0 (triplet); 0 below the diagonal.
  if (c >= nb || d >= nb || c > d) return 0.0;
  if (mult == 0) {
    const int64_t idx = (int64_t)c * nb - (int64_t)c * (c - 1) / 2 + (d - c);
    const double v = zk[idx];
    return c == d ? v * 0.70710678118654752440 : v;
  }
  if (c == d) return 0.0;
  const int64_t idx = (int64_t)c * (nb - 1) - (int64_t)c * (c - 1) / 2 + (d - c - 1);
  return zk[idx];
}

template <typename T>
__global__ void k_unpack(const double* __restrict__ z, int64_t n, int64_t nvv, int nv, int no,
                         int nvp, int nop, int nmop, int mult, T* __restrict__ ZT) {
  const int kv = blockIdx.y;
  int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nvb = (int64_t)nvp * nvp;
  int d, c, off;
  double v;
  if (e < nvb) {
    d = (int)(e / nvp);
    c = (int)(e % nvp);
    off = 0;
    v = unpacked_value(z + (int64_t)kv * n, nv, mult, c, d);
  } else {
    e -= nvb;
    if (e >= (int64_t)nop * nop) return;
    d = (int)(e / nop);
    c = (int)(e % nop);
    off = nvp;
    v = unpacked_value(z + (int64_t)kv * n + nvv, no, mult, c, d);
  }
  ZT[((int64_t)kv * nmop + off + d) * nmop + off + c] = (T)v;
}

// BF16 planes of U (not transposed: the BF16 kernel reads 8 consecutive d of a row c).
__global__ void k_unpack_bf16(const double* __restrict__ z, int64_t n, int64_t nvv, int nv,
                              int no, int nvp, int nop, int nmop, int mult,
                              unsigned short* __restrict__ ZT, size_t zplane) {
  const int kv = blockIdx.y;
  int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nvb = (int64_t)nvp * nvp;
  int d, c, off;
  double v;
  if (e < nvb) {
    d = (int)(e / nvp);
    c = (int)(e % nvp);
    off = 0;
    v = unpacked_value(z + (int64_t)kv * n, nv, mult, c, d);
  } else {
    e -= nvb;
    if (e >= (int64_t)nop * nop) return;
    d = (int)(e / nop);
    c = (int)(e % nop);
    off = nvp;
    v = unpacked_value(z + (int64_t)kv * n + nvv, no, mult, c, d);
  }
  const unsigned short h = bf16_rne((float)v);
  const double r1 = v - (double)bf16_to_f(h);
  const unsigned short m = bf16_rne((float)r1);
  const double r2 = r1 - (double)bf16_to_f(m);
  const unsigned short l = bf16_rne((float)r2);
  const size_t o = ((size_t)kv * nmop + off + c) * nmop + off + d;  // U itself, row c
  ZT[o] = h;
  ZT[o + zplane] = m;
  ZT[o + 2 * zplane] = l;
}

// ------------------------------------------------------------------------------------------
// Fused sandwich kernel (FP64 / FP32 MFMA).
// ------------------------------------------------------------------------------------------


template <typename T, int CT, int RT>
struct SandCfg {
  // LDS tiles are packed row-major (row stride = staged width) because direct global->LDS loads
  // write each wave's 64 x 16 bytes contiguously.
  static constexpr int SR1 = 3 * TILE;                            // contraction-1 rows (3 tiles)
  static constexpr int SR = 2 * TILE;                             // contraction-2 rows (2 tiles)
  static constexpr int S1 = SR1 * CT * TILE + SR1 * 4 * TILE;    // contraction-1 stage
  static constexpr int S2 = SR * RT * TILE;                      // contraction-2 stage, full rows
  // elements per LDS buffer (two workgroups per CU leave room for small kernels beside them; a
  // contraction-2 stage holds as many c tiles as fit at its row width)
  static constexpr int BUF = S1 > S2 ? S1 : S2;
  static constexpr int VEC = 16 / sizeof(T);                     // elements per lane per load
  static constexpr int CHUNK = 1024 / sizeof(T);                 // elements per wave load
};

// Q = sum_P L^P U L^P for one vector, a panel of up to 4 column tiles of one diagonal block and a
// range of up to RT row tiles of that block (U: upper triangle of the unpacked vector; the sigma
// block is Q + s Q^T, formed in the epilogue). Every wave of a panel does the same work. Each
// stage is staged by direct global->LDS loads into one buffer; two workgroups per CU overlap one
// another's staging with their MFMA work.
// Work unit u of one sigma product (u < a.nunits): unit -> (work item, vector, aux split).
template <typename T, int CT, int RT>
__device__ __forceinline__ void sandwich_unit(const T* __restrict__ L, const T* __restrict__ UT,
                                              T* __restrict__ Qp, const SandParams& a, int u,
                                              T* __restrict__ buf) {
  using V = typename AccT<T>::V;
  using Cfg = SandCfg<T, CT, RT>;
  constexpr int GRP = 2;  // tiles per unrolled MFMA group
  static_assert(CT % GRP == 0 && RT % GRP == 0, "tile groups");
  static_assert(2 * CT * 4 * 64 <= Cfg::BUF, "T exchange of a two-column panel fits the buffer");
  static_assert(2 * TILE * RT * TILE <= Cfg::BUF && 2 * TILE * (RT - 1) * TILE + TILE <= Cfg::BUF,
                "two contraction-2 c tiles at any row count");

  const int item = a.items[(u / a.k) % a.nitems];
  const int kv = u % a.k;
  const int sp = u / (a.nitems * a.k);
  const int pn = item >> 16;
  const int R0 = item & 0xFFFF;  // first row tile of the range (local to the block)

  const bool vblk = pn < a.npan_v;
  const int t0 = vblk ? 4 * pn : 4 * (pn - a.npan_v);
  const int bnt = vblk ? a.nvt : (a.nct - a.nvt);
  const int brow0 = vblk ? 0 : a.nvp;
  const int npt = min(4, bnt - t0);
  // the wave index is uniform: kept in a scalar register, the per-wave conditions below become
  // scalar branches
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  // a panel of one or two column tiles puts parts = 4 / npt waves on each column: in
  // contraction 1 they share out the column's c groups (g % parts == rsel), exchange their T
  // tiles through LDS, and in contraction 2 they share out its row groups the same way; a
  // three-tile panel idles one wave
  const int parts = npt == 1 ? 4 : (npt == 2 ? 2 : 1);
  const bool active = w < npt * parts;
  const int wc = parts == 1 ? min(w, npt - 1) : w % npt;  // column tile (idle waves: the last)
  const int rsel = parts == 1 ? 0 : w / npt;               // c and row groups g with g % parts == rsel
  const int rend = min(bnt, R0 + RT);
  const int nrt = rend - R0;
  const int col0 = brow0 + t0 * TILE;
  const int ncol = npt * TILE;
  const int row0 = brow0 + R0 * TILE;
  const int wl = nrt * TILE;  // row stride of a staged L^P row tile (contraction 2)
  // c tiles per contraction-2 stage: FP32 takes as many as the buffer holds at this row width
  // (>= 2; with an odd row count TILE elements stay free past the last one for the unused second
  // tile of the last row group), FP64 two (wider FP64 stages measured ~1 % slower in the solve)
  const int nb2 = sizeof(T) == 8 ? 2 : min(CT, (Cfg::BUF - ((nrt & 1) ? TILE : 0)) / (TILE * wl));
  const int P0 = (int)((int64_t)a.naux * sp / a.nsplit);
  const int P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  const T* __restrict__ Z = UT + (int64_t)kv * a.zstride;

  V S[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) S[r] = V{0, 0, 0, 0};

  T* const sB = buf + Cfg::SR1 * CT * TILE;
  for (int P = P0; P < P1; ++P) {
    const T* __restrict__ Lp = L + (int64_t)P * a.zstride;
    for (int cc0 = 0; cc0 < a.nct; cc0 += CT) {
      const int cc1 = min(cc0 + CT, a.nct);
      V Tacc[CT];
#pragma unroll
      for (int i = 0; i < CT; ++i) Tacc[i] = V{0, 0, 0, 0};
      // contraction 1: T[c][cols] = sum_{d >= c} U[c][d] L^P[d][cols], d in c's block, three d
      // tiles per stage
      for (int part = 0; part < 2; ++part) {
        const int lo = part == 0 ? cc0 : max(cc0, a.nvt);
        const int hi = part == 0 ? (cc0 < a.nvt ? a.nvt : cc0) : (cc1 > a.nvt ? a.nct : lo);
        for (int dt = lo; dt < hi; dt += 3) {
          const int nd = min(3, hi - dt);
          int g0, g1, h0, h1;
          c_range(dt, cc0, cc1, a.nvt, &g0, &g1);
          c_range(dt + nd - 1, cc0, cc1, a.nvt, &h0, &h1);
          const int wa = (h1 - g0) * TILE;
          __syncthreads();
          dma_tile(Z + (int64_t)(dt * TILE) * a.nmop + g0 * TILE, a.nmop, nd * TILE, wa, buf, w, lane);
          dma_tile(Lp + (int64_t)(dt * TILE) * a.nmop + col0, a.nmop, nd * TILE, ncol, sB, w, lane);
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
#pragma unroll
          for (int sub = 0; sub < 3; ++sub) {
            if (sub < nd) {
              int q0, q1g;
              c_range(dt + sub, cc0, cc1, a.nvt, &q0, &q1g);
              const int q1 = min(cc1, dt + sub + 1);  // end of the nonzero c tiles (c <= d)
              const T* sA = buf + sub * TILE * wa;
              const T* sBs = sB + sub * TILE * ncol;
              T bv[4];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) bv[ks] = sBs[(4 * ks + lk) * ncol + wc * TILE + li];
#pragma unroll
              for (int grp = 0; grp < CT / GRP; ++grp) {
                const int cg = cc0 + GRP * grp;
                // groups that reach past d multiply exact zeros of U^T (c > d)
                if (active && cg >= q0 && cg < q1 && grp % parts == rsel) {
                  // all four k steps of the group's A operands first: one LDS wait per group
                  T av[4][GRP];
#pragma unroll
                  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = 0; j < GRP; ++j)
                      av[ks][j] = sA[(4 * ks + lk) * wa + (cg - g0 + j) * TILE + li];
                  __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
#pragma unroll
                  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = 0; j < GRP; ++j)
                      Tacc[GRP * grp + j] = mfma(av[ks][j], bv[ks], Tacc[GRP * grp + j]);
                }
              }
            }
          }
        }
      }
      if (parts > 1) {
        // narrow panel: every wave of a column takes the T tiles of the other waves' c groups
        // (same values, same summation order as computing them itself); layout [col][tile][reg]
        // [lane], conflict-free
        T* const sT = buf;
        __syncthreads();  // contraction-1 operands no longer read
#pragma unroll
        for (int i = 0; i < CT; ++i)
          if ((i / GRP) % parts == rsel)
#pragma unroll
            for (int j = 0; j < 4; ++j) sT[((wc * CT + i) * 4 + j) * 64 + lane] = Tacc[i][j];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < CT; ++i)
          if ((i / GRP) % parts != rsel)
#pragma unroll
            for (int j = 0; j < 4; ++j) Tacc[i][j] = sT[((wc * CT + i) * 4 + j) * 64 + lane];
      }
      // contraction 2: Q[r][cols] += sum_c L^P[r][c] T[c][cols], T from registers, nb2 c tiles
      // per stage
      // slot of c tile i in its stage: i % 2 for FP64 (known at compile time), a running count
      // for FP32 (a run-time i % nb2 made the FP32 kernel ~15 % slower)
      int run = 0;
#pragma unroll
      for (int i = 0; i < CT; ++i) {
        if (cc0 + i < cc1) {
          const int slot = sizeof(T) == 8 ? i % 2 : run;
          if (slot == 0) {
            const int nb = min(nb2, cc1 - cc0 - i);
            __syncthreads();
            dma_tile(Lp + (int64_t)((cc0 + i) * TILE) * a.nmop + row0, a.nmop, nb * TILE, wl, buf, w, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
          }
          const T* sL = buf + slot * TILE * wl;
#pragma unroll
          for (int grp = 0; grp < RT / GRP; ++grp) {
            // row tiles at or beyond nrt in the last group read other data of the buffer (in
            // bounds); their results are never stored
            if (active && GRP * grp < nrt && grp % parts == rsel) {
              T av[4][GRP];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                for (int j = 0; j < GRP; ++j)
                  av[ks][j] = sL[acc_row<T>(lk, ks) * wl + (GRP * grp + j) * TILE + li];
              __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
#pragma unroll
              for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                for (int j = 0; j < GRP; ++j)
                  S[GRP * grp + j] = mfma(av[ks][j], Tacc[i][ks], S[GRP * grp + j]);
            }
          }
          run = run + 1 == nb2 ? 0 : run + 1;
        }
      }
    }
  }

  if (active) {
    T* __restrict__ out = Qp + ((int64_t)sp * a.k + kv) * a.zstride;
    const int col = col0 + wc * TILE + li;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (rt < nrt && (rt / GRP) % parts == rsel) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          out[(int64_t)(row0 + rt * TILE + acc_row<T>(lk, j)) * a.nmop + col] = S[rt][j];
      }
    }
  }
}

// One workgroup per work unit; consecutive units go to the same XCD (workgroups are dealt to
// the 8 XCDs round-robin), so the units sharing a panel of L^P share that XCD's L2.
template <typename T, int CT, int RT, int OCC>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(OCC, OCC)))
void k_sandwich(const T* __restrict__ L, const T* __restrict__ UT, T* __restrict__ Qp,
                SandParams a) {
  __shared__ __attribute__((aligned(1024))) T buf[SandCfg<T, CT, RT>::BUF];
  const int g = blockIdx.x;
  const int u = (g & 7) * a.per_xcd + (g >> 3);
  if (u >= a.nunits) return;
  sandwich_unit<T, CT, RT>(L, UT, Qp, a, u, buf);
}

// Grouped launch: the work units of several independent sigma products (one per entry, each with
// its own integrals, vectors, partial-sum buffer and decomposition) laid end to end. A unit does
// exactly what it does in a launch of its own product, so each product's result does not depend
// on what it is grouped with.
template <typename T, int CT, int RT, int OCC>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(OCC, OCC)))
void k_sandwich_group(GroupArgs ga) {
  __shared__ __attribute__((aligned(1024))) T buf[SandCfg<T, CT, RT>::BUF];
  const int g = blockIdx.x;
  const int u = (g & 7) * ga.per_xcd + (g >> 3);
  if (u >= ga.u0[ga.n]) return;
  int e = 0;
  while (e + 1 < ga.n && u >= ga.u0[e + 1]) ++e;
  sandwich_unit<T, CT, RT>((const T*)ga.e[e].L, (const T*)ga.e[e].UT, (T*)ga.e[e].Qp, ga.e[e].p,
                           u - ga.u0[e], buf);
}

// ------------------------------------------------------------------------------------------
// Epilogue: sigma = E z + N * (Q + s Q^T), Q summed over the aux splits in a fixed order, FP64.
// One workgroup per 16 x 16 tile (I, J), I <= J, of the upper triangle of a diagonal block and
// one vector: thread (r, c) sums Q[I r][J c] and the mirror tile's Q[J r][I c] over the splits
// (both read with 128-byte row segments), the mirror goes through LDS transposed, and the
// packed pairs (p, q) of the tile get sigma. (Reading Q[q][p] directly for each packed pair
// touches one memory line per element.)
// ------------------------------------------------------------------------------------------
constexpr int ET = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_epilogue(const double* __restrict__ z, int64_t n,
                                                  int64_t nvv, int nv, int no, int nvp, int nmop,
                                                  int mult, const T* __restrict__ Sp, int nsplit,
                                                  int64_t split_stride, int ntv, int npv,
                                                  const double* __restrict__ epair,
                                                  double* __restrict__ sigma) {
  __shared__ double mirror[ET][ET + 1];
  const int kv = blockIdx.y;
  int tp = blockIdx.x;
  const bool vblk = tp < npv;
  if (!vblk) tp -= npv;
  const int nb = vblk ? nv : no;
  const int nt = (nb + ET - 1) / ET;
  const int off = vblk ? 0 : nvp;
  int I = 0;  // tile pair tp -> (I, J), row-major over the upper triangle of tiles
  while (tp >= nt - I) {
    tp -= nt - I;
    ++I;
  }
  const int J = I + tp;
  const int r = threadIdx.x / ET, c = threadIdx.x % ET;
  const int pa = I * ET + r, qa = J * ET + c;  // element of the tile
  const int pb = J * ET + r, qb = I * ET + c;  // element of the mirror tile
  const bool oka = pa < nb && qa < nb, okb = pb < nb && qb < nb;
  const T* Q = Sp + (int64_t)kv * nmop * nmop;
  const int64_t ia = (int64_t)(off + pa) * nmop + off + qa;
  const int64_t ib = (int64_t)(off + pb) * nmop + off + qb;
  // both elements lie in the padded block, which every split writes in full: the loads are
  // unconditional (so that the unrolled iterations issue them together), the padding is
  // discarded afterwards
  double a = 0.0, b = 0.0;
#pragma unroll 8
  for (int t = 0; t < nsplit; ++t) {
    a += (double)Q[t * split_stride + ia];
    b += (double)Q[t * split_stride + ib];
  }
  if (!oka) a = 0.0;
  if (!okb) b = 0.0;
  mirror[r][c] = b;
  __syncthreads();
  const int k = mult == 0 ? 0 : 1;
  if (!oka || qa < pa + k) return;
  // Q[q][p] for (p, q) = (pa, qa) is the mirror tile's element (qa - J ET, pa - I ET) = (c, r)
  const double s = mult == 0 ? a + mirror[c][r] : a - mirror[c][r];
  const int64_t p = pa, q = qa;
  const int64_t e = (vblk ? 0 : nvv) + p * (nb - k) - p * (p - 1) / 2 + (q - p - k);
  const double nrm = (mult == 0 && p == q) ? 0.70710678118654752440 : 1.0;
  sigma[(int64_t)kv * n + e] = epair[e] * z[(int64_t)kv * n + e] + nrm * s;
}

}  // namespace

// ==========================================================================================
// Launchers
// ==========================================================================================
hipError_t launch_check_finite(const double* x, size_t n, int* d_bad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, s, x, n, d_bad);
  return hipGetLastError();
}

hipError_t launch_stage_L(const Geometry& g, Store st, const double* Lin, int nin, int p0, int np,
                          const int* d_src, void* Lout, size_t plane, int* d_bad,
                          hipStream_t s) {
  if (np <= 0) return hipSuccess;
  const int64_t e = (int64_t)g.nmop * g.nmop;
  dim3 grid((unsigned)((e + 255) / 256), (unsigned)np);
  if (st == Store::F64)
    hipLaunchKernelGGL(k_stage_L<double>, grid, dim3(256), 0, s, Lin, nin, p0, d_src, g.nmop,
                       (double*)Lout, d_bad);
  else if (st == Store::F32)
    hipLaunchKernelGGL(k_stage_L<float>, grid, dim3(256), 0, s, Lin, nin, p0, d_src, g.nmop,
                       (float*)Lout, d_bad);
  else
    hipLaunchKernelGGL(k_stage_L_bf16, grid, dim3(256), 0, s, Lin, nin, p0, d_src, g.nmop,
                       (unsigned short*)Lout, plane, d_bad);
  return hipGetLastError();
}

hipError_t launch_unpack(const Geometry& g, Store st, const double* z, int k, const int* d_ptab,
                         void* ZT, size_t zplane, hipStream_t s) {
  (void)d_ptab;
  const int64_t e = (int64_t)g.nvp * g.nvp + (int64_t)g.nop * g.nop;
  dim3 grid((unsigned)((e + 255) / 256), (unsigned)k);
  if (st == Store::F64)
    hipLaunchKernelGGL(k_unpack<double>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nv, g.no, g.nvp,
                       g.nop, g.nmop, g.mult, (double*)ZT);
  else if (st == Store::F32)
    hipLaunchKernelGGL(k_unpack<float>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nv, g.no, g.nvp,
                       g.nop, g.nmop, g.mult, (float*)ZT);
  else
    hipLaunchKernelGGL(k_unpack_bf16, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nv, g.no, g.nvp,
                       g.nop, g.nmop, g.mult, (unsigned short*)ZT, zplane);
  return hipGetLastError();
}

hipError_t launch_epilogue(const Geometry& g, Store st, const double* z, int k, const void* Sp,
                           int nsplit, const int* d_ptab, const double* d_epair, double* sigma,
                           hipStream_t s) {
  (void)d_ptab;
  const int ntv = (g.nv + ET - 1) / ET, nto = (g.no + ET - 1) / ET;
  const int npv = ntv * (ntv + 1) / 2, npo = nto * (nto + 1) / 2;
  dim3 grid((unsigned)(npv + npo), (unsigned)k);
  const int64_t split_stride = (int64_t)k * g.nmop * g.nmop;
  if (st == Store::F64)
    hipLaunchKernelGGL(k_epilogue<double>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nv, g.no, g.nvp,
                       g.nmop, g.mult, (const double*)Sp, nsplit, split_stride, ntv, npv, d_epair,
                       sigma);
  else
    hipLaunchKernelGGL(k_epilogue<float>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nv, g.no, g.nvp,
                       g.nmop, g.mult, (const float*)Sp, nsplit, split_stride, ntv, npv, d_epair,
                       sigma);
  return hipGetLastError();
}

// Work items: (panel, first row tile) pairs; a panel spans up to 4 column tiles of one block.
void make_sigma_items(const Geometry& g, int RT, std::vector<int>& items, int& npan_v, int pw) {
  items.clear();
  const int not_ = g.nct - g.nvt;
  npan_v = (g.nvt + pw - 1) / pw;
  const int npan_o = (not_ + pw - 1) / pw;
  for (int pn = 0; pn < npan_v + npan_o; ++pn) {
    const int bnt = pn < npan_v ? g.nvt : not_;
    for (int R0 = 0; R0 < bnt; R0 += RT) items.push_back((pn << 16) | R0);
  }
}

int sigma_variant(const Geometry& g, Store st, int nprod, int* RT) {
  if (st == Store::F64) {
    // the software-pipelined kernel (k_sigma_f64.hip) for large virtual blocks; below that its
    // units are too short to keep the pipeline full and the two-workgroup kernel is faster
    if (g.nvt >= F64_PIPE_MIN_NVT) {
      *RT = 32;
      return 5;
    }
    *RT = 16;
    return 1;
  }
  if (st == Store::F32) { *RT = 32; return 4; }
  *RT = 32;
  // BF16 split, six products: the double-buffered wide-panel kernel (k_sigma_bf16.hip) for
  // large virtual blocks that it tiles with full 8-tile panels (a ragged last panel idles waves
  // of its workgroup: at 26 tiles = 3 x 8 + 2 it measured no faster than the 4-tile kernel)
  return nprod == 6 && g.nvt >= BF16_WIDE_MIN_NVT && g.nvt % 8 == 0 ? 7 : 3;
}

template <typename T, int CC, int RT, int OCC>
static hipError_t run_sandwich(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                               hipStream_t s) {
  const SandParams p = sand_params(g, plan, la);
  hipLaunchKernelGGL((k_sandwich<T, CC, RT, OCC>), dim3(p.per_xcd * 8), dim3(256), 0, s,
                     (const T*)la.L, (const T*)la.ZT, (T*)la.Sp, p);
  return hipGetLastError();
}

template <typename T, int CC, int RT, int OCC>
static hipError_t run_group(const GroupMember* m, int n, hipStream_t s) {
  const GroupArgs ga = group_args(m, n);
  hipLaunchKernelGGL((k_sandwich_group<T, CC, RT, OCC>), dim3(ga.per_xcd * 8), dim3(256), 0, s, ga);
  return hipGetLastError();
}

hipError_t launch_sigma_group_bf16(const GroupMember* m, int n, hipStream_t s);
hipError_t launch_sigma_group_f64(const GroupMember* m, int n, hipStream_t s);
hipError_t launch_sigma_f64(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                            hipStream_t s);

hipError_t launch_sigma_group(const GroupMember* m, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > GROUP_MAX) return hipErrorInvalidValue;
  const int variant = m[0].plan->variant;
  for (int i = 1; i < n; ++i)
    if (m[i].plan->variant != variant || m[i].la.nprod != m[0].la.nprod) return hipErrorInvalidValue;
  switch (variant) {
    case 1: return run_group<double, 8, 16, 2>(m, n, s);
    case 5: return launch_sigma_group_f64(m, n, s);
    case 4: return run_group<float, 16, 32, 2>(m, n, s);
    default: return launch_sigma_group_bf16(m, n, s);
  }
}

hipError_t launch_sigma_bf16(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                             hipStream_t s);

hipError_t launch_sigma(const Geometry& g, Store st, const SigmaPlan& plan, const SigmaLaunch& la,
                        hipStream_t s) {
  switch (plan.variant) {
    case 1: return run_sandwich<double, 8, 16, 2>(g, plan, la, s);
    case 5: return launch_sigma_f64(g, plan, la, s);
    case 4: return run_sandwich<float, 16, 32, 2>(g, plan, la, s);
    default: return launch_sigma_bf16(g, plan, la, s);
  }
}

}  // namespace pprpa
