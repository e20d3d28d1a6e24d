// BF16-split sigma product on CDNA4 (gfx950): the same sandwich S = sum_P L^P U L^P as the
// FP64/FP32 kernel in k_sigma.hip (same work units, same partial-sum layout, same epilogue),
// with every product done on the BF16 matrix cores (MFMA 16x16x32, FP32 accumulation).
//
// Precision: each operand v is carried as three BF16 planes, hi = bf16(v), mid = bf16(v - hi),
// lo = bf16(v - hi - mid) (round to nearest even), so hi + mid + lo holds v to about 24 bits. A
// product a b is formed as the six terms hh + hm + mh + mm + hl + lh (BF16x6, about FP32
// accuracy) or the three terms hh + hm + mh (BF16x3, about 2^-16 relative); terms below that are
// dropped. L and the unpacked vectors are split when staged; the intermediate T of contraction 1
// is split in registers before it enters contraction 2.
//
// Layout differences from the FP32 kernel, both dictated by the BF16 MFMA operand shape (each lane
// supplies 8 consecutive reduction indices of one row of A and of one column of B):
//   * contraction 1, T[c][col] = sum_d U[c][d] L^P[d][col]: U is stored row-major (not transposed)
//     so a lane reads 8 consecutive d of row c; L^P[d][col] is read as row col of L^P (symmetric),
//     again 8 consecutive d;
//   * contraction 2, S[r][col] += sum_c L^P[r][c] T[c][col], in two forms:
//     - six products (sandwich_bf16_cols): wave w keeps column tile w; T comes from its own
//       accumulators, in which a lane holds rows 4 lk .. 4 lk + 3 of a 16-row tile, so two c
//       tiles give the lane's 8 reduction slots and the A operand is read with the same
//       permutation (two 4-element pieces of a row of L^P);
//     - three products (sandwich_bf16_rows): each wave's T is split and written to LDS once per
//       chunk, transposed (c contiguous); the waves share the row tiles out and each covers all
//       column tiles of the panel, so a staged row of L^P feeds the MFMAs of every column (about
//       a third of the LDS reads per product; the six-product form cannot hold the third plane
//       of four columns in registers);
//   * the diagonal blocks are padded to multiples of 32 orbitals (two tiles), so every 32-wide
//     reduction block lies inside one block.
// Virtual blocks of 32 or more tiles in full 8-tile panels take, for six products, a third form
// (sandwich_bf16_cols_pipe): the columns form on panels of 8 column tiles with 8 waves and two
// LDS stage buffers (loads of the next stage in flight during the current stage's products). The
// wider panel halves the staged U and L^P rows per product, which is what bounds these kernels
// at that size (a timing probe of an 8-wave form on 4-tile panels ran 1.44x faster with its
// loads removed; double-buffering alone did not help it).
#include "sigma_common.h"
#include "sigma_bf16.h"

namespace pprpa {
namespace {

constexpr int RT = 32;  // row tiles per work unit (equals the FP32 kernel's, same work items)

// Six products (two planes more than three) use the columns-per-wave kernel; its LDS holds one
// staging buffer (a contraction-1 stage or a contraction-2 stage of RH row tiles).
struct Bf16ColsCfg {
  static constexpr int NPL = 3, CT = 8, RH = 16;
  static constexpr int US = CT * TILE * KB;  // U rows of a chunk x one reduction block
  static constexpr int LS = 4 * TILE * KB;   // L^P rows of a panel x one reduction block
  static constexpr int S1 = NPL * (US + LS);
  static constexpr int RS = RH * TILE * KB;  // L^P rows of a contraction-2 stage x one block
  static constexpr int S2 = NPL * RS;
  static constexpr int BUF = S1 > S2 ? S1 : S2;  // u16 elements
};

// Three products use the rows-shared kernel: a staging buffer, then T of the current chunk as
// NPL BF16 planes [64 columns][TWP] (c contiguous; rows padded by 8 elements against bank
// conflicts).
struct Bf16RowsCfg {
  static constexpr int NPL = 2, CT = 8, RH = 16;
  static constexpr int US = CT * TILE * KB;
  static constexpr int LS = 4 * TILE * KB;
  static constexpr int S1 = NPL * (US + LS);
  static constexpr int RS = RH * TILE * KB;
  static constexpr int S2 = NPL * RS;
  static constexpr int STAGE = S1 > S2 ? S1 : S2;  // u16 elements
  static constexpr int TWP = CT * TILE + 8;         // padded row of T
  static constexpr int TS = 4 * TILE * TWP;         // one plane of T
  static constexpr int BUF = STAGE + NPL * TS;      // u16 elements
};

template <int NPROD>
constexpr int bf16_buf() {
  return NPROD == 6 ? Bf16ColsCfg::BUF : Bf16RowsCfg::BUF;
}

// acc[i][j] += a_i b_j over the split planes for an NA x NB grid of tiles, the products taken in
// the same order as split_mfma for every tile but interleaved over the grid (independent
// accumulators between two products into the same one).
template <int NPROD, int NA, int NB, int NPL>
__device__ __forceinline__ void split_mfma_grid(const bf8 (&A)[NA][NPL], const bf8 (&B)[NB][NPL],
                                                f4 (&acc)[NA][NB]) {
  constexpr int pa[6] = {0, 0, 1, 1, 0, 2}, pb[6] = {0, 1, 0, 1, 2, 0};
#pragma unroll
  for (int t = 0; t < NPROD; ++t)
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = mfma(A[i][pa[t]], B[j][pb[t]], acc[i][j]);
}

// Six products: wave w keeps column tile w of the panel through both contractions, T stays in
// its registers (split there) and the rows of L^P are read by every wave.
__device__ __forceinline__ void sandwich_bf16_cols(const u16* __restrict__ L, size_t plane,
                                                   const u16* __restrict__ ZU, size_t zplane,
                                                   float* __restrict__ Qp, const SandParams& a,
                                                   int u, u16* __restrict__ buf) {
  constexpr int NPROD = 6, NPL = 3;
  using Cfg = Bf16ColsCfg;
  constexpr int CT = Cfg::CT, RH = Cfg::RH;
  const int item = a.items[(u / a.k) % a.nitems];
  const int kv = u % a.k;
  const int sp = u / (a.nitems * a.k);
  const int pn = item >> 16;
  const int R0 = item & 0xFFFF;

  const bool vblk = pn < a.npan_v;
  const int t0 = vblk ? 4 * pn : 4 * (pn - a.npan_v);
  const int bnt = vblk ? a.nvt : (a.nct - a.nvt);
  const int brow0 = vblk ? 0 : a.nvp;
  const int npt = min(4, bnt - t0);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  // (waves of a short panel stay idle: giving them rows, as the FP32 kernel does, would repeat
  // contraction 1 and its LDS reads, which bound this kernel)
  const bool active = w < npt;
  const int wc = min(w, npt - 1);
  const int nrt = min(bnt, R0 + RT) - R0;
  const int col0 = brow0 + t0 * TILE;
  const int ncol = npt * TILE;
  const int row0 = brow0 + R0 * TILE;
  const int P0 = (int)((int64_t)a.naux * sp / a.nsplit);
  const int P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  const u16* __restrict__ Z = ZU + (int64_t)kv * a.zstride;

  u16* const sU = buf;
  u16* const sL = buf + NPL * Cfg::US;

  f4 S[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) S[r] = f4{0, 0, 0, 0};

  for (int P = P0; P < P1; ++P) {
    const u16* __restrict__ Lp = L + (int64_t)P * a.zstride;
    for (int cc0 = 0; cc0 < a.nct; cc0 += CT) {
      const int cc1 = min(cc0 + CT, a.nct);
      f4 Tacc[CT];
#pragma unroll
      for (int i = 0; i < CT; ++i) Tacc[i] = f4{0, 0, 0, 0};
      // contraction 1: T[c][cols] = sum_d U[c][d] L^P[d][cols] over d in c's block, d >= c;
      // one 32-wide block of d per stage (both tiles in one diagonal block)
      for (int part = 0; part < 2; ++part) {
        const int lo = part == 0 ? cc0 : max(cc0, a.nvt);
        const int hi = part == 0 ? (cc0 < a.nvt ? a.nvt : cc0) : (cc1 > a.nvt ? a.nct : lo);
        for (int dt = lo; dt < hi; dt += 2) {
          int g0, g1, h0, h1;
          c_range(dt, cc0, cc1, a.nvt, &g0, &g1);
          c_range(dt + 1, cc0, cc1, a.nvt, &h0, &h1);
          const int blo = dt < a.nvt ? 0 : a.nvt;
          const int clo = max(cc0, blo), chi = min(cc1, dt + 2);  // c tiles with U[c][d] != 0
          __syncthreads();
#pragma unroll
          for (int p = 0; p < NPL; ++p) {
            dma_tile32(Z + p * zplane + (int64_t)(g0 * TILE) * a.nmop + dt * TILE, a.nmop,
                       (h1 - g0) * TILE, sU + p * Cfg::US, w, lane);
            dma_tile32(Lp + p * plane + (int64_t)col0 * a.nmop + dt * TILE, a.nmop, ncol,
                       sL + p * Cfg::LS, w, lane);
          }
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
          if (active) {
            const int lrow = (wc * TILE + li) * KB + 8 * (lk ^ swz(li));
            const bf8 bh = *(const bf8*)(sL + lrow);
            const bf8 bm = *(const bf8*)(sL + Cfg::LS + lrow);
            const bf8 bl = *(const bf8*)(sL + 2 * Cfg::LS + lrow);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const int cg = cc0 + ct;
              if (cg >= clo && cg < chi) {
                const int urow = ((cg - g0) * TILE + li) * KB + 8 * (lk ^ swz(li));
                const bf8 ah = *(const bf8*)(sU + urow);
                const bf8 am = *(const bf8*)(sU + Cfg::US + urow);
                const bf8 al = *(const bf8*)(sU + 2 * Cfg::US + urow);
                Tacc[ct] = split_mfma<NPROD>(ah, am, al, bh, bm, bl, Tacc[ct]);
              }
            }
          }
        }
      }
      // contraction 2: S[r][cols] += sum_c L^P[r][c] T[c][cols], 32 c (two tiles of T) per
      // reduction block; the lane's slots 0-3 are rows 4 lk .. 4 lk + 3 of the first tile, slots
      // 4-7 the same rows of the second
#pragma unroll
      for (int i = 0; i < CT; i += 2) {
        if (cc0 + i < cc1) {
          bf8 th, tm, tl;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            __bf16 h, m, l;
            split3(t < 4 ? Tacc[i][t] : Tacc[i + 1][t - 4], h, m, l);
            th[t] = h;
            tm[t] = m;
            tl[t] = l;
          }
#pragma unroll
          for (int half = 0; half < RT / RH; ++half) {
            const int rh0 = half * RH;
            if (rh0 < nrt) {
              const int nr = min(RH, nrt - rh0);
              __syncthreads();
#pragma unroll
              for (int p = 0; p < NPL; ++p)
                dma_tile32(Lp + p * plane + (int64_t)(row0 + rh0 * TILE) * a.nmop + (cc0 + i) * TILE,
                           a.nmop, nr * TILE, buf + p * Cfg::RS, w, lane);
              __builtin_amdgcn_s_waitcnt(0);
              __syncthreads();
              if (active) {
#pragma unroll
                for (int rt = 0; rt < RH; ++rt) {
                  if (rt < nr) {
                    // c offsets 4 lk and 16 + 4 lk: chunks lk / 2 and 2 + lk / 2, half lk & 1
                    const int o = (rt * TILE + li) * KB + 4 * (lk & 1);
                    const int o0 = o + 8 * ((lk >> 1) ^ swz(li));
                    const int o1 = o + 8 * ((2 + (lk >> 1)) ^ swz(li));
                    bf8 av[3];
#pragma unroll
                    for (int p = 0; p < NPL; ++p) {
                      const bf4 x0 = *(const bf4*)(buf + p * Cfg::RS + o0);
                      const bf4 x1 = *(const bf4*)(buf + p * Cfg::RS + o1);
                      av[p] = __builtin_shufflevector(x0, x1, 0, 1, 2, 3, 4, 5, 6, 7);
                    }
                    S[rh0 + rt] = split_mfma<NPROD>(av[0], av[1], av[2], th, tm, tl, S[rh0 + rt]);
                  }
                }
              }
            }
          }
        }
      }
    }
  }

  if (active) {
    float* __restrict__ out = Qp + ((int64_t)sp * a.k + kv) * a.zstride;
    const int col = col0 + wc * TILE + li;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (rt < nrt) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          out[(int64_t)(row0 + rt * TILE + 4 * lk + j) * a.nmop + col] = S[rt][j];
      }
    }
  }
}

// Three products: contraction 2 with the rows shared out (T through LDS). Work unit u of one
// product (u < a.nunits), as in the FP32 kernel.
__device__ __forceinline__ void sandwich_bf16_rows(const u16* __restrict__ L, size_t plane,
                                                   const u16* __restrict__ ZU, size_t zplane,
                                                   float* __restrict__ Qp, const SandParams& a,
                                                   int u, u16* __restrict__ buf) {
  constexpr int NPROD = 3, NPL = 2;  // planes used: hi, mid
  using Cfg = Bf16RowsCfg;
  const int item = a.items[(u / a.k) % a.nitems];
  const int kv = u % a.k;
  const int sp = u / (a.nitems * a.k);
  const int pn = item >> 16;
  const int R0 = item & 0xFFFF;

  const bool vblk = pn < a.npan_v;
  const int t0 = vblk ? 4 * pn : 4 * (pn - a.npan_v);
  const int bnt = vblk ? a.nvt : (a.nct - a.nvt);
  const int brow0 = vblk ? 0 : a.nvp;
  const int npt = min(4, bnt - t0);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const bool active = w < npt;  // contraction 1: wave w computes T for column tile w
  const int wc = min(w, npt - 1);
  const int nrt = min(bnt, R0 + RT) - R0;
  const int col0 = brow0 + t0 * TILE;
  const int ncol = npt * TILE;
  const int row0 = brow0 + R0 * TILE;
  const int P0 = (int)((int64_t)a.naux * sp / a.nsplit);
  const int P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  const u16* __restrict__ Z = ZU + (int64_t)kv * a.zstride;

  constexpr int RH = Cfg::RH, CT = Cfg::CT;
  u16* const sU = buf;
  u16* const sL = buf + NPL * Cfg::US;
  u16* const sT = buf + Cfg::STAGE;

  // S[q][cw]: row tile 4 q + w of the unit (rows are dealt round-robin to the waves), column
  // tile cw of the panel
  f4 S[RT / 4][4];
#pragma unroll
  for (int q = 0; q < RT / 4; ++q)
#pragma unroll
    for (int cw = 0; cw < 4; ++cw) S[q][cw] = f4{0, 0, 0, 0};

  for (int P = P0; P < P1; ++P) {
    const u16* __restrict__ Lp = L + (int64_t)P * a.zstride;
    for (int cc0 = 0; cc0 < a.nct; cc0 += CT) {
      const int cc1 = min(cc0 + CT, a.nct);
      f4 Tacc[CT];
#pragma unroll
      for (int i = 0; i < CT; ++i) Tacc[i] = f4{0, 0, 0, 0};
      // contraction 1: T[c][cols] = sum_d U[c][d] L^P[d][cols] over d in c's block, d >= c;
      // one 32-wide block of d per stage (both tiles in one diagonal block)
      for (int part = 0; part < 2; ++part) {
        const int lo = part == 0 ? cc0 : max(cc0, a.nvt);
        const int hi = part == 0 ? (cc0 < a.nvt ? a.nvt : cc0) : (cc1 > a.nvt ? a.nct : lo);
        for (int dt = lo; dt < hi; dt += 2) {
          int g0, g1, h0, h1;
          c_range(dt, cc0, cc1, a.nvt, &g0, &g1);
          c_range(dt + 1, cc0, cc1, a.nvt, &h0, &h1);
          const int blo = dt < a.nvt ? 0 : a.nvt;
          const int clo = max(cc0, blo), chi = min(cc1, dt + 2);  // c tiles with U[c][d] != 0
          __syncthreads();
#pragma unroll
          for (int p = 0; p < NPL; ++p) {
            dma_tile32(Z + p * zplane + (int64_t)(g0 * TILE) * a.nmop + dt * TILE, a.nmop,
                       (h1 - g0) * TILE, sU + p * Cfg::US, w, lane);
            dma_tile32(Lp + p * plane + (int64_t)col0 * a.nmop + dt * TILE, a.nmop, ncol,
                       sL + p * Cfg::LS, w, lane);
          }
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
          if (active) {
            const int lrow = (wc * TILE + li) * KB + 8 * (lk ^ swz(li));
            const bf8 bh = *(const bf8*)(sL + lrow);
            const bf8 bm = *(const bf8*)(sL + Cfg::LS + lrow);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const int cg = cc0 + ct;
              if (cg >= clo && cg < chi) {
                const int urow = ((cg - g0) * TILE + li) * KB + 8 * (lk ^ swz(li));
                const bf8 ah = *(const bf8*)(sU + urow);
                const bf8 am = *(const bf8*)(sU + Cfg::US + urow);
                Tacc[ct] = split_mfma<NPROD>(ah, am, ah, bh, bm, bh, Tacc[ct]);
              }
            }
          }
        }
      }
      // T of this chunk into LDS, split, transposed: sT[p][col][c]; a lane holds rows
      // 4 lk .. 4 lk + 3 of each c tile for column li of its tile. (The previous chunk's reads of
      // sT finished before the first stage barrier of this chunk's contraction 1.)
      if (active) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          bf4 th, tm;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            __bf16 h, m, l;
            split3(Tacc[ct][j], h, m, l);
            th[j] = h;
            tm[j] = m;
          }
          const int o = (wc * TILE + li) * Cfg::TWP + ct * TILE + 4 * lk;
          *(bf4*)(sT + o) = th;
          *(bf4*)(sT + Cfg::TS + o) = tm;
        }
      }
      __syncthreads();
      // contraction 2: S[r][cols] += sum_c L^P[r][c] T[c][cols], one 32-wide block of c (two
      // tiles of T) at a time; B operands (T of every column tile) from LDS, A (rows of L^P)
      // staged RH row tiles at a time
#pragma unroll
      for (int cb = 0; cb < CT / 2; ++cb) {
        if (cc0 + 2 * cb < cc1) {
          bf8 B[4][NPL];
#pragma unroll
          for (int cw = 0; cw < 4; ++cw)
#pragma unroll
            for (int p = 0; p < NPL; ++p)
              B[cw][p] = cw < npt ? *(const bf8*)(sT + p * Cfg::TS + (cw * TILE + li) * Cfg::TWP +
                                                  cb * KB + 8 * lk)
                                  : B[0][p];
#pragma unroll
          for (int half = 0; half < RT / RH; ++half) {
            const int rh0 = half * RH;
            if (rh0 < nrt) {
              const int nr = min(RH, nrt - rh0);
              __syncthreads();
#pragma unroll
              for (int p = 0; p < NPL; ++p)
                dma_tile32(Lp + p * plane + (int64_t)(row0 + rh0 * TILE) * a.nmop +
                               (cc0 + 2 * cb) * TILE,
                           a.nmop, nr * TILE, buf + p * Cfg::RS, w, lane);
              __builtin_amdgcn_s_waitcnt(0);
              __syncthreads();
#pragma unroll
              for (int rr = 0; rr < RH / 4; ++rr) {
                const int r = 4 * rr + w;
                if (r < nr) {
                  const int o = (r * TILE + li) * KB + 8 * (lk ^ swz(li));
                  const bf8 ah = *(const bf8*)(buf + o);
                  const bf8 am = *(const bf8*)(buf + Cfg::RS + o);
#pragma unroll
                  for (int cw = 0; cw < 4; ++cw)
                    if (cw < npt)
                      S[half * (RH / 4) + rr][cw] = split_mfma<NPROD>(
                          ah, am, ah, B[cw][0], B[cw][1], B[cw][0], S[half * (RH / 4) + rr][cw]);
                }
              }
            }
          }
        }
      }
    }
  }

  float* __restrict__ out = Qp + ((int64_t)sp * a.k + kv) * a.zstride;
#pragma unroll
  for (int half = 0; half < RT / RH; ++half)
#pragma unroll
    for (int rr = 0; rr < RH / 4; ++rr) {
      const int rt = half * RH + 4 * rr + w;
      if (rt < nrt) {
#pragma unroll
        for (int cw = 0; cw < 4; ++cw)
          if (cw < npt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              out[(int64_t)(row0 + rt * TILE + 4 * lk + j) * a.nmop + col0 + cw * TILE + li] =
                  S[half * (RH / 4) + rr][cw][j];
      }
    }
}

// ---------------------------------------------------------------------------------------------
// Double-buffered columns form on wide panels: wave w keeps column tile w of an 8-tile panel
// (T in its registers, split there), one 8-wave workgroup per CU with two stage buffers, so the
// direct loads of stage s + 1 run during the products of stage s. The panel of 8 column tiles
// (twice the other kernels') halves the staged U and L^P rows per product: every staged tile of
// U feeds 8 columns' products in contraction 1 and every staged row of L^P 8 columns' in
// contraction 2.
// ---------------------------------------------------------------------------------------------
constexpr int QNW = 8;  // waves per workgroup = column tiles per panel

template <int NPL>
struct ColsPipeCfg {
  static constexpr int CT = 8;                           // c tiles per chunk
  static constexpr int RH = NPL == 3 ? 16 : 32;           // row tiles per contraction-2 stage
  static constexpr int US = CT * TILE * KB;               // U rows of a chunk x one d block
  static constexpr int LS = QNW * TILE * KB;              // L^P rows of a panel x one d block
  static constexpr int S1 = NPL * (US + LS);
  static constexpr int RS = RH * TILE * KB;               // L^P rows of a stage x one c block
  static constexpr int S2 = NPL * RS;
  static constexpr int BUF = S1 > S2 ? S1 : S2;           // u16 per stage buffer
};

// Stage order of a unit (as StageB, with rh row tiles per contraction-2 stage).
struct StageQ {
  int nvt, nct, P1, nrt, rh;
  int P, cc0, cc1, part, pos, hh;
  bool valid;

  __device__ __forceinline__ int hi() const {
    if (part == 0) return cc0 < nvt ? nvt : cc0;
    if (part == 1) return cc1 > nvt ? nct : max(cc0, nvt);
    return cc1;
  }
  __device__ __forceinline__ void settle() {
    for (;;) {
      if (pos < hi()) return;
      if (part == 0) {
        part = 1;
        pos = max(cc0, nvt);
      } else if (part == 1) {
        part = 2;
        pos = cc0;
        hh = 0;
      } else {
        cc0 += 8;
        if (cc0 >= nct) {
          cc0 = 0;
          if (++P >= P1) {
            valid = false;
            return;
          }
        }
        cc1 = min(cc0 + 8, nct);
        part = 0;
        pos = cc0;
      }
    }
  }
  __device__ __forceinline__ void advance() {
    if (part < 2) {
      pos += 2;
    } else if (++hh * rh >= nrt) {
      hh = 0;
      pos += 2;
    }
    settle();
  }
};

template <int NPROD>
__device__ __forceinline__ void sandwich_bf16_cols_pipe(const u16* __restrict__ L, size_t plane,
                                                        const u16* __restrict__ ZU, size_t zplane,
                                                        float* __restrict__ Qp,
                                                        const SandParams& a, int u,
                                                        u16* __restrict__ lds) {
  constexpr int NPL = NPROD == 6 ? 3 : 2;
  using Cfg = ColsPipeCfg<NPL>;
  constexpr int CT = Cfg::CT, RH = Cfg::RH;
  constexpr int NH = (RT + RH - 1) / RH;  // contraction-2 stages per c block at the widest unit
  const int item = a.items[(u / a.k) % a.nitems];
  const int kv = u % a.k;
  const int sp = u / (a.nitems * a.k);
  const int pn = item >> 16;
  const int R0 = item & 0xFFFF;

  const bool vblk = pn < a.npan_v;
  const int t0 = vblk ? QNW * pn : QNW * (pn - a.npan_v);
  const int bnt = vblk ? a.nvt : (a.nct - a.nvt);
  const int brow0 = vblk ? 0 : a.nvp;
  const int npt = min(QNW, bnt - t0);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const bool active = w < npt;
  const int wc = min(w, npt - 1);
  const int nrt = min(bnt, R0 + RT) - R0;
  const int col0 = brow0 + t0 * TILE;
  const int ncol = npt * TILE;
  const int row0 = brow0 + R0 * TILE;
  const u16* __restrict__ Z = ZU + (int64_t)kv * a.zstride;
  const int sw = 8 * (lk ^ swz(li));

  StageQ it;
  it.nvt = a.nvt;
  it.nct = a.nct;
  it.nrt = nrt;
  it.rh = RH;
  it.P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  it.P = (int)((int64_t)a.naux * sp / a.nsplit);
  it.cc0 = 0;
  it.cc1 = min(CT, a.nct);
  it.part = 0;
  it.pos = 0;
  it.hh = 0;
  it.valid = it.P < it.P1;
  if (it.valid) it.settle();

  auto issue = [&](const StageQ& s, u16* b) {
    const u16* __restrict__ Lp = L + (int64_t)s.P * a.zstride;
    if (s.part < 2) {
      int g0, g1, h0, h1;
      c_range(s.pos, s.cc0, s.cc1, a.nvt, &g0, &g1);
      c_range(s.pos + 1, s.cc0, s.cc1, a.nvt, &h0, &h1);
#pragma unroll
      for (int p = 0; p < NPL; ++p) {
        dma_tile32<QNW>(Z + p * zplane + (int64_t)(g0 * TILE) * a.nmop + s.pos * TILE, a.nmop,
                        (h1 - g0) * TILE, b + p * Cfg::US, w, lane);
        dma_tile32<QNW>(Lp + p * plane + (int64_t)col0 * a.nmop + s.pos * TILE, a.nmop, ncol,
                        b + NPL * Cfg::US + p * Cfg::LS, w, lane);
      }
    } else {
      const int nr = min(RH, s.nrt - s.hh * RH);
#pragma unroll
      for (int p = 0; p < NPL; ++p)
        dma_tile32<QNW>(Lp + p * plane + (int64_t)(row0 + s.hh * RH * TILE) * a.nmop +
                            s.pos * TILE,
                        a.nmop, nr * TILE, b + p * Cfg::RS, w, lane);
    }
  };
  StageQ nx = it;
  if (nx.valid) {
    issue(nx, lds);
    nx.advance();
  }
  int stage = 0;
  u16* cur = lds;
  auto next_stage = [&]() {
    cur = lds + (stage & 1) * Cfg::BUF;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (nx.valid) {
      issue(nx, lds + ((stage + 1) & 1) * Cfg::BUF);
      nx.advance();
    }
    ++stage;
  };

  f4 S[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) S[r] = f4{0, 0, 0, 0};

  const int P0 = it.P, P1 = it.P1;
  for (int P = P0; P < P1; ++P) {
    for (int cc0 = 0; cc0 < a.nct; cc0 += CT) {
      const int cc1 = min(cc0 + CT, a.nct);
      f4 Tacc[CT];
#pragma unroll
      for (int i = 0; i < CT; ++i) Tacc[i] = f4{0, 0, 0, 0};
      // contraction 1: T[c][col tile w] = sum_{d >= c} U[c][d] L^P[d][cols], d in c's block
      for (int part = 0; part < 2; ++part) {
        const int lo = part == 0 ? cc0 : max(cc0, a.nvt);
        const int hi = part == 0 ? (cc0 < a.nvt ? a.nvt : cc0) : (cc1 > a.nvt ? a.nct : lo);
        for (int dt = lo; dt < hi; dt += 2) {
          next_stage();
          int g0, g1;
          c_range(dt, cc0, cc1, a.nvt, &g0, &g1);
          const int blo = dt < a.nvt ? 0 : a.nvt;
          const int clo = max(cc0, blo), chi = min(cc1, dt + 2);
          if (active) {
            const u16* __restrict__ sU = cur;
            const u16* __restrict__ sL = cur + NPL * Cfg::US;
            bf8 bv[NPL];
#pragma unroll
            for (int p = 0; p < NPL; ++p)
              bv[p] = *(const bf8*)(sL + p * Cfg::LS + (wc * TILE + li) * KB + sw);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const int cg = cc0 + ct;
              if (cg >= clo && cg < chi) {
                bf8 av[NPL];
#pragma unroll
                for (int p = 0; p < NPL; ++p)
                  av[p] = *(const bf8*)(sU + p * Cfg::US + ((cg - g0) * TILE + li) * KB + sw);
                Tacc[ct] = split_mfma<NPROD>(av[0], av[1], av[NPL - 1], bv[0], bv[1], bv[NPL - 1],
                                             Tacc[ct]);
              }
            }
          }
        }
      }
      // contraction 2: S[r][col tile w] += sum_c L^P[r][c] T[c][col tile w], one 32-wide c block
      // (two T tiles, split in registers) per stage group, RH row tiles per stage
#pragma unroll
      for (int i = 0; i < CT; i += 2) {
        if (cc0 + i < cc1) {
          bf8 tb[NPL];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            __bf16 h, m, l;
            split3(t < 4 ? Tacc[i][t] : Tacc[i + 1][t - 4], h, m, l);
            tb[0][t] = h;
            tb[1][t] = m;
            if (NPL == 3) tb[NPL - 1][t] = l;
          }
#pragma unroll
          for (int hh = 0; hh < NH; ++hh) {
            if (hh * RH < nrt) {
              next_stage();
              const int nr = min(RH, nrt - hh * RH);
              if (active) {
#pragma unroll
                for (int rt = 0; rt < RH; ++rt) {
                  if (hh * RH + rt < RT && rt < nr) {
                    const int o = (rt * TILE + li) * KB + 4 * (lk & 1);
                    const int o0 = o + 8 * ((lk >> 1) ^ swz(li));
                    const int o1 = o + 8 * ((2 + (lk >> 1)) ^ swz(li));
                    bf8 av[NPL];
#pragma unroll
                    for (int p = 0; p < NPL; ++p) {
                      const bf4 x0 = *(const bf4*)(cur + p * Cfg::RS + o0);
                      const bf4 x1 = *(const bf4*)(cur + p * Cfg::RS + o1);
                      av[p] = __builtin_shufflevector(x0, x1, 0, 1, 2, 3, 4, 5, 6, 7);
                    }
                    S[hh * RH + rt] = split_mfma<NPROD>(av[0], av[1], av[NPL - 1], tb[0], tb[1],
                                                        tb[NPL - 1], S[hh * RH + rt]);
                  }
                }
              }
            }
          }
        }
      }
    }
  }

  if (active) {
    float* __restrict__ out = Qp + ((int64_t)sp * a.k + kv) * a.zstride;
    const int col = col0 + wc * TILE + li;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (rt < nrt) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          out[(int64_t)(row0 + rt * TILE + 4 * lk + j) * a.nmop + col] = S[rt][j];
      }
    }
  }
}

__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
void k_sandwich_bf16w(const u16* __restrict__ L, size_t plane, const u16* __restrict__ ZU,
                      size_t zplane, float* __restrict__ Qp, SandParams a) {
  __shared__ __attribute__((aligned(1024))) u16 lds[2 * ColsPipeCfg<3>::BUF];
  const int g = blockIdx.x;
  const int u = (g & 7) * a.per_xcd + (g >> 3);
  if (u >= a.nunits) return;
  sandwich_bf16_cols_pipe<6>(L, plane, ZU, zplane, Qp, a, u, lds);
}

// Grouped launch (serving): each member's units exactly as in its own launch.
__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
void k_sandwich_bf16w_group(GroupArgs ga) {
  __shared__ __attribute__((aligned(1024))) u16 lds[2 * ColsPipeCfg<3>::BUF];
  const int g = blockIdx.x;
  const int u = (g & 7) * ga.per_xcd + (g >> 3);
  if (u >= ga.u0[ga.n]) return;
  int e = 0;
  while (e + 1 < ga.n && u >= ga.u0[e + 1]) ++e;
  const GroupEntry& m = ga.e[e];
  sandwich_bf16_cols_pipe<6>((const u16*)m.L, m.plane, (const u16*)m.UT, m.zplane, (float*)m.Qp,
                             m.p, u - ga.u0[e], lds);
}

template <int NPROD>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
void k_sandwich_bf16(const u16* __restrict__ L, size_t plane, const u16* __restrict__ ZU,
                     size_t zplane, float* __restrict__ Qp, SandParams a) {
  __shared__ __attribute__((aligned(1024))) u16 buf[bf16_buf<NPROD>()];
  const int g = blockIdx.x;
  const int u = (g & 7) * a.per_xcd + (g >> 3);
  if (u >= a.nunits) return;
  if constexpr (NPROD == 6)
    sandwich_bf16_cols(L, plane, ZU, zplane, Qp, a, u, buf);
  else
    sandwich_bf16_rows(L, plane, ZU, zplane, Qp, a, u, buf);
}

// Grouped launch (serving): each member's units exactly as in its own launch.
template <int NPROD>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
void k_sandwich_bf16_group(GroupArgs ga) {
  __shared__ __attribute__((aligned(1024))) u16 buf[bf16_buf<NPROD>()];
  const int g = blockIdx.x;
  const int u = (g & 7) * ga.per_xcd + (g >> 3);
  if (u >= ga.u0[ga.n]) return;
  int e = 0;
  while (e + 1 < ga.n && u >= ga.u0[e + 1]) ++e;
  const GroupEntry& m = ga.e[e];
  if constexpr (NPROD == 6)
    sandwich_bf16_cols((const u16*)m.L, m.plane, (const u16*)m.UT, m.zplane, (float*)m.Qp, m.p,
                       u - ga.u0[e], buf);
  else
    sandwich_bf16_rows((const u16*)m.L, m.plane, (const u16*)m.UT, m.zplane, (float*)m.Qp, m.p,
                       u - ga.u0[e], buf);
}

}  // namespace

hipError_t launch_sigma_bf16(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                             hipStream_t s) {
  if (g.nvp % (2 * TILE) || g.nop % (2 * TILE)) return hipErrorInvalidValue;
  const SandParams p = sand_params(g, plan, la);
  const dim3 grid(p.per_xcd * 8);
  if (plan.variant == 7) {
    if (la.nprod != 6) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sandwich_bf16w, grid, dim3(QNW * 64), 0, s, (const u16*)la.L, la.plane,
                       (const u16*)la.ZT, la.zplane, (float*)la.Sp, p);
    return hipGetLastError();
  }
  if (la.nprod == 3)
    hipLaunchKernelGGL(k_sandwich_bf16<3>, grid, dim3(256), 0, s, (const u16*)la.L, la.plane,
                       (const u16*)la.ZT, la.zplane, (float*)la.Sp, p);
  else
    hipLaunchKernelGGL(k_sandwich_bf16<6>, grid, dim3(256), 0, s, (const u16*)la.L, la.plane,
                       (const u16*)la.ZT, la.zplane, (float*)la.Sp, p);
  return hipGetLastError();
}

hipError_t launch_sigma_group_bf16(const GroupMember* m, int n, hipStream_t s) {
  for (int i = 0; i < n; ++i)
    if (m[i].g->nvp % (2 * TILE) || m[i].g->nop % (2 * TILE)) return hipErrorInvalidValue;
  const GroupArgs ga = group_args(m, n);
  if (m[0].plan->variant == 7) {
    if (m[0].la.nprod != 6) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sandwich_bf16w_group, dim3(ga.per_xcd * 8), dim3(QNW * 64), 0, s, ga);
    return hipGetLastError();
  }
  if (m[0].la.nprod == 3)
    hipLaunchKernelGGL(k_sandwich_bf16_group<3>, dim3(ga.per_xcd * 8), dim3(256), 0, s, ga);
  else
    hipLaunchKernelGGL(k_sandwich_bf16_group<6>, dim3(ga.per_xcd * 8), dim3(256), 0, s, ga);
  return hipGetLastError();
}

}  // namespace pprpa
