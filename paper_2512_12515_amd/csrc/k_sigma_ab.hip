// Density-fitted sigma product of the alpha-beta sector of spin-unrestricted ppRPA on CDNA4
// (gfx950), FP64 MFMA.
//
// Method (arXiv 2512.12515, section "Implementation Details": the unrestricted matrix splits into
// three spin subspaces). In the alpha-beta sector a pair joins an alpha orbital with a beta one
// and the exchange integral vanishes, so with (pq|rs) = sum_P La^P_pq Lb^P_rs
//   A x (ab) = sum_cd (ac|bd) x_cd,  B y (ab) = sum_kl (ak|bl) y_kl,
//   B^T x (ij) = sum_cd (ic|jd) x_cd,  C y (ij) = sum_kl (ik|jl) y_kl.
// With Z = blockdiag(X, Y) (X: nv_a x nv_b, Y: no_a x no_b; every pair, alpha index outer) over
// the orbitals ordered [virtual; occupied] of each spin,
//   Q = sum_P La^P Z Lb^P   (nmo_a x nmo_b)
// holds A x + B y in its virtual-virtual block and B^T x + C y in its occupied-occupied block:
//   sigma_x(ab) = (e^a_a + e^b_b) x_ab + Q[a][b],   sigma_y(ij) = -(e^a_i + e^b_j) y_ij + Q[i][j].
//
// BF16-split sigma (k_sandwich_ab_bf16): the integrals and Z carried as BF16 planes, contraction 1
// reducing over d and contraction 2 over c in blocks of 32 on the BF16 MFMA (blocks padded to 32
// orbitals), T split into planes in LDS between them, as the restricted rows-form BF16 kernel.
//
// Kernel design: the two contractions of the restricted sandwich kernel, one workgroup of 4
// waves per (vector, panel of up to 4 beta column tiles, range of up to RT alpha row tiles, aux
// range), wave w owning column tile w: contraction 1, T[c][cols] = sum_d Z[c][d] Lb^P[d][cols]
// with d over the whole beta block that pairs with c's alpha block (Z is rectangular: no
// triangle), accumulates in registers; contraction 2, Q[r][cols] += sum_c La^P[r][c] T[c][cols],
// takes T from those registers. Operands are staged in LDS by direct global->LDS loads; the aux
// index is split over workgroups and the partial Q are summed in a fixed order by the epilogue.
#include "internal.h"
#include "sigma_common.h"
#include "sigma_bf16.h"

namespace pprpa {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int AB_CT = 8;   // c tiles per chunk (T tiles held in registers)
constexpr int AB_RT = 16;  // alpha row tiles per work unit
constexpr int AB_ND = 3;   // d tiles per contraction-1 stage
constexpr int AB_SR1 = AB_ND * TILE;
constexpr int AB_BUF = AB_SR1 * AB_CT * TILE + AB_SR1 * 4 * TILE;  // 72 KiB of doubles
static_assert(2 * TILE * AB_RT * TILE <= AB_BUF, "two contraction-2 c tiles fit the buffer");

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// c tiles of chunk [cc0, cc1) paired with beta d tile dt (all of the alpha block that matches d's
// beta block), rounded out to pairs counted from cc0; tiles outside the block hold exact zeros of
// Z^T.
__device__ __forceinline__ void ab_c_range(int dt, int cc0, int cc1, int nvta, int ncta, int nvtb,
                                           int* g0, int* g1, int* hi_out) {
  const bool virt = dt < nvtb;
  const int lo = max(cc0, virt ? 0 : nvta);
  const int hi = min(cc1, virt ? nvta : ncta);
  *hi_out = hi;
  *g0 = cc0 + ((lo - cc0) & ~1);
  *g1 = min(cc1, cc0 + ((hi - cc0 + 1) & ~1));
}

// Unpack the packed alpha-beta vectors into Z^T[kv][d][c] (beta row d, alpha column c), the
// layout contraction 1 stages. Positions outside the two blocks keep the zeros they were
// cleared to at build.
template <typename T>
__global__ void k_unpack_ab(const double* __restrict__ z, int64_t n, int64_t nvv, int nvb,
                            int nob, int nvpa, int nvpb, int nmopa, int nmopb,
                            T* __restrict__ ZT) {
  const int kv = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  int c, d;
  if (e < nvv) {
    c = (int)(e / nvb);
    d = (int)(e % nvb);
  } else {
    const int64_t s = e - nvv;
    c = nvpa + (int)(s / nob);
    d = nvpb + (int)(s % nob);
  }
  ZT[((int64_t)kv * nmopb + d) * nmopa + c] = (T)z[(int64_t)kv * n + e];
}

template <typename T> struct AbAcc;
template <> struct AbAcc<double> { using V = d4; };
template <> struct AbAcc<float> { using V = f4; };
__device__ __forceinline__ f4 mfma64(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// accumulator register j of lane group lk holds output row ab_acc_row(lk, j) of the tile
// (FP64 16x16x4: lk + 4 j; FP32 16x16x4: 4 lk + j)
template <typename T> __device__ __forceinline__ int ab_acc_row(int lk, int j);
template <> __device__ __forceinline__ int ab_acc_row<double>(int lk, int j) { return lk + 4 * j; }
template <> __device__ __forceinline__ int ab_acc_row<float>(int lk, int j) { return 4 * lk + j; }

template <typename T, int CT, int RT>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
void k_sandwich_ab(const T* __restrict__ La, const T* __restrict__ Lb,
                   const T* __restrict__ UT, T* __restrict__ Qp, AbParams a) {
  using V = typename AbAcc<T>::V;
  __shared__ __attribute__((aligned(1024))) T buf[AB_BUF];
  constexpr int GRP = 2;
  static_assert(CT % GRP == 0 && RT % GRP == 0, "tile groups");
  static_assert(2 * CT * 4 * 64 <= AB_BUF, "T exchange of a two-column panel fits the buffer");
  const int g = blockIdx.x;
  const int u = (g & 7) * a.per_xcd + (g >> 3);
  if (u >= a.nunits) return;

  // unit u -> (vector u % k, work item (u / k) % nitems, aux split u / (nitems k))
  const int item = a.items[(u / a.k) % a.nitems];
  const int kv = u % a.k;
  const int sp = u / (a.nitems * a.k);
  const int pn = item >> 16;
  const int R0 = item & 0xFFFF;  // first alpha row tile of the range (local to the block)
  const bool vblk = pn < a.npan_v;
  const int t0 = vblk ? 4 * pn : 4 * (pn - a.npan_v);            // first beta column tile
  const int bntb = vblk ? a.nvtb : (a.nctb - a.nvtb);             // beta column tiles of block
  const int bnta = vblk ? a.nvta : (a.ncta - a.nvta);             // alpha row tiles of block
  const int col0 = (vblk ? 0 : a.nvpb) + t0 * TILE;
  const int row0 = (vblk ? 0 : a.nvpa) + R0 * TILE;
  const int npt = min(4, bntb - t0);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  // a panel of one or two column tiles puts parts = 4 / npt waves on each column: in
  // contraction 1 they share out the column's c groups (g % parts == rsel), exchange their T
  // tiles through LDS, and in contraction 2 they share out its row groups the same way; a
  // three-tile panel idles one wave
  const int parts = npt == 1 ? 4 : (npt == 2 ? 2 : 1);
  const bool active = w < npt * parts;
  const int wc = parts == 1 ? min(w, npt - 1) : w % npt;
  const int rsel = parts == 1 ? 0 : w / npt;
  const int nrt = min(bnta, R0 + RT) - R0;
  const int ncol = npt * TILE;
  const int wl = nrt * TILE;
  const int P0 = (int)((int64_t)a.naux * sp / a.nsplit);
  const int P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  const T* __restrict__ Z = UT + (int64_t)kv * a.zt_stride;

  V S[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) S[r] = V{0, 0, 0, 0};

  T* const sB = buf + AB_SR1 * CT * TILE;
  for (int P = P0; P < P1; ++P) {
    const T* __restrict__ Lap = La + (int64_t)P * a.la_stride;
    const T* __restrict__ Lbp = Lb + (int64_t)P * a.lb_stride;
    for (int cc0 = 0; cc0 < a.ncta; cc0 += CT) {
      const int cc1 = min(cc0 + CT, a.ncta);
      V Tacc[CT];
#pragma unroll
      for (int i = 0; i < CT; ++i) Tacc[i] = V{0, 0, 0, 0};
      // contraction 1: part 0 pairs the chunk's alpha virtual c tiles with every beta virtual d
      // tile, part 1 its alpha occupied c tiles with every beta occupied d tile
      for (int part = 0; part < 2; ++part) {
        const bool has = part == 0 ? cc0 < a.nvta : cc1 > a.nvta;
        const int lo = part == 0 ? 0 : a.nvtb;
        const int hi = has ? (part == 0 ? a.nvtb : a.nctb) : lo;
        for (int dt = lo; dt < hi; dt += AB_ND) {
          const int nd = min(AB_ND, hi - dt);
          int g0, g1, chi;
          ab_c_range(dt, cc0, cc1, a.nvta, a.ncta, a.nvtb, &g0, &g1, &chi);
          const int wa = (g1 - g0) * TILE;
          __syncthreads();
          dma_tile(Z + (int64_t)(dt * TILE) * a.nmopa + g0 * TILE, a.nmopa, nd * TILE, wa, buf, w,
                   lane);
          dma_tile(Lbp + (int64_t)(dt * TILE) * a.nmopb + col0, a.nmopb, nd * TILE, ncol, sB, w,
                   lane);
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
#pragma unroll
          for (int sub = 0; sub < AB_ND; ++sub) {
            if (sub < nd) {
              const T* sA = buf + sub * TILE * wa;
              const T* sBs = sB + sub * TILE * ncol;
              T bv[4];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) bv[ks] = sBs[(4 * ks + lk) * ncol + wc * TILE + li];
#pragma unroll
              for (int grp = 0; grp < CT / GRP; ++grp) {
                const int cg = cc0 + GRP * grp;
                if (active && cg >= g0 && cg < chi && grp % parts == rsel) {
                  T av[4][GRP];
#pragma unroll
                  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = 0; j < GRP; ++j)
                      av[ks][j] = sA[(4 * ks + lk) * wa + (cg - g0 + j) * TILE + li];
                  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = 0; j < GRP; ++j)
                      Tacc[GRP * grp + j] = mfma64(av[ks][j], bv[ks], Tacc[GRP * grp + j]);
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
      // contraction 2: Q[r][cols] += sum_c La^P[r][c] T[c][cols] (La^P symmetric: the staged
      // rows c of La^P give the A operand, read with the reduction index permuted to T's
      // accumulator layout), two c tiles per stage
#pragma unroll
      for (int i = 0; i < CT; i += 2) {
        if (cc0 + i < cc1) {
          const int nb = min(2, cc1 - cc0 - i);
          __syncthreads();
          dma_tile(Lap + (int64_t)((cc0 + i) * TILE) * a.nmopa + row0, a.nmopa, nb * TILE, wl, buf, w,
                   lane);
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
#pragma unroll
          for (int sub = 0; sub < 2; ++sub) {
            if (sub < nb) {
              const T* sL = buf + sub * TILE * wl;
#pragma unroll
              for (int grp = 0; grp < RT / GRP; ++grp) {
                // a row tile at nrt in the last group reads other staged data (in bounds); its
                // result is never stored
                if (active && GRP * grp < nrt && grp % parts == rsel) {
                  T av[4][GRP];
#pragma unroll
                  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = 0; j < GRP; ++j)
                      av[ks][j] = sL[ab_acc_row<T>(lk, ks) * wl + (GRP * grp + j) * TILE + li];
                  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = 0; j < GRP; ++j)
                      S[GRP * grp + j] = mfma64(av[ks][j], Tacc[i + sub][ks], S[GRP * grp + j]);
                }
              }
            }
          }
        }
      }
    }
  }

  if (active) {
    T* __restrict__ out = Qp + ((int64_t)sp * a.k + kv) * a.q_stride;
    const int col = col0 + wc * TILE + li;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (rt < nrt && (rt / GRP) % parts == rsel) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          out[(int64_t)(row0 + rt * TILE + ab_acc_row<T>(lk, j)) * a.nmopb + col] = S[rt][j];
      }
    }
  }
}

// sigma[e] = epair[e] z[e] + sum over splits of Q[row][col] (fixed order), with epair the signed
// pair energies (+ for vv, - for oo pairs).
template <typename T>
__global__ __launch_bounds__(256) void k_epilogue_ab(const double* __restrict__ z, int64_t n,
                                                     int64_t nvv, int nvb, int nob, int nvpa,
                                                     int nvpb, int nmopb, const T* __restrict__ Qp,
                                                     int nsplit, int64_t split_stride,
                                                     int64_t q_stride,
                                                     const double* __restrict__ epair,
                                                     double* __restrict__ sigma) {
  const int kv = blockIdx.y;
  const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t e = e0 < n ? e0 : n - 1;  // clamped: every thread's loads stay in bounds
  int r, c;
  if (e < nvv) {
    r = (int)(e / nvb);
    c = (int)(e % nvb);
  } else {
    const int64_t s = e - nvv;
    r = nvpa + (int)(s / nob);
    c = nvpb + (int)(s % nob);
  }
  const T* Q = Qp + (int64_t)kv * q_stride + (int64_t)r * nmopb + c;
  double acc = 0.0;
#pragma unroll 8
  for (int t = 0; t < nsplit; ++t) acc += (double)Q[t * split_stride];
  if (e0 < n) sigma[(int64_t)kv * n + e] = epair[e] * z[(int64_t)kv * n + e] + acc;
}

// Z[kv][c][d] (alpha row c, beta column d contiguous) of the packed alpha-beta vectors as three
// BF16 planes (hi, mid, lo) zplane elements apart; positions outside the two blocks keep the
// zeros they were cleared to at build.
__global__ void k_unpack_ab_bf16(const double* __restrict__ z, int64_t n, int64_t nvv, int nvb,
                                 int nob, int nvpa, int nvpb, int nmopb, int64_t zstride,
                                 u16* __restrict__ ZU, size_t zplane) {
  const int kv = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  int c, d;
  if (e < nvv) {
    c = (int)(e / nvb);
    d = (int)(e % nvb);
  } else {
    const int64_t s = e - nvv;
    c = nvpa + (int)(s / nob);
    d = nvpb + (int)(s % nob);
  }
  const double v = z[(int64_t)kv * n + e];
  const unsigned short h = bf16_rne((float)v);
  const double r1 = v - (double)bf16_to_f(h);
  const unsigned short m = bf16_rne((float)r1);
  const double r2 = r1 - (double)bf16_to_f(m);
  const unsigned short l = bf16_rne((float)r2);
  const size_t o = (size_t)kv * zstride + (size_t)c * nmopb + d;
  ZU[o] = h;
  ZU[o + zplane] = m;
  ZU[o + 2 * zplane] = l;
}

// LDS plan of the BF16 alpha-beta kernel (u16 elements): a staging buffer (contraction 1: rows c
// of Z and rows of Lb^P for the panel's columns, one 32-wide d block; contraction 2: RH rows of
// La^P, one 32-wide c block), then T of the current chunk as NPL planes [64 columns][TWP] (c
// contiguous; rows padded by 8 elements against bank conflicts).
template <int NPL>
struct AbBf16Cfg {
  static constexpr int CT = NPL == 3 ? 6 : 8;   // alpha c tiles per chunk (three planes: 69 KiB,
                                                // two workgroups per CU)
  static constexpr int RH = NPL == 3 ? 8 : 16;  // alpha row tiles per contraction-2 stage
  static constexpr int US = CT * TILE * KB;
  static constexpr int LS = 4 * TILE * KB;
  static constexpr int S1 = NPL * (US + LS);
  static constexpr int RS = RH * TILE * KB;
  static constexpr int S2 = NPL * RS;
  static constexpr int STAGE = S1 > S2 ? S1 : S2;
  static constexpr int TWP = CT * TILE + 8;
  static constexpr int TS = 4 * TILE * TWP;
  static constexpr int BUF = STAGE + NPL * TS;
};

// One work unit as in k_sandwich_ab (vector, panel of up to 4 beta column tiles, AB_RT alpha row
// tiles, aux range), 4 waves: contraction 1 by column (wave w: T of column tile w), contraction 2
// by rows (row tile 4 q + w of each contraction-2 stage to wave w, every column of the panel);
// NPROD = 6 (planes hi, mid, lo) or 3 (hi, mid) products per pair of operands. Partial Q in FP32.
template <int NPROD>
__global__ __launch_bounds__(256) void k_sandwich_ab_bf16(const u16* __restrict__ La,
                                                          const u16* __restrict__ Lb,
                                                          const u16* __restrict__ ZU,
                                                          float* __restrict__ Qp, AbParams a,
                                                          size_t plane_a, size_t plane_b,
                                                          size_t zplane) {
  constexpr int NPL = NPROD == 6 ? 3 : 2;
  using Cfg = AbBf16Cfg<NPL>;
  constexpr int RT = AB_RT, RH = Cfg::RH, CT = Cfg::CT;
  static_assert(RT % RH == 0 && RH % 4 == 0 && CT % 2 == 0, "tile groups");
  __shared__ __attribute__((aligned(1024))) u16 buf[Cfg::BUF];
  const int g = blockIdx.x;
  const int u = (g & 7) * a.per_xcd + (g >> 3);
  if (u >= a.nunits) return;
  const int item = a.items[(u / a.k) % a.nitems];
  const int kv = u % a.k;
  const int sp = u / (a.nitems * a.k);
  const int pn = item >> 16;
  const int R0 = item & 0xFFFF;
  const bool vblk = pn < a.npan_v;
  const int t0 = vblk ? 4 * pn : 4 * (pn - a.npan_v);
  const int bntb = vblk ? a.nvtb : (a.nctb - a.nvtb);
  const int bnta = vblk ? a.nvta : (a.ncta - a.nvta);
  const int col0 = (vblk ? 0 : a.nvpb) + t0 * TILE;
  const int row0 = (vblk ? 0 : a.nvpa) + R0 * TILE;
  const int npt = min(4, bntb - t0);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const bool active = w < npt;  // contraction 1: wave w computes T for column tile w
  const int wc = min(w, npt - 1);
  const int nrt = min(bnta, R0 + RT) - R0;
  const int ncol = npt * TILE;
  const int P0 = (int)((int64_t)a.naux * sp / a.nsplit);
  const int P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  const u16* __restrict__ Z = ZU + (int64_t)kv * a.zt_stride;
  u16* const sU = buf;
  u16* const sL = buf + NPL * Cfg::US;
  u16* const sT = buf + Cfg::STAGE;

  f4 S[RT / 4][4];
#pragma unroll
  for (int q = 0; q < RT / 4; ++q)
#pragma unroll
    for (int cw = 0; cw < 4; ++cw) S[q][cw] = f4{0, 0, 0, 0};

  for (int P = P0; P < P1; ++P) {
    const u16* __restrict__ Lap = La + (int64_t)P * a.la_stride;
    const u16* __restrict__ Lbp = Lb + (int64_t)P * a.lb_stride;
    for (int cc0 = 0; cc0 < a.ncta; cc0 += CT) {
      const int cc1 = min(cc0 + CT, a.ncta);
      f4 Tacc[CT];
#pragma unroll
      for (int i = 0; i < CT; ++i) Tacc[i] = f4{0, 0, 0, 0};
      // contraction 1: T[c][cols] = sum_d Z[c][d] Lb^P[d][cols]; part 0 pairs the chunk's alpha
      // virtual c tiles with the beta virtual d, part 1 its alpha occupied c tiles with the beta
      // occupied d; one 32-wide block of d per stage
      for (int part = 0; part < 2; ++part) {
        const int clo = part == 0 ? cc0 : max(cc0, a.nvta);
        const int chi = part == 0 ? min(cc1, a.nvta) : cc1;
        const int dlo = part == 0 ? 0 : a.nvtb, dhi = part == 0 ? a.nvtb : a.nctb;
        if (clo >= chi) continue;  // uniform
        for (int dt = dlo; dt < dhi; dt += 2) {
          __syncthreads();
#pragma unroll
          for (int p = 0; p < NPL; ++p) {
            dma_tile32(Z + p * zplane + (int64_t)(clo * TILE) * a.nmopb + dt * TILE, a.nmopb,
                       (chi - clo) * TILE, sU + p * Cfg::US, w, lane);
            dma_tile32(Lbp + p * plane_b + (int64_t)col0 * a.nmopb + dt * TILE, a.nmopb, ncol,
                       sL + p * Cfg::LS, w, lane);
          }
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
          if (active) {
            const int lrow = (wc * TILE + li) * KB + 8 * (lk ^ swz(li));
            bf8 bv[NPL];
#pragma unroll
            for (int p = 0; p < NPL; ++p) bv[p] = *(const bf8*)(sL + p * Cfg::LS + lrow);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const int cg = cc0 + ct;
              if (cg >= clo && cg < chi) {
                const int urow = ((cg - clo) * TILE + li) * KB + 8 * (lk ^ swz(li));
                bf8 av[NPL];
#pragma unroll
                for (int p = 0; p < NPL; ++p) av[p] = *(const bf8*)(sU + p * Cfg::US + urow);
                Tacc[ct] = split_mfma<NPROD>(av[0], av[1], av[NPL - 1], bv[0], bv[1], bv[NPL - 1],
                                             Tacc[ct]);
              }
            }
          }
        }
      }
      // T of this chunk into LDS, split, transposed: sT[p][col][c]; a lane holds rows
      // 4 lk .. 4 lk + 3 of each c tile for column li of its tile (the barrier: the previous
      // chunk's contraction 2 has read sT, also when this chunk had no contraction-1 stage)
      __syncthreads();
      if (active) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          bf4 tp[NPL];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            __bf16 h, m, l;
            split3(Tacc[ct][j], h, m, l);
            tp[0][j] = h;
            tp[1][j] = m;
            if (NPL == 3) tp[NPL - 1][j] = l;
          }
          const int o = (wc * TILE + li) * Cfg::TWP + ct * TILE + 4 * lk;
#pragma unroll
          for (int p = 0; p < NPL; ++p) *(bf4*)(sT + p * Cfg::TS + o) = tp[p];
        }
      }
      __syncthreads();
      // contraction 2: S[r][cols] += sum_c La^P[r][c] T[c][cols] over every c of the chunk (La^P
      // couples the alpha blocks), one 32-wide block of c (two tiles of T) at a time; B operands
      // from LDS, A (rows of La^P) staged RH row tiles at a time
#pragma unroll
      for (int cb = 0; cb < CT / 2; ++cb) {
        if (cc0 + 2 * cb < cc1) {
          bf8 B[4][NPL];
#pragma unroll
          for (int cw = 0; cw < 4; ++cw)
#pragma unroll
            for (int p = 0; p < NPL; ++p)
              B[cw][p] = *(const bf8*)(sT + p * Cfg::TS + (min(cw, npt - 1) * TILE + li) * Cfg::TWP +
                                       cb * KB + 8 * lk);
#pragma unroll
          for (int half = 0; half < RT / RH; ++half) {
            const int rh0 = half * RH;
            if (rh0 < nrt) {
              const int nr = min(RH, nrt - rh0);
              __syncthreads();
#pragma unroll
              for (int p = 0; p < NPL; ++p)
                dma_tile32(Lap + p * plane_a + (int64_t)(row0 + rh0 * TILE) * a.nmopa +
                               (cc0 + 2 * cb) * TILE,
                           a.nmopa, nr * TILE, buf + p * Cfg::RS, w, lane);
              __builtin_amdgcn_s_waitcnt(0);
              __syncthreads();
#pragma unroll
              for (int rr = 0; rr < RH / 4; ++rr) {
                const int r = 4 * rr + w;
                if (r < nr) {
                  const int o = (r * TILE + li) * KB + 8 * (lk ^ swz(li));
                  bf8 av[NPL];
#pragma unroll
                  for (int p = 0; p < NPL; ++p) av[p] = *(const bf8*)(buf + p * Cfg::RS + o);
#pragma unroll
                  for (int cw = 0; cw < 4; ++cw)
                    if (cw < npt)
                      S[half * (RH / 4) + rr][cw] =
                          split_mfma<NPROD>(av[0], av[1], av[NPL - 1], B[cw][0], B[cw][1],
                                            B[cw][NPL - 1], S[half * (RH / 4) + rr][cw]);
                }
              }
            }
          }
        }
      }
    }
  }

  float* __restrict__ out = Qp + ((int64_t)sp * a.k + kv) * a.q_stride;
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
              out[(int64_t)(row0 + rt * TILE + 4 * lk + j) * a.nmopb + col0 + cw * TILE + li] =
                  S[half * (RH / 4) + rr][cw][j];
      }
    }
}

}  // namespace

hipError_t launch_unpack_ab(const AbGeometry& g, Store st, const double* z, int k, void* ZT,
                            size_t zplane, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.n + 255) / 256), (unsigned)k);
  if (st == Store::BF16)
    hipLaunchKernelGGL(k_unpack_ab_bf16, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nvb, g.nob,
                       g.nvpa, g.nvpb, g.nmopb, (int64_t)g.nmopa * g.nmopb, (u16*)ZT, zplane);
  else if (st == Store::F64)
    hipLaunchKernelGGL(k_unpack_ab<double>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nvb, g.nob,
                       g.nvpa, g.nvpb, g.nmopa, g.nmopb, (double*)ZT);
  else if (st == Store::F32)
    hipLaunchKernelGGL(k_unpack_ab<float>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nvb, g.nob,
                       g.nvpa, g.nvpb, g.nmopa, g.nmopb, (float*)ZT);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sigma_ab(const AbGeometry& g, Store st, int nprod, const SigmaPlan& plan,
                           const void* La, const void* Lb, const void* ZT, size_t zplane, void* Qp,
                           int k, int nsplit, hipStream_t s) {
  AbParams p;
  p.nvta = g.nvta;
  p.ncta = g.ncta;
  p.nvtb = g.nvtb;
  p.nctb = g.nctb;
  p.nvpa = g.nvpa;
  p.nvpb = g.nvpb;
  p.nmopa = g.nmopa;
  p.nmopb = g.nmopb;
  p.naux = g.naux;
  p.k = k;
  p.nsplit = nsplit;
  p.nitems = plan.nitems;
  p.nunits = p.nitems * k * nsplit;
  p.per_xcd = (p.nunits + 7) / 8;
  p.npan_v = plan.npan_v;
  p.items = plan.d_items;
  p.la_stride = (int64_t)g.nmopa * g.nmopa;
  p.lb_stride = (int64_t)g.nmopb * g.nmopb;
  p.zt_stride = (int64_t)g.nmopb * g.nmopa;
  p.q_stride = (int64_t)g.nmopa * g.nmopb;
  if (st == Store::F64)
    hipLaunchKernelGGL((k_sandwich_ab<double, AB_CT, AB_RT>), dim3(p.per_xcd * 8), dim3(256), 0, s,
                       (const double*)La, (const double*)Lb, (const double*)ZT, (double*)Qp, p);
  else if (st == Store::F32)
    hipLaunchKernelGGL((k_sandwich_ab<float, AB_CT, AB_RT>), dim3(p.per_xcd * 8), dim3(256), 0, s,
                       (const float*)La, (const float*)Lb, (const float*)ZT, (float*)Qp, p);
  else if (nprod == 6)
    hipLaunchKernelGGL(k_sandwich_ab_bf16<6>, dim3(p.per_xcd * 8), dim3(256), 0, s,
                       (const u16*)La, (const u16*)Lb, (const u16*)ZT, (float*)Qp, p,
                       (size_t)g.naux * p.la_stride, (size_t)g.naux * p.lb_stride, zplane);
  else if (nprod == 3)
    hipLaunchKernelGGL(k_sandwich_ab_bf16<3>, dim3(p.per_xcd * 8), dim3(256), 0, s,
                       (const u16*)La, (const u16*)Lb, (const u16*)ZT, (float*)Qp, p,
                       (size_t)g.naux * p.la_stride, (size_t)g.naux * p.lb_stride, zplane);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_epilogue_ab(const AbGeometry& g, Store st, const double* z, int k,
                              const void* Qp, int nsplit, const double* epair, double* sigma,
                              hipStream_t s) {
  if (k <= 0) return hipSuccess;
  const int64_t q_stride = (int64_t)g.nmopa * g.nmopb;
  dim3 grid((unsigned)((g.n + 255) / 256), (unsigned)k);
  if (st == Store::F64)
    hipLaunchKernelGGL(k_epilogue_ab<double>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nvb, g.nob,
                       g.nvpa, g.nvpb, g.nmopb, (const double*)Qp, nsplit, (int64_t)k * q_stride,
                       q_stride, epair, sigma);
  else if (st == Store::F32 || st == Store::BF16)
    hipLaunchKernelGGL(k_epilogue_ab<float>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nvb, g.nob,
                       g.nvpa, g.nvpb, g.nmopb, (const float*)Qp, nsplit, (int64_t)k * q_stride,
                       q_stride, epair, sigma);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Work items of the alpha-beta sigma kernel: panels of up to 4 beta column tiles of each
// diagonal block, with the alpha row tiles of the block in ranges of AB_RT.
void make_sigma_items_ab(const AbGeometry& g, std::vector<int>& items, int& npan_v) {
  items.clear();
  npan_v = (g.nvtb + 3) / 4;
  const int npan_o = (g.nctb - g.nvtb + 3) / 4;
  const int rows_v = g.nvta, rows_o = g.ncta - g.nvta;
  for (int pn = 0; pn < npan_v + npan_o; ++pn) {
    const int rows = pn < npan_v ? rows_v : rows_o;
    for (int R0 = 0; R0 < rows; R0 += AB_RT) items.push_back((pn << 16) | R0);
  }
}

}  // namespace pprpa
