// FP64 density-fitted sigma contraction on CDNA4 (gfx950): the sandwich Q = sum_P L^P U L^P of
// the ppRPA sigma product (arXiv 2512.12515, section "ppRPA Equation", Eq. eigen_equation with the
// spin-adapted A, B, C; the algebra, the packed layouts and the epilogue are those of
// k_sigma.hip) in a software-pipelined form:
//
//   * one workgroup of 8 waves per CU (two waves per SIMD, so one wave's LDS operand waits are
//     covered by the other's MFMAs) with two LDS stage buffers of 72 KiB: while the waves run
//     the MFMAs of stage s from one buffer, the direct global->LDS loads of stage s + 1 fill the
//     other, so the staging latency hides behind the products (one barrier per stage);
//   * a work unit is one vector, a panel of up to 4 adjacent 16-column tiles of one diagonal
//     block, up to 32 row tiles of that block and a range of the aux index; the waves of a
//     column (two for a four-tile panel) share out its c groups in contraction 1, exchange their
//     T tiles through the buffer just used, and split its row tiles in contraction 2, so
//     contraction 1 (T = U L^P[:, cols], the triangle d >= c) is computed once for up to 32 row
//     tiles and each wave holds at most 16 row tiles of Q and 8 c tiles of T in registers;
//   * the stage sequence of a unit (per P, per chunk of 8 c tiles: contraction-1 stages of three
//     d tiles of U^T and L^P[:, cols], then contraction-2 stages of as many c tiles of
//     L^P[c][rows] as a buffer holds) is walked by a small iterator in uniform registers, one
//     step ahead for the loads;
//   * partial Q per aux split, summed in a fixed order by the epilogue (deterministic); unit ids
//     remapped so each XCD runs a contiguous range, vector index fastest (the units sharing a
//     panel's L^P tiles run together on one XCD and share its L2).
#include "internal.h"
#include "sigma_common.h"

namespace pprpa {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FP64 16x16x4: row lk + 4 j of the output tile sits in accumulator register j of lane group lk.
__device__ __forceinline__ int acc_row64(int lk, int j) { return lk + 4 * j; }

constexpr int NW = 8;     // waves per workgroup
constexpr int CT = 8;     // c tiles per chunk (T tiles per wave)
constexpr int RW = 16;    // row tiles of Q per wave
constexpr int RTU = 32;   // row tiles per work unit
constexpr int GRP = 2;    // tiles per unrolled MFMA group
constexpr int ND = 3;     // d tiles per contraction-1 stage
constexpr int S1 = ND * TILE * CT * TILE + ND * TILE * 4 * TILE;  // a contraction-1 stage
constexpr int S2 = TILE * RTU * TILE;  // one contraction-2 c tile at the widest row range
constexpr int BUF = S1 > S2 ? S1 : S2;  // doubles per stage buffer
constexpr int SBOFF = ND * TILE * CT * TILE;  // offset of the L^P[d][cols] tile in a C1 stage
static_assert(4 * CT * 4 * 64 <= BUF, "the T exchange of a four-column panel fits a buffer");

// Stages of one unit in order: for P in [P, P1): for each chunk [cc0, cc1) of CT c tiles:
// contraction-1 part 0 (d over [cc0, nvt): the virtual block, when the chunk starts in it), part 1
// (d over [max(cc0, nvt), nct): the occupied block, when the chunk reaches it), ND d tiles per
// stage; then part 2, contraction 2 over the chunk's c tiles, nb2 per stage. pos is the first d
// (parts 0, 1) or c (part 2) tile of the stage.
struct StageIt {
  int nvt, nct, P1, nb2;
  int P, cc0, cc1, part, pos;
  bool valid;

  __device__ __forceinline__ int hi() const {
    if (part == 0) return cc0 < nvt ? nvt : cc0;
    if (part == 1) return cc1 > nvt ? nct : max(cc0, nvt);
    return cc1;
  }
  // move forward to the next non-empty position (from a position that may be past its part's end)
  __device__ __forceinline__ void settle() {
    for (;;) {
      if (pos < hi()) return;
      if (part == 0) {
        part = 1;
        pos = max(cc0, nvt);
      } else if (part == 1) {
        part = 2;
        pos = cc0;
      } else {
        cc0 += CT;
        if (cc0 >= nct) {
          cc0 = 0;
          if (++P >= P1) {
            valid = false;
            return;
          }
        }
        cc1 = min(cc0 + CT, nct);
        part = 0;
        pos = cc0;
      }
    }
  }
  __device__ __forceinline__ void advance() {
    pos += part < 2 ? ND : nb2;
    settle();
  }
  __device__ __forceinline__ int count() const { return min(part < 2 ? ND : nb2, hi() - pos); }
};

__device__ __forceinline__ void sandwich_f64_unit(const double* __restrict__ L,
                                                  const double* __restrict__ UT,
                                                  double* __restrict__ Qp, const SandParams& a,
                                                  int u, double* __restrict__ buf) {
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
  // parts waves per column tile: they share out its c groups in contraction 1 (group g to the
  // wave with g % parts == rsel) and split its row tiles in contraction 2; a three-tile panel
  // idles two waves
  const int parts = npt == 1 ? 8 : (npt == 2 ? 4 : 2);
  const bool active = w < npt * parts;
  const int wc = w % npt;
  const int rsel = w / npt;
  const int nrt = min(bnt - R0, RTU);
  // contraction 2: the waves of a column take contiguous runs of its row tiles, rwp each (a
  // multiple of GRP), wave rsel from row tile rsel * rwp
  const int rwp = ((nrt + parts - 1) / parts + GRP - 1) / GRP * GRP;
  const int rlo = rsel * rwp;                   // first row tile of this wave
  const int rcnt = max(0, min(rwp, nrt - rlo)); // its row tiles
  const int col0 = brow0 + t0 * TILE;
  const int ncol = npt * TILE;
  const int row0 = brow0 + R0 * TILE;
  const int wl = nrt * TILE;  // row stride of a staged contraction-2 tile
  const double* __restrict__ Z = UT + (int64_t)kv * a.zstride;

  StageIt it;
  it.nvt = a.nvt;
  it.nct = a.nct;
  it.P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  // contraction-2 c tiles per stage: as many as a buffer holds at this row width (with an odd
  // row count TILE elements stay free past the last tile for the unused second tile of the last
  // row group)
  it.nb2 = min(CT, (BUF - ((nrt & 1) ? TILE : 0)) / (TILE * wl));
  it.P = (int)((int64_t)a.naux * sp / a.nsplit);
  it.cc0 = 0;
  it.cc1 = min(CT, a.nct);
  it.part = 0;
  it.pos = 0;
  it.valid = it.P < it.P1;
  if (it.valid) it.settle();

  d4 S[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) S[r] = d4{0, 0, 0, 0};
  d4 Tacc[CT];
#pragma unroll
  for (int i = 0; i < CT; ++i) Tacc[i] = d4{0, 0, 0, 0};

  // loads of the stage at `s` into buffer b
  auto issue = [&](const StageIt& s, double* b) {
    const double* __restrict__ Lp = L + (int64_t)s.P * a.zstride;
    const int n = s.count();
    if (s.part < 2) {
      int g0, g1, h0, h1;
      c_range(s.pos, s.cc0, s.cc1, a.nvt, &g0, &g1);
      c_range(s.pos + n - 1, s.cc0, s.cc1, a.nvt, &h0, &h1);
      const int wa = (h1 - g0) * TILE;
      dma_tile<double, NW>(Z + (int64_t)(s.pos * TILE) * a.nmop + g0 * TILE, a.nmop, n * TILE, wa,
                           b, w, lane);
      dma_tile<double, NW>(Lp + (int64_t)(s.pos * TILE) * a.nmop + col0, a.nmop, n * TILE, ncol,
                           b + SBOFF, w, lane);
    } else {
      dma_tile<double, NW>(Lp + (int64_t)(s.pos * TILE) * a.nmop + row0, a.nmop, n * TILE, wl, b,
                           w, lane);
    }
  };

  // The nested loops below walk the stages in the iterator's order; nx, one stage ahead, names
  // the stage whose loads are issued while the current one computes.
  StageIt nx = it;
  if (nx.valid) {
    issue(nx, buf);
    nx.advance();
  }
  int stage = 0;
  double* cur = buf;
  // wait for the current stage's loads (this wave's, then everyone's: the barrier also means the
  // other buffer is no longer read) and start the next stage's loads into the other buffer
  auto next_stage = [&]() {
    cur = buf + (stage & 1) * BUF;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (nx.valid) {
      issue(nx, buf + ((stage + 1) & 1) * BUF);
      nx.advance();
    }
    ++stage;
  };
  const int P0 = it.P, P1 = it.P1;
  for (int P = P0; P < P1; ++P) {
    for (int cc0 = 0; cc0 < a.nct; cc0 += CT) {
      const int cc1 = min(cc0 + CT, a.nct);
      // contraction 1: T[c][cols] = sum_{d >= c} U[c][d] L^P[d][cols], d in c's block
      for (int part = 0; part < 2; ++part) {
        const int lo = part == 0 ? cc0 : max(cc0, a.nvt);
        const int hi = part == 0 ? (cc0 < a.nvt ? a.nvt : cc0) : (cc1 > a.nvt ? a.nct : lo);
        for (int dt = lo; dt < hi; dt += ND) {
          next_stage();
          const int n = min(ND, hi - dt);
          int g0, g1, h0, h1;
          c_range(dt, cc0, cc1, a.nvt, &g0, &g1);
          c_range(dt + n - 1, cc0, cc1, a.nvt, &h0, &h1);
          const int wa = (h1 - g0) * TILE;
#pragma unroll
          for (int sub = 0; sub < ND; ++sub) {
            if (sub < n) {
              int q0, q1g;
              c_range(dt + sub, cc0, cc1, a.nvt, &q0, &q1g);
              const int q1 = min(cc1, dt + sub + 1);  // end of the nonzero c tiles (c <= d)
              const double* sA = cur + sub * TILE * wa;
              const double* sB = cur + SBOFF + sub * TILE * ncol;
              double bv[4];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) bv[ks] = sB[(4 * ks + lk) * ncol + wc * TILE + li];
#pragma unroll
              for (int grp = 0; grp < CT / GRP; ++grp) {
                const int cg = cc0 + GRP * grp;
                if (active && cg >= q0 && cg < q1 && grp % parts == rsel) {
                  double av[4][GRP];
#pragma unroll
                  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = 0; j < GRP; ++j)
                      av[ks][j] = sA[(4 * ks + lk) * wa + (cg - g0 + j) * TILE + li];
                  __builtin_amdgcn_sched_barrier(0);  // the group's operands ahead of its products
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
      // each wave of a column takes the T tiles of the other waves' c groups (same values, same
      // summation order as computing them itself) through the buffer of the last contraction-1
      // stage, which nothing reads or loads into until the next stage; layout [column][tile]
      // [register][lane], conflict-free
      __syncthreads();  // every wave is done reading that stage
      if (active) {
#pragma unroll
        for (int i = 0; i < CT; ++i)
          if ((i / GRP) % parts == rsel)
#pragma unroll
            for (int j = 0; j < 4; ++j) cur[((wc * CT + i) * 4 + j) * 64 + lane] = Tacc[i][j];
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int i = 0; i < CT; ++i)
          if ((i / GRP) % parts != rsel)
#pragma unroll
            for (int j = 0; j < 4; ++j) Tacc[i][j] = cur[((wc * CT + i) * 4 + j) * 64 + lane];
      }
      // contraction 2: Q[rows][cols] += sum_c L^P[rows][c] T[c][cols], T from registers (the
      // reduction index permuted to its accumulator layout), nb2 c tiles per stage
      for (int ci = cc0; ci < cc1; ci += it.nb2) {
        next_stage();
        const int n = min(it.nb2, cc1 - ci);
#pragma unroll
        for (int i = 0; i < CT; ++i) {
          const int slot = cc0 + i - ci;
          if (slot >= 0 && slot < n) {
            // this lane's element of the wave's first row tile, reduction row lk (the A operand
            // of step ks is 4 ks rows further down)
            const double* sL = cur + slot * TILE * wl + lk * wl + rlo * TILE + li;
#pragma unroll
            for (int jg = 0; jg < RW / GRP; ++jg) {
              // a last group reaching past nrt reads other data of the buffer (in bounds); its
              // second tile's results are never stored
              if (active && GRP * jg < rcnt) {
                double av[4][GRP];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                  for (int j = 0; j < GRP; ++j)
                    av[ks][j] = sL[4 * ks * wl + (GRP * jg + j) * TILE];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                  for (int j = 0; j < GRP; ++j)
                    S[GRP * jg + j] = mfma64(av[ks][j], Tacc[i][ks], S[GRP * jg + j]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < CT; ++i) Tacc[i] = d4{0, 0, 0, 0};
    }
  }

  if (active) {
    double* __restrict__ out = Qp + ((int64_t)sp * a.k + kv) * a.zstride;
    const int col = col0 + wc * TILE + li;
#pragma unroll
    for (int jg = 0; jg < RW / GRP; ++jg) {
#pragma unroll
      for (int j = 0; j < GRP; ++j) {
        const int rt = rlo + GRP * jg + j;
        if (GRP * jg + j < rcnt) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            out[(int64_t)(row0 + rt * TILE + acc_row64(lk, r)) * a.nmop + col] = S[GRP * jg + j][r];
        }
      }
    }
  }
}

__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
void k_sandwich_f64(const double* __restrict__ L, const double* __restrict__ UT,
                    double* __restrict__ Qp, SandParams a) {
  __shared__ __attribute__((aligned(1024))) double buf[2 * BUF];
  const int g = blockIdx.x;
  const int u = (g & 7) * a.per_xcd + (g >> 3);
  if (u >= a.nunits) return;
  sandwich_f64_unit(L, UT, Qp, a, u, buf);
}

// Grouped launch (serving): the units of several products laid end to end; a unit does exactly
// what it does in its own product's launch.
__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
void k_sandwich_f64_group(GroupArgs ga) {
  __shared__ __attribute__((aligned(1024))) double buf[2 * BUF];
  const int g = blockIdx.x;
  const int u = (g & 7) * ga.per_xcd + (g >> 3);
  if (u >= ga.u0[ga.n]) return;
  int e = 0;
  while (e + 1 < ga.n && u >= ga.u0[e + 1]) ++e;
  sandwich_f64_unit((const double*)ga.e[e].L, (const double*)ga.e[e].UT, (double*)ga.e[e].Qp,
                    ga.e[e].p, u - ga.u0[e], buf);
}

}  // namespace

hipError_t launch_sigma_f64(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                            hipStream_t s) {
  const SandParams p = sand_params(g, plan, la);
  hipLaunchKernelGGL(k_sandwich_f64, dim3(p.per_xcd * 8), dim3(NW * 64), 0, s, (const double*)la.L,
                     (const double*)la.ZT, (double*)la.Sp, p);
  return hipGetLastError();
}

hipError_t launch_sigma_group_f64(const GroupMember* m, int n, hipStream_t s) {
  const GroupArgs ga = group_args(m, n);
  hipLaunchKernelGGL(k_sandwich_f64_group, dim3(ga.per_xcd * 8), dim3(NW * 64), 0, s, ga);
  return hipGetLastError();
}

}  // namespace pprpa
