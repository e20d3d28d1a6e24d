// Pieces shared by the sigma kernels (k_sigma.hip: FP64/FP32, k_sigma_bf16.hip: BF16-split).
#pragma once

#include "internal.h"

namespace pprpa {

// One sigma product's decomposition into work units (one workgroup each): unit u ->
// (vector u % k, work item (u / k) % nitems, aux split u / (nitems k)). The vector index runs
// fastest, so the k units that stage the same L^P tiles are launched together.
struct SandParams {
  int nvp, nop, nmop, nvt, nct, naux;
  int k, nsplit, nitems, nunits, per_xcd;
  int64_t zstride;  // nmop * nmop
  const int* items; // [nitems]: panel index << 16 | first row tile of the range
  int npan_v;
};

// Entries of a grouped sigma launch (passed by value as the kernel argument).
struct GroupEntry {
  const void* L;
  const void* UT;
  void* Qp;
  size_t plane, zplane;  // BF16 plane strides (elements)
  SandParams p;
};
struct GroupArgs {
  int n, per_xcd;
  int u0[GROUP_MAX + 1];  // first unit of each entry; u0[n] = total units
  GroupEntry e[GROUP_MAX];
};

// Host-side parameters of one product's launch (shared by the single and grouped launchers).
inline SandParams sand_params(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la) {
  SandParams p;
  p.nvp = g.nvp;
  p.nop = g.nop;
  p.nmop = g.nmop;
  p.nvt = g.nvt;
  p.nct = g.nct;
  p.naux = g.naux;
  p.k = la.k;
  p.nsplit = la.nsplit;
  p.nitems = plan.nitems;
  p.nunits = p.nitems * la.k * la.nsplit;
  const int nwg = (p.nunits + 7) / 8 * 8;
  p.per_xcd = nwg / 8;
  p.zstride = (int64_t)g.nmop * g.nmop;
  p.npan_v = plan.npan_v;
  p.items = plan.d_items;
  return p;
}

// Grouped launch arguments for members m[0..n): units laid end to end.
inline GroupArgs group_args(const GroupMember* m, int n) {
  GroupArgs ga{};
  ga.n = n;
  int total = 0;
  for (int i = 0; i < n; ++i) {
    ga.e[i].L = m[i].la.L;
    ga.e[i].UT = m[i].la.ZT;
    ga.e[i].Qp = m[i].la.Sp;
    ga.e[i].plane = m[i].la.plane;
    ga.e[i].zplane = m[i].la.zplane;
    ga.e[i].p = sand_params(*m[i].g, *m[i].plan, m[i].la);
    ga.u0[i] = total;
    total += ga.e[i].p.nunits;
  }
  ga.u0[n] = total;
  ga.per_xcd = (total + 7) / 8;
  return ga;
}

// c tiles of the chunk a contraction-1 step on d tile dt touches, rounded out to pairs counted
// from cc0 (the MFMA loops take tiles two at a time; columns outside the valid range hold exact
// zeros in U^T: c > d, or the other block).
__device__ __forceinline__ void c_range(int dt, int cc0, int cc1, int nvt, int* g0, int* g1) {
  const int blo = dt < nvt ? 0 : nvt;            // first c tile of d's block
  const int lo = max(cc0, blo);                   // lowest c tile used
  const int hi = min(cc1, dt + 1);                // one past the highest (c <= d)
  *g0 = cc0 + ((lo - cc0) & ~1);
  *g1 = min(cc1, cc0 + ((hi - cc0 + 1) & ~1));
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Issue this wave's share (wave w of NWAVES) of the direct global->LDS loads of a rows x cols
// tile (packed in LDS at dst, row stride cols). Each wave load moves 64 lanes x 16 bytes into
// 1 KiB of contiguous LDS.
template <typename T, int NWAVES = 4>
__device__ __forceinline__ void dma_tile(const T* __restrict__ src, int64_t ld, int rows, int cols,
                                         T* dst, int w, int lane) {
  constexpr int VEC = 16 / sizeof(T), CHUNK = 1024 / sizeof(T);
  const int nchunk = rows * cols / CHUNK;
  for (int j = w; j < nchunk; j += NWAVES) {
    const int e = j * CHUNK + lane * VEC;
    const int row = e / cols, col = e - row * cols;
    __builtin_amdgcn_global_load_lds((const void*)(src + row * ld + col), (lds_ptr_t)(dst + j * CHUNK),
                                     16, 0, 0);
  }
}

}  // namespace pprpa
