// Pieces shared by the sigma kernels (k_sigma.hip: FP64/FP32, k_sigma_bf16.hip: BF16-split).
#pragma once

#include "internal.h"

namespace pprpa {

// One sigma product's decomposition into work units (one workgroup each): unit u ->
// (work item u % nitems, vector (u / nitems) % k, aux split u / (nitems k)).
struct SandParams {
  int nvp, nop, nmop, nvt, nct, naux;
  int k, nsplit, nitems, nunits, per_xcd;
  int64_t zstride;  // nmop * nmop
  const int* items; // [nitems]: panel index << 16 | first row tile of the range
  int npan_v;
};

// c tiles of the chunk a contraction-1 step on d tile dt touches, rounded out to groups of 4
// (columns outside the valid range hold exact zeros in U^T: c > d, or the other block).
__device__ __forceinline__ void c_range(int dt, int cc0, int cc1, int nvt, int* g0, int* g1) {
  const int blo = dt < nvt ? 0 : nvt;            // first c tile of d's block
  const int lo = max(cc0, blo);                   // lowest c tile used
  const int hi = min(cc1, dt + 1);                // one past the highest (c <= d)
  *g0 = cc0 + ((lo - cc0) & ~3);
  *g1 = min(cc1, cc0 + ((hi - cc0 + 3) & ~3));
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Issue this wave's share of the direct global->LDS loads of a rows x cols tile (packed in LDS at
// dst, row stride cols). Each wave load moves 64 lanes x 16 bytes into 1 KiB of contiguous LDS.
template <typename T>
__device__ __forceinline__ void dma_tile(const T* __restrict__ src, int64_t ld, int rows, int cols,
                                         T* dst, int w, int lane) {
  constexpr int VEC = 16 / sizeof(T), CHUNK = 1024 / sizeof(T);
  const int nchunk = rows * cols / CHUNK;
  for (int j = w; j < nchunk; j += 4) {
    const int e = j * CHUNK + lane * VEC;
    const int row = e / cols, col = e - row * cols;
    __builtin_amdgcn_global_load_lds((const void*)(src + row * ld + col), (lds_ptr_t)(dst + j * CHUNK),
                                     16, 0, 0);
  }
}

}  // namespace pprpa
