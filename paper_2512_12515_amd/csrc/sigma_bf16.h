// BF16-split pieces shared by the sigma kernels (the restricted kernels of k_sigma_bf16.hip,
// the staging and unpack kernels of k_sigma.hip, the alpha-beta kernel of k_sigma_ab.hip): a
// value x is carried as three BF16 planes hi + mid + lo (hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid)); a product takes the six (or three) largest of the nine plane
// products on the BF16 MFMA with FP32 accumulation.
#pragma once

#include "sigma_common.h"

namespace pprpa {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int KB = 32;  // reduction block of one MFMA

// Round to nearest even into BF16 (the bits of a float's upper half), and back.
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  unsigned r = 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)((u + r) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

// LDS layout of a staged rows x 32 BF16 tile: each 64-byte row holds four 16-byte chunks, stored
// at position kc ^ swz(row) so that the lanes one LDS cycle serves (rows r .. r+7 or r .. r+15 of
// one chunk column) fall in distinct banks. The direct global->LDS loads write each wave's 1 KiB
// contiguously, so the permutation is applied to the global addresses instead.
__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

template <int NWV = 4>
__device__ __forceinline__ void dma_tile32(const u16* __restrict__ src, int64_t ld, int rows,
                                           u16* dst, int w, int lane) {
  const int nchunk = rows / 16;  // 16 rows x 64 bytes per wave load
  for (int j = w; j < nchunk; j += NWV) {
    const int row = j * 16 + (lane >> 2), pos = lane & 3;
    __builtin_amdgcn_global_load_lds((const void*)(src + row * ld + 8 * (pos ^ swz(row))),
                                     (lds_ptr_t)(dst + j * 512), 16, 0, 0);
  }
}

__device__ __forceinline__ f4 mfma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// a b over the split planes (NPROD = 6 or 3 products).
template <int NPROD>
__device__ __forceinline__ f4 split_mfma(bf8 ah, bf8 am, bf8 al, bf8 bh, bf8 bm, bf8 bl, f4 c) {
  c = mfma(ah, bh, c);
  c = mfma(ah, bm, c);
  c = mfma(am, bh, c);
  if (NPROD == 6) {
    c = mfma(am, bm, c);
    c = mfma(ah, bl, c);
    c = mfma(al, bh, c);
  }
  return c;
}

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r1 = x - (float)h;  // exact
  m = (__bf16)r1;
  const float r2 = r1 - (float)m;  // exact
  l = (__bf16)r2;
}

}  // namespace
}  // namespace pprpa
