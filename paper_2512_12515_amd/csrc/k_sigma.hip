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
//   * a workgroup owns one vector, a panel of up to 4 adjacent 16-column tiles of one diagonal
//     block of S, a range of up to RT row tiles, and a contiguous range of the aux index P;
//     wave w owns column tile w of the panel;
//   * per P: contraction 1, T[c][cols] = sum_d Zh[c][d] L^P[d][cols], accumulates in registers
//     (CC row blocks of T at a time); contraction 2, S[r][cols] += sum_c L^P[r][c] T[c][cols],
//     takes T straight from those registers as its B operand (the reduction index c is
//     permuted to match the MFMA output layout, acc_row, and the A operand is read with the
//     same permutation), so T never leaves the register file;
//   * the A operands (rows of Zh and of L^P) are shared by the 4 waves and staged in LDS with
//     coalesced 16-byte loads; L^P and Zh being symmetric (antisymmetric), every staged tile is a
//     contiguous row segment in HBM;
//   * S is symmetric (antisymmetric for the triplet) so only row tiles <= the column tile are
//     computed (upper triangle of tiles);
//   * the aux index is split over workgroups; partial S per split are summed in the epilogue in
//     a fixed order (deterministic);
//   * workgroup ids are remapped so the 8 XCDs each take a contiguous range of work units, which
//     share P ranges and vectors in that XCD's L2.
#include "internal.h"

namespace pprpa {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

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

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  unsigned r = 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)((u + r) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

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
// Unpack packed vectors into ZT[k][nmop][nmop] = Zh^T (only the two diagonal blocks written).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double unpacked_value(const double* __restrict__ zk, int nb, int mult,
                                                 int c, int d) {
  // Zh[c][d] for one diagonal block of size nb; zk points at the block's packed entries.
  if (c >= nb || d >= nb) return 0.0;
  const int p = c < d ? c : d, q = c < d ? d : c;
  if (mult == 0) {
    const int64_t idx = (int64_t)p * nb - (int64_t)p * (p - 1) / 2 + (q - p);
    const double v = zk[idx];
    return p == q ? v * 1.4142135623730951 : v;
  }
  if (p == q) return 0.0;
  const int64_t idx = (int64_t)p * (nb - 1) - (int64_t)p * (p - 1) / 2 + (q - p - 1);
  const double v = zk[idx];
  return c < d ? v : -v;
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
  const size_t o = ((size_t)kv * nmop + off + d) * nmop + off + c;
  ZT[o] = h;
  ZT[o + zplane] = m;
  ZT[o + 2 * zplane] = l;
}

// ------------------------------------------------------------------------------------------
// Fused sandwich kernel (FP64 / FP32 MFMA).
// ------------------------------------------------------------------------------------------
struct SandParams {
  int nvp, nop, nmop, nvt, nct, naux;
  int k, nsplit, nitems, nunits, per_xcd;
  int64_t zstride;  // nmop * nmop
  const int* items; // [nitems]: panel index << 16 | first row tile of the range
  int npan_v;
};

// Copy a rows x cols tile (cols a multiple of 16 elements, 16-byte aligned rows) into LDS.
template <typename T>
__device__ __forceinline__ void stage_tile(T* __restrict__ dst, int ldd, const T* __restrict__ src,
                                           int64_t lds, int rows, int cols) {
  constexpr int VEC = 16 / sizeof(T);
  const int nvr = cols / VEC;
  const int total = rows * nvr;
  for (int v = threadIdx.x; v < total; v += 256) {
    const int r = v / nvr, c = (v - r * nvr) * VEC;
    const uint4 x = *reinterpret_cast<const uint4*>(src + r * lds + c);
    *reinterpret_cast<uint4*>(dst + r * ldd + c) = x;
  }
}

template <typename T, int CC, int RT>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 2)))
void k_sandwich(const T* __restrict__ L, const T* __restrict__ ZT, T* __restrict__ Sp,
                SandParams a) {
  using V = typename AccT<T>::V;
  constexpr int PAD = 16 / sizeof(T);
  constexpr int WA = CC * TILE + PAD;
  constexpr int WB = 4 * TILE + PAD;
  constexpr int WL = RT * TILE + PAD;
  __shared__ __attribute__((aligned(16))) T sA[TILE * WA];
  __shared__ __attribute__((aligned(16))) T sB[TILE * WB];
  __shared__ __attribute__((aligned(16))) T sL[TILE * WL];

  const int g = blockIdx.x;
  const int u = (g & 7) * a.per_xcd + (g >> 3);
  if (u >= a.nunits) return;
  const int item = a.items[u % a.nitems];
  const int kv = (u / a.nitems) % a.k;
  const int sp = u / (a.nitems * a.k);
  const int pn = item >> 16;
  const int R0 = item & 0xFFFF;  // first row tile (local to the block)

  const bool vblk = pn < a.npan_v;
  const int t0 = vblk ? 4 * pn : 4 * (pn - a.npan_v);
  const int bnt = vblk ? a.nvt : (a.nct - a.nvt);
  const int brow0 = vblk ? 0 : a.nvp;
  const int npt = min(4, bnt - t0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mytile = t0 + w;
  const bool active = w < npt;
  const int rend = min(t0 + npt, R0 + RT);            // row tiles [R0, rend) staged
  const int nrt = active ? max(0, min(mytile + 1, R0 + RT) - R0) : 0;
  const int P0 = (int)((int64_t)a.naux * sp / a.nsplit);
  const int P1 = (int)((int64_t)a.naux * (sp + 1) / a.nsplit);
  const T* __restrict__ Z = ZT + (int64_t)kv * a.zstride;

  V S[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) S[r] = V{0, 0, 0, 0};

  for (int P = P0; P < P1; ++P) {
    const T* __restrict__ Lp = L + (int64_t)P * a.zstride;
    for (int cc0 = 0; cc0 < a.nct; cc0 += CC) {
      const int cc1 = min(cc0 + CC, a.nct);
      V Tacc[CC];
#pragma unroll
      for (int i = 0; i < CC; ++i) Tacc[i] = V{0, 0, 0, 0};

      // contraction 1: T[c][cols] = sum_d Zh[c][d] L^P[d][cols], d in the block of c
      for (int part = 0; part < 2; ++part) {
        const int cb0 = part == 0 ? cc0 : max(cc0, a.nvt);
        const int cb1 = part == 0 ? min(cc1, a.nvt) : cc1;
        if (cb0 >= cb1) continue;
        const int dbase = part == 0 ? 0 : a.nvp;
        const int dlen = part == 0 ? a.nvp : a.nop;
        const int ncol = (cb1 - cb0) * TILE;
        for (int d0 = 0; d0 < dlen; d0 += TILE) {
          __syncthreads();
          stage_tile(sA, WA, Z + (int64_t)(dbase + d0) * a.nmop + cb0 * TILE, a.nmop, TILE, ncol);
          stage_tile(sB, WB, Lp + (int64_t)(dbase + d0) * a.nmop + brow0 + t0 * TILE, a.nmop, TILE,
                     npt * TILE);
          __syncthreads();
          if (active) {
            T b[4];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) b[ks] = sB[(4 * ks + lk) * WB + w * TILE + li];
#pragma unroll
            for (int i = 0; i < CC; ++i) {
              const int cb = cc0 + i;
              if (cb >= cb0 && cb < cb1) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                  const T av = sA[(4 * ks + lk) * WA + (cb - cb0) * TILE + li];
                  Tacc[i] = mfma(av, b[ks], Tacc[i]);
                }
              }
            }
          }
        }
      }

      // contraction 2: S[r][cols] += sum_c L^P[r][c] T[c][cols], T from registers
#pragma unroll
      for (int i = 0; i < CC; ++i) {
        const int cb = cc0 + i;
        if (cb < cc1) {
          __syncthreads();
          stage_tile(sL, WL, Lp + (int64_t)(cb * TILE) * a.nmop + brow0 + R0 * TILE, a.nmop, TILE,
                     (rend - R0) * TILE);
          __syncthreads();
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            if (rt < nrt) {
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) {
                const T av = sL[acc_row<T>(lk, ks) * WL + rt * TILE + li];
                S[rt] = mfma(av, Tacc[i][ks], S[rt]);
              }
            }
          }
        }
      }
    }
  }

  if (active) {
    T* __restrict__ out = Sp + ((int64_t)sp * a.k + kv) * a.zstride;
    const int col = brow0 + mytile * TILE + li;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (rt < nrt) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          out[(int64_t)(brow0 + (R0 + rt) * TILE + acc_row<T>(lk, j)) * a.nmop + col] = S[rt][j];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Epilogue: sigma = E z + N * sum_splits S (upper triangle), FP64.
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_epilogue(const double* __restrict__ z, int64_t n, int64_t nvv, int nvp,
                           int nmop, int mult, const T* __restrict__ Sp, int nsplit,
                           int64_t split_stride, const int* __restrict__ ptab,
                           const double* __restrict__ epair, double* __restrict__ sigma) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int kv = blockIdx.y;
  if (e >= n) return;
  const int pq = ptab[e];
  const int p = pq >> 16, q = pq & 0xFFFF;
  const int off = e < nvv ? 0 : nvp;
  const int64_t si = ((int64_t)kv * nmop + off + p) * nmop + off + q;
  double s = 0.0;
  for (int t = 0; t < nsplit; ++t) s += (double)Sp[t * split_stride + si];
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
  dim3 grid((unsigned)((g.n + 255) / 256), (unsigned)k);
  const int64_t split_stride = (int64_t)k * g.nmop * g.nmop;
  if (st == Store::F64)
    hipLaunchKernelGGL(k_epilogue<double>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nvp, g.nmop,
                       g.mult, (const double*)Sp, nsplit, split_stride, d_ptab, d_epair, sigma);
  else
    hipLaunchKernelGGL(k_epilogue<float>, grid, dim3(256), 0, s, z, g.n, g.nvv, g.nvp, g.nmop,
                       g.mult, (const float*)Sp, nsplit, split_stride, d_ptab, d_epair, sigma);
  return hipGetLastError();
}

// Work items: (panel, first row tile) pairs; a panel spans up to 4 column tiles of one block.
void make_sigma_items(const Geometry& g, int RT, std::vector<int>& items, int& npan_v) {
  items.clear();
  const int not_ = g.nct - g.nvt;
  npan_v = (g.nvt + 3) / 4;
  const int npan_o = (not_ + 3) / 4;
  for (int pn = 0; pn < npan_v + npan_o; ++pn) {
    const bool v = pn < npan_v;
    const int t0 = v ? 4 * pn : 4 * (pn - npan_v);
    const int bnt = v ? g.nvt : not_;
    const int tend = std::min(t0 + 4, bnt);
    for (int R0 = 0; R0 < tend; R0 += RT) items.push_back((pn << 16) | R0);
  }
}

int sigma_variant(const Geometry& g, Store st, int* RT) {
  if (st == Store::F64) {
    if (g.nct <= 16) { *RT = 16; return 0; }
    *RT = 16;
    return 1;
  }
  if (st == Store::F32) { *RT = 32; return 2; }
  *RT = 32;
  return 3;
}

template <typename T, int CC, int RT>
static hipError_t run_sandwich(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                               hipStream_t s) {
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
  hipLaunchKernelGGL((k_sandwich<T, CC, RT>), dim3(nwg), dim3(256), 0, s, (const T*)la.L,
                     (const T*)la.ZT, (T*)la.Sp, p);
  return hipGetLastError();
}

hipError_t launch_sigma_bf16(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                             hipStream_t s);

hipError_t launch_sigma(const Geometry& g, Store st, const SigmaPlan& plan, const SigmaLaunch& la,
                        hipStream_t s) {
  switch (plan.variant) {
    case 0: return run_sandwich<double, 16, 16>(g, plan, la, s);
    case 1: return run_sandwich<double, 8, 16>(g, plan, la, s);
    case 2: return run_sandwich<float, 16, 32>(g, plan, la, s);
    default: return launch_sigma_bf16(g, plan, la, s);
  }
}

}  // namespace pprpa
