// C ABI of libpprpa: argument checks, ownership, staging, sigma and dense entry points.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>

#include "solver.h"

namespace pprpa {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

static pprpa_status einval(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return PPRPA_EINVAL;
}

// Orbital energies as the ABI requires them: finite, ascending within the occupied block
// [0, nocc) and within the virtual block [nocc, nmo), and the highest occupied below the lowest
// virtual. The definite shift 2 mu = e_HOMO + e_LUMO and the active window (the highest occupied,
// the lowest virtual orbitals) both read the energies in this order.
static pprpa_status check_energies(const std::vector<double>& e, int nocc, const char* name) {
  const int nmo = (int)e.size();
  for (int i = 0; i < nmo; ++i)
    if (!std::isfinite(e[i])) return einval("%s[%d] is not finite", name, i);
  for (int i = 1; i < nmo; ++i)
    if (i != nocc && e[i] < e[i - 1])
      return einval("%s is not ascending within its %s block (%s[%d] = %.17g < %s[%d] = %.17g)",
                    name, i < nocc ? "occupied" : "virtual", name, i, e[i], name, i - 1, e[i - 1]);
  if (nocc > 0 && nocc < nmo && !(e[nocc - 1] < e[nocc]))
    return einval("highest occupied %s[%d] = %.17g is not below the lowest virtual %s[%d] = %.17g",
                  name, nocc - 1, e[nocc - 1], name, nocc, e[nocc]);
  return PPRPA_OK;
}

pprpa_status dalloc(pprpa_ctx* c, size_t bytes, void** p) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (c->slab) {
    const size_t b = (bytes + 255) / 256 * 256;
    if (c->slab->top + b > c->slab->size) {
      set_error("request footprint exceeded: %zu + %zu > %zu bytes reserved", c->slab->top, b,
                c->slab->size);
      return PPRPA_ENOMEM;
    }
    *p = c->slab->base + c->slab->top;
    c->slab->top += b;
    return PPRPA_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    *p = nullptr;
    return PPRPA_ENOMEM;
  }
  c->allocs.push_back(*p);
  return PPRPA_OK;
}

// Aux-index splits of a sigma launch: about 8192 workgroups (32 per CU), which measured best on
// MI355X (shorter tails and better balance than 1.5k-4k; partial sums stay small).
int nsplit_of(int variant, int nitems, int naux, int k) {
  // work units per launch: the FP64 kernel runs one 8-wave workgroup per CU, the others two
  // 4-wave workgroups
  const int target = variant == 5 ? UNITS_F64 : 8192;
  const int per = std::max(1, nitems * k);
  int ns = (target + per - 1) / per;
  ns = std::min(ns, std::min(naux, 256));
  return std::max(1, ns);
}

int nsplit_for(const pprpa_ctx* c, int k) {
  return nsplit_of(c->plan.variant, c->plan.nitems, c->g.naux, k);
}

static pprpa_status get_event(pprpa_ctx* c, hipEvent_t* e) {
  if (!c->pool.empty()) {
    *e = c->pool.back();
    c->pool.pop_back();
    return PPRPA_OK;
  }
  PPRPA_HIP(hipEventCreate(e));
  return PPRPA_OK;
}

pprpa_status harvest_timing(pprpa_ctx* c) {
  for (auto& t : c->pend) {
    float ms = 0.f;
    PPRPA_HIP(hipEventElapsedTime(&ms, t.a, t.b));
    c->stats.launches += 1;
    c->stats.seconds += ms * 1e-3;
    c->stats.flops += t.flops;
    c->stats.bytes += t.bytes;
    c->pool.push_back(t.a);
    c->pool.push_back(t.b);
  }
  c->pend.clear();
  return PPRPA_OK;
}

// Order of sandwich launches on one device across contexts: each launch waits, on the GPU, for
// the end of the previous launch issued on the same device by any context, so the sandwiches of
// solves running side by side on several streams do not split the compute units between them
// (each one fills the chip alone, and its per-launch time is its own) while their other kernels
// still overlap. The event lives until the process ends; the host is never blocked.
namespace {
struct SigmaGate {
  std::mutex mu;
  hipEvent_t last = nullptr;
};
constexpr int GATE_DEVICES = 64;
SigmaGate g_gate[GATE_DEVICES];
}  // namespace

// Run one sandwich launch behind the device's sigma gate, with its timing events.
template <typename F>
static pprpa_status gated_launch(pprpa_ctx* c, pprpa_ctx::Timed& tm, F&& launch) {
  if (c->device >= 0 && c->device < GATE_DEVICES) {
    SigmaGate& gt = g_gate[c->device];
    std::lock_guard<std::mutex> lk(gt.mu);
    if (!gt.last) PPRPA_HIP(hipEventCreateWithFlags(&gt.last, hipEventDisableTiming));
    PPRPA_HIP(hipStreamWaitEvent(c->stream, gt.last, 0));
    PPRPA_HIP(hipEventRecord(tm.a, c->stream));
    PPRPA_HIP(launch());
    PPRPA_HIP(hipEventRecord(tm.b, c->stream));
    PPRPA_HIP(hipEventRecord(gt.last, c->stream));
  } else {
    PPRPA_HIP(hipEventRecord(tm.a, c->stream));
    PPRPA_HIP(launch());
    PPRPA_HIP(hipEventRecord(tm.b, c->stream));
  }
  c->pend.push_back(tm);
  return PPRPA_OK;
}

pprpa_status sigma_device(pprpa_ctx* c, int k, const double* dz, double* ds) {
  const int64_t n = c->g.n;
  if (c->ab && c->ab_df) {  // density-fitted alpha-beta sector
    const AbGeometry& ag = c->abg;
    for (int k0 = 0; k0 < k; k0 += c->kcap) {
      const int kk = std::min(c->kcap, k - k0);
      const double* z = dz + (int64_t)k0 * n;
      double* s = ds + (int64_t)k0 * n;
      const int ns = nsplit_for(c, kk);
      PPRPA_HIP(launch_unpack_ab(ag, c->st, z, kk, c->ZT, c->zplane, c->stream));
      pprpa_ctx::Timed tm;
      PPRPA_TRY(get_event(c, &tm.a));
      PPRPA_TRY(get_event(c, &tm.b));
      const double esz = c->st == Store::F64 ? 8.0 : (c->st == Store::F32 ? 4.0 : 2.0 * (c->nprod == 3 ? 2 : 3));
      tm.flops = 2.0 * ag.naux * (double)n * ((ag.nva + ag.noa) + (ag.nvb + ag.nob)) * kk;
      tm.bytes = (double)ag.naux * ((double)ag.nmopa * ag.nmopa + (double)ag.nmopb * ag.nmopb) * esz +
                 2.0 * kk * (double)n * 8.0;
      PPRPA_TRY(gated_launch(c, tm, [&] {
        return launch_sigma_ab(ag, c->st, c->nprod, c->plan, c->L, c->Lb, c->ZT, c->zplane, c->Sp, kk,
                               ns, c->stream);
      }));
      PPRPA_HIP(launch_epilogue_ab(ag, c->st, z, kk, c->Sp, ns, c->epair, s, c->stream));
    }
    return PPRPA_OK;
  }
  if (c->ab) {  // dense context (alpha-beta sector): sigma = M z
    PPRPA_HIP(launch_dense_sigma(c->M, n, dz, k, ds, c->stream));
    return PPRPA_OK;
  }
  for (int k0 = 0; k0 < k; k0 += c->kcap) {
    const int kk = std::min(c->kcap, k - k0);
    const double* z = dz + (int64_t)k0 * n;
    double* s = ds + (int64_t)k0 * n;
    const int ns = nsplit_for(c, kk);
    PPRPA_HIP(launch_unpack(c->g, c->st, z, kk, c->ptab, c->ZT, c->zplane, c->stream));
    SigmaLaunch la;
    la.L = c->L;
    la.ZT = c->ZT;
    la.Sp = c->Sp;
    la.k = kk;
    la.nsplit = ns;
    la.npan_v = c->plan.npan_v;
    la.npan_o = 0;
    la.plane = c->plane;
    la.zplane = c->zplane;
    la.nprod = c->nprod;
    pprpa_ctx::Timed tm;
    PPRPA_TRY(get_event(c, &tm.a));
    PPRPA_TRY(get_event(c, &tm.b));
    const Geometry& g = c->g;
    const double nmo = g.nv + g.no;
    tm.flops = 4.0 * g.naux * nmo * ((double)g.nv * g.nv + (double)g.no * g.no) * kk;
    const double esz = c->st == Store::F64 ? 8.0 : (c->st == Store::F32 ? 4.0 : 2.0 * (c->nprod == 3 ? 2 : 3));
    tm.bytes = (double)g.naux * ((double)g.nv * g.nv + (double)g.nv * g.no + (double)g.no * g.no) * esz +
               2.0 * kk * (double)n * 8.0;
    PPRPA_TRY(gated_launch(c, tm, [&] { return launch_sigma(c->g, c->st, c->plan, la, c->stream); }));
    PPRPA_HIP(launch_epilogue(c->g, c->st, z, kk, c->Sp, ns, c->ptab, c->epair, s, c->stream));
  }
  return PPRPA_OK;
}

}  // namespace pprpa

using namespace pprpa;

namespace {

struct Busy {
  std::atomic<int>& b;
  bool ok;
  explicit Busy(std::atomic<int>& x) : b(x) {
    int e = 0;
    ok = b.compare_exchange_strong(e, 1);
  }
  ~Busy() {
    if (ok) b.store(0);
  }
};

void destroy(pprpa_ctx* c) {
  if (!c) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != c->device) (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->dws.base && !c->slab) (void)hipFree(c->dws.base);
  if (c->pinned && c->own_pinned) (void)hipHostFree(c->pinned);
  for (auto& t : c->pend) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->e0) (void)hipEventDestroy(c->e0);
  if (c->e1) (void)hipEventDestroy(c->e1);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  if (cur != c->device) (void)hipSetDevice(cur);
  delete c;
}

// Window, padded layout and pair counts of a problem (argument errors -> EINVAL).
pprpa_status geometry_of(const pprpa_build_args* a, Geometry* out) {
  const int nmo = a->nmo, nocc = a->nocc;
  const int nvir = nmo - nocc;
  if (a->nocc_act > nocc) return einval("nocc_act=%d exceeds nocc=%d", a->nocc_act, nocc);
  if (a->nvir_act > nvir) return einval("nvir_act=%d exceeds nvir=%d", a->nvir_act, nvir);
  const int no = a->nocc_act > 0 ? a->nocc_act : nocc;
  const int nv = a->nvir_act > 0 ? a->nvir_act : nvir;
  if (nv <= 0) return einval("no virtual orbitals in the window");
  if (nv > 16000 || no > 16000) return einval("window too large (nv=%d, no=%d)", nv, no);
  Geometry g;
  g.nv = nv;
  g.no = no;
  g.naux = a->naux;
  g.mult = a->mult;
  // BF16-split sigma reduces over 32 orbitals per MFMA: its blocks are padded to two tiles
  const int pad = (a->prec == PPRPA_BF16X6 || a->prec == PPRPA_BF16X3) ? 2 * TILE : TILE;
  g.nvp = round_up(nv, pad);
  g.nop = round_up(no, pad);
  g.nmop = g.nvp + g.nop;
  g.nvt = g.nvp / TILE;
  g.nct = g.nmop / TILE;
  const int k = a->mult == PPRPA_SINGLET ? 0 : 1;
  g.nvv = (int64_t)nv * (nv + 1) / 2 - (int64_t)k * nv;
  g.noo = (int64_t)no * (no + 1) / 2 - (int64_t)k * no;
  g.n = g.nvv + g.noo;
  if (g.nvv <= 0) return einval("no particle pairs (nv=%d, triplet)", nv);
  *out = g;
  return PPRPA_OK;
}

// Aux slices per host-to-device staging copy: all naux of them, or about 256 MB of FP64 input
// at a time when L is larger (the staging buffer holds one chunk).
int staging_chunk(size_t per, int naux) {
  const size_t cap = std::min<size_t>(65535, (size_t(256) << 20) / (per * 8));
  return (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(naux, 1), cap));
}

// Stream (the caller's or a new non-blocking one), timing events and the pinned status buffer of
// a context, on the current device.
pprpa_status setup_runtime(pprpa_ctx* c, void* stream) {
  PPRPA_HIP(hipGetDevice(&c->device));
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    PPRPA_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  PPRPA_HIP(hipEventCreate(&c->e0));
  PPRPA_HIP(hipEventCreate(&c->e1));
  c->pinned_elems = PINNED_ELEMS;
  if (!c->pinned)
    PPRPA_HIP(hipHostMalloc((void**)&c->pinned, c->pinned_elems * sizeof(double), hipHostMallocDefault));
  PPRPA_HIP(prepare_kernels());
  return PPRPA_OK;
}

pprpa_status build_impl(const pprpa_build_args* a, pprpa_ctx* c) {
  // ---- sizes and window ----------------------------------------------------------------
  const int nmo = a->nmo, nocc = a->nocc, naux = a->naux;
  PPRPA_TRY(geometry_of(a, &c->g));
  Geometry& g = c->g;
  const int no = g.no, nv = g.nv;
  const int k = a->mult == PPRPA_SINGLET ? 0 : 1;
  c->prec = a->prec;
  c->st = a->prec == PPRPA_FP64 ? Store::F64 : (a->prec == PPRPA_FP32 ? Store::F32 : Store::BF16);
  c->nprod = a->prec == PPRPA_BF16X3 ? 3 : 6;
  c->kcap = a->max_block > 0 ? std::min(a->max_block, 64) : 32;

  // ---- energies (host copy; validated) -------------------------------------------------
  std::vector<double> eps(nmo);
  if (a->on_device) {
    PPRPA_HIP(hipMemcpy(eps.data(), a->eps, nmo * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(eps.data(), a->eps, nmo * sizeof(double));
  }
  PPRPA_TRY(check_energies(eps, nocc, "eps"));
  c->eo_h.assign(eps.begin() + (nocc - no), eps.begin() + nocc);
  c->ev_h.assign(eps.begin() + nocc, eps.begin() + nocc + nv);
  c->mu2 = no > 0 ? c->eo_h.back() + c->ev_h.front() : 2.0 * (c->ev_h.front() - 1.0);

  PPRPA_TRY(setup_runtime(c, a->stream));

  // ---- pair table and pair energies ----------------------------------------------------
  c->ptab_h.resize(g.n);
  {
    int64_t e = 0;
    for (int p = 0; p < nv; ++p)
      for (int q = p + k; q < nv; ++q) c->ptab_h[e++] = (p << 16) | q;
    for (int p = 0; p < no; ++p)
      for (int q = p + k; q < no; ++q) c->ptab_h[e++] = (p << 16) | q;
  }
  c->epair_h.resize(g.n);
  for (int64_t e = 0; e < g.n; ++e) {
    const int p = c->ptab_h[e] >> 16, q = c->ptab_h[e] & 0xFFFF;
    c->epair_h[e] = e < g.nvv ? c->ev_h[p] + c->ev_h[q] : -(c->eo_h[p] + c->eo_h[q]);
  }
  PPRPA_TRY(dalloc(c, g.n * sizeof(int), (void**)&c->ptab));
  PPRPA_TRY(dalloc(c, nv * sizeof(double), (void**)&c->ev));
  PPRPA_TRY(dalloc(c, std::max(no, 1) * sizeof(double), (void**)&c->eo));
  PPRPA_TRY(dalloc(c, g.n * sizeof(double), (void**)&c->epair));
  PPRPA_HIP(hipMemcpyAsync(c->ptab, c->ptab_h.data(), g.n * sizeof(int), hipMemcpyHostToDevice, c->stream));
  PPRPA_HIP(hipMemcpyAsync(c->ev, c->ev_h.data(), nv * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (no > 0)
    PPRPA_HIP(hipMemcpyAsync(c->eo, c->eo_h.data(), no * sizeof(double), hipMemcpyHostToDevice, c->stream));
  PPRPA_HIP(launch_epair(g, c->ptab, c->ev, c->eo, c->epair, c->stream));

  // ---- stage L ---------------------------------------------------------------------------
  const int nin = a->lpq_is_active ? no + nv : nmo;
  std::vector<int> src(g.nmop, -1);
  for (int r = 0; r < nv; ++r) src[r] = a->lpq_is_active ? no + r : nocc + r;
  for (int r = 0; r < no; ++r) src[g.nvp + r] = a->lpq_is_active ? r : nocc - no + r;
  int* d_src = nullptr;
  int* d_bad = nullptr;
  PPRPA_TRY(dalloc(c, g.nmop * sizeof(int), (void**)&d_src));
  PPRPA_TRY(dalloc(c, sizeof(int), (void**)&d_bad));
  PPRPA_HIP(hipMemcpyAsync(d_src, src.data(), g.nmop * sizeof(int), hipMemcpyHostToDevice, c->stream));
  PPRPA_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), c->stream));
  c->plane = (size_t)naux * g.nmop * g.nmop;
  const size_t esz = c->st == Store::F64 ? 8 : (c->st == Store::F32 ? 4 : 2);
  const size_t nplanes = c->st == Store::BF16 ? 3 : 1;
  PPRPA_TRY(dalloc(c, c->plane * esz * nplanes, &c->L));
  double* tmp = nullptr;  // host-input staging buffer
  bool own_tmp = false;
  struct FreeTmp {
    double*& p;
    bool& own;
    ~FreeTmp() {
      if (own && p) (void)hipFree(p);
    }
  } free_tmp{tmp, own_tmp};
  auto stage = [&](Store st, void* dst, size_t plane) -> pprpa_status {
    if (a->on_device) {
      for (int p0 = 0; p0 < naux; p0 += 65535) {
        const int np = std::min(65535, naux - p0);
        PPRPA_HIP(launch_stage_L(g, st, a->Lpq + (size_t)p0 * nin * nin, nin, p0, np, d_src, dst,
                                 plane, d_bad, c->stream));
      }
      return PPRPA_OK;
    }
    const size_t per = (size_t)nin * nin;
    const int chunk = staging_chunk(per, naux);
    if (!tmp) {
      if (c->slab) {
        PPRPA_TRY(dalloc(c, (size_t)chunk * per * sizeof(double), (void**)&tmp));
      } else {
        PPRPA_HIP(hipMalloc((void**)&tmp, (size_t)chunk * per * sizeof(double)));
        own_tmp = true;
      }
    }
    pprpa_status rc = PPRPA_OK;
    for (int p0 = 0; p0 < naux && rc == PPRPA_OK; p0 += chunk) {
      const int np = std::min(chunk, naux - p0);
      hipError_t e = hipMemcpyAsync(tmp, a->Lpq + (size_t)p0 * per, (size_t)np * per * sizeof(double),
                                    hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = launch_stage_L(g, st, tmp, nin, p0, np, d_src, dst, plane, d_bad, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        set_error("staging L: %s", hipGetErrorString(e));
        rc = PPRPA_EDEVICE;
      }
    }
    return rc;
  };
  PPRPA_TRY(stage(c->st, c->L, c->plane));
  if (own_tmp) {
    (void)hipFree(tmp);
    tmp = nullptr;
    own_tmp = false;
  }
  if (a->dense) {
    if (c->st == Store::F64) {
      c->L64 = (double*)c->L;
    } else {
      PPRPA_TRY(dalloc(c, c->plane * sizeof(double), (void**)&c->L64));
      PPRPA_TRY(stage(Store::F64, c->L64, c->plane));
    }
  }
  int bad = 0;
  PPRPA_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  if (bad) return einval("Lpq contains non-finite values");

  // ---- sigma plan and workspaces ---------------------------------------------------------
  int RT = 16;
  c->plan.variant = sigma_variant(g, c->st, c->nprod, &RT);
  c->plan.RT = RT;
  std::vector<int> items;
  make_sigma_items(g, RT, items, c->plan.npan_v, panel_width(c->plan.variant));
  c->plan.nitems = (int)items.size();
  PPRPA_TRY(dalloc(c, items.size() * sizeof(int), (void**)&c->plan.d_items));
  PPRPA_HIP(hipMemcpyAsync(c->plan.d_items, items.data(), items.size() * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
  size_t sp_max = 0;
  for (int kk = 1; kk <= c->kcap; ++kk)
    sp_max = std::max(sp_max, (size_t)nsplit_for(c, kk) * kk);
  const size_t zz = (size_t)g.nmop * g.nmop;
  c->zplane = (size_t)c->kcap * zz;
  PPRPA_TRY(dalloc(c, c->zplane * esz * nplanes, &c->ZT));
  PPRPA_HIP(hipMemsetAsync(c->ZT, 0, c->zplane * esz * nplanes, c->stream));
  const size_t spsz = c->st == Store::F64 ? 8 : 4;
  PPRPA_TRY(dalloc(c, sp_max * zz * spsz, &c->Sp));
  PPRPA_TRY(dalloc(c, (size_t)c->kcap * g.n * sizeof(double), (void**)&c->zbuf));
  PPRPA_TRY(dalloc(c, (size_t)c->kcap * g.n * sizeof(double), (void**)&c->sbuf));

  // ---- dense matrix ------------------------------------------------------------------------
  if (a->dense) {
    if (g.n > 46000) return einval("dense build needs n <= 46000 (n=%lld)", (long long)g.n);
    PPRPA_TRY(dalloc(c, (size_t)g.n * g.n * sizeof(double), (void**)&c->M));
    PPRPA_HIP(launch_dense_build(g, c->L64, c->ptab, c->epair, c->M, c->stream));
  }
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  return PPRPA_OK;
}

// Alpha-beta sector of spin-unrestricted ppRPA: a dense context (the matrix built on the device,
// sigma = M z by the dense product) or a density-fitted one (both spins' integrals staged, sigma
// by the alpha-beta sandwich kernel).
pprpa_status build_ab_impl(const pprpa_build_ab_args* a, pprpa_ctx* c) {
  const int nmo = a->nmo, noa = a->nocc_a, nob = a->nocc_b, naux = a->naux;
  const int nva = nmo - noa, nvb = nmo - nob;
  Geometry& g = c->g;
  g.nv = nva;
  g.no = noa;
  g.naux = naux;
  g.mult = 0;
  g.nvv = (int64_t)nva * nvb;
  g.noo = (int64_t)noa * nob;
  g.n = g.nvv + g.noo;
  if (!a->density_fitted && g.n > 32768)
    return einval("dense alpha-beta sector of order %lld exceeds 32768", (long long)g.n);
  if (nva >= 65536 || nvb >= 65536 || noa >= 65536 || nob >= 65536)
    return einval("orbital counts must be below 65536");
  c->ab = true;
  c->ab_df = a->density_fitted != 0;
  c->ab_nocc_b = nob;
  c->prec = a->prec;
  c->st = a->prec == PPRPA_FP32 ? Store::F32
          : (a->prec == PPRPA_BF16X6 || a->prec == PPRPA_BF16X3) ? Store::BF16 : Store::F64;
  c->nprod = a->prec == PPRPA_BF16X3 ? 3 : 6;
  c->kcap = a->max_block > 0 ? std::min(a->max_block, 64) : 32;

  std::vector<double> ea(nmo), eb(nmo);
  const hipMemcpyKind kind = a->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  PPRPA_HIP(hipMemcpy(ea.data(), a->eps_a, nmo * sizeof(double), kind));
  PPRPA_HIP(hipMemcpy(eb.data(), a->eps_b, nmo * sizeof(double), kind));
  PPRPA_TRY(check_energies(ea, noa, "eps_a"));
  PPRPA_TRY(check_energies(eb, nob, "eps_b"));
  c->eo_h.assign(ea.begin(), ea.begin() + noa);
  c->ev_h.assign(ea.begin() + noa, ea.end());
  const double lumo = ea[noa] + eb[nob];
  c->mu2 = (noa > 0 && nob > 0) ? 0.5 * (lumo + ea[noa - 1] + eb[nob - 1]) : lumo - 2.0;

  PPRPA_TRY(setup_runtime(c, a->stream));

  c->ptab_h.resize(g.n);
  c->epair_h.resize(g.n);
  {
    int64_t e = 0;
    for (int p = 0; p < nva; ++p)
      for (int q = 0; q < nvb; ++q, ++e) {
        c->ptab_h[e] = (p << 16) | q;
        c->epair_h[e] = ea[noa + p] + eb[nob + q];
      }
    for (int p = 0; p < noa; ++p)
      for (int q = 0; q < nob; ++q, ++e) {
        c->ptab_h[e] = (p << 16) | q;
        c->epair_h[e] = -(ea[p] + eb[q]);
      }
  }
  PPRPA_TRY(dalloc(c, g.n * sizeof(int), (void**)&c->ptab));
  PPRPA_TRY(dalloc(c, g.n * sizeof(double), (void**)&c->epair));
  PPRPA_HIP(hipMemcpyAsync(c->ptab, c->ptab_h.data(), g.n * sizeof(int), hipMemcpyHostToDevice, c->stream));
  PPRPA_HIP(hipMemcpyAsync(c->epair, c->epair_h.data(), g.n * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));

  // integrals of both spins on the device (the caller's, or temporary copies of host inputs)
  const size_t per = (size_t)naux * nmo * nmo;
  const double* La = a->Lpq_a;
  const double* Lb = a->Lpq_b;
  double* tmp = nullptr;
  struct FreeTmp {
    double*& p;
    ~FreeTmp() {
      if (p) (void)hipFree(p);
    }
  } free_tmp{tmp};
  if (!a->on_device) {
    hipError_t e = hipMalloc((void**)&tmp, 2 * per * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      tmp = nullptr;
      set_error("staging %zu bytes of integrals: %s", 2 * per * sizeof(double), hipGetErrorString(e));
      return PPRPA_ENOMEM;
    }
    PPRPA_HIP(hipMemcpyAsync(tmp, a->Lpq_a, per * sizeof(double), hipMemcpyHostToDevice, c->stream));
    PPRPA_HIP(hipMemcpyAsync(tmp + per, a->Lpq_b, per * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    La = tmp;
    Lb = tmp + per;
  }
  int* d_bad = nullptr;
  PPRPA_TRY(dalloc(c, sizeof(int), (void**)&d_bad));
  PPRPA_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), c->stream));
  PPRPA_HIP(launch_check_finite(La, per, d_bad, c->stream));
  PPRPA_HIP(launch_check_finite(Lb, per, d_bad, c->stream));
  if (c->ab_df) {
    // both spins' integrals in the padded [virtual; occupied] layout of the sigma kernels
    AbGeometry& ag = c->abg;
    ag.nva = nva;
    ag.noa = noa;
    ag.nvb = nvb;
    ag.nob = nob;
    ag.naux = naux;
    // BF16-split sigma reduces over 32 orbitals per MFMA: its blocks are padded to two tiles
    const int pad = c->st == Store::BF16 ? 2 * TILE : TILE;
    ag.nvpa = round_up(nva, pad);
    ag.nopa = round_up(noa, pad);
    ag.nmopa = ag.nvpa + ag.nopa;
    ag.nvta = ag.nvpa / TILE;
    ag.ncta = ag.nmopa / TILE;
    ag.nvpb = round_up(nvb, pad);
    ag.nopb = round_up(nob, pad);
    ag.nmopb = ag.nvpb + ag.nopb;
    ag.nvtb = ag.nvpb / TILE;
    ag.nctb = ag.nmopb / TILE;
    ag.nvv = g.nvv;
    ag.noo = g.noo;
    ag.n = g.n;
    const size_t esz = c->st == Store::F64 ? 8 : (c->st == Store::F32 ? 4 : 2);
    const size_t nplanes = c->st == Store::BF16 ? 3 : 1;  // BF16: hi, mid, lo
    auto stage_spin = [&](const double* Lin, int nocc_s, int nv_s, int nvp_s, int nmop_s,
                          void** out) -> pprpa_status {
      std::vector<int> src(nmop_s, -1);
      for (int r = 0; r < nv_s; ++r) src[r] = nocc_s + r;
      for (int r = 0; r < nocc_s; ++r) src[nvp_s + r] = r;
      int* d_src = nullptr;
      PPRPA_TRY(dalloc(c, nmop_s * sizeof(int), (void**)&d_src));
      PPRPA_HIP(hipMemcpyAsync(d_src, src.data(), nmop_s * sizeof(int), hipMemcpyHostToDevice,
                               c->stream));
      const size_t plane_s = (size_t)naux * nmop_s * nmop_s;
      PPRPA_TRY(dalloc(c, plane_s * esz * nplanes, out));
      Geometry gs;
      gs.nmop = nmop_s;
      for (int p0 = 0; p0 < naux; p0 += 65535) {
        const int np = std::min(65535, naux - p0);
        PPRPA_HIP(launch_stage_L(gs, c->st, Lin + (size_t)p0 * nmo * nmo, nmo, p0, np, d_src,
                                 *out, plane_s, d_bad, c->stream));
      }
      return PPRPA_OK;
    };
    void* la_p = nullptr;
    void* lb_p = nullptr;
    PPRPA_TRY(stage_spin(La, noa, nva, ag.nvpa, ag.nmopa, &la_p));
    PPRPA_TRY(stage_spin(Lb, nob, nvb, ag.nvpb, ag.nmopb, &lb_p));
    c->L = la_p;
    c->Lb = lb_p;
    const size_t zt = (size_t)c->kcap * ag.nmopb * ag.nmopa;
    c->zplane = zt;
    PPRPA_TRY(dalloc(c, zt * esz * nplanes, &c->ZT));
    PPRPA_HIP(hipMemsetAsync(c->ZT, 0, zt * esz * nplanes, c->stream));
    std::vector<int> items;
    make_sigma_items_ab(ag, items, c->plan.npan_v);
    c->plan.nitems = (int)items.size();
    PPRPA_TRY(dalloc(c, items.size() * sizeof(int), (void**)&c->plan.d_items));
    PPRPA_HIP(hipMemcpyAsync(c->plan.d_items, items.data(), items.size() * sizeof(int),
                             hipMemcpyHostToDevice, c->stream));
    size_t sp_max = 0;
    for (int kk = 1; kk <= c->kcap; ++kk)
      sp_max = std::max(sp_max, (size_t)nsplit_for(c, kk) * kk);
    PPRPA_TRY(dalloc(c, sp_max * ag.nmopa * ag.nmopb * (c->st == Store::F64 ? 8 : 4), &c->Sp));
  } else {
    PPRPA_TRY(dalloc(c, (size_t)g.n * g.n * sizeof(double), (void**)&c->M));
    PPRPA_HIP(launch_dense_build_ab(La, Lb, naux, nmo, noa, nob, g.n, g.nvv, c->ptab, c->epair,
                                    c->M, c->stream));
  }
  PPRPA_TRY(dalloc(c, (size_t)c->kcap * g.n * sizeof(double), (void**)&c->zbuf));
  PPRPA_TRY(dalloc(c, (size_t)c->kcap * g.n * sizeof(double), (void**)&c->sbuf));
  int bad = 0;
  PPRPA_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  if (bad) return einval("Lpq_a or Lpq_b contains non-finite values");
  return PPRPA_OK;
}

}  // namespace

namespace pprpa {

pprpa_status check_build_args(const pprpa_build_args* a) {
  if (!a) return einval("args is NULL");
  if (a->nmo <= 0 || a->naux <= 0) return einval("nmo=%d and naux=%d must be positive", a->nmo, a->naux);
  if (a->nocc < 0 || a->nocc > a->nmo) return einval("nocc=%d outside [0, nmo=%d]", a->nocc, a->nmo);
  if (!a->eps || !a->Lpq) return einval("eps and Lpq must not be NULL");
  if (a->mult != PPRPA_SINGLET && a->mult != PPRPA_TRIPLET) return einval("mult=%d", a->mult);
  if (a->prec < PPRPA_FP64 || a->prec > PPRPA_BF16X3) return einval("prec=%d", a->prec);
  return PPRPA_OK;
}

// Every device allocation build_impl makes (plus the Davidson workspace), each rounded up to the
// 256-byte granule of the slab allocator. Kept in step with build_impl and get_ws: a served
// build whose allocations outrun this figure fails with ENOMEM instead of overrunning its slab.
size_t context_footprint(const pprpa_build_args* a, const pprpa_davidson_args* d) {
  Geometry g;
  if (check_build_args(a) != PPRPA_OK || geometry_of(a, &g) != PPRPA_OK) return 0;
  auto al = [](size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; };
  const Store st = a->prec == PPRPA_FP64 ? Store::F64 : (a->prec == PPRPA_FP32 ? Store::F32 : Store::BF16);
  const size_t esz = st == Store::F64 ? 8 : (st == Store::F32 ? 4 : 2);
  const size_t nplanes = st == Store::BF16 ? 3 : 1;
  const int kcap = a->max_block > 0 ? std::min(a->max_block, 64) : 32;
  const size_t plane = (size_t)g.naux * g.nmop * g.nmop;
  const size_t zz = (size_t)g.nmop * g.nmop;
  size_t b = 0;
  b += al(g.n * sizeof(int));                      // pair table
  b += al(g.nv * sizeof(double));                  // virtual energies
  b += al(std::max(g.no, 1) * sizeof(double));     // occupied energies
  b += al(g.n * sizeof(double));                   // pair energies
  b += al(g.nmop * sizeof(int));                   // source rows
  b += al(sizeof(int));                            // bad-value flag
  b += al(plane * esz * nplanes);                  // staged L
  if (!a->on_device) {
    const int nin = a->lpq_is_active ? g.no + g.nv : a->nmo;
    const size_t per = (size_t)nin * nin;
    b += al((size_t)staging_chunk(per, g.naux) * per * sizeof(double));
  }
  if (a->dense && st != Store::F64) b += al(plane * sizeof(double));
  int RT = 16, npan_v = 0;
  const int variant = sigma_variant(g, st, a->prec == PPRPA_BF16X3 ? 3 : 6, &RT);
  std::vector<int> items;
  make_sigma_items(g, RT, items, npan_v, panel_width(variant));
  b += al(items.size() * sizeof(int));
  b += al((size_t)kcap * zz * esz * nplanes);       // unpacked vectors
  size_t sp_max = 0;
  for (int kk = 1; kk <= kcap; ++kk)
    sp_max = std::max(sp_max, (size_t)nsplit_of(variant, (int)items.size(), g.naux, kk) * kk);
  b += al(sp_max * zz * (st == Store::F64 ? 8 : 4));  // partial sums
  b += 2 * al((size_t)kcap * g.n * sizeof(double));   // host-vector staging
  if (a->dense) b += al((size_t)g.n * g.n * sizeof(double));
  if (d) {
    const size_t ws = davidson_workspace_bytes(g, *d);
    if (ws == 0) return 0;
    b += al(ws);
  }
  return b;
}

pprpa_status build_context(const pprpa_build_args* a, Slab* slab, double* pinned,
                           pprpa_ctx** out) {
  *out = nullptr;
  PPRPA_TRY(check_build_args(a));
  pprpa_ctx* c = new (std::nothrow) pprpa_ctx();
  if (!c) return einval("host allocation failed");
  c->slab = slab;
  c->pinned = pinned;
  c->own_pinned = pinned == nullptr;
  pprpa_status s = build_impl(a, c);
  if (s != PPRPA_OK) {
    std::string keep = g_err;
    destroy(c);
    g_err = keep;
    return s;
  }
  *out = c;
  return PPRPA_OK;
}

void free_context(pprpa_ctx* c) { destroy(c); }

}  // namespace pprpa

namespace {

// Checks shared by both correlation-energy entry points (max_n: the largest order accepted).
pprpa_status corr_energy_checks(pprpa_ctx* c, pprpa_corr_energy* out, int64_t max_n) {
  if (!c) return einval("ctx is NULL");
  if (!out) return einval("out is NULL");
  if (!c->M) {
    set_error("the correlation energy needs a dense build (dense=1)");
    return PPRPA_EUNSUPPORTED;
  }
  if (c->g.n > max_n) {
    set_error("the whole-spectrum solve on the device is limited to n <= %lld (n=%lld)",
              (long long)max_n, (long long)c->g.n);
    return PPRPA_EUNSUPPORTED;
  }
  return PPRPA_OK;
}

// The whole-spectrum solve into the workspace `work` (3 n^2 doubles, then 4 doubles and 3 ints
// of outputs), results copied out through the context's pinned buffer. No allocation.
pprpa_status corr_energy_run(pprpa_ctx* c, double* work, pprpa_corr_energy* out) {
  TraceRange tr("pprpa_correlation_energy");
  const int64_t n = c->g.n, nvv = c->g.nvv;
  double* dout = work + 3 * (size_t)n * n;  // 4 doubles, then 3 ints
  int* dinfo = (int*)(dout + 4);
  double* hp = c->pinned;
  // one workgroup up to order 96, many above (the no-allocation entry point goes to 512)
  hipError_t le = n <= DENSE_ONE_WG_MAX ? launch_pencil_energy(c->M, (int)n, nvv, c->mu2, dout, work, dinfo, c->stream)
                           : launch_pencil_energy_mw(c->M, (int)n, nvv, c->mu2, dout, work, dinfo,
                                                     c->stream);
  if (le == hipSuccess) le = hipMemcpyAsync(hp, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (le == hipSuccess) le = hipMemcpyAsync(hp + 4, dinfo, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (le == hipSuccess) le = hipStreamSynchronize(c->stream);
  if (le != hipSuccess) {
    set_error("correlation energy: %s", hipGetErrorString(le));
    return PPRPA_EDEVICE;
  }
  const int* info = (const int*)(hp + 4);
  if (info[0] == 1) {
    set_error("M - 2 mu W is not positive definite");
    return PPRPA_ENONDEF;
  }
  pprpa_corr_energy r{};
  r.ec_pp = hp[0];
  r.ec_hh = hp[1];
  r.trace_a = hp[2];
  r.trace_c = hp[3];
  r.n_pp_roots = info[1];
  r.n_hh_roots = info[2];
  *out = r;
  if (info[1] != nvv || info[2] != n - nvv) {
    set_error("the spectrum splits into %d pp and %d hh roots, not %lld and %lld", info[1], info[2],
              (long long)nvv, (long long)(n - nvv));
    return PPRPA_ENONDEF;
  }
  return PPRPA_OK;
}

// Scratch of pprpa_correlation_energy_noalloc: the workspace of the whole-spectrum solve at the
// largest order it accepts, plus its outputs. Each device the library runs on holds its own copy
// for the life of the process; every call on a device shares it (calls that overlap on one
// device race). Nothing in it needs clearing between calls: the solve writes every element it
// reads.
constexpr int64_t NOALLOC_MAX_N = 512;
constexpr size_t NOALLOC_ELEMS = 3 * (size_t)NOALLOC_MAX_N * NOALLOC_MAX_N + 32;
static __device__ __align__(256) double scratch[NOALLOC_ELEMS];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device: the device address of `scratch`

// The device address of this device's copy of `scratch` (looked up once per device, with that
// device current; the host-side name is not a device address).
pprpa_status scratch_of(int device, double** ptr) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error("device address of the static scratch: %s", hipGetErrorString(e));
      return PPRPA_EDEVICE;
    }
    g_scratch_ptr[device] = (double*)p;
  }
  *ptr = g_scratch_ptr[device];
  return PPRPA_OK;
}

}  // namespace

extern "C" {

const char* pprpa_strerror(pprpa_status s) {
  // A C caller may pass any int; reading it as the enum type would be undefined outside the
  // enum's range of values, so the bytes are compared as an int.
  static_assert(sizeof(pprpa_status) == sizeof(int), "pprpa_status is an int on this ABI");
  int v;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case PPRPA_OK: return "ok";
    case PPRPA_EINVAL: return "invalid argument";
    case PPRPA_ENOMEM: return "out of device memory";
    case PPRPA_EDEVICE: return "device error";
    case PPRPA_ENOCONV: return "not converged";
    case PPRPA_ENONDEF: return "pencil not definite";
    case PPRPA_EUNSUPPORTED: return "unsupported";
    case PPRPA_EBUSY: return "context busy";
  }
  return "unknown status";
}

const char* pprpa_last_error(void) { return pprpa::g_err.c_str(); }

pprpa_status pprpa_build(const pprpa_build_args* a, pprpa_ctx** out) {
  TraceRange tr("pprpa_build");
  g_err.clear();
  if (!out) return einval("out is NULL");
  *out = nullptr;
  return build_context(a, nullptr, nullptr, out);
}

pprpa_status pprpa_build_ab(const pprpa_build_ab_args* a, pprpa_ctx** out) {
  TraceRange tr("pprpa_build_ab");
  g_err.clear();
  if (!out) return einval("out is NULL");
  *out = nullptr;
  if (!a) return einval("args is NULL");
  if (a->nmo <= 0 || a->naux <= 0) return einval("nmo=%d and naux=%d must be positive", a->nmo, a->naux);
  if (a->nocc_a < 0 || a->nocc_a >= a->nmo || a->nocc_b < 0 || a->nocc_b >= a->nmo)
    return einval("nocc_a=%d, nocc_b=%d outside [0, nmo=%d)", a->nocc_a, a->nocc_b, a->nmo);
  if (a->nmo > 65535) return einval("nmo=%d exceeds 65535", a->nmo);
  if (a->density_fitted != 0 && a->density_fitted != 1)
    return einval("density_fitted=%d must be 0 or 1", a->density_fitted);
  if (!a->eps_a || !a->eps_b || !a->Lpq_a || !a->Lpq_b)
    return einval("eps_a, eps_b, Lpq_a and Lpq_b must not be NULL");
  if (a->prec < PPRPA_FP64 || a->prec > PPRPA_BF16X3) return einval("prec=%d", a->prec);
  if (a->prec != PPRPA_FP64 && !(a->prec >= PPRPA_FP32 && a->prec <= PPRPA_BF16X3 && a->density_fitted)) {
    set_error("the alpha-beta sector takes FP64, or FP32 or BF16-split sigma when density fitted (prec=%d)",
              a->prec);
    return PPRPA_EUNSUPPORTED;
  }
  pprpa_ctx* c = new (std::nothrow) pprpa_ctx();
  if (!c) return einval("host allocation failed");
  pprpa_status s = build_ab_impl(a, c);
  if (s != PPRPA_OK) {
    std::string keep = g_err;
    destroy(c);
    g_err = keep;
    return s;
  }
  *out = c;
  return PPRPA_OK;
}

pprpa_status pprpa_dims(const pprpa_ctx* c, int64_t* n_pp, int64_t* n_hh) {
  if (!c) return einval("ctx is NULL");
  if (n_pp) *n_pp = c->g.nvv;
  if (n_hh) *n_hh = c->g.noo;
  return PPRPA_OK;
}

pprpa_status pprpa_matvec(pprpa_ctx* c, int32_t k, const double* z, double* sigma,
                          int32_t on_device) {
  TraceRange tr("pprpa_matvec");
  g_err.clear();
  if (!c) return einval("ctx is NULL");
  if (k <= 0) return einval("k=%d must be positive", k);
  if (!z || !sigma) return einval("z and sigma must not be NULL");
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  const int64_t n = c->g.n;
  if (on_device) {
    PPRPA_TRY(sigma_device(c, k, z, sigma));
  } else {
    for (int k0 = 0; k0 < k; k0 += c->kcap) {
      const int kk = std::min(c->kcap, k - k0);
      PPRPA_HIP(hipMemcpyAsync(c->zbuf, z + (size_t)k0 * n, (size_t)kk * n * sizeof(double),
                               hipMemcpyHostToDevice, c->stream));
      PPRPA_TRY(sigma_device(c, kk, c->zbuf, c->sbuf));
      PPRPA_HIP(hipMemcpyAsync(sigma + (size_t)k0 * n, c->sbuf, (size_t)kk * n * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
      PPRPA_HIP(hipStreamSynchronize(c->stream));
    }
  }
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  return harvest_timing(c);
}

pprpa_status pprpa_sigma_stats(pprpa_ctx* c, pprpa_kernel_stats* out, int32_t reset) {
  g_err.clear();
  if (!c) return einval("ctx is NULL");
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  PPRPA_TRY(harvest_timing(c));
  if (out) *out = c->stats;
  if (reset) c->stats = pprpa_kernel_stats{};
  return PPRPA_OK;
}

pprpa_status pprpa_dense_matrix(pprpa_ctx* c, double* M, int32_t on_device) {
  g_err.clear();
  if (!c) return einval("ctx is NULL");
  if (!M) return einval("M is NULL");
  if (!c->M) {
    set_error("context was built without dense=1");
    return PPRPA_EUNSUPPORTED;
  }
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  const size_t bytes = (size_t)c->g.n * c->g.n * sizeof(double);
  PPRPA_HIP(hipMemcpyAsync(M, c->M, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream));
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  return PPRPA_OK;
}

pprpa_status pprpa_correlation_energy(pprpa_ctx* c, pprpa_corr_energy* out) {
  g_err.clear();
  PPRPA_TRY(corr_energy_checks(c, out, DENSE_ENERGY_MAX));
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  const int64_t n = c->g.n;
  const size_t work_bytes = 3 * (size_t)n * n * sizeof(double) + 256;
  void* work = nullptr;
  hipError_t e = hipMalloc(&work, work_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("correlation-energy workspace of %zu bytes: %s", work_bytes, hipGetErrorString(e));
    return PPRPA_ENOMEM;
  }
  const pprpa_status st = corr_energy_run(c, (double*)work, out);
  (void)hipFree(work);
  return st;
}

pprpa_status pprpa_correlation_energy_noalloc(pprpa_ctx* c, pprpa_corr_energy* out) {
  g_err.clear();
  PPRPA_TRY(corr_energy_checks(c, out, NOALLOC_MAX_N));
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  double* work = nullptr;
  PPRPA_TRY(scratch_of(c->device, &work));
  return corr_energy_run(c, work, out);
}

// NTOs of alpha-beta roots (pprpa_nto on an alpha-beta context): the rectangular blocks are the
// packed vectors themselves, so only the Gram products and their eigenvalues run.
static pprpa_status nto_ab(pprpa_ctx* c, int k, const double* z, int on_device, double* lam_p,
                           double* lam_h, double* d_vv, double* d_oo) {
  const Geometry& g = c->g;
  const int nmo = g.nv + g.no, nva = g.nv, noa = g.no, nob = c->ab_nocc_b, nvb = nmo - nob;
  if (nva > 512 || nvb > 512 || noa > 512 || nob > 512) {
    set_error("NTOs on the device are limited to orbital blocks <= 512 (nvir %d/%d, nocc %d/%d)",
              nva, nvb, noa, nob);
    return PPRPA_EUNSUPPORTED;
  }
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  const size_t zv = (size_t)k * g.n;
  const size_t gv = (size_t)k * nva * nva, go = (size_t)k * noa * noa;
  const size_t dv = (size_t)k * ((size_t)nva * nva + (size_t)nvb * nvb);
  const size_t dov = (size_t)k * ((size_t)noa * noa + (size_t)nob * nob);
  const size_t lv = (size_t)k * nva, lo = (size_t)k * noa;
  // z (when on the host), Gx, Gy, Dv, Do, lam_p, lam_h
  const size_t total = (on_device ? 0 : zv) + gv + go + dv + dov + lv + lo;
  double* buf = nullptr;
  hipError_t e = hipMalloc((void**)&buf, std::max<size_t>(total, 1) * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("NTO workspace of %zu bytes: %s", total * sizeof(double), hipGetErrorString(e));
    return PPRPA_ENOMEM;
  }
  double* p = buf;
  const double* dz = z;
  if (!on_device) {
    dz = p;
    p += zv;
  }
  double* Gx = p; p += gv;
  double* Gy = p; p += go;
  double* Dv = p; p += dv;
  double* Do = p; p += dov;
  double* lp = p; p += lv;
  double* lh = p;
  hipStream_t s = c->stream;
  hipError_t le = hipSuccess;
  if (!on_device) le = hipMemcpyAsync((void*)dz, z, zv * sizeof(double), hipMemcpyHostToDevice, s);
  if (le == hipSuccess)
    le = launch_nto_ab(dz, g.n, k, nva, nvb, noa, nob, Gx, Gy, Dv, Do, lp, lh, s);
  if (le == hipSuccess) le = hipMemcpyAsync(lam_p, lp, lv * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && lo) le = hipMemcpyAsync(lam_h, lh, lo * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && d_vv) le = hipMemcpyAsync(d_vv, Dv, dv * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && d_oo && dov)
    le = hipMemcpyAsync(d_oo, Do, dov * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess) le = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (le != hipSuccess) {
    set_error("NTO analysis: %s", hipGetErrorString(le));
    return PPRPA_EDEVICE;
  }
  return PPRPA_OK;
}

pprpa_status pprpa_nto(pprpa_ctx* c, int32_t k, const double* z, int32_t on_device, double* lam_p,
                       double* lam_h, double* d_vv, double* d_oo) {
  TraceRange tr("pprpa_nto");
  g_err.clear();
  if (!c) return einval("ctx is NULL");
  if (!z || !lam_p || (!lam_h && c->g.no > 0)) return einval("z, lam_p and lam_h must not be NULL");
  if (k < 1 || k > 64) return einval("k=%d outside [1, 64]", k);
  if (c->ab) return nto_ab(c, k, z, on_device, lam_p, lam_h, d_vv, d_oo);
  const Geometry& g = c->g;
  if (g.nv > 512 || g.no > 512) {
    set_error("NTOs on the device are limited to nv, no <= 512 (nv=%d, no=%d)", g.nv, g.no);
    return PPRPA_EUNSUPPORTED;
  }
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  const size_t zv = (size_t)k * g.n, mv = (size_t)k * g.nv * g.nv, mo = (size_t)k * g.no * g.no;
  const size_t lv = (size_t)k * g.nv, lo = (size_t)k * g.no;
  // z (when on the host), X, Y, Gx, Gy, Dv, Do, lam_p, lam_h
  const size_t total = (on_device ? 0 : zv) + 3 * mv + 3 * mo + lv + lo;
  double* buf = nullptr;
  hipError_t e = hipMalloc((void**)&buf, std::max<size_t>(total, 1) * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("NTO workspace of %zu bytes: %s", total * sizeof(double), hipGetErrorString(e));
    return PPRPA_ENOMEM;
  }
  double* p = buf;
  const double* dz = z;
  if (!on_device) {
    dz = p;
    p += zv;
  }
  double* X = p; p += mv;
  double* Gx = p; p += mv;
  double* Dv = p; p += mv;
  double* Y = p; p += mo;
  double* Gy = p; p += mo;
  double* Do = p; p += mo;
  double* lp = p; p += lv;
  double* lh = p;
  hipStream_t s = c->stream;
  hipError_t le = hipSuccess;
  if (!on_device) le = hipMemcpyAsync((void*)dz, z, zv * sizeof(double), hipMemcpyHostToDevice, s);
  if (le == hipSuccess)
    le = launch_nto(dz, g.n, k, g, c->ptab, X, Y, Gx, Gy, Dv, Do, lp, lh, s);
  if (le == hipSuccess) le = hipMemcpyAsync(lam_p, lp, lv * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && lo) le = hipMemcpyAsync(lam_h, lh, lo * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && d_vv) le = hipMemcpyAsync(d_vv, Dv, mv * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && d_oo && mo) le = hipMemcpyAsync(d_oo, Do, mo * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess) le = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (le != hipSuccess) {
    set_error("NTO analysis: %s", hipGetErrorString(le));
    return PPRPA_EDEVICE;
  }
  return PPRPA_OK;
}

pprpa_status pprpa_nto_vectors(pprpa_ctx* c, int32_t k, const double* z, int32_t on_device,
                               int32_t nvec, double* c_p1, double* c_p2, double* c_h1,
                               double* c_h2) {
  TraceRange tr("pprpa_nto_vectors");
  g_err.clear();
  if (!c) return einval("ctx is NULL");
  if (!z) return einval("z must not be NULL");
  if (k < 1 || k > 64) return einval("k=%d outside [1, 64]", k);
  if (nvec < 1 || nvec > 64) return einval("nvec=%d outside [1, 64]", nvec);
  const Geometry& g = c->g;
  // the amplitude blocks: rows x cols of the pp and hh parts
  const int rp = g.nv, cp = c->ab ? (g.nv + g.no) - c->ab_nocc_b : g.nv;
  const int rh = g.no, ch = c->ab ? c->ab_nocc_b : g.no;
  if (rp > 512 || cp > 512 || rh > 512 || ch > 512) {
    set_error("NTO vectors on the device are limited to orbital blocks <= 512");
    return PPRPA_EUNSUPPORTED;
  }
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  const bool hh = rh > 0 && ch > 0;
  const size_t zv = (size_t)k * g.n;
  const size_t xs = c->ab ? 0 : (size_t)k * ((size_t)rp * rp + (size_t)rh * rh);  // unpacked X, Y
  const size_t wp = svd_vectors_work(k, rp, cp, nvec), wh = hh ? svd_vectors_work(k, rh, ch, nvec) : 0;
  const size_t op = (size_t)k * nvec * ((size_t)rp + cp), oh = hh ? (size_t)k * nvec * ((size_t)rh + ch) : 0;
  const size_t total = (on_device ? 0 : zv) + xs + std::max(wp, wh) + op + oh;
  double* buf = nullptr;
  hipError_t e = hipMalloc((void**)&buf, std::max<size_t>(total, 1) * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("NTO workspace of %zu bytes: %s", total * sizeof(double), hipGetErrorString(e));
    return PPRPA_ENOMEM;
  }
  double* p = buf;
  const double* dz = z;
  if (!on_device) {
    dz = p;
    p += zv;
  }
  const double *Ap, *Ah;
  int64_t sp_, sh_;
  hipStream_t s = c->stream;
  hipError_t le = hipSuccess;
  if (!on_device) le = hipMemcpyAsync((void*)dz, z, zv * sizeof(double), hipMemcpyHostToDevice, s);
  if (c->ab) {  // the packed alpha-beta vector is X then Y, row-major (alpha index outer)
    Ap = dz;
    Ah = dz + g.nvv;
    sp_ = sh_ = g.n;
  } else {
    double* X = p;
    double* Y = p + (size_t)k * rp * rp;
    p += xs;
    if (le == hipSuccess) le = launch_unpack_triangular(dz, g.n, k, g, c->ptab, X, Y, s);
    Ap = X;
    Ah = Y;
    sp_ = (int64_t)rp * rp;
    sh_ = (int64_t)rh * rh;
  }
  double* work = p;
  p += std::max(wp, wh);
  double* U1 = p;
  double* V1 = U1 + (size_t)k * nvec * rp;
  double* U2 = V1 + (size_t)k * nvec * cp;
  double* V2 = U2 + (size_t)k * nvec * rh;
  if (le == hipSuccess) le = launch_svd_vectors(Ap, sp_, rp, cp, k, nvec, work, U1, V1, s);
  if (le == hipSuccess && hh) le = launch_svd_vectors(Ah, sh_, rh, ch, k, nvec, work, U2, V2, s);
  const size_t np1 = (size_t)k * nvec * rp, np2 = (size_t)k * nvec * cp;
  const size_t nh1 = (size_t)k * nvec * rh, nh2 = (size_t)k * nvec * ch;
  if (le == hipSuccess && c_p1) le = hipMemcpyAsync(c_p1, U1, np1 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && c_p2) le = hipMemcpyAsync(c_p2, V1, np2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (le == hipSuccess && c_h1 && nh1) {
    if (hh) le = hipMemcpyAsync(c_h1, U2, nh1 * sizeof(double), hipMemcpyDeviceToHost, s);
    else std::fill(c_h1, c_h1 + nh1, 0.0);
  }
  if (le == hipSuccess && c_h2 && nh2) {
    if (hh) le = hipMemcpyAsync(c_h2, V2, nh2 * sizeof(double), hipMemcpyDeviceToHost, s);
    else std::fill(c_h2, c_h2 + nh2, 0.0);
  }
  if (le == hipSuccess) le = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (le != hipSuccess) {
    set_error("NTO vectors: %s", hipGetErrorString(le));
    return PPRPA_EDEVICE;
  }
  return PPRPA_OK;
}

pprpa_status pprpa_davidson(pprpa_ctx* c, const pprpa_davidson_args* a, double* omega,
                            double* vecs, double* resid, pprpa_report* rep) {
  g_err.clear();
  if (!c) return einval("ctx is NULL");
  if (!a || !omega) return einval("args and omega must not be NULL");
  Busy busy(c->busy);
  if (!busy.ok) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  PPRPA_HIP(hipSetDevice(c->device));
  pprpa_status st = run_davidson(c, a, omega, vecs, resid, rep);
  if (hipStreamSynchronize(c->stream) == hipSuccess) (void)harvest_timing(c);
  return st;
}

// A Davidson solve advanced by the caller. It holds its context (other calls on the context
// return EBUSY) from pprpa_solve_begin until pprpa_solve_end.
struct pprpa_solve {
  pprpa_ctx* c = nullptr;
  std::unique_ptr<Solver> sv;
};

pprpa_status pprpa_solve_begin(pprpa_ctx* c, const pprpa_davidson_args* a, pprpa_solve** out) {
  g_err.clear();
  if (!out) return einval("out is NULL");
  *out = nullptr;
  if (!c) return einval("ctx is NULL");
  if (!a) return einval("args is NULL");
  if (a->direct) {
    set_error("pprpa_solve_begin runs the Davidson solver only (direct=0); use pprpa_davidson");
    return PPRPA_EUNSUPPORTED;
  }
  int expect = 0;
  if (!c->busy.compare_exchange_strong(expect, 1)) {
    set_error("context in use by another thread");
    return PPRPA_EBUSY;
  }
  std::unique_ptr<pprpa_solve> s(new (std::nothrow) pprpa_solve());
  if (!s) {
    c->busy.store(0);
    return einval("host allocation failed");
  }
  s->c = c;
  pprpa_status rc = PPRPA_OK;
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipSetDevice(%d) failed", c->device);
    rc = PPRPA_EDEVICE;
  } else {
    s->sv.reset(new Solver(c, *a));
    s->sv->start();
    if (s->sv->phase == Solver::DONE && s->sv->status != PPRPA_OK) {
      set_error("%s", s->sv->message.c_str());
      rc = s->sv->status;
    }
  }
  if (rc != PPRPA_OK) {
    c->busy.store(0);
    return rc;
  }
  *out = s.release();
  return PPRPA_OK;
}

pprpa_status pprpa_solve_iterate(pprpa_solve* s, int32_t n_iter, int32_t* iters_done,
                                 int32_t* done) {
  g_err.clear();
  if (!s) return einval("solve is NULL");
  if (n_iter < 0) return einval("n_iter=%d must not be negative", n_iter);
  PPRPA_HIP(hipSetDevice(s->c->device));
  int it = 0;
  pprpa_status rc = iterate_solver(s->c, *s->sv, n_iter, &it);
  if (iters_done) *iters_done = it;
  if (done) *done = s->sv->phase == Solver::DONE ? 1 : 0;
  if (rc != PPRPA_OK) {
    s->sv->phase = Solver::DONE;
    s->sv->status = rc;
    s->sv->message = pprpa_last_error();
  }
  return rc;
}

pprpa_status pprpa_solve_stats(pprpa_solve* s, pprpa_kernel_stats* out, int32_t reset) {
  g_err.clear();
  if (!s) return einval("solve is NULL");
  pprpa_ctx* c = s->c;
  PPRPA_HIP(hipSetDevice(c->device));
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  PPRPA_TRY(harvest_timing(c));
  if (out) *out = c->stats;
  if (reset) c->stats = pprpa_kernel_stats{};
  return PPRPA_OK;
}

pprpa_status pprpa_solve_end(pprpa_solve* s, double* omega, double* vecs, double* resid,
                             pprpa_report* rep) {
  g_err.clear();
  if (!s) return einval("solve is NULL");
  pprpa_ctx* c = s->c;
  pprpa_status st = PPRPA_OK;
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipSetDevice(%d) failed", c->device);
    st = PPRPA_EDEVICE;
  } else {
    st = finish_solver(*s->sv, omega, vecs, resid, rep);
    const std::string msg = pprpa_last_error();
    if (hipStreamSynchronize(c->stream) == hipSuccess) (void)harvest_timing(c);
    if (!msg.empty()) set_error("%s", msg.c_str());
  }
  s->sv.reset();
  delete s;
  c->busy.store(0);
  return st;
}

void pprpa_free(pprpa_ctx* c) { destroy(c); }

}  // extern "C"
