// The context behind the opaque pprpa_ctx handle.
#pragma once

#include "internal.h"

struct pprpa_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  pprpa::Geometry g;
  int prec = PPRPA_FP64;
  pprpa::Store st = pprpa::Store::F64;
  int nprod = 6;      // BF16 products (3 or 6)
  double mu2 = 0.0;   // 2 mu = e_HOMO + e_LUMO of the active window
  int kcap = 32;      // largest sigma block
  int nsplit_max = 1;

  void* L = nullptr;  // staged integrals [naux][nmop][nmop] (3 planes for BF16)
  size_t plane = 0;   // elements per plane
  double* L64 = nullptr;  // FP64 staged integrals for the dense build (may alias L)
  int* ptab = nullptr;    // packed pair -> (p << 16 | q)
  double* ev = nullptr;   // active virtual energies
  double* eo = nullptr;   // active occupied energies
  double* epair = nullptr;  // +(e_a+e_b) / -(e_i+e_j) per packed pair
  void* ZT = nullptr;       // unpacked vectors [kcap][nmop][nmop] (3 planes for BF16)
  size_t zplane = 0;
  void* Sp = nullptr;       // sigma partial sums
  double* zbuf = nullptr;   // [kcap][n] staging of host vectors
  double* sbuf = nullptr;
  double* M = nullptr;      // dense matrix [n][n] (dense builds)
  pprpa::SigmaPlan plan;

  std::vector<double> ev_h, eo_h;  // active virtual / occupied energies (alpha for the ab sector)
  std::vector<double> epair_h;     // host copy of epair
  bool ab = false;                 // alpha-beta sector of unrestricted ppRPA
  bool ab_df = false;              // ... with the density-fitted sigma (else dense: sigma = M z)
  int ab_nocc_b = 0;
  pprpa::AbGeometry abg;           // density-fitted alpha-beta layout
  void* Lb = nullptr;              // staged beta integrals [naux][nmopb][nmopb] (L holds alpha)
  std::vector<int> ptab_h;
  std::atomic<int> busy{0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double* pinned = nullptr;  // small pinned host buffer for per-iteration status
  size_t pinned_elems = 0;
  bool own_pinned = true;
  pprpa::Slab* slab = nullptr;  // served contexts: every device allocation comes from here
  std::vector<void*> allocs;

  // per-launch timing of the sandwich kernel (events harvested after stream synchronisation)
  struct Timed {
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Timed> pend;
  std::vector<hipEvent_t> pool;
  pprpa_kernel_stats stats{};

  // Davidson workspace (grown on demand, reused across calls)
  struct {
    size_t bytes = 0;
    void* base = nullptr;
  } dws;
};

namespace pprpa {
// sigma = M z for k vectors already on the device ([k][n] each), on the context's stream.
pprpa_status sigma_device(pprpa_ctx* c, int k, const double* dz, double* ds);
int nsplit_for(const pprpa_ctx* c, int k);
int nsplit_of(int variant, int nitems, int naux, int k);

pprpa_status dalloc(pprpa_ctx* c, size_t bytes, void** p);
// Fold completed launch timings into c->stats (call after synchronising the stream).
pprpa_status harvest_timing(pprpa_ctx* c);
// Served contexts (the serving loop): argument checks shared with pprpa_build; exact device
// footprint of a context plus one Davidson solve; build into a slab with a caller-owned pinned
// buffer (pinned_elems doubles) and stream; release.
pprpa_status check_build_args(const pprpa_build_args* a);
size_t context_footprint(const pprpa_build_args* a, const pprpa_davidson_args* d);
pprpa_status build_context(const pprpa_build_args* a, Slab* slab, double* pinned,
                           pprpa_ctx** out);
void free_context(pprpa_ctx* c);
constexpr size_t PINNED_ELEMS = 4096;
pprpa_status run_davidson(pprpa_ctx* c, const pprpa_davidson_args* a, double* omega,
                          double* vecs, double* resid, pprpa_report* rep);
class Solver;
pprpa_status iterate_solver(pprpa_ctx* c, Solver& sv, int n_iter, int* done_iters);
pprpa_status finish_solver(Solver& sv, double* omega, double* vecs, double* resid,
                           pprpa_report* rep);
}  // namespace pprpa
