// Resumable block Davidson solver (one context, one solve). The solve is a sequence of phases;
// each phase queues device work on the context's stream, ending with a small device-to-host copy
// into the context's pinned buffer that the next phase reads. The caller waits for the stream
// (synchronise, or poll it) before advancing a phase other than RR_LAUNCH, and may run other work
// in between (another solve's phases, a grouped sigma launch), which is how the serving loop
// overlaps solves. The sigma product of a new block is the caller's: in phase NEED_SIGMA,
// sigma of rows [sig_m0, sig_m0 + sig_k) of V goes into the same rows of SV, queued on the
// context's stream (or ordered before it), then sigma_done() is called.
#pragma once

#include <chrono>
#include <string>
#include <vector>

#include "ctx.h"

namespace pprpa {

struct DavWork {
  double *V, *SV, *Vt, *SVt, *Ms, *Ws_, *Mt, *Wt, *Cc, *Q, *Z, *SZ, *R, *Tn, *Tn2, *Cp, *Gb, *Tm;
  double *omega, *rnorm, *part, *pwork;
  int* info;
};

// Sizes of one Davidson solve.
struct Shape {
  int nroot, blk, max_iter, mmax, nguess, nb0, tblk, nret, nch;
};

// Device workspace of a Davidson solve of this geometry (0 if the arguments are invalid).
size_t davidson_workspace_bytes(const Geometry& g, const pprpa_davidson_args& a);

class Solver {
 public:
  enum Phase { NEED_SIGMA, RR_LAUNCH, RR_READ, RESTART_READ, ORTH1_READ, ORTH2_READ, DONE };

  Solver(pprpa_ctx* c, const pprpa_davidson_args& a) : c_(c), a_(a) {}

  // Validate, take the workspace, queue the initial subspace. Ends in NEED_SIGMA, or DONE (the
  // direct path, or an error in status/message).
  pprpa_status start();
  // Run the current phase (RR_LAUNCH and the *_READ phases).
  pprpa_status advance();
  // sigma of the requested block is queued: continue with the Rayleigh-Ritz step. timed: the
  // context's events e0/e1 bracket the sigma work.
  void sigma_done(bool timed = false) {
    sig_timed_ = timed;
    phase = RR_LAUNCH;
  }
  // Outputs of a finished solve (each may be NULL): the last iterate's roots, vectors (host) and
  // residual norms, and the report.
  pprpa_status results(double* omega, double* vecs, double* resid, pprpa_report* rep);

  Phase phase = DONE;
  pprpa_status status = PPRPA_OK;  // final status once DONE
  std::string message;             // error text once DONE with an error
  int sig_m0 = 0, sig_k = 0;       // block awaiting sigma
  DavWork w{};
  double t_sigma = 0.0;  // seconds of timed sigma work
  int nroot() const { return nroot_; }
  int iters() const { return iter_; }
  const double* omega() const { return om_; }

 private:
  pprpa_status fail(pprpa_status s);  // error: record the message, finish
  pprpa_status done(pprpa_status s);  // finish with OK or ENOCONV
  pprpa_status run_direct();
  pprpa_status initial_subspace(const Shape& sh);
  pprpa_status orth_pass1(int nsel);
  pprpa_status orth_pass2(int kept);
  pprpa_status orth_commit(int kept, int kept2);
  pprpa_status rr_launch();
  pprpa_status rr_read();
  pprpa_status restart_read();
  pprpa_status launch_corrections();
  pprpa_status orth1_read();
  pprpa_status orth2_read();
  pprpa_status stagnated();
  void log_iteration(int nconv, double maxr, int sweeps);

  pprpa_ctx* c_;
  pprpa_davidson_args a_;
  std::chrono::steady_clock::time_point t0_;
  int nroot_ = 0, blk_ = 0, max_iter_ = 0, mmax_ = 0, nret_ = 0, tblk_ = 0, nch_ = 0, nres_ = 64;
  int m_ = 0, mnew0_ = 0, iter_ = 0, nsig_ = 0;
  int npos_ = 0, nsel_ = 0, kept_ = 0;
  bool sig_timed_ = false, have_iterate_ = false;
  std::vector<int> sel_;
  double om_[64] = {0}, rn_[64] = {0};
  int nconv_ = 0;
  double maxr_ = 0.0;
};

}  // namespace pprpa
