// Block Davidson solver for the lowest pp roots (or the hh roots nearest the gap) of
// M z = Omega W z, and the direct dense path.
//
// arXiv 2512.12515 (sections "ppRPA Equation" and "Implementation Details") names the Davidson
// algorithm and direct diagonalisation as the two solvers but gives no algorithmic detail; the
// design here:
//  * subspace V (orthonormal rows, Euclidean) grown by blocks; projected pencil
//    (V M V^T, V W V^T) solved on the device through the definite shift M - 2 mu W
//    (mu = mid-gap of the active window), whose positive-theta roots are the pp roots, so the
//    wanted roots are the nroot largest theta (lowest Omega > 2 mu); in the hh channel the
//    negative-theta roots are the hh roots and the wanted ones the nroot smallest theta (the
//    largest Omega < 2 mu, nearest the gap);
//  * Ritz vectors z = V^T c with z^T W z = +1 (pp) or -1 (hh) (Eq. xy_norm); residual
//    r = M z - Omega W z,
//    converged when ||r||_2 <= tol for every wanted root;
//  * corrections t = r / (Omega w - D) from the diagonal pair energies D, normalised, projected
//    out of V twice (classical Gram-Schmidt, two passes) and orthonormalised within the block
//    from their Gram matrix (eigenvalue cut drops dependent directions), twice;
//  * restart when the subspace would exceed max_subspace: keep the 2*nroot best Ritz vectors,
//    orthonormalised in the small space, and rotate V, sigma(V) and the projected matrices with
//    them (no new sigma products).
// All arithmetic is FP64 on the device; the host runs the control loop and reads back nroot
// eigenvalues, nroot residual norms and a few counters per iteration.
//
// The loop is a phase machine (Solver): every phase queues device work on the context's stream
// and ends with a small device-to-host copy that the next phase reads, so a caller can interleave
// the phases of many solves and batch their sigma products (the serving loop does).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <numeric>

#include "solver.h"

namespace pprpa {
namespace {

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// Sizes of one Davidson solve (shared by the workspace allocation and the footprint estimate).
pprpa_status shape_of(const Geometry& g, const pprpa_davidson_args* a, Shape* sh) {
  const int64_t n = g.n;
  if (a->channel != 0 && a->channel != 1) {
    set_error("channel=%d is neither 0 (pp) nor 1 (hh)", a->channel);
    return PPRPA_EINVAL;
  }
  // pair space of the wanted channel: virtual pairs (pp) or occupied pairs (hh)
  const int64_t nwant = a->channel == 0 ? g.nvv : g.n - g.nvv;
  Shape s{};
  s.nroot = a->nroot;
  if (s.nroot < 1 || s.nroot > nwant) {
    set_error("nroot=%d outside [1, n_%s=%lld]", s.nroot, a->channel == 0 ? "pp" : "hh",
              (long long)nwant);
    return PPRPA_EINVAL;
  }
  if (s.nroot > 64) {
    set_error("nroot=%d exceeds 64", s.nroot);
    return PPRPA_EUNSUPPORTED;
  }
  if (!(a->tol > 0.0) && !a->direct) {
    set_error("tol must be positive");
    return PPRPA_EINVAL;
  }
  int blk = a->block > 0 ? a->block : s.nroot;
  blk = std::max(blk, 1);
  s.blk = (int)std::min<int64_t>(std::min(blk, 64), nwant);
  s.max_iter = a->max_iter > 0 ? a->max_iter : 100;
  int mmax = a->max_subspace > 0 ? a->max_subspace : std::max(8 * s.nroot, s.nroot + 4 * s.blk);
  s.mmax = (int)std::min<int64_t>(std::min(mmax, 256), n);
  s.nguess = (a->guess && a->nguess > 0) ? std::min(a->nguess, s.mmax) : 0;
  int nb0 = s.nguess > 0 ? s.nguess : (int)std::min<int64_t>(std::max(s.blk, s.nroot), nwant);
  s.nb0 = std::min(nb0, s.mmax);
  s.tblk = std::max(s.blk, s.nb0);  // rows of the correction buffers
  if (s.mmax < s.nroot + 1 && s.mmax < n) {
    set_error("max_subspace=%d too small for nroot=%d", s.mmax, s.nroot);
    return PPRPA_EINVAL;
  }
  s.nret = std::max(s.nroot, std::min(2 * s.nroot, s.mmax / 2));
  s.nch = (int)std::min<int64_t>(256, std::max<int64_t>(1, n / 128));  // t-chunks of the dots
  *sh = s;
  return PPRPA_OK;
}

// Workspace element counts, in the order of the DavWork members.
int ws_sizes(int64_t n, int mmax, int nret, int blk, size_t pwork_elems, size_t part_elems,
             size_t* sizes) {
  const size_t vecs = (size_t)mmax * n;
  const size_t list[] = {vecs, vecs, vecs, vecs,                                         // V SV Vt SVt
                         (size_t)mmax * mmax, (size_t)mmax * mmax, (size_t)mmax * mmax,  // Ms Ws Mt
                         (size_t)mmax * mmax,                                            // Wt
                         (size_t)mmax * nret, (size_t)mmax * nret,                       // Cc Q
                         (size_t)nret * n, (size_t)nret * n, (size_t)nret * n,           // Z SZ R
                         (size_t)blk * n, (size_t)blk * n,                               // Tn Tn2
                         (size_t)mmax * blk, (size_t)blk * blk, (size_t)blk * blk,       // Cp Gb Tm
                         (size_t)nret, (size_t)nret, part_elems, pwork_elems, 16};
  const int nb = sizeof(list) / sizeof(list[0]);
  std::copy(list, list + nb, sizes);
  return nb;
}

size_t ws_total(int64_t n, int mmax, int nret, int blk, size_t pwork, size_t part) {
  size_t sizes[32];
  const int nb = ws_sizes(n, mmax, nret, blk, pwork, part, sizes);
  size_t total = 0;
  for (int i = 0; i < nb; ++i) total += align_up(sizes[i] * sizeof(double));
  return total;
}

pprpa_status get_ws(pprpa_ctx* c, int mmax, int nret, int blk, size_t pwork_elems,
                    size_t part_elems, DavWork* w) {
  size_t sizes[32];
  const int nb = ws_sizes(c->g.n, mmax, nret, blk, pwork_elems, part_elems, sizes);
  size_t total = 0;
  for (int i = 0; i < nb; ++i) total += align_up(sizes[i] * sizeof(double));
  if (c->dws.bytes < total) {
    if (c->slab) {
      // a slab-backed context (served request) allocates its workspace once from its slab
      if (c->dws.base) {
        set_error("workspace of %zu bytes exceeds the request's reservation", total);
        return PPRPA_ENOMEM;
      }
      PPRPA_TRY(dalloc(c, total, &c->dws.base));
    } else {
      if (c->dws.base) (void)hipFree(c->dws.base);
      c->dws.base = nullptr;
      c->dws.bytes = 0;
      hipError_t e = hipMalloc(&c->dws.base, total);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        c->dws.base = nullptr;
        set_error("Davidson workspace of %zu bytes: %s", total, hipGetErrorString(e));
        return PPRPA_ENOMEM;
      }
    }
    c->dws.bytes = total;
  }
  char* p = (char*)c->dws.base;
  double** slots[] = {&w->V,  &w->SV, &w->Vt, &w->SVt, &w->Ms, &w->Ws_, &w->Mt, &w->Wt,
                      &w->Cc, &w->Q,  &w->Z,  &w->SZ,  &w->R,  &w->Tn,  &w->Tn2, &w->Cp,
                      &w->Gb, &w->Tm, &w->omega, &w->rnorm, &w->part, &w->pwork, nullptr};
  for (int i = 0; i < nb; ++i) {
    if (slots[i])
      *slots[i] = (double*)p;
    else
      w->info = (int*)p;
    p += align_up(sizes[i] * sizeof(double));
  }
  return PPRPA_OK;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

size_t davidson_workspace_bytes(const Geometry& g, const pprpa_davidson_args& a) {
  Shape sh;
  if (shape_of(g, &a, &sh) != PPRPA_OK) return 0;
  return ws_total(g.n, sh.mmax, sh.nret, sh.tblk, (size_t)7 * sh.mmax * sh.mmax,
                  std::max((size_t)sh.nch * sh.mmax * sh.tblk, (size_t)sh.nret * 64));
}

pprpa_status Solver::fail(pprpa_status s) {
  status = s;
  message = pprpa_last_error();
  phase = DONE;
  return s;
}

pprpa_status Solver::done(pprpa_status s) {
  status = s;
  message = s == PPRPA_OK ? std::string() : std::string(pprpa_last_error());
  phase = DONE;
  return PPRPA_OK;
}

void Solver::log_iteration(int nconv, double maxr, int sweeps) {
  if (!a_.log) return;
  char buf[320];
  snprintf(buf, sizeof buf,
           "{\"iter\": %d, \"subspace\": %d, \"n_conv\": %d, \"max_resid\": %.3e, \"omega0\": %.12f, "
           "\"n_sigma\": %d, \"rr_sweeps\": %d}",
           iter_, m_, nconv, maxr, om_[0], nsig_, sweeps);
  a_.log(a_.user, buf);
}

pprpa_status Solver::start() {
  t0_ = std::chrono::steady_clock::now();
  status = PPRPA_OK;
  Shape sh;
  pprpa_status rc = shape_of(c_->g, &a_, &sh);
  if (rc != PPRPA_OK) return fail(rc);
  if (a_.direct) {
    rc = run_direct();
    return rc == PPRPA_OK ? PPRPA_OK : fail(rc);
  }
  nroot_ = sh.nroot;
  blk_ = sh.blk;
  max_iter_ = sh.max_iter;
  mmax_ = sh.mmax;
  nret_ = sh.nret;
  tblk_ = sh.tblk;
  nch_ = sh.nch;
  rc = get_ws(c_, mmax_, nret_, tblk_, (size_t)7 * mmax_ * mmax_,
              std::max((size_t)nch_ * mmax_ * tblk_, (size_t)nret_ * nres_), &w);
  if (rc != PPRPA_OK) return fail(rc);
  rc = initial_subspace(sh);
  if (rc != PPRPA_OK) return fail(rc);
  sig_m0 = 0;
  sig_k = m_;
  nsig_ = m_;
  mnew0_ = 0;
  phase = NEED_SIGMA;
  return PPRPA_OK;
}

pprpa_status Solver::initial_subspace(const Shape& sh) {
  const int64_t n = c_->g.n, nvv = c_->g.nvv;
  hipStream_t s = c_->stream;
  if (sh.nguess > 0) {
    PPRPA_HIP(hipMemcpyAsync(w.Tn, a_.guess, (size_t)sh.nguess * n * sizeof(double),
                             hipMemcpyHostToDevice, s));
    m_ = 0;
    PPRPA_TRY(orth_pass1(sh.nguess));
    PPRPA_HIP(hipStreamSynchronize(s));
    const int kept = *(int*)c_->pinned;
    int added = 0;
    if (kept > 0) {
      PPRPA_TRY(orth_pass2(kept));
      PPRPA_HIP(hipStreamSynchronize(s));
      added = std::max(*(int*)c_->pinned, 0);
      if (added > 0) PPRPA_TRY(orth_commit(kept, added));
    }
    if (added < nroot_) {
      set_error("initial guesses span only %d directions", added);
      return PPRPA_EINVAL;
    }
    m_ = added;
    return PPRPA_OK;
  }
  // unit vectors on the nb0 lowest virtual-pair energies (pp) or the nb0 highest occupied-pair
  // energies (hh), ties: lowest index
  // (the diagonal pair energies: +(e_a + e_b) for pp pairs, -(e_i + e_j) for hh pairs, so both
  // channels take the smallest values)
  const bool hh = a_.channel == 1;
  std::vector<int64_t> idx(hh ? n - nvv : nvv);
  std::iota(idx.begin(), idx.end(), hh ? nvv : 0);
  const std::vector<double>& ep = c_->epair_h;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return ep[x] < ep[y]; });
  PPRPA_HIP(launch_fill(w.V, (size_t)sh.nb0 * n, 0.0, s));
  PPRPA_HIP(launch_set_units(w.V, n, idx.data(), sh.nb0, s));
  m_ = sh.nb0;
  return PPRPA_OK;
}

// Orthonormalisation of the correction rows Tn[0:nsel] against V[0:m] and among themselves, in
// two passes: pass 1 normalises, projects out V twice and forms the block's Gram matrix
// transform (count kept -> pinned[0]); pass 2 applies it into Tn2, projects out V once more and
// repeats the Gram step (count -> pinned[0]); commit appends the result to V at row m.
pprpa_status Solver::orth_pass1(int nsel) {
  const int64_t n = c_->g.n;
  hipStream_t s = c_->stream;
  PPRPA_HIP(launch_normalize_rows(w.Tn, n, nsel, n, s));
  for (int pass = 0; pass < 2 && m_ > 0; ++pass) {
    PPRPA_HIP(launch_dots(w.V, n, m_, w.Tn, n, nsel, n, 0, 0, w.Cp, tblk_, w.part, nch_, s));
    PPRPA_HIP(launch_combine(w.V, n, m_, w.Cp, tblk_, nsel, n, -1.0, 1.0, w.Tn, n, s));
  }
  PPRPA_HIP(launch_dots(w.Tn, n, nsel, w.Tn, n, nsel, n, 0, 0, w.Gb, tblk_, w.part, nch_, s));
  PPRPA_HIP(launch_gram_orth(w.Gb, tblk_, nsel, 1e-10, w.Tm, tblk_, w.info + 4, w.pwork, s));
  PPRPA_HIP(hipMemcpyAsync(c_->pinned, w.info + 4, sizeof(int), hipMemcpyDeviceToHost, s));
  nsel_ = nsel;
  return PPRPA_OK;
}

pprpa_status Solver::orth_pass2(int kept) {
  const int64_t n = c_->g.n;
  hipStream_t s = c_->stream;
  PPRPA_HIP(launch_combine(w.Tn, n, nsel_, w.Tm, tblk_, kept, n, 1.0, 0.0, w.Tn2, n, s));
  if (m_ > 0) {
    PPRPA_HIP(launch_dots(w.V, n, m_, w.Tn2, n, kept, n, 0, 0, w.Cp, tblk_, w.part, nch_, s));
    PPRPA_HIP(launch_combine(w.V, n, m_, w.Cp, tblk_, kept, n, -1.0, 1.0, w.Tn2, n, s));
  }
  PPRPA_HIP(launch_dots(w.Tn2, n, kept, w.Tn2, n, kept, n, 0, 0, w.Gb, tblk_, w.part, nch_, s));
  PPRPA_HIP(launch_gram_orth(w.Gb, tblk_, kept, 1e-10, w.Tm, tblk_, w.info + 4, w.pwork, s));
  PPRPA_HIP(hipMemcpyAsync(c_->pinned, w.info + 4, sizeof(int), hipMemcpyDeviceToHost, s));
  kept_ = kept;
  return PPRPA_OK;
}

pprpa_status Solver::orth_commit(int kept, int kept2) {
  const int64_t n = c_->g.n;
  PPRPA_HIP(launch_combine(w.Tn2, n, kept, w.Tm, tblk_, kept2, n, 1.0, 0.0, w.V + (size_t)m_ * n, n,
                           c_->stream));
  return PPRPA_OK;
}

pprpa_status Solver::rr_launch() {
  const int64_t n = c_->g.n, nvv = c_->g.nvv;
  hipStream_t s = c_->stream;
  double* hp = c_->pinned;  // [0,64) omega, [64,128) rnorm, [128,..) ints
  const int nb = m_ - mnew0_;
  if (nb > 0) {
    PPRPA_HIP(launch_dots(w.V, n, m_, w.SV + (size_t)mnew0_ * n, n, nb, n, 0, 0, w.Ms + mnew0_,
                          mmax_, w.part, nch_, s));
    PPRPA_HIP(launch_dots(w.V, n, m_, w.V + (size_t)mnew0_ * n, n, nb, n, nvv, 1, w.Ws_ + mnew0_,
                          mmax_, w.part, nch_, s));
  }
  PPRPA_HIP(launch_pencil(w.Ms, w.Ws_, mmax_, m_, c_->mu2, nroot_, std::min(nret_, m_),
                          a_.channel, w.omega, w.Cc, nret_, w.pwork, w.info, s));
  PPRPA_HIP(launch_combine(w.V, n, m_, w.Cc, nret_, nroot_, n, 1.0, 0.0, w.Z, n, s));
  PPRPA_HIP(launch_combine(w.SV, n, m_, w.Cc, nret_, nroot_, n, 1.0, 0.0, w.SZ, n, s));
  PPRPA_HIP(launch_residual(w.Z, w.SZ, n, nroot_, n, nvv, w.omega, w.R, w.part, nres_, s));
  PPRPA_HIP(launch_reduce_norms(w.part, nres_, nroot_, w.rnorm, s));
  PPRPA_HIP(hipMemcpyAsync(hp, w.omega, nroot_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PPRPA_HIP(hipMemcpyAsync(hp + 64, w.rnorm, nroot_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PPRPA_HIP(hipMemcpyAsync(hp + 128, w.info, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  phase = RR_READ;
  return PPRPA_OK;
}

pprpa_status Solver::rr_read() {
  const double* hp = c_->pinned;
  if (sig_timed_) {
    float ms = 0.f;
    PPRPA_HIP(hipEventElapsedTime(&ms, c_->e0, c_->e1));
    t_sigma += ms * 1e-3;
    sig_timed_ = false;
  }
  PPRPA_TRY(harvest_timing(c_));
  const int* info = (const int*)(hp + 128);
  npos_ = info[1];
  if (info[0] == 1) {
    set_error("projected pencil V(M - 2 mu W)V^T not positive definite at iteration %d", iter_);
    return fail(PPRPA_ENONDEF);
  }
  if (info[0] == 2) {
    set_error("projected pencil has %d %s roots, fewer than nroot=%d", npos_,
              a_.channel == 0 ? "pp" : "hh", nroot_);
    return fail(PPRPA_ENONDEF);
  }
  std::copy(hp, hp + nroot_, om_);
  std::copy(hp + 64, hp + 64 + nroot_, rn_);
  have_iterate_ = true;
  ++iter_;
  nconv_ = 0;
  maxr_ = 0.0;
  sel_.clear();
  for (int j = 0; j < nroot_; ++j) {
    if (!std::isfinite(rn_[j])) {
      set_error("non-finite residual at iteration %d", iter_);
      return fail(PPRPA_EDEVICE);
    }
    maxr_ = std::max(maxr_, rn_[j]);
    if (rn_[j] <= a_.tol)
      ++nconv_;
    else if ((int)sel_.size() < blk_)
      sel_.push_back(j);
  }
  log_iteration(nconv_, maxr_, info[2]);
  if (nconv_ == nroot_) return done(PPRPA_OK);
  if (iter_ >= max_iter_) {
    set_error("Davidson not converged in %d iterations (max residual %.3e)", iter_, maxr_);
    return done(PPRPA_ENOCONV);
  }
  const int nsel = (int)sel_.size();
  // restart if the new block does not fit
  if (m_ + nsel > mmax_) {
    int nkeep = std::min(std::min(nret_, m_), std::max(npos_, nroot_));
    nkeep = std::max(nroot_, std::min(nkeep, mmax_ - nsel));
    PPRPA_HIP(launch_small_orth(w.Cc, nret_, m_, nkeep, w.Q, nret_, w.info + 6, c_->stream));
    PPRPA_HIP(hipMemcpyAsync(c_->pinned + 130, w.info + 6, sizeof(int), hipMemcpyDeviceToHost,
                             c_->stream));
    phase = RESTART_READ;
    return PPRPA_OK;
  }
  return launch_corrections();
}

pprpa_status Solver::restart_read() {
  const int64_t n = c_->g.n;
  hipStream_t s = c_->stream;
  const int rank = *(const int*)(c_->pinned + 130);
  if (rank < nroot_) {
    set_error("restart basis lost rank (%d < %d)", rank, nroot_);
    return done(PPRPA_ENOCONV);
  }
  PPRPA_HIP(launch_combine(w.V, n, m_, w.Q, nret_, rank, n, 1.0, 0.0, w.Vt, n, s));
  PPRPA_HIP(launch_combine(w.SV, n, m_, w.Q, nret_, rank, n, 1.0, 0.0, w.SVt, n, s));
  PPRPA_HIP(launch_small_congruence(w.Ms, mmax_, m_, w.Q, nret_, rank, w.Mt, mmax_, w.pwork, s));
  PPRPA_HIP(launch_small_congruence(w.Ws_, mmax_, m_, w.Q, nret_, rank, w.Wt, mmax_, w.pwork, s));
  std::swap(w.V, w.Vt);
  std::swap(w.SV, w.SVt);
  std::swap(w.Ms, w.Mt);
  std::swap(w.Ws_, w.Wt);
  m_ = rank;
  mnew0_ = m_;
  return launch_corrections();
}

pprpa_status Solver::launch_corrections() {
  const int64_t n = c_->g.n, nvv = c_->g.nvv;
  const int nsel = (int)sel_.size();
  PPRPA_HIP(launch_precond(w.R, n, sel_.data(), nsel, n, nvv, c_->epair, w.omega, w.Tn, n,
                           c_->stream));
  PPRPA_TRY(orth_pass1(nsel));
  phase = ORTH1_READ;
  return PPRPA_OK;
}

pprpa_status Solver::orth1_read() {
  const int kept = *(const int*)c_->pinned;
  if (kept <= 0) return stagnated();
  PPRPA_TRY(orth_pass2(kept));
  phase = ORTH2_READ;
  return PPRPA_OK;
}

pprpa_status Solver::orth2_read() {
  const int kept2 = *(const int*)c_->pinned;
  if (kept2 <= 0) return stagnated();
  PPRPA_TRY(orth_commit(kept_, kept2));
  sig_m0 = m_;
  sig_k = kept2;
  nsig_ += kept2;
  mnew0_ = m_;
  m_ += kept2;
  phase = NEED_SIGMA;
  return PPRPA_OK;
}

pprpa_status Solver::stagnated() {
  set_error("Davidson stagnated: corrections lie in the subspace (max residual %.3e)", maxr_);
  return done(PPRPA_ENOCONV);
}

pprpa_status Solver::advance() {
  pprpa_status rc = PPRPA_OK;
  switch (phase) {
    case RR_LAUNCH: rc = rr_launch(); break;
    case RR_READ: rc = rr_read(); break;
    case RESTART_READ: rc = restart_read(); break;
    case ORTH1_READ: rc = orth1_read(); break;
    case ORTH2_READ: rc = orth2_read(); break;
    default:
      set_error("solver advanced in phase %d", (int)phase);
      rc = PPRPA_EINVAL;
  }
  if (rc != PPRPA_OK && phase != DONE) return fail(rc);
  return rc;
}

pprpa_status Solver::results(double* omega, double* vecs, double* resid, pprpa_report* rep) {
  const int64_t n = c_->g.n;
  const bool filled = (status == PPRPA_OK || status == PPRPA_ENOCONV) && have_iterate_;
  if (filled) {
    if (omega) std::copy(om_, om_ + nroot_, omega);
    if (resid) std::copy(rn_, rn_ + nroot_, resid);
    if (vecs) {
      PPRPA_HIP(launch_scale_sign(w.Z, n, nroot_, n, c_->stream));
      PPRPA_HIP(hipMemcpyAsync(vecs, w.Z, (size_t)nroot_ * n * sizeof(double),
                               hipMemcpyDeviceToHost, c_->stream));
    }
    PPRPA_HIP(hipStreamSynchronize(c_->stream));
  }
  if (rep) {
    pprpa_report R{};
    R.iters = iter_;
    R.n_sigma = nsig_;
    R.n_conv = nconv_;
    R.subspace = m_;
    R.max_resid = maxr_;
    R.t_sigma_s = t_sigma;
    R.t_total_s = seconds_since(t0_);
    *rep = R;
  }
  return PPRPA_OK;
}

// Direct diagonalisation of the dense pencil (M, W) with the same device pencil solver.
pprpa_status Solver::run_direct() {
  TraceRange tr("davidson.direct");
  const Geometry& g = c_->g;
  const int64_t n = g.n, nvv = g.nvv;
  hipStream_t s = c_->stream;
  nroot_ = a_.nroot;
  if (!c_->M) {
    set_error("direct diagonalisation needs a dense build");
    return PPRPA_EUNSUPPORTED;
  }
  if (n > DENSE_SOLVE_MAX) {
    set_error("direct diagonalisation on the device is limited to n <= %d (n=%lld)",
              DENSE_SOLVE_MAX, (long long)n);
    return PPRPA_EUNSUPPORTED;
  }
  const int m = (int)n;
  PPRPA_TRY(get_ws(c_, m, nroot_, 1,
                   std::max({(size_t)4 * m * m, (size_t)3 * m * m + 4 * 64 * m,
                             direct_pencil_mw_work(m, nroot_)}),
                   (size_t)nroot_ * 64, &w));
  double* hp = c_->pinned;
  PPRPA_HIP(launch_metric_matrix(w.Ws_, n, nvv, s));
  if (m <= DENSE_ONE_WG_MAX)  // W as a dense matrix: the Davidson pencil solver on the whole problem
    PPRPA_HIP(launch_pencil(c_->M, w.Ws_, m, m, c_->mu2, nroot_, nroot_, a_.channel, w.omega,
                            w.Cc, nroot_, w.pwork, w.info, s));
  else  // W diagonal, many workgroups
    PPRPA_HIP(launch_direct_pencil_mw(c_->M, m, nvv, c_->mu2, nroot_, a_.channel, w.omega, w.Cc,
                                      nroot_, w.pwork, w.info, s));
  PPRPA_HIP(launch_transpose(w.Cc, nroot_, m, nroot_, w.Z, n, s));
  PPRPA_HIP(launch_combine(c_->M, n, m, w.Cc, nroot_, nroot_, n, 1.0, 0.0, w.SZ, n, s));
  PPRPA_HIP(launch_residual(w.Z, w.SZ, n, nroot_, n, nvv, w.omega, w.R, w.part, 64, s));
  PPRPA_HIP(launch_reduce_norms(w.part, 64, nroot_, w.rnorm, s));
  PPRPA_HIP(hipMemcpyAsync(hp, w.omega, nroot_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PPRPA_HIP(hipMemcpyAsync(hp + 64, w.rnorm, nroot_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PPRPA_HIP(hipMemcpyAsync(hp + 128, w.info, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  PPRPA_HIP(hipStreamSynchronize(s));
  const int* info = (const int*)(hp + 128);
  if (info[0] == 1) {
    set_error("M - 2 mu W is not positive definite");
    return PPRPA_ENONDEF;
  }
  if (info[0] == 2) {
    set_error("fewer than nroot %s roots (%d)", a_.channel == 0 ? "pp" : "hh", info[1]);
    return PPRPA_ENONDEF;
  }
  std::copy(hp, hp + nroot_, om_);
  std::copy(hp + 64, hp + 64 + nroot_, rn_);
  have_iterate_ = true;
  nconv_ = nroot_;
  maxr_ = *std::max_element(rn_, rn_ + nroot_);
  m_ = m;
  if (info[0] == 3) {
    set_error("dense pencil eigensolver did not converge");
    return done(PPRPA_ENOCONV);
  }
  return done(PPRPA_OK);
}

static const char* phase_name(Solver::Phase p) {
  switch (p) {
    case Solver::RR_LAUNCH: return "davidson.rayleigh_ritz";
    case Solver::RR_READ: return "davidson.ritz_read";
    case Solver::RESTART_READ: return "davidson.restart";
    case Solver::ORTH1_READ: return "davidson.orth1";
    case Solver::ORTH2_READ: return "davidson.orth2";
    default: return "davidson.phase";
  }
}

// Up to n_iter iterations of a started solve, phases run back to back. An iteration starts with
// the sigma product of the pending block and ends when the next block is requested or the solve
// is done; *done_iters counts the iterations run.
pprpa_status iterate_solver(pprpa_ctx* c, Solver& sv, int n_iter, int* done_iters) {
  int it = 0;
  while (sv.phase != Solver::DONE && it < n_iter) {
    if (sv.phase == Solver::NEED_SIGMA) {
      TraceRange tr("davidson.sigma");
      const int64_t n = c->g.n;
      PPRPA_HIP(hipEventRecord(c->e0, c->stream));
      pprpa_status rc = sigma_device(c, sv.sig_k, sv.w.V + (size_t)sv.sig_m0 * n,
                                     sv.w.SV + (size_t)sv.sig_m0 * n);
      if (rc != PPRPA_OK) return rc;
      PPRPA_HIP(hipEventRecord(c->e1, c->stream));
      sv.sigma_done(true);
    }
    while (sv.phase != Solver::DONE && sv.phase != Solver::NEED_SIGMA) {
      if (sv.phase != Solver::RR_LAUNCH) {
        TraceRange tw("davidson.wait");
        PPRPA_HIP(hipStreamSynchronize(c->stream));
      }
      TraceRange tp(phase_name(sv.phase));
      sv.advance();
    }
    ++it;
  }
  if (done_iters) *done_iters = it;
  return PPRPA_OK;
}

// Outputs of a solve as pprpa_davidson returns them: its final status (ENOCONV if the caller
// stopped it before convergence), with omega/resid/rep filled from the last iterate.
pprpa_status finish_solver(Solver& sv, double* omega, double* vecs, double* resid,
                           pprpa_report* rep) {
  if (sv.phase != Solver::DONE) {
    set_error("Davidson stopped by the caller after %d iterations (not converged)", sv.iters());
    sv.status = PPRPA_ENOCONV;
    sv.message = pprpa_last_error();
  }
  if (sv.status != PPRPA_OK && !sv.message.empty()) set_error("%s", sv.message.c_str());
  const pprpa_status st = sv.status;
  if (st == PPRPA_OK || st == PPRPA_ENOCONV || rep) {
    const std::string keep = sv.message;
    pprpa_status f = sv.results(omega, vecs, resid, rep);
    if (f != PPRPA_OK) return f;
    if (!keep.empty()) set_error("%s", keep.c_str());
  }
  return st;
}

// One solve on one context, phases run back to back.
pprpa_status run_davidson(pprpa_ctx* c, const pprpa_davidson_args* a, double* omega, double* vecs,
                          double* resid, pprpa_report* rep) {
  TraceRange tr("pprpa_davidson");
  Solver sv(c, *a);
  sv.start();
  PPRPA_TRY(iterate_solver(c, sv, INT32_MAX, nullptr));
  return finish_solver(sv, omega, vecs, resid, rep);
}

}  // namespace pprpa
