// Block Davidson solver for the lowest pp roots of M z = Omega W z, and the direct dense path.
//
// arXiv 2512.12515 (sections "ppRPA Equation" and "Implementation Details") names the Davidson
// algorithm and direct diagonalisation as the two solvers but gives no algorithmic detail; the
// design here:
//  * subspace V (orthonormal rows, Euclidean) grown by blocks; projected pencil
//    (V M V^T, V W V^T) solved on the device through the definite shift M - 2 mu W
//    (mu = mid-gap of the active window), whose positive-theta roots are the pp roots, so the
//    wanted roots are the nroot largest theta (lowest Omega > 2 mu);
//  * Ritz vectors z = V^T c with z^T W z = +1 (Eq. xy_norm); residual r = M z - Omega W z,
//    converged when ||r||_2 <= tol for every wanted root;
//  * corrections t = r / (Omega w - D) from the diagonal pair energies D, normalised, projected
//    out of V twice (classical Gram-Schmidt, two passes) and orthonormalised within the block
//    from their Gram matrix (eigenvalue cut drops dependent directions), twice;
//  * restart when the subspace would exceed max_subspace: keep the 2*nroot best Ritz vectors,
//    orthonormalised in the small space, and rotate V, sigma(V) and the projected matrices with
//    them (no new sigma products).
// All arithmetic is FP64 on the device; the host runs the control loop and reads back nroot
// eigenvalues, nroot residual norms and a few counters per iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <numeric>

#include "ctx.h"

namespace pprpa {
namespace {

struct Ws {
  double *V, *SV, *Vt, *SVt, *Ms, *Ws_, *Mt, *Wt, *Cc, *Q, *Z, *SZ, *R, *Tn, *Tn2, *Cp, *Gb, *Tm;
  double *omega, *rnorm, *part, *pwork, *Up;
  int* info;
};

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

static pprpa_status get_ws(pprpa_ctx* c, int mmax, int nret, int blk, size_t pwork_elems,
                           size_t part_elems, Ws* w) {
  const int64_t n = c->g.n;
  const size_t vecs = (size_t)mmax * n;
  size_t sizes[] = {vecs, vecs, vecs, vecs,                                          // V SV Vt SVt
                    (size_t)mmax * mmax, (size_t)mmax * mmax, (size_t)mmax * mmax,   // Ms Ws Mt
                    (size_t)mmax * mmax,                                             // Wt
                    (size_t)mmax * nret, (size_t)mmax * nret,                        // Cc Q
                    (size_t)nret * n, (size_t)nret * n, (size_t)nret * n,            // Z SZ R
                    (size_t)blk * n, (size_t)blk * n,                                // Tn Tn2
                    (size_t)mmax * blk, (size_t)blk * blk, (size_t)blk * blk,        // Cp Gb Tm
                    (size_t)nret, (size_t)nret, part_elems, pwork_elems, (size_t)mmax * mmax, 16};
  const int nb = sizeof(sizes) / sizeof(sizes[0]);
  size_t total = 0;
  for (int i = 0; i < nb; ++i) total += align_up(sizes[i] * sizeof(double));
  if (c->dws.bytes < total) {
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
    c->dws.bytes = total;
  }
  char* p = (char*)c->dws.base;
  double** slots[] = {&w->V,  &w->SV, &w->Vt, &w->SVt, &w->Ms, &w->Ws_, &w->Mt, &w->Wt,
                      &w->Cc, &w->Q,  &w->Z,  &w->SZ,  &w->R,  &w->Tn,  &w->Tn2, &w->Cp,
                      &w->Gb, &w->Tm, &w->omega, &w->rnorm, &w->part, &w->pwork, &w->Up, nullptr};
  for (int i = 0; i < nb; ++i) {
    if (slots[i])
      *slots[i] = (double*)p;
    else
      w->info = (int*)p;
    p += align_up(sizes[i] * sizeof(double));
  }
  return PPRPA_OK;
}

// Orthonormalise rows Tn[0:nsel] against V[0:m] and among themselves; append to V at row m.
// Returns the number of vectors appended in *added.
static pprpa_status add_vectors(pprpa_ctx* c, Ws& w, int m, int nsel, int blk, int* added) {
  const int64_t n = c->g.n;
  const int nch = (int)std::min<int64_t>(512, std::max<int64_t>(1, n / 256));
  hipStream_t s = c->stream;
  PPRPA_HIP(launch_normalize_rows(w.Tn, n, nsel, n, s));
  for (int pass = 0; pass < 2 && m > 0; ++pass) {
    PPRPA_HIP(launch_dots(w.V, n, m, w.Tn, n, nsel, n, 0, 0, w.Cp, blk, w.part, nch, s));
    PPRPA_HIP(launch_combine(w.V, n, m, w.Cp, blk, nsel, n, -1.0, 1.0, w.Tn, n, s));
  }
  PPRPA_HIP(launch_dots(w.Tn, n, nsel, w.Tn, n, nsel, n, 0, 0, w.Gb, blk, w.part, nch, s));
  PPRPA_HIP(launch_gram_orth(w.Gb, blk, nsel, 1e-10, w.Tm, blk, w.info + 4, w.pwork, s));
  PPRPA_HIP(hipMemcpyAsync(c->pinned, w.info + 4, sizeof(int), hipMemcpyDeviceToHost, s));
  PPRPA_HIP(hipStreamSynchronize(s));
  const int kept = *(int*)c->pinned;
  if (kept <= 0) {
    *added = 0;
    return PPRPA_OK;
  }
  PPRPA_HIP(launch_combine(w.Tn, n, nsel, w.Tm, blk, kept, n, 1.0, 0.0, w.Tn2, n, s));
  if (m > 0) {
    PPRPA_HIP(launch_dots(w.V, n, m, w.Tn2, n, kept, n, 0, 0, w.Cp, blk, w.part, nch, s));
    PPRPA_HIP(launch_combine(w.V, n, m, w.Cp, blk, kept, n, -1.0, 1.0, w.Tn2, n, s));
  }
  PPRPA_HIP(launch_dots(w.Tn2, n, kept, w.Tn2, n, kept, n, 0, 0, w.Gb, blk, w.part, nch, s));
  PPRPA_HIP(launch_gram_orth(w.Gb, blk, kept, 1e-10, w.Tm, blk, w.info + 4, w.pwork, s));
  PPRPA_HIP(hipMemcpyAsync(c->pinned, w.info + 4, sizeof(int), hipMemcpyDeviceToHost, s));
  PPRPA_HIP(hipStreamSynchronize(s));
  const int kept2 = *(int*)c->pinned;
  if (kept2 > 0)
    PPRPA_HIP(launch_combine(w.Tn2, n, kept, w.Tm, blk, kept2, n, 1.0, 0.0, w.V + (size_t)m * n, n, s));
  *added = std::max(kept2, 0);
  return PPRPA_OK;
}

static void emit_log(const pprpa_davidson_args* a, int iter, int m, int nconv, double maxr,
                     double om0, int nsig, int sweeps) {
  if (!a->log) return;
  char buf[320];
  snprintf(buf, sizeof buf,
           "{\"iter\": %d, \"subspace\": %d, \"n_conv\": %d, \"max_resid\": %.3e, \"omega0\": %.12f, "
           "\"n_sigma\": %d, \"rr_sweeps\": %d}",
           iter, m, nconv, maxr, om0, nsig, sweeps);
  a->log(a->user, buf);
}

static pprpa_status finish(pprpa_ctx* c, Ws& w, int nroot, double* omega, double* vecs,
                           double* resid, pprpa_report* rep, const double* h_omega,
                           const double* h_rn) {
  const int64_t n = c->g.n;
  for (int j = 0; j < nroot; ++j) omega[j] = h_omega[j];
  if (resid)
    for (int j = 0; j < nroot; ++j) resid[j] = h_rn[j];
  if (vecs) {
    PPRPA_HIP(launch_scale_sign(w.Z, n, nroot, n, c->stream));
    PPRPA_HIP(hipMemcpyAsync(vecs, w.Z, (size_t)nroot * n * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  }
  PPRPA_HIP(hipStreamSynchronize(c->stream));
  (void)rep;
  return PPRPA_OK;
}

pprpa_status run_davidson(pprpa_ctx* c, const pprpa_davidson_args* a, double* omega, double* vecs,
                          double* resid, pprpa_report* rep) {
  const auto t_start = std::chrono::steady_clock::now();
  const Geometry& g = c->g;
  const int64_t n = g.n, nvv = g.nvv;
  hipStream_t s = c->stream;
  const int nroot = a->nroot;
  if (nroot < 1 || nroot > nvv) {
    set_error("nroot=%d outside [1, n_pp=%lld]", nroot, (long long)nvv);
    return PPRPA_EINVAL;
  }
  if (nroot > 64) {
    set_error("nroot=%d exceeds 64", nroot);
    return PPRPA_EUNSUPPORTED;
  }
  if (!(a->tol > 0.0) && !a->direct) {
    set_error("tol must be positive");
    return PPRPA_EINVAL;
  }
  pprpa_report R{};
  double* hp = c->pinned;  // [0,64) omega, [64,128) rnorm, [128,..) ints

  // ------------------------------------------------------------------ direct diagonalisation
  if (a->direct) {
    if (!c->M) {
      set_error("direct diagonalisation needs a dense build");
      return PPRPA_EUNSUPPORTED;
    }
    if (n > 512) {
      set_error("direct diagonalisation on the device is limited to n <= 512 (n=%lld)", (long long)n);
      return PPRPA_EUNSUPPORTED;
    }
    Ws w{};
    const int m = (int)n;
    PPRPA_TRY(get_ws(c, m, nroot, 1, (size_t)4 * m * m, (size_t)nroot * 64, &w));
    // W as a dense matrix in Ws_, M itself as the "projected" matrix
    PPRPA_HIP(launch_metric_matrix(w.Ws_, n, nvv, s));
    PPRPA_HIP(launch_pencil(c->M, w.Ws_, m, m, c->mu2, nroot, nroot, w.omega, w.Cc, nroot, w.pwork,
                            w.info, nullptr, 0, 0, s));
    PPRPA_HIP(launch_transpose(w.Cc, nroot, m, nroot, w.Z, n, s));
    PPRPA_HIP(launch_combine(c->M, n, m, w.Cc, nroot, nroot, n, 1.0, 0.0, w.SZ, n, s));
    PPRPA_HIP(launch_residual(w.Z, w.SZ, n, nroot, n, nvv, w.omega, w.R, w.part, 64, s));
    PPRPA_HIP(launch_reduce_norms(w.part, 64, nroot, w.rnorm, s));
    PPRPA_HIP(hipMemcpyAsync(hp, w.omega, nroot * sizeof(double), hipMemcpyDeviceToHost, s));
    PPRPA_HIP(hipMemcpyAsync(hp + 64, w.rnorm, nroot * sizeof(double), hipMemcpyDeviceToHost, s));
    PPRPA_HIP(hipMemcpyAsync(hp + 128, w.info, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    PPRPA_HIP(hipStreamSynchronize(s));
    const int* info = (const int*)(hp + 128);
    if (info[0] == 1) {
      set_error("M - 2 mu W is not positive definite");
      return PPRPA_ENONDEF;
    }
    if (info[0] == 2) {
      set_error("fewer than nroot pp roots (%d)", info[1]);
      return PPRPA_ENONDEF;
    }
    double om[64], rn[64];
    std::copy(hp, hp + nroot, om);
    std::copy(hp + 64, hp + 64 + nroot, rn);
    PPRPA_TRY(finish(c, w, nroot, omega, vecs, resid, rep, om, rn));
    R.iters = 0;
    R.n_conv = nroot;
    R.max_resid = *std::max_element(rn, rn + nroot);
    R.subspace = m;
    R.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (rep) *rep = R;
    return info[0] == 3 ? PPRPA_ENOCONV : PPRPA_OK;
  }

  // ------------------------------------------------------------------ Davidson
  int blk = a->block > 0 ? a->block : nroot;
  blk = std::max(blk, 1);
  blk = std::min<int64_t>(std::min(blk, 64), nvv);
  const int max_iter = a->max_iter > 0 ? a->max_iter : 100;
  int mmax = a->max_subspace > 0 ? a->max_subspace : std::max(8 * nroot, nroot + 4 * blk);
  mmax = (int)std::min<int64_t>(std::min(mmax, 256), n);
  const int nguess = (a->guess && a->nguess > 0) ? std::min(a->nguess, mmax) : 0;
  int nb0 = nguess > 0 ? nguess : (int)std::min<int64_t>(std::max(blk, nroot), nvv);
  nb0 = std::min(nb0, mmax);
  const int tblk = std::max(blk, nb0);  // rows of the correction buffers
  if (mmax < nroot + 1 && mmax < n) {
    set_error("max_subspace=%d too small for nroot=%d", mmax, nroot);
    return PPRPA_EINVAL;
  }
  const int nret = std::max(nroot, std::min(2 * nroot, mmax / 2));
  const int nch = (int)std::min<int64_t>(512, std::max<int64_t>(1, n / 256));
  const int nres = 64;
  Ws w{};
  PPRPA_TRY(get_ws(c, mmax, nret, tblk, (size_t)4 * mmax * mmax,
                   std::max((size_t)nch * mmax * tblk, (size_t)nret * nres), &w));

  // initial subspace
  int m = 0;
  if (nguess > 0) {
    PPRPA_HIP(hipMemcpyAsync(w.Tn, a->guess, (size_t)nguess * n * sizeof(double),
                             hipMemcpyHostToDevice, s));
    int added = 0;
    PPRPA_TRY(add_vectors(c, w, 0, nguess, tblk, &added));
    if (added < nroot) {
      set_error("initial guesses span only %d directions", added);
      return PPRPA_EINVAL;
    }
    m = added;
  } else {
    // unit vectors on the nb0 lowest virtual-pair energies (ties: lowest index)
    std::vector<int64_t> idx(nvv);
    std::iota(idx.begin(), idx.end(), 0);
    auto epair = [&](int64_t e) {
      const int pq = c->ptab_h[e];
      return c->ev_h[pq >> 16] + c->ev_h[pq & 0xFFFF];
    };
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return epair(x) < epair(y); });
    PPRPA_HIP(launch_fill(w.V, (size_t)nb0 * n, 0.0, s));
    PPRPA_HIP(launch_set_units(w.V, n, idx.data(), nb0, s));
    m = nb0;
  }
  PPRPA_HIP(hipEventRecord(c->e0, s));
  PPRPA_TRY(sigma_device(c, m, w.V, w.SV));
  PPRPA_HIP(hipEventRecord(c->e1, s));
  int nsig = m;
  int mnew0 = 0;
  int mprev = 0;  // pencil size of the previous iteration (0: no warm start)
  double t_sigma = 0.0;
  bool sigma_pending = true;

  double om[64], rn[64];
  pprpa_status status = PPRPA_ENOCONV;
  int iter = 0;
  for (;;) {
    const int nb = m - mnew0;
    if (nb > 0) {
      PPRPA_HIP(launch_dots(w.V, n, m, w.SV + (size_t)mnew0 * n, n, nb, n, 0, 0, w.Ms + mnew0,
                            mmax, w.part, nch, s));
      PPRPA_HIP(launch_dots(w.V, n, m, w.V + (size_t)mnew0 * n, n, nb, n, nvv, 1, w.Ws_ + mnew0,
                            mmax, w.part, nch, s));
    }
    PPRPA_HIP(launch_pencil(w.Ms, w.Ws_, mmax, m, c->mu2, nroot, std::min(nret, m), w.omega, w.Cc,
                            nret, w.pwork, w.info, w.Up, mmax, mprev, s));
    mprev = m;
    PPRPA_HIP(launch_combine(w.V, n, m, w.Cc, nret, nroot, n, 1.0, 0.0, w.Z, n, s));
    PPRPA_HIP(launch_combine(w.SV, n, m, w.Cc, nret, nroot, n, 1.0, 0.0, w.SZ, n, s));
    PPRPA_HIP(launch_residual(w.Z, w.SZ, n, nroot, n, nvv, w.omega, w.R, w.part, nres, s));
    PPRPA_HIP(launch_reduce_norms(w.part, nres, nroot, w.rnorm, s));
    PPRPA_HIP(hipMemcpyAsync(hp, w.omega, nroot * sizeof(double), hipMemcpyDeviceToHost, s));
    PPRPA_HIP(hipMemcpyAsync(hp + 64, w.rnorm, nroot * sizeof(double), hipMemcpyDeviceToHost, s));
    PPRPA_HIP(hipMemcpyAsync(hp + 128, w.info, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    PPRPA_HIP(hipStreamSynchronize(s));
    if (sigma_pending) {
      float ms = 0.f;
      PPRPA_HIP(hipEventElapsedTime(&ms, c->e0, c->e1));
      t_sigma += ms * 1e-3;
      sigma_pending = false;
    }
    PPRPA_TRY(harvest_timing(c));
    const int* info = (const int*)(hp + 128);
    const int npos = info[1];
    if (info[0] == 1) {
      set_error("projected pencil V(M - 2 mu W)V^T not positive definite at iteration %d", iter);
      status = PPRPA_ENONDEF;
      break;
    }
    if (info[0] == 2) {
      set_error("projected pencil has %d pp roots, fewer than nroot=%d", npos, nroot);
      status = PPRPA_ENONDEF;
      break;
    }
    std::copy(hp, hp + nroot, om);
    std::copy(hp + 64, hp + 64 + nroot, rn);
    ++iter;
    int nconv = 0;
    double maxr = 0.0;
    std::vector<int> sel;
    for (int j = 0; j < nroot; ++j) {
      if (!std::isfinite(rn[j])) {
        set_error("non-finite residual at iteration %d", iter);
        return PPRPA_EDEVICE;
      }
      maxr = std::max(maxr, rn[j]);
      if (rn[j] <= a->tol)
        ++nconv;
      else if ((int)sel.size() < blk)
        sel.push_back(j);
    }
    emit_log(a, iter, m, nconv, maxr, om[0], nsig, info[2]);
    R.n_conv = nconv;
    R.max_resid = maxr;
    if (nconv == nroot) {
      status = PPRPA_OK;
      break;
    }
    if (iter >= max_iter) {
      set_error("Davidson not converged in %d iterations (max residual %.3e)", iter, maxr);
      status = PPRPA_ENOCONV;
      break;
    }
    const int nsel = (int)sel.size();
    // restart if the new block does not fit
    if (m + nsel > mmax) {
      int nkeep = std::min(std::min(nret, m), std::max(npos, nroot));
      nkeep = std::max(nroot, std::min(nkeep, mmax - nsel));
      PPRPA_HIP(launch_small_orth(w.Cc, nret, m, nkeep, w.Q, nret, w.info + 6, s));
      PPRPA_HIP(hipMemcpyAsync(hp + 130, w.info + 6, sizeof(int), hipMemcpyDeviceToHost, s));
      PPRPA_HIP(hipStreamSynchronize(s));
      const int rank = *(int*)(hp + 130);
      if (rank < nroot) {
        set_error("restart basis lost rank (%d < %d)", rank, nroot);
        status = PPRPA_ENOCONV;
        break;
      }
      PPRPA_HIP(launch_combine(w.V, n, m, w.Q, nret, rank, n, 1.0, 0.0, w.Vt, n, s));
      PPRPA_HIP(launch_combine(w.SV, n, m, w.Q, nret, rank, n, 1.0, 0.0, w.SVt, n, s));
      PPRPA_HIP(launch_small_congruence(w.Ms, mmax, m, w.Q, nret, rank, w.Mt, mmax, w.pwork, s));
      PPRPA_HIP(launch_small_congruence(w.Ws_, mmax, m, w.Q, nret, rank, w.Wt, mmax, w.pwork, s));
      std::swap(w.V, w.Vt);
      std::swap(w.SV, w.SVt);
      std::swap(w.Ms, w.Mt);
      std::swap(w.Ws_, w.Wt);
      m = rank;
      mnew0 = m;
      mprev = 0;  // the basis was rotated: no warm start
    }
    PPRPA_HIP(launch_precond(w.R, n, sel.data(), nsel, n, nvv, c->epair, w.omega, w.Tn, n, s));
    int added = 0;
    PPRPA_TRY(add_vectors(c, w, m, nsel, tblk, &added));
    if (added == 0) {
      set_error("Davidson stagnated: corrections lie in the subspace (max residual %.3e)", maxr);
      status = PPRPA_ENOCONV;
      break;
    }
    PPRPA_HIP(hipEventRecord(c->e0, s));
    PPRPA_TRY(sigma_device(c, added, w.V + (size_t)m * n, w.SV + (size_t)m * n));
    PPRPA_HIP(hipEventRecord(c->e1, s));
    sigma_pending = true;
    nsig += added;
    mnew0 = m;
    m += added;
  }
  if (status == PPRPA_OK || status == PPRPA_ENOCONV) {
    pprpa_status f = finish(c, w, nroot, omega, vecs, resid, rep, om, rn);
    if (f != PPRPA_OK) return f;
  }
  R.iters = iter;
  R.n_sigma = nsig;
  R.subspace = m;
  R.t_sigma_s = t_sigma;
  R.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (rep) *rep = R;
  return status;
}

}  // namespace pprpa
