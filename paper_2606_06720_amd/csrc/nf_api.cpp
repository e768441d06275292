// Host side of the C ABI declared in include/nf.h: handle and workspace
// management, the PCG driver loop, the time step, the time loop with its
// stopping criteria (Algorithm 1, Sec. 2.5) and the discrete energy.
#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "nf.h"
#include "nf_handle.h"
#include "nf_internal.h"

using namespace nf;

namespace nf {

// Wait for an event of the polling loops by querying it, which returns as soon
// as the event completes; a blocking wait can return later, while the queued
// work (a single PCG iteration once the first chunk is done) runs out.  After
// about a millisecond the wait blocks instead.
hipError_t poll_event(hipEvent_t e) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t q = hipEventQuery(e);
    if (q != hipErrorNotReady) return q;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(1000)) return hipEventSynchronize(e);
  }
}

}  // namespace nf

namespace {

const char* kVersion = "nf-mi355x 0.3 (gfx950; 2D and 3D; FP64 and FP32-refined solves; adjoint step; ensembles)";

// message of the last nf_create_grid failure on this thread (nf_last_error(NULL))
thread_local std::string create_err;

int fail(nf_grid* g, int code, const std::string& msg) {
  if (g) g->err = msg;
  return code;
}

#define HIPCHK(g, expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((g), NF_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));      \
  } while (0)

bool is_pow2_in_range(int64_t v) { return v >= 8 && v <= 4096 && (v & (v - 1)) == 0; }
// 2D sizes: powers of two in [8, 4096] and 50 * 2^k in [50, 1600] (mixed radix 2, 5)
bool is_2d_size(int64_t v) {
  if (is_pow2_in_range(v)) return true;
  for (int64_t s = 50; s <= 1600; s *= 2)
    if (v == s) return true;
  return false;
}
int64_t gcd64(int64_t a, int64_t b) { return b == 0 ? a : gcd64(b, a % b); }

int ilog2i(int v) {
  int p = 0;
  while ((1 << p) < v) ++p;
  return p;
}

// exp(-2 pi i u / N) for u < N, from long double arithmetic with the octant
// symmetries so that each entry is the correctly rounded value in practice.
template <typename T>
void make_twiddles(int N, T* out /* 2N */) {
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int u = 0; u < N; ++u) {
    // reduce to the first octant: angle = 2 pi u / N = (pi/4) * (8u/N)
    long double a = two_pi * (long double)u / (long double)N;
    long double c = cosl(a), s = sinl(a);
    if ((8LL * u) % N == 0) {  // exact multiples of pi/4
      const int oct = (int)((8LL * u) / N);
      const long double r2 = 0.707106781186547524400844362104849039L;
      const long double cs[8] = {1.0L, r2, 0.0L, -r2, -1.0L, -r2, 0.0L, r2};
      const long double sn[8] = {0.0L, r2, 1.0L, r2, 0.0L, -r2, -1.0L, -r2};
      c = cs[oct];
      s = sn[oct];
    }
    out[2 * u] = (T)c;
    out[2 * u + 1] = (T)(-s);
  }
}

int check_launch(nf_grid* g, hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(g, NF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return NF_OK;
}

#define LCHK(g, expr)                               \
  do {                                              \
    int rc_ = check_launch((g), (expr), #expr);     \
    if (rc_ != NF_OK) return rc_;                   \
  } while (0)

int read_status(nf_grid* g, DevStatus* dst) {
  HIPCHK(g, hipMemcpyAsync(dst, g->st, sizeof(DevStatus), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return NF_OK;
}

// b_hat = F(Pi S) and the compatibility partials of S
int compute_rhs(nf_grid* g, const double* S) {
  const Geo& G = g->geo;
  if (g->dim == 3) {
    LCHK(g, launch3_row_r2c(G, S, g->mix[0], 1, g->stream));
    LCHK(g, launch3_ypass(G, false, 1, -1, g->mix[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, g->stream));
    LCHK(g, launch3_zfwd(G, g->mix[0], g->bh, 1, g->stream));
    return NF_OK;
  }
  LCHK(g, launch_row_r2c(G, S, g->mix[0], slot_ptr(g->part, SLOT_SCHK), g->stream));
  LCHK(g, launch_col_fwd(G, g->mix[0], g->bh, 0, nullptr, nullptr, g->stream));
  return NF_OK;
}

enum XSource { X_FROM_P = 0, X_FROM_XH = 1, X_ZERO = 2 };

// Timing hooks: when the handle times kernel `which`, the kernel stamps, for
// each loop iteration, the earliest workgroup start and the latest workgroup
// end on the device wall clock (Geo::tclk).  The stamps are cleared before
// each PCG loop and copied out after it without waiting (pinned buffer, event);
// the host adds them up before the next copy or when the totals are read, so
// timing adds no synchronisation to the loop.  Launches queued after the
// solver stopped (no-ops) are discarded.  The launch events are no longer used.
int timed_events(nf_grid* g, int which, int it, hipEvent_t* e0, hipEvent_t* e1) {
  (void)g;
  (void)which;
  (void)it;
  *e0 = *e1 = nullptr;
  return NF_OK;
}
int timed_reset(nf_grid* g) {
  if (g->timed < 0) return NF_OK;
  LCHK(g, launch_tclk_reset(g->tclk, g->stream));
  return NF_OK;
}
// adds the stamps of the last copy (waits for it if it is still in flight)
int timed_flush(nf_grid* g) {
  if (!g->tclk_pending) return NF_OK;
  g->tclk_pending = 0;
  HIPCHK(g, hipEventSynchronize(g->tclk_ev));
  for (int it = g->tclk_lo; it <= g->tclk_hi; ++it) {
    unsigned long long t0 = ~0ULL, t1 = 0;
    for (int w = 0; w < TCLK_W; ++w) {
      const unsigned long long a = g->htclk[2 * ((size_t)it * TCLK_W + w)], b = g->htclk[2 * ((size_t)it * TCLK_W + w) + 1];
      if (a < t0) t0 = a;
      if (b > t1) t1 = b;
    }
    if (t0 == ~0ULL || t1 < t0) continue;
    g->timed_ms += (double)(t1 - t0) / g->wall_khz;
    g->timed_count++;
  }
  return NF_OK;
}
// after a PCG loop whose stop iteration is known; flux and div of iteration it
// did work iff it < conv_at, the update stamped with it iff 1 <= it <= conv_at
int timed_collect(nf_grid* g, int conv_at) {
  if (g->timed < 0) return NF_OK;
  int rc = timed_flush(g);
  if (rc) return rc;
  const int lo = g->timed == NF_KERNEL_COL_UPDATE ? 1 : 0;
  int hi = g->timed == NF_KERNEL_COL_UPDATE ? conv_at : conv_at - 1;
  if (hi > TCLK_CAP - 1) hi = TCLK_CAP - 1;
  if (hi < lo) return NF_OK;
  const size_t n = (size_t)(hi + 1) * TCLK_W * 2;
  HIPCHK(g, hipMemcpyAsync(g->htclk, g->tclk, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipEventRecord(g->tclk_ev, g->stream));
  g->tclk_lo = lo;
  g->tclk_hi = hi;
  g->tclk_pending = 1;
  return NF_OK;
}

struct SolveOut {
  int iters = 0, converged = 0, flags = 0, sticky = 0;
  double rel_res = 0.0, true_rel_res = -1.0;
};

// Operator apply on the current iterate x_hat: leaves r_hat = b_hat - A x_hat,
// partials <r,M^-1 r>, <r,r>, <b,b> in SLOT_P3INIT and Kbar in the status.
// lo: also write the FP32 copies of m and r (mixed-precision solve).
int init_residual(nf_grid* g, const double* m, const double* r, float* lo = nullptr) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  if (g->dim == 3) {
    LCHK(g, launch3_row_flux(G, false, g->mix[0], g->mix[1], g->mix[2], m, r, -1, 1, lo, s));
    LCHK(g, launch3_ypass(G, false, 3, -1, g->mix[0], g->mix[1], g->mix[2], nullptr, -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_zdiv(G, false, 1, g->mix[0], g->mix[1], g->mix[2], g->qh, g->dh, g->rh, g->bh, 0, s));
    return NF_OK;
  }
  LCHK(g, launch_row_flux(G, g->mix[0], g->mix[1], m, r, -1, slot_ptr(g->part, SLOT_KBAR), 0.0, s, nullptr, nullptr,
                          lo));
  LCHK(g, launch_col_div(G, 1, g->mix[0], g->mix[1], g->qh, g->dh, g->rh, g->bh, 0, row_nwg(G), s));
  return NF_OK;
}

// Iterations it = 0, 1, ... of the PCG loop after its first update, queued in
// chunks; after each chunk the status is copied to pinned memory, and the host
// waits on the copy of the PREVIOUS chunk, so the GPU always has queued work.
// Kernels launched after the stop are no-ops.  f32 selects the FP32 passes of
// the mixed-precision inner solve.  `expect` sizes the first chunk.  On return
// the stream is synchronised and *fin holds the final status.
int pcg_loop(nf_grid* g, bool f32, const double* m, const double* r, int max_iter, double tol2, int expect,
             DevStatus* fin) {
  const Geo& G = f32 ? g->geo32 : g->geo;
  hipStream_t s = g->stream;
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  int rc = timed_reset(g);
  if (rc) return rc;
  int it = 0;
  int slot = 0, pending = -1;
  bool first_chunk = true, stopped = false;
  while (it < max_iter) {
    // up to one iteration short of the last solve's count, then one iteration per
    // chunk: the host polls one chunk behind, so at most about one chunk of
    // launches is queued past the stop (they return at once)
    int nk = first_chunk ? (expect > 3 ? expect - 1 : 2) : 1;
    if (!g->hst) nk = 8;  // synchronous polling: a few iterations per wait
    first_chunk = false;
    if (nk > max_iter - it) nk = max_iter - it;
    for (int k = 0; k < nk; ++k) {
      hipEvent_t e0, e1;
      if (g->dim == 3) {
        void* const* F = f32 ? g->mix32 : g->mix;
        LCHK(g, launch3_ypass(G, f32, 3, +1, F[0], F[1], F[2], nullptr, it, 1, tol2, -1.0, s));
        if ((rc = timed_events(g, NF_KERNEL_ROW_FLUX, it, &e0, &e1))) return rc;
        LCHK(g, launch3_row_flux(G, f32, F[0], F[1], F[2], f32 ? (const void*)g->lo : (const void*)m,
                                 f32 ? (const void*)(g->lo + 3 * n) : (const void*)r, it, 0, nullptr, s, e0, e1));
        LCHK(g, launch3_ypass(G, f32, 3, -1, F[0], F[1], F[2], nullptr, it, 0, 0.0, -1.0, s));
        if ((rc = timed_events(g, NF_KERNEL_COL_DIV, it, &e0, &e1))) return rc;
        LCHK(g, launch3_zdiv(G, f32, 0, F[0], F[1], F[2], f32 ? g->q32 : g->qh, f32 ? g->d32 : g->dh,
                             f32 ? g->r32 : g->rh, g->bh, it, s, e0, e1));
        if ((rc = timed_events(g, NF_KERNEL_COL_UPDATE, it, &e0, &e1))) return rc;
        LCHK(g, launch3_zupdate(G, f32, 0, f32 ? g->x32 : g->xh, f32 ? g->r32 : g->rh, f32 ? g->d32 : g->dh,
                                f32 ? g->q32 : g->qh, F[0], F[1], F[2], it + 1, max_iter, tol2, s, e0, e1));
        ++it;
        continue;
      }
      if ((rc = timed_events(g, NF_KERNEL_ROW_FLUX, it, &e0, &e1))) return rc;
      if (f32)
        LCHK(g, launch_row_flux32(G, g->mix32[0], g->mix32[1], g->lo, g->lo + 2 * n, it, tol2, s, e0, e1));
      else
        LCHK(g, launch_row_flux(G, g->mix[0], g->mix[1], m, r, it, nullptr, tol2, s, e0, e1));
      if ((rc = timed_events(g, NF_KERNEL_COL_DIV, it, &e0, &e1))) return rc;
      if (f32)
        LCHK(g, launch_col_div32(G, g->mix32[0], g->mix32[1], g->q32, g->d32, g->r32, it, s, e0, e1));
      else
        LCHK(g, launch_col_div(G, 0, g->mix[0], g->mix[1], g->qh, g->dh, g->rh, g->bh, it, 0, s, e0, e1));
      // the update of iteration it+1 does work iff the solver had not stopped before it
      if ((rc = timed_events(g, NF_KERNEL_COL_UPDATE, it, &e0, &e1))) return rc;
      if (f32)
        LCHK(g, launch_col_update32(G, g->x32, g->r32, g->d32, g->q32, g->mix32[0], g->mix32[1], it + 1, max_iter,
                                    tol2, s, e0, e1));
      else
        LCHK(g, launch_col_update(G, 0, g->xh, g->rh, g->dh, g->qh, g->mix[0], g->mix[1], it + 1, max_iter, tol2,
                                  s, e0, e1));
      ++it;
    }
    if (!g->hst) {
      // allocation-free solve (no pinned buffer, no events): wait for the chunk
      DevStatus cur;
      HIPCHK(g, hipMemcpyAsync(&cur, g->st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
      HIPCHK(g, hipStreamSynchronize(s));
      if (cur.conv_at != INT_MAX) break;
      continue;
    }
    HIPCHK(g, hipMemcpyAsync(&g->hst[slot], g->st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(g, hipEventRecord(g->ev[slot], s));
    if (pending >= 0) {
      HIPCHK(g, poll_event(g->ev[pending]));
      if (g->hst[pending].conv_at != INT_MAX) {
        stopped = true;
        break;
      }
    }
    pending = slot;
    slot ^= 1;
  }
  if (stopped) {
    // Once conv_at is set no later kernel of the loop writes the status, so the
    // copy that showed the stop is final: no need to wait for the queued tail
    // (no-op launches), and the caller's next launches queue behind it.
    *fin = g->hst[pending];
  } else {
    rc = read_status(g, fin);
    if (rc) return rc;
  }
  if ((rc = timed_collect(g, fin->conv_at))) return rc;
  return NF_OK;
}

// 3D: gradient of x_hat through the inverse z and y transforms into mix[0..2]
int grad_to_mixed3(nf_grid* g) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  LCHK(g, launch3_zinv(G, 2, g->xh, nullptr, g->mix[0], g->mix[1], g->mix[2], s));
  LCHK(g, launch3_ypass(G, false, 3, +1, g->mix[0], g->mix[1], g->mix[2], nullptr, -1, 0, 0.0, -1.0, s));
  return NF_OK;
}

// p = F^-1 x_hat
int write_p(nf_grid* g, double* p) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  if (g->dim == 3) {
    LCHK(g, launch3_zinv(G, 1, g->xh, g->mix[0], nullptr, nullptr, nullptr, s));
    LCHK(g, launch3_ypass(G, false, 1, +1, g->mix[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_row_c2r(G, g->mix[0], p, s));
    return NF_OK;
  }
  LCHK(g, launch_col_grad(G, g->xh, g->mix[0], nullptr, nullptr, s));
  LCHK(g, launch_row_c2r(G, g->mix[0], p, s));
  return NF_OK;
}

// Initial iterate x_hat from p (X_FROM_P), kept (X_FROM_XH) or zero, and its
// gradient in the mixed buffers for the first operator pass.
int prepare_iterate(nf_grid* g, XSource src, const double* p) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  if (g->dim == 3) {
    if (src == X_FROM_P) {
      LCHK(g, launch3_row_r2c(G, p, g->mix[0], 0, s));
      LCHK(g, launch3_ypass(G, false, 1, -1, g->mix[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, s));
      LCHK(g, launch3_zfwd(G, g->mix[0], g->xh, 1, s));
    } else if (src == X_ZERO) {
      LCHK(g, launch_zero_spec(G, g->xh, s));
    }
    return grad_to_mixed3(g);
  }
  if (src == X_FROM_P) {
    LCHK(g, launch_row_r2c(G, p, g->mix[0], nullptr, s));
    LCHK(g, launch_col_fwd(G, g->mix[0], g->xh, 1, g->mix[0], g->mix[1], s));
  } else {
    if (src == X_ZERO) LCHK(g, launch_zero_spec(G, g->xh, s));
    LCHK(g, launch_col_grad(G, g->xh, nullptr, g->mix[0], g->mix[1], s));
  }
  return NF_OK;
}

// Mixed-precision PCG (dtype NF_F32_REFINED): iterative refinement of
// A x = Pi S with x and the residual b - A x in FP64 and each correction
// A e = r solved by the same PCG in FP32 storage and arithmetic (FP64 inner
// products and scalars).  The solve stops on the FP64 residual, so rtol means
// what it means for the FP64 solver.  max_iter bounds the sum of the inner
// iterations; a correction that does not lower the FP64 residual ends the
// solve as not converged.  The decisions are taken on the device (status
// fields outer_done, itot, orr_prev); the host only repeats the passes until
// the status reports the end.
int pcg_refined(nf_grid* g, const double* m, const double* r, XSource src, const double* p, double rtol,
                int max_iter, bool want_true, SolveOut* out) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  LCHK(g, launch_status_reset(G, 0, s));
  int rc = prepare_iterate(g, src, p);
  if (rc) return rc;
  const double tol2 = rtol * rtol;
  DevStatus fin;
  for (int outer = 0;; ++outer) {
    // FP64 residual r = b - A x (and, on the first pass, the FP32 copies of m, r)
    rc = init_residual(g, m, r, outer == 0 ? g->lo : nullptr);
    if (rc) return rc;
    if (g->dim == 3)
      LCHK(g, launch3_zrefine_start(g->geo32, g->rh, g->xh, g->x32, g->r32, g->d32, g->mix32[0], g->mix32[1],
                                    g->mix32[2], tol2, g->inner_floor, max_iter, s));
    else
      LCHK(g, launch_col_refine_start(g->geo32, g->rh, g->xh, g->x32, g->r32, g->d32, g->mix32[0], g->mix32[1],
                                      tol2, g->inner_floor, max_iter, s));
    const int slot = outer < 3 ? outer : 3;
    rc = pcg_loop(g, true, m, r, max_iter, 1.0, g->last_inner[slot], &fin);
    if (rc) return rc;
    if (fin.outer_done) break;
    if (fin.iters > 0) g->last_inner[slot] = fin.iters;
    // x += ||r|| e and the gradient of the new x for the next residual
    if (g->dim == 3) {
      LCHK(g, launch3_zrefine_acc(G, g->xh, g->x32, g->mix[0], g->mix[1], g->mix[2], s));
      LCHK(g, launch3_ypass(G, false, 3, +1, g->mix[0], g->mix[1], g->mix[2], nullptr, -1, 0, 0.0, -1.0, s));
    } else {
      LCHK(g, launch_col_refine_acc(G, g->xh, g->x32, g->mix[0], g->mix[1], s));
    }
  }
  out->iters = fin.itot;
  out->converged = fin.converged;
  out->flags = fin.flags;
  out->sticky = fin.sticky;
  out->rel_res = fin.obb > 0.0 ? std::sqrt(fin.orr > 0.0 ? fin.orr : 0.0) / std::sqrt(fin.obb) : 0.0;
  // the stopping test is already on the FP64 residual of the returned iterate
  out->true_rel_res = (want_true && !(fin.flags & FLAG_INCOMPAT)) ? out->rel_res : -1.0;
  return NF_OK;
}

// PCG for A x = Pi S (Sec. 2.4) with b_hat already in place.
int pcg(nf_grid* g, const double* m, const double* r, XSource src, const double* p, double rtol, int max_iter,
        bool want_true, SolveOut* out) {
  if (g->dtype == NF_F32_REFINED) return pcg_refined(g, m, r, src, p, rtol, max_iter, want_true, out);
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  LCHK(g, launch_status_reset(G, 0, s));
  int rc = prepare_iterate(g, src, p);
  if (rc) return rc;
  rc = init_residual(g, m, r);
  if (rc) return rc;
  const double tol2 = rtol * rtol;
  if (g->dim == 3)
    LCHK(g, launch3_zupdate(G, false, 1, g->xh, g->rh, g->dh, g->qh, g->mix[0], g->mix[1], g->mix[2], 0, max_iter,
                            tol2, s));
  else
    LCHK(g, launch_col_update(G, 1, g->xh, g->rh, g->dh, g->qh, g->mix[0], g->mix[1], 0, max_iter, tol2, s));
  DevStatus fin;
  rc = pcg_loop(g, false, m, r, max_iter, tol2, g->last_iters, &fin);
  if (rc) return rc;
  if (!fin.converged && fin.conv_at == max_iter && max_iter > 0 && !(fin.flags & (FLAG_NONFINITE | FLAG_INCOMPAT))) {
    // stopped by max_iter: take the stopping test on the final residual here
    if (g->dim == 3)
      LCHK(g, launch3_copy_tot(G, SLOT_RR, 1, 11, s));
    else
      LCHK(g, launch_sum_slot(G, slot_ptr(g->part, SLOT_RR), 1, rr_nwg(G, false), 11, s));
    rc = read_status(g, &fin);
    if (rc) return rc;
    fin.rr[0] = fin.out[11];
    fin.converged = fin.out[11] <= tol2 * fin.bb ? 1 : 0;
  }
  out->iters = fin.iters;
  out->converged = fin.converged;
  out->flags = fin.flags;
  out->sticky = fin.sticky;
  const double rrf = fin.rr[0];
  out->rel_res = fin.bb > 0.0 ? std::sqrt(rrf > 0.0 ? rrf : 0.0) / std::sqrt(fin.bb) : 0.0;
  out->true_rel_res = -1.0;
  if (fin.iters > 0 || fin.converged) g->last_iters = fin.iters;
  if (want_true && !(fin.flags & FLAG_INCOMPAT)) {
    if (g->dim == 3) {
      rc = grad_to_mixed3(g);
      if (rc) return rc;
    } else {
      LCHK(g, launch_col_grad(G, g->xh, nullptr, g->mix[0], g->mix[1], s));
    }
    rc = init_residual(g, m, r);
    if (rc) return rc;
    if (g->dim == 3)
      LCHK(g, launch3_copy_tot(G, SLOT_P3INIT, 3, 0, s));
    else
      LCHK(g, launch_sum_slot(G, slot_ptr(g->part, SLOT_P3INIT), 3, col_nwg(G), 0, s));
    DevStatus t;
    rc = read_status(g, &t);
    if (rc) return rc;
    out->true_rel_res = t.out[2] > 0.0 ? std::sqrt(t.out[1] / t.out[2]) : 0.0;
  }
  return NF_OK;
}

int check_fields(nf_grid* g, std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs)
    if (!q) return fail(g, NF_EINVAL, "NULL field pointer");
  return NF_OK;
}

int check_params(nf_grid* g, const nf_params* prm, double dt) {
  if (!prm) return fail(g, NF_EINVAL, "NULL params");
  if (!(dt > 0.0)) return fail(g, NF_EINVAL, "dt must be > 0");
  if (!(prm->gamma > 0.0)) return fail(g, NF_EINVAL, "gamma must be > 0");
  if (!(prm->c2 >= 0.0)) return fail(g, NF_EINVAL, "c2 must be >= 0");
  if (!(prm->D2 >= 0.0)) return fail(g, NF_EINVAL, "D2 must be >= 0");
  return NF_OK;
}

int solve_status_code(nf_grid* g, const SolveOut& so) {
  if ((so.flags | so.sticky) & FLAG_NONFINITE)
    return fail(g, NF_ENONFINITE, "non-finite values (activation overflow: c^2 |grad p|^2 dt too large, or NaN input)");
  if (so.flags & FLAG_INCOMPAT) return fail(g, NF_EINCOMPAT, "S violates the solvability condition (sum S != 0)");
  if (!so.converged) return fail(g, NF_ENOTCONV, "PCG did not reach the tolerance within max_iter");
  return NF_OK;
}

// Step 2 of Algorithm 1 on the current x_hat: writes p = F^-1 x_hat, advances
// m in place, leaves the partials of Delta m (and of ||grad m_new||^2 if egm).
int split_update(nf_grid* g, const nf_params* prm, double dt, double* m, double* p, bool egm) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  if (g->dim == 3) {
    void* const* M = g->mix;
    const double D2dt = prm->D2 * dt;
    LCHK(g, launch3_zinv(G, 3, g->xh, M[0], M[1], M[2], M[3], s));
    LCHK(g, launch3_ypass(G, false, 4, +1, M[0], M[1], M[2], M[3], -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_row_split(G, M[0], M[1], M[2], M[3], m, p, prm->c2 * dt, prm->gamma, dt, std::exp(-dt), D2dt, s));
    LCHK(g, launch3_ypass(G, false, 3, -1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, D2dt, s));
    LCHK(g, launch3_zheat(G, M[0], M[1], M[2], D2dt, s));
    LCHK(g, launch3_ypass(G, false, 3, +1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_row_final(G, M[0], M[1], M[2], m, s));
    return NF_OK;
  }
  LCHK(g, launch_col_grad(G, g->xh, g->mix[0], g->mix[1], g->mix[2], s));
  LCHK(g, launch_row_split(G, g->mix[0], g->mix[1], g->mix[2], m, p, prm->c2 * dt, prm->gamma, dt, std::exp(-dt), s));
  LCHK(g, launch_col_heat(G, g->mix[0], g->mix[1], prm->D2 * dt, egm ? slot_ptr(g->part, SLOT_EGM) : nullptr, s));
  LCHK(g, launch_row_final(G, g->mix[0], g->mix[1], m, slot_ptr(g->part, SLOT_DM), s));
  return NF_OK;
}

// partials of Delta m of the last split update into status.out[8..9]
int dm_to_status(nf_grid* g) {
  if (g->dim == 3) {
    LCHK(g, launch3_copy_tot(g->geo, SLOT_DM, 2, 8, g->stream));
  } else {
    LCHK(g, launch_sum_slot(g->geo, slot_ptr(g->part, SLOT_DM), 2, row_nwg(g->geo), 8, g->stream));
  }
  return NF_OK;
}

// Pointwise energy terms of (m, p = F^-1 x_hat) into status.out[4..6]
int energy_pointwise(nf_grid* g, const nf_params* prm, const double* m, const double* r) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  LCHK(g, launch_col_grad(G, g->xh, nullptr, g->mix[0], g->mix[1], s));
  LCHK(g, launch_row_energy(G, g->mix[0], g->mix[1], m, r, prm->gamma, slot_ptr(g->part, SLOT_EPT), s));
  LCHK(g, launch_sum_slot(G, slot_ptr(g->part, SLOT_EPT), 3, row_nwg(G), 4, s));
  return NF_OK;
}

double assemble_energy(const nf_grid* g, const nf_params* prm, double gradm2_phys, const double* pt, double* terms) {
  const double n = (double)g->nx * g->ny * g->nz;
  const double hvol = g->lx * g->ly * g->lz / n;  // lz = 1, nz = 1 in 2D
  const double e_diff = 0.5 * prm->D2 * hvol * gradm2_phys;
  const double e_relax = hvol * pt[2] / (2.0 * prm->gamma);
  const double e_act = 0.5 * prm->c2 * hvol * pt[1];
  const double e_flow = 0.5 * prm->c2 * hvol * pt[0];
  const double tot = e_diff + e_relax + e_act + e_flow;
  if (terms) {
    terms[0] = tot;
    terms[1] = e_diff;
    terms[2] = e_relax;
    terms[3] = e_act;
    terms[4] = e_flow;
  }
  return tot;
}

// 3D energy of (m, p = F^-1 x_hat): grad p through the inverse z and y passes
// and three row passes into physical scratch fields (the PCG vectors r, d, q,
// free between solves), the pointwise terms, then the three spectra of m into
// the same scratch fields and their Parseval gradient norm.  Returns E_h and
// fills terms (5 entries) if non-NULL.
int energy3(nf_grid* g, const nf_params* prm, const double* m, const double* r, double* e_out, double* terms) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  double* P[3] = {(double*)g->rh, (double*)g->dh, (double*)g->qh};
  void* const* M = g->mix;
  LCHK(g, launch3_zinv(G, 2, g->xh, nullptr, M[0], M[1], M[2], s));
  LCHK(g, launch3_ypass(G, false, 3, +1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, -1.0, s));
  for (int c = 0; c < 3; ++c) LCHK(g, launch3_row_c2r(G, M[c], P[c], s));
  LCHK(g, launch3_energy_pt(G, m, r, P[0], P[1], P[2], prm->gamma, s));
  LCHK(g, launch3_copy_tot(G, SLOT_EPT, 3, 4, s));
  for (int c = 0; c < 3; ++c) {
    LCHK(g, launch3_row_r2c(G, m + c * n, M[0], 0, s));
    LCHK(g, launch3_ypass(G, false, 1, -1, M[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_zfwd(G, M[0], P[c], 0, s));
  }
  LCHK(g, launch3_spec_gradnorm(G, P[0], P[1], P[2], s));
  LCHK(g, launch3_copy_tot(G, SLOT_EGM, 1, 3, s));
  DevStatus fin;
  int rc = read_status(g, &fin);
  if (rc) return rc;
  const double e = assemble_energy(g, prm, fin.out[3] / (double)n, &fin.out[4], terms);
  if (e_out) *e_out = e;
  return NF_OK;
}

// end of nf_step_adjoint: wait, report the adjoint solve, map its outcome to a code
int adjoint_epilogue(nf_grid* g, const SolveOut& so, nf_solve_info* info) {
  DevStatus fin;
  int rc = read_status(g, &fin);
  if (rc) return rc;
  if (info) {
    info->iters = so.iters;
    info->converged = so.converged;
    info->rel_res = so.rel_res;
    info->true_rel_res = so.true_rel_res;
  }
  if ((so.flags | fin.flags) & FLAG_NONFINITE) return fail(g, NF_ENONFINITE, "non-finite values in the adjoint step");
  if (!so.converged) return fail(g, NF_ENOTCONV, "adjoint PCG did not reach the tolerance within max_iter");
  return NF_OK;
}

// 3D: the gradient of a physical field f as three physical fields (transforms
// of f into spec, its gradient back through the inverse passes; mix[0..2] are
// intermediates, out may include spec)
int grad_phys3(nf_grid* g, const double* f, void* spec, double* const* out) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  void* const* M = g->mix;
  LCHK(g, launch3_row_r2c(G, f, M[0], 0, s));
  LCHK(g, launch3_ypass(G, false, 1, -1, M[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, s));
  LCHK(g, launch3_zfwd(G, M[0], spec, 0, s));
  LCHK(g, launch3_zinv(G, 2, spec, nullptr, M[0], M[1], M[2], s));
  LCHK(g, launch3_ypass(G, false, 3, +1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, -1.0, s));
  for (int c = 0; c < 3; ++c) LCHK(g, launch3_row_c2r(G, M[c], out[c], s));
  return NF_OK;
}

// Adjoint of one 3D step: the 2D sequence with a third component, the pointwise
// parts as grid-stride passes over physical fields.
int step_adjoint3(nf_grid* g, const nf_params* prm, double dt, const double* m, const double* p, const double* r,
                  const double* lam_next, double* lam_k, double* grad_r, double* grad_S, double* mu, double rtol,
                  int max_iter, bool want_true, SolveOut* so) {
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  void* const* M = g->mix;
  const double D2dt = prm->D2 * dt;
  // diffusion stage (H symmetric): lam_k = H lam_next through the passes of the
  // split update with activation and relaxation switched off (c^2 = 0, gamma = 1
  // with factor 1) and a zero pressure (its scratch output goes to qh)
  if (lam_k != lam_next)
    HIPCHK(g, hipMemcpyAsync(lam_k, lam_next, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  LCHK(g, launch_zero_doubles((double*)g->xh, n, s));
  LCHK(g, launch3_zinv(G, 3, g->xh, M[0], M[1], M[2], M[3], s));
  LCHK(g, launch3_ypass(G, false, 4, +1, M[0], M[1], M[2], M[3], -1, 0, 0.0, -1.0, s));
  LCHK(g, launch3_row_split(G, M[0], M[1], M[2], M[3], lam_k, (double*)g->qh, 0.0, 1.0, dt, 1.0, D2dt, s));
  LCHK(g, launch3_ypass(G, false, 3, -1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, D2dt, s));
  LCHK(g, launch3_zheat(G, M[0], M[1], M[2], D2dt, s));
  LCHK(g, launch3_ypass(G, false, 3, +1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, -1.0, s));
  LCHK(g, launch3_row_final(G, M[0], M[1], M[2], lam_k, s));
  // grad p^k, then the reverse of relaxation and activation: lam_k <- lam_m, Gp <- lam_g
  double* Gp[3] = {(double*)g->rh, (double*)g->dh, (double*)g->qh};
  int rc = grad_phys3(g, p, g->bh, Gp);
  if (rc) return rc;
  LCHK(g, launch3_adj1(G, m, lam_k, Gp[0], Gp[1], Gp[2], prm->c2 * dt, prm->gamma, dt, std::exp(-dt), s));
  // adjoint pressure: A mu = Pi G^T lam_g, b_hat = -i xi_tilde . F(lam_g)
  void* F[3] = {g->xh, M[1], M[2]};
  for (int c = 0; c < 3; ++c) {
    LCHK(g, launch3_row_r2c(G, Gp[c], M[0], 0, s));
    LCHK(g, launch3_ypass(G, false, 1, -1, M[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_zfwd(G, M[0], F[c], 0, s));
  }
  LCHK(g, launch3_spec_divrhs(G, F[0], F[1], F[2], g->bh, s));
  // S does not enter: the compatibility totals of the solve's check are cleared
  LCHK(g, launch_zero_doubles(G.tot + SLOT_SCHK * SLOT_K, 2, s));
  rc = pcg(g, m, r, X_FROM_P, mu, rtol, max_iter, want_true, so);
  if (rc) return rc;
  // mu, grad mu (rh, dh, qh) and grad p^k again (xh, mix[3], bh)
  rc = write_p(g, mu);
  if (rc) return rc;
  LCHK(g, launch3_zinv(G, 2, g->xh, nullptr, M[0], M[1], M[2], s));
  LCHK(g, launch3_ypass(G, false, 3, +1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, -1.0, s));
  double* U[3] = {(double*)g->rh, (double*)g->dh, (double*)g->qh};
  for (int c = 0; c < 3; ++c) LCHK(g, launch3_row_c2r(G, M[c], U[c], s));
  double* P[3] = {(double*)g->xh, (double*)M[3], (double*)g->bh};
  rc = grad_phys3(g, p, g->bh, P);
  if (rc) return rc;
  LCHK(g, launch3_adj2(G, m, mu, U[0], U[1], U[2], P[0], P[1], P[2], lam_k, grad_r, grad_S, s));
  return NF_OK;
}

}  // namespace

extern "C" {

const char* nf_version(void) { return kVersion; }

const char* nf_last_error(const nf_grid* g) { return g ? g->err.c_str() : create_err.c_str(); }

int nf_set_stream(nf_grid* g, void* stream) {
  if (!g) return NF_EINVAL;
  // A solve returns with its last no-op launches still queued; they must run
  // before work of the handle on another stream touches the workspace.
  if ((hipStream_t)stream != g->stream) HIPCHK(g, hipStreamSynchronize(g->stream));
  g->stream = (hipStream_t)stream;
  return NF_OK;
}

int nf_create_grid(nf_grid** out, int ndim, const int64_t n[3], const double L[3], int dtype, void* stream) {
  if (!out) return NF_EINVAL;
  *out = nullptr;
  if ((ndim != 2 && ndim != 3) || !n || !L || (dtype != NF_F64 && dtype != NF_F32_REFINED)) return NF_EINVAL;
  if (ndim == 2 && (!is_2d_size(n[0]) || !is_2d_size(n[1]))) return NF_EINVAL;
  if (ndim == 3)
    for (int c = 0; c < 3; ++c)
      if (!is_pow2_in_range(n[c]) || n[c] > 1024) return NF_EINVAL;
  for (int c = 0; c < ndim; ++c)
    if (!(L[c] > 0.0)) return NF_EINVAL;
  nf_grid* g = new nf_grid();
  g->dim = ndim;
  // default floor of the FP32 corrections, measured per dimension: 3e-6 saves
  // a correction per solve on 2D grids; on 256^3 1e-5 was 3% faster
  g->inner_floor = ndim == 3 ? 1e-5 : 3e-6;
  g->nx = (int)n[0];
  g->ny = (int)n[1];
  g->nz = ndim == 3 ? (int)n[2] : 1;
  g->h = g->nx / 2;
  g->lx = L[0];
  g->ly = L[1];
  g->lz = ndim == 3 ? L[2] : 1.0;
  g->stream = (hipStream_t)stream;
  g->dtype = dtype;
  int rc = NF_OK;
  create_err.clear();
  hipError_t herr = hipSuccess;
  auto bail = [&](int code, const char* what) {
    create_err = std::string(what) + (herr != hipSuccess ? std::string(": ") + hipGetErrorString(herr) : "");
    nf_destroy_grid(g);
    return code;
  };
#define CREATE_CHK(expr, code)                          \
  do {                                                  \
    if ((herr = (expr)) != hipSuccess) return bail(code, #expr); \
  } while (0)
  CREATE_CHK(hipGetDevice(&g->device), NF_EDEVICE);
  // twiddle table length: the least common multiple of the axis lengths, so
  // that every stage's angle unit is a whole number of table steps
  int64_t twl = g->nx / gcd64(g->nx, g->ny) * g->ny;
  twl = twl / gcd64(twl, g->nz) * g->nz;
  const int twn = (int)twl;
  g->twn = twn;
  const size_t npts = (size_t)g->nx * g->ny * g->nz;
  const size_t spec_bytes = (size_t)g->h * g->ny * g->nz * 2 * sizeof(double);
  const int nmix = ndim == 3 ? 4 : 3;
  void** bufs[] = {&g->xh, &g->rh, &g->dh, &g->qh, &g->bh};
  for (void** b : bufs) CREATE_CHK(hipMalloc(b, spec_bytes), NF_ENOMEM);
  for (int i = 0; i < nmix; ++i) CREATE_CHK(hipMalloc(&g->mix[i], spec_bytes), NF_ENOMEM);
  CREATE_CHK(hipMalloc(&g->tw, (size_t)twn * 2 * sizeof(double)), NF_ENOMEM);
  // partial sums: 2D keeps MAX_WG per array; 3D sizes them to the largest pass.
  // The reduced totals follow them.
  int pstride = MAX_WG;
  if (ndim == 3) {
    Geo tmp{};
    tmp.nx = g->nx;
    tmp.ny = g->ny;
    tmp.nz = g->nz;
    tmp.h = g->h;
    pstride = nwg3_row(tmp);
    if (nwg3_y(tmp) > pstride) pstride = nwg3_y(tmp);
    if (nwg3_z(tmp) > pstride) pstride = nwg3_z(tmp);
  }
  const size_t part_doubles = (size_t)NSLOTS * SLOT_K * pstride + NSLOTS * SLOT_K;
  CREATE_CHK(hipMalloc((void**)&g->part, part_doubles * sizeof(double)), NF_ENOMEM);
  CREATE_CHK(hipMalloc((void**)&g->st, sizeof(DevStatus)), NF_ENOMEM);
  g->st_own = g->st;
  CREATE_CHK(hipHostMalloc((void**)&g->hst, 2 * sizeof(DevStatus), hipHostMallocDefault), NF_ENOMEM);
  for (int i = 0; i < 2; ++i) CREATE_CHK(hipEventCreateWithFlags(&g->ev[i], hipEventDisableTiming), NF_EDEVICE);
  {
    double* h = new double[2 * (size_t)twn];
    make_twiddles(twn, h);
    herr = hipMemcpy(g->tw, h, (size_t)twn * 2 * sizeof(double), hipMemcpyHostToDevice);
    delete[] h;
    if (herr != hipSuccess) return bail(NF_EDEVICE, "hipMemcpy(twiddles)");
  }
  CREATE_CHK(hipMemset(g->part, 0, part_doubles * sizeof(double)), NF_EDEVICE);
  CREATE_CHK(hipMemset(g->st, 0, sizeof(DevStatus)), NF_EDEVICE);
  CREATE_CHK(hipMemset(g->xh, 0, spec_bytes), NF_EDEVICE);
  if (dtype == NF_F32_REFINED) {
    const size_t spec32 = spec_bytes / 2;
    void** b32[] = {&g->x32, &g->r32, &g->d32, &g->q32};
    for (void** b : b32) CREATE_CHK(hipMalloc(b, spec32), NF_ENOMEM);
    for (int i = 0; i < ndim; ++i) CREATE_CHK(hipMalloc(&g->mix32[i], spec32), NF_ENOMEM);
    CREATE_CHK(hipMalloc((void**)&g->lo, (size_t)(ndim + 1) * npts * sizeof(float)), NF_ENOMEM);
    CREATE_CHK(hipMalloc(&g->tw32, (size_t)twn * 2 * sizeof(float)), NF_ENOMEM);
    float* h = new float[2 * (size_t)twn];
    make_twiddles(twn, h);
    herr = hipMemcpy(g->tw32, h, (size_t)twn * 2 * sizeof(float), hipMemcpyHostToDevice);
    delete[] h;
    if (herr != hipSuccess) return bail(NF_EDEVICE, "hipMemcpy(twiddles32)");
  }
#undef CREATE_CHK
  Geo& G = g->geo;
  G.nx = g->nx;
  G.ny = g->ny;
  G.h = g->h;
  G.twn = g->twn;
  G.lx = g->lx;
  G.ly = g->ly;
  G.inv_n = 1.0 / ((double)g->nx * (double)g->ny * (double)g->nz);
  G.tw = g->tw;
  G.st = g->st;
  G.part = g->part;
  G.nz = g->nz;
  G.lz = g->lz;
  G.pstride = pstride;
  G.tot = g->part + (size_t)NSLOTS * SLOT_K * pstride;
  G.tclk = nullptr;
  G.tkind = -1;
  for (int k = 0; k < 2; ++k) G.var_flux[k] = G.var_div[k] = G.var_upd[k] = VAR_DEFAULT;
  g->geo32 = G;
  g->geo32.tw = g->tw32;
  // tile variants of the PCG loop for this grid shape (tuned once per process)
  rc = nf::tune_handle(g);
  if (rc != NF_OK) {
    create_err = g->err;
    nf_destroy_grid(g);
    return rc;
  }
  *out = g;
  return rc;
}

int nf_set_inner_tolerance(nf_grid* g, double floor_rtol) {
  if (!g) return NF_EINVAL;
  if (!(floor_rtol > 0.0 && floor_rtol < 0.5)) return fail(g, NF_EINVAL, "inner tolerance must lie in (0, 0.5)");
  g->inner_floor = floor_rtol;
  return NF_OK;
}

int nf_time_kernel(nf_grid* g, int which) {
  if (!g || which < -1 || which > NF_KERNEL_COL_UPDATE) return NF_EINVAL;
  if (g->tclk_pending) {
    // stamps of the previous setting still in flight: let the copy land, drop them
    HIPCHK(g, hipEventSynchronize(g->tclk_ev));
    g->tclk_pending = 0;
  }
  if (which >= 0 && !g->tclk) {
    const size_t nb = 2 * sizeof(unsigned long long) * TCLK_CAP * TCLK_W;
    HIPCHK(g, hipMalloc((void**)&g->tclk, nb));
    HIPCHK(g, hipHostMalloc((void**)&g->htclk, nb, hipHostMallocDefault));
    HIPCHK(g, hipEventCreateWithFlags(&g->tclk_ev, hipEventDisableTiming));
    int khz = 0;
    HIPCHK(g, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device));
    if (khz <= 0) return fail(g, NF_EDEVICE, "device wall-clock rate unavailable");
    g->wall_khz = (double)khz;
  }
  g->timed = which;
  g->geo.tclk = g->geo32.tclk = which >= 0 ? g->tclk : nullptr;
  g->geo.tkind = g->geo32.tkind = which;
  g->timed_ms = 0.0;
  g->timed_count = 0;
  return NF_OK;
}

int nf_time_kernel_read(nf_grid* g, double* total_ms, int64_t* count) {
  if (!g || !total_ms || !count) return NF_EINVAL;
  const int rc = timed_flush(g);
  if (rc) return rc;
  *total_ms = g->timed_ms;
  *count = g->timed_count;
  return NF_OK;
}

int nf_destroy_grid(nf_grid* g) {
  if (!g) return NF_OK;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  else (void)hipDeviceSynchronize();
  void* bufs[] = {g->xh,     g->rh,     g->dh,   g->qh,  g->bh,  g->mix[0],  g->mix[1],  g->mix[2],
                  g->mix[3], g->tw,     g->part, g->st_own, g->x32, g->r32, g->d32, g->q32,
                  g->mix32[0], g->mix32[1], g->mix32[2], g->lo, g->tw32};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (g->hst) (void)hipHostFree(g->hst);
  if (g->tclk) (void)hipFree(g->tclk);
  if (g->htclk) (void)hipHostFree(g->htclk);
  if (g->tclk_ev) (void)hipEventDestroy(g->tclk_ev);
  for (int i = 0; i < 2; ++i)
    if (g->ev[i]) (void)hipEventDestroy(g->ev[i]);
  delete g;
  return NF_OK;
}

int nf_transform_forward(nf_grid* g, const double* f, double* out) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  int rc = check_fields(g, {f, out});
  if (rc) return rc;
  if (g->dim == 3) {
    LCHK(g, launch3_row_r2c(g->geo, f, g->mix[0], 0, g->stream));
    LCHK(g, launch3_ypass(g->geo, false, 1, -1, g->mix[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, g->stream));
    LCHK(g, launch3_zfwd(g->geo, g->mix[0], out, 0, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return NF_OK;
  }
  LCHK(g, launch_row_r2c(g->geo, f, g->mix[0], nullptr, g->stream));
  LCHK(g, launch_col_fwd(g->geo, g->mix[0], out, 2, nullptr, nullptr, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return NF_OK;
}

int nf_transform_inverse(nf_grid* g, const double* spec, double* f) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  int rc = check_fields(g, {spec, f});
  if (rc) return rc;
  if (g->dim == 3) {
    LCHK(g, launch3_zinv(g->geo, 1, spec, g->mix[0], nullptr, nullptr, nullptr, g->stream));
    LCHK(g, launch3_ypass(g->geo, false, 1, +1, g->mix[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, g->stream));
    LCHK(g, launch3_row_c2r(g->geo, g->mix[0], f, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return NF_OK;
  }
  LCHK(g, launch_col_grad(g->geo, spec, g->mix[0], nullptr, nullptr, g->stream));
  LCHK(g, launch_row_c2r(g->geo, g->mix[0], f, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return NF_OK;
}

int nf_gradient(nf_grid* g, const double* f, double* grad) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  int rc = check_fields(g, {f, grad});
  if (rc) return rc;
  if (g->dim != 2) return fail(g, NF_EINVAL, "nf_gradient is available for 2D grids only");
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  const size_t n = (size_t)g->nx * g->ny;
  LCHK(g, launch_row_r2c(G, f, g->mix[0], nullptr, s));
  LCHK(g, launch_col_fwd(G, g->mix[0], g->qh, 1, g->mix[1], g->mix[2], s));
  LCHK(g, launch_row_c2r(G, g->mix[1], grad, s));
  LCHK(g, launch_row_c2r(G, g->mix[2], grad + n, s));
  HIPCHK(g, hipStreamSynchronize(s));
  return NF_OK;
}

int nf_apply_operator(nf_grid* g, const double* m, const double* r, const double* p, double* out) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  int rc = check_fields(g, {m, r, p, out});
  if (rc) return rc;
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  LCHK(g, launch_status_reset(G, 1, s));
  if (g->dim == 3) {
    rc = prepare_iterate(g, X_FROM_P, p);
    if (rc) return rc;
    void* const* M = g->mix;
    LCHK(g, launch3_row_flux(G, false, M[0], M[1], M[2], m, r, -1, 0, nullptr, s));
    LCHK(g, launch3_ypass(G, false, 3, -1, M[0], M[1], M[2], nullptr, -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_zdiv(G, false, 0, M[0], M[1], M[2], g->qh, g->xh, g->xh, g->bh, 0, s));
    LCHK(g, launch3_zinv(G, 1, g->qh, M[0], nullptr, nullptr, nullptr, s));
    LCHK(g, launch3_ypass(G, false, 1, +1, M[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, s));
    LCHK(g, launch3_row_c2r(G, M[0], out, s));
    HIPCHK(g, hipStreamSynchronize(s));
    return NF_OK;
  }
  LCHK(g, launch_row_r2c(G, p, g->mix[0], nullptr, s));
  LCHK(g, launch_col_fwd(G, g->mix[0], g->xh, 1, g->mix[0], g->mix[1], s));
  LCHK(g, launch_row_flux(G, g->mix[0], g->mix[1], m, r, -1, nullptr, 0.0, s));
  LCHK(g, launch_col_div(G, 0, g->mix[0], g->mix[1], g->qh, g->xh, g->xh, g->bh, 0, 0, s));
  LCHK(g, launch_col_grad(G, g->qh, g->mix[0], nullptr, nullptr, s));
  LCHK(g, launch_row_c2r(G, g->mix[0], out, s));
  HIPCHK(g, hipStreamSynchronize(s));
  return NF_OK;
}

int nf_pressure_solve(nf_grid* g, const double* m, const double* r, const double* S, double* p, double rtol,
                      int max_iter, nf_solve_info* info) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  LCHK(g, launch_status_reset(g->geo, 1, g->stream));
  int rc = check_fields(g, {m, r, S, p});
  if (rc) return rc;
  if (!(rtol >= 0.0) || max_iter < 0) return fail(g, NF_EINVAL, "rtol must be >= 0 and max_iter >= 0");
  rc = compute_rhs(g, S);
  if (rc) return rc;
  SolveOut so;
  rc = pcg(g, m, r, X_FROM_P, p, rtol, max_iter, info != nullptr, &so);
  if (rc) return rc;
  if (so.flags & FLAG_INCOMPAT) return solve_status_code(g, so);
  rc = write_p(g, p);
  if (rc) return rc;
  if (info) {
    info->iters = so.iters;
    info->converged = so.converged;
    info->rel_res = so.rel_res;
    info->true_rel_res = so.true_rel_res;
  }
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return solve_status_code(g, so);
}

int nf_pressure_solve_noalloc(const int64_t n[2], const double L[2], void* stream, const double* m, const double* r,
                              const double* S, double* p, double rtol, int max_iter, nf_solve_info* info) {
  create_err.clear();
  auto reject = [](const char* msg) {
    create_err = msg;
    return NF_EINVAL;
  };
  // every argument is checked before the device is touched
  if (!n || !L) return reject("NULL grid size or box length");
  const int64_t nx = n[0], ny = n[1];
  if (!is_pow2_in_range(nx) || !is_pow2_in_range(ny))
    return reject("allocation-free solve: Nx and Ny must be powers of two in [8, 4096]");
  if (nx * ny > NOALLOC_MAX_POINTS)
    return reject("allocation-free solve: Nx * Ny exceeds the fixed workspace (at most 65536 grid points)");
  if (!(L[0] > 0.0) || !(L[1] > 0.0)) return reject("box lengths must be > 0");
  if (!m || !r || !S || !p) return reject("NULL field pointer");
  if (!(rtol >= 0.0) || max_iter < 0) return reject("rtol must be >= 0 and max_iter >= 0");
  void* base = nullptr;
  hipError_t herr = noalloc_scratch(&base);
  if (herr != hipSuccess) {
    create_err = std::string("device address of the fixed workspace: ") + hipGetErrorString(herr);
    return NF_EDEVICE;
  }
  // A handle on the stack whose workspace is carved from the fixed array: no
  // pinned status buffer and no events (the PCG loop then polls synchronously).
  nf_grid G;
  nf_grid* g = &G;
  g->dim = 2;
  g->nx = (int)nx;
  g->ny = (int)ny;
  g->nz = 1;
  g->h = g->nx / 2;
  g->lx = L[0];
  g->ly = L[1];
  g->stream = (hipStream_t)stream;
  g->dtype = NF_F64;
  g->twn = (int)(nx > ny ? nx : ny);  // lcm of two powers of two
  (void)hipGetDevice(&g->device);
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    void* q = (char*)base + off;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  const size_t spec_bytes = (size_t)g->h * g->ny * 2 * sizeof(double);
  void** spec[] = {&g->xh, &g->rh, &g->dh, &g->qh, &g->bh, &g->mix[0], &g->mix[1], &g->mix[2]};
  for (void** b : spec) *b = carve(spec_bytes);
  const size_t part_doubles = (size_t)NSLOTS * SLOT_K * MAX_WG + NSLOTS * SLOT_K;
  g->part = (double*)carve(part_doubles * sizeof(double));
  g->st = (DevStatus*)carve(sizeof(DevStatus));
  g->tw = carve((size_t)g->twn * 2 * sizeof(double));
  if (off > NOALLOC_SCRATCH_BYTES) return reject("allocation-free solve: workspace layout exceeds the fixed array");
  // twiddles from the same long-double table as nf_create_grid (host copy per thread)
  static thread_local double twh[2 * NOALLOC_MAX_TWIDDLES];
  make_twiddles(g->twn, twh);
  herr = hipMemcpyAsync(g->tw, twh, (size_t)g->twn * 2 * sizeof(double), hipMemcpyHostToDevice, g->stream);
  if (herr != hipSuccess) {
    create_err = std::string("twiddle upload: ") + hipGetErrorString(herr);
    return NF_EDEVICE;
  }
  Geo& Gg = g->geo;
  Gg.nx = g->nx;
  Gg.ny = g->ny;
  Gg.h = g->h;
  Gg.twn = g->twn;
  Gg.lx = g->lx;
  Gg.ly = g->ly;
  Gg.inv_n = 1.0 / ((double)g->nx * (double)g->ny);
  Gg.tw = g->tw;
  Gg.st = g->st;
  Gg.part = g->part;
  Gg.nz = 1;
  Gg.lz = 1.0;
  Gg.pstride = MAX_WG;
  Gg.tot = g->part + (size_t)NSLOTS * SLOT_K * MAX_WG;
  Gg.tclk = nullptr;
  Gg.tkind = -1;
  // the tile variants tuned for this shape by an earlier nf_create_grid, if any
  int var[3] = {VAR_DEFAULT, VAR_DEFAULT, VAR_DEFAULT};
  (void)nf::tune_lookup(g->device, g->nx, g->ny, false, var);
  for (int k = 0; k < 2; ++k) {
    Gg.var_flux[k] = var[0];
    Gg.var_div[k] = var[1];
    Gg.var_upd[k] = var[2];
  }
  // the array keeps the previous call's contents: clear the partial sums (a
  // fill kernel, no memset node) before the solve resets the status
  int rc = check_launch(g, launch_zero_doubles(g->part, part_doubles, g->stream), "clear workspace");
  if (rc == NF_OK) rc = nf_pressure_solve(g, m, r, S, p, rtol, max_iter, info);
  if (rc != NF_OK) create_err = g->err;
  return rc;
}

int nf_step(nf_grid* g, const nf_params* prm, double dt, double* m, double* p, const double* r, const double* S,
            double rtol, int max_iter, nf_step_info* info) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  LCHK(g, launch_status_reset(g->geo, 1, g->stream));
  int rc = check_fields(g, {m, p, r, S});
  if (rc) return rc;
  rc = check_params(g, prm, dt);
  if (rc) return rc;
  if (!(rtol >= 0.0) || max_iter < 0) return fail(g, NF_EINVAL, "rtol must be >= 0 and max_iter >= 0");
  rc = compute_rhs(g, S);
  if (rc) return rc;
  SolveOut so;
  rc = pcg(g, m, r, X_FROM_P, p, rtol, max_iter, false, &so);
  if (rc) return rc;
  if (so.flags & FLAG_INCOMPAT) return solve_status_code(g, so);
  // E_h(m^k) with p[m^k]: the spectral solution is still in x_hat (as in nf_run)
  double e_step = NAN;
  if (g->step_energy) {
    if (g->dim == 3) {
      rc = energy3(g, prm, m, r, &e_step, nullptr);
      if (rc) return rc;
    } else {
      const Geo& G = g->geo;
      const size_t n = (size_t)g->nx * g->ny;
      LCHK(g, launch_row_r2c(G, m, g->mix[0], nullptr, g->stream));
      LCHK(g, launch_row_r2c(G, m + n, g->mix[1], nullptr, g->stream));
      LCHK(g, launch_col_gradnorm(G, g->mix[0], g->mix[1], slot_ptr(g->part, SLOT_EGM), g->stream));
      LCHK(g, launch_sum_slot(G, slot_ptr(g->part, SLOT_EGM), 1, col_nwg(G), 3, g->stream));
      rc = energy_pointwise(g, prm, m, r);
      if (rc) return rc;
      DevStatus t;
      rc = read_status(g, &t);
      if (rc) return rc;
      e_step = assemble_energy(g, prm, t.out[3] / (double)n, &t.out[4], nullptr);
    }
  }
  rc = split_update(g, prm, dt, m, p, false);
  if (rc) return rc;
  rc = dm_to_status(g);
  if (rc) return rc;
  DevStatus fin;
  rc = read_status(g, &fin);
  if (rc) return rc;
  if (info) {
    info->solve.iters = so.iters;
    info->solve.converged = so.converged;
    info->solve.rel_res = so.rel_res;
    info->solve.true_rel_res = so.true_rel_res;
    info->dm_rel = fin.out[9] > 0.0 ? std::sqrt(fin.out[8] / fin.out[9]) / dt : 0.0;
    info->energy = e_step;
    info->energy_valid = g->step_energy ? 1 : 0;
  }
  if (fin.sticky & FLAG_NONFINITE)
    return fail(g, NF_ENONFINITE, "activation overflow: c^2 |grad p|^2 dt too large for the time step");
  return solve_status_code(g, so);
}

int nf_set_step_energy(nf_grid* g, int on) {
  if (!g) return NF_EINVAL;
  g->step_energy = on ? 1 : 0;
  return NF_OK;
}

int nf_step_adjoint(nf_grid* g, const nf_params* prm, double dt, const double* m, const double* p, const double* r,
                    const double* S, const double* lam_next, double* lam_k, double* grad_r, double* grad_S,
                    double* mu, double rtol, int max_iter, nf_solve_info* info) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  int rc = check_fields(g, {m, p, r, S, lam_next, lam_k, grad_r, grad_S, mu});
  if (rc) return rc;
  rc = check_params(g, prm, dt);
  if (rc) return rc;
  if (!(rtol >= 0.0) || max_iter < 0) return fail(g, NF_EINVAL, "rtol must be >= 0 and max_iter >= 0");
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  const size_t n = (size_t)g->nx * g->ny;
  LCHK(g, launch_status_reset(G, 1, s));
  if (g->dim == 3) {
    SolveOut so3;
    rc = step_adjoint3(g, prm, dt, m, p, r, lam_next, lam_k, grad_r, grad_S, mu, rtol, max_iter, info != nullptr, &so3);
    if (rc) return rc;
    return adjoint_epilogue(g, so3, info);
  }
  // adjoint through the diffusion stage: H lam (H symmetric)
  LCHK(g, launch_row_r2c(G, lam_next, g->mix[0], nullptr, s));
  LCHK(g, launch_row_r2c(G, lam_next + n, g->mix[1], nullptr, s));
  LCHK(g, launch_col_heat(G, g->mix[0], g->mix[1], prm->D2 * dt, nullptr, s));
  // grad p^k
  LCHK(g, launch_row_r2c(G, p, g->mix[2], nullptr, s));
  LCHK(g, launch_col_fwd(G, g->mix[2], g->dh, 1, g->mix[2], g->qh, s));
  // through relaxation and activation: lam_m -> lam_k, lam_g -> mix[0..1]
  LCHK(g, launch_row_adj1(G, g->mix[0], g->mix[1], g->mix[2], g->qh, m, lam_k, prm->c2 * dt, prm->gamma, dt,
                          std::exp(-dt), s));
  // adjoint pressure: A mu = Pi G^T lam_g
  LCHK(g, launch_col_divrhs(G, g->mix[0], g->mix[1], g->bh, s));
  LCHK(g, launch_zero_doubles(slot_ptr(g->part, SLOT_SCHK), 2 * (size_t)MAX_WG, s));
  SolveOut so;
  rc = pcg(g, m, r, X_FROM_P, mu, rtol, max_iter, info != nullptr, &so);
  if (rc) return rc;
  // gradients
  LCHK(g, launch_col_grad(G, g->xh, g->mix[0], g->mix[1], g->mix[2], s));
  LCHK(g, launch_row_c2r(G, g->mix[0], mu, s));
  LCHK(g, launch_row_r2c(G, p, g->rh, nullptr, s));
  LCHK(g, launch_col_fwd(G, g->rh, g->dh, 1, g->rh, g->qh, s));
  LCHK(g, launch_row_adj2(G, g->mix[1], g->mix[2], g->rh, g->qh, m, mu, lam_k, grad_r, grad_S, s));
  return adjoint_epilogue(g, so, info);
}

int nf_energy(nf_grid* g, const nf_params* prm, const double* m, const double* p, const double* r, const double* S,
              double out[5]) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  LCHK(g, launch_status_reset(g->geo, 1, g->stream));
  int rc = check_fields(g, {m, r, S, out});
  if (rc) return rc;
  if (!prm || !(prm->gamma > 0.0)) return fail(g, NF_EINVAL, "invalid params");
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  if (p) {
    if (g->dim == 3) {
      LCHK(g, launch3_row_r2c(G, p, g->mix[0], 0, s));
      LCHK(g, launch3_ypass(G, false, 1, -1, g->mix[0], nullptr, nullptr, nullptr, -1, 0, 0.0, -1.0, s));
      LCHK(g, launch3_zfwd(G, g->mix[0], g->xh, 0, s));
    } else {
      LCHK(g, launch_row_r2c(G, p, g->mix[0], nullptr, s));
      LCHK(g, launch_col_fwd(G, g->mix[0], g->xh, 0, nullptr, nullptr, s));
    }
  } else {
    rc = compute_rhs(g, S);
    if (rc) return rc;
    SolveOut so;
    rc = pcg(g, m, r, X_ZERO, nullptr, 1e-12, 1000, false, &so);
    if (rc) return rc;
    rc = solve_status_code(g, so);
    if (rc) return rc;
  }
  if (g->dim == 3) return energy3(g, prm, m, r, nullptr, out);
  const size_t n = (size_t)g->nx * g->ny;
  LCHK(g, launch_row_r2c(G, m, g->mix[0], nullptr, s));
  LCHK(g, launch_row_r2c(G, m + n, g->mix[1], nullptr, s));
  LCHK(g, launch_col_gradnorm(G, g->mix[0], g->mix[1], slot_ptr(g->part, SLOT_EGM), s));
  LCHK(g, launch_sum_slot(G, slot_ptr(g->part, SLOT_EGM), 1, col_nwg(G), 3, s));
  rc = energy_pointwise(g, prm, m, r);
  if (rc) return rc;
  DevStatus fin;
  rc = read_status(g, &fin);
  if (rc) return rc;
  const double gradm2 = fin.out[3] / (double)n;  // (1/n) sum w |xi|^2 |DFT m|^2
  assemble_energy(g, prm, gradm2, &fin.out[4], out);
  return NF_OK;
}

int nf_run(nf_grid* g, const nf_params* prm, double dt, int64_t max_steps, double eps_dm,
           int stop_on_energy_increase, double* m, double* p, const double* r, const double* S, double rtol,
           int max_iter, nf_run_info* info) {
  if (!g) return NF_EINVAL;
  g->err.clear();
  LCHK(g, launch_status_reset(g->geo, 1, g->stream));
  int rc = check_fields(g, {m, p, r, S});
  if (rc) return rc;
  rc = check_params(g, prm, dt);
  if (rc) return rc;
  if (!(rtol >= 0.0) || max_iter < 0 || max_steps < 1)
    return fail(g, NF_EINVAL, "rtol >= 0, max_iter >= 0 and max_steps >= 1 required");
  const Geo& G = g->geo;
  hipStream_t s = g->stream;
  const size_t n = (size_t)g->nx * g->ny;
  nf_run_info ri;
  ri.steps = 0;
  ri.stop_reason = NF_STOP_MAX_STEPS;
  ri.last_dm = NAN;
  ri.last_energy = NAN;
  ri.prev_energy = NAN;
  ri.total_cg_iters = 0;
  ri.unconverged_solves = 0;
  const bool en = stop_on_energy_increase != 0;
  const bool en2 = en && g->dim == 2;  // 2D: the gradient norm comes with the heat pass
  const bool need_sync = en || eps_dm > 0.0;

  rc = compute_rhs(g, S);
  if (rc) return rc;
  SolveOut so;
  rc = pcg(g, m, r, X_FROM_P, p, rtol, max_iter, false, &so);
  if (rc) return rc;
  ri.total_cg_iters += so.iters;
  rc = solve_status_code(g, so);
  if (rc == NF_ENOTCONV) {
    ri.unconverged_solves++;
    rc = NF_OK;
    g->err.clear();
  }
  if (rc) {
    if (info) *info = ri;
    return rc;
  }
  double e_prev = NAN;
  if (en && g->dim == 3) {
    rc = energy3(g, prm, m, r, &e_prev, nullptr);
    if (rc) return rc;
    ri.last_energy = e_prev;
  } else if (en) {
    LCHK(g, launch_row_r2c(G, m, g->mix[0], nullptr, s));
    LCHK(g, launch_row_r2c(G, m + n, g->mix[1], nullptr, s));
    LCHK(g, launch_col_gradnorm(G, g->mix[0], g->mix[1], slot_ptr(g->part, SLOT_EGM), s));
    LCHK(g, launch_sum_slot(G, slot_ptr(g->part, SLOT_EGM), 1, col_nwg(G), 3, s));
    rc = energy_pointwise(g, prm, m, r);
    if (rc) return rc;
    DevStatus t;
    rc = read_status(g, &t);
    if (rc) return rc;
    e_prev = assemble_energy(g, prm, t.out[3] / (double)n, &t.out[4], nullptr);
    ri.last_energy = e_prev;
  }
  while (ri.steps < max_steps) {
    rc = split_update(g, prm, dt, m, p, en2);
    if (rc) return rc;
    // keep Delta m and ||grad m_new||^2 before the solve reuses the status block
    rc = dm_to_status(g);
    if (rc) return rc;
    if (en2) LCHK(g, launch_sum_slot(G, slot_ptr(g->part, SLOT_EGM), 1, col_nwg(G), 10, s));
    DevStatus pre;
    if (need_sync) {
      rc = read_status(g, &pre);
      if (rc) return rc;
    }
    rc = pcg(g, m, r, X_FROM_XH, nullptr, rtol, max_iter, false, &so);
    if (rc) return rc;
    ri.steps += 1;
    ri.total_cg_iters += so.iters;
    if ((so.flags | so.sticky) & FLAG_NONFINITE) {
      ri.stop_reason = NF_STOP_ERROR;
      if (info) *info = ri;
      return fail(g, NF_ENONFINITE, "activation overflow: c^2 |grad p|^2 dt too large for the time step");
    }
    rc = solve_status_code(g, so);
    if (rc == NF_ENOTCONV) {
      ri.unconverged_solves++;
      rc = NF_OK;
      g->err.clear();
    }
    if (rc) {
      ri.stop_reason = NF_STOP_ERROR;
      if (info) *info = ri;
      return rc;
    }
    if (need_sync) {
      const double dm = pre.out[9] > 0.0 ? std::sqrt(pre.out[8] / pre.out[9]) / dt : 0.0;
      ri.last_dm = dm;
      if (en) {
        double e = 0.0;
        if (g->dim == 3) {
          rc = energy3(g, prm, m, r, &e, nullptr);
          if (rc) return rc;
        } else {
          rc = energy_pointwise(g, prm, m, r);
          if (rc) return rc;
          DevStatus t;
          rc = read_status(g, &t);
          if (rc) return rc;
          e = assemble_energy(g, prm, pre.out[10] * (double)n, &t.out[4], nullptr);
        }
        ri.prev_energy = e_prev;
        ri.last_energy = e;
        if (e >= e_prev) {
          ri.stop_reason = NF_STOP_ENERGY_INCREASE;
          break;
        }
        e_prev = e;
      }
      if (dm <= eps_dm) {
        ri.stop_reason = NF_STOP_DM_BELOW_EPS;
        break;
      }
    }
  }
  if (!need_sync) {
    // Delta m of the last step (its partials are still in place)
    rc = dm_to_status(g);
    if (rc) return rc;
    DevStatus t;
    rc = read_status(g, &t);
    if (rc) return rc;
    ri.last_dm = t.out[9] > 0.0 ? std::sqrt(t.out[8] / t.out[9]) / dt : 0.0;
    if (t.sticky & FLAG_NONFINITE) {
      ri.stop_reason = NF_STOP_ERROR;
      if (info) *info = ri;
      return fail(g, NF_ENONFINITE, "activation overflow: c^2 |grad p|^2 dt too large for the time step");
    }
  }
  // p = p[m_final]
  rc = write_p(g, p);
  if (rc) return rc;
  HIPCHK(g, hipStreamSynchronize(s));
  if (info) *info = ri;
  return NF_OK;
}

}  // extern "C"
