// Host side of the ensemble entry points (nf_batch_*, include/nf.h).
//
// Each instance owns the workspace of one nf_grid; their status blocks are
// moved into one contiguous array so that a single copy polls them all.
// Instances of equal grid shape form a launch group: every pass of the time
// step (Algorithm 1) and every PCG iteration is one launch per group, with the
// instance as the second grid dimension and its pointers and parameters read
// from a device table of per-instance argument structs.  The kernel bodies are
// those of the single-instance entry points, so each instance computes exactly
// what nf_run computes for it.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "nf.h"
#include "nf_handle.h"
#include "nf_internal.h"

using namespace nf;

namespace {

thread_local std::string batch_create_err;

// device argument tables of one launch group (k entries each)
struct Tables {
  FluxArgs *flux_init = nullptr, *flux_init_lo = nullptr, *flux_loop = nullptr, *flux32 = nullptr;
  DivArgs *div64 = nullptr, *div32 = nullptr;
  UpdArgs *upd64 = nullptr, *upd32 = nullptr;
  ColGradArgs *grad_x = nullptr, *split_p = nullptr, *split_g = nullptr;
  SplitArgs* split = nullptr;
  HeatArgs* heat = nullptr;
  FinalArgs* fin = nullptr;
  RefStartArgs* rstart = nullptr;
  RefAccArgs* racc = nullptr;
  SumArgs *sum_rr = nullptr, *sum_dm = nullptr;
};

}  // namespace

struct nf_batch {
  int count = 0;
  int dtype = NF_F64;
  hipStream_t stream = nullptr;
  std::vector<nf_grid*> inst;
  DevStatus* st = nullptr;   // count contiguous statuses
  DevStatus* hst = nullptr;  // pinned, 2 * count
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct Group {
    std::vector<int> idx;
    Geo shape;
    char* dev = nullptr;
    size_t bytes = 0;
    std::vector<char> host;
    Tables t;
  };
  std::vector<Group> groups;
  std::vector<DevStatus> fin;
  int last_iters = 0;
  int last_inner[4] = {0, 0, 0, 0};
  std::string err;
};

namespace {

int bfail(nf_batch* b, int code, const std::string& msg) {
  b->err = msg;
  return code;
}

#define BCHK(b, expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return bfail((b), NF_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));    \
  } while (0)

// Offsets of the tables in a group's allocation (256-byte aligned).
struct Layout {
  size_t off[18];
  size_t total;
};
Layout layout(int k) {
  const size_t sz[18] = {sizeof(FluxArgs),    sizeof(FluxArgs),     sizeof(FluxArgs),    sizeof(FluxArgs),
                         sizeof(DivArgs),     sizeof(DivArgs),      sizeof(UpdArgs),     sizeof(UpdArgs),
                         sizeof(ColGradArgs), sizeof(ColGradArgs),  sizeof(ColGradArgs), sizeof(SplitArgs),
                         sizeof(HeatArgs),    sizeof(FinalArgs),    sizeof(RefStartArgs), sizeof(RefAccArgs),
                         sizeof(SumArgs),     sizeof(SumArgs)};
  Layout L;
  size_t o = 0;
  for (int i = 0; i < 18; ++i) {
    L.off[i] = o;
    o += (sz[i] * k + 255) & ~(size_t)255;
  }
  L.total = o;
  return L;
}

template <typename T>
T* at(char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

void bind_tables(nf_batch::Group& G, char* base, const Layout& L) {
  Tables& t = G.t;
  t.flux_init = at<FluxArgs>(base, L.off[0]);
  t.flux_init_lo = at<FluxArgs>(base, L.off[1]);
  t.flux_loop = at<FluxArgs>(base, L.off[2]);
  t.flux32 = at<FluxArgs>(base, L.off[3]);
  t.div64 = at<DivArgs>(base, L.off[4]);
  t.div32 = at<DivArgs>(base, L.off[5]);
  t.upd64 = at<UpdArgs>(base, L.off[6]);
  t.upd32 = at<UpdArgs>(base, L.off[7]);
  t.grad_x = at<ColGradArgs>(base, L.off[8]);
  t.split_p = at<ColGradArgs>(base, L.off[9]);
  t.split_g = at<ColGradArgs>(base, L.off[10]);
  t.split = at<SplitArgs>(base, L.off[11]);
  t.heat = at<HeatArgs>(base, L.off[12]);
  t.fin = at<FinalArgs>(base, L.off[13]);
  t.rstart = at<RefStartArgs>(base, L.off[14]);
  t.racc = at<RefAccArgs>(base, L.off[15]);
  t.sum_rr = at<SumArgs>(base, L.off[16]);
  t.sum_dm = at<SumArgs>(base, L.off[17]);
}

// Fill the host image of a group's tables for one run and copy it to the device.
int upload_tables(nf_batch* b, nf_batch::Group& G, const nf_params* prm, double dt, double* const* m,
                  double* const* p, const double* const* r) {
  const int k = (int)G.idx.size();
  const Layout L = layout(k);
  char* hb = G.host.data();
  nf_batch::Group H;  // host-side view of the same layout
  bind_tables(H, hb, L);
  for (int j = 0; j < k; ++j) {
    const int i = G.idx[j];
    nf_grid* g = b->inst[i];
    const size_t n = (size_t)g->nx * g->ny;
    const Geo& g64 = g->geo;
    const Geo& g32 = g->geo32;
    H.t.flux_init[j] = FluxArgs{g64, g->mix[0], g->mix[1], m[i], r[i], slot_ptr(g->part, SLOT_KBAR), nullptr};
    H.t.flux_init_lo[j] = FluxArgs{g64, g->mix[0], g->mix[1], m[i], r[i], slot_ptr(g->part, SLOT_KBAR), g->lo};
    H.t.flux_loop[j] = FluxArgs{g64, g->mix[0], g->mix[1], m[i], r[i], nullptr, nullptr};
    H.t.flux32[j] = FluxArgs{g32, g->mix32[0], g->mix32[1], g->lo, g->lo ? g->lo + 2 * n : nullptr, nullptr, nullptr};
    H.t.div64[j] = DivArgs{g64, g->mix[0], g->mix[1], g->qh, g->dh, g->rh, g->bh};
    H.t.div32[j] = DivArgs{g32, g->mix32[0], g->mix32[1], g->q32, g->d32, g->r32, nullptr};
    H.t.upd64[j] = UpdArgs{g64, g->xh, g->rh, g->dh, g->qh, g->mix[0], g->mix[1]};
    H.t.upd32[j] = UpdArgs{g32, g->x32, g->r32, g->d32, g->q32, g->mix32[0], g->mix32[1]};
    H.t.grad_x[j] = ColGradArgs{g64, g->xh, nullptr, g->mix[0], g->mix[1]};
    H.t.split_p[j] = ColGradArgs{g64, g->xh, g->mix[0], nullptr, nullptr};
    H.t.split_g[j] = ColGradArgs{g64, g->xh, nullptr, g->mix[1], g->mix[2]};
    H.t.split[j] = SplitArgs{g64,        g->mix[0], g->mix[1],        g->mix[2],       m[i],
                             p[i],       prm[i].c2 * dt, prm[i].gamma, dt, std::exp(-dt)};
    H.t.heat[j] = HeatArgs{g64, g->mix[0], g->mix[1], prm[i].D2 * dt, nullptr};
    H.t.fin[j] = FinalArgs{g64, g->mix[0], g->mix[1], m[i], slot_ptr(g->part, SLOT_DM)};
    H.t.rstart[j] = RefStartArgs{g32, g->rh, g->xh, g->x32, g->r32, g->d32, g->mix32[0], g->mix32[1]};
    H.t.racc[j] = RefAccArgs{g64, g->xh, g->x32, g->mix[0], g->mix[1]};
    H.t.sum_rr[j] = SumArgs{slot_ptr(g->part, SLOT_RR), g->st};
    H.t.sum_dm[j] = SumArgs{slot_ptr(g->part, SLOT_DM), g->st};
  }
  BCHK(b, hipMemcpyAsync(G.dev, hb, L.total, hipMemcpyHostToDevice, b->stream));
  return NF_OK;
}

int read_all(nf_batch* b) {
  BCHK(b, hipMemcpyAsync(b->fin.data(), b->st, sizeof(DevStatus) * b->count, hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  return NF_OK;
}

// PCG iterations of all instances, chunked and polled as in the single-instance
// loop; stops once every instance's status reports a stop.
int batch_loop(nf_batch* b, bool f32, int max_iter, double tol2, int expect) {
  hipStream_t s = b->stream;
  const int c = b->count;
  int it = 0, slot = 0, pending = -1;
  bool first_chunk = true;
  while (it < max_iter) {
    int nk = first_chunk ? (expect > 6 ? expect - 4 : 2) : 3;
    first_chunk = false;
    if (nk > max_iter - it) nk = max_iter - it;
    for (int q = 0; q < nk; ++q) {
      for (auto& G : b->groups) {
        const int k = (int)G.idx.size();
        BCHK(b, launchb_row_flux(G.shape, f32, f32 ? G.t.flux32 : G.t.flux_loop, k, it, tol2, s));
        BCHK(b, launchb_col_div(G.shape, f32, false, f32 ? G.t.div32 : G.t.div64, k, it, s));
        BCHK(b, launchb_col_update(G.shape, f32, f32 ? G.t.upd32 : G.t.upd64, k, 0, it + 1, max_iter, tol2, s));
      }
      ++it;
    }
    BCHK(b, hipMemcpyAsync(b->hst + (size_t)slot * c, b->st, sizeof(DevStatus) * c, hipMemcpyDeviceToHost, s));
    BCHK(b, hipEventRecord(b->ev[slot], s));
    if (pending >= 0) {
      BCHK(b, hipEventSynchronize(b->ev[pending]));
      bool all = true;
      for (int i = 0; i < c && all; ++i) all = b->hst[(size_t)pending * c + i].conv_at != INT_MAX;
      if (all) break;
    }
    pending = slot;
    slot ^= 1;
  }
  return read_all(b);
}

struct SolveRes {
  std::vector<int> iters, converged;
};

// Pressure solves of all instances (the pcg / pcg_refined sequence of the
// single-instance path, batched).  first: warm start from p, else from the
// spectral iterate kept from the previous solve.
int batch_solve(nf_batch* b, bool first, double* const* p, double rtol, int max_iter, SolveRes* out) {
  hipStream_t s = b->stream;
  const int c = b->count;
  BCHK(b, launchb_status_reset(b->st, c, 0, s));
  if (first) {
    for (int i = 0; i < c; ++i) {
      nf_grid* g = b->inst[i];
      BCHK(b, launch_row_r2c(g->geo, p[i], g->mix[0], nullptr, s));
      BCHK(b, launch_col_fwd(g->geo, g->mix[0], g->xh, 1, g->mix[0], g->mix[1], s));
    }
  } else {
    for (auto& G : b->groups) BCHK(b, launchb_col_grad(G.shape, G.t.grad_x, (int)G.idx.size(), true, s));
  }
  const double tol2 = rtol * rtol;
  out->iters.assign(c, 0);
  out->converged.assign(c, 0);
  if (b->dtype == NF_F64) {
    for (auto& G : b->groups) {
      const int k = (int)G.idx.size();
      BCHK(b, launchb_row_flux(G.shape, false, G.t.flux_init, k, -1, 0.0, s));
      BCHK(b, launchb_col_div(G.shape, false, true, G.t.div64, k, 0, s));
      BCHK(b, launchb_col_update(G.shape, false, G.t.upd64, k, 1, 0, max_iter, tol2, s));
    }
    int rc = batch_loop(b, false, max_iter, tol2, b->last_iters);
    if (rc) return rc;
    // final convergence test of solves stopped by max_iter, on the last residual
    for (auto& G : b->groups)
      BCHK(b, launchb_sum_slot(G.t.sum_rr, (int)G.idx.size(), 1, col_nwg(G.shape), 11, s));
    rc = read_all(b);
    if (rc) return rc;
    int mx = 0;
    for (int i = 0; i < c; ++i) {
      const DevStatus& f = b->fin[i];
      bool conv = f.converged != 0;
      if (!conv && f.conv_at == max_iter && max_iter > 0 && !(f.flags & (FLAG_NONFINITE | FLAG_INCOMPAT)))
        conv = f.out[11] <= tol2 * f.bb;
      out->iters[i] = f.iters;
      out->converged[i] = conv ? 1 : 0;
      mx = f.iters > mx ? f.iters : mx;
    }
    if (mx > 0) b->last_iters = mx;
    return NF_OK;
  }
  for (int outer = 0;; ++outer) {
    for (auto& G : b->groups) {
      const int k = (int)G.idx.size();
      BCHK(b, launchb_row_flux(G.shape, false, outer == 0 ? G.t.flux_init_lo : G.t.flux_init, k, -1, 0.0, s));
      BCHK(b, launchb_col_div(G.shape, false, true, G.t.div64, k, 0, s));
      BCHK(b, launchb_col_refine_start(G.shape, G.t.rstart, k, tol2, b->inst[G.idx[0]]->inner_floor, max_iter, s));
    }
    const int slot = outer < 3 ? outer : 3;
    int rc = batch_loop(b, true, max_iter, 1.0, b->last_inner[slot]);
    if (rc) return rc;
    bool all = true;
    int mx = 0;
    for (int i = 0; i < c; ++i) {
      all = all && b->fin[i].outer_done;
      mx = b->fin[i].iters > mx ? b->fin[i].iters : mx;
    }
    if (all) break;
    if (mx > 0) b->last_inner[slot] = mx;
    for (auto& G : b->groups) BCHK(b, launchb_col_refine_acc(G.shape, G.t.racc, (int)G.idx.size(), s));
  }
  for (int i = 0; i < c; ++i) {
    out->iters[i] = b->fin[i].itot;
    out->converged[i] = b->fin[i].converged;
  }
  return NF_OK;
}

}  // namespace

extern "C" {

const char* nf_batch_last_error(const nf_batch* b) { return b ? b->err.c_str() : batch_create_err.c_str(); }

int nf_batch_destroy(nf_batch* b) {
  if (!b) return NF_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  for (nf_grid* g : b->inst) {
    if (!g) continue;
    g->st = g->st_own;
    g->geo.st = g->st_own;
    g->geo32.st = g->st_own;
    nf_destroy_grid(g);
  }
  for (auto& G : b->groups)
    if (G.dev) (void)hipFree(G.dev);
  if (b->st) (void)hipFree(b->st);
  if (b->hst) (void)hipHostFree(b->hst);
  for (int i = 0; i < 2; ++i)
    if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
  delete b;
  return NF_OK;
}

int nf_batch_set_stream(nf_batch* b, void* stream) {
  if (!b) return NF_EINVAL;
  b->stream = (hipStream_t)stream;
  return NF_OK;
}

int nf_batch_create(nf_batch** out, int count, const int64_t* n, const double* L, int dtype, void* stream) {
  if (!out) return NF_EINVAL;
  *out = nullptr;
  batch_create_err.clear();
  if (count < 1 || !n || !L || (dtype != NF_F64 && dtype != NF_F32_REFINED)) {
    batch_create_err = "count >= 1, non-NULL n and L and a valid dtype are required";
    return NF_EINVAL;
  }
  nf_batch* b = new nf_batch();
  b->count = count;
  b->dtype = dtype;
  b->stream = (hipStream_t)stream;
  b->inst.assign(count, nullptr);
  hipError_t herr = hipSuccess;
  auto bail = [&](int code, const std::string& what) {
    batch_create_err = what + (herr != hipSuccess ? std::string(": ") + hipGetErrorString(herr) : "");
    nf_batch_destroy(b);
    return code;
  };
  for (int i = 0; i < count; ++i) {
    const int64_t nn[3] = {n[2 * i], n[2 * i + 1], 1};
    const double LL[3] = {L[2 * i], L[2 * i + 1], 1.0};
    const int rc = nf_create_grid(&b->inst[i], 2, nn, LL, dtype, stream);
    if (rc != NF_OK) return bail(rc, "instance " + std::to_string(i) + ": " + nf_last_error(nullptr));
  }
  if ((herr = hipMalloc((void**)&b->st, sizeof(DevStatus) * count)) != hipSuccess) return bail(NF_ENOMEM, "hipMalloc(st)");
  if ((herr = hipMemset(b->st, 0, sizeof(DevStatus) * count)) != hipSuccess) return bail(NF_EDEVICE, "hipMemset(st)");
  if ((herr = hipHostMalloc((void**)&b->hst, 2 * sizeof(DevStatus) * count, hipHostMallocDefault)) != hipSuccess)
    return bail(NF_ENOMEM, "hipHostMalloc(status)");
  for (int i = 0; i < 2; ++i)
    if ((herr = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming)) != hipSuccess)
      return bail(NF_EDEVICE, "hipEventCreate");
  b->fin.resize(count);
  for (int i = 0; i < count; ++i) {
    nf_grid* g = b->inst[i];
    g->st = b->st + i;
    g->geo.st = g->st;
    g->geo32.st = g->st;
    // group by shape and box
    nf_batch::Group* grp = nullptr;
    for (auto& G : b->groups) {
      const nf_grid* h = b->inst[G.idx[0]];
      if (h->nx == g->nx && h->ny == g->ny && h->lx == g->lx && h->ly == g->ly) grp = &G;
    }
    if (!grp) {
      b->groups.emplace_back();
      grp = &b->groups.back();
      grp->shape = g->geo;
    }
    grp->idx.push_back(i);
  }
  for (auto& G : b->groups) {
    const Layout Lo = layout((int)G.idx.size());
    G.bytes = Lo.total;
    G.host.assign(Lo.total, 0);
    if ((herr = hipMalloc((void**)&G.dev, Lo.total)) != hipSuccess) return bail(NF_ENOMEM, "hipMalloc(tables)");
    bind_tables(G, G.dev, Lo);
  }
  *out = b;
  return NF_OK;
}

int nf_batch_run(nf_batch* b, const nf_params* prm, double dt, int64_t steps, double* const* m, double* const* p,
                 const double* const* r, const double* const* S, double rtol, int max_iter, nf_run_info* info) {
  if (!b) return NF_EINVAL;
  b->err.clear();
  const int c = b->count;
  if (!prm || !m || !p || !r || !S) return bfail(b, NF_EINVAL, "NULL argument array");
  if (!(dt > 0.0)) return bfail(b, NF_EINVAL, "dt must be > 0");
  if (!(rtol >= 0.0) || max_iter < 0 || steps < 1)
    return bfail(b, NF_EINVAL, "rtol >= 0, max_iter >= 0 and steps >= 1 required");
  for (int i = 0; i < c; ++i) {
    if (!m[i] || !p[i] || !r[i] || !S[i]) return bfail(b, NF_EINVAL, "NULL field pointer of instance " + std::to_string(i));
    if (!(prm[i].gamma > 0.0) || !(prm[i].c2 >= 0.0) || !(prm[i].D2 >= 0.0))
      return bfail(b, NF_EINVAL, "invalid params of instance " + std::to_string(i));
  }
  hipStream_t s = b->stream;
  std::vector<nf_run_info> ri(c);
  for (auto& x : ri) {
    x.steps = 0;
    x.stop_reason = NF_STOP_MAX_STEPS;
    x.last_dm = NAN;
    x.last_energy = NAN;
    x.prev_energy = NAN;
    x.total_cg_iters = 0;
    x.unconverged_solves = 0;
  }
  auto finish = [&](int rc) {
    if (info)
      for (int i = 0; i < c; ++i) info[i] = ri[i];
    return rc;
  };
  for (auto& G : b->groups) {
    const int rc = upload_tables(b, G, prm, dt, m, p, r);
    if (rc) return finish(rc);
  }
  BCHK(b, launchb_status_reset(b->st, c, 1, s));
  for (int i = 0; i < c; ++i) {
    nf_grid* g = b->inst[i];
    BCHK(b, launch_row_r2c(g->geo, S[i], g->mix[0], slot_ptr(g->part, SLOT_SCHK), s));
    BCHK(b, launch_col_fwd(g->geo, g->mix[0], g->bh, 0, nullptr, nullptr, s));
  }
  SolveRes sr;
  int rc = batch_solve(b, true, p, rtol, max_iter, &sr);
  if (rc) return finish(rc);
  for (int i = 0; i < c; ++i) {
    ri[i].total_cg_iters += sr.iters[i];
    if (b->fin[i].flags & FLAG_INCOMPAT) {
      ri[i].stop_reason = NF_STOP_ERROR;
      rc = bfail(b, NF_EINCOMPAT, "instance " + std::to_string(i) + ": S violates the solvability condition");
    } else if (!sr.converged[i]) {
      ri[i].unconverged_solves++;
    }
  }
  if (rc) return finish(rc);
  for (int64_t step = 0; step < steps; ++step) {
    for (auto& G : b->groups) {
      const int k = (int)G.idx.size();
      BCHK(b, launchb_col_grad(G.shape, G.t.split_p, k, false, s));
      BCHK(b, launchb_col_grad(G.shape, G.t.split_g, k, true, s));
      BCHK(b, launchb_row_split(G.shape, G.t.split, k, s));
      BCHK(b, launchb_col_heat(G.shape, G.t.heat, k, s));
      BCHK(b, launchb_row_final(G.shape, G.t.fin, k, s));
    }
    rc = batch_solve(b, false, p, rtol, max_iter, &sr);
    if (rc) return finish(rc);
    bool bad = false;
    for (int i = 0; i < c; ++i) {
      ri[i].steps += 1;
      ri[i].total_cg_iters += sr.iters[i];
      if ((b->fin[i].flags | b->fin[i].sticky) & FLAG_NONFINITE) {
        ri[i].stop_reason = NF_STOP_ERROR;
        bad = true;
      } else if (!sr.converged[i]) {
        ri[i].unconverged_solves++;
      }
    }
    if (bad) return finish(bfail(b, NF_ENONFINITE, "activation overflow: c^2 |grad p|^2 dt too large for the time step"));
  }
  // Delta m of the last step and p = p[m_final]
  for (auto& G : b->groups)
    BCHK(b, launchb_sum_slot(G.t.sum_dm, (int)G.idx.size(), 2, row_nwg(G.shape), 8, s));
  for (int i = 0; i < c; ++i) {
    nf_grid* g = b->inst[i];
    BCHK(b, launch_col_grad(g->geo, g->xh, g->mix[0], nullptr, nullptr, s));
    BCHK(b, launch_row_c2r(g->geo, g->mix[0], p[i], s));
  }
  rc = read_all(b);
  if (rc) return finish(rc);
  for (int i = 0; i < c; ++i) {
    const DevStatus& f = b->fin[i];
    ri[i].last_dm = f.out[9] > 0.0 ? std::sqrt(f.out[8] / f.out[9]) / dt : 0.0;
    if (f.sticky & FLAG_NONFINITE) {
      ri[i].stop_reason = NF_STOP_ERROR;
      rc = bfail(b, NF_ENONFINITE, "activation overflow: c^2 |grad p|^2 dt too large for the time step");
    }
  }
  return finish(rc);
}

}  // extern "C"
