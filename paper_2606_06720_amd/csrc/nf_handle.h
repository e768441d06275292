// Host-side solver handle (opaque to callers of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "nf.h"
#include "nf_internal.h"

struct nf_grid {
  using DevStatus = nf::DevStatus;
  using Geo = nf::Geo;
  int dim = 2;  // 2 or 3
  int nx = 0, ny = 0, nz = 1, h = 0;
  double lx = 1.0, ly = 1.0, lz = 1.0;
  hipStream_t stream = nullptr;
  int device = 0;
  void* tw = nullptr;
  int twn = 0;  // twiddle table length
  void* xh = nullptr;  // PCG iterate (spectral)
  void* rh = nullptr;  // residual
  void* dh = nullptr;  // search direction
  void* qh = nullptr;  // A d
  void* bh = nullptr;  // projected right-hand side
  void* mix[4] = {nullptr, nullptr, nullptr, nullptr};  // 2D uses 3, 3D uses 4
  double* part = nullptr;
  DevStatus* st = nullptr;
  DevStatus* hst = nullptr;  // pinned, 2 slots
  hipEvent_t ev[2] = {nullptr, nullptr};
  int last_iters = 0;
  DevStatus* st_own = nullptr;  // the handle's own status block (st may point into a batch's array)
  std::string err;
  Geo geo;
  // mixed-precision solve (dtype NF_F32_REFINED): FP32 inner PCG state
  int dtype = NF_F64;
  void* tw32 = nullptr;
  void* x32 = nullptr;  // inner iterate (correction e)
  void* r32 = nullptr;
  void* d32 = nullptr;
  void* q32 = nullptr;
  void* mix32[3] = {nullptr, nullptr, nullptr};  // 2D uses 2, 3D uses 3
  float* lo = nullptr;  // FP32 copies of m (d n) and r (n)
  double inner_floor = 1e-5;
  int last_inner[4] = {0, 0, 0, 0};
  Geo geo32;
  // optional per-kernel timing of one PCG-loop kernel: execution-span stamps
  // written by the kernel itself (Geo::tclk), read back after each PCG loop
  int timed = -1;
  int step_energy = 0;  // nf_step evaluates E_h(m^k) (nf_set_step_energy)
  unsigned long long* tclk = nullptr;   // device, 2 * TCLK_CAP
  unsigned long long* htclk = nullptr;  // pinned copy
  hipEvent_t tclk_ev = nullptr;         // marks the completion of the last stamp copy
  int tclk_pending = 0, tclk_lo = 0, tclk_hi = -1;  // iterations of that copy not yet added
  double wall_khz = 0.0;                // device wall-clock ticks per ms
  double timed_ms = 0.0;
  int64_t timed_count = 0;
  // tile variants of the PCG-loop passes (Geo::var_*): whether they came from
  // the tuner, and for the operator middle, end and update the number of
  // candidates timed, the chosen variant's and the default tile's time per launch
  int tuned = 0;
  int tune_ncand[3] = {1, 1, 1};
  double tune_us[3] = {0.0, 0.0, 0.0};
  double tune_us_default[3] = {0.0, 0.0, 0.0};
};

namespace nf {
// Wait for an event of a polling loop: query it, block after about a millisecond.
hipError_t poll_event(hipEvent_t e);
// Set the handle's tile variants for its grid shape and real type: from the
// process-wide cache, else by timing the candidates on its buffers (2D grids
// with tuned sizes, when autotuning is on); otherwise the default tiles.
int tune_handle(nf_grid* g);
// The cached variants (operator middle, end, update) of a shape, if any.
bool tune_lookup(int device, int nx, int ny, bool f32, int var[3]);
}  // namespace nf
