// Structures shared by the host driver and the kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nf {

// Device-resident solver status.  Written by exactly one workgroup (block 0)
// of the kernel that owns each field; read by later launches and copied to the
// host for convergence checks.
struct DevStatus {
  double kbar[8];   // grid mean of K = m m^T + r I: 2D Kxx, Kxy, Kyy; 3D Kxx, Kxy, Kxz, Kyy, Kyz, Kzz
  double bb;        // weighted ||b_hat||^2 of the projected right-hand side
  double rho[2];    // <r, M^-1 r> by iteration parity (expanded value used for beta)
  double rr[2];     // rr[0]: ||r||^2 of the residual at which the solve stopped
  double rr0;       // initial ||r||^2
  double orr, obb;  // mixed-precision solve: FP64 ||r||^2 and ||b||^2 at the last correction start
  double rscale;    // mixed-precision solve: ||r|| scaling the FP32 correction
  double orr_prev;  // mixed-precision solve: ||r||^2 at the previous correction start (+inf before the first)
  double out[16];   // results of the final reductions (energy terms, dm, ...)
  int conv_at;      // iteration at which PCG stopped (converged or max_iter); INT_MAX while running
  int converged;    // 1 if the stop was convergence
  int iters;        // PCG iterations done
  int flags;        // FLAG_* bits of the current PCG solve
  int sticky;       // FLAG_* bits raised since the last full reset (split update)
  int outer_done;   // mixed-precision solve: 1 once the FP64 residual test has ended it
  int itot;         // mixed-precision solve: FP32 iterations of the finished corrections
  int budget;       // iteration limit of the current (inner) PCG run, INT_MAX when unused
};

enum { FLAG_NONFINITE = 1, FLAG_INCOMPAT = 2 };

// Slots of the partial-sum area; each slot holds up to SLOT_K arrays of
// MAX_WG doubles.
enum {
  SLOT_P3 = 0,      // <d,q>, <q,M^-1 r>, <q,M^-1 q>, <r,M^-1 r>
  SLOT_P3INIT = 1,  // <r,M^-1 r>, <r,r>, <b,b>
  SLOT_KBAR = 2,    // sum mx^2, mx my, my^2, r
  SLOT_SCHK = 3,    // sum S, sum |S|
  SLOT_DM = 4,      // sum (m_new - m_old)^2, sum m_old^2
  SLOT_EPT = 5,     // sum r|g|^2, sum (m.g)^2, sum |m|^{2 gamma}
  SLOT_EGM = 6,     // sum w |xi|^2 |m_hat|^2 (both components)
  SLOT_RR = 7,      // ||r||^2 of the residual written by the last PCG update
  NSLOTS = 8,
  SLOT_K = 8,
  MAX_WG = 4096,
};

// Geometry and workspace pointers passed by value to every kernel.
struct Geo {
  int nx, ny, h, twn;
  double lx, ly;
  double inv_n;       // 1 / (number of grid points)
  const void* tw;     // cx<double>[twn] (cx<float> for the FP32 passes), tw[u] = exp(-2 pi i u / twn);
                      // twn is a common multiple of every transform length
  DevStatus* st;
  double* part;       // 2D: NSLOTS * SLOT_K * MAX_WG doubles; 3D: NSLOTS * SLOT_K * pstride doubles
  // 3D only (nz = 1 in 2D)
  int nz;
  double lz;
  int pstride;        // stride of the partial-sum arrays of one slot
  double* tot;        // NSLOTS * SLOT_K totals of the 3D partials (formed by a one-workgroup pass)
  // optional execution-span timing of one PCG-loop pass (nullptr = off): for
  // iteration it, the workgroups of kind tkind fold their start and end stamps
  // (device wall clock) into TCLK_W (min, max) pairs at
  // tclk[2 (it TCLK_W + (block mod TCLK_W))]; the host reduces them
  unsigned long long* tclk;
  int tkind;
  // tile variants of the PCG-loop passes chosen by the tuner (index 0: FP64
  // passes, 1: FP32 passes; VAR_DEFAULT = 1 is the untuned tile): operator
  // middle (row variant), operator end and update (column variants).  Read by
  // the launchers only.
  int var_flux[2], var_div[2], var_upd[2];
};

enum { TCLK_CAP = 2048, TCLK_W = 64 };
// tile variants of the PCG-loop passes (codes 0 .. NVAR-1, see nf_tiles.hpp);
// VAR_DEFAULT is the untuned tile
enum { VAR_DEFAULT = 1, NVAR = 12 };  // timed iterations per PCG loop, stamp slots per iteration

__host__ __device__ inline double* slot_ptr(double* part, int slot) {
  return part + (size_t)slot * SLOT_K * MAX_WG;
}

// ---- per-instance arguments of the batched passes --------------------------------
// A batched launch covers `count` instances of one grid shape: blockIdx.y picks
// the instance, whose pointers and parameters are read from a device array of
// these structs (same names and meaning as the single-instance launchers'
// arguments; void* fields hold complex double, complex float or double data
// as the pass expects).
struct RowR2cArgs {
  Geo g;
  const double* f;
  void* out;
  double* schk;
};
struct ColFwdArgs {
  Geo g;
  void* in;
  void* out;
  void* Gx;
  void* Gy;
};
struct ColGradArgs {
  Geo g;
  const void* xh;
  void* P;
  void* Gx;
  void* Gy;
};
struct FluxArgs {
  Geo g;
  void* G0;
  void* G1;
  const void* m;
  const void* r;
  double* kslot;
  float* lo;
};
struct DivArgs {
  Geo g;
  const void* Fx;
  const void* Fy;
  void* qh;
  const void* dh;
  void* rh;
  const void* bh;
};
struct UpdArgs {
  Geo g;
  void* xh;
  void* rh;
  void* dh;
  const void* qh;
  void* Gx;
  void* Gy;
};
struct SplitArgs {
  Geo g;
  void* P;
  void* Gx;
  const void* Gy;
  const double* m;
  double* p_out;
  double c2dt, gamma, dt, relax1;
};
struct HeatArgs {
  Geo g;
  void* Mx;
  void* My;
  double D2dt;
  double* eslot;
};
struct FinalArgs {
  Geo g;
  const void* Mx;
  const void* My;
  double* m;
  double* dslot;
};
struct RefStartArgs {
  Geo g;
  const void* r64;
  void* x64;
  void* x32;
  void* r32;
  void* d32;
  void* Gx;
  void* Gy;
};
struct RefAccArgs {
  Geo g;
  void* x64;
  const void* x32;
  void* Gx;
  void* Gy;
};
struct SumArgs {
  const double* slot;
  DevStatus* st;
};

// ---- fixed workspace of the allocation-free solve (nf_noalloc.hip) ------------------
// Size of the per-GPU device array and the largest grid it serves: 2D FP64,
// Nx * Ny <= NOALLOC_MAX_POINTS (8 complex half-spectrum fields of 8 bytes per
// grid point, the partial-sum slots, the status block and a twiddle table of
// at most 4096 entries).
enum : size_t { NOALLOC_SCRATCH_BYTES = 8u << 20 };
enum { NOALLOC_MAX_POINTS = 65536, NOALLOC_MAX_TWIDDLES = 4096, NOALLOC_MAX_DEVICES = 64 };
// Device address of the current GPU's copy of the array (looked up on the
// first call for that GPU and kept).
hipError_t noalloc_scratch(void** out);

// ---- host-callable launchers (defined in nf_kernels.hip) --------------------------
// All take the stream last and return hipError_t of the launch.
struct Bufs;

hipError_t launch_status_reset(const Geo& g, int full, hipStream_t s);

// ---- 3D passes (nf_kernels3d.hip).  g: the 3D geometry (ny = Ny, nz = Nz);
// row passes take the same geometry and treat the Ny*Nz lines (z, y) as rows.
// Mixed buffers hold [kx][z][y] (after x) or, in place, [kx][z][ky] (after
// x and y); spectral buffers hold [kx][ky][kz].
int nwg3_row(const Geo& g);
int nwg3_y(const Geo& g);
int nwg3_z(const Geo& g, bool f32 = false);  // workgroups of the z passes (FP32 loop passes: f32)
hipError_t launch3_row_r2c(const Geo& g, const double* f, void* out, int schk, hipStream_t s);
hipError_t launch3_row_c2r(const Geo& g, const void* in, double* f, hipStream_t s);
// lo: FP32 copies of m (3n) then r (n), written when non-null; kbar: write the Kbar partials
hipError_t launch3_row_flux(const Geo& g, bool f32, void* G0, void* G1, void* G2, const void* m, const void* r, int it,
                            int kbar, float* lo, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch3_row_split(const Geo& g, void* P, void* G0, void* G1, void* G2, const double* m, double* p_out,
                             double c2dt, double gamma, double dt, double relax1, double D2dt, hipStream_t s);
hipError_t launch3_row_final(const Geo& g, const void* M0, const void* M1, const void* M2, double* m, hipStream_t s);
// y passes over nf fields (1..4) in place; dir -1 forward, +1 inverse; stop_test: PCG
// stopping decision of iteration it (it >= 1); heat_D2dt >= 0: multiply by exp(-D2dt xi_y^2)
hipError_t launch3_ypass(const Geo& g, bool f32, int nf, int dir, void* F0, void* F1, void* F2, void* F3, int it,
                         int stop_test, double tol2, double heat_D2dt, hipStream_t s);
// z passes
hipError_t launch3_zfwd(const Geo& g, const void* in, void* out, int project, hipStream_t s);
// mode 1: P = x/n; 2: gradient (G0..G2); 3: both
hipError_t launch3_zinv(const Geo& g, int mode, const void* xh, void* P, void* G0, void* G1, void* G2, hipStream_t s);
hipError_t launch3_zdiv(const Geo& g, bool f32, int init, const void* F0, const void* F1, const void* F2, void* qh,
                        const void* dh, void* rh, const void* bh, int it, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch3_zupdate(const Geo& g, bool f32, int first, void* xh, void* rh, void* dh, const void* qh, void* G0,
                           void* G1, void* G2, int it, int max_iter, double tol2, hipStream_t s,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch3_zheat(const Geo& g, void* M0, void* M1, void* M2, double D2dt, hipStream_t s);
hipError_t launch3_zrefine_start(const Geo& g32, const void* r64, void* x64, void* x32, void* r32, void* d32,
                                 void* G0, void* G1, void* G2, double tol2, double floor_in, int max_iter,
                                 hipStream_t s);
hipError_t launch3_zrefine_acc(const Geo& g, void* x64, const void* x32, void* G0, void* G1, void* G2,
                               hipStream_t s);
// reduced totals of a slot into st->out[o..o+K)
hipError_t launch3_copy_tot(const Geo& g, int slot, int K, int o, hipStream_t s);
// energy terms (Sec. 2.5) in 3D: totals of sum r|g|^2, sum (m.g)^2, sum |m|^{2 gamma}
// into the SLOT_EPT totals (g = grad p as three physical fields), and of the
// Parseval sum of the three spectra of m into the SLOT_EGM total
hipError_t launch3_energy_pt(const Geo& g, const double* m, const double* r, const double* gx, const double* gy,
                             const double* gz, double gamma, hipStream_t s);
hipError_t launch3_spec_gradnorm(const Geo& g, const void* F0, const void* F1, const void* F2, hipStream_t s);
// adjoint of one 3D step (grid-stride passes): reverse of activation and
// relaxation (lam in: after diffusion, out: lam_m; G in: grad p, out: lam_g),
// the right-hand side -i xi_tilde . F(v) of the adjoint pressure from three
// spectra, and the final gradient terms (U = grad mu, P = grad p)
hipError_t launch3_adj1(const Geo& g, const double* m, double* lam, double* G0, double* G1, double* G2, double c2dt,
                        double gamma, double dt, double relax1, hipStream_t s);
hipError_t launch3_spec_divrhs(const Geo& g, const void* F0, const void* F1, const void* F2, void* bh, hipStream_t s);
hipError_t launch3_adj2(const Geo& g, const double* m, const double* mu, const double* U0, const double* U1,
                        const double* U2, const double* P0, const double* P1, const double* P2, double* lam,
                        double* grad_r, double* grad_S, hipStream_t s);
// g.tot of a slot from the n partials the passes of the PCG loop store (one
// workgroup; K = 1 or 7 arrays)
hipError_t launch3_sum_tot(const Geo& g, int slot, int K, int n, hipStream_t s);
hipError_t launch_zero_spec(const Geo& g, void* xh, hipStream_t s);
// row passes (physical <-> mixed)
int row_nwg(const Geo& g);
int col_nwg(const Geo& g);
// workgroups of the row variant rv of the operator middle / column variant cv
// of the operator end and update
int row_nwg_var(const Geo& g, int rv);
int col_nwg_var(const Geo& g, int cv);
// whether a variant exists for the grid of g and the real type (f32) and can run
bool flux_var_valid(const Geo& g, bool f32, int rv);
bool div_var_valid(const Geo& g, bool f32, int cv);
// partial sums of ||r||^2 written by the update of the PCG loop
int rr_nwg(const Geo& g, bool f32);
// rows per workgroup of row variant rv, columns per workgroup of column variant cv
int flux_var_rows(const Geo& g, int rv);
int flux_var_threads(const Geo& g, int rv);
int flux_var_plan(int rv);
int div_var_cols(const Geo& g, int cv);
int div_var_threads(const Geo& g, int cv);
// whether the grid sizes have tuned variants at all
bool var_grid(const Geo& g);
// fill n doubles with a value (a kernel, so that no memset node is recorded)
hipError_t launch_fill_doubles(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_row_r2c(const Geo& g, const double* f, void* out_mixed, double* schk_slot, hipStream_t s);
hipError_t launch_row_c2r(const Geo& g, const void* in_mixed, double* f, hipStream_t s);
// e0/e1: optional start/stop events timestamped by the dispatch (nullptr = none)
// lo: optional FP32 copies of m then r (3n floats), written when non-null
hipError_t launch_row_flux(const Geo& g, void* G0, void* G1, const double* m, const double* r, int it,
                           double* kbar_slot, double tol2, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr, float* lo = nullptr);
hipError_t launch_row_split(const Geo& g, void* P, void* Gx, void* Gy, const double* m, double* p_out,
                            double c2dt, double gamma, double dt, double relax_gamma1, hipStream_t s);
hipError_t launch_row_final(const Geo& g, const void* Mx, const void* My, double* m, double* dm_slot,
                            hipStream_t s);
hipError_t launch_row_energy(const Geo& g, const void* Gx, const void* Gy, const double* m, const double* r,
                             double gamma, double* slot, hipStream_t s);
// column passes (mixed <-> spectral)
hipError_t launch_col_fwd(const Geo& g, void* in_mixed, void* out_spec, int with_grad, void* Gx, void* Gy,
                          hipStream_t s);
hipError_t launch_col_grad(const Geo& g, const void* xh, void* P, void* Gx, void* Gy, hipStream_t s);
hipError_t launch_col_div(const Geo& g, int init, const void* Fx, const void* Fy, void* qh, const void* dh,
                          void* rh, const void* bh, int it, int nwg_row, hipStream_t s, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);
hipError_t launch_col_update(const Geo& g, int first, void* xh, void* rh, void* dh, const void* qh, void* Gx,
                             void* Gy, int it, int max_iter, double tol2, hipStream_t s, hipEvent_t e0 = nullptr,
                             hipEvent_t e1 = nullptr);
// FP32 instantiations of the PCG-loop passes (g.tw points at the FP32 table;
// m32/r32 are the FP32 copies written by launch_row_flux)
hipError_t launch_row_flux32(const Geo& g, void* G0, void* G1, const float* m32, const float* r32, int it,
                             double tol2, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_col_div32(const Geo& g, const void* Fx, const void* Fy, void* qh, const void* dh, void* rh, int it,
                            hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_col_update32(const Geo& g, void* xh, void* rh, void* dh, const void* qh, void* Gx, void* Gy, int it,
                               int max_iter, double tol2, hipStream_t s, hipEvent_t e0 = nullptr,
                               hipEvent_t e1 = nullptr);
// mixed-precision correction start / accumulation (g32: FP32 twiddles)
hipError_t launch_col_refine_start(const Geo& g32, const void* r64, void* x64, void* x32, void* r32, void* d32,
                                   void* Gx32, void* Gy32, double tol2, double floor_in, int max_iter, hipStream_t s);
hipError_t launch_col_refine_acc(const Geo& g, void* x64, const void* x32, void* Gx, void* Gy, hipStream_t s);
hipError_t launch_col_heat(const Geo& g, void* Mx, void* My, double D2dt, double* egm_slot, hipStream_t s);
hipError_t launch_col_gradnorm(const Geo& g, const void* Mx, const void* My, double* egm_slot, hipStream_t s);
// adjoint passes
hipError_t launch_row_adj1(const Geo& g, void* A0, void* A1, const void* G0, const void* G1, const double* m,
                           double* lam_out, double c2dt, double gamma, double dt, double relax1, hipStream_t s);
hipError_t launch_row_adj2(const Geo& g, const void* M1, const void* M2, const void* P1, const void* P2,
                           const double* m, const double* mu, double* lam, double* grad_r, double* grad_S,
                           hipStream_t s);
hipError_t launch_col_divrhs(const Geo& g, const void* V0, const void* V1, void* bh, hipStream_t s);
hipError_t launch_zero_doubles(double* p, size_t n, hipStream_t s);
// set the TCLK_CAP * TCLK_W stamp pairs to (max, 0)
hipError_t launch_tclk_reset(unsigned long long* t, hipStream_t s);
// reduce K arrays of n partials of a slot into st->out[o..o+K)
hipError_t launch_sum_slot(const Geo& g, const double* slot, int K, int n, int o, hipStream_t s);

// Batched launchers: `shape` gives the grid shape shared by the instances
// (sizes only), A points at `count` device-resident argument structs; the
// remaining arguments are common to the batch.  st0: `count` contiguous statuses.
hipError_t launchb_status_reset(DevStatus* st0, int count, int full, hipStream_t s);
hipError_t launchb_sum_slot(const SumArgs* A, int count, int K, int n, int o, hipStream_t s);
hipError_t launchb_row_r2c(const Geo& shape, const RowR2cArgs* A, int count, hipStream_t s);
hipError_t launchb_col_fwd(const Geo& shape, const ColFwdArgs* A, int count, int mode, hipStream_t s);
hipError_t launchb_col_grad(const Geo& shape, const ColGradArgs* A, int count, bool grad, hipStream_t s);
hipError_t launchb_row_flux(const Geo& shape, bool f32, const FluxArgs* A, int count, int it, double tol2,
                            hipStream_t s);
hipError_t launchb_col_div(const Geo& shape, bool f32, bool init, const DivArgs* A, int count, int it,
                           hipStream_t s);
hipError_t launchb_col_update(const Geo& shape, bool f32, const UpdArgs* A, int count, int first, int it,
                              int max_iter, double tol2, hipStream_t s);
hipError_t launchb_row_split(const Geo& shape, const SplitArgs* A, int count, hipStream_t s);
hipError_t launchb_col_heat(const Geo& shape, const HeatArgs* A, int count, hipStream_t s);
hipError_t launchb_row_final(const Geo& shape, const FinalArgs* A, int count, hipStream_t s);
hipError_t launchb_col_refine_start(const Geo& shape, const RefStartArgs* A, int count, double tol2,
                                    double floor_in, int max_iter, hipStream_t s);
hipError_t launchb_col_refine_acc(const Geo& shape, const RefAccArgs* A, int count, hipStream_t s);

}  // namespace nf
