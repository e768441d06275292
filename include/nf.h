/*
 * nf.h -- C ABI of the MI355X (gfx950) implementation of the per-time-step hot
 * path of the Fourier spectral scheme for the periodic Hu-Cai network-formation
 * system (Aceves-Sanchez, Degond, Merino-Aceituno, Wytrzens, "A Spectral-Based
 * Method for Network-Formation PDEs").
 *
 * The system (Sec. 1.1, eqs. p and m):
 *     -div((m (x) m + r I) grad p) = S,
 *     d_t m - D^2 lap m - c^2 (m . grad p) grad p + |m|^{2(gamma-1)} m = 0,
 * on a periodic box, S time independent with zero integral.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Grid: n[0] = Nx, n[1] = Ny (2D), n[2] = Nz (3D), with the sizes listed
 *   under nf_create_grid; nodes x_i = i Lx / Nx, i < Nx (Sec. 2.2, node Nx
 *   identified with node 0).
 * - Fields are caller-owned DEVICE buffers of double, C-contiguous, x fastest:
 *   scalars (p, r, S) are [Ny][Nx]; the conductivity m is [2][Ny][Nx] with
 *   component 0 = m_x.  The library never frees, reallocates or retains them.
 * - The handle owns all workspace (allocated once by nf_create_grid); the
 *   solver entry points allocate no device memory.  Exceptions, outside the
 *   solver: nf_time_kernel allocates its stamp buffer, and an ensemble
 *   allocates the state of its partitions when they are set or tuned
 *   (nf_batch_set_partitions, the first nf_batch_run), the tuning also a
 *   scratch copy of m and p that it frees before the run.
 * - All work is enqueued on the handle's HIP stream (an ensemble's partitions
 *   run on streams of their own, forked from and joined to the batch's
 *   stream).  Entry points that run a
 *   PCG solve synchronise with that stream to test convergence; they return
 *   after the last kernel of the call has been queued and every host-visible
 *   result has been read back.
 * - Errors are reported by return code; on error the outputs are unspecified
 *   (exception: NF_ENOTCONV still writes the last iterate and fills info).
 *   nf_last_error() gives a message for the last failing call on a handle.
 * - Discrete pressure (reading of Sec. 2.4): the minimum-norm solution of the
 *   spectral operator of eq. p_discrete, whose first-derivative multipliers use
 *   the discrete Fourier variable of Sec. 2.3.3 with the Nyquist entry set to
 *   zero.  The 2^d Fourier modes on which those multipliers all vanish are
 *   projected out of S and of p.
 * - One handle per stream; calls on one handle must not overlap.
 */
#ifndef NF_H
#define NF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nf_grid nf_grid;

enum {
  NF_OK = 0,
  NF_EINVAL = -1,      /* invalid argument (size, dtype, dt <= 0, gamma <= 0, c2 < 0, D2 < 0, NULL field) */
  NF_ENOMEM = -2,      /* workspace allocation failed */
  NF_EDEVICE = -3,     /* a HIP runtime call or kernel launch failed */
  NF_ENOTCONV = -4,    /* PCG reached max_iter before the tolerance */
  NF_EINCOMPAT = -5,   /* |sum S| > 1e-12 sum |S|: solvability condition of eq. p violated */
  NF_ENONFINITE = -6   /* activation produced Inf/NaN: c^2 |grad p|^2 dt too large (Sec. 2.3.1, Remark) */
};

/*
 * Precision of the pressure solve (every other pass is FP64 in both):
 *   NF_F64          FP64 storage and arithmetic throughout;
 *   NF_F32_REFINED  iterative refinement: the iterate and the residual
 *                   Pi S - A p are FP64, each correction is the same PCG run
 *                   with FP32 transforms, fields and vector updates (FP64 inner
 *                   products and scalars).  The stopping test is on the FP64
 *                   residual, so rtol has the same meaning as for NF_F64 and
 *                   rel_res is the true relative residual.
 */
enum { NF_F64 = 0, NF_F32_REFINED = 1 };

enum { NF_STOP_MAX_STEPS = 0, NF_STOP_DM_BELOW_EPS = 1, NF_STOP_ENERGY_INCREASE = 2, NF_STOP_ERROR = 3 };

/* c^2, D^2 and the metabolic exponent gamma of eq. m. */
typedef struct {
  double c2, D2, gamma;
} nf_params;

typedef struct {
  int iters;           /* PCG iterations taken */
  int converged;       /* 1 if ||r|| <= rtol ||Pi S|| was reached */
  double rel_res;      /* recurrence residual / ||Pi S|| */
  double true_rel_res; /* ||Pi S - A p|| / ||Pi S|| (-1 when not computed) */
} nf_solve_info;

typedef struct {
  nf_solve_info solve;
  double dm_rel;       /* Delta m = ||m^{k+1} - m^k|| / (dt ||m^k||) (Sec. 2.5) */
  double energy;       /* E_h(m^k) with p[m^k] (Sec. 2.5), if energy_valid */
  int energy_valid;    /* 1 if the handle evaluates it (nf_set_step_energy), else 0 (energy NaN) */
} nf_step_info;

typedef struct {
  int64_t steps;          /* time steps taken */
  int stop_reason;        /* NF_STOP_* */
  double last_dm;         /* Delta m of the last step */
  double last_energy;     /* E_h of the final state (NaN if energy stopping was off) */
  double prev_energy;     /* E_h of the state before it (NaN if off) */
  int64_t total_cg_iters; /* PCG iterations over the whole run */
  int64_t unconverged_solves; /* solves that reached max_iter (the run continues with the last iterate) */
} nf_run_info;

/*
 * Create a solver handle for a 2D or 3D periodic grid (the scheme is the same
 * in 3D, with m in R^3 and the 3x3 tensor m m^T + r I; Sec. 2 and Sec. 5).
 *   ndim    2 or 3;
 *   n       grid sizes (Nx, Ny[, Nz]): 2D powers of two in [8, 4096] or
 *           50 * 2^k in [50, 1600] (the paper's grids; radix-5 stages);
 *           3D powers of two in [8, 1024];
 *   L       box lengths (Lx, Ly[, Lz]), > 0;
 *   dtype   NF_F64 or NF_F32_REFINED;
 *   stream  hipStream_t to enqueue on (NULL = default stream).
 * Allocates the workspace (8 complex half-spectrum fields plus tables, 9 in
 * 3D; with NF_F32_REFINED also 6 (3D: 7) single-precision half-spectrum
 * fields and FP32 copies of m and r) on the current HIP device.
 * Layouts of the caller's fields: 2D p, r, S [Ny][Nx], m [2][Ny][Nx]; 3D
 * p, r, S [Nz][Ny][Nx], m [3][Nz][Ny][Nx]; x fastest.
 * The first handle of a 2D shape and precision in a process also tunes the
 * tiles of the PCG loop (see nf_set_autotune).  Returns NF_EINVAL, NF_ENOMEM
 * or NF_EDEVICE on failure (*out is then NULL).
 */
int nf_create_grid(nf_grid **out, int ndim, const int64_t n[3], const double L[3], int dtype, void *stream);

/* Release the handle and its workspace (after synchronising its stream). NULL is a no-op. */
int nf_destroy_grid(nf_grid *g);

/* Change the stream the handle enqueues on (after synchronising the previous one,
 * whose queue may still hold the handle's last launches). */
int nf_set_stream(nf_grid *g, void *stream);

/*
 * NF_F32_REFINED handles: smallest relative residual reduction asked of one
 * FP32 correction (default 3e-6 in 2D, 1e-5 in 3D; each correction asks for
 * the reduction that reaches rtol with a margin of 2, but not below this
 * floor).  Must lie in (0, 0.5); NF_EINVAL otherwise.  No effect on NF_F64
 * handles.
 */
int nf_set_inner_tolerance(nf_grid *g, double floor_rtol);

/*
 * Pressure solve, Sec. 2.4 (eq. p_discrete by CG, warm started from p):
 * solves -div((m m^T + r I) grad p) = S for the minimum-norm p by preconditioned
 * CG with the constant-coefficient preconditioner -div(Kbar grad), Kbar the grid
 * mean of m m^T + r I (Sec. 5 mentions it).  Stops when
 * ||r_k||_2 <= rtol ||Pi S||_2 (recurrence residual; for NF_F32_REFINED handles
 * the FP64 residual of the refined iterate, max_iter then bounding the sum of
 * the FP32 iterations) or after max_iter iterations.
 *   m [2][Ny][Nx], r [Ny][Nx] (r > 0 is the caller's responsibility), S [Ny][Nx];
 *   p [Ny][Nx] in: initial guess, out: the solution (null modes removed);
 *   info may be NULL; if not, the true residual is computed as well.
 * Returns NF_OK, NF_ENOTCONV, NF_EINCOMPAT, NF_EINVAL or NF_EDEVICE.
 */
int nf_pressure_solve(nf_grid *g, const double *m, const double *r, const double *S, double *p, double rtol,
                      int max_iter, nf_solve_info *info);

/*
 * Allocation-free pressure solve, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Computes what nf_pressure_solve computes on an FP64
 * handle for the same grid (same kernels, same results), without a handle:
 *   n    (Nx, Ny), powers of two in [8, 4096] with Nx * Ny <= 65536;
 *   L    (Lx, Ly) > 0;  stream as for nf_create_grid;
 *   m, r, S, p, rtol, max_iter, info as for nf_pressure_solve.
 * Workspace: a fixed device array of 8 MiB per GPU (the library's own,
 * held by every GPU it runs on until the process ends); no hipMalloc,
 * hipFree, pinned host memory or events are used.  All calls on one GPU share
 * that array and each call overwrites it, so calls that overlap on one GPU
 * (several streams or host threads) race and must be serialised by the
 * caller.  The call synchronises its stream (convergence is polled).
 * Returns NF_EINVAL for sizes outside the limits above (message in
 * nf_last_error(NULL)), before any device work; otherwise the codes of
 * nf_pressure_solve.
 */
int nf_pressure_solve_noalloc(const int64_t n[2], const double L[2], void *stream, const double *m, const double *r,
                              const double *S, double *p, double rtol, int max_iter, nf_solve_info *info);

/*
 * One pass of the time loop of Algorithm 1:
 *   Step 1: p <- p[m^k] (as nf_pressure_solve, warm start from p on entry);
 *   Step 2: with g = grad p, exact activation (eq. m_activation_discrete), exact
 *           relaxation (eq. m_relaxation_discrete), exact diffusion by the heat
 *           multiplier exp(-D^2 |xi|^2 dt) in Fourier space (eq.
 *           diffusion_space_discrete), in that order.
 *   m [2][Ny][Nx] in: m^k, out: m^{k+1};  p out: p[m^k].
 * info may be NULL.  Each call forms the transformed right-hand side F(Pi S)
 * from S again (one forward transform, a few percent of a step; S may change
 * between calls); nf_run forms it once per run.  With nf_set_step_energy(g, 1)
 * the step also evaluates the discrete energy E_h of the state it starts from,
 * m^k with the pressure p[m^k] of Step 1 (as nf_energy does, 2D and 3D; a few
 * passes and one host synchronisation more), into info->energy; successive
 * calls thus give E_h(m^0), E_h(m^1), ...  Returns NF_OK, NF_ENOTCONV (m
 * is still advanced with the last PCG iterate), NF_EINCOMPAT, NF_ENONFINITE,
 * NF_EINVAL or NF_EDEVICE.
 */
int nf_step(nf_grid *g, const nf_params *prm, double dt, double *m, double *p, const double *r, const double *S,
            double rtol, int max_iter, nf_step_info *info);
/* on = 1: nf_step fills info->energy (see nf_step); 0 (the default): it does not.  NF_EINVAL for a NULL handle. */
int nf_set_step_energy(nf_grid *g, int on);

/*
 * Time loop of Algorithm 1 with the stopping criteria of Sec. 2.5.
 * Solves p[m^0] (warm start from p), then repeats: split update of m^k with
 * p[m^k]; solve p[m^{k+1}] (warm start from the previous solution);
 * Delta m^k; stop if stop_on_energy_increase and E_h(m^{k+1}) >= E_h(m^k), or
 * if Delta m <= eps_dm, or after max_steps steps.  At least one step is taken.
 * On return m holds the final state and p = p[m] for that state.  A solve that
 * reaches max_iter does not stop the run (its last iterate is used and counted
 * in info->unconverged_solves).
 * Returns NF_OK (see info->stop_reason) or the first error of a step
 * (NF_EINCOMPAT, NF_ENONFINITE, NF_EINVAL, NF_EDEVICE).
 */
int nf_run(nf_grid *g, const nf_params *prm, double dt, int64_t max_steps, double eps_dm,
           int stop_on_energy_increase, double *m, double *p, const double *r, const double *S, double rtol,
           int max_iter, nf_run_info *info);

/*
 * Discrete energy E_h of Sec. 2.5 (the energy functional of Sec. 1.1 on the grid):
 *   out[0] total,
 *   out[1] D^2/2 ||grad m||^2,
 *   out[2] || |m|^gamma ||^2 / (2 gamma),
 *   out[3] c^2/2 ||m . grad p||^2,
 *   out[4] c^2/2 sum h^d r |grad p|^2,
 * with ||f||^2 = h^d sum f^2 (h^d = hx hy, or hx hy hz on 3D handles) and the
 * spectral gradient.  p must be p[m]; if p is NULL the pressure is solved
 * (cold start, rtol 1e-12, 1000 iterations).  2D and 3D handles.
 */
int nf_energy(nf_grid *g, const nf_params *prm, const double *m, const double *p, const double *r, const double *S,
              double out[5]);

/*
 * Discrete adjoint (reverse mode) of one nf_step.  The step maps
 * (m^k, r, S) -> m^{k+1} = H Rel(Act(m^k, grad p)), p = p[m^k].  Given
 * lam_next = dL/dm^{k+1}, this computes, by transposing each stage:
 *   diffusion (H symmetric), relaxation (Jacobian of eq. m_relaxation_discrete),
 *   activation (Jacobian of eq. m_activation_discrete w.r.t. m and grad p),
 *   the gradient grad p, and the pressure equation (eq. p_discrete): since the
 *   operator A is symmetric, the adjoint pressure mu solves A mu = Pi G^T lam_g
 *   with the same PCG as nf_pressure_solve.
 * Inputs (device, layouts as above): m = m^k [d][Ny][Nx] (3D [3][Nz][Ny][Nx]),
 * p = p[m^k] (as returned by nf_step for that step), r, S, lam_next (as m).
 * Outputs: lam_k (as m) = dL/dm^k (overwritten); grad_r, grad_S (as p) are
 * ACCUMULATED (+=) with this step's dL/dr and dL/dS; mu (as p) is the adjoint
 * pressure (in: warm start, out: solution).  rtol/max_iter as in
 * nf_pressure_solve; info may be NULL.  2D and 3D handles; on 3D handles the
 * diffusion stage runs through the passes of the split update with activation
 * and relaxation switched off, and the pointwise stages as passes over physical
 * fields.
 * Returns NF_OK, NF_ENOTCONV (outputs written with the last iterate),
 * NF_ENONFINITE, NF_EINVAL or NF_EDEVICE.
 */
int nf_step_adjoint(nf_grid *g, const nf_params *prm, double dt, const double *m, const double *p, const double *r,
                    const double *S, const double *lam_next, double *lam_k, double *grad_r, double *grad_S,
                    double *mu, double rtol, int max_iter, nf_solve_info *info);

/*
 * Diagnostic entry points exposing single stages of the path, for unit checks
 * of the transforms and of the operator against independent references.
 *
 * nf_transform_forward: out = unnormalised 2D DFT of the real field f [Ny][Nx],
 *   in the packed half-spectrum layout used internally: out is [Nx/2][Ny]
 *   complex (interleaved re, im; 2 * Nx/2 * Ny doubles), entry [kx][ky] =
 *   F(kx, ky) for 1 <= kx < Nx/2, and column kx = 0 holds
 *   F(0, ky) + i F(Nx/2, ky) (both columns are spectra of real sequences).
 *   3D: out is [Nx/2][Ny][Nz] complex, entry [kx][ky][kz] = F(kx, ky, kz) for
 *   1 <= kx < Nx/2 and slot kx = 0 holds F(0, ky, kz) + i F(Nx/2, ky, kz).
 * nf_transform_inverse: f = inverse DFT (normalised by 1/n) of a packed
 *   half spectrum in the same layout.
 * nf_apply_operator: out = A p, the left-hand side of eq. p_discrete for the
 *   given m and r, p [Ny][Nx], out [Ny][Nx].
 * nf_gradient: grad = G f, the spectral gradient of eq. p_discrete (the
 *   first-derivative multipliers with the Nyquist entry zeroed, Sec. 2.3.3),
 *   f [Ny][Nx], grad [2][Ny][Nx] (component 0 = d/dx); 2D handles only
 *   (NF_EINVAL otherwise).
 * All four are enqueued on the handle's stream and return after synchronising it.
 */
int nf_transform_forward(nf_grid *g, const double *f, double *out);
int nf_transform_inverse(nf_grid *g, const double *spec, double *f);
int nf_apply_operator(nf_grid *g, const double *m, const double *r, const double *p, double *out);
int nf_gradient(nf_grid *g, const double *f, double *grad);

/*
 * Ensembles: independent instances of the problem of Sec. 2 advanced together.
 * Every pass of a time step is one launch per grid shape covering all the
 * instances of that shape (the instance is the second grid dimension), and
 * each PCG iteration is launched for all instances at once; an instance whose
 * solve has stopped does no work in the later iterations of that solve.
 *
 * nf_batch_create: count >= 1 instances; n [count][2] grid sizes (Nx, Ny),
 *   2D sizes as for nf_create_grid; L [count][2] box lengths (> 0); dtype
 *   NF_F64 or NF_F32_REFINED for every instance; stream as for
 *   nf_create_grid.  Each instance owns the workspace of one nf_grid.
 *   Returns NF_EINVAL, NF_ENOMEM or NF_EDEVICE on failure (*out is then NULL;
 *   nf_batch_last_error(NULL) holds the message).
 * nf_batch_run: for every instance i the computation of
 *   nf_run(g_i, &prm[i], dt, steps, 0.0, 0, m[i], p[i], r[i], S[i], rtol,
 *          max_iter, &info[i])
 *   (fixed step count, no Delta m or energy stopping).  The fields written
 *   are bitwise those of that single-instance call.  prm: count entries;
 *   m, p, r, S: count device pointers each, with the layouts of nf_run;
 *   info: count entries or NULL.  Returns NF_OK, NF_EINCOMPAT (some S_i
 *   violates the solvability condition; nothing is advanced), NF_ENONFINITE
 *   (the run stops for all instances after the step that produced it),
 *   NF_EINVAL or NF_EDEVICE.  Unconverged solves are counted per instance as
 *   in nf_run.  The call returns when all the work is complete.
 *
 * Partitions: the instances are split into 1 to 4 partitions of about equal
 * grid-point counts, each with its own HIP stream (created by the batch,
 * default priority) and host thread, forked from and complete before the
 * return to the batch's stream.  Partitions overlap each other's transform
 * and memory phases.  They meet after the first solve and after every step,
 * so a stop (NF_EINCOMPAT, NF_ENONFINITE, a device error) ends all of them at
 * the same point; the fields are those above for every partition count.
 * nf_batch_set_partitions: parts 0 (the default) tunes the count at the next
 *   nf_batch_run: every count from 1 to min(4, count) runs two steps on
 *   scratch copies of m and p (device memory for 3 doubles per grid point,
 *   freed before the run; the caller's fields are not written) and the fastest
 *   is kept for the following runs (one partition if that memory is not
 *   available).  parts in [1, min(4, count)] fixes it.
 *   NF_EINVAL otherwise.
 * nf_batch_set_graphs: on records each chunk of PCG iterations a partition
 *   launches (the three passes of every iteration for every grid shape) as a
 *   HIP graph on first use and replays it afterwards; 0 (the default)
 *   launches the kernels one by one.  The results are the same either way.
 *   NF_EINVAL for a NULL handle.
 * nf_batch_partitions: the partition count in use (0 before the first run
 *   when tuning); tune_ms (NULL or 4 entries) receives the tuning time of
 *   each candidate count (ms for the two steps, -1 where none was taken).
 *   Returns NF_EINVAL (< 0) for a NULL handle.
 */
typedef struct nf_batch nf_batch;
int nf_batch_create(nf_batch **out, int count, const int64_t *n, const double *L, int dtype, void *stream);
int nf_batch_destroy(nf_batch *b);
/* Change the stream the batch enqueues on. */
int nf_batch_set_stream(nf_batch *b, void *stream);
int nf_batch_run(nf_batch *b, const nf_params *prm, double dt, int64_t steps, double *const *m, double *const *p,
                 const double *const *r, const double *const *S, double rtol, int max_iter, nf_run_info *info);
int nf_batch_set_partitions(nf_batch *b, int parts);
int nf_batch_set_graphs(nf_batch *b, int on);
int nf_batch_partitions(const nf_batch *b, double *tune_ms);
const char *nf_batch_last_error(const nf_batch *b);

/*
 * Tile tuning of the PCG loop (2D grids with a side of 256 to 4096, powers of
 * two).  The three passes of a PCG iteration (operator middle: x transforms
 * and the flux (m m^T + r I) grad p; operator end: y transform, divergence and
 * the inner products; update) exist in several tile variants: rows per
 * workgroup of the operator middle, columns and threads per workgroup of the
 * other two, and the order of the radix-8 and radix-4 stages of their
 * transforms.  When
 * autotuning is on (the default), the first nf_create_grid of a grid shape
 * and precision in a process times every variant of each pass on the new
 * handle's workspace and keeps the fastest (the default tile unless a variant
 * is more than 3% faster); later handles, ensembles and allocation-free solves
 * of that shape use the same choice, so their results agree bit for bit.
 * The variants change the work split and the rounding of the transforms and
 * inner products only.
 * nf_set_autotune: 2 (the default) times each candidate's throughput with three
 *   concurrent launches on separate buffers on grids of at most 2^21 points
 *   (the choice for solves that share the GPU, as ensemble partitions and
 *   concurrent handles do; the tuning then allocates two scratch copies of the
 *   loop's buffers, freed before nf_create_grid returns) and alone on larger
 *   grids, which fill the GPU by themselves, each timed launch after an
 *   untimed fill of a 320 MiB scratch buffer (freed likewise) that clears the
 *   Infinity Cache as the loop's other passes do; 1 times each candidate alone
 *   on every grid; 0 turns tuning off
 *   (default tiles for handles created afterwards).  Shapes already tuned
 *   keep their choice.  NF_EINVAL for other values.
 * nf_tuning: the variants of a handle.  us / us_default: time per launch of the
 *   chosen variant / the default tile measured by the tuner (0 if not tuned);
 *   candidates: variants timed per pass.
 */
typedef struct {
  int tuned;          /* 1 if the variants were set by the tuner */
  int flux_rows;      /* operator middle: grid rows per workgroup */
  int flux_plan;      /* 0: radix-8 stages first, 1: radix-4 stages first */
  int div_cols;       /* operator end: spectral columns per workgroup */
  int div_plan;
  int div_threads;    /* threads per workgroup */
  int update_cols;    /* update: spectral columns per workgroup */
  int update_plan;
  int update_threads;
  int candidates[3];  /* operator middle, operator end, update */
  double us[3];
  double us_default[3];
  int flux_threads;   /* operator middle: threads per workgroup */
} nf_tuning_info;
int nf_set_autotune(int mode);
int nf_tuning(const nf_grid *g, nf_tuning_info *out);
/*
 * Fix the variants of one handle (2D), overriding the tuner: variant code v
 * selects half (v % 3 == 0), the default (1) or twice (2) the default rows
 * (operator middle) or columns (operator end, update) per workgroup; v / 3
 * selects the radix plan (0: radix-8 stages first, 1: radix-4 first); for the
 * operator middle v / 3 = 2 is the first plan with half the threads (only
 * where the tile would have 1024 threads), for the operator end and update
 * v / 3 = 2 or 3 the first plan with twice or four times the threads.  Codes:
 * operator middle [0, 8], the others [0, 11]; 1 is the untuned pass, -1 keeps
 * the current one.  NF_EINVAL if a variant does not exist for the grid and
 * precision.
 */
int nf_set_tiles(nf_grid *g, int flux_var, int div_var, int update_var);

/*
 * Kernel timing: nf_time_kernel(g, k) makes the PCG-loop kernel k (NF_KERNEL_*)
 * stamp, for every loop iteration, the start of its first and the end of its
 * last workgroup on the device wall clock; after each PCG loop the handle adds
 * the spans of the launches that did work (launches queued after the solver
 * stopped are discarded).  k = -1 switches timing off.  Both calls reset the
 * accumulators.  nf_time_kernel_read returns the summed span (ms) and the
 * launch count.  Handles of a batch are not timed.
 */
enum { NF_KERNEL_ROW_FLUX = 0, NF_KERNEL_COL_DIV = 1, NF_KERNEL_COL_UPDATE = 2 };
int nf_time_kernel(nf_grid *g, int which);
int nf_time_kernel_read(nf_grid *g, double *total_ms, int64_t *count);

/* Message describing the last error on the handle ("" if none). */
const char *nf_last_error(const nf_grid *g);

/* Version string of the library. */
const char *nf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NF_H */
