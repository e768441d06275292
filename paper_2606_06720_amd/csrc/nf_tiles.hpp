// Tile geometry and global<->register images shared by the 2D and 3D passes:
// row passes (x direction, transposing to the column-major mixed layout) and
// column passes (contiguous lines), wavenumbers, the XCD-aware block order and
// the partial-sum writer.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "nf_fft.hpp"
#include "nf_internal.h"

namespace nf {

typedef cx<double> cd;

static constexpr double TWO_PI = 6.283185307179586476925286766559;

// ---------------------------------------------------------------- tile configs
// A row pass works on R physical rows of NX points (R*H complex pairs per
// field, H = NX/2) and transforms NF fields of the block together in one
// batched LDS FFT of NF*R lines; a column pass works on C columns of NY
// complex values, NF fields at once.
// Elements of one field held by a workgroup.  At 1024^2 this gives 512
// workgroups per pass, two per CU, so that one workgroup's transform overlaps
// the other's memory phase.
static constexpr int TILE = 1024;
static constexpr int TPF = TILE / 8;  // threads per field: one radix-8 butterfly per stage

// Rows of a row tile of t complex elements per field over lines of h pairs.
__host__ __device__ constexpr int tile_rows(int h, int t) { return t / h < 1 ? 1 : (t / h > 64 ? 64 : t / h); }
// Tile of the 2D row passes.  From Nx = 4096 on, the passes over one or two
// fields hold two rows per workgroup instead of one: the transposed stores then
// move runs twice as long and leave half as many partial cache lines open in
// L2 (one 16-wave workgroup per compute unit instead of two 8-wave ones).  The
// passes over three and four fields keep TILE.
__host__ __device__ constexpr int row_tile(int nx, int nf) { return (nf <= 2 && nx >= 4096) ? nx : TILE; }

template <int NX, int NF, int RT = TILE, int PL = 0, int TD = 1>
struct RowCfg {
  static constexpr int H = NX / 2;
  static constexpr int R = tile_rows(H, RT);                    // rows per workgroup
  static constexpr int NFv = NF;
  static constexpr int PLAN = PL;                               // radix plan of the x transforms
  // one radix-8 butterfly per thread, at most 1024 threads (wider tiles give
  // each thread several butterflies per stage); TD divides the thread count
  // (each thread then runs TD times the butterflies)
  static constexpr int NT = ((RT / 8) * NF > 1024 ? 1024 : (RT / 8) * NF) / TD;
  // LDS line stride: room for the FFT's padded layout, rounded so that the R
  // rows a group of 8 lanes touches in the row-interleaved phases (transposed
  // and paired loads and stores, consecutive lanes running over the rows of
  // one kx) start on different 32-byte quarters of the banks' 128 bytes:
  // stride = 8 / R (mod 8) complex for R < 8, 1 (mod 8) from R = 8 on
  static constexpr int LS0 = lpad_use(H) ? lpad_len(H) + 1 : H + 2;
  static constexpr int LSM = R >= 8 ? 1 : (R == 1 ? LS0 % 8 : 8 / R);
  static constexpr int LS = LS0 + ((LSM - LS0 % 8) + 8) % 8;
  static constexpr int RH = R * H;                              // pairs per field in the block
  static constexpr int NB = NF * R;                             // LDS lines
  static constexpr int ET = (NF * RH + NT - 1) / NT;            // transposed-image elements per thread
  static constexpr int EP = (RH + NT - 1) / NT;                 // pointwise elements per thread
};
// configuration of the 2D row passes
template <int NX, int NF>
using Row2D = RowCfg<NX, NF, row_tile(NX, NF)>;

// Default thread multiple of a column tile: columns of 4096 (one column per
// workgroup whose two FP64 fields take 131 KB of LDS, one workgroup per
// compute unit) take twice the threads, so that a compute unit runs 8 waves
// rather than 4.
__host__ __device__ constexpr int col_tm_default(int ny) { return ny >= 4096 ? 2 : 1; }
__host__ __device__ constexpr int col_threads(int ny, int nf) { return TPF * nf * col_tm_default(ny); }
template <int NY, int NF, int CT = TILE, int PL = 0, int TM = 0>
struct ColCfg {
  static constexpr int C0 = CT / NY;
  static constexpr int C = C0 < 1 ? 1 : (C0 > 64 ? 64 : C0);   // columns per workgroup
  static constexpr int PLAN = PL;                               // radix plan of the y transforms
  static constexpr int NYv = NY;
  // TM: thread multiple of the tile (0: the default of the column length)
  static constexpr int NT = TPF * NF * (TM > 0 ? TM : col_tm_default(NY));
  static constexpr int LS = lpad_use(NY) ? lpad_len(NY) : NY;   // room for the FFT's padded layout
  static constexpr int CN = C * NY;                             // elements per field in the block
  static constexpr int NB = NF * C;                             // LDS lines
  static constexpr int ET = (NF * CN + NT - 1) / NT;
  static constexpr int EP = (CN + NT - 1) / NT;
};

// ---------------------------------------------------------------- tuned variants
// The PCG-loop passes (operator middle, operator end, update) come in variants
// that a run-time tuner chooses between per grid shape and real type:
//   row variant rv (operator middle): rows per workgroup RD/2, RD or 2 RD for
//     rv % 3 = 0, 1, 2 (RD the default rows of Row2D<NX, 2>); rv / 3 = 0: radix
//     plan 0, 1: plan 1, 2: plan 0 with half the threads, for tiles that would
//     have 1024 threads (whose 128-register limit per thread makes them spill);
//   column variant cv (operator end, update): columns per workgroup CD/2, CD or
//     2 CD for cv % 3 = 0, 1, 2 (CD the default of ColCfg<NY, 2>); cv / 3 = 0:
//     radix plan 0, 1: plan 1, 2 and 3: plan 0 with twice and four times the
//     threads (long columns, where each thread of the default tile would
//     otherwise run several butterflies per stage, one wave per SIMD).
// Variant 1 (default tile, plan 0) is the untuned pass.  Variants that would
// repeat another (a radix plan without an alternative), fall below one row or
// column, leave threads without a radix-8 butterfly, or exceed the LDS of a
// workgroup do not exist.  Row variants use the codes below 9 only.
enum { LDS_LIMIT = 160 * 1024 };  // VAR_DEFAULT, NVAR: nf_internal.h

__host__ __device__ constexpr int rv_rows(int nx, int rv) {
  const int rd = tile_rows(nx / 2, row_tile(nx, 2));
  return rv % 3 == 0 ? rd / 2 : (rv % 3 == 1 ? rd : 2 * rd);
}
__host__ __device__ constexpr int cv_cols_default(int ny) {
  return TILE / ny < 1 ? 1 : (TILE / ny > 64 ? 64 : TILE / ny);
}
__host__ __device__ constexpr int cv_cols(int ny, int cv) {
  return cv % 3 == 0 ? cv_cols_default(ny) / 2 : (cv % 3 == 1 ? cv_cols_default(ny) : 2 * cv_cols_default(ny));
}
// LDS bytes of the operator-middle and operator-end passes for element size es
__host__ __device__ constexpr int flux_lds(int nx, int rows, int es) {
  return 2 * rows * ((lpad_use(nx / 2) ? lpad_len(nx / 2) + 1 : nx / 2 + 2) + 7) * es;
}
__host__ __device__ constexpr int div_lds(int ny, int cols, int es) {
  return 2 * cols * ((lpad_use(ny) ? lpad_len(ny) : ny) * es);
}
__host__ __device__ constexpr int cv_plan(int cv) { return cv / 3 == 1 ? 1 : 0; }
__host__ __device__ constexpr int cv_tm(int cv) { return cv / 3 == 2 ? 2 : (cv / 3 == 3 ? 4 : 1); }
__host__ __device__ constexpr int rv_plan(int rv) { return rv / 3 == 1 ? 1 : 0; }
__host__ __device__ constexpr int rv_td(int rv) { return rv / 3 == 2 ? 2 : 1; }
__host__ __device__ constexpr bool rv_ok(int nx, int ny, int rv, int es) {
  return rv >= 0 && rv < 9 && (rv / 3 != 1 || plan_has_alt(ilog2(nx / 2))) && rv_rows(nx, rv) >= 1 &&
         rv_rows(nx, rv) <= 64 && (rv % 3 != 2 || rv_rows(nx, rv) <= ny) &&
         (rv / 3 != 2 || rv_rows(nx, rv) * (nx / 2) / 8 * 2 >= 1024) &&
         flux_lds(nx, rv_rows(nx, rv), es) + 4096 <= LDS_LIMIT;
}
__host__ __device__ constexpr bool cv_ok(int ny, int h, int cv, int es) {
  return cv >= 0 && cv < NVAR && (cv / 3 != 1 || plan_has_alt(ilog2(ny))) && cv_cols(ny, cv) >= 1 &&
         cv_cols(ny, cv) <= 64 && (cv % 3 != 2 || cv_cols(ny, cv) <= h) &&
         cv_cols(ny, cv) * ny >= cv_tm(cv) * TILE && div_lds(ny, cv_cols(ny, cv), es) + 4096 <= LDS_LIMIT;
}
// grid sizes that have tuned variants (every size has the default)
__host__ __device__ constexpr bool var_size(int n) { return n >= 256 && n <= 4096 && (n & (n - 1)) == 0; }
// configurations of the variants (the default is exactly the untuned tile)
template <int NX, int RV>
using FluxCfg = typename std::conditional<RV == VAR_DEFAULT, Row2D<NX, 2>,
                                          RowCfg<NX, 2, rv_rows(NX, RV) * (NX / 2), rv_plan(RV), rv_td(RV)>>::type;
template <int NY, int CV>
using DivCfg = typename std::conditional<CV == VAR_DEFAULT, ColCfg<NY, 2>,
                                         ColCfg<NY, 2, cv_cols(NY, CV) * NY, cv_plan(CV), cv_tm(CV)>>::type;
// variants that can be built for a size (the row count against Ny is checked at run time)
template <int NX, int RV, int ES>
constexpr bool flux_var_exists() {
  return RV == VAR_DEFAULT || (var_size(NX) && rv_ok(NX, 1 << 20, RV, ES));
}
template <int NY, int CV, int ES>
constexpr bool div_var_exists() {
  return CV == VAR_DEFAULT || (var_size(NY) && cv_ok(NY, 1 << 20, CV, ES));
}

// first-derivative wavenumber (Nyquist zeroed) and full wavenumber
__device__ __forceinline__ double xi_tilde(int k, int n, double L) {
  if (2 * k == n) return 0.0;
  const int kk = (2 * k < n) ? k : k - n;
  return TWO_PI * (double)kk / L;
}
__device__ __forceinline__ double xi_full(int k, int n, double L) {
  const int kk = (2 * k <= n) ? k : k - n;
  return TWO_PI * (double)kk / L;
}
// x wavenumber of packed column kx (zero on the packed kx = 0 / Nx/2 column)
__device__ __forceinline__ double xi_col(int kx, double lx) { return kx == 0 ? 0.0 : TWO_PI * kx / lx; }

// Workgroups are dealt round-robin over the 8 XCDs; map them so that
// consecutive logical blocks (adjacent row blocks, which share cache lines of
// the column-major mixed layout) run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

template <typename V>
__device__ __forceinline__ const V* pick(int f, const V* a, const V* b, const V* c) {
  return f == 0 ? a : (f == 1 ? b : c);
}
template <typename V>
__device__ __forceinline__ V* pickw(int f, V* a, V* b, V* c) { return f == 0 ? a : (f == 1 ? b : c); }
// non-deduced context: optional pointer arguments may be passed as nullptr
template <typename V>
struct same_t {
  using type = V;
};
template <typename V>
using same = typename same_t<V>::type;

template <typename T>
struct vec2;
template <>
struct vec2<double> {
  using type = double2;
};
template <>
struct vec2<float> {
  using type = float2;
};

template <typename V>
__device__ __forceinline__ V vzero() {
  V v;
  v.x = 0;
  v.y = 0;
  return v;
}

// ---------------------------------------------------------------- row images
// "T" image: element e -> field e / RH, row (e % RH) % R, column (e % RH) / R;
// coalesced over the column-major mixed layout M[kx][y].  LDS line of (field,
// row) is field * R + row.
template <class C, typename V>
__device__ __forceinline__ void rowT_gload(V (&v)[(C::ET)], const V* s0, const same<V>* s1, const same<V>* s2,
                                           int ny, int y0, int nrow) {
  constexpr int NF = C::NFv;
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::RH, ee = e % C::RH;
    const int rr = ee % C::R, kx = ee / C::R;
    v[i] = (e < NF * C::RH && rr < nrow) ? pick<V>(f, s0, s1, s2)[(size_t)kx * ny + y0 + rr] : vzero<V>();
  }
}
template <class C, typename V>
__device__ __forceinline__ void rowT_put(V* buf, const V (&v)[(C::ET)]) {
  constexpr int NF = C::NFv;
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::RH, ee = e % C::RH;
    if (e < NF * C::RH) buf[(f * C::R + ee % C::R) * C::LS + ee / C::R] = v[i];
  }
}
// store the first NFS fields of the block back to the mixed layout
template <class C, int NFS, typename V>
__device__ __forceinline__ void rowT_store(const V* buf, same<V>* d0, same<V>* d1, same<V>* d2, int ny, int y0, int nrow) {
  for (int e = threadIdx.x; e < NFS * C::RH; e += C::NT) {
    const int f = e / C::RH, ee = e % C::RH;
    const int rr = ee % C::R, kx = ee / C::R;
    if (rr < nrow) pickw<V>(f, d0, d1, d2)[(size_t)kx * ny + y0 + rr] = buf[(f * C::R + rr) * C::LS + kx];
  }
}
// Pair images of the row passes, which fold the real-transform pre- and
// post-processing (irfft_pre / rfft_post of nf_fft.hpp, same arithmetic) into
// the transposed loads and stores: task t -> field t / (R NP), row
// (t % (R NP)) % R, pair k = (t % (R NP)) / R, covering the entries k and
// mirror(k) of that line (mirror(0) = H/2, the self-paired entry for even H;
// mirror(k) = H - k otherwise).  Consecutive tasks run along the R rows of one
// k, as the transposed images do.
template <class C>
struct RowPairs {
  static constexpr int NP = (C::H + 1) / 2;
  static constexpr int NTK = C::NFv * C::R * NP;          // tasks
  static constexpr int ETP = (NTK + C::NT - 1) / C::NT;   // tasks per thread
};
__host__ __device__ constexpr int pair_mirror(int k, int h) { return k == 0 ? h / 2 : h - k; }

template <class C, typename V>
__device__ __forceinline__ void rowTP_gload(V (&a)[RowPairs<C>::ETP], V (&b)[RowPairs<C>::ETP], const V* s0,
                                            const same<V>* s1, const same<V>* s2, int ny, int y0, int nrow) {
  using PT = RowPairs<C>;
  constexpr int H = C::H;
#pragma unroll
  for (int i = 0; i < PT::ETP; ++i) {
    const int t = threadIdx.x + i * C::NT;
    const int f = t / (C::R * PT::NP), u = t % (C::R * PT::NP);
    const int rr = u % C::R, k = u / C::R;
    const bool ok = t < PT::NTK && rr < nrow;
    const V* src = pick<V>(f, s0, s1, s2);
    a[i] = ok ? src[(size_t)k * ny + y0 + rr] : vzero<V>();
    b[i] = (ok && (k != 0 || H % 2 == 0)) ? src[(size_t)pair_mirror(k, H) * ny + y0 + rr] : vzero<V>();
  }
}
// Write the loaded pairs into the LDS lines (field * R + row) after the
// pre-processing of the inverse real transform: rebuilds 2 Z from the packed
// half spectrum X (see irfft_pre).  Rows beyond nrow carry zeros, as they do
// in the transposed image.
template <class C, typename T>
__device__ __forceinline__ void rowTP_put_pre(cx<T>* buf, const cx<T> (&a)[RowPairs<C>::ETP],
                                              const cx<T> (&b)[RowPairs<C>::ETP], const cx<T>* __restrict__ tw,
                                              int twn) {
  using PT = RowPairs<C>;
  constexpr int H = C::H;
  const int mult = twn / (2 * H);
#pragma unroll
  for (int i = 0; i < PT::ETP; ++i) {
    const int t = threadIdx.x + i * C::NT;
    if (t >= PT::NTK) continue;
    const int f = t / (C::R * PT::NP), u = t % (C::R * PT::NP);
    const int rr = u % C::R, k = u / C::R;
    cx<T>* l = buf + (f * C::R + rr) * C::LS;
    if (k == 0) {
      const cx<T> p = a[i];  // X[0] + i X[H]
      l[0] = mk<T>(p.x + p.y, p.x - p.y);
      if (H % 2 == 0) {
        const cx<T> xh = b[i];
        l[H / 2] = mk<T>(xh.x + xh.x, -(xh.y + xh.y));
      }
    } else {
      const cx<T> xk = a[i], xm = b[i];
      const cx<T> w = tw[k * mult];
      const cx<T> e1 = add(xk, conj(xm)), o1 = sub(xk, conj(xm));
      const cx<T> e2 = add(xm, conj(xk)), o2 = sub(xm, conj(xk));
      l[k] = add(e1, mul_i<+1>(mul(conj(w), o1)));
      l[H - k] = add(e2, mul_i<-1>(mul(w, o2)));
    }
  }
}
// Post-processing of the forward real transform (see rfft_post) of the first
// NFS fields' lines, stored straight to the mixed layout.
template <class C, int NFS, typename T>
__device__ __forceinline__ void rowTP_store_post(const cx<T>* buf, same<cx<T>>* d0, same<cx<T>>* d1,
                                                 same<cx<T>>* d2, const cx<T>* __restrict__ tw, int twn, int ny,
                                                 int y0, int nrow) {
  using PT = RowPairs<C>;
  constexpr int H = C::H;
  const int mult = twn / (2 * H);
  for (int t = threadIdx.x; t < NFS * C::R * PT::NP; t += C::NT) {
    const int f = t / (C::R * PT::NP), u = t % (C::R * PT::NP);
    const int rr = u % C::R, k = u / C::R;
    if (rr >= nrow) continue;
    const cx<T>* l = buf + (f * C::R + rr) * C::LS;
    cx<T>* dst = pickw<cx<T>>(f, d0, d1, d2) + y0 + rr;
    if (k == 0) {
      const cx<T> z0 = l[0];
      dst[0] = mk<T>(z0.x + z0.y, z0.x - z0.y);
      if (H % 2 == 0) dst[(size_t)(H / 2) * ny] = conj(l[H / 2]);
    } else {
      const cx<T> zk = l[k], zm = l[H - k];
      const cx<T> w = tw[k * mult];
      const cx<T> e1 = add(zk, conj(zm)), o1 = sub(zk, conj(zm));
      const cx<T> e2 = add(zm, conj(zk)), o2 = sub(zm, conj(zk));
      const cx<T> t1 = mul_i<-1>(mul(w, o1));
      const cx<T> t2 = mul_i<+1>(mul(conj(w), o2));
      dst[(size_t)k * ny] = scl(add(e1, t1), (T)0.5);
      dst[(size_t)(H - k) * ny] = scl(add(e2, t2), (T)0.5);
    }
  }
}

// "P" image of a physical field: element p -> row p / H, pair p % H (the
// grid points 2j, 2j+1 of the row), coalesced over the row-major layout
template <class C, typename P, typename S>
__device__ __forceinline__ void rowP_gload(P (&v)[(C::EP)], const S* __restrict__ f, int y0, int nrow) {
  constexpr int NX = 2 * C::H;
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    v[i] = (p < C::RH && rr < nrow) ? *(const P*)(f + (size_t)(y0 + rr) * NX + 2 * j) : vzero<P>();
  }
}

// ---------------------------------------------------------------- column images
// C is a ColCfg: C::NYv lines of C::C columns per field.
template <class C, int NFL, typename V>
__device__ __forceinline__ void colT_gload(V (&v)[(C::ET)], const V* s0, const same<V>* s1, int kx0, int h) {
  constexpr int NY = C::NYv;
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::CN, ee = e % C::CN;
    const int c = ee / NY, ky = ee % NY;
    v[i] = (e < NFL * C::CN && kx0 + c < h) ? (f == 0 ? s0 : s1)[(size_t)(kx0 + c) * NY + ky] : vzero<V>();
  }
}
template <class C, int NFL, typename V>
__device__ __forceinline__ void colT_put(V* buf, const V (&v)[(C::ET)]) {
  constexpr int NY = C::NYv;
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::CN, ee = e % C::CN;
    if (e < NFL * C::CN) buf[(f * C::C + ee / NY) * C::LS + ee % NY] = v[i];
  }
}
template <class C, int NFS, typename V>
__device__ __forceinline__ void colT_store(const V* buf, same<V>* d0, same<V>* d1, int kx0, int h) {
  constexpr int NY = C::NYv;
  for (int e = threadIdx.x; e < NFS * C::CN; e += C::NT) {
    const int f = e / C::CN, ee = e % C::CN;
    const int c = ee / NY, ky = ee % NY;
    if (kx0 + c < h) (f == 0 ? d0 : d1)[(size_t)(kx0 + c) * NY + ky] = buf[(f * C::C + c) * C::LS + ky];
  }
}
// pointwise image of one field: p -> column p / NY, row p % NY
template <class C, typename V>
__device__ __forceinline__ void colP_gload(V (&v)[(C::EP)], const V* __restrict__ src, int kx0, int h) {
  constexpr int NY = C::NYv;
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NY, ky = p % NY;
    v[i] = (p < C::CN && kx0 + c < h) ? src[(size_t)(kx0 + c) * NY + ky] : vzero<V>();
  }
}

// Execution-span stamps of a timed pass (see Geo::tclk): the first thread of
// every workgroup lowers the start stamp on entry and, after the workgroup's
// last instruction, raises the end stamp.  Uniform per workgroup.
__device__ __forceinline__ bool tclk_on(const Geo& g, int kind, int it) {
  return g.tclk != nullptr && g.tkind == kind && it >= 0 && it < TCLK_CAP;
}
__device__ __forceinline__ unsigned long long* tclk_slot(const Geo& g, int it) {
  return g.tclk + 2 * ((size_t)it * TCLK_W + (blockIdx.x & (TCLK_W - 1)));
}
__device__ __forceinline__ void tclk_start(const Geo& g, int kind, int it) {
  if (tclk_on(g, kind, it) && threadIdx.x == 0) atomicMin(tclk_slot(g, it), (unsigned long long)wall_clock64());
}
__device__ __forceinline__ void tclk_end(const Geo& g, int kind, int it) {
  if (tclk_on(g, kind, it)) {
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(tclk_slot(g, it) + 1, (unsigned long long)wall_clock64());
  }
}

template <int NT>
__device__ __forceinline__ void write_partials(double* slot, const double* v, int K) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) slot[(size_t)k * MAX_WG + blockIdx.x] = v[k];
  }
}

__device__ __forceinline__ double precond_symbol_inv(const double* K, double xx, double yy) {
  const double s = K[0] * xx * xx + 2.0 * K[1] * xx * yy + K[2] * yy * yy;
  return s > 0.0 ? 1.0 / s : 0.0;
}

}  // namespace nf
