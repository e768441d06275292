// HIP kernels (gfx950, FP64) of the per-time-step hot path:
//   * row passes   -- the x-direction real transforms, fused with the pointwise
//                     work that needs physical values (flux K grad p, activation,
//                     relaxation, energy terms), transposing to column-major;
//   * column passes -- the y-direction complex transforms of the packed
//                     half spectrum, fused with the spectral multipliers
//                     (gradient, divergence, preconditioner, heat kernel) and the
//                     PCG vector updates / inner products.
//
// Data layout (2D, n = Nx*Ny, H = Nx/2):
//   physical   f[y][x]                 (double, x fastest, caller-owned)
//   mixed      M[kx][y]  kx < H        (complex, after the x transform)
//   spectral   F[kx][ky] kx < H        (complex, after both transforms)
// Column kx = 0 packs the real kx = 0 and kx = Nx/2 columns as X0 + i X_{Nx/2}.
// Every multiplier used on it (first-derivative wavenumbers with the Nyquist
// entry zeroed, preconditioner) is identical for both packed halves; the heat
// kernel, which differs, unpacks the pair (ky, -ky) first.
//
// Spectral vectors hold the unnormalised DFT of the physical field.  Inner
// products are sum_k w_k Re(a conj b) with w = 1 on the packed column and 2
// elsewhere, which is n times the physical Euclidean product (Parseval).
#include <hip/hip_ext.h>

#include <climits>

#include "nf_fft.hpp"
#include "nf_internal.h"
#include "nf_tiles.hpp"

namespace nf {

// ================================================================ small kernels
__device__ __forceinline__ void k_status_reset_one(DevStatus* st, int full) {
  if (threadIdx.x == 0) {
    if (full) st->sticky = 0;
    for (int i = 0; i < 8; ++i) st->kbar[i] = 0.0;
    st->bb = 0.0;
    st->rho[0] = st->rho[1] = 0.0;
    st->rr[0] = st->rr[1] = 0.0;
    st->rr0 = 0.0;
    st->orr = st->obb = st->rscale = 0.0;
    st->orr_prev = __builtin_inf();
    st->outer_done = 0;
    st->itot = 0;
    st->budget = INT_MAX;
    for (int i = 0; i < 16; ++i) st->out[i] = 0.0;
    st->conv_at = INT_MAX;
    st->converged = 0;
    st->iters = 0;
    st->flags = 0;
  }
}

__global__ void k_status_reset(DevStatus* st, int full) {
  if (blockIdx.x == 0) k_status_reset_one(st, full);
}
__global__ void kb_status_reset(DevStatus* st0, int full) { k_status_reset_one(st0 + blockIdx.x, full); }
__global__ void k_zero(cd* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = mk<double>(0.0, 0.0);
}

__device__ __forceinline__ void sum_slot_body(const double* __restrict__ slot, int K, int n, int o, DevStatus* st) {
  __shared__ double scratch[8 * 4];
  double v[8];
  for (int k = 0; k < 8; ++k) v[k] = 0.0;
  for (int k = 0; k < K; ++k)
    for (int i = threadIdx.x; i < n; i += 256) v[k] += slot[(size_t)k * MAX_WG + i];
  block_sum<256, 8>(v, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) st->out[o + k] = v[k];
}
__global__ void __launch_bounds__(256) k_sum_slot(const double* __restrict__ slot, int K, int n, int o, DevStatus* st) {
  sum_slot_body(slot, K, n, o, st);
}
__global__ void __launch_bounds__(256) kb_sum_slot(const SumArgs* __restrict__ A, int K, int n, int o) {
  sum_slot_body(A[blockIdx.y].slot, K, n, o, A[blockIdx.y].st);
}

// ================================================================ row kernels
// physical -> mixed; optional partials sum f, sum |f| (compatibility of S)
template <int NX>
__device__ __forceinline__ void row_r2c_body(Geo g, const double* __restrict__ f, cd* __restrict__ out,
                                                 double* schk) {
  using C = Row2D<NX, 1>;
  __shared__ cd buf[C::NB * C::LS];
  __shared__ double red[2 * (C::NT / 64)];
  const cd* tw = (const cd*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  double2 v[C::EP];
  rowP_gload<C>(v, f, y0, nrow);
  double s[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    if (p < C::RH) {
      buf[(p / C::H) * C::LS + p % C::H] = mk<double>(v[i].x, v[i].y);
      s[0] += v[i].x + v[i].y;
      s[1] += fabs(v[i].x) + fabs(v[i].y);
    }
  }
  __syncthreads();
  lds_fft<double, -1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  rfft_post<double, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  rowT_store<C, 1>(buf, out, nullptr, nullptr, g.ny, y0, nrow);
  if (schk) {
    block_sum<C::NT, 2>(s, red);
    write_partials<C::NT>(schk, s, 2);
  }
}
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 1>::NT)) k_row_r2c(Geo g, const double* __restrict__ f, cd* __restrict__ out,
                                                 double* schk) {
  row_r2c_body<NX>(g, f, out, schk);
}
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 1>::NT)) kb_row_r2c(const RowR2cArgs* __restrict__ A) {
  const RowR2cArgs& a = A[blockIdx.y];
  row_r2c_body<NX>(a.g, (const double*)a.f, (cd*)a.out, (double*)a.schk);
}

// mixed -> physical (unnormalised inverse: the caller folds 1/n into the spectral side)
template <int NX>
__device__ __forceinline__ void row_c2r_body(Geo g, const cd* __restrict__ in, double* __restrict__ f) {
  using C = Row2D<NX, 1>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  cd tv[C::ET];
  rowT_gload<C>(tv, in, nullptr, nullptr, g.ny, y0, nrow);
  rowT_put<C>(buf, tv);
  __syncthreads();
  irfft_pre<double, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  lds_fft<double, +1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  for (int p = threadIdx.x; p < C::RH; p += C::NT) {
    const int rr = p / C::H, j = p % C::H;
    if (rr < nrow) {
      const cd v = buf[rr * C::LS + j];
      *(double2*)(f + (size_t)(y0 + rr) * NX + 2 * j) = make_double2(v.x, v.y);
    }
  }
}
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 1>::NT)) k_row_c2r(Geo g, const cd* __restrict__ in, double* __restrict__ f) {
  row_c2r_body<NX>(g, in, f);
}
// the pressure of a split update written out on its own (see launch_row_split)
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 1>::NT)) kb_row_split_p(const SplitArgs* __restrict__ A) {
  const SplitArgs& a = A[blockIdx.y];
  row_c2r_body<NX>(a.g, (const cd*)a.P, (double*)a.p_out);
}

// Operator middle: gradient fields (mixed) -> physical g -> flux K g -> mixed,
// both components in one batched transform each way.  In place: G0/G1 hold
// grad_x/grad_y on entry and F_x/F_y on exit.  Optional partials: sum mx^2,
// mx my, my^2, r (the preconditioner's Kbar).  Optional lo: FP32 copies of
// m (2n values) followed by r (n values) for the single-precision inner solve.
// In the PCG loop (it >= 1) the pass first takes the stopping decision for the
// residual r_it left by k_col_update: ||r_it||^2 (reduced directly from that
// kernel's partials) <= tol2 * status.bb ends the solve at iteration it.
// T is the arithmetic and storage type of the transforms and fields; the
// reductions are FP64 in both instantiations.
template <int NX, typename T, int RV>
__device__ __forceinline__ void row_flux_body(Geo g, cx<T>* G0, cx<T>* G1, const T* __restrict__ m,
                                                  const T* __restrict__ r, int it, double* kslot, int nwg_col,
                                                  double tol2, float* lo) {
  using C = FluxCfg<NX, RV>;
  using V = cx<T>;
  using P = typename vec2<T>::type;
  if (it >= 0 ? g.st->conv_at <= it : g.st->outer_done != 0) return;
  tclk_start(g, 0, it);
  __shared__ V buf[C::NB * C::LS];
  __shared__ double red[4 * (C::NT / 64)];
  const V* tw = (const V*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  // Tiles of fewer than 1024 threads load the pairs (k, H - k) of each line, so
  // that the pre-processing of the inverse real transform happens on the way
  // into LDS; 1024-thread tiles (at most 128 registers per thread) load the
  // plain transposed image and pre-process in LDS, since the paired form
  // spills there.
  constexpr bool PAIRS = C::NT < 1024;
  constexpr int NA = PAIRS ? RowPairs<C>::ETP : C::ET, NBP = PAIRS ? RowPairs<C>::ETP : 1;
  V ta[NA], tb[NBP];
  if constexpr (PAIRS)
    rowTP_gload<C>(ta, tb, G0, G1, nullptr, g.ny, y0, nrow);
  else
    rowT_gload<C>(ta, G0, G1, nullptr, g.ny, y0, nrow);
  if (it >= 1) {
    double rr[1];
    sum_partials<C::NT, 1>(slot_ptr(g.part, SLOT_RR), nwg_col, MAX_WG, rr, red);
    const double bb = g.st->bb;
    const bool bad = !isfinite(rr[0]);
    if (bad || rr[0] <= tol2 * bb) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        g.st->rr[0] = rr[0];
        g.st->converged = bad ? 0 : 1;
        if (bad) g.st->flags |= FLAG_NONFINITE;
        g.st->conv_at = it;
      }
      return;
    }
  }
  if constexpr (PAIRS) {
    rowTP_put_pre<C>(buf, ta, tb, tw, g.twn);
    __syncthreads();
  } else {
    rowT_put<C>(buf, ta);
    __syncthreads();
    irfft_pre<T, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  }
  lds_fft<T, +1, C::H, C::NB, C::LS, C::NT, C::PLAN>(buf, tw, g.twn);
  // m and r are loaded only now: held across the transform they would cost
  // about 48 registers, and a workgroup with fewer registers shares a compute
  // unit more easily with the passes of concurrent solves
  P mx[C::EP], my[C::EP], rv[C::EP];
  rowP_gload<C>(mx, m, y0, nrow);
  rowP_gload<C>(my, m + n, y0, nrow);
  rowP_gload<C>(rv, r, y0, nrow);
  if (lo) {
#pragma unroll
    for (int i = 0; i < C::EP; ++i) {
      const int p = threadIdx.x + i * C::NT;
      const int rr = p / C::H, j = p % C::H;
      if (p < C::RH && rr < nrow) {
        const size_t o = (size_t)(y0 + rr) * NX + 2 * j;
        *(float2*)(lo + o) = make_float2((float)mx[i].x, (float)mx[i].y);
        *(float2*)(lo + n + o) = make_float2((float)my[i].x, (float)my[i].y);
        *(float2*)(lo + 2 * n + o) = make_float2((float)rv[i].x, (float)rv[i].y);
      }
    }
  }
  double ks[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    if (p < C::RH && rr < nrow) {
      V* px = buf + rr * C::LS + j;
      V* py = buf + (C::R + rr) * C::LS + j;
      const V gx = *px, gy = *py;
      // K g = (m.g) m + r g at the two grid points packed in this element
      const T a0 = mx[i].x * gx.x + my[i].x * gy.x;
      const T a1 = mx[i].y * gx.y + my[i].y * gy.y;
      *px = mk<T>(fma(a0, mx[i].x, rv[i].x * gx.x), fma(a1, mx[i].y, rv[i].y * gx.y));
      *py = mk<T>(fma(a0, my[i].x, rv[i].x * gy.x), fma(a1, my[i].y, rv[i].y * gy.y));
      if (kslot) {
        ks[0] += (double)mx[i].x * mx[i].x + (double)mx[i].y * mx[i].y;
        ks[1] += (double)mx[i].x * my[i].x + (double)mx[i].y * my[i].y;
        ks[2] += (double)my[i].x * my[i].x + (double)my[i].y * my[i].y;
        ks[3] += (double)rv[i].x + (double)rv[i].y;
      }
    }
  }
  __syncthreads();
  lds_fft<T, -1, C::H, C::NB, C::LS, C::NT, C::PLAN>(buf, tw, g.twn);
  // post-processing of the forward real transform on the way out
  if constexpr (PAIRS) {
    rowTP_store_post<C, 2>(buf, G0, G1, nullptr, tw, g.twn, g.ny, y0, nrow);
  } else {
    rfft_post<T, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
    rowT_store<C, 2>(buf, G0, G1, nullptr, g.ny, y0, nrow);
  }
  if (kslot) {
    block_sum<C::NT, 4>(ks, red);
    write_partials<C::NT>(kslot, ks, 4);
  }
  tclk_end(g, 0, it);
}
template <int NX, typename T, int RV>
__global__ void __launch_bounds__((FluxCfg<NX, RV>::NT)) k_row_flux(Geo g, cx<T>* G0, cx<T>* G1, const T* __restrict__ m,
                                                  const T* __restrict__ r, int it, double* kslot, int nwg_col,
                                                  double tol2, float* lo) {
  row_flux_body<NX, T, RV>(g, G0, G1, m, r, it, kslot, nwg_col, tol2, lo);
}
template <int NX, typename T, int RV>
__global__ void __launch_bounds__((FluxCfg<NX, RV>::NT)) kb_row_flux(const FluxArgs* __restrict__ A, int it, int nwg_col, double tol2) {
  const FluxArgs& a = A[blockIdx.y];
  row_flux_body<NX, T, RV>(a.g, (cx<T>*)a.G0, (cx<T>*)a.G1, (const T*)a.m, (const T*)a.r, it, (double*)a.kslot, nwg_col, tol2, (float*)a.lo);
}

// Split update, pointwise part: p = F^-1 x_hat (written out), g = grad p,
// exact activation then exact relaxation of m, forward x transform of the
// result.  In place: P, Gx hold the transformed m_x, m_y on exit.
// WITHP: the three fields (P, Gx, Gy) in one tile, p written here; otherwise
// only Gx, Gy (p is written by a pass of its own before), in the two-row tile
// SplitCfg: rows of 2048 and more hold one row per workgroup with three fields
// (16-byte runs through the mixed layout) but two with two.
template <int NX>
using SplitCfg = RowCfg<NX, 2, NX, 0, ((NX / 8) * 2 >= 1024 ? 2 : 1)>;
template <int NX>
constexpr bool split_separate_p() { return Row2D<NX, 3>::R < 2 && (NX & (NX - 1)) == 0; }
template <int NX, bool WITHP>
using SplitTile = typename std::conditional<WITHP, Row2D<NX, 3>, SplitCfg<NX>>::type;
template <int NX, bool WITHP>
__device__ __forceinline__ void row_split_body(Geo g, cd* P, cd* Gx, const cd* __restrict__ Gy,
                                                   const double* __restrict__ m, double* __restrict__ p_out,
                                                   double c2dt, double gamma, double dt, double relax1) {
  using C = SplitTile<NX, WITHP>;
  constexpr int OFF = WITHP ? C::R : 0;  // first line of Gx
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd tv[C::ET];
  if constexpr (WITHP)
    rowT_gload<C>(tv, P, Gx, Gy, g.ny, y0, nrow);
  else
    rowT_gload<C>(tv, Gx, Gy, nullptr, g.ny, y0, nrow);
  double2 mxv[C::EP], myv[C::EP];
  rowP_gload<C>(mxv, m, y0, nrow);
  rowP_gload<C>(myv, m + n, y0, nrow);
  rowT_put<C>(buf, tv);
  __syncthreads();
  irfft_pre<double, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  lds_fft<double, +1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);

  const double e1 = 1.0 - gamma;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    if (p < C::RH && rr < nrow) {
      // m_x and m_y replace the first two fields' lines
      cd* pp = buf + rr * C::LS + j;
      cd* px = buf + (C::R + rr) * C::LS + j;
      const cd gxv = buf[(OFF + rr) * C::LS + j], gyv = buf[(OFF + C::R + rr) * C::LS + j];
      if constexpr (WITHP) {
        const cd pv = *pp;
        *(double2*)(p_out + (size_t)(y0 + rr) * NX + 2 * j) = make_double2(pv.x, pv.y);
      }
      double mx[2] = {mxv[i].x, mxv[i].y}, my[2] = {myv[i].x, myv[i].y};
      const double gxa[2] = {gxv.x, gxv.y}, gya[2] = {gyv.x, gyv.y};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // activation: m + c^2 dt phi1(c^2 dt |g|^2) (g.m) g, phi1(z) = expm1(z)/z
        const double g2 = gxa[t] * gxa[t] + gya[t] * gya[t];
        const double z = c2dt * g2;
        const double phi = z > 0.0 ? expm1(z) / z : 1.0;
        const double coef = c2dt * phi * (gxa[t] * mx[t] + gya[t] * my[t]);
        double qx = fma(coef, gxa[t], mx[t]);
        double qy = fma(coef, gya[t], my[t]);
        // relaxation: exact decay of |m| along m/|m|
        double fac;
        if (gamma == 1.0) {
          fac = relax1;
        } else {
          const double s2 = qx * qx + qy * qy;
          if (s2 == 0.0) {
            fac = 1.0;
          } else {
            const double u = 2.0 * e1 * dt * exp(-e1 * log(s2));
            fac = (u >= 1.0) ? 0.0 : exp(log1p(-u) / (2.0 * e1));
          }
        }
        qx *= fac;
        qy *= fac;
        if (!isfinite(qx) || !isfinite(qy)) bad = true;
        mx[t] = qx;
        my[t] = qy;
      }
      *pp = mk<double>(mx[0], mx[1]);
      *px = mk<double>(my[0], my[1]);
    }
  }
  if (bad) atomicOr(&g.st->sticky, (int)FLAG_NONFINITE);
  __syncthreads();
  lds_fft<double, -1, C::H, 2 * C::R, C::LS, C::NT>(buf, tw, g.twn);
  rfft_post<double, C::H, 2 * C::R, C::LS, C::NT>(buf, tw, g.twn);
  rowT_store<C, 2>(buf, P, Gx, nullptr, g.ny, y0, nrow);
}
template <int NX, bool WITHP>
__global__ void __launch_bounds__((SplitTile<NX, WITHP>::NT)) k_row_split(Geo g, cd* P, cd* Gx, const cd* __restrict__ Gy,
                                                   const double* __restrict__ m, double* __restrict__ p_out,
                                                   double c2dt, double gamma, double dt, double relax1) {
  row_split_body<NX, WITHP>(g, P, Gx, Gy, m, p_out, c2dt, gamma, dt, relax1);
}
template <int NX, bool WITHP>
__global__ void __launch_bounds__((SplitTile<NX, WITHP>::NT)) kb_row_split(const SplitArgs* __restrict__ A) {
  const SplitArgs& a = A[blockIdx.y];
  row_split_body<NX, WITHP>(a.g, (cd*)a.P, (cd*)a.Gx, (const cd*)a.Gy, (const double*)a.m, (double*)a.p_out, a.c2dt, a.gamma, a.dt, a.relax1);
}

// Last pass of the step: inverse x transform of the diffused m, written over
// m; partials sum (m_new - m_old)^2 and sum m_old^2.
template <int NX>
__device__ __forceinline__ void row_final_body(Geo g, const cd* __restrict__ Mx, const cd* __restrict__ My,
                                                   double* m, double* dslot) {
  using C = Row2D<NX, 2>;
  __shared__ cd buf[C::NB * C::LS];
  __shared__ double red[2 * (C::NT / 64)];
  const cd* tw = (const cd*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd tv[C::ET];
  rowT_gload<C>(tv, Mx, My, nullptr, g.ny, y0, nrow);
  double2 o0[C::EP], o1[C::EP];
  rowP_gload<C>(o0, m, y0, nrow);
  rowP_gload<C>(o1, m + n, y0, nrow);
  rowT_put<C>(buf, tv);
  __syncthreads();
  irfft_pre<double, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  lds_fft<double, +1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  double s[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    if (p < C::RH && rr < nrow) {
      const cd a0 = buf[rr * C::LS + j], a1 = buf[(C::R + rr) * C::LS + j];
      const size_t idx = (size_t)(y0 + rr) * NX + 2 * j;
      const double d0 = a0.x - o0[i].x, d1 = a0.y - o0[i].y;
      const double d2 = a1.x - o1[i].x, d3 = a1.y - o1[i].y;
      s[0] += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
      s[1] += o0[i].x * o0[i].x + o0[i].y * o0[i].y + o1[i].x * o1[i].x + o1[i].y * o1[i].y;
      *(double2*)(m + idx) = make_double2(a0.x, a0.y);
      *(double2*)(m + n + idx) = make_double2(a1.x, a1.y);
    }
  }
  if (dslot) {
    block_sum<C::NT, 2>(s, red);
    write_partials<C::NT>(dslot, s, 2);
  }
}
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 2>::NT)) k_row_final(Geo g, const cd* __restrict__ Mx, const cd* __restrict__ My,
                                                   double* m, double* dslot) {
  row_final_body<NX>(g, Mx, My, m, dslot);
}
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 2>::NT)) kb_row_final(const FinalArgs* __restrict__ A) {
  const FinalArgs& a = A[blockIdx.y];
  row_final_body<NX>(a.g, (const cd*)a.Mx, (const cd*)a.My, (double*)a.m, (double*)a.dslot);
}

// Pointwise energy terms: sum r|g|^2, sum (m.g)^2, sum |m|^{2 gamma}
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 2>::NT)) k_row_energy(Geo g, const cd* __restrict__ Gx, const cd* __restrict__ Gy,
                                                    const double* __restrict__ m, const double* __restrict__ r,
                                                    double gamma, double* eslot) {
  using C = Row2D<NX, 2>;
  __shared__ cd buf[C::NB * C::LS];
  __shared__ double red[3 * (C::NT / 64)];
  const cd* tw = (const cd*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd tv[C::ET];
  rowT_gload<C>(tv, Gx, Gy, nullptr, g.ny, y0, nrow);
  double2 mx[C::EP], my[C::EP], rv[C::EP];
  rowP_gload<C>(mx, m, y0, nrow);
  rowP_gload<C>(my, m + n, y0, nrow);
  rowP_gload<C>(rv, r, y0, nrow);
  rowT_put<C>(buf, tv);
  __syncthreads();
  irfft_pre<double, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  lds_fft<double, +1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    if (p < C::RH && rr < nrow) {
      const cd gxv = buf[rr * C::LS + j], gyv = buf[(C::R + rr) * C::LS + j];
      const double gxa[2] = {gxv.x, gxv.y}, gya[2] = {gyv.x, gyv.y};
      const double mxa[2] = {mx[i].x, mx[i].y}, mya[2] = {my[i].x, my[i].y}, ra[2] = {rv[i].x, rv[i].y};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double mg = mxa[t] * gxa[t] + mya[t] * gya[t];
        s[0] += ra[t] * (gxa[t] * gxa[t] + gya[t] * gya[t]);
        s[1] += mg * mg;
        const double mm = mxa[t] * mxa[t] + mya[t] * mya[t];
        s[2] += (mm == 0.0) ? 0.0 : exp(gamma * log(mm));
      }
    }
  }
  block_sum<C::NT, 3>(s, red);
  write_partials<C::NT>(eslot, s, 3);
}

// ================================================================ adjoint row kernels
// phi1'(z) = (e^z (z - 1) + 1) / z^2, by its Taylor series near 0
__device__ __forceinline__ double dphi1(double z) {
  if (fabs(z) < 1e-3) return 0.5 + z * (1.0 / 3.0 + z * (0.125 + z * (1.0 / 30.0)));
  return (expm1(z) * (z - 1.0) + z) / (z * z);
}

// Reverse of the pointwise part of the split update at one grid point.
// In: m (= m^k), g (= grad p^k), lam2 (= H^T lam^{k+1}, the adjoint after the
// diffusion stage).  Out: lam_m (adjoint of m through activation and
// relaxation) and lam_g (adjoint of g).
__device__ __forceinline__ void adjoint_point(double mx, double my, double gx, double gy, double lx, double ly,
                                              double c2dt, double gamma, double dt, double relax1, double& lmx,
                                              double& lmy, double& lgx, double& lgy) {
  // forward activation intermediates
  const double g2 = gx * gx + gy * gy;
  const double z = c2dt * g2;
  const double kap = c2dt * (z > 0.0 ? expm1(z) / z : 1.0);
  const double dkap = c2dt * dphi1(z);
  const double gm = gx * mx + gy * my;
  const double sx = fma(kap * gm, gx, mx), sy = fma(kap * gm, gy, my);  // m*
  // relaxation Jacobian (symmetric): fac (I - u u^T) + rho' u u^T
  double ax, ay;
  if (gamma == 1.0) {
    ax = relax1 * lx;
    ay = relax1 * ly;
  } else {
    const double s2 = sx * sx + sy * sy;
    const double e1 = 1.0 - gamma;
    if (s2 == 0.0) {
      ax = gamma > 1.0 ? lx : 0.0;
      ay = gamma > 1.0 ? ly : 0.0;
    } else {
      const double u = 2.0 * e1 * dt * exp(-e1 * log(s2));
      if (u >= 1.0) {
        ax = ay = 0.0;
      } else {
        const double fac = exp(log1p(-u) / (2.0 * e1));   // rho / s
        const double drho = exp((1.0 - 2.0 * e1) * log(fac));  // rho'(s) = (s/rho)^{2e-1}
        const double is = 1.0 / sqrt(s2);
        const double ux = sx * is, uy = sy * is;
        const double ul = ux * lx + uy * ly;
        ax = fac * (lx - ux * ul) + drho * ul * ux;
        ay = fac * (ly - uy * ul) + drho * ul * uy;
      }
    }
  }
  // activation: d m*/d m = I + kap g g^T;  d m*/d g as in the oracle
  const double gl = gx * ax + gy * ay;
  lmx = fma(kap * gl, gx, ax);
  lmy = fma(kap * gl, gy, ay);
  const double t = 2.0 * c2dt * dkap * gm * gl;
  lgx = t * gx + kap * gl * mx + kap * gm * ax;
  lgy = t * gy + kap * gl * my + kap * gm * ay;
}

// Adjoint, first pass: c2r of (H lam_x, H lam_y, grad_x p, grad_y p); the
// pointwise reverse of relaxation and activation; lam_m written to lam_out,
// lam_g transformed forward back into A0 / A1 (in place).
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 4>::NT)) k_row_adj1(Geo g, cd* A0, cd* A1, const cd* __restrict__ G0,
                                                      const cd* __restrict__ G1, const double* __restrict__ m,
                                                      double* __restrict__ lam_out, double c2dt, double gamma,
                                                      double dt, double relax1) {
  using C = Row2D<NX, 4>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd tv[C::ET];
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::RH, ee = e % C::RH;
    const int rr = ee % C::R, kx = ee / C::R;
    const cd* src = f == 0 ? A0 : (f == 1 ? A1 : (f == 2 ? G0 : G1));
    tv[i] = (e < 4 * C::RH && rr < nrow) ? src[(size_t)kx * g.ny + y0 + rr] : mk<double>(0.0, 0.0);
  }
  double2 mx[C::EP], my[C::EP];
  rowP_gload<C>(mx, m, y0, nrow);
  rowP_gload<C>(my, m + n, y0, nrow);
  rowT_put<C>(buf, tv);
  __syncthreads();
  irfft_pre<double, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  lds_fft<double, +1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    if (p < C::RH && rr < nrow) {
      cd* plx = buf + rr * C::LS + j;
      cd* ply = buf + (C::R + rr) * C::LS + j;
      const cd lx = *plx, ly = *ply;
      const cd gxv = buf[(2 * C::R + rr) * C::LS + j], gyv = buf[(3 * C::R + rr) * C::LS + j];
      double lm[2][2], lg[2][2];
      adjoint_point(mx[i].x, my[i].x, gxv.x, gyv.x, lx.x, ly.x, c2dt, gamma, dt, relax1, lm[0][0], lm[1][0], lg[0][0],
                    lg[1][0]);
      adjoint_point(mx[i].y, my[i].y, gxv.y, gyv.y, lx.y, ly.y, c2dt, gamma, dt, relax1, lm[0][1], lm[1][1], lg[0][1],
                    lg[1][1]);
      const size_t idx = (size_t)(y0 + rr) * NX + 2 * j;
      *(double2*)(lam_out + idx) = make_double2(lm[0][0], lm[0][1]);
      *(double2*)(lam_out + n + idx) = make_double2(lm[1][0], lm[1][1]);
      *plx = mk<double>(lg[0][0], lg[0][1]);
      *ply = mk<double>(lg[1][0], lg[1][1]);
    }
  }
  __syncthreads();
  lds_fft<double, -1, C::H, 2 * C::R, C::LS, C::NT>(buf, tw, g.twn);
  rfft_post<double, C::H, 2 * C::R, C::LS, C::NT>(buf, tw, g.twn);
  rowT_store<C, 2>(buf, A0, A1, nullptr, g.ny, y0, nrow);
}

// Adjoint, second pass: c2r of (grad mu, grad p); with mu (physical) and m:
// dL/dS += mu, dL/dr -= grad mu . grad p, and
// lam -= (m.grad p) grad mu + (m.grad mu) grad p.
template <int NX>
__global__ void __launch_bounds__((Row2D<NX, 4>::NT)) k_row_adj2(Geo g, const cd* __restrict__ M1, const cd* __restrict__ M2,
                                                      const cd* __restrict__ P1, const cd* __restrict__ P2,
                                                      const double* __restrict__ m, const double* __restrict__ mu,
                                                      double* lam, double* grad_r, double* grad_S) {
  using C = Row2D<NX, 4>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd tv[C::ET];
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::RH, ee = e % C::RH;
    const int rr = ee % C::R, kx = ee / C::R;
    const cd* src = f == 0 ? M1 : (f == 1 ? M2 : (f == 2 ? P1 : P2));
    tv[i] = (e < 4 * C::RH && rr < nrow) ? src[(size_t)kx * g.ny + y0 + rr] : mk<double>(0.0, 0.0);
  }
  double2 mx[C::EP], my[C::EP], muv[C::EP];
  rowP_gload<C>(mx, m, y0, nrow);
  rowP_gload<C>(my, m + n, y0, nrow);
  rowP_gload<C>(muv, mu, y0, nrow);
  rowT_put<C>(buf, tv);
  __syncthreads();
  irfft_pre<double, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  lds_fft<double, +1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    if (p < C::RH && rr < nrow) {
      const cd umx = buf[rr * C::LS + j], umy = buf[(C::R + rr) * C::LS + j];
      const cd upx = buf[(2 * C::R + rr) * C::LS + j], upy = buf[(3 * C::R + rr) * C::LS + j];
      const size_t idx = (size_t)(y0 + rr) * NX + 2 * j;
      double2 gS = *(const double2*)(grad_S + idx);
      double2 gr = *(const double2*)(grad_r + idx);
      double2 l0 = *(const double2*)(lam + idx);
      double2 l1 = *(const double2*)(lam + n + idx);
      gS.x += muv[i].x;
      gS.y += muv[i].y;
      gr.x -= umx.x * upx.x + umy.x * upy.x;
      gr.y -= umx.y * upx.y + umy.y * upy.y;
      const double mgp0 = mx[i].x * upx.x + my[i].x * upy.x, mgp1 = mx[i].y * upx.y + my[i].y * upy.y;
      const double mgm0 = mx[i].x * umx.x + my[i].x * umy.x, mgm1 = mx[i].y * umx.y + my[i].y * umy.y;
      l0.x -= mgp0 * umx.x + mgm0 * upx.x;
      l0.y -= mgp1 * umx.y + mgm1 * upx.y;
      l1.x -= mgp0 * umy.x + mgm0 * upy.x;
      l1.y -= mgp1 * umy.y + mgm1 * upy.y;
      *(double2*)(grad_S + idx) = gS;
      *(double2*)(grad_r + idx) = gr;
      *(double2*)(lam + idx) = l0;
      *(double2*)(lam + n + idx) = l1;
    }
  }
}

// ================================================================ column kernels
// Write the gradient multipliers i xi_c f_hat / n of one spectral value into
// the two gradient lines of the column block.
template <class C, typename T>
__device__ __forceinline__ void put_grad(cx<T>* buf, int c, int ky, int kx, const cx<T> v, const Geo& g) {
  constexpr int NY = C::NYv;
  const T sx = (T)(xi_col(kx, g.lx) * g.inv_n), sy = (T)(xi_tilde(ky, NY, g.ly) * g.inv_n);
  buf[c * C::LS + ky] = mk<T>(-sx * v.y, sx * v.x);
  buf[(C::C + c) * C::LS + ky] = mk<T>(-sy * v.y, sy * v.x);
}

// mixed -> spectral (null modes zeroed unless bit 1 of mode is set); with bit 0
// of mode also the gradient of the result back to mixed:
// Gx = F_y^-1(i xi_x f_hat / n), Gy likewise.
template <int NY>
__device__ __forceinline__ void col_fwd_body(Geo g, cd* in, cd* __restrict__ out, int mode, cd* Gx, cd* Gy) {
  using C = ColCfg<NY, 2>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  cd tv[C::ET];
  colT_gload<C, 1>(tv, in, nullptr, kx0, g.h);
  colT_put<C, 1>(buf, tv);
  __syncthreads();
  lds_fft<double, -1, NY, C::C, C::LS, C::NT>(buf, tw, g.twn);
  cd v[C::EP];
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NY, ky = p % NY;
    cd a = p < C::CN ? buf[c * C::LS + ky] : mk<double>(0.0, 0.0);
    if (!(mode & 2) && kx0 + c == 0 && (ky == 0 || 2 * ky == NY)) a = mk<double>(0.0, 0.0);
    v[i] = a;
    if (p < C::CN && kx0 + c < g.h) out[(size_t)(kx0 + c) * NY + ky] = a;
  }
  if (!(mode & 1)) return;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    if (p < C::CN) put_grad<C>(buf, p / NY, p % NY, kx0 + p / NY, v[i], g);
  }
  __syncthreads();
  lds_fft<double, +1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  colT_store<C, 2>(buf, Gx, Gy, kx0, g.h);
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) k_col_fwd(Geo g, cd* in, cd* __restrict__ out, int mode, cd* Gx, cd* Gy) {
  col_fwd_body<NY>(g, in, out, mode, Gx, Gy);
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) kb_col_fwd(const ColFwdArgs* __restrict__ A, int mode) {
  const ColFwdArgs& a = A[blockIdx.y];
  col_fwd_body<NY>(a.g, (cd*)a.in, (cd*)a.out, mode, (cd*)a.Gx, (cd*)a.Gy);
}

// spectral -> mixed: P = F_y^-1(x_hat / n)  (GRAD false)  or
//                    Gx, Gy as in k_col_fwd (GRAD true)
template <int NY, bool GRAD>
__device__ __forceinline__ void col_grad_body(Geo g, const cd* __restrict__ xh, cd* P, cd* Gx,
                                                               cd* Gy) {
  using C = ColCfg<NY, GRAD ? 2 : 1>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  cd v[C::EP];
  colP_gload<C>(v, xh, kx0, g.h);
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    if (p < C::CN) {
      if (GRAD) put_grad<C>(buf, p / NY, p % NY, kx0 + p / NY, v[i], g);
      else buf[(p / NY) * C::LS + p % NY] = scl(v[i], g.inv_n);
    }
  }
  __syncthreads();
  lds_fft<double, +1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  if (GRAD) colT_store<C, 2>(buf, Gx, Gy, kx0, g.h);
  else colT_store<C, 1>(buf, P, nullptr, kx0, g.h);
}
template <int NY, bool GRAD>
__global__ void __launch_bounds__((ColCfg<NY, GRAD ? 2 : 1>::NT)) k_col_grad(Geo g, const cd* __restrict__ xh, cd* P, cd* Gx,
                                                               cd* Gy) {
  col_grad_body<NY, GRAD>(g, xh, P, Gx, Gy);
}
template <int NY, bool GRAD>
__global__ void __launch_bounds__((ColCfg<NY, GRAD ? 2 : 1>::NT)) kb_col_grad(const ColGradArgs* __restrict__ A) {
  const ColGradArgs& a = A[blockIdx.y];
  col_grad_body<NY, GRAD>(a.g, (const cd*)a.xh, (cd*)a.P, (cd*)a.Gx, (cd*)a.Gy);
}


// Operator end: forward y transform of the fluxes, q_hat = -i xi . F_hat.
// INIT: r_hat = b_hat - q_hat (stored), partials <r,M^-1 r>, <r,r>, <b,b>;
//       also reduces the Kbar and compatibility partials of the row pass.
// else: q_hat stored, partials <d,q>, <q,M^-1 r>, <q,M^-1 q>, <r,M^-1 r> (the
//       inner products the update's alpha and beta need).
// INIT exists for T = double only (the residual of the refinement is FP64).
template <int NY, bool INIT, typename T, int CV>
__device__ __forceinline__ void col_div_body(Geo g, const cx<T>* __restrict__ Fx,
                                                 const cx<T>* __restrict__ Fy, cx<T>* __restrict__ qh,
                                                 const cx<T>* __restrict__ dh, cx<T>* rh,
                                                 const cx<T>* __restrict__ bh, int it, int nwg_row) {
  using C = DivCfg<NY, CV>;
  static_assert(!INIT || CV == VAR_DEFAULT, "the INIT pass uses the default tile");
  using V = cx<T>;
  static_assert(!INIT || sizeof(T) == sizeof(double), "INIT pass is FP64");
  if (INIT ? g.st->outer_done != 0 : g.st->conv_at <= it) return;
  if (!INIT) tclk_start(g, 1, it);
  __shared__ V buf[C::NB * C::LS];
  __shared__ double red[4 * (C::NT / 64)];
  __shared__ double Ks[4];
  const V* tw = (const V*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  V tv[C::ET];
  colT_gload<C, 2>(tv, Fx, Fy, kx0, g.h);
  if (INIT) {
    double kb[4], sc[2];
    sum_partials<C::NT, 4>(slot_ptr(g.part, SLOT_KBAR), nwg_row, MAX_WG, kb, red);
    sum_partials<C::NT, 2>(slot_ptr(g.part, SLOT_SCHK), nwg_row, MAX_WG, sc, red);
    if (threadIdx.x == 0) {
      Ks[0] = kb[0] * g.inv_n + kb[3] * g.inv_n;
      Ks[1] = kb[1] * g.inv_n;
      Ks[2] = kb[2] * g.inv_n + kb[3] * g.inv_n;
      Ks[3] = 0.0;
      if (blockIdx.x == 0) {
        for (int i = 0; i < 4; ++i) g.st->kbar[i] = Ks[i];
        if (fabs(sc[0]) > 1e-12 * sc[1]) atomicOr(&g.st->flags, (int)FLAG_INCOMPAT);
      }
    }
  } else if (threadIdx.x < 4) {
    Ks[threadIdx.x] = g.st->kbar[threadIdx.x];
  }
  colT_put<C, 2>(buf, tv);
  __syncthreads();
  lds_fft<T, -1, NY, C::NB, C::LS, C::NT, C::PLAN>(buf, tw, g.twn);
  // the vectors of the dot products are loaded after the transform (fewer
  // registers held across it)
  V av[C::EP], bv[C::EP];
  if (INIT) {
    colP_gload<C>(av, bh, kx0, g.h);
  } else {
    colP_gload<C>(av, dh, kx0, g.h);
    colP_gload<C>(bv, rh, kx0, g.h);
  }
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NY, ky = p % NY;
    const int kx = kx0 + c;
    if (p < C::CN && kx < g.h) {
      const V fx = buf[c * C::LS + ky], fy = buf[(C::C + c) * C::LS + ky];
      const double xx = xi_col(kx, g.lx);
      const double yy = xi_tilde(ky, NY, g.ly);
      // q = -i (xx Fx + yy Fy)
      const T ax = (T)xx * fx.x + (T)yy * fy.x, ay = (T)xx * fx.y + (T)yy * fy.y;
      const V q = mk<T>(ay, -ax);
      const double w = kx == 0 ? 1.0 : 2.0;
      const double sig = precond_symbol_inv(Ks, xx, yy);
      const size_t idx = (size_t)kx * NY + ky;
      const double qx = q.x, qy = q.y;
      if (INIT) {
        const V b = av[i];
        const V rn = sub(b, q);
        rh[idx] = rn;
        const double rr = (double)rn.x * rn.x + (double)rn.y * rn.y;
        s[0] += w * sig * rr;
        s[1] += w * rr;
        s[2] += w * ((double)b.x * b.x + (double)b.y * b.y);
      } else {
        qh[idx] = q;
        const double dx = av[i].x, dy = av[i].y, rx = bv[i].x, ry = bv[i].y;
        const double qq = qx * qx + qy * qy;
        const double rq = rx * qx + ry * qy;
        s[0] += w * (dx * qx + dy * qy);
        s[1] += w * sig * rq;
        s[2] += w * sig * qq;
        s[3] += w * sig * (rx * rx + ry * ry);
      }
    }
  }
  if (INIT) {
    double s3[3] = {s[0], s[1], s[2]};
    block_sum<C::NT, 3>(s3, red);
    write_partials<C::NT>(slot_ptr(g.part, SLOT_P3INIT), s3, 3);
  } else {
    block_sum<C::NT, 4>(s, red);
    write_partials<C::NT>(slot_ptr(g.part, SLOT_P3), s, 4);
  }
  if (!INIT) tclk_end(g, 1, it);
}
template <int NY, bool INIT, typename T, int CV>
__global__ void __launch_bounds__((DivCfg<NY, CV>::NT)) k_col_div(Geo g, const cx<T>* __restrict__ Fx,
                                                 const cx<T>* __restrict__ Fy, cx<T>* __restrict__ qh,
                                                 const cx<T>* __restrict__ dh, cx<T>* rh,
                                                 const cx<T>* __restrict__ bh, int it, int nwg_row) {
  col_div_body<NY, INIT, T, CV>(g, Fx, Fy, qh, dh, rh, bh, it, nwg_row);
}
template <int NY, bool INIT, typename T, int CV>
__global__ void __launch_bounds__((DivCfg<NY, CV>::NT)) kb_col_div(const DivArgs* __restrict__ A, int it, int nwg_row) {
  const DivArgs& a = A[blockIdx.y];
  col_div_body<NY, INIT, T, CV>(a.g, (const cx<T>*)a.Fx, (const cx<T>*)a.Fy, (cx<T>*)a.qh, (const cx<T>*)a.dh, (cx<T>*)a.rh, (const cx<T>*)a.bh, it, nwg_row);
}

// PCG scalar step + vector update + next direction + its gradient (mixed).
// first: d = M^-1 r.  else: alpha, beta from the partials of k_col_div (the
// new <r,M^-1 r> follows from the expansion of <r - alpha q, M^-1 (r - alpha q)>
// around the directly computed old value; it is used for beta only), then
// x += alpha d, r -= alpha q, d = M^-1 r + beta d.  The stopping test on the
// new residual is taken by the next pass from its direct norm (SLOT_RR).
// The scalars are FP64; the vector updates run in T.  `first` exists for
// T = double only (the single-precision solve starts in k_col_refine_start).
template <int NY, typename T, int CV>
__device__ __forceinline__ void col_update_body(Geo g, int first, cx<T>* xh, cx<T>* rh, cx<T>* dh,
                                                    const cx<T>* __restrict__ qh, cx<T>* Gx, cx<T>* Gy, int it,
                                                    int max_iter, double tol2, int nwg_col) {
  using C = DivCfg<NY, CV>;
  using V = cx<T>;
  DevStatus* st = g.st;
  if (st->conv_at < it) return;
  const int tit = first ? -1 : it;  // timing slot (the first update is not a loop pass)
  tclk_start(g, 2, tit);
  __shared__ V buf[C::NB * C::LS];
  __shared__ double red[7 * (C::NT / 64)];
  const V* tw = (const V*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
  double K[4];
  for (int i = 0; i < 4; ++i) K[i] = st->kbar[i];
  // vectors of the block, loaded before the scalar reduction so that both
  // latencies overlap
  V xv[C::EP], rv0[C::EP], dv0[C::EP], qv[C::EP];
  colP_gload<C>(rv0, rh, kx0, g.h);
  if (!first) {
    colP_gload<C>(xv, xh, kx0, g.h);
    colP_gload<C>(dv0, dh, kx0, g.h);
    colP_gload<C>(qv, qh, kx0, g.h);
  }
  double alpha = 0.0, beta = 0.0;
  bool stop = false, zero_x = false;
  if (first) {
    double s[3];
    sum_partials<C::NT, 3>(slot_ptr(g.part, SLOT_P3INIT), nwg_col, MAX_WG, s, red);
    const double rho = s[0], rr = s[1], bb = s[2];
    const bool incompat = (st->flags & FLAG_INCOMPAT) != 0;
    zero_x = (bb == 0.0);
    const bool bad = !isfinite(rr) || !isfinite(bb);
    const bool conv = !bad && (incompat || zero_x || rr <= tol2 * bb);
    if (bad) zero_x = false;
    if (lead) {
      st->rho[0] = rho;
      st->rr[0] = zero_x ? 0.0 : rr;
      st->rr0 = rr;
      st->bb = bb;
      st->iters = 0;
      if (bad) st->flags |= FLAG_NONFINITE;
      if (conv || bad || max_iter <= 0) {
        st->conv_at = 0;
        st->converged = conv ? 1 : 0;
      }
    }
    if (!zero_x && (conv || bad || max_iter <= 0)) return;
    stop = zero_x;
  } else {
    // rho = <r,M^-1 r> of the residual the last operator pass read, computed
    // directly from it
    double s[4];
    sum_partials<C::NT, 4>(slot_ptr(g.part, SLOT_P3), nwg_col, MAX_WG, s, red);
    const double rho = s[3];
    alpha = rho / s[0];
    const double rhon = rho - 2.0 * alpha * s[1] + alpha * alpha * s[2];
    beta = rhon / rho;
    const bool bad = !isfinite(rhon) || !isfinite(alpha);
    stop = bad || it >= max_iter || it >= st->budget;
    if (lead) {
      if (bad) st->flags |= FLAG_NONFINITE;
      st->rho[it & 1] = rhon;
      st->iters = it;
      if (stop) {
        st->conv_at = it;
        st->converged = 0;
      }
    }
  }
  const T a = (T)alpha, bt = (T)beta;
  double rrp[1] = {0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NY, ky = p % NY;
    const int kx = kx0 + c;
    V d = vzero<V>();
    if (p < C::CN && kx < g.h) {
      const size_t idx = (size_t)kx * NY + ky;
      if (zero_x) {
        xh[idx] = vzero<V>();
      } else {
        V rv = rv0[i];
        if (!first) {
          d = dv0[i];
          xh[idx] = add(xv[i], scl(d, a));
          rv = sub(rv, scl(qv[i], a));
          rh[idx] = rv;
          rrp[0] += (kx == 0 ? 1.0 : 2.0) * ((double)rv.x * rv.x + (double)rv.y * rv.y);
        }
        if (!stop) {
          const T sig = (T)precond_symbol_inv(K, xi_col(kx, g.lx), xi_tilde(ky, NY, g.ly));
          d = add(scl(rv, sig), scl(d, bt));
          dh[idx] = d;
        }
      }
    }
    if (!stop && p < C::CN) put_grad<C>(buf, c, ky, kx, d, g);
  }
  if (!first && !zero_x) {
    block_sum<C::NT, 1>(rrp, red);
    write_partials<C::NT>(slot_ptr(g.part, SLOT_RR), rrp, 1);
  }
  if (stop) {
    tclk_end(g, 2, tit);
    return;
  }
  __syncthreads();
  lds_fft<T, +1, NY, C::NB, C::LS, C::NT, C::PLAN>(buf, tw, g.twn);
  colT_store<C, 2>(buf, Gx, Gy, kx0, g.h);
  tclk_end(g, 2, tit);
}
template <int NY, typename T, int CV>
__global__ void __launch_bounds__((DivCfg<NY, CV>::NT)) k_col_update(Geo g, int first, cx<T>* xh, cx<T>* rh, cx<T>* dh,
                                                    const cx<T>* __restrict__ qh, cx<T>* Gx, cx<T>* Gy, int it,
                                                    int max_iter, double tol2, int nwg_col) {
  col_update_body<NY, T, CV>(g, first, xh, rh, dh, qh, Gx, Gy, it, max_iter, tol2, nwg_col);
}
template <int NY, typename T, int CV>
__global__ void __launch_bounds__((DivCfg<NY, CV>::NT)) kb_col_update(const UpdArgs* __restrict__ A, int first, int it, int max_iter, double tol2, int nwg_col) {
  const UpdArgs& a = A[blockIdx.y];
  col_update_body<NY, T, CV>(a.g, first, (cx<T>*)a.xh, (cx<T>*)a.rh, (cx<T>*)a.dh, (const cx<T>*)a.qh, (cx<T>*)a.Gx, (cx<T>*)a.Gy, it, max_iter, tol2, nwg_col);
}

// Start of one correction of the mixed-precision solve (iterative refinement
// of A x = b: the inner solve A e = r runs in FP32, x and the residual
// r = b - A x in FP64).  Reads the FP64 residual partials <r,M^-1 r>, <r,r>,
// <b,b> left by the FP64 operator pass.  If ||r||^2 <= tol2 ||b||^2 (or b = 0,
// or S is incompatible, or the values are not finite) the solve is over: the
// status records the outcome and every later inner launch is a no-op.
// Otherwise the inner right-hand side is r / ||r|| in FP32, the inner
// iterate starts at 0, its first direction is M^-1 r with the gradient of it
// in the FP32 mixed buffers, and the inner stopping threshold (a relative
// residual of tol_in on the unit right-hand side, kept in status.bb for the
// passes' test with tol2 = 1) asks for the reduction that reaches tol2 with a
// margin of 2, but no less than `floor_in`.  A residual no smaller than the
// previous correction's means the refinement has stalled: the solve ends
// unconverged, as it does when max_iter FP32 iterations have been spent.
// Instances that have finished repeat their final decision unchanged (their
// residual passes are skipped), so a batch can run until all have finished.
// Status fields read here are written only by other launches.
template <int NY>
__device__ __forceinline__ void col_refine_start_body(Geo g, const cd* __restrict__ r64, cd* x64,
                                                          cx<float>* x32, cx<float>* r32, cx<float>* d32,
                                                          cx<float>* Gx, cx<float>* Gy, double tol2,
                                                          double floor_in, int max_iter, int nwg_col) {
  using C = ColCfg<NY, 2>;
  using V = cx<float>;
  DevStatus* st = g.st;
  __shared__ V buf[C::NB * C::LS];
  __shared__ double red[3 * (C::NT / 64)];
  const V* tw = (const V*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
  double K[4];
  for (int i = 0; i < 4; ++i) K[i] = st->kbar[i];
  cd rv[C::EP];
  colP_gload<C>(rv, r64, kx0, g.h);
  double s[3];
  sum_partials<C::NT, 3>(slot_ptr(g.part, SLOT_P3INIT), nwg_col, MAX_WG, s, red);
  const double rho = s[0], rr = s[1], bb = s[2];
  const int budget = max_iter - st->itot;
  const double rr_cap = st->orr_prev;
  const bool incompat = (st->flags & FLAG_INCOMPAT) != 0;
  const bool bad = !isfinite(rr) || !isfinite(bb);
  const bool zero_b = !bad && bb == 0.0;
  const bool conv = !bad && (incompat || zero_b || rr <= tol2 * bb);
  if (conv || bad || budget <= 0 || rr >= rr_cap) {
    if (lead) {
      st->rr[0] = zero_b ? 0.0 : rr;
      st->bb = bb;
      st->orr = zero_b ? 0.0 : rr;
      st->obb = bb;
      if (bad) st->flags |= FLAG_NONFINITE;
      st->conv_at = 0;
      st->converged = conv ? 1 : 0;
      st->iters = 0;
      st->outer_done = 1;
    }
    if (zero_b) {
#pragma unroll
      for (int i = 0; i < C::EP; ++i) {
        const int p = threadIdx.x + i * C::NT;
        const int kx = kx0 + p / NY;
        if (p < C::CN && kx < g.h) x64[(size_t)kx * NY + p % NY] = mk<double>(0.0, 0.0);
      }
    }
    return;
  }
  const double scale = 1.0 / sqrt(rr);
  double tin = 0.5 * sqrt(tol2 * bb / rr);
  tin = tin < floor_in ? floor_in : (tin > 0.5 ? 0.5 : tin);
  if (lead) {
    st->orr = rr;
    st->obb = bb;
    st->rscale = sqrt(rr);
    st->bb = tin * tin;
    st->rho[0] = rho * scale * scale;
    st->rr[0] = 1.0;
    st->rr0 = 1.0;
    st->iters = 0;
    st->budget = budget;
    st->converged = 0;
    st->conv_at = INT_MAX;
  }
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NY, ky = p % NY;
    const int kx = kx0 + c;
    V d = vzero<V>();
    if (p < C::CN && kx < g.h) {
      const size_t idx = (size_t)kx * NY + ky;
      const double sig = precond_symbol_inv(K, xi_col(kx, g.lx), xi_tilde(ky, NY, g.ly));
      const double ux = rv[i].x * scale, uy = rv[i].y * scale;
      r32[idx] = mk<float>((float)ux, (float)uy);
      d = mk<float>((float)(sig * ux), (float)(sig * uy));
      d32[idx] = d;
      x32[idx] = vzero<V>();
    }
    if (p < C::CN) put_grad<C>(buf, c, ky, kx, d, g);
  }
  __syncthreads();
  lds_fft<float, +1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  colT_store<C, 2>(buf, Gx, Gy, kx0, g.h);
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) k_col_refine_start(Geo g, const cd* __restrict__ r64, cd* x64,
                                                          cx<float>* x32, cx<float>* r32, cx<float>* d32,
                                                          cx<float>* Gx, cx<float>* Gy, double tol2,
                                                          double floor_in, int max_iter, int nwg_col) {
  col_refine_start_body<NY>(g, r64, x64, x32, r32, d32, Gx, Gy, tol2, floor_in, max_iter, nwg_col);
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) kb_col_refine_start(const RefStartArgs* __restrict__ A, double tol2, double floor_in, int max_iter, int nwg_col) {
  const RefStartArgs& a = A[blockIdx.y];
  col_refine_start_body<NY>(a.g, (const cd*)a.r64, (cd*)a.x64, (cx<float>*)a.x32, (cx<float>*)a.r32, (cx<float>*)a.d32, (cx<float>*)a.Gx, (cx<float>*)a.Gy, tol2, floor_in, max_iter, nwg_col);
}

// End of one correction: x64 += ||r|| e32 (status.rscale), then the gradient
// of the new x64 into the FP64 mixed buffers for the next residual; the
// correction's FP32 iterations are added to the total.  No-op for a finished
// solve.
template <int NY>
__device__ __forceinline__ void col_refine_acc_body(Geo g, cd* x64, const cx<float>* __restrict__ x32,
                                                        cd* Gx, cd* Gy) {
  using C = ColCfg<NY, 2>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  if (g.st->outer_done) return;
  const double sc = g.st->rscale;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g.st->itot += g.st->iters;
    g.st->orr_prev = g.st->orr;
  }
  cd xv[C::EP];
  cx<float> ev[C::EP];
  colP_gload<C>(xv, x64, kx0, g.h);
  colP_gload<C>(ev, x32, kx0, g.h);
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NY, ky = p % NY;
    const int kx = kx0 + c;
    cd x = mk<double>(0.0, 0.0);
    if (p < C::CN && kx < g.h) {
      x = mk<double>(fma(sc, (double)ev[i].x, xv[i].x), fma(sc, (double)ev[i].y, xv[i].y));
      x64[(size_t)kx * NY + ky] = x;
    }
    if (p < C::CN) put_grad<C>(buf, c, ky, kx, x, g);
  }
  __syncthreads();
  lds_fft<double, +1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  colT_store<C, 2>(buf, Gx, Gy, kx0, g.h);
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) k_col_refine_acc(Geo g, cd* x64, const cx<float>* __restrict__ x32,
                                                        cd* Gx, cd* Gy) {
  col_refine_acc_body<NY>(g, x64, x32, Gx, Gy);
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) kb_col_refine_acc(const RefAccArgs* __restrict__ A) {
  const RefAccArgs& a = A[blockIdx.y];
  col_refine_acc_body<NY>(a.g, (cd*)a.x64, (const cx<float>*)a.x32, (cd*)a.Gx, (cd*)a.Gy);
}

// Diffusion: forward y transform, multiply by exp(-D^2 |xi|^2 dt) / n (the
// packed column is unpacked into its kx = 0 and kx = Nx/2 halves for this),
// inverse y transform; both components batched.  Optional partial sum
// w |xi_tilde|^2 |m_hat_new|^2.
template <int NY>
__device__ __forceinline__ void col_heat_body(Geo g, cd* Mx, cd* My, double D2dt, double* eslot) {
  using C = ColCfg<NY, 2>;
  __shared__ cd buf[C::NB * C::LS];
  __shared__ double red[1 * (C::NT / 64)];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  const double xnyq = TWO_PI * (g.nx / 2) / g.lx;  // full wavenumber of the kx = Nx/2 column
  cd tv[C::ET];
  colT_gload<C, 2>(tv, Mx, My, kx0, g.h);
  colT_put<C, 2>(buf, tv);
  __syncthreads();
  lds_fft<double, -1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  double s[1] = {0.0};
  cd v[2][C::EP];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
#pragma unroll
    for (int i = 0; i < C::EP; ++i) {
      const int p = threadIdx.x + i * C::NT;
      const int c = p / NY, ky = p % NY;
      const int kx = kx0 + c;
      if (p >= C::CN) continue;
      const double yf = xi_full(ky, NY, g.ly);
      const cd* line = buf + (f * C::C + c) * C::LS;
      const cd a = line[ky];
      cd out;
      if (kx == 0) {
        const cd b = line[ky == 0 ? 0 : NY - ky];
        const double hA = exp(-D2dt * (yf * yf)) * g.inv_n;
        const double hB = exp(-D2dt * (xnyq * xnyq + yf * yf)) * g.inv_n;
        // P' = (hA+hB)/2 P(ky) + (hA-hB)/2 conj P(-ky)
        out = add(scl(a, 0.5 * (hA + hB)), scl(conj(b), 0.5 * (hA - hB)));
      } else {
        const double xx = TWO_PI * kx / g.lx;
        out = scl(a, exp(-D2dt * (xx * xx + yf * yf)) * g.inv_n);
      }
      v[f][i] = out;
      if (eslot && kx < g.h) {
        const double xt = xi_col(kx, g.lx), yt = xi_tilde(ky, NY, g.ly);
        const double w = kx == 0 ? 1.0 : 2.0;
        s[0] += w * (xt * xt + yt * yt) * (out.x * out.x + out.y * out.y);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < 2; ++f) {
#pragma unroll
    for (int i = 0; i < C::EP; ++i) {
      const int p = threadIdx.x + i * C::NT;
      if (p < C::CN) buf[(f * C::C + p / NY) * C::LS + p % NY] = v[f][i];
    }
  }
  __syncthreads();
  lds_fft<double, +1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  colT_store<C, 2>(buf, Mx, My, kx0, g.h);
  if (eslot) {
    block_sum<C::NT, 1>(s, red);
    write_partials<C::NT>(eslot, s, 1);
  }
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) k_col_heat(Geo g, cd* Mx, cd* My, double D2dt, double* eslot) {
  col_heat_body<NY>(g, Mx, My, D2dt, eslot);
}
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) kb_col_heat(const HeatArgs* __restrict__ A) {
  const HeatArgs& a = A[blockIdx.y];
  col_heat_body<NY>(a.g, (cd*)a.Mx, (cd*)a.My, a.D2dt, (double*)a.eslot);
}

// Adjoint right-hand side: b_hat = Pi F(G^T v) = -i xi_tilde . F(v) for the
// two mixed fields of v (null modes vanish since xi_tilde does).
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) k_col_divrhs(Geo g, const cd* __restrict__ V0, const cd* __restrict__ V1,
                                                        cd* __restrict__ bh) {
  using C = ColCfg<NY, 2>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  cd tv[C::ET];
  colT_gload<C, 2>(tv, V0, V1, kx0, g.h);
  colT_put<C, 2>(buf, tv);
  __syncthreads();
  lds_fft<double, -1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  for (int p = threadIdx.x; p < C::CN; p += C::NT) {
    const int c = p / NY, ky = p % NY;
    const int kx = kx0 + c;
    if (kx < g.h) {
      const cd fx = buf[c * C::LS + ky], fy = buf[(C::C + c) * C::LS + ky];
      const double xx = xi_col(kx, g.lx), yy = xi_tilde(ky, NY, g.ly);
      const double ax = xx * fx.x + yy * fy.x, ay = xx * fx.y + yy * fy.y;
      bh[(size_t)kx * NY + ky] = mk<double>(ay, -ax);
    }
  }
}

__global__ void k_zero_d(double* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Parseval sum w |xi_tilde|^2 |f_hat|^2 over two mixed fields (||grad m||^2 * n)
template <int NY>
__global__ void __launch_bounds__((ColCfg<NY, 2>::NT)) k_col_gradnorm(Geo g, const cd* __restrict__ Mx, const cd* __restrict__ My,
                                                      double* eslot) {
  using C = ColCfg<NY, 2>;
  __shared__ cd buf[C::NB * C::LS];
  __shared__ double red[1 * (C::NT / 64)];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  cd tv[C::ET];
  colT_gload<C, 2>(tv, Mx, My, kx0, g.h);
  colT_put<C, 2>(buf, tv);
  __syncthreads();
  lds_fft<double, -1, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  double s[1] = {0.0};
  for (int e = threadIdx.x; e < 2 * C::CN; e += C::NT) {
    const int f = e / C::CN, ee = e % C::CN;
    const int c = ee / NY, ky = ee % NY;
    const int kx = kx0 + c;
    if (kx < g.h) {
      const cd a = buf[(f * C::C + c) * C::LS + ky];
      const double xt = xi_col(kx, g.lx), yt = xi_tilde(ky, NY, g.ly);
      const double w = kx == 0 ? 1.0 : 2.0;
      s[0] += w * (xt * xt + yt * yt) * (a.x * a.x + a.y * a.y);
    }
  }
  block_sum<C::NT, 1>(s, red);
  write_partials<C::NT>(eslot, s, 1);
}

// ================================================================ launchers
#define NF_DISPATCH(N, MACRO)                \
  switch (N) {                               \
    case 8: MACRO(8); break;                 \
    case 16: MACRO(16); break;               \
    case 32: MACRO(32); break;               \
    case 64: MACRO(64); break;               \
    case 128: MACRO(128); break;             \
    case 256: MACRO(256); break;             \
    case 512: MACRO(512); break;             \
    case 1024: MACRO(1024); break;           \
    case 2048: MACRO(2048); break;           \
    case 4096: MACRO(4096); break;           \
    case 50: MACRO(50); break;               \
    case 100: MACRO(100); break;             \
    case 200: MACRO(200); break;             \
    case 400: MACRO(400); break;             \
    case 800: MACRO(800); break;             \
    case 1600: MACRO(1600); break;           \
    default: return hipErrorInvalidValue;    \
  }

// Launch through hipExtLaunchKernelGGL when a start/stop event pair is given
// (the events are then timestamped by the dispatch itself).
#define NF_LAUNCH(K, GRID, BLK, S, E0, E1, ...)                                   \
  do {                                                                             \
    if (E0) hipExtLaunchKernelGGL(K, GRID, BLK, 0, S, E0, E1, 0, __VA_ARGS__);     \
    else hipLaunchKernelGGL(K, GRID, BLK, 0, S, __VA_ARGS__);                      \
  } while (0)

static int row_threads(int nx, int nf) {
  const int t = row_tile(nx, nf) / 8 * nf;
  return t > 1024 ? 1024 : t;
}
static int row_nwg(const Geo& g, int nf) {
  const int R = tile_rows(g.nx / 2, row_tile(g.nx, nf));
  return (g.ny + R - 1) / R;
}
static int col_cols(int ny) {
  int c = TILE / ny;
  return c < 1 ? 1 : (c > 64 ? 64 : c);
}
// workgroups of the 2D row passes over one or two fields (the writers of row partials)
int row_nwg(const Geo& g) { return row_nwg(g, 2); }
int col_nwg(const Geo& g) {
  const int C = col_cols(g.ny);
  return (g.h + C - 1) / C;
}
int row_nwg_var(const Geo& g, int rv) {
  if (rv == VAR_DEFAULT) return row_nwg(g, 2);
  const int R = rv_rows(g.nx, rv);
  return (g.ny + R - 1) / R;
}
int col_nwg_var(const Geo& g, int cv) {
  if (cv == VAR_DEFAULT) return col_nwg(g);
  const int C = cv_cols(g.ny, cv);
  return (g.h + C - 1) / C;
}
bool flux_var_valid(const Geo& g, bool f32, int rv) {
  if (rv == VAR_DEFAULT) return true;
  const int es = f32 ? 8 : 16;
  return var_size(g.nx) && g.nz == 1 && rv_ok(g.nx, g.ny, rv, es);
}
bool div_var_valid(const Geo& g, bool f32, int cv) {
  if (cv == VAR_DEFAULT) return true;
  const int es = f32 ? 8 : 16;
  return var_size(g.ny) && g.nz == 1 && cv_ok(g.ny, g.h, cv, es);
}
__global__ void k_fill_d(double* p, size_t n, double v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_doubles(double* p, size_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Variant dispatch of the PCG-loop passes: a switch over the variant code that
// instantiates only the variants that exist for the size and real type.
template <int NX, typename T, int RV>
static hipError_t flux_go(const Geo& g, cx<T>* G0, cx<T>* G1, const T* m, const T* r, int it, double* kslot,
                          int nwg_col, double tol2, float* lo, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (flux_var_exists<NX, RV, (int)sizeof(cx<T>)>()) {
    const dim3 grid(row_nwg_var(g, RV)), blk(FluxCfg<NX, RV>::NT);
    NF_LAUNCH((k_row_flux<NX, T, RV>), grid, blk, s, e0, e1, g, G0, G1, m, r, it, kslot, nwg_col, tol2, lo);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}
template <int NX, typename T>
static hipError_t flux_var(int rv, const Geo& g, cx<T>* G0, cx<T>* G1, const T* m, const T* r, int it,
                           double* kslot, int nwg_col, double tol2, float* lo, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  switch (rv) {
#define V_(K) \
  case K: return flux_go<NX, T, K>(g, G0, G1, m, r, it, kslot, nwg_col, tol2, lo, s, e0, e1);
    V_(0) V_(1) V_(2) V_(3) V_(4) V_(5) V_(6) V_(7) V_(8) V_(9) V_(10) V_(11)
#undef V_
    default: return hipErrorInvalidValue;
  }
}
template <int NX, typename T, int RV>
static hipError_t fluxb_go(const Geo& g, const FluxArgs* A, int count, int it, int nwg_col, double tol2,
                           hipStream_t s) {
  if constexpr (flux_var_exists<NX, RV, (int)sizeof(cx<T>)>()) {
    const dim3 grid(row_nwg_var(g, RV), count), blk(FluxCfg<NX, RV>::NT);
    hipLaunchKernelGGL((kb_row_flux<NX, T, RV>), grid, blk, 0, s, A, it, nwg_col, tol2);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}
template <int NX, typename T>
static hipError_t fluxb_var(int rv, const Geo& g, const FluxArgs* A, int count, int it, int nwg_col, double tol2,
                            hipStream_t s) {
  switch (rv) {
#define V_(K) \
  case K: return fluxb_go<NX, T, K>(g, A, count, it, nwg_col, tol2, s);
    V_(0) V_(1) V_(2) V_(3) V_(4) V_(5) V_(6) V_(7) V_(8) V_(9) V_(10) V_(11)
#undef V_
    default: return hipErrorInvalidValue;
  }
}
template <int NY, typename T, int CV>
static hipError_t div_go(const Geo& g, const cx<T>* Fx, const cx<T>* Fy, cx<T>* qh, const cx<T>* dh, cx<T>* rh,
                         int it, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (div_var_exists<NY, CV, (int)sizeof(cx<T>)>()) {
    const dim3 grid(col_nwg_var(g, CV)), blk(DivCfg<NY, CV>::NT);
    NF_LAUNCH((k_col_div<NY, false, T, CV>), grid, blk, s, e0, e1, g, Fx, Fy, qh, dh, rh, (const cx<T>*)nullptr, it,
              0);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}
template <int NY, typename T>
static hipError_t div_var(int cv, const Geo& g, const cx<T>* Fx, const cx<T>* Fy, cx<T>* qh, const cx<T>* dh,
                          cx<T>* rh, int it, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (cv) {
#define V_(K) \
  case K: return div_go<NY, T, K>(g, Fx, Fy, qh, dh, rh, it, s, e0, e1);
    V_(0) V_(1) V_(2) V_(3) V_(4) V_(5) V_(6) V_(7) V_(8) V_(9) V_(10) V_(11)
#undef V_
    default: return hipErrorInvalidValue;
  }
}
template <int NY, typename T, int CV>
static hipError_t divb_go(const Geo& g, const DivArgs* A, int count, int it, hipStream_t s) {
  if constexpr (div_var_exists<NY, CV, (int)sizeof(cx<T>)>()) {
    const dim3 grid(col_nwg_var(g, CV), count), blk(DivCfg<NY, CV>::NT);
    hipLaunchKernelGGL((kb_col_div<NY, false, T, CV>), grid, blk, 0, s, A, it, 0);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}
template <int NY, typename T>
static hipError_t divb_var(int cv, const Geo& g, const DivArgs* A, int count, int it, hipStream_t s) {
  switch (cv) {
#define V_(K) \
  case K: return divb_go<NY, T, K>(g, A, count, it, s);
    V_(0) V_(1) V_(2) V_(3) V_(4) V_(5) V_(6) V_(7) V_(8) V_(9) V_(10) V_(11)
#undef V_
    default: return hipErrorInvalidValue;
  }
}
template <int NY, typename T, int CV>
static hipError_t upd_go(const Geo& g, int first, cx<T>* xh, cx<T>* rh, cx<T>* dh, const cx<T>* qh, cx<T>* Gx,
                         cx<T>* Gy, int it, int max_iter, double tol2, int nwg, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  if constexpr (div_var_exists<NY, CV, (int)sizeof(cx<T>)>()) {
    const dim3 grid(col_nwg_var(g, CV)), blk(DivCfg<NY, CV>::NT);
    NF_LAUNCH((k_col_update<NY, T, CV>), grid, blk, s, e0, e1, g, first, xh, rh, dh, qh, Gx, Gy, it, max_iter, tol2,
              nwg);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}
template <int NY, typename T>
static hipError_t upd_var(int cv, const Geo& g, int first, cx<T>* xh, cx<T>* rh, cx<T>* dh, const cx<T>* qh,
                          cx<T>* Gx, cx<T>* Gy, int it, int max_iter, double tol2, int nwg, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1) {
  switch (cv) {
#define V_(K) \
  case K: return upd_go<NY, T, K>(g, first, xh, rh, dh, qh, Gx, Gy, it, max_iter, tol2, nwg, s, e0, e1);
    V_(0) V_(1) V_(2) V_(3) V_(4) V_(5) V_(6) V_(7) V_(8) V_(9) V_(10) V_(11)
#undef V_
    default: return hipErrorInvalidValue;
  }
}
template <int NY, typename T, int CV>
static hipError_t updb_go(const Geo& g, const UpdArgs* A, int count, int first, int it, int max_iter, double tol2,
                          int nwg, hipStream_t s) {
  if constexpr (div_var_exists<NY, CV, (int)sizeof(cx<T>)>()) {
    const dim3 grid(col_nwg_var(g, CV), count), blk(DivCfg<NY, CV>::NT);
    hipLaunchKernelGGL((kb_col_update<NY, T, CV>), grid, blk, 0, s, A, first, it, max_iter, tol2, nwg);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}
template <int NY, typename T>
static hipError_t updb_var(int cv, const Geo& g, const UpdArgs* A, int count, int first, int it, int max_iter,
                           double tol2, int nwg, hipStream_t s) {
  switch (cv) {
#define V_(K) \
  case K: return updb_go<NY, T, K>(g, A, count, first, it, max_iter, tol2, nwg, s);
    V_(0) V_(1) V_(2) V_(3) V_(4) V_(5) V_(6) V_(7) V_(8) V_(9) V_(10) V_(11)
#undef V_
    default: return hipErrorInvalidValue;
  }
}
// variant codes in use (a variant that cannot run on this grid falls back to the default)
static int use_rv(const Geo& g, bool f32, int it) {
  const int rv = it >= 0 ? g.var_flux[f32 ? 1 : 0] : VAR_DEFAULT;
  return flux_var_valid(g, f32, rv) ? rv : VAR_DEFAULT;
}
static int use_cvd(const Geo& g, bool f32) {
  const int cv = g.var_div[f32 ? 1 : 0];
  return div_var_valid(g, f32, cv) ? cv : VAR_DEFAULT;
}
static int use_cvu(const Geo& g, bool f32) {
  const int cv = g.var_upd[f32 ? 1 : 0];
  return div_var_valid(g, f32, cv) ? cv : VAR_DEFAULT;
}
int rr_nwg(const Geo& g, bool f32) { return col_nwg_var(g, use_cvu(g, f32)); }
int flux_var_rows(const Geo& g, int rv) {
  return rv == VAR_DEFAULT ? tile_rows(g.nx / 2, row_tile(g.nx, 2)) : rv_rows(g.nx, rv);
}
int flux_var_plan(int rv) { return rv_plan(rv); }
int flux_var_threads(const Geo& g, int rv) {
  const int rt = rv == VAR_DEFAULT ? row_tile(g.nx, 2) : rv_rows(g.nx, rv) * (g.nx / 2);
  const int nt = (rt / 8) * 2 > 1024 ? 1024 : (rt / 8) * 2;
  return nt / (rv == VAR_DEFAULT ? 1 : rv_td(rv));
}
int div_var_cols(const Geo& g, int cv) { return cv == VAR_DEFAULT ? col_cols(g.ny) : cv_cols(g.ny, cv); }
int div_var_threads(const Geo& g, int cv) { return cv == VAR_DEFAULT ? col_threads(g.ny, 2) : 2 * TPF * cv_tm(cv); }
bool var_grid(const Geo& g) { return g.nz == 1 && (var_size(g.nx) || var_size(g.ny)); }

hipError_t launch_status_reset(const Geo& g, int full, hipStream_t s) {
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, s, g.st, full);
  return hipGetLastError();
}
hipError_t launch_zero_spec(const Geo& g, void* xh, hipStream_t s) {
  const size_t n = (size_t)g.h * g.ny;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (cd*)xh, n);
  return hipGetLastError();
}
hipError_t launch_sum_slot(const Geo& g, const double* slot, int K, int n, int o, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_slot, dim3(1), dim3(256), 0, s, slot, K, n, o, g.st);
  return hipGetLastError();
}

hipError_t launch_row_r2c(const Geo& g, const double* f, void* out, double* schk, hipStream_t s) {
  const dim3 grid(row_nwg(g, 1)), blk(row_threads(g.nx, 1));
#define L_(N) hipLaunchKernelGGL(k_row_r2c<N>, grid, blk, 0, s, g, f, (cd*)out, schk)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_c2r(const Geo& g, const void* in, double* f, hipStream_t s) {
  const dim3 grid(row_nwg(g, 1)), blk(row_threads(g.nx, 1));
#define L_(N) hipLaunchKernelGGL(k_row_c2r<N>, grid, blk, 0, s, g, (const cd*)in, f)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
// The operator middle: the initial pass (it < 0, which may write the Kbar
// partials read with the default workgroup count) uses the default tile, the
// loop passes the tuned variant; the stopping test of the loop reads the
// partials of the update's variant.
hipError_t launch_row_flux(const Geo& g, void* G0, void* G1, const double* m, const double* r, int it,
                           double* kslot, double tol2, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* lo) {
  const int rv = use_rv(g, false, it);
  const int nwg_col = rr_nwg(g, false);
#define L_(N) return flux_var<N, double>(rv, g, (cd*)G0, (cd*)G1, m, r, it, kslot, nwg_col, tol2, lo, s, e0, e1)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipErrorInvalidValue;
}
hipError_t launch_row_flux32(const Geo& g, void* G0, void* G1, const float* m32, const float* r32, int it,
                             double tol2, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int rv = use_rv(g, true, it);
  const int nwg_col = rr_nwg(g, true);
#define L_(N)                                                                                                  \
  return flux_var<N, float>(rv, g, (cx<float>*)G0, (cx<float>*)G1, m32, r32, it, (double*)nullptr, nwg_col,    \
                            tol2, (float*)nullptr, s, e0, e1)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipErrorInvalidValue;
}
// Split update, pointwise part.  Where the three-field tile holds one row per
// workgroup (rows of 2048 and more), p is written by a one-field pass first and
// the activation and relaxation run in the two-field, two-row tile: the same
// bytes in runs of twice the length.
template <int NX>
static hipError_t split_go(const Geo& g, void* P, void* Gx, void* Gy, const double* m, double* p_out, double c2dt,
                           double gamma, double dt, double relax1, hipStream_t s) {
  if constexpr (split_separate_p<NX>()) {
    hipLaunchKernelGGL(k_row_c2r<NX>, dim3(row_nwg(g, 1)), dim3(row_threads(g.nx, 1)), 0, s, g, (const cd*)P, p_out);
    const int R = SplitCfg<NX>::R;
    hipLaunchKernelGGL((k_row_split<NX, false>), dim3((g.ny + R - 1) / R), dim3(SplitCfg<NX>::NT), 0, s, g, (cd*)P,
                       (cd*)Gx, (const cd*)Gy, m, p_out, c2dt, gamma, dt, relax1);
  } else {
    hipLaunchKernelGGL((k_row_split<NX, true>), dim3(row_nwg(g, 3)), dim3(row_threads(g.nx, 3)), 0, s, g, (cd*)P,
                       (cd*)Gx, (const cd*)Gy, m, p_out, c2dt, gamma, dt, relax1);
  }
  return hipGetLastError();
}
hipError_t launch_row_split(const Geo& g, void* P, void* Gx, void* Gy, const double* m, double* p_out,
                            double c2dt, double gamma, double dt, double relax1, hipStream_t s) {
#define L_(N) return split_go<N>(g, P, Gx, Gy, m, p_out, c2dt, gamma, dt, relax1, s)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipErrorInvalidValue;
}
hipError_t launch_row_final(const Geo& g, const void* Mx, const void* My, double* m, double* dslot,
                            hipStream_t s) {
  const dim3 grid(row_nwg(g, 2)), blk(row_threads(g.nx, 2));
#define L_(N) hipLaunchKernelGGL(k_row_final<N>, grid, blk, 0, s, g, (const cd*)Mx, (const cd*)My, m, dslot)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_energy(const Geo& g, const void* Gx, const void* Gy, const double* m, const double* r,
                             double gamma, double* slot, hipStream_t s) {
  const dim3 grid(row_nwg(g, 2)), blk(row_threads(g.nx, 2));
#define L_(N) \
  hipLaunchKernelGGL(k_row_energy<N>, grid, blk, 0, s, g, (const cd*)Gx, (const cd*)Gy, m, r, gamma, slot)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_col_fwd(const Geo& g, void* in, void* out, int with_grad, void* Gx, void* Gy, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(col_threads(g.ny, 2));
#define L_(N) hipLaunchKernelGGL(k_col_fwd<N>, grid, blk, 0, s, g, (cd*)in, (cd*)out, with_grad, (cd*)Gx, (cd*)Gy)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_grad(const Geo& g, const void* xh, void* P, void* Gx, void* Gy, hipStream_t s) {
  const dim3 grid(col_nwg(g));
  if (P) {
#define L_(N) hipLaunchKernelGGL((k_col_grad<N, false>), grid, dim3(col_threads(g.ny, 1)), 0, s, g, (const cd*)xh, (cd*)P, (cd*)Gx, (cd*)Gy)
    NF_DISPATCH(g.ny, L_)
#undef L_
  }
  if (Gx) {
#define L_(N) hipLaunchKernelGGL((k_col_grad<N, true>), grid, dim3(col_threads(g.ny, 2)), 0, s, g, (const cd*)xh, (cd*)P, (cd*)Gx, (cd*)Gy)
    NF_DISPATCH(g.ny, L_)
#undef L_
  }
  return hipGetLastError();
}
// The operator end: the initial (INIT) pass uses the default tile, the loop
// passes the tuned variant.
hipError_t launch_col_div(const Geo& g, int init, const void* Fx, const void* Fy, void* qh, const void* dh,
                          void* rh, const void* bh, int it, int nwg_row, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
  if (init) {
    const dim3 grid(col_nwg(g)), blk(col_threads(g.ny, 2));
#define L_(N)                                                                                                  \
  NF_LAUNCH((k_col_div<N, true, double, VAR_DEFAULT>), grid, blk, s, e0, e1, g, (const cd*)Fx, (const cd*)Fy,  \
            (cd*)qh, (const cd*)dh, (cd*)rh, (const cd*)bh, it, nwg_row)
    NF_DISPATCH(g.ny, L_)
#undef L_
    return hipGetLastError();
  }
  const int cv = use_cvd(g, false);
#define L_(N) \
  return div_var<N, double>(cv, g, (const cd*)Fx, (const cd*)Fy, (cd*)qh, (const cd*)dh, (cd*)rh, it, s, e0, e1)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipErrorInvalidValue;
}
hipError_t launch_col_div32(const Geo& g, const void* Fx, const void* Fy, void* qh, const void* dh, void* rh, int it,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  typedef cx<float> cf;
  const int cv = use_cvd(g, true);
#define L_(N) \
  return div_var<N, float>(cv, g, (const cf*)Fx, (const cf*)Fy, (cf*)qh, (const cf*)dh, (cf*)rh, it, s, e0, e1)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipErrorInvalidValue;
}
// The update: the first one reads the partials of the INIT pass (default
// tile), the others those of the operator end's variant.
hipError_t launch_col_update(const Geo& g, int first, void* xh, void* rh, void* dh, const void* qh, void* Gx,
                             void* Gy, int it, int max_iter, double tol2, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
  const int cv = use_cvu(g, false);
  const int nwg = first ? col_nwg(g) : col_nwg_var(g, use_cvd(g, false));
#define L_(N)                                                                                                    \
  return upd_var<N, double>(cv, g, first, (cd*)xh, (cd*)rh, (cd*)dh, (const cd*)qh, (cd*)Gx, (cd*)Gy, it,        \
                            max_iter, tol2, nwg, s, e0, e1)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipErrorInvalidValue;
}
hipError_t launch_col_update32(const Geo& g, void* xh, void* rh, void* dh, const void* qh, void* Gx, void* Gy, int it,
                               int max_iter, double tol2, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  typedef cx<float> cf;
  const int cv = use_cvu(g, true);
  const int nwg = col_nwg_var(g, use_cvd(g, true));
#define L_(N)                                                                                                    \
  return upd_var<N, float>(cv, g, 0, (cf*)xh, (cf*)rh, (cf*)dh, (const cf*)qh, (cf*)Gx, (cf*)Gy, it, max_iter,  \
                           tol2, nwg, s, e0, e1)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipErrorInvalidValue;
}
hipError_t launch_col_refine_start(const Geo& g, const void* r64, void* x64, void* x32, void* r32, void* d32,
                                   void* Gx, void* Gy, double tol2, double floor_in, int max_iter, hipStream_t s) {
  typedef cx<float> cf;
  const dim3 grid(col_nwg(g)), blk(col_threads(g.ny, 2));
  const int nwg = col_nwg(g);
#define L_(N)                                                                                                 \
  hipLaunchKernelGGL(k_col_refine_start<N>, grid, blk, 0, s, g, (const cd*)r64, (cd*)x64, (cf*)x32, (cf*)r32,  \
                     (cf*)d32, (cf*)Gx, (cf*)Gy, tol2, floor_in, max_iter, nwg)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_refine_acc(const Geo& g, void* x64, const void* x32, void* Gx, void* Gy, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(col_threads(g.ny, 2));
#define L_(N)                                                                                                 \
  hipLaunchKernelGGL(k_col_refine_acc<N>, grid, blk, 0, s, g, (cd*)x64, (const cx<float>*)x32, (cd*)Gx, (cd*)Gy)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_heat(const Geo& g, void* Mx, void* My, double D2dt, double* eslot, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(col_threads(g.ny, 2));
#define L_(N) hipLaunchKernelGGL(k_col_heat<N>, grid, blk, 0, s, g, (cd*)Mx, (cd*)My, D2dt, eslot)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_gradnorm(const Geo& g, const void* Mx, const void* My, double* eslot, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(col_threads(g.ny, 2));
#define L_(N) hipLaunchKernelGGL(k_col_gradnorm<N>, grid, blk, 0, s, g, (const cd*)Mx, (const cd*)My, eslot)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}

// ---------------------------------------------------------------- batched launchers
hipError_t launchb_status_reset(DevStatus* st0, int count, int full, hipStream_t s) {
  hipLaunchKernelGGL(kb_status_reset, dim3(count), dim3(64), 0, s, st0, full);
  return hipGetLastError();
}
hipError_t launchb_sum_slot(const SumArgs* A, int count, int K, int n, int o, hipStream_t s) {
  hipLaunchKernelGGL(kb_sum_slot, dim3(1, count), dim3(256), 0, s, A, K, n, o);
  return hipGetLastError();
}
hipError_t launchb_row_r2c(const Geo& g, const RowR2cArgs* A, int count, hipStream_t s) {
  const dim3 grid(row_nwg(g, 1), count), blk(row_threads(g.nx, 1));
#define L_(N) hipLaunchKernelGGL(kb_row_r2c<N>, grid, blk, 0, s, A)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launchb_col_fwd(const Geo& g, const ColFwdArgs* A, int count, int mode, hipStream_t s) {
  const dim3 grid(col_nwg(g), count), blk(col_threads(g.ny, 2));
#define L_(N) hipLaunchKernelGGL(kb_col_fwd<N>, grid, blk, 0, s, A, mode)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launchb_col_grad(const Geo& g, const ColGradArgs* A, int count, bool grad, hipStream_t s) {
  const dim3 grid(col_nwg(g), count);
  if (grad) {
#define L_(N) hipLaunchKernelGGL((kb_col_grad<N, true>), grid, dim3(col_threads(g.ny, 2)), 0, s, A)
    NF_DISPATCH(g.ny, L_)
#undef L_
  } else {
#define L_(N) hipLaunchKernelGGL((kb_col_grad<N, false>), grid, dim3(col_threads(g.ny, 1)), 0, s, A)
    NF_DISPATCH(g.ny, L_)
#undef L_
  }
  return hipGetLastError();
}
hipError_t launchb_row_flux(const Geo& g, bool f32, const FluxArgs* A, int count, int it, double tol2,
                            hipStream_t s) {
  const int rv = use_rv(g, f32, it);
  const int nwg_col = rr_nwg(g, f32);
  if (f32) {
#define L_(N) return fluxb_var<N, float>(rv, g, A, count, it, nwg_col, tol2, s)
    NF_DISPATCH(g.nx, L_)
#undef L_
  } else {
#define L_(N) return fluxb_var<N, double>(rv, g, A, count, it, nwg_col, tol2, s)
    NF_DISPATCH(g.nx, L_)
#undef L_
  }
  return hipErrorInvalidValue;
}
hipError_t launchb_col_div(const Geo& g, bool f32, bool init, const DivArgs* A, int count, int it, hipStream_t s) {
  if (init) {
    const dim3 grid(col_nwg(g), count), blk(col_threads(g.ny, 2));
    const int nwg_row = row_nwg(g);
#define L_(N) hipLaunchKernelGGL((kb_col_div<N, true, double, VAR_DEFAULT>), grid, blk, 0, s, A, it, nwg_row)
    NF_DISPATCH(g.ny, L_)
#undef L_
    return hipGetLastError();
  }
  const int cv = use_cvd(g, f32);
  if (f32) {
#define L_(N) return divb_var<N, float>(cv, g, A, count, it, s)
    NF_DISPATCH(g.ny, L_)
#undef L_
  } else {
#define L_(N) return divb_var<N, double>(cv, g, A, count, it, s)
    NF_DISPATCH(g.ny, L_)
#undef L_
  }
  return hipErrorInvalidValue;
}
hipError_t launchb_col_update(const Geo& g, bool f32, const UpdArgs* A, int count, int first, int it, int max_iter,
                              double tol2, hipStream_t s) {
  const int cv = use_cvu(g, f32);
  const int nwg = (first && !f32) ? col_nwg(g) : col_nwg_var(g, use_cvd(g, f32));
  if (f32) {
#define L_(N) return updb_var<N, float>(cv, g, A, count, 0, it, max_iter, tol2, nwg, s)
    NF_DISPATCH(g.ny, L_)
#undef L_
  } else {
#define L_(N) return updb_var<N, double>(cv, g, A, count, first, it, max_iter, tol2, nwg, s)
    NF_DISPATCH(g.ny, L_)
#undef L_
  }
  return hipErrorInvalidValue;
}
template <int NX>
static hipError_t splitb_go(const Geo& g, const SplitArgs* A, int count, hipStream_t s) {
  if constexpr (split_separate_p<NX>()) {
    hipLaunchKernelGGL(kb_row_split_p<NX>, dim3(row_nwg(g, 1), count), dim3(row_threads(g.nx, 1)), 0, s, A);
    const int R = SplitCfg<NX>::R;
    hipLaunchKernelGGL((kb_row_split<NX, false>), dim3((g.ny + R - 1) / R, count), dim3(SplitCfg<NX>::NT), 0, s, A);
  } else {
    hipLaunchKernelGGL((kb_row_split<NX, true>), dim3(row_nwg(g, 3), count), dim3(row_threads(g.nx, 3)), 0, s, A);
  }
  return hipGetLastError();
}
hipError_t launchb_row_split(const Geo& g, const SplitArgs* A, int count, hipStream_t s) {
#define L_(N) return splitb_go<N>(g, A, count, s)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipErrorInvalidValue;
}
hipError_t launchb_col_heat(const Geo& g, const HeatArgs* A, int count, hipStream_t s) {
  const dim3 grid(col_nwg(g), count), blk(col_threads(g.ny, 2));
#define L_(N) hipLaunchKernelGGL(kb_col_heat<N>, grid, blk, 0, s, A)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launchb_row_final(const Geo& g, const FinalArgs* A, int count, hipStream_t s) {
  const dim3 grid(row_nwg(g, 2), count), blk(row_threads(g.nx, 2));
#define L_(N) hipLaunchKernelGGL(kb_row_final<N>, grid, blk, 0, s, A)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launchb_col_refine_start(const Geo& g, const RefStartArgs* A, int count, double tol2, double floor_in,
                                    int max_iter, hipStream_t s) {
  const dim3 grid(col_nwg(g), count), blk(col_threads(g.ny, 2));
  const int nwg = col_nwg(g);
#define L_(N) hipLaunchKernelGGL(kb_col_refine_start<N>, grid, blk, 0, s, A, tol2, floor_in, max_iter, nwg)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launchb_col_refine_acc(const Geo& g, const RefAccArgs* A, int count, hipStream_t s) {
  const dim3 grid(col_nwg(g), count), blk(col_threads(g.ny, 2));
#define L_(N) hipLaunchKernelGGL(kb_col_refine_acc<N>, grid, blk, 0, s, A)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}

}  // namespace nf

namespace nf {
hipError_t launch_row_adj1(const Geo& g, void* A0, void* A1, const void* G0, const void* G1, const double* m,
                           double* lam_out, double c2dt, double gamma, double dt, double relax1, hipStream_t s) {
  const dim3 grid(row_nwg(g, 4)), blk(row_threads(g.nx, 4));
#define L_(N)                                                                                                    \
  hipLaunchKernelGGL(k_row_adj1<N>, grid, blk, 0, s, g, (cd*)A0, (cd*)A1, (const cd*)G0, (const cd*)G1, m, lam_out, \
                     c2dt, gamma, dt, relax1)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_adj2(const Geo& g, const void* M1, const void* M2, const void* P1, const void* P2,
                           const double* m, const double* mu, double* lam, double* grad_r, double* grad_S,
                           hipStream_t s) {
  const dim3 grid(row_nwg(g, 4)), blk(row_threads(g.nx, 4));
#define L_(N)                                                                                                 \
  hipLaunchKernelGGL(k_row_adj2<N>, grid, blk, 0, s, g, (const cd*)M1, (const cd*)M2, (const cd*)P1,           \
                     (const cd*)P2, m, mu, lam, grad_r, grad_S)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_divrhs(const Geo& g, const void* V0, const void* V1, void* bh, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(col_threads(g.ny, 2));
#define L_(N) hipLaunchKernelGGL(k_col_divrhs<N>, grid, blk, 0, s, g, (const cd*)V0, (const cd*)V1, (cd*)bh)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_zero_doubles(double* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
}  // namespace nf
