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
#include <climits>

#include "nf_fft.hpp"
#include "nf_internal.h"

namespace nf {

typedef cx<double> cd;

static constexpr double TWO_PI = 6.283185307179586476925286766559;

// ---------------------------------------------------------------- tile configs
template <int NX>
struct RowCfg {
  static constexpr int H = NX / 2;
  static constexpr int R0 = 2048 / H;
  static constexpr int R = R0 < 1 ? 1 : (R0 > 64 ? 64 : R0);  // rows per workgroup
  static constexpr int NT = 256;
  static constexpr int LS = H + 1;                              // padded LDS line stride
  static constexpr int E = (R * H + NT - 1) / NT;               // complex elements per thread
};

template <int NY>
struct ColCfg {
  static constexpr int C0 = 2048 / NY;
  static constexpr int C = C0 < 1 ? 1 : (C0 > 64 ? 64 : C0);   // columns per workgroup
  static constexpr int NT = 256;
  static constexpr int LS = NY;
  static constexpr int E = (C * NY + NT - 1) / NT;
};

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

// ---------------------------------------------------------------- row helpers
// mixed [kx][y] (global) -> LDS lines [row][kx]
template <int NX>
__device__ __forceinline__ void row_load_mixed(cd* buf, const cd* __restrict__ src, int ny, int y0, int nrow) {
  using C = RowCfg<NX>;
  for (int e = threadIdx.x; e < C::R * C::H; e += C::NT) {
    const int rr = e % C::R, kx = e / C::R;
    if (rr < nrow) buf[rr * C::LS + kx] = src[(size_t)kx * ny + y0 + rr];
  }
}
template <int NX>
__device__ __forceinline__ void row_store_mixed(const cd* buf, cd* __restrict__ dst, int ny, int y0, int nrow) {
  using C = RowCfg<NX>;
  for (int e = threadIdx.x; e < C::R * C::H; e += C::NT) {
    const int rr = e % C::R, kx = e / C::R;
    if (rr < nrow) dst[(size_t)kx * ny + y0 + rr] = buf[rr * C::LS + kx];
  }
}
// inverse x transform of the block in LDS (mixed -> physical pairs, times Nx)
template <int NX>
__device__ __forceinline__ void row_c2r(cd* buf, const cd* tw, int twlog) {
  using C = RowCfg<NX>;
  irfft_pre<double, C::H, C::R, C::LS, C::NT>(buf, tw, twlog);
  lds_fft<double, +1, C::H, C::R, C::LS, C::NT>(buf, tw, twlog);
}
// forward x transform of the block in LDS (physical pairs -> mixed)
template <int NX>
__device__ __forceinline__ void row_r2c(cd* buf, const cd* tw, int twlog) {
  using C = RowCfg<NX>;
  lds_fft<double, -1, C::H, C::R, C::LS, C::NT>(buf, tw, twlog);
  rfft_post<double, C::H, C::R, C::LS, C::NT>(buf, tw, twlog);
}

// ---------------------------------------------------------------- column helpers
template <int NY>
__device__ __forceinline__ void col_load(cd* buf, const cd* __restrict__ src, int kx0, int h) {
  using C = ColCfg<NY>;
  for (int e = threadIdx.x; e < C::C * NY; e += C::NT) {
    const int c = e / NY, ky = e % NY;
    if (kx0 + c < h) buf[c * C::LS + ky] = src[(size_t)(kx0 + c) * NY + ky];
  }
}
template <int NY>
__device__ __forceinline__ void col_store(const cd* buf, cd* __restrict__ dst, int kx0, int h) {
  using C = ColCfg<NY>;
  for (int e = threadIdx.x; e < C::C * NY; e += C::NT) {
    const int c = e / NY, ky = e % NY;
    if (kx0 + c < h) dst[(size_t)(kx0 + c) * NY + ky] = buf[c * C::LS + ky];
  }
}

__device__ __forceinline__ void write_partials(double* slot, const double* v, int K) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) slot[(size_t)k * MAX_WG + blockIdx.x] = v[k];
  }
}

// ================================================================ small kernels
__global__ void k_status_reset(DevStatus* st, int full) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (full) st->sticky = 0;
    for (int i = 0; i < 4; ++i) st->kbar[i] = 0.0;
    st->bb = 0.0;
    st->rho[0] = st->rho[1] = 0.0;
    st->rr[0] = st->rr[1] = 0.0;
    st->rr0 = 0.0;
    for (int i = 0; i < 16; ++i) st->out[i] = 0.0;
    st->conv_at = INT_MAX;
    st->converged = 0;
    st->iters = 0;
    st->flags = 0;
  }
}

__global__ void k_zero(cd* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = mk<double>(0.0, 0.0);
}

__global__ void __launch_bounds__(256) k_sum_slot(const double* __restrict__ slot, int K, int n, int o, DevStatus* st) {
  __shared__ double scratch[8 * 4];
  double v[8];
  for (int k = 0; k < 8; ++k) v[k] = 0.0;
  for (int k = 0; k < K; ++k)
    for (int i = threadIdx.x; i < n; i += 256) v[k] += slot[(size_t)k * MAX_WG + i];
  block_sum<256, 8>(v, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) st->out[o + k] = v[k];
}

// ================================================================ row kernels
// physical -> mixed; optional partials sum f, sum |f| (compatibility of S)
template <int NX>
__global__ void __launch_bounds__(256) k_row_r2c(Geo g, const double* __restrict__ f, cd* __restrict__ out,
                                                 double* schk) {
  using C = RowCfg<NX>;
  __shared__ cd buf[C::R * C::LS];
  __shared__ double red[2 * 4];
  const cd* tw = (const cd*)g.tw;
  const int y0 = blockIdx.x * C::R;
  const int nrow = min(C::R, g.ny - y0);
  double s[2] = {0.0, 0.0};
  for (int e = threadIdx.x; e < C::R * C::H; e += C::NT) {
    const int rr = e / C::H, j = e % C::H;
    if (rr < nrow) {
      const double2 v = *(const double2*)(f + (size_t)(y0 + rr) * NX + 2 * j);
      buf[rr * C::LS + j] = mk<double>(v.x, v.y);
      s[0] += v.x + v.y;
      s[1] += fabs(v.x) + fabs(v.y);
    }
  }
  __syncthreads();
  row_r2c<NX>(buf, tw, g.twlog);
  row_store_mixed<NX>(buf, out, g.ny, y0, nrow);
  if (schk) {
    block_sum<C::NT, 2>(s, red);
    write_partials(schk, s, 2);
  }
}

// mixed -> physical (times 1: the caller folds 1/n into the spectral side)
template <int NX>
__global__ void __launch_bounds__(256) k_row_c2r(Geo g, const cd* __restrict__ in, double* __restrict__ f) {
  using C = RowCfg<NX>;
  __shared__ cd buf[C::R * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int y0 = blockIdx.x * C::R;
  const int nrow = min(C::R, g.ny - y0);
  row_load_mixed<NX>(buf, in, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
  for (int e = threadIdx.x; e < C::R * C::H; e += C::NT) {
    const int rr = e / C::H, j = e % C::H;
    if (rr < nrow) {
      const cd v = buf[rr * C::LS + j];
      *(double2*)(f + (size_t)(y0 + rr) * NX + 2 * j) = make_double2(v.x, v.y);
    }
  }
}

// Operator middle: gradient fields (mixed) -> physical g -> flux K g -> mixed.
// In place: G0/G1 hold grad_x/grad_y on entry and F_x/F_y on exit.
// Optional partials: sum mx^2, mx my, my^2, r (the preconditioner's Kbar).
// In the PCG loop (it >= 1) the pass first takes the stopping decision for the
// residual r_it left by k_col_update: ||r_it||^2 (reduced directly from that
// kernel's partials) <= tol2 ||b||^2 ends the solve at iteration it.
template <int NX>
__global__ void __launch_bounds__(256) k_row_flux(Geo g, cd* G0, cd* G1, const double* __restrict__ m,
                                                  const double* __restrict__ r, int it, double* kslot, int nwg_col,
                                                  double tol2) {
  using C = RowCfg<NX>;
  if (it >= 0 && g.st->conv_at <= it) return;
  __shared__ cd buf[C::R * C::LS];
  __shared__ double red[4 * 4];
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
  const cd* tw = (const cd*)g.tw;
  const int y0 = blockIdx.x * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd gx[C::E], gy[C::E];

  row_load_mixed<NX>(buf, G0, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) gx[i] = buf[(e / C::H) * C::LS + e % C::H];
  }
  __syncthreads();
  row_load_mixed<NX>(buf, G1, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) gy[i] = buf[(e / C::H) * C::LS + e % C::H];
  }
  __syncthreads();

  double ks[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int rr = e / C::H, j = e % C::H;
    if (e < C::R * C::H && rr < nrow) {
      const size_t idx = (size_t)(y0 + rr) * NX + 2 * j;
      const double2 mx = *(const double2*)(m + idx);
      const double2 my = *(const double2*)(m + n + idx);
      const double2 rv = *(const double2*)(r + idx);
      // K g = (m.g) m + r g at the two grid points packed in this element
      const double a0 = mx.x * gx[i].x + my.x * gy[i].x;
      const double a1 = mx.y * gx[i].y + my.y * gy[i].y;
      const cd fx = mk<double>(fma(a0, mx.x, rv.x * gx[i].x), fma(a1, mx.y, rv.y * gx[i].y));
      const cd fy = mk<double>(fma(a0, my.x, rv.x * gy[i].x), fma(a1, my.y, rv.y * gy[i].y));
      gx[i] = fx;
      gy[i] = fy;
      if (kslot) {
        ks[0] += mx.x * mx.x + mx.y * mx.y;
        ks[1] += mx.x * my.x + mx.y * my.y;
        ks[2] += my.x * my.x + my.y * my.y;
        ks[3] += rv.x + rv.y;
      }
    }
  }
  // forward x transform of F_x, then F_y
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) buf[(e / C::H) * C::LS + e % C::H] = gx[i];
  }
  __syncthreads();
  row_r2c<NX>(buf, tw, g.twlog);
  row_store_mixed<NX>(buf, G0, g.ny, y0, nrow);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) buf[(e / C::H) * C::LS + e % C::H] = gy[i];
  }
  __syncthreads();
  row_r2c<NX>(buf, tw, g.twlog);
  row_store_mixed<NX>(buf, G1, g.ny, y0, nrow);
  if (kslot) {
    block_sum<C::NT, 4>(ks, red);
    write_partials(kslot, ks, 4);
  }
}

// Split update, pointwise part: p = F^-1 x_hat (written out), g = grad p,
// exact activation then exact relaxation of m, forward x transform of the
// result.  In place: P, Gx hold the transformed m_x, m_y on exit.
template <int NX>
__global__ void __launch_bounds__(256) k_row_split(Geo g, cd* P, cd* Gx, const cd* __restrict__ Gy,
                                                   const double* __restrict__ m, double* __restrict__ p_out,
                                                   double c2dt, double gamma, double dt, double relax1) {
  using C = RowCfg<NX>;
  __shared__ cd buf[C::R * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int y0 = blockIdx.x * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd gx[C::E], gy[C::E];

  // pressure: write p to the caller's buffer
  row_load_mixed<NX>(buf, P, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
  for (int e = threadIdx.x; e < C::R * C::H; e += C::NT) {
    const int rr = e / C::H, j = e % C::H;
    if (rr < nrow) {
      const cd v = buf[rr * C::LS + j];
      *(double2*)(p_out + (size_t)(y0 + rr) * NX + 2 * j) = make_double2(v.x, v.y);
    }
  }
  __syncthreads();
  row_load_mixed<NX>(buf, Gx, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) gx[i] = buf[(e / C::H) * C::LS + e % C::H];
  }
  __syncthreads();
  row_load_mixed<NX>(buf, Gy, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) gy[i] = buf[(e / C::H) * C::LS + e % C::H];
  }
  __syncthreads();

  const double e1 = 1.0 - gamma;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int rr = e / C::H, j = e % C::H;
    if (e < C::R * C::H && rr < nrow) {
      const size_t idx = (size_t)(y0 + rr) * NX + 2 * j;
      const double2 mxv = *(const double2*)(m + idx);
      const double2 myv = *(const double2*)(m + n + idx);
      double mx[2] = {mxv.x, mxv.y}, my[2] = {myv.x, myv.y};
      const double gxa[2] = {gx[i].x, gx[i].y}, gya[2] = {gy[i].x, gy[i].y};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // activation: m + c^2 dt phi1(c^2 dt |g|^2) (g.m) g, phi1(z) = expm1(z)/z
        const double g2 = gxa[t] * gxa[t] + gya[t] * gya[t];
        const double z = c2dt * g2;
        const double phi = z > 0.0 ? expm1(z) / z : 1.0;
        const double coef = c2dt * phi * (gxa[t] * mx[t] + gya[t] * my[t]);
        double ax = fma(coef, gxa[t], mx[t]);
        double ay = fma(coef, gya[t], my[t]);
        // relaxation: exact decay of |m| along m/|m|
        double fac;
        if (gamma == 1.0) {
          fac = relax1;
        } else {
          const double s2 = ax * ax + ay * ay;
          if (s2 == 0.0) {
            fac = 1.0;
          } else {
            const double u = 2.0 * e1 * dt * exp(-e1 * log(s2));
            fac = (u >= 1.0) ? 0.0 : exp(log1p(-u) / (2.0 * e1));
          }
        }
        ax *= fac;
        ay *= fac;
        if (!isfinite(ax) || !isfinite(ay)) bad = true;
        mx[t] = ax;
        my[t] = ay;
      }
      gx[i] = mk<double>(mx[0], mx[1]);
      gy[i] = mk<double>(my[0], my[1]);
    }
  }
  if (bad) atomicOr(&g.st->sticky, (int)FLAG_NONFINITE);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) buf[(e / C::H) * C::LS + e % C::H] = gx[i];
  }
  __syncthreads();
  row_r2c<NX>(buf, tw, g.twlog);
  row_store_mixed<NX>(buf, P, g.ny, y0, nrow);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) buf[(e / C::H) * C::LS + e % C::H] = gy[i];
  }
  __syncthreads();
  row_r2c<NX>(buf, tw, g.twlog);
  row_store_mixed<NX>(buf, Gx, g.ny, y0, nrow);
}

// Last pass of the step: inverse x transform of the diffused m, written over
// m; partials sum (m_new - m_old)^2 and sum m_old^2.
template <int NX>
__global__ void __launch_bounds__(256) k_row_final(Geo g, const cd* __restrict__ Mx, const cd* __restrict__ My,
                                                   double* m, double* dslot) {
  using C = RowCfg<NX>;
  __shared__ cd buf[C::R * C::LS];
  __shared__ double red[2 * 4];
  const cd* tw = (const cd*)g.tw;
  const int y0 = blockIdx.x * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  double s[2] = {0.0, 0.0};
  for (int comp = 0; comp < 2; ++comp) {
    row_load_mixed<NX>(buf, comp == 0 ? Mx : My, g.ny, y0, nrow);
    __syncthreads();
    row_c2r<NX>(buf, tw, g.twlog);
    for (int e = threadIdx.x; e < C::R * C::H; e += C::NT) {
      const int rr = e / C::H, j = e % C::H;
      if (rr < nrow) {
        const cd v = buf[rr * C::LS + j];
        double* dst = m + comp * n + (size_t)(y0 + rr) * NX + 2 * j;
        const double2 old = *(const double2*)dst;
        const double d0 = v.x - old.x, d1 = v.y - old.y;
        s[0] += d0 * d0 + d1 * d1;
        s[1] += old.x * old.x + old.y * old.y;
        *(double2*)dst = make_double2(v.x, v.y);
      }
    }
    __syncthreads();
  }
  if (dslot) {
    block_sum<C::NT, 2>(s, red);
    write_partials(dslot, s, 2);
  }
}

// Pointwise energy terms: sum r|g|^2, sum (m.g)^2, sum |m|^{2 gamma}
template <int NX>
__global__ void __launch_bounds__(256) k_row_energy(Geo g, const cd* __restrict__ Gx, const cd* __restrict__ Gy,
                                                    const double* __restrict__ m, const double* __restrict__ r,
                                                    double gamma, double* eslot) {
  using C = RowCfg<NX>;
  __shared__ cd buf[C::R * C::LS];
  __shared__ double red[3 * 4];
  const cd* tw = (const cd*)g.tw;
  const int y0 = blockIdx.x * C::R;
  const int nrow = min(C::R, g.ny - y0);
  const size_t n = (size_t)g.nx * g.ny;
  cd gx[C::E], gy[C::E];
  row_load_mixed<NX>(buf, Gx, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) gx[i] = buf[(e / C::H) * C::LS + e % C::H];
  }
  __syncthreads();
  row_load_mixed<NX>(buf, Gy, g.ny, y0, nrow);
  __syncthreads();
  row_c2r<NX>(buf, tw, g.twlog);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < C::R * C::H) gy[i] = buf[(e / C::H) * C::LS + e % C::H];
  }
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int rr = e / C::H, j = e % C::H;
    if (e < C::R * C::H && rr < nrow) {
      const size_t idx = (size_t)(y0 + rr) * NX + 2 * j;
      const double2 mx = *(const double2*)(m + idx);
      const double2 my = *(const double2*)(m + n + idx);
      const double2 rv = *(const double2*)(r + idx);
      const double gxa[2] = {gx[i].x, gx[i].y}, gya[2] = {gy[i].x, gy[i].y};
      const double mxa[2] = {mx.x, mx.y}, mya[2] = {my.x, my.y}, ra[2] = {rv.x, rv.y};
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
  write_partials(eslot, s, 3);
}

// ================================================================ column kernels
// mixed -> spectral (null modes zeroed unless bit 1 of mode is set); with bit 0
// of mode also the gradient of the result back to mixed:
// Gx = F_y^-1(i xi_x f_hat / n), Gy likewise.
template <int NY>
__global__ void __launch_bounds__(256) k_col_fwd(Geo g, cd* in, cd* __restrict__ out, int with_grad, cd* Gx,
                                                 cd* Gy) {
  using C = ColCfg<NY>;
  __shared__ cd buf[C::C * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  col_load<NY>(buf, in, kx0, g.h);
  __syncthreads();
  lds_fft<double, -1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
  cd v[C::E];
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int c = e / NY, ky = e % NY;
    cd a = buf[c * C::LS + ky];
    if (!(with_grad & 2) && kx0 + c == 0 && (ky == 0 || 2 * ky == NY)) a = mk<double>(0.0, 0.0);
    v[i] = a;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    buf[(e / NY) * C::LS + e % NY] = v[i];
  }
  __syncthreads();
  col_store<NY>(buf, out, kx0, g.h);
  if (!(with_grad & 1)) return;
  __syncthreads();
  for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      const int e = threadIdx.x + i * C::NT;
      const int c = e / NY, ky = e % NY;
      const int kx = kx0 + c;
      const double xi = comp == 0 ? (kx == 0 ? 0.0 : TWO_PI * kx / g.lx) : xi_tilde(ky, NY, g.ly);
      const double s = xi * g.inv_n;
      buf[c * C::LS + ky] = mk<double>(-s * v[i].y, s * v[i].x);
    }
    __syncthreads();
    lds_fft<double, +1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
    col_store<NY>(buf, comp == 0 ? Gx : Gy, kx0, g.h);
    __syncthreads();
  }
}

// spectral -> mixed: optional P = F_y^-1(x_hat / n), Gx, Gy as in k_col_fwd
template <int NY>
__global__ void __launch_bounds__(256) k_col_grad(Geo g, const cd* __restrict__ xh, cd* P, cd* Gx, cd* Gy) {
  using C = ColCfg<NY>;
  __shared__ cd buf[C::C * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  cd v[C::E];
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int c = e / NY, ky = e % NY;
    v[i] = (kx0 + c < g.h) ? xh[(size_t)(kx0 + c) * NY + ky] : mk<double>(0.0, 0.0);
  }
  for (int comp = (P ? -1 : 0); comp < (Gx ? 2 : 0); ++comp) {
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      const int e = threadIdx.x + i * C::NT;
      const int c = e / NY, ky = e % NY;
      const int kx = kx0 + c;
      if (comp < 0) {
        buf[c * C::LS + ky] = scl(v[i], g.inv_n);
      } else {
        const double xi = comp == 0 ? (kx == 0 ? 0.0 : TWO_PI * kx / g.lx) : xi_tilde(ky, NY, g.ly);
        const double s = xi * g.inv_n;
        buf[c * C::LS + ky] = mk<double>(-s * v[i].y, s * v[i].x);
      }
    }
    __syncthreads();
    lds_fft<double, +1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
    col_store<NY>(buf, comp < 0 ? P : (comp == 0 ? Gx : Gy), kx0, g.h);
    __syncthreads();
  }
}

__device__ __forceinline__ double precond_symbol_inv(const double* K, double xx, double yy) {
  const double s = K[0] * xx * xx + 2.0 * K[1] * xx * yy + K[2] * yy * yy;
  return s > 0.0 ? 1.0 / s : 0.0;
}

// Operator end: forward y transform of the fluxes, q_hat = -i xi . F_hat.
// INIT: r_hat = b_hat - q_hat (stored), partials <r,M^-1 r>, <r,r>, <b,b>;
//       also reduces the Kbar and compatibility partials of the row pass.
// else: q_hat stored, partials <d,q>, <q,M^-1 r>, <q,M^-1 q>, <r,q>, <q,q>,
//       <r,M^-1 r>, <r,r>.
template <int NY, bool INIT>
__global__ void __launch_bounds__(256) k_col_div(Geo g, const cd* __restrict__ Fx, const cd* __restrict__ Fy,
                                                 cd* __restrict__ qh, const cd* __restrict__ dh, cd* rh,
                                                 const cd* __restrict__ bh, int it, int nwg_row) {
  using C = ColCfg<NY>;
  if (!INIT && g.st->conv_at <= it) return;
  __shared__ cd buf[C::C * C::LS];
  __shared__ double red[7 * 4];
  __shared__ double Ks[4];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
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
  cd fx[C::E];
  col_load<NY>(buf, Fx, kx0, g.h);
  __syncthreads();
  lds_fft<double, -1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    fx[i] = buf[(e / NY) * C::LS + e % NY];
  }
  __syncthreads();
  col_load<NY>(buf, Fy, kx0, g.h);
  __syncthreads();
  lds_fft<double, -1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
  double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int c = e / NY, ky = e % NY;
    const int kx = kx0 + c;
    if (kx < g.h) {
      const cd fy = buf[c * C::LS + ky];
      const double xx = kx == 0 ? 0.0 : TWO_PI * kx / g.lx;
      const double yy = xi_tilde(ky, NY, g.ly);
      // q = -i (xx Fx + yy Fy)
      const double ax = xx * fx[i].x + yy * fy.x, ay = xx * fx[i].y + yy * fy.y;
      const cd q = mk<double>(ay, -ax);
      const double w = kx == 0 ? 1.0 : 2.0;
      const double sig = precond_symbol_inv(Ks, xx, yy);
      const size_t idx = (size_t)kx * NY + ky;
      if (INIT) {
        const cd b = bh[idx];
        const cd rn = sub(b, q);
        rh[idx] = rn;
        const double rr = rn.x * rn.x + rn.y * rn.y;
        s[0] += w * sig * rr;
        s[1] += w * rr;
        s[2] += w * (b.x * b.x + b.y * b.y);
      } else {
        qh[idx] = q;
        const cd d = dh[idx], rv = rh[idx];
        const double qq = q.x * q.x + q.y * q.y;
        const double rq = rv.x * q.x + rv.y * q.y;
        s[0] += w * (d.x * q.x + d.y * q.y);
        s[1] += w * sig * rq;
        s[2] += w * sig * qq;
        s[3] += w * rq;
        s[4] += w * qq;
        const double r2 = rv.x * rv.x + rv.y * rv.y;
        s[5] += w * sig * r2;
        s[6] += w * r2;
      }
    }
  }
  block_sum<C::NT, 7>(s, red);
  write_partials(slot_ptr(g.part, INIT ? SLOT_P3INIT : SLOT_P3), s, INIT ? 3 : 7);
}

// PCG scalar step + vector update + next direction + its gradient (mixed).
// first: d = M^-1 r.  else: alpha, beta from the partials of k_col_div (the
// new <r,M^-1 r> and ||r||^2 follow from the expansion of r - alpha q around
// the directly computed old values), then x += alpha d, r -= alpha q,
// d = M^-1 r + beta d.
template <int NY>
__global__ void __launch_bounds__(256) k_col_update(Geo g, int first, cd* xh, cd* rh, cd* dh,
                                                    const cd* __restrict__ qh, cd* Gx, cd* Gy, int it,
                                                    int max_iter, double tol2, int nwg_col) {
  using C = ColCfg<NY>;
  DevStatus* st = g.st;
  if (st->conv_at < it) return;
  __shared__ cd buf[C::C * C::LS];
  __shared__ double red[7 * 4];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
  double K[4];
  for (int i = 0; i < 4; ++i) K[i] = st->kbar[i];
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
    // directly from it; the new rho (for beta only) follows from the
    // expansion of <r - alpha q, M^-1 (r - alpha q)> around it.  The stopping
    // test on the new residual is taken by the next pass from its direct norm.
    double s[7];
    sum_partials<C::NT, 7>(slot_ptr(g.part, SLOT_P3), nwg_col, MAX_WG, s, red);
    const double rho = s[5];
    alpha = rho / s[0];
    const double rhon = rho - 2.0 * alpha * s[1] + alpha * alpha * s[2];
    beta = rhon / rho;
    const bool bad = !isfinite(rhon) || !isfinite(alpha);
    stop = bad || it >= max_iter;
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
  double rrp[1] = {0.0};
  cd dv[C::E];
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int c = e / NY, ky = e % NY;
    const int kx = kx0 + c;
    if (kx < g.h) {
      const size_t idx = (size_t)kx * NY + ky;
      if (zero_x) {
        xh[idx] = mk<double>(0.0, 0.0);
        continue;
      }
      cd rv = rh[idx];
      cd d;
      if (first) {
        d = mk<double>(0.0, 0.0);
      } else {
        d = dh[idx];
        const cd q = qh[idx];
        xh[idx] = add(xh[idx], scl(d, alpha));
        rv = sub(rv, scl(q, alpha));
        rh[idx] = rv;
        rrp[0] += (kx == 0 ? 1.0 : 2.0) * (rv.x * rv.x + rv.y * rv.y);
      }
      if (!stop) {
        const double xx = kx == 0 ? 0.0 : TWO_PI * kx / g.lx;
        const double yy = xi_tilde(ky, NY, g.ly);
        const double sig = precond_symbol_inv(K, xx, yy);
        d = add(scl(rv, sig), scl(d, beta));
        dh[idx] = d;
      }
      dv[i] = d;
    } else {
      dv[i] = mk<double>(0.0, 0.0);
    }
  }
  if (!first && !zero_x) {
    block_sum<C::NT, 1>(rrp, red);
    write_partials(slot_ptr(g.part, SLOT_RR), rrp, 1);
  }
  if (stop) return;
  for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      const int e = threadIdx.x + i * C::NT;
      const int c = e / NY, ky = e % NY;
      const int kx = kx0 + c;
      const double xi = comp == 0 ? (kx == 0 ? 0.0 : TWO_PI * kx / g.lx) : xi_tilde(ky, NY, g.ly);
      const double s = xi * g.inv_n;
      buf[c * C::LS + ky] = mk<double>(-s * dv[i].y, s * dv[i].x);
    }
    __syncthreads();
    lds_fft<double, +1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
    col_store<NY>(buf, comp == 0 ? Gx : Gy, kx0, g.h);
    __syncthreads();
  }
}

// Diffusion: forward y transform, multiply by exp(-D^2 |xi|^2 dt) / n (the
// packed column is unpacked into its kx = 0 and kx = Nx/2 halves for this),
// inverse y transform.  Optional partial sum w |xi_tilde|^2 |m_hat_new|^2.
template <int NY>
__global__ void __launch_bounds__(256) k_col_heat(Geo g, cd* Mx, cd* My, double D2dt, double* eslot) {
  using C = ColCfg<NY>;
  __shared__ cd buf[C::C * C::LS];
  __shared__ double red[1 * 4];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  const double xnyq = TWO_PI * (g.nx / 2) / g.lx;  // full wavenumber of the kx = Nx/2 column
  double s[1] = {0.0};
  for (int comp = 0; comp < 2; ++comp) {
    cd* F = comp == 0 ? Mx : My;
    col_load<NY>(buf, F, kx0, g.h);
    __syncthreads();
    lds_fft<double, -1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
    cd v[C::E];
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      const int e = threadIdx.x + i * C::NT;
      const int c = e / NY, ky = e % NY;
      const int kx = kx0 + c;
      const double yf = xi_full(ky, NY, g.ly);
      const cd a = buf[c * C::LS + ky];
      cd out;
      if (kx == 0) {
        const cd b = buf[c * C::LS + ((NY - ky) & (NY - 1))];
        const double hA = exp(-D2dt * (yf * yf)) * g.inv_n;
        const double hB = exp(-D2dt * (xnyq * xnyq + yf * yf)) * g.inv_n;
        // P' = (hA+hB)/2 P(ky) + (hA-hB)/2 conj P(-ky)
        out = add(scl(a, 0.5 * (hA + hB)), scl(conj(b), 0.5 * (hA - hB)));
      } else {
        const double xx = TWO_PI * kx / g.lx;
        out = scl(a, exp(-D2dt * (xx * xx + yf * yf)) * g.inv_n);
      }
      v[i] = out;
      if (eslot && kx < g.h) {
        const double xt = kx == 0 ? 0.0 : TWO_PI * kx / g.lx;
        const double yt = xi_tilde(ky, NY, g.ly);
        const double w = kx == 0 ? 1.0 : 2.0;
        s[0] += w * (xt * xt + yt * yt) * (out.x * out.x + out.y * out.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      const int e = threadIdx.x + i * C::NT;
      buf[(e / NY) * C::LS + e % NY] = v[i];
    }
    __syncthreads();
    lds_fft<double, +1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
    col_store<NY>(buf, F, kx0, g.h);
    __syncthreads();
  }
  if (eslot) {
    block_sum<C::NT, 1>(s, red);
    write_partials(eslot, s, 1);
  }
}

// Parseval sum w |xi_tilde|^2 |f_hat|^2 over two mixed fields (||grad m||^2 * n)
template <int NY>
__global__ void __launch_bounds__(256) k_col_gradnorm(Geo g, const cd* __restrict__ Mx, const cd* __restrict__ My,
                                                      double* eslot) {
  using C = ColCfg<NY>;
  __shared__ cd buf[C::C * C::LS];
  __shared__ double red[1 * 4];
  const cd* tw = (const cd*)g.tw;
  const int kx0 = blockIdx.x * C::C;
  double s[1] = {0.0};
  for (int comp = 0; comp < 2; ++comp) {
    col_load<NY>(buf, comp == 0 ? Mx : My, kx0, g.h);
    __syncthreads();
    lds_fft<double, -1, NY, C::C, C::LS, C::NT>(buf, tw, g.twlog);
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      const int e = threadIdx.x + i * C::NT;
      const int c = e / NY, ky = e % NY;
      const int kx = kx0 + c;
      if (kx < g.h) {
        const cd a = buf[c * C::LS + ky];
        const double xt = kx == 0 ? 0.0 : TWO_PI * kx / g.lx;
        const double yt = xi_tilde(ky, NY, g.ly);
        const double w = kx == 0 ? 1.0 : 2.0;
        s[0] += w * (xt * xt + yt * yt) * (a.x * a.x + a.y * a.y);
      }
    }
    __syncthreads();
  }
  block_sum<C::NT, 1>(s, red);
  write_partials(eslot, s, 1);
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
    default: return hipErrorInvalidValue;    \
  }

static int row_rows(int nx) {
  const int h = nx / 2;
  int r = 2048 / h;
  return r < 1 ? 1 : (r > 64 ? 64 : r);
}
static int col_cols(int ny) {
  int c = 2048 / ny;
  return c < 1 ? 1 : (c > 64 ? 64 : c);
}
int row_nwg(const Geo& g) {
  const int R = row_rows(g.nx);
  return (g.ny + R - 1) / R;
}
int col_nwg(const Geo& g) {
  const int C = col_cols(g.ny);
  return (g.h + C - 1) / C;
}

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
  const dim3 grid(row_nwg(g)), blk(256);
#define L_(N) hipLaunchKernelGGL(k_row_r2c<N>, grid, blk, 0, s, g, f, (cd*)out, schk)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_c2r(const Geo& g, const void* in, double* f, hipStream_t s) {
  const dim3 grid(row_nwg(g)), blk(256);
#define L_(N) hipLaunchKernelGGL(k_row_c2r<N>, grid, blk, 0, s, g, (const cd*)in, f)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_flux(const Geo& g, void* G0, void* G1, const double* m, const double* r, int it,
                           double* kslot, double tol2, hipStream_t s) {
  const dim3 grid(row_nwg(g)), blk(256);
  const int nwg_col = col_nwg(g);
#define L_(N) hipLaunchKernelGGL(k_row_flux<N>, grid, blk, 0, s, g, (cd*)G0, (cd*)G1, m, r, it, kslot, nwg_col, tol2)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_split(const Geo& g, void* P, void* Gx, void* Gy, const double* m, double* p_out,
                            double c2dt, double gamma, double dt, double relax1, hipStream_t s) {
  const dim3 grid(row_nwg(g)), blk(256);
#define L_(N)                                                                                            \
  hipLaunchKernelGGL(k_row_split<N>, grid, blk, 0, s, g, (cd*)P, (cd*)Gx, (const cd*)Gy, m, p_out, c2dt, \
                     gamma, dt, relax1)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_final(const Geo& g, const void* Mx, const void* My, double* m, double* dslot,
                            hipStream_t s) {
  const dim3 grid(row_nwg(g)), blk(256);
#define L_(N) hipLaunchKernelGGL(k_row_final<N>, grid, blk, 0, s, g, (const cd*)Mx, (const cd*)My, m, dslot)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_row_energy(const Geo& g, const void* Gx, const void* Gy, const double* m, const double* r,
                             double gamma, double* slot, hipStream_t s) {
  const dim3 grid(row_nwg(g)), blk(256);
#define L_(N) \
  hipLaunchKernelGGL(k_row_energy<N>, grid, blk, 0, s, g, (const cd*)Gx, (const cd*)Gy, m, r, gamma, slot)
  NF_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_col_fwd(const Geo& g, void* in, void* out, int with_grad, void* Gx, void* Gy, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(256);
#define L_(N) hipLaunchKernelGGL(k_col_fwd<N>, grid, blk, 0, s, g, (cd*)in, (cd*)out, with_grad, (cd*)Gx, (cd*)Gy)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_grad(const Geo& g, const void* xh, void* P, void* Gx, void* Gy, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(256);
#define L_(N) hipLaunchKernelGGL(k_col_grad<N>, grid, blk, 0, s, g, (const cd*)xh, (cd*)P, (cd*)Gx, (cd*)Gy)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_div(const Geo& g, int init, const void* Fx, const void* Fy, void* qh, const void* dh,
                          void* rh, const void* bh, int it, int nwg_row, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(256);
  if (init) {
#define L_(N)                                                                                                 \
  hipLaunchKernelGGL((k_col_div<N, true>), grid, blk, 0, s, g, (const cd*)Fx, (const cd*)Fy, (cd*)qh,         \
                     (const cd*)dh, (cd*)rh, (const cd*)bh, it, nwg_row)
    NF_DISPATCH(g.ny, L_)
#undef L_
  } else {
#define L_(N)                                                                                                 \
  hipLaunchKernelGGL((k_col_div<N, false>), grid, blk, 0, s, g, (const cd*)Fx, (const cd*)Fy, (cd*)qh,        \
                     (const cd*)dh, (cd*)rh, (const cd*)bh, it, nwg_row)
    NF_DISPATCH(g.ny, L_)
#undef L_
  }
  return hipGetLastError();
}
hipError_t launch_col_update(const Geo& g, int first, void* xh, void* rh, void* dh, const void* qh, void* Gx,
                             void* Gy, int it, int max_iter, double tol2, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(256);
  const int nwg = col_nwg(g);
#define L_(N)                                                                                              \
  hipLaunchKernelGGL(k_col_update<N>, grid, blk, 0, s, g, first, (cd*)xh, (cd*)rh, (cd*)dh, (const cd*)qh, \
                     (cd*)Gx, (cd*)Gy, it, max_iter, tol2, nwg)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_heat(const Geo& g, void* Mx, void* My, double D2dt, double* eslot, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(256);
#define L_(N) hipLaunchKernelGGL(k_col_heat<N>, grid, blk, 0, s, g, (cd*)Mx, (cd*)My, D2dt, eslot)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch_col_gradnorm(const Geo& g, const void* Mx, const void* My, double* eslot, hipStream_t s) {
  const dim3 grid(col_nwg(g)), blk(256);
#define L_(N) hipLaunchKernelGGL(k_col_gradnorm<N>, grid, blk, 0, s, g, (const cd*)Mx, (const cd*)My, eslot)
  NF_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}

}  // namespace nf
