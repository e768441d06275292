// HIP kernels (gfx950) of the 3D time step: the same spectral scheme as the 2D
// passes, with one more transform direction.
//
// Data layout (n = Nx*Ny*Nz, H = Nx/2):
//   physical   f[z][y][x]                (x fastest, caller-owned)
//   mixed      M[kx][z][y]               after the x transform; the y passes
//                                        transform the contiguous lines (kx, z)
//                                        in place, giving M[kx][z][ky]
//   spectral   F[kx][ky][kz]             after the z transform
// The row (x) passes treat the Ny*Nz lines (z, y) as rows.  A z pass gathers the
// lines (kx, ky) from the mixed layout at stride Ny, C consecutive ky per
// workgroup, and reads or writes the spectral layout contiguously.
// Slot kx = 0 packs the real kx = 0 and kx = Nx/2 planes as X0 + i X_{Nx/2};
// every multiplier applied to it is real or equal on both halves: the first
// derivative wavenumbers (Nyquist zeroed), the preconditioner symbol and the
// factors of the separable heat kernel, whose x factor is applied in the row
// pass before the planes are mixed.
// Inner products use the weights of the 2D path (1 on slot 0, 2 elsewhere).
// Reductions: every workgroup stores its block sums as partials and a
// one-workgroup pass launched right after the producing pass adds them in
// index order (deterministic) into the totals (see store_partials).
#include <hip/hip_ext.h>

#include <climits>

#include "nf_fft.hpp"
#include "nf_internal.h"
#include "nf_tiles.hpp"

namespace nf {

// ---------------------------------------------------------------- reductions
// Block sums of this workgroup stored as partials only; a one-workgroup pass
// (k3_sum_tot) launched right after the producing pass adds them in a fixed
// order into g.tot.  (A pass can have more workgroups than a consumer could
// re-read in every workgroup.)  A last-workgroup reduction would need an
// agent-scope release fence in every workgroup, which writes back the dirty
// lines of that XCD's L2 and cost a fifth to a third of the z passes.
template <int NT, int K>
__device__ __forceinline__ void store_partials(double (&v)[K], const Geo& g, int slot, double* red) {
  block_sum<NT, K>(v, red);
  if (threadIdx.x == 0) {
    double* part = g.part + (size_t)slot * SLOT_K * g.pstride;
    for (int k = 0; k < K; ++k) part[(size_t)k * g.pstride + blockIdx.x] = v[k];
  }
}

__device__ __forceinline__ double precond3_inv(const double* K, double a, double b, double c) {
  const double s = K[0] * a * a + K[3] * b * b + K[5] * c * c + 2.0 * (K[1] * a * b + K[2] * a * c + K[4] * b * c);
  return s > 0.0 ? 1.0 / s : 0.0;
}

// ---------------------------------------------------------------- z tiles
// A z tile holds 2 * TILE elements per field: at Nz = 256 that is 8 lines, so
// the strided gathers and scatters move 128-byte runs (full cache lines).
// Tiles of 8-byte elements (ES = 8, the FP32 loop passes) hold twice the lines
// with twice the threads, so that their runs stay 128 bytes long for the same
// LDS and the same registers per thread.
template <int NZ, int NF, int ES = 16, int TW = 1>
struct ZCfg {
  static constexpr int W = ES == 8 ? 2 : 1;
  static constexpr int C0 = 2 * TILE * W / NZ;
  static constexpr int C = C0 < 1 ? 1 : (C0 > 64 ? 64 : C0);  // lines (kx, ky) per workgroup
  static constexpr int NT = TPF * NF * W * TW;  // TW: extra thread multiple (same lines)
  static constexpr int LS = lpad_use(NZ) ? lpad_len(NZ) : NZ + 1;  // room for the FFT's padded layout
  static constexpr int CN = C * NZ;
  static constexpr int NB = NF * C;
  static constexpr int ET = (NF * CN + NT - 1) / NT;
  static constexpr int EP = (CN + NT - 1) / NT;
};

template <typename V>
__device__ __forceinline__ const V* pick4(int f, const V* a, const V* b, const V* c, const V* d) {
  return f == 0 ? a : (f == 1 ? b : (f == 2 ? c : d));
}
template <typename V>
__device__ __forceinline__ V* pick4w(int f, V* a, V* b, V* c, V* d) {
  return f == 0 ? a : (f == 1 ? b : (f == 2 ? c : d));
}

// gathered image: element e -> field e / CN, line (e % CN) % C, z (e % CN) / C;
// consecutive threads read consecutive ky of one z (coalesced runs of C)
template <int NZ, int NF, int NFL, typename V, int ES = 16, int TW = 1>
__device__ __forceinline__ void zT_gload(V (&v)[(ZCfg<NZ, NF, ES, TW>::ET)], const V* s0, const same<V>* s1,
                                         const same<V>* s2, const same<V>* s3, int lam0, int nlam, int ny) {
  using C = ZCfg<NZ, NF, ES, TW>;
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::CN, ee = e % C::CN;
    const int c = ee % C::C, z = ee / C::C;
    const int lam = lam0 + c;
    V x = vzero<V>();
    if (e < NFL * C::CN && lam < nlam) {
      const int kx = lam / ny, ky = lam - kx * ny;
      x = pick4<V>(f, s0, s1, s2, s3)[((size_t)kx * NZ + z) * ny + ky];
    }
    v[i] = x;
  }
}
template <int NZ, int NF, int NFL, typename V, int ES = 16, int TW = 1>
__device__ __forceinline__ void zT_put(V* buf, const V (&v)[(ZCfg<NZ, NF, ES, TW>::ET)]) {
  using C = ZCfg<NZ, NF, ES, TW>;
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::CN, ee = e % C::CN;
    if (e < NFL * C::CN) buf[(f * C::C + ee % C::C) * C::LS + ee / C::C] = v[i];
  }
}
template <int NZ, int NF, int NFS, typename V, int ES = 16, int TW = 1>
__device__ __forceinline__ void zT_store(const V* buf, same<V>* d0, same<V>* d1, same<V>* d2, same<V>* d3, int lam0,
                                         int nlam, int ny) {
  using C = ZCfg<NZ, NF, ES, TW>;
  for (int e = threadIdx.x; e < NFS * C::CN; e += C::NT) {
    const int f = e / C::CN, ee = e % C::CN;
    const int c = ee % C::C, z = ee / C::C;
    const int lam = lam0 + c;
    if (lam < nlam) {
      const int kx = lam / ny, ky = lam - kx * ny;
      pick4w<V>(f, d0, d1, d2, d3)[((size_t)kx * NZ + z) * ny + ky] = buf[(f * C::C + c) * C::LS + z];
    }
  }
}
// contiguous spectral image of one field: p -> line p / NZ, kz = p % NZ
template <int NZ, int NF, typename V, int ES = 16, int TW = 1>
__device__ __forceinline__ void zP_gload(V (&v)[(ZCfg<NZ, NF, ES, TW>::EP)], const V* __restrict__ src, int lam0, int nlam) {
  using C = ZCfg<NZ, NF, ES, TW>;
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NZ, kz = p % NZ;
    v[i] = (p < C::CN && lam0 + c < nlam) ? src[(size_t)(lam0 + c) * NZ + kz] : vzero<V>();
  }
}

// gradient multipliers i xi_c v / n of one spectral value into lines f0..f0+2
template <int NZ, int NF, typename T, int ES = 16, int TW = 1>
__device__ __forceinline__ void put_grad3(cx<T>* buf, int f0, int c, int kz, const cx<T> v, double xx, double yy,
                                          double zz, double inv_n) {
  using C = ZCfg<NZ, NF, ES, TW>;
  const T sx = (T)(xx * inv_n), sy = (T)(yy * inv_n), sz = (T)(zz * inv_n);
  buf[(f0 * C::C + c) * C::LS + kz] = mk<T>(-sx * v.y, sx * v.x);
  buf[((f0 + 1) * C::C + c) * C::LS + kz] = mk<T>(-sy * v.y, sy * v.x);
  buf[((f0 + 2) * C::C + c) * C::LS + kz] = mk<T>(-sz * v.y, sz * v.x);
}

// wavenumbers of spectral line lam = kx * Ny + ky
__device__ __forceinline__ void line_xi(const Geo& g, int lam, double& xx, double& yy) {
  const int kx = lam / g.ny, ky = lam - kx * g.ny;
  xx = xi_col(kx, g.lx);
  yy = xi_tilde(ky, g.ny, g.ly);
}

// ================================================================ row (x) passes
// physical -> mixed, one field; optional compatibility partials (sum S, sum |S|)
template <int NX>
__global__ void __launch_bounds__(TPF) k3_row_r2c(Geo g, const double* __restrict__ f, cd* __restrict__ out,
                                                  int schk) {
  using C = RowCfg<NX, 1>;
  __shared__ cd buf[C::NB * C::LS];
  __shared__ double red[2 * (C::NT / 64)];
  const cd* tw = (const cd*)g.tw;
  const int rows = g.ny * g.nz;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, rows - y0);
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
  rowT_store<C, 1>(buf, out, nullptr, nullptr, rows, y0, nrow);
  if (schk) store_partials<C::NT, 2>(s, g, SLOT_SCHK, red);
}

template <int NX>
__global__ void __launch_bounds__(TPF) k3_row_c2r(Geo g, const cd* __restrict__ in, double* __restrict__ f) {
  using C = RowCfg<NX, 1>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int rows = g.ny * g.nz;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, rows - y0);
  cd tv[C::ET];
  rowT_gload<C>(tv, in, nullptr, nullptr, rows, y0, nrow);
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

// Operator middle: gradient (mixed, 3 fields) -> physical g -> K g -> mixed,
// in place.  K = m m^T + r I.  it >= 0: no-op once the solve has stopped.
template <int NX, typename T>
__global__ void __launch_bounds__(3 * TPF) k3_row_flux(Geo g, cx<T>* G0, cx<T>* G1, cx<T>* G2,
                                                     const T* __restrict__ m, const T* __restrict__ r, int it,
                                                     int kbar, float* lo) {
  using C = RowCfg<NX, 3>;
  using V = cx<T>;
  using P = typename vec2<T>::type;
  if (it >= 0 ? g.st->conv_at <= it : g.st->outer_done != 0) return;
  tclk_start(g, 0, it);
  __shared__ V buf[C::NB * C::LS];
  __shared__ double red[7 * (C::NT / 64)];
  const V* tw = (const V*)g.tw;
  const int rows = g.ny * g.nz;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, rows - y0);
  const size_t n = (size_t)g.nx * rows;
  V tv[C::ET];
  rowT_gload<C>(tv, G0, G1, G2, rows, y0, nrow);
  P mx[C::EP], my[C::EP], mz[C::EP], rv[C::EP];
  rowP_gload<C>(mx, m, y0, nrow);
  rowP_gload<C>(my, m + n, y0, nrow);
  rowP_gload<C>(mz, m + 2 * n, y0, nrow);
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
        *(float2*)(lo + 2 * n + o) = make_float2((float)mz[i].x, (float)mz[i].y);
        *(float2*)(lo + 3 * n + o) = make_float2((float)rv[i].x, (float)rv[i].y);
      }
    }
  }
  rowT_put<C>(buf, tv);
  __syncthreads();
  irfft_pre<T, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  lds_fft<T, +1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  double ks[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int rr = p / C::H, j = p % C::H;
    if (p < C::RH && rr < nrow) {
      V* px = buf + rr * C::LS + j;
      V* py = buf + (C::R + rr) * C::LS + j;
      V* pz = buf + (2 * C::R + rr) * C::LS + j;
      const V gx = *px, gy = *py, gz = *pz;
      const T a0 = mx[i].x * gx.x + my[i].x * gy.x + mz[i].x * gz.x;
      const T a1 = mx[i].y * gx.y + my[i].y * gy.y + mz[i].y * gz.y;
      *px = mk<T>(fma(a0, mx[i].x, rv[i].x * gx.x), fma(a1, mx[i].y, rv[i].y * gx.y));
      *py = mk<T>(fma(a0, my[i].x, rv[i].x * gy.x), fma(a1, my[i].y, rv[i].y * gy.y));
      *pz = mk<T>(fma(a0, mz[i].x, rv[i].x * gz.x), fma(a1, mz[i].y, rv[i].y * gz.y));
      if (kbar) {
        const double ax[2] = {mx[i].x, mx[i].y}, ay[2] = {my[i].x, my[i].y}, az[2] = {mz[i].x, mz[i].y};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          ks[0] += ax[t] * ax[t];
          ks[1] += ax[t] * ay[t];
          ks[2] += ax[t] * az[t];
          ks[3] += ay[t] * ay[t];
          ks[4] += ay[t] * az[t];
          ks[5] += az[t] * az[t];
        }
        ks[6] += (double)rv[i].x + (double)rv[i].y;
      }
    }
  }
  __syncthreads();
  lds_fft<T, -1, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  rfft_post<T, C::H, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  rowT_store<C, 3>(buf, G0, G1, G2, rows, y0, nrow);
  if (kbar) store_partials<C::NT, 7>(ks, g, SLOT_KBAR, red);
  tclk_end(g, 0, it);
}

// Split update, pointwise part: P, G0..G2 hold x/n, and the gradient (mixed,
// after the inverse y transform).  Writes p, advances m by exact activation and
// exact relaxation, forward x transform of the three components times the x
// factor exp(-D2dt xi_x^2) of the heat kernel, into P, G0, G1.
template <int NX>
__global__ void __launch_bounds__(4 * TPF) k3_row_split(Geo g, cd* P, cd* G0, cd* G1, const cd* __restrict__ G2,
                                                      const double* __restrict__ m, double* __restrict__ p_out,
                                                      double c2dt, double gamma, double dt, double relax1,
                                                      double D2dt) {
  using C = RowCfg<NX, 4>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int rows = g.ny * g.nz;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, rows - y0);
  const size_t n = (size_t)g.nx * rows;
  cd tv[C::ET];
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::RH, ee = e % C::RH;
    const int rr = ee % C::R, kx = ee / C::R;
    const cd* src = f == 0 ? P : (f == 1 ? G0 : (f == 2 ? G1 : G2));
    tv[i] = (e < 4 * C::RH && rr < nrow) ? src[(size_t)kx * rows + y0 + rr] : mk<double>(0.0, 0.0);
  }
  double2 m0v[C::EP], m1v[C::EP], m2v[C::EP];
  rowP_gload<C>(m0v, m, y0, nrow);
  rowP_gload<C>(m1v, m + n, y0, nrow);
  rowP_gload<C>(m2v, m + 2 * n, y0, nrow);
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
      cd* l0 = buf + rr * C::LS + j;
      cd* l1 = buf + (C::R + rr) * C::LS + j;
      cd* l2 = buf + (2 * C::R + rr) * C::LS + j;
      const cd pv = *l0, ga = *l1, gb = *l2, gc = buf[(3 * C::R + rr) * C::LS + j];
      *(double2*)(p_out + (size_t)(y0 + rr) * NX + 2 * j) = make_double2(pv.x, pv.y);
      double q[3][2] = {{m0v[i].x, m0v[i].y}, {m1v[i].x, m1v[i].y}, {m2v[i].x, m2v[i].y}};
      const double gg[3][2] = {{ga.x, ga.y}, {gb.x, gb.y}, {gc.x, gc.y}};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // activation: m + c^2 dt phi1(c^2 dt |g|^2) (g.m) g
        const double g2 = gg[0][t] * gg[0][t] + gg[1][t] * gg[1][t] + gg[2][t] * gg[2][t];
        const double z = c2dt * g2;
        const double phi = z > 0.0 ? expm1(z) / z : 1.0;
        const double coef = c2dt * phi * (gg[0][t] * q[0][t] + gg[1][t] * q[1][t] + gg[2][t] * q[2][t]);
        double a[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] = fma(coef, gg[c][t], q[c][t]);
        // relaxation: exact decay of |m| along m/|m|
        double fac;
        if (gamma == 1.0) {
          fac = relax1;
        } else {
          const double s2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
          if (s2 == 0.0) {
            fac = 1.0;
          } else {
            const double u = 2.0 * e1 * dt * exp(-e1 * log(s2));
            fac = (u >= 1.0) ? 0.0 : exp(log1p(-u) / (2.0 * e1));
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          q[c][t] = a[c] * fac;
          if (!isfinite(q[c][t])) bad = true;
        }
      }
      *l0 = mk<double>(q[0][0], q[0][1]);
      *l1 = mk<double>(q[1][0], q[1][1]);
      *l2 = mk<double>(q[2][0], q[2][1]);
    }
  }
  if (bad) atomicOr(&g.st->sticky, (int)FLAG_NONFINITE);
  __syncthreads();
  lds_fft<double, -1, C::H, 3 * C::R, C::LS, C::NT>(buf, tw, g.twn);
  rfft_post<double, C::H, 3 * C::R, C::LS, C::NT>(buf, tw, g.twn);
  // x factor of the heat kernel; slot 0 holds the kx = 0 (real part) and kx = Nx/2
  // (imaginary part) coefficients
  for (int t = threadIdx.x; t < 3 * C::R * C::H; t += C::NT) {
    const int line = t / C::H, kx = t % C::H;
    cd* e = buf + line * C::LS + kx;
    if (kx == 0) {
      const double xn = xi_full(NX / 2, NX, g.lx);
      e->y *= exp(-D2dt * xn * xn);
    } else {
      const double xk = xi_full(kx, NX, g.lx);
      *e = scl(*e, exp(-D2dt * xk * xk));
    }
  }
  __syncthreads();
  rowT_store<C, 3>(buf, P, G0, G1, rows, y0, nrow);
}

// Last pass of the step: inverse x transform of the three components (already
// diffused and normalised), writes m and the partials of Delta m.
template <int NX>
__global__ void __launch_bounds__(3 * TPF) k3_row_final(Geo g, const cd* __restrict__ M0, const cd* __restrict__ M1,
                                                      const cd* __restrict__ M2, double* m) {
  using C = RowCfg<NX, 3>;
  __shared__ cd buf[C::NB * C::LS];
  __shared__ double red[2 * (C::NT / 64)];
  const cd* tw = (const cd*)g.tw;
  const int rows = g.ny * g.nz;
  const int y0 = xcd_block() * C::R;
  const int nrow = min(C::R, rows - y0);
  const size_t n = (size_t)g.nx * rows;
  cd tv[C::ET];
  rowT_gload<C>(tv, M0, M1, M2, rows, y0, nrow);
  double2 o0[C::EP], o1[C::EP], o2[C::EP];
  rowP_gload<C>(o0, m, y0, nrow);
  rowP_gload<C>(o1, m + n, y0, nrow);
  rowP_gload<C>(o2, m + 2 * n, y0, nrow);
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
      const cd a0 = buf[rr * C::LS + j], a1 = buf[(C::R + rr) * C::LS + j], a2 = buf[(2 * C::R + rr) * C::LS + j];
      const size_t idx = (size_t)(y0 + rr) * NX + 2 * j;
      const double d[6] = {a0.x - o0[i].x, a0.y - o0[i].y, a1.x - o1[i].x, a1.y - o1[i].y, a2.x - o2[i].x,
                           a2.y - o2[i].y};
      for (int k = 0; k < 6; ++k) s[0] += d[k] * d[k];
      s[1] += o0[i].x * o0[i].x + o0[i].y * o0[i].y + o1[i].x * o1[i].x + o1[i].y * o1[i].y + o2[i].x * o2[i].x +
              o2[i].y * o2[i].y;
      *(double2*)(m + idx) = make_double2(a0.x, a0.y);
      *(double2*)(m + n + idx) = make_double2(a1.x, a1.y);
      *(double2*)(m + 2 * n + idx) = make_double2(a2.x, a2.y);
    }
  }
  store_partials<C::NT, 2>(s, g, SLOT_DM, red);
}

// ================================================================ y passes
// NF fields, lines (kx, z) of length NY, transformed in place (DIR -1 forward,
// +1 inverse).  stop_test: take the PCG stopping decision of iteration it
// (it >= 1) from the totals of the last update.  heat_D2dt >= 0: multiply by
// the y factor exp(-D2dt xi_y^2) of the heat kernel after the transform.
template <int NY, int NF, int DIR, typename T>
__global__ void __launch_bounds__(NF * TPF) k3_ypass(Geo g, cx<T>* F0, cx<T>* F1, cx<T>* F2, cx<T>* F3, int it,
                                                   int stop_test, double tol2, double heat_D2dt) {
  using C = ColCfg<NY, NF>;
  using V = cx<T>;
  if (it >= 0 && g.st->conv_at <= it) return;
  __shared__ V buf[C::NB * C::LS];
  const V* tw = (const V*)g.tw;
  const int nl = g.h * g.nz;
  const int l0 = xcd_block() * C::C;
  V tv[C::ET];
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    const int f = e / C::CN, ee = e % C::CN;
    const int c = ee / NY, ky = ee % NY;
    tv[i] = (e < NF * C::CN && l0 + c < nl) ? pick4<V>(f, F0, F1, F2, F3)[(size_t)(l0 + c) * NY + ky] : vzero<V>();
  }
  if (stop_test && it >= 1) {
    const double rr = g.tot[SLOT_RR * SLOT_K];
    const double bb = g.st->bb;
    const bool bad = !isfinite(rr);
    if (bad || rr <= tol2 * bb) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        g.st->rr[0] = rr;
        g.st->converged = bad ? 0 : 1;
        if (bad) g.st->flags |= FLAG_NONFINITE;
        g.st->conv_at = it;
      }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < C::ET; ++i) {
    const int e = threadIdx.x + i * C::NT;
    if (e < NF * C::CN) buf[(e / C::CN * C::C + (e % C::CN) / NY) * C::LS + e % NY] = tv[i];
  }
  __syncthreads();
  lds_fft<T, DIR, NY, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  for (int e = threadIdx.x; e < NF * C::CN; e += C::NT) {
    const int f = e / C::CN, ee = e % C::CN;
    const int c = ee / NY, ky = ee % NY;
    if (l0 + c < nl) {
      V v = buf[(f * C::C + c) * C::LS + ky];
      if (heat_D2dt >= 0.0) {
        const double yk = xi_full(ky, NY, g.ly);
        v = scl(v, (T)exp(-heat_D2dt * yk * yk));
      }
      pick4w<V>(f, F0, F1, F2, F3)[(size_t)(l0 + c) * NY + ky] = v;
    }
  }
}

// ================================================================ z passes
// mixed [kx][z][ky] -> spectral [kx][ky][kz], one field; project: zero the
// null modes (slot 0, ky in {0, Ny/2}, kz in {0, Nz/2})
template <int NZ>
__global__ void __launch_bounds__(TPF) k3_zfwd(Geo g, const cd* __restrict__ in, cd* __restrict__ out, int project) {
  using C = ZCfg<NZ, 1>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int nlam = g.h * g.ny;
  const int lam0 = xcd_block() * C::C;
  cd tv[C::ET];
  zT_gload<NZ, 1, 1>(tv, in, nullptr, nullptr, nullptr, lam0, nlam, g.ny);
  zT_put<NZ, 1, 1>(buf, tv);
  __syncthreads();
  lds_fft<double, -1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NZ, kz = p % NZ;
    const int lam = lam0 + c;
    if (p < C::CN && lam < nlam) {
      cd a = buf[c * C::LS + kz];
      const int kx = lam / g.ny, ky = lam - kx * g.ny;
      if (project && kx == 0 && (ky == 0 || 2 * ky == g.ny) && (kz == 0 || 2 * kz == NZ)) a = mk<double>(0.0, 0.0);
      out[(size_t)lam * NZ + kz] = a;
    }
  }
}

// spectral -> mixed after the inverse z transform: MODE 1 P = x/n; MODE 2 the
// gradient i xi x / n into G0..G2; MODE 3 both (P first)
template <int NZ, int MODE>
__global__ void __launch_bounds__((MODE == 1 ? 1 : (MODE == 2 ? 3 : 4)) * TPF)
    k3_zinv(Geo g, const cd* __restrict__ xh, cd* P, cd* G0, cd* G1, cd* G2) {
  constexpr int NF = MODE == 1 ? 1 : (MODE == 2 ? 3 : 4);
  using C = ZCfg<NZ, NF>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int nlam = g.h * g.ny;
  const int lam0 = xcd_block() * C::C;
  cd v[C::EP];
  zP_gload<NZ, NF>(v, xh, lam0, nlam);
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NZ, kz = p % NZ;
    if (p < C::CN) {
      if (MODE & 1) buf[c * C::LS + kz] = scl(v[i], g.inv_n);
      if (MODE & 2) {
        double xx, yy;
        line_xi(g, lam0 + c, xx, yy);
        put_grad3<NZ, NF, double>(buf, MODE == 3 ? 1 : 0, c, kz, v[i], xx, yy, xi_tilde(kz, NZ, g.lz), g.inv_n);
      }
    }
  }
  __syncthreads();
  lds_fft<double, +1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  if (MODE == 1) zT_store<NZ, NF, 1>(buf, P, nullptr, nullptr, nullptr, lam0, nlam, g.ny);
  if (MODE == 2) zT_store<NZ, NF, 3>(buf, G0, G1, G2, nullptr, lam0, nlam, g.ny);
  if (MODE == 3) zT_store<NZ, NF, 4>(buf, P, G0, G1, G2, lam0, nlam, g.ny);
}

// Operator end: forward z transform of the three fluxes, q = -i xi . F.
// INIT (FP64 only): r = b - q (stored); totals <r,M^-1 r>, <r,r>, <b,b>;
//   also turns the Kbar and compatibility totals of the row passes into
//   status.kbar and the incompatibility flag.
// else: q stored; totals <d,q>, <q,M^-1 r>, <q,M^-1 q>, <r,q>, <q,q>,
//   <r,M^-1 r>, <r,r>.
// z tile of the loop passes: 128-byte runs in both precisions (section of
// ZCfg); FP64 with twice the threads (the tile's 111 KB of LDS admit one
// workgroup per compute unit: 12 waves rather than 6)
template <typename T>
constexpr int z_tw() { return sizeof(T) == sizeof(double) ? 2 : 1; }
template <int NZ, bool INIT, typename T>
__global__ void __launch_bounds__((ZCfg<NZ, 3, sizeof(cx<T>), z_tw<T>()>::NT))
    k3_zdiv(Geo g, const cx<T>* F0, const cx<T>* F1, const cx<T>* F2, cx<T>* __restrict__ qh,
            const cx<T>* __restrict__ dh, cx<T>* rh, const cx<T>* __restrict__ bh, int it) {
  constexpr int ES = sizeof(cx<T>), TW = z_tw<T>();
  using C = ZCfg<NZ, 3, ES, TW>;
  using V = cx<T>;
  static_assert(!INIT || sizeof(T) == sizeof(double), "INIT pass is FP64");
  if (INIT ? g.st->outer_done != 0 : g.st->conv_at <= it) return;
  if (!INIT) tclk_start(g, 1, it);
  __shared__ V buf[C::NB * C::LS];
  __shared__ double red[7 * (C::NT / 64)];
  __shared__ double Ks[6];
  const V* tw = (const V*)g.tw;
  const int nlam = g.h * g.ny;
  const int lam0 = xcd_block() * C::C;
  V tv[C::ET], av[C::EP], bv[C::EP];
  zT_gload<NZ, 3, 3, V, ES, TW>(tv, F0, F1, F2, nullptr, lam0, nlam, g.ny);
  if (INIT) {
    zP_gload<NZ, 3, V, ES, TW>(av, bh, lam0, nlam);
  } else {
    zP_gload<NZ, 3, V, ES, TW>(av, dh, lam0, nlam);
    zP_gload<NZ, 3, V, ES, TW>(bv, rh, lam0, nlam);
  }
  if (INIT) {
    if (threadIdx.x == 0) {
      const double* kb = g.tot + SLOT_KBAR * SLOT_K;
      const double* sc = g.tot + SLOT_SCHK * SLOT_K;
      const double rm = kb[6] * g.inv_n;
      Ks[0] = kb[0] * g.inv_n + rm;
      Ks[1] = kb[1] * g.inv_n;
      Ks[2] = kb[2] * g.inv_n;
      Ks[3] = kb[3] * g.inv_n + rm;
      Ks[4] = kb[4] * g.inv_n;
      Ks[5] = kb[5] * g.inv_n + rm;
      if (blockIdx.x == 0) {
        for (int i = 0; i < 6; ++i) g.st->kbar[i] = Ks[i];
        if (fabs(sc[0]) > 1e-12 * sc[1]) atomicOr(&g.st->flags, (int)FLAG_INCOMPAT);
      }
    }
  } else if (threadIdx.x < 6) {
    Ks[threadIdx.x] = g.st->kbar[threadIdx.x];
  }
  zT_put<NZ, 3, 3, V, ES, TW>(buf, tv);
  __syncthreads();
  lds_fft<T, -1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  constexpr int KP = INIT ? 3 : 4;  // partial sums stored (see below)
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NZ, kz = p % NZ;
    const int lam = lam0 + c;
    if (p < C::CN && lam < nlam) {
      const V fx = buf[c * C::LS + kz], fy = buf[(C::C + c) * C::LS + kz], fz = buf[(2 * C::C + c) * C::LS + kz];
      double xx, yy;
      line_xi(g, lam, xx, yy);
      const double zz = xi_tilde(kz, NZ, g.lz);
      const T ax = (T)xx * fx.x + (T)yy * fy.x + (T)zz * fz.x;
      const T ay = (T)xx * fx.y + (T)yy * fy.y + (T)zz * fz.y;
      const V q = mk<T>(ay, -ax);
      const double w = lam < g.ny ? 1.0 : 2.0;  // slot kx = 0 <=> lam < Ny
      const double sig = precond3_inv(Ks, xx, yy, zz);
      const size_t idx = (size_t)lam * NZ + kz;
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
  // INIT: <r,M^-1 r>, <r,r>, <b,b>; else <d,q>, <q,M^-1 r>, <q,M^-1 q>, <r,M^-1 r>
  double sk[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) sk[k] = s[k];
  store_partials<C::NT, KP>(sk, g, INIT ? SLOT_P3INIT : SLOT_P3, red);
  if (!INIT) tclk_end(g, 1, it);
}

// PCG scalar step + vector update + next direction + its gradient through the
// inverse z transform (the 2D column update with three gradient fields).
template <int NZ, typename T>
__global__ void __launch_bounds__((ZCfg<NZ, 3, sizeof(cx<T>), z_tw<T>()>::NT))
    k3_zupdate(Geo g, int first, cx<T>* xh, cx<T>* rh, cx<T>* dh, const cx<T>* __restrict__ qh, cx<T>* G0,
               cx<T>* G1, cx<T>* G2, int it, int max_iter, double tol2) {
  constexpr int ES = sizeof(cx<T>), TW = z_tw<T>();
  using C = ZCfg<NZ, 3, ES, TW>;
  using V = cx<T>;
  DevStatus* st = g.st;
  if (st->conv_at < it) return;
  const int tit = first ? -1 : it;  // timing slot (the first update is not a loop pass)
  tclk_start(g, 2, tit);
  __shared__ V buf[C::NB * C::LS];
  __shared__ double red[7 * (C::NT / 64)];
  const V* tw = (const V*)g.tw;
  const int nlam = g.h * g.ny;
  const int lam0 = xcd_block() * C::C;
  const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
  double K[6];
  for (int i = 0; i < 6; ++i) K[i] = st->kbar[i];
  V xv[C::EP], rv0[C::EP], dv0[C::EP], qv[C::EP];
  zP_gload<NZ, 3, V, ES, TW>(rv0, rh, lam0, nlam);
  if (!first) {
    zP_gload<NZ, 3, V, ES, TW>(xv, xh, lam0, nlam);
    zP_gload<NZ, 3, V, ES, TW>(dv0, dh, lam0, nlam);
    zP_gload<NZ, 3, V, ES, TW>(qv, qh, lam0, nlam);
  }
  double alpha = 0.0, beta = 0.0;
  bool stop = false, zero_x = false;
  if (first) {
    const double* s = g.tot + SLOT_P3INIT * SLOT_K;
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
    const double* s = g.tot + SLOT_P3 * SLOT_K;
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
    const int c = p / NZ, kz = p % NZ;
    const int lam = lam0 + c;
    V d = vzero<V>();
    double xx = 0.0, yy = 0.0;
    const double zz = xi_tilde(kz, NZ, g.lz);
    if (p < C::CN && lam < nlam) {
      line_xi(g, lam, xx, yy);
      const size_t idx = (size_t)lam * NZ + kz;
      if (zero_x) {
        xh[idx] = vzero<V>();
      } else {
        V rv = rv0[i];
        if (!first) {
          d = dv0[i];
          xh[idx] = add(xv[i], scl(d, a));
          rv = sub(rv, scl(qv[i], a));
          rh[idx] = rv;
          rrp[0] += (lam < g.ny ? 1.0 : 2.0) * ((double)rv.x * rv.x + (double)rv.y * rv.y);
        }
        if (!stop) {
          const T sig = (T)precond3_inv(K, xx, yy, zz);
          d = add(scl(rv, sig), scl(d, bt));
          dh[idx] = d;
        }
      }
    }
    if (!stop && p < C::CN) put_grad3<NZ, 3, T, ES, TW>(buf, 0, c, kz, d, xx, yy, zz, g.inv_n);
  }
  if (!first && !zero_x) store_partials<C::NT, 1>(rrp, g, SLOT_RR, red);
  if (stop) {
    tclk_end(g, 2, tit);
    return;
  }
  __syncthreads();
  lds_fft<T, +1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  zT_store<NZ, 3, 3, V, ES, TW>(buf, G0, G1, G2, nullptr, lam0, nlam, g.ny);
  tclk_end(g, 2, tit);
}

// Diffusion, z part: forward z transform of the three components, multiply by
// the z factor exp(-D2dt xi_z^2) and 1/n, inverse z transform; in place.
template <int NZ>
__global__ void __launch_bounds__(3 * TPF) k3_zheat(Geo g, cd* M0, cd* M1, cd* M2, double D2dt) {
  using C = ZCfg<NZ, 3>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int nlam = g.h * g.ny;
  const int lam0 = xcd_block() * C::C;
  cd tv[C::ET];
  zT_gload<NZ, 3, 3>(tv, M0, M1, M2, nullptr, lam0, nlam, g.ny);
  zT_put<NZ, 3, 3>(buf, tv);
  __syncthreads();
  lds_fft<double, -1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  for (int e = threadIdx.x; e < 3 * C::CN; e += C::NT) {
    const int line = e / NZ, kz = e % NZ;
    const double zk = xi_full(kz, NZ, g.lz);
    cd* v = buf + line * C::LS + kz;
    *v = scl(*v, exp(-D2dt * zk * zk) * g.inv_n);
  }
  __syncthreads();
  lds_fft<double, +1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  zT_store<NZ, 3, 3>(buf, M0, M1, M2, nullptr, lam0, nlam, g.ny);
}

// Mixed-precision solve in 3D: correction start and accumulation (the 2D
// kernels with the z transform and three gradient fields).
template <int NZ>
__global__ void __launch_bounds__(3 * TPF) k3_zrefine_start(Geo g, const cd* __restrict__ r64, cd* x64,
                                                          cx<float>* x32, cx<float>* r32, cx<float>* d32,
                                                          cx<float>* G0, cx<float>* G1, cx<float>* G2, double tol2,
                                                          double floor_in, int max_iter) {
  using C = ZCfg<NZ, 3>;
  using V = cx<float>;
  DevStatus* st = g.st;
  __shared__ V buf[C::NB * C::LS];
  const V* tw = (const V*)g.tw;
  const int nlam = g.h * g.ny;
  const int lam0 = xcd_block() * C::C;
  const bool lead = (blockIdx.x == 0 && threadIdx.x == 0);
  double K[6];
  for (int i = 0; i < 6; ++i) K[i] = st->kbar[i];
  cd rv[C::EP];
  zP_gload<NZ, 3>(rv, r64, lam0, nlam);
  const double* s = g.tot + SLOT_P3INIT * SLOT_K;
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
        const int lam = lam0 + p / NZ;
        if (p < C::CN && lam < nlam) x64[(size_t)lam * NZ + p % NZ] = mk<double>(0.0, 0.0);
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
    const int c = p / NZ, kz = p % NZ;
    const int lam = lam0 + c;
    V d = vzero<V>();
    double xx = 0.0, yy = 0.0;
    const double zz = xi_tilde(kz, NZ, g.lz);
    if (p < C::CN && lam < nlam) {
      line_xi(g, lam, xx, yy);
      const size_t idx = (size_t)lam * NZ + kz;
      const double sig = precond3_inv(K, xx, yy, zz);
      const double ux = rv[i].x * scale, uy = rv[i].y * scale;
      r32[idx] = mk<float>((float)ux, (float)uy);
      d = mk<float>((float)(sig * ux), (float)(sig * uy));
      d32[idx] = d;
      x32[idx] = vzero<V>();
    }
    if (p < C::CN) put_grad3<NZ, 3, float>(buf, 0, c, kz, d, xx, yy, zz, g.inv_n);
  }
  __syncthreads();
  lds_fft<float, +1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  zT_store<NZ, 3, 3>(buf, G0, G1, G2, nullptr, lam0, nlam, g.ny);
}

template <int NZ>
__global__ void __launch_bounds__(3 * TPF) k3_zrefine_acc(Geo g, cd* x64, const cx<float>* __restrict__ x32, cd* G0,
                                                        cd* G1, cd* G2) {
  using C = ZCfg<NZ, 3>;
  __shared__ cd buf[C::NB * C::LS];
  const cd* tw = (const cd*)g.tw;
  const int nlam = g.h * g.ny;
  const int lam0 = xcd_block() * C::C;
  if (g.st->outer_done) return;
  const double sc = g.st->rscale;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g.st->itot += g.st->iters;
    g.st->orr_prev = g.st->orr;
  }
  cd xv[C::EP];
  cx<float> ev[C::EP];
  zP_gload<NZ, 3>(xv, x64, lam0, nlam);
  zP_gload<NZ, 3>(ev, x32, lam0, nlam);
#pragma unroll
  for (int i = 0; i < C::EP; ++i) {
    const int p = threadIdx.x + i * C::NT;
    const int c = p / NZ, kz = p % NZ;
    const int lam = lam0 + c;
    cd x = mk<double>(0.0, 0.0);
    double xx = 0.0, yy = 0.0;
    if (p < C::CN && lam < nlam) {
      line_xi(g, lam, xx, yy);
      x = mk<double>(fma(sc, (double)ev[i].x, xv[i].x), fma(sc, (double)ev[i].y, xv[i].y));
      x64[(size_t)lam * NZ + kz] = x;
    }
    if (p < C::CN) put_grad3<NZ, 3, double>(buf, 0, c, kz, x, xx, yy, xi_tilde(kz, NZ, g.lz), g.inv_n);
  }
  __syncthreads();
  lds_fft<double, +1, NZ, C::NB, C::LS, C::NT>(buf, tw, g.twn);
  zT_store<NZ, 3, 3>(buf, G0, G1, G2, nullptr, lam0, nlam, g.ny);
}

__global__ void k_tclk_reset(unsigned long long* t, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    t[2 * i] = ~0ULL;
    t[2 * i + 1] = 0ULL;
  }
}
hipError_t launch_tclk_reset(unsigned long long* t, hipStream_t s) {
  const int n = TCLK_CAP * TCLK_W;
  hipLaunchKernelGGL(k_tclk_reset, dim3((n + 255) / 256), dim3(256), 0, s, t, n);
  return hipGetLastError();
}

__global__ void k3_copy_tot(Geo g, int slot, int K, int o) {
  if (threadIdx.x < K) g.st->out[o + threadIdx.x] = g.tot[slot * SLOT_K + threadIdx.x];
}

// ---------------------------------------------------------------- energy (Sec. 2.5)
// Pointwise terms of the discrete energy: partials of sum r |g|^2,
// sum (m . g)^2 and sum |m|^{2 gamma} over the physical grid, with g = grad p
// given as three physical fields.  Grid-stride over the n points.
__global__ void __launch_bounds__(256) k3_energy_pt(Geo g, const double* __restrict__ m,
                                                     const double* __restrict__ r, const double* __restrict__ gx,
                                                     const double* __restrict__ gy, const double* __restrict__ gz,
                                                     double gamma) {
  __shared__ double red[3 * 4];
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  double s[3] = {0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double mx = m[i], my = m[n + i], mz = m[2 * n + i];
    const double ax = gx[i], ay = gy[i], az = gz[i];
    const double mg = mx * ax + my * ay + mz * az;
    s[0] += r[i] * (ax * ax + ay * ay + az * az);
    s[1] += mg * mg;
    const double mm = mx * mx + my * my + mz * mz;
    s[2] += (mm == 0.0) ? 0.0 : exp(gamma * log(mm));
  }
  store_partials<256, 3>(s, g, SLOT_EPT, red);
}

// Parseval sum w |xi_tilde|^2 |F_c|^2 over three spectral fields ([kx][ky][kz],
// slot kx = 0 packed as in the other passes, weight 1 there and 2 elsewhere):
// n times sum_c ||grad m_c||^2 for the spectra of the components of m.
__global__ void __launch_bounds__(256) k3_spec_gradnorm(Geo g, const cd* __restrict__ F0, const cd* __restrict__ F1,
                                                         const cd* __restrict__ F2) {
  __shared__ double red[4];
  const size_t ns = (size_t)g.h * g.ny * g.nz;
  double s[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < ns; i += (size_t)gridDim.x * 256) {
    const int kx = (int)(i / ((size_t)g.ny * g.nz));
    const int rem = (int)(i % ((size_t)g.ny * g.nz));
    const int ky = rem / g.nz, kz = rem % g.nz;
    const double xt = xi_col(kx, g.lx), yt = xi_tilde(ky, g.ny, g.ly), zt = xi_tilde(kz, g.nz, g.lz);
    const double w = (kx == 0 ? 1.0 : 2.0) * (xt * xt + yt * yt + zt * zt);
    const cd a = F0[i], b = F1[i], c = F2[i];
    s[0] += w * (a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y + c.x * c.x + c.y * c.y);
  }
  store_partials<256, 1>(s, g, SLOT_EGM, red);
}

// ================================================================ adjoint (grid-stride, physical/spectral)
// phi1'(z) = (e^z (z - 1) + 1) / z^2, by its Taylor series near 0
static __device__ __forceinline__ double dphi1_3(double z) {
  if (fabs(z) < 1e-3) return 0.5 + z * (1.0 / 3.0 + z * (0.125 + z * (1.0 / 30.0)));
  return (expm1(z) * (z - 1.0) + z) / (z * z);
}

// Reverse of activation then relaxation at one grid point (m, g = grad p^k and
// lam = the adjoint after the diffusion stage, three components each): lam_m
// (through both stages) and lam_g (of g), as the 2D adjoint with a third
// component.
static __device__ __forceinline__ void adjoint_point3(const double (&m)[3], const double (&g)[3], const double (&l)[3],
                                                      double c2dt, double gamma, double dt, double relax1,
                                                      double (&lm)[3], double (&lg)[3]) {
  const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  const double z = c2dt * g2;
  const double kap = c2dt * (z > 0.0 ? expm1(z) / z : 1.0);
  const double dkap = c2dt * dphi1_3(z);
  const double gm = g[0] * m[0] + g[1] * m[1] + g[2] * m[2];
  double sv[3];
  for (int c = 0; c < 3; ++c) sv[c] = fma(kap * gm, g[c], m[c]);  // m*
  // relaxation Jacobian (symmetric): fac (I - u u^T) + rho'(s) u u^T, u = m*/|m*|
  double a[3];
  if (gamma == 1.0) {
    for (int c = 0; c < 3; ++c) a[c] = relax1 * l[c];
  } else {
    const double s2 = sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
    const double e1 = 1.0 - gamma;
    if (s2 == 0.0) {
      for (int c = 0; c < 3; ++c) a[c] = gamma > 1.0 ? l[c] : 0.0;
    } else {
      const double u = 2.0 * e1 * dt * exp(-e1 * log(s2));
      if (u >= 1.0) {
        a[0] = a[1] = a[2] = 0.0;
      } else {
        const double fac = exp(log1p(-u) / (2.0 * e1));        // rho / s
        const double drho = exp((1.0 - 2.0 * e1) * log(fac));  // rho'(s) = (s / rho)^{2e - 1}
        const double is = 1.0 / sqrt(s2);
        double uv[3];
        for (int c = 0; c < 3; ++c) uv[c] = sv[c] * is;
        const double ul = uv[0] * l[0] + uv[1] * l[1] + uv[2] * l[2];
        for (int c = 0; c < 3; ++c) a[c] = fac * (l[c] - uv[c] * ul) + drho * ul * uv[c];
      }
    }
  }
  // activation: d m*/d m = I + kap g g^T, and the derivative in g
  const double gl = g[0] * a[0] + g[1] * a[1] + g[2] * a[2];
  const double t = 2.0 * c2dt * dkap * gm * gl;
  for (int c = 0; c < 3; ++c) {
    lm[c] = fma(kap * gl, g[c], a[c]);
    lg[c] = t * g[c] + kap * gl * m[c] + kap * gm * a[c];
  }
}

// lam [3][n] in: the adjoint after the diffusion stage, out: lam_m; G0..G2 in:
// grad p^k (physical), out: lam_g
__global__ void __launch_bounds__(256) k3_adj1(Geo g, const double* __restrict__ m, double* lam, double* G0,
                                                double* G1, double* G2, double c2dt, double gamma, double dt,
                                                double relax1) {
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double mv[3] = {m[i], m[n + i], m[2 * n + i]};
    const double gv[3] = {G0[i], G1[i], G2[i]};
    const double lv[3] = {lam[i], lam[n + i], lam[2 * n + i]};
    double lm[3], lg[3];
    adjoint_point3(mv, gv, lv, c2dt, gamma, dt, relax1, lm, lg);
    lam[i] = lm[0];
    lam[n + i] = lm[1];
    lam[2 * n + i] = lm[2];
    G0[i] = lg[0];
    G1[i] = lg[1];
    G2[i] = lg[2];
  }
}

// Adjoint right-hand side from the spectra of v (three components, [kx][ky][kz],
// slot kx = 0 packed): b_hat = -i xi_tilde . F(v), i.e. F(Pi G^T v) (the null
// modes vanish with xi_tilde; the x multiplier of slot 0 is 0 on both halves)
__global__ void __launch_bounds__(256) k3_spec_divrhs(Geo g, const cd* __restrict__ F0, const cd* __restrict__ F1,
                                                       const cd* __restrict__ F2, cd* __restrict__ bh) {
  const size_t ns = (size_t)g.h * g.ny * g.nz;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < ns; i += (size_t)gridDim.x * 256) {
    const int kx = (int)(i / ((size_t)g.ny * g.nz));
    const int rem = (int)(i % ((size_t)g.ny * g.nz));
    const int ky = rem / g.nz, kz = rem % g.nz;
    const double xt = xi_col(kx, g.lx), yt = xi_tilde(ky, g.ny, g.ly), zt = xi_tilde(kz, g.nz, g.lz);
    const cd a = F0[i], b = F1[i], c = F2[i];
    const double ax = xt * a.x + yt * b.x + zt * c.x, ay = xt * a.y + yt * b.y + zt * c.y;
    bh[i] = mk<double>(ay, -ax);
  }
}

// dL/dS += mu, dL/dr -= grad mu . grad p, lam -= (m.grad p) grad mu + (m.grad mu) grad p
__global__ void __launch_bounds__(256) k3_adj2(Geo g, const double* __restrict__ m, const double* __restrict__ mu,
                                                const double* __restrict__ U0, const double* __restrict__ U1,
                                                const double* __restrict__ U2, const double* __restrict__ P0,
                                                const double* __restrict__ P1, const double* __restrict__ P2,
                                                double* lam, double* grad_r, double* grad_S) {
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double mv[3] = {m[i], m[n + i], m[2 * n + i]};
    const double uv[3] = {U0[i], U1[i], U2[i]}, pv[3] = {P0[i], P1[i], P2[i]};
    const double mgp = mv[0] * pv[0] + mv[1] * pv[1] + mv[2] * pv[2];
    const double mgu = mv[0] * uv[0] + mv[1] * uv[1] + mv[2] * uv[2];
    grad_S[i] += mu[i];
    grad_r[i] -= uv[0] * pv[0] + uv[1] * pv[1] + uv[2] * pv[2];
    for (int c = 0; c < 3; ++c) lam[c * n + i] -= mgp * uv[c] + mgu * pv[c];
  }
}

// totals of the n partials of each of the K arrays of a slot, in a fixed order
template <int K>
__global__ void __launch_bounds__(256) k3_sum_tot(Geo g, int slot, int n) {
  __shared__ double red[K * 4];
  const double* part = g.part + (size_t)slot * SLOT_K * g.pstride;
  double s[K];
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0.0;
  // the loads of all arrays and of several indices are independent: keep many
  // in flight (the sum is latency-bound)
#pragma unroll 4
  for (int i = threadIdx.x; i < n; i += 256) {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] += part[(size_t)k * g.pstride + i];
  }
  block_sum<256, K>(s, red);
  if (threadIdx.x < K) g.tot[slot * SLOT_K + threadIdx.x] = s[threadIdx.x];
}

// ================================================================ launchers
// 3D sizes: powers of two in [8, 1024] per axis.
#define NF3_DISPATCH(N, L_)         \
  switch (N) {                      \
    case 8: L_(8); break;           \
    case 16: L_(16); break;         \
    case 32: L_(32); break;         \
    case 64: L_(64); break;         \
    case 128: L_(128); break;       \
    case 256: L_(256); break;       \
    case 512: L_(512); break;       \
    case 1024: L_(1024); break;     \
    default: return hipErrorInvalidValue; \
  }

#define NF3_LAUNCH(K, GRID, BLK, S, E0, E1, ...)                               \
  do {                                                                         \
    if (E0) hipExtLaunchKernelGGL(K, GRID, BLK, 0, S, E0, E1, 0, __VA_ARGS__); \
    else hipLaunchKernelGGL(K, GRID, BLK, 0, S, __VA_ARGS__);                  \
  } while (0)

static int clamp_tile(int n) {
  const int c = TILE / n;
  return c < 1 ? 1 : (c > 64 ? 64 : c);
}
int nwg3_row(const Geo& g) {
  const int R = clamp_tile(g.nx / 2);
  return (g.ny * g.nz + R - 1) / R;
}
int nwg3_y(const Geo& g) {
  const int C = clamp_tile(g.ny);
  return (g.h * g.nz + C - 1) / C;
}
int nwg3_z(const Geo& g, bool f32) {
  // lines per workgroup of ZCfg: 2 TILE / Nz (FP64), 4 TILE / Nz (FP32 loop passes), in [1, 64]
  const int c0 = (f32 ? 4 : 2) * TILE / g.nz;
  const int C = c0 < 1 ? 1 : (c0 > 64 ? 64 : c0);
  return (g.h * g.ny + C - 1) / C;
}

hipError_t launch3_row_r2c(const Geo& g, const double* f, void* out, int schk, hipStream_t s) {
  const dim3 grid(nwg3_row(g)), blk(TPF);
#define L_(N) hipLaunchKernelGGL(k3_row_r2c<N>, grid, blk, 0, s, g, f, (cd*)out, schk)
  NF3_DISPATCH(g.nx, L_)
#undef L_
  if (schk) {
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch3_sum_tot(g, SLOT_SCHK, 2, nwg3_row(g), s);
  }
  return hipGetLastError();
}
hipError_t launch3_row_c2r(const Geo& g, const void* in, double* f, hipStream_t s) {
  const dim3 grid(nwg3_row(g)), blk(TPF);
#define L_(N) hipLaunchKernelGGL(k3_row_c2r<N>, grid, blk, 0, s, g, (const cd*)in, f)
  NF3_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch3_row_flux(const Geo& g, bool f32, void* G0, void* G1, void* G2, const void* m, const void* r, int it,
                            int kbar, float* lo, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(nwg3_row(g)), blk(3 * TPF);
  if (f32) {
    typedef cx<float> cf;
#define L_(N)                                                                                                   \
  NF3_LAUNCH((k3_row_flux<N, float>), grid, blk, s, e0, e1, g, (cf*)G0, (cf*)G1, (cf*)G2, (const float*)m,     \
             (const float*)r, it, kbar, (float*)nullptr)
    NF3_DISPATCH(g.nx, L_)
#undef L_
  } else {
#define L_(N)                                                                                                   \
  NF3_LAUNCH((k3_row_flux<N, double>), grid, blk, s, e0, e1, g, (cd*)G0, (cd*)G1, (cd*)G2, (const double*)m,    \
             (const double*)r, it, kbar, lo)
    NF3_DISPATCH(g.nx, L_)
#undef L_
  }
  if (kbar) {
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch3_sum_tot(g, SLOT_KBAR, 7, nwg3_row(g), s);
  }
  return hipGetLastError();
}
hipError_t launch3_row_split(const Geo& g, void* P, void* G0, void* G1, void* G2, const double* m, double* p_out,
                             double c2dt, double gamma, double dt, double relax1, double D2dt, hipStream_t s) {
  const dim3 grid(nwg3_row(g)), blk(4 * TPF);
#define L_(N)                                                                                                    \
  hipLaunchKernelGGL(k3_row_split<N>, grid, blk, 0, s, g, (cd*)P, (cd*)G0, (cd*)G1, (const cd*)G2, m, p_out, c2dt, \
                     gamma, dt, relax1, D2dt)
  NF3_DISPATCH(g.nx, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch3_row_final(const Geo& g, const void* M0, const void* M1, const void* M2, double* m, hipStream_t s) {
  const dim3 grid(nwg3_row(g)), blk(3 * TPF);
#define L_(N) hipLaunchKernelGGL(k3_row_final<N>, grid, blk, 0, s, g, (const cd*)M0, (const cd*)M1, (const cd*)M2, m)
  NF3_DISPATCH(g.nx, L_)
#undef L_
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch3_sum_tot(g, SLOT_DM, 2, nwg3_row(g), s);
}

template <int NF, int DIR, typename T>
static hipError_t ypass_t(const Geo& g, void* F0, void* F1, void* F2, void* F3, int it, int stop_test, double tol2,
                          double heat, hipStream_t s) {
  typedef cx<T> cv;
  const dim3 grid(nwg3_y(g)), blk(NF * TPF);
#define L_(N)                                                                                                   \
  hipLaunchKernelGGL((k3_ypass<N, NF, DIR, T>), grid, blk, 0, s, g, (cv*)F0, (cv*)F1, (cv*)F2, (cv*)F3, it,     \
                     stop_test, tol2, heat)
  NF3_DISPATCH(g.ny, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch3_ypass(const Geo& g, bool f32, int nf, int dir, void* F0, void* F1, void* F2, void* F3, int it,
                         int stop_test, double tol2, double heat_D2dt, hipStream_t s) {
#define Y_(NFv, D)                                                                                 \
  return f32 ? ypass_t<NFv, D, float>(g, F0, F1, F2, F3, it, stop_test, tol2, heat_D2dt, s)       \
             : ypass_t<NFv, D, double>(g, F0, F1, F2, F3, it, stop_test, tol2, heat_D2dt, s)
  if (dir < 0) {
    if (nf == 1) Y_(1, -1);
    if (nf == 3) Y_(3, -1);
  } else {
    if (nf == 1) Y_(1, +1);
    if (nf == 3) Y_(3, +1);
    if (nf == 4) Y_(4, +1);
  }
#undef Y_
  return hipErrorInvalidValue;
}

hipError_t launch3_zfwd(const Geo& g, const void* in, void* out, int project, hipStream_t s) {
  const dim3 grid(nwg3_z(g)), blk(TPF);
#define L_(N) hipLaunchKernelGGL(k3_zfwd<N>, grid, blk, 0, s, g, (const cd*)in, (cd*)out, project)
  NF3_DISPATCH(g.nz, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch3_zinv(const Geo& g, int mode, const void* xh, void* P, void* G0, void* G1, void* G2, hipStream_t s) {
  const dim3 grid(nwg3_z(g));
  if (mode == 1) {
#define L_(N) \
  hipLaunchKernelGGL((k3_zinv<N, 1>), grid, dim3(TPF), 0, s, g, (const cd*)xh, (cd*)P, (cd*)G0, (cd*)G1, (cd*)G2)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  } else if (mode == 2) {
#define L_(N) \
  hipLaunchKernelGGL((k3_zinv<N, 2>), grid, dim3(3 * TPF), 0, s, g, (const cd*)xh, (cd*)P, (cd*)G0, (cd*)G1, (cd*)G2)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  } else {
#define L_(N) \
  hipLaunchKernelGGL((k3_zinv<N, 3>), grid, dim3(4 * TPF), 0, s, g, (const cd*)xh, (cd*)P, (cd*)G0, (cd*)G1, (cd*)G2)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  }
  return hipGetLastError();
}
hipError_t launch3_zdiv(const Geo& g, bool f32, int init, const void* F0, const void* F1, const void* F2, void* qh,
                        const void* dh, void* rh, const void* bh, int it, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  const bool lo = f32 && !init;
  const dim3 grid(nwg3_z(g, lo)), blk(6 * TPF);  // FP32: twice the lines, FP64: twice the threads
  if (init) {
#define L_(N)                                                                                                  \
  NF3_LAUNCH((k3_zdiv<N, true, double>), grid, blk, s, e0, e1, g, (const cd*)F0, (const cd*)F1, (const cd*)F2, \
             (cd*)qh, (const cd*)dh, (cd*)rh, (const cd*)bh, it)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  } else if (f32) {
    typedef cx<float> cf;
#define L_(N)                                                                                                    \
  NF3_LAUNCH((k3_zdiv<N, false, float>), grid, blk, s, e0, e1, g, (const cf*)F0, (const cf*)F1, (const cf*)F2,   \
             (cf*)qh, (const cf*)dh, (cf*)rh, (const cf*)nullptr, it)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  } else {
#define L_(N)                                                                                                   \
  NF3_LAUNCH((k3_zdiv<N, false, double>), grid, blk, s, e0, e1, g, (const cd*)F0, (const cd*)F1, (const cd*)F2, \
             (cd*)qh, (const cd*)dh, (cd*)rh, (const cd*)bh, it)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  }
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch3_sum_tot(g, init ? SLOT_P3INIT : SLOT_P3, init ? 3 : 4, nwg3_z(g, lo), s);
}
hipError_t launch3_zupdate(const Geo& g, bool f32, int first, void* xh, void* rh, void* dh, const void* qh, void* G0,
                           void* G1, void* G2, int it, int max_iter, double tol2, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  const dim3 grid(nwg3_z(g, f32)), blk(6 * TPF);  // FP32: twice the lines, FP64: twice the threads
  if (f32) {
    typedef cx<float> cf;
#define L_(N)                                                                                               \
  NF3_LAUNCH((k3_zupdate<N, float>), grid, blk, s, e0, e1, g, 0, (cf*)xh, (cf*)rh, (cf*)dh, (const cf*)qh,  \
             (cf*)G0, (cf*)G1, (cf*)G2, it, max_iter, tol2)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  } else {
#define L_(N)                                                                                                 \
  NF3_LAUNCH((k3_zupdate<N, double>), grid, blk, s, e0, e1, g, first, (cd*)xh, (cd*)rh, (cd*)dh, (const cd*)qh, \
             (cd*)G0, (cd*)G1, (cd*)G2, it, max_iter, tol2)
    NF3_DISPATCH(g.nz, L_)
#undef L_
  }
  const hipError_t e = hipGetLastError();
  // the first update writes no residual norm
  return e != hipSuccess || first ? e : launch3_sum_tot(g, SLOT_RR, 1, nwg3_z(g, f32), s);
}
hipError_t launch3_zheat(const Geo& g, void* M0, void* M1, void* M2, double D2dt, hipStream_t s) {
  const dim3 grid(nwg3_z(g)), blk(3 * TPF);
#define L_(N) hipLaunchKernelGGL(k3_zheat<N>, grid, blk, 0, s, g, (cd*)M0, (cd*)M1, (cd*)M2, D2dt)
  NF3_DISPATCH(g.nz, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch3_zrefine_start(const Geo& g, const void* r64, void* x64, void* x32, void* r32, void* d32, void* G0,
                                 void* G1, void* G2, double tol2, double floor_in, int max_iter, hipStream_t s) {
  typedef cx<float> cf;
  const dim3 grid(nwg3_z(g)), blk(3 * TPF);
#define L_(N)                                                                                                    \
  hipLaunchKernelGGL(k3_zrefine_start<N>, grid, blk, 0, s, g, (const cd*)r64, (cd*)x64, (cf*)x32, (cf*)r32,       \
                     (cf*)d32, (cf*)G0, (cf*)G1, (cf*)G2, tol2, floor_in, max_iter)
  NF3_DISPATCH(g.nz, L_)
#undef L_
  return hipGetLastError();
}
hipError_t launch3_zrefine_acc(const Geo& g, void* x64, const void* x32, void* G0, void* G1, void* G2,
                               hipStream_t s) {
  const dim3 grid(nwg3_z(g)), blk(3 * TPF);
#define L_(N)                                                                                                  \
  hipLaunchKernelGGL(k3_zrefine_acc<N>, grid, blk, 0, s, g, (cd*)x64, (const cx<float>*)x32, (cd*)G0, (cd*)G1, \
                     (cd*)G2)
  NF3_DISPATCH(g.nz, L_)
#undef L_
  return hipGetLastError();
}
// workgroups of the grid-stride energy passes (at most the partial-sum stride)
static int nwg3_energy(const Geo& g) { return g.pstride < 1024 ? g.pstride : 1024; }
static int nwg3_pt(size_t n) {
  const size_t b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}
hipError_t launch3_adj1(const Geo& g, const double* m, double* lam, double* G0, double* G1, double* G2, double c2dt,
                        double gamma, double dt, double relax1, hipStream_t s) {
  hipLaunchKernelGGL(k3_adj1, dim3(nwg3_pt((size_t)g.nx * g.ny * g.nz)), dim3(256), 0, s, g, m, lam, G0, G1, G2, c2dt,
                     gamma, dt, relax1);
  return hipGetLastError();
}
hipError_t launch3_spec_divrhs(const Geo& g, const void* F0, const void* F1, const void* F2, void* bh, hipStream_t s) {
  hipLaunchKernelGGL(k3_spec_divrhs, dim3(nwg3_pt((size_t)g.h * g.ny * g.nz)), dim3(256), 0, s, g, (const cd*)F0,
                     (const cd*)F1, (const cd*)F2, (cd*)bh);
  return hipGetLastError();
}
hipError_t launch3_adj2(const Geo& g, const double* m, const double* mu, const double* U0, const double* U1,
                        const double* U2, const double* P0, const double* P1, const double* P2, double* lam,
                        double* grad_r, double* grad_S, hipStream_t s) {
  hipLaunchKernelGGL(k3_adj2, dim3(nwg3_pt((size_t)g.nx * g.ny * g.nz)), dim3(256), 0, s, g, m, mu, U0, U1, U2, P0,
                     P1, P2, lam, grad_r, grad_S);
  return hipGetLastError();
}
hipError_t launch3_energy_pt(const Geo& g, const double* m, const double* r, const double* gx, const double* gy,
                             const double* gz, double gamma, hipStream_t s) {
  const int nwg = nwg3_energy(g);
  hipLaunchKernelGGL(k3_energy_pt, dim3(nwg), dim3(256), 0, s, g, m, r, gx, gy, gz, gamma);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch3_sum_tot(g, SLOT_EPT, 3, nwg, s);
}
hipError_t launch3_spec_gradnorm(const Geo& g, const void* F0, const void* F1, const void* F2, hipStream_t s) {
  const int nwg = nwg3_energy(g);
  hipLaunchKernelGGL(k3_spec_gradnorm, dim3(nwg), dim3(256), 0, s, g, (const cd*)F0, (const cd*)F1, (const cd*)F2);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch3_sum_tot(g, SLOT_EGM, 1, nwg, s);
}

hipError_t launch3_copy_tot(const Geo& g, int slot, int K, int o, hipStream_t s) {
  hipLaunchKernelGGL(k3_copy_tot, dim3(1), dim3(64), 0, s, g, slot, K, o);
  return hipGetLastError();
}
hipError_t launch3_sum_tot(const Geo& g, int slot, int K, int n, hipStream_t s) {
  if (n < 1 || n > g.pstride) return hipErrorInvalidValue;
  switch (K) {
    case 1: hipLaunchKernelGGL(k3_sum_tot<1>, dim3(1), dim3(256), 0, s, g, slot, n); break;
    case 2: hipLaunchKernelGGL(k3_sum_tot<2>, dim3(1), dim3(256), 0, s, g, slot, n); break;
    case 3: hipLaunchKernelGGL(k3_sum_tot<3>, dim3(1), dim3(256), 0, s, g, slot, n); break;
    case 4: hipLaunchKernelGGL(k3_sum_tot<4>, dim3(1), dim3(256), 0, s, g, slot, n); break;
    case 7: hipLaunchKernelGGL(k3_sum_tot<7>, dim3(1), dim3(256), 0, s, g, slot, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nf
