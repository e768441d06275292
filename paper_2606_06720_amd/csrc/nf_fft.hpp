// Device-side building blocks of the spectral solver: complex arithmetic,
// radix-2/4/8 butterflies, an in-LDS Stockham autosort FFT over a batch of
// lines, the real<->half-complex post/pre-processing of the x transform, and
// deterministic workgroup reductions.
//
// The FFT replaces the paper's CPU FFT library (Sec. 2.3.3); transforms are
// unnormalised in both directions, normalisation is folded into the spectral
// multipliers by the callers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nf {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> scl(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk<T>(a.x, -a.y); }
// a * b
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
  return mk<T>(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// multiply by i (DIR=+1) or -i (DIR=-1)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  return DIR > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
// multiply by e^{DIR i pi/4}
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_w8(cx<T> a) {
  const T s = (T)0.70710678118654752440;
  return DIR > 0 ? mk<T>((a.x - a.y) * s, (a.x + a.y) * s) : mk<T>((a.x + a.y) * s, (a.y - a.x) * s);
}
// multiply by e^{DIR 3 i pi/4}
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_w83(cx<T> a) {
  const T s = (T)0.70710678118654752440;
  return DIR > 0 ? mk<T>(-(a.x + a.y) * s, (a.x - a.y) * s) : mk<T>((a.y - a.x) * s, -(a.x + a.y) * s);
}

// ---------------------------------------------------------------- butterflies
// In-place DFT of size R on v[0..R-1]: v_m <- sum_q v_q e^{DIR 2 pi i q m / R}.
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = add(a, b);
  v[1] = sub(a, b);
}
template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>& b0, cx<T>& b1, cx<T>& b2, cx<T>& b3) {
  cx<T> s02 = add(b0, b2), d02 = sub(b0, b2);
  cx<T> s13 = add(b1, b3), d13 = mul_i<DIR>(sub(b1, b3));
  b0 = add(s02, s13);
  b2 = sub(s02, s13);
  b1 = add(d02, d13);
  b3 = sub(d02, d13);
}
template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  dft4<DIR>(v[0], v[1], v[2], v[3]);
}
template <int DIR, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  // decimation in frequency: even outputs from v_q + v_{q+4}, odd outputs from
  // (v_q - v_{q+4}) w8^q, each followed by a 4-point DFT
  cx<T> a0 = add(v[0], v[4]), a4 = sub(v[0], v[4]);
  cx<T> a1 = add(v[1], v[5]), a5 = sub(v[1], v[5]);
  cx<T> a2 = add(v[2], v[6]), a6 = sub(v[2], v[6]);
  cx<T> a3 = add(v[3], v[7]), a7 = sub(v[3], v[7]);
  a5 = mul_w8<DIR>(a5);
  a6 = mul_i<DIR>(a6);
  a7 = mul_w83<DIR>(a7);
  dft4<DIR>(a0, a1, a2, a3);
  dft4<DIR>(a4, a5, a6, a7);
  v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
  v[1] = a4; v[3] = a5; v[5] = a6; v[7] = a7;
}
// 5-point DFT: with t1 = v1 + v4, t2 = v2 + v3, t3 = v1 - v4, t4 = v2 - v3 the
// outputs are X0 = v0 + t1 + t2, X1,4 = a1 +- DIR i b1, X2,3 = a2 +- DIR i b2 where
// a1 = v0 + c1 t1 + c2 t2, a2 = v0 + c2 t1 + c1 t2, b1 = s1 t3 + s2 t4,
// b2 = s2 t3 - s1 t4 (c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5)).
template <int DIR, typename T>
__device__ __forceinline__ void dft5(cx<T>* v) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
  const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
  const cx<T> t1 = add(v[1], v[4]), t2 = add(v[2], v[3]);
  const cx<T> t3 = sub(v[1], v[4]), t4 = sub(v[2], v[3]);
  const cx<T> a1 = add(v[0], add(scl(t1, c1), scl(t2, c2)));
  const cx<T> a2 = add(v[0], add(scl(t1, c2), scl(t2, c1)));
  const cx<T> b1 = mul_i<DIR>(add(scl(t3, s1), scl(t4, s2)));
  const cx<T> b2 = mul_i<DIR>(sub(scl(t3, s2), scl(t4, s1)));
  v[0] = add(v[0], add(t1, t2));
  v[1] = add(a1, b1);
  v[4] = sub(a1, b1);
  v[2] = add(a2, b2);
  v[3] = sub(a2, b2);
}
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 5) dft5<DIR>(v);
  else dft8<DIR>(v);
}

// ---------------------------------------------------------------- radix plan
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }
// Radices of a length-2^p transform: as many 8s as possible with a tail of 4,
// 4,4 or a lone 2.  Plan 0 runs the 8s first, plan 1 the tail first (the two
// differ when p is not a multiple of 3); the run-time tuner picks between them.
constexpr int plan_nstages(int p) {
  return p <= 2 ? 1 : (p % 3 == 0 ? p / 3 : (p % 3 == 2 ? p / 3 + 1 : p / 3 + 1));
}
constexpr int plan_radix(int p, int s, int pl = 0) {
  if (p == 1) return 2;
  if (p == 2) return 4;
  if (p % 3 == 0) return 8;
  // number of tail stages: one 4 (p % 3 == 2) or two 4s (p % 3 == 1)
  const int nt = p % 3 == 2 ? 1 : 2;
  const int n8 = plan_nstages(p) - nt;
  return pl == 0 ? (s < n8 ? 8 : 4) : (s < nt ? 4 : 8);
}
constexpr int plan_ns(int p, int s, int pl = 0) {  // product of radices before stage s
  return s == 0 ? 1 : plan_ns(p, s - 1, pl) * plan_radix(p, s - 1, pl);
}
// whether plan 1 differs from plan 0 for a length-2^p transform
constexpr bool plan_has_alt(int p) { return p > 2 && p % 3 != 0; }
// Lengths n = 5^k 2^p: k radix-5 stages first, then the power-of-two plan above.
constexpr int f5(int n) { return n % 5 == 0 ? 1 + f5(n / 5) : 0; }
constexpr int pow5(int k) { return k == 0 ? 1 : 5 * pow5(k - 1); }
constexpr int mplan_nstages(int n) {
  return f5(n) + (n / pow5(f5(n)) == 1 ? 0 : plan_nstages(ilog2(n / pow5(f5(n)))));
}
constexpr int mplan_radix(int n, int s, int pl = 0) {
  return s < f5(n) ? 5 : plan_radix(ilog2(n / pow5(f5(n))), s - f5(n), pl);
}
constexpr int mplan_ns(int n, int s, int pl = 0) {
  return s == 0 ? 1 : mplan_ns(n, s - 1, pl) * mplan_radix(n, s - 1, pl);
}
constexpr bool plan_ok(int n) { return pow5(f5(n)) * (1 << ilog2(n / pow5(f5(n)))) == n; }

// Twiddle e^{DIR 2 pi i t / M} from the table tw[u] = e^{-2 pi i u / TWN}, where
// mult = TWN / M (TWN is a common multiple of every transform length).
template <int DIR, typename T>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int t, int mult) {
  cx<T> w = tw[t * mult];
  return DIR > 0 ? conj(w) : w;
}

// One Stockham stage over B lines of length L stored at buf + line*LS.
// Inputs are read at stride L/R, outputs written in autosort order.
// Intermediate results between stages live in a padded line layout (one
// spare slot after every 8 elements, lpad below): the first stage's outputs,
// 8 consecutive elements per butterfly, then fall on distinct LDS banks.  The
// first stage reads and the last stage writes the natural layout, so a line
// needs LS >= lpad_len(L) slots (the padding is used when it has them).
__host__ __device__ constexpr int lpad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lpad_len(int L) { return L + (L >> 3) + 1; }
// Lines longer than 1024 keep the natural layout: there the extra index
// arithmetic costs more registers than the bank conflicts cost time.
__host__ __device__ constexpr bool lpad_use(int L) { return L <= 1024; }

// Order the LDS accesses of one wave without a workgroup barrier: the LDS
// executes a wave's instructions in issue order, so a compiler fence that keeps
// the accesses of two stages apart is enough when the data stays in the wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// WL: every wave reads and writes only lines it owns (see wave_local_ok), so
// the stage's barriers are wave-level, except a workgroup barrier after the
// last stage (LAST) for the cross-wave phase that follows.
template <typename T, int DIR, int L, int B, int LS, int NT, int R, int NS, bool PIN, bool POUT, bool WL = false,
          bool LAST = true>
__device__ __forceinline__ void fft_stage(cx<T>* buf, const cx<T>* __restrict__ tw, int twn) {
  static_assert(!(PIN || POUT) || LS >= lpad_len(L), "line stride too small for the padded layout");
  constexpr int Q = L / R;          // butterflies per line
  constexpr int NBF = B * Q;        // butterflies in the batch
  constexpr int PER = (NBF + NT - 1) / NT;
  constexpr bool EXACT = (PER * NT == NBF);
  const int tid = threadIdx.x;
  cx<T> v[PER][R];
  cx<T> w[PER][R];
  // the table has twn entries, this stage needs angles in units of
  // 2 pi / (NS R).  The table loads are issued before the barrier so that
  // their latency overlaps the LDS traffic.
  const int mult = twn / (NS * R);
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int f = tid + b * NT;
    if (EXACT || f < NBF) {
      const int line = f / Q, j = f % Q;
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int q = 1; q < R; ++q) w[b][q] = twiddle<DIR>(tw, q * k, mult);
      }
      if constexpr (PIN) {
        const cx<T>* src = buf + line * LS;
#pragma unroll
        for (int q = 0; q < R; ++q) v[b][q] = src[lpad(j + q * Q)];
      } else {
        const cx<T>* src = buf + line * LS + j;
#pragma unroll
        for (int q = 0; q < R; ++q) v[b][q] = src[q * Q];
      }
    }
  }
  if constexpr (WL) wave_sync();
  else __syncthreads();
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int f = tid + b * NT;
    if (EXACT || f < NBF) {
      const int line = f / Q, j = f % Q;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) v[b][q] = mul(v[b][q], w[b][q]);
      }
      dft<R, DIR>(v[b]);
      if constexpr (POUT) {
        cx<T>* dst = buf + line * LS;
        const int o = (j / NS) * NS * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) dst[lpad(o + q * NS)] = v[b][q];
      } else {
        cx<T>* dst = buf + line * LS + (j / NS) * NS * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) dst[q * NS] = v[b][q];
      }
    }
  }
  if constexpr (WL && !LAST) wave_sync();
  else __syncthreads();
}

// Whether every wave owns whole lines, the same ones in every stage: all
// stages of one radix R0 (so the butterflies per line, Q = L / R0, are the same
// in each stage), at most 64 butterflies per line with 64 a multiple of Q, and
// whole waves.
template <int L, int NT, int PL>
constexpr bool wave_local_ok() {
  if (mplan_nstages(L) < 1 || NT % 64 != 0) return false;
  const int r0 = mplan_radix(L, 0, PL);
  for (int s = 1; s < mplan_nstages(L); ++s)
    if (mplan_radix(L, s, PL) != r0) return false;
  const int q = L / r0;
  return q <= 64 && 64 % q == 0;
}

template <typename T, int DIR, int L, int B, int LS, int NT, int S, int PL>
__device__ __forceinline__ void fft_stages(cx<T>* buf, const cx<T>* __restrict__ tw, int twn) {
  static_assert(plan_ok(L), "transform lengths are 5^k 2^p");
  if constexpr (S < mplan_nstages(L)) {
    constexpr bool PAD = lpad_use(L) && LS >= lpad_len(L);
    constexpr bool WL = wave_local_ok<L, NT, PL>();
    fft_stage<T, DIR, L, B, LS, NT, mplan_radix(L, S, PL), mplan_ns(L, S, PL), PAD && (S > 0),
              PAD && (S + 1 < mplan_nstages(L)), WL, S + 1 == mplan_nstages(L)>(buf, tw, twn);
    fft_stages<T, DIR, L, B, LS, NT, S + 1, PL>(buf, tw, twn);
  }
}

// In-LDS FFT of B lines of length L (line stride LS), all NT threads taking part,
// with radix plan PL (see plan_radix).
// Caller must __syncthreads() before (data written) -- the routine ends with a barrier.
template <typename T, int DIR, int L, int B, int LS, int NT, int PL = 0>
__device__ __forceinline__ void lds_fft(cx<T>* buf, const cx<T>* __restrict__ tw, int twn) {
  fft_stages<T, DIR, L, B, LS, NT, 0, PL>(buf, tw, twn);
}

// ------------------------------------------------- real <-> half-complex (x axis)
// A real line f[0..N-1], N = 2H, is packed as z[j] = f[2j] + i f[2j+1] and
// transformed with a length-H complex FFT Z.  rfft_post turns Z into the first H
// coefficients X[0..H-1] of the length-N DFT, with the (real) X[0] and X[H]
// packed into slot 0 as X[0] + i X[H].  irfft_pre is its inverse (up to the
// factor N of an unnormalised inverse): it rebuilds 2 Z from the packed X, so
// that an unnormalised length-H inverse FFT gives N (f[2j] + i f[2j+1]).
// Both work on B lines in place; one thread per pair (k, H-k), k in [1, H/2),
// and one for slot 0 (which also handles the self-paired k = H/2 when H is even).
template <typename T, int H, int B, int LS, int NT>
__device__ __forceinline__ void rfft_post(cx<T>* buf, const cx<T>* __restrict__ tw, int twn) {
  constexpr int NP = (H + 1) / 2;
  constexpr int NTASK = B * NP;
  const int mult = twn / (2 * H);
  for (int t = threadIdx.x; t < NTASK; t += NT) {
    const int line = t / NP, k = t % NP;
    cx<T>* l = buf + line * LS;
    if (k == 0) {
      cx<T> z0 = l[0];
      l[0] = mk<T>(z0.x + z0.y, z0.x - z0.y);
      if (H % 2 == 0) {
        // self-paired k = H/2: w^{H/2} = -i, X = conj(Z)
        cx<T> zh = l[H / 2];
        l[H / 2] = conj(zh);
      }
    } else {
      cx<T> zk = l[k], zm = l[H - k];
      cx<T> w = tw[k * mult];                        // e^{-2 pi i k / N}
      // X[k]   = (zk + conj zm)/2 - (i/2) w (zk - conj zm)
      // X[H-k] = (zm + conj zk)/2 + (i/2) conj(w) (zm - conj zk)
      cx<T> e1 = add(zk, conj(zm)), o1 = sub(zk, conj(zm));
      cx<T> e2 = add(zm, conj(zk)), o2 = sub(zm, conj(zk));
      cx<T> t1 = mul_i<-1>(mul(w, o1));
      cx<T> t2 = mul_i<+1>(mul(conj(w), o2));
      l[k] = scl(add(e1, t1), (T)0.5);
      l[H - k] = scl(add(e2, t2), (T)0.5);
    }
  }
  __syncthreads();
}

template <typename T, int H, int B, int LS, int NT>
__device__ __forceinline__ void irfft_pre(cx<T>* buf, const cx<T>* __restrict__ tw, int twn) {
  constexpr int NP = (H + 1) / 2;
  constexpr int NTASK = B * NP;
  const int mult = twn / (2 * H);
  for (int t = threadIdx.x; t < NTASK; t += NT) {
    const int line = t / NP, k = t % NP;
    cx<T>* l = buf + line * LS;
    if (k == 0) {
      cx<T> p = l[0];  // X[0] + i X[H]
      l[0] = mk<T>(p.x + p.y, p.x - p.y);
      if (H % 2 == 0) {
        // self-paired k = H/2: 2 Z = 2 conj(X)
        cx<T> xh = l[H / 2];
        l[H / 2] = mk<T>(xh.x + xh.x, -(xh.y + xh.y));
      }
    } else {
      cx<T> xk = l[k], xm = l[H - k];
      cx<T> w = tw[k * mult];  // e^{-2 pi i k / N}
      // 2Z[k]   = (xk + conj xm) + i conj(w) (xk - conj xm)
      // 2Z[H-k] = (xm + conj xk) - i w (xm - conj xk)
      cx<T> e1 = add(xk, conj(xm)), o1 = sub(xk, conj(xm));
      cx<T> e2 = add(xm, conj(xk)), o2 = sub(xm, conj(xk));
      l[k] = add(e1, mul_i<+1>(mul(conj(w), o1)));
      l[H - k] = add(e2, mul_i<-1>(mul(w, o2)));
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- reductions
// Deterministic workgroup sum of K doubles per thread: wavefront butterfly via
// shuffles, then a fixed-order pass over the waves.  Every thread gets the result.
template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* scratch /* >= K*NT/64 */) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) scratch[k * NW + wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += scratch[k * NW + w];
    v[k] = s;
  }
  __syncthreads();
}

// Sum K arrays of n partials (layout part[k*stride + i]) in a fixed order; the
// result is bitwise identical in every workgroup that calls it.
template <int NT, int K>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int n, int stride,
                                             double (&out)[K], double* scratch) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) s += part[k * stride + i];
    out[k] = s;
  }
  block_sum<NT, K>(out, scratch);
}

}  // namespace nf
