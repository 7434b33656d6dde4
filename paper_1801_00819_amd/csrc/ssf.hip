// Split-step Fourier shot-profile operators on gfx950: the de-migration /
// migration family of the paper's examples (Examples section), with the
// operator defined in brrlsm_ssf.h.
//
// One workgroup marches one (shot, frequency) pair through every depth
// level. The lateral wavefield (nx = N complex points) lives in registers,
// four points per thread at positions t + r N/4; each depth step is a
// forward FFT, the wavenumber-domain phase, an inverse FFT and the
// split-step phase and taper. The FFTs are radix-4 Stockham passes (a
// radix-2 pass first when log2 N is odd) whose first input and last output
// are already in the register layout, so an N-point FFT needs
// ceil(log2 N / 2) - 1 exchanges through LDS, one barrier each (two LDS
// buffers used alternately). Twiddles depend only on the thread and the
// pass, so they sit in registers for the whole march.
//
// Phase angles (kz dz and w theta) are formed and reduced in double and
// only then rounded to float for sincos: the same rounded factor is applied
// at every level, so a float error in the angle would grow linearly with
// depth.
#include <hip/hip_runtime.h>

#include "ssf_kernels.h"

namespace brls {
namespace {

constexpr double kTwoPi = 6.283185307179586;
constexpr double kInvTwoPi = 0.15915494309189535;

// Complex numbers as (x, y) pairs in float (the operator marches) or double
// (the source march, whose result every later application reuses).
template <typename T>
struct Cplx;
template <>
struct Cplx<float> {
  using V = float2;
};
template <>
struct Cplx<double> {
  using V = double2;
};

template <typename V>
__device__ inline V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename V>
__device__ inline V cadd(V a, V b) {
  V r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename V>
__device__ inline V csub(V a, V b) {
  V r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <typename V, typename S>
__device__ inline V cscale(V a, S s) {
  V r;
  r.x = a.x * s;
  r.y = a.y * s;
  return r;
}
template <typename V>
__device__ inline V czero() {
  V r;
  r.x = 0;
  r.y = 0;
  return r;
}

// e^{i a}. Float: the angle reduced to [-pi, pi] in double before the float
// sincos. Double: sincos of the angle.
template <typename T>
__device__ inline typename Cplx<T>::V cis(double a);
template <>
__device__ inline float2 cis<float>(double a) {
  const double r = fma(-kTwoPi, rint(a * kInvTwoPi), a);
  float s, c;
  sincosf((float)r, &s, &c);
  return make_float2(c, s);
}
template <>
__device__ inline double2 cis<double>(double a) {
  double s, c;
  sincos(a, &s, &c);
  return make_double2(c, s);
}

template <int L>
struct Geo {
  static constexpr int N = 1 << L;
  static constexpr int Q = N / 4;
  static constexpr int kBlock = Q < 64 ? 64 : Q;
  static constexpr int kOdd = L & 1;
  static constexpr int kPasses = L / 2;  // radix-4 passes
};

// Per-thread twiddles of every radix-4 pass: tw^(r jm N / (4 Ns)), r = 1..3.
template <int L, typename V>
struct Twiddles {
  V w[Geo<L>::kPasses][3];
};

template <int L, typename V>
__device__ void load_twiddles(Twiddles<L, V>& T, const V* __restrict__ tw,
                              int t) {
  constexpr int N = Geo<L>::N;
#pragma unroll
  for (int p = 0; p < Geo<L>::kPasses; ++p) {
    const int Ns = (Geo<L>::kOdd ? 2 : 1) << (2 * p);
    const int jm = t & (Ns - 1);
    const int st = N / (4 * Ns);
#pragma unroll
    for (int r = 1; r <= 3; ++r)
      T.w[p][r - 1] = (t < Geo<L>::Q) ? tw[(r * jm * st) & (N - 1)]
                                      : czero<V>();
  }
}

// Forward DFT (e^{-2 pi i q x / N}) of the N points held four per thread,
// in place in the same layout (frequency q = t + r N/4 afterwards).
template <int L, typename V>
__device__ void fft(V v[4], V* __restrict__ b0, V* __restrict__ b1,
                    const Twiddles<L, V>& T, int t, int& pb) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  const bool on = t < Q;
  if constexpr (Geo<L>::kOdd) {
    V* y = pb ? b1 : b0;
    if (on) {
      y[2 * t] = cadd(v[0], v[2]);
      y[2 * t + 1] = csub(v[0], v[2]);
      y[2 * t + 2 * Q] = cadd(v[1], v[3]);
      y[2 * t + 2 * Q + 1] = csub(v[1], v[3]);
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = y[t + r * Q];
    }
    pb ^= 1;
  }
#pragma unroll
  for (int p = 0; p < Geo<L>::kPasses; ++p) {
    const int Ns = (Geo<L>::kOdd ? 2 : 1) << (2 * p);
    if (Ns > 1) {
      v[1] = cmul(v[1], T.w[p][0]);
      v[2] = cmul(v[2], T.w[p][1]);
      v[3] = cmul(v[3], T.w[p][2]);
    }
    const V a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const V a2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    V a3;  // -i d
    a3.x = d.y;
    a3.y = -d.x;
    v[0] = cadd(a0, a2);
    v[1] = cadd(a1, a3);
    v[2] = csub(a0, a2);
    v[3] = csub(a1, a3);
    if (Ns == Q) break;  // last pass: outputs already at t + r N/4
    V* y = pb ? b1 : b0;
    const int jm = t & (Ns - 1);
    const int base = (t - jm) * 4 + jm;
    if (on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) y[base + r * Ns] = v[r];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = y[t + r * Q];
    }
    pb ^= 1;
  }
  (void)N;
}

// Unscaled inverse DFT through the forward one: conj(F(conj(v))).
template <int L, typename V>
__device__ void ifft(V v[4], V* b0, V* b1, const Twiddles<L, V>& T, int t,
                     int& pb) {
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r].y = -v[r].y;
  fft<L, V>(v, b0, b1, T, t, pb);
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r].y = -v[r].y;
}

// Wavenumber-domain factor e^{-i kz dz} (e^{-|kz| dz} where evanescent).
template <typename T>
__device__ inline typename Cplx<T>::V kz_phase(double ws0, double kx2,
                                               double dz) {
  const double a = ws0 * ws0 - kx2;
  if (a >= 0.0) return cis<T>(-sqrt(a) * dz);
  typename Cplx<T>::V r;
  r.x = (T)exp(-sqrt(-a) * dz);
  r.y = 0;
  return r;
}

// State of one workgroup's march: its frequency and the thread's columns.
template <int L, typename T>
struct March {
  using V = typename Cplx<T>::V;
  int t;
  double w;        // angular frequency
  double kx2[4];   // squared wavenumbers of the thread's four q
  Twiddles<L, V> tw;
  int pb = 0;
};

template <int L, typename T>
__device__ void march_init(March<L, T>& s, const SsfArgs& a, int k,
                           const typename Cplx<T>::V* tw) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  s.t = threadIdx.x;
  s.w = (double)(a.k0 + k) * a.dw;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = s.t + r * Q;
    const int qs = r < 2 ? q : q - N;
    const double kx = qs * a.kx_unit;
    s.kx2[r] = kx * kx;
  }
  load_twiddles<L>(s.tw, tw, s.t);
}

// v <- E_j v
template <int L, typename T, typename V>
__device__ void step_down(March<L, T>& s, const SsfArgs& a, int j, V v[4],
                          V* b0, V* b1) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  constexpr T kInvN = T(1) / N;
  fft<L, V>(v, b0, b1, s.tw, s.t, s.pb);
  const double ws0 = s.w * a.s0[j];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    v[r] = cscale(cmul(v[r], kz_phase<T>(ws0, s.kx2[r], a.dz)), kInvN);
  ifft<L, V>(v, b0, b1, s.tw, s.t, s.pb);
  if (s.t < Q) {
    const double* th = a.theta + (int64_t)j * N;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = s.t + r * Q;
      v[r] = cscale(cmul(v[r], cis<T>(-s.w * th[x])), (T)a.tau[x]);
    }
  }
}

// v <- E_j^H v
template <int L, typename T, typename V>
__device__ void step_up_adj(March<L, T>& s, const SsfArgs& a, int j, V v[4],
                            V* b0, V* b1) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  constexpr T kInvN = T(1) / N;
  if (s.t < Q) {
    const double* th = a.theta + (int64_t)j * N;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = s.t + r * Q;
      v[r] = cscale(cmul(v[r], cis<T>(s.w * th[x])), (T)a.tau[x]);
    }
  }
  fft<L, V>(v, b0, b1, s.tw, s.t, s.pb);
  const double ws0 = s.w * a.s0[j];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    V p = kz_phase<T>(ws0, s.kx2[r], a.dz);
    p.y = -p.y;
    v[r] = cscale(cmul(v[r], p), kInvN);
  }
  ifft<L, V>(v, b0, b1, s.tw, s.t, s.pb);
}

// --- source: Born weights W_j = -i (w dz/2) s_j S_j for one slot ---------
// The source field is marched in double (it runs once per shot and every
// later application of A and A^T reads its result); W is stored in float.
template <int L>
__global__ __launch_bounds__(Geo<L>::kBlock) void k_ssf_source(
    SsfArgs a, int slot, int xs) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  __shared__ double2 b0[N], b1[N];
  const int k = blockIdx.x;
  March<L, double> s;
  march_init<L, double>(s, a, k, a.tw64);
  const bool on = s.t < Q;
  double2 v[4];
  const double2 f = a.wav[(int64_t)slot * a.nw + k];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    v[r] = (on && s.t + r * Q == xs) ? f : czero<double2>();
  float2* Wb = a.W + ((int64_t)slot * a.nw + k) * a.nz * N;
  const double c = 0.5 * s.w * a.dz;
  for (int j = 0; j < a.nz; ++j) {
    if (on) {
      const double* th = a.theta + (int64_t)j * N;
      const double s0 = a.s0[j];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = s.t + r * Q;
        const double cs = c * (s0 + th[x] / a.dz);  // (w dz / 2) s_j(x)
        Wb[(int64_t)j * N + x] =
            make_float2((float)(cs * v[r].y), (float)(-cs * v[r].x));
      }
    }
    if (j + 1 < a.nz) step_down<L, double>(s, a, j, v, b0, b1);
  }
}

// --- A: upward recursion R_j = W_j m_j + E_j R_{j+1}, receivers of R_0 ---
template <int L>
__global__ __launch_bounds__(Geo<L>::kBlock) void k_ssf_born(
    SsfArgs a, const float* __restrict__ m, float* __restrict__ d) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  __shared__ float2 b0[N], b1[N];
  const int item = blockIdx.x;
  const int i = item / a.nw, k = item - i * a.nw;
  const SsfShotDev sh = a.tab[i];
  March<L, float> s;
  march_init<L, float>(s, a, k, a.tw);
  const bool on = s.t < Q;
  const float2* Wb = a.W + ((int64_t)sh.slot * a.nw + k) * a.nz * N;
  float2 v[4];
  {
    const int j = a.nz - 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = s.t + r * Q;
      v[r] = on ? cscale(Wb[(int64_t)j * N + x], m[(int64_t)j * N + x])
                : czero<float2>();
    }
  }
  for (int j = a.nz - 2; j >= 0; --j) {
    step_down<L, float>(s, a, j, v, b0, b1);
    if (on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = s.t + r * Q;
        const float2 wv = Wb[(int64_t)j * N + x];
        const float mv = m[(int64_t)j * N + x];
        v[r].x = fmaf(wv.x, mv, v[r].x);
        v[r].y = fmaf(wv.y, mv, v[r].y);
      }
    }
  }
  // gather the receivers' columns of R_0
  __syncthreads();
  if (on) {
#pragma unroll
    for (int r = 0; r < 4; ++r) b0[s.t + r * Q] = v[r];
  }
  __syncthreads();
  const int* rec = a.rec + (int64_t)sh.slot * a.nrec_max;
  float* out = d + (int64_t)sh.slot * a.seg + (int64_t)k * sh.nrec * 2;
  for (int r = s.t; r < sh.nrec; r += Geo<L>::kBlock) {
    const float2 val = b0[rec[r]];
    out[2 * r] = val.x;
    out[2 * r + 1] = val.y;
  }
}

// --- A^T: downward adjoint recursion, per-item image contributions ---------
template <int L>
__global__ __launch_bounds__(Geo<L>::kBlock) void k_ssf_adjoint(
    SsfArgs a, const float* __restrict__ d, float* __restrict__ part) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  __shared__ float2 b0[N], b1[N];
  const int item = blockIdx.x;
  const int i = item / a.nw, k = item - i * a.nw;
  const SsfShotDev sh = a.tab[i];
  March<L, float> s;
  march_init<L, float>(s, a, k, a.tw);
  const bool on = s.t < Q;
  const float2* Wb = a.W + ((int64_t)sh.slot * a.nw + k) * a.nz * N;
  // the receivers' data placed in their columns (repeats summed in order)
  float2 v[4];
  {
    const int* cp = a.colptr + (int64_t)sh.slot * (N + 1);
    const int* ci = a.cidx + (int64_t)sh.slot * a.nrec_max;
    const float* din = d + (int64_t)sh.slot * a.seg + (int64_t)k * sh.nrec * 2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float2 acc = make_float2(0.f, 0.f);
      if (on) {
        const int x = s.t + r * Q;
        for (int e = cp[x]; e < cp[x + 1]; ++e) {
          const int ri = ci[e];
          acc.x += din[2 * ri];
          acc.y += din[2 * ri + 1];
        }
      }
      v[r] = acc;
    }
  }
  float* pb = part + (int64_t)item * a.nz * N;
  for (int j = 0; j < a.nz; ++j) {
    if (on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = s.t + r * Q;
        const float2 wv = Wb[(int64_t)j * N + x];
        pb[(int64_t)j * N + x] = fmaf(wv.x, v[r].x, wv.y * v[r].y);
      }
    }
    if (j + 1 < a.nz) step_up_adj<L, float>(s, a, j, v, b0, b1);
  }
}

__global__ void k_ssf_image_sum(const float* __restrict__ part, int items,
                                int64_t npts, float* __restrict__ img) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  double acc = 0.0;
  for (int i = 0; i < items; ++i) acc += part[(int64_t)i * npts + p];
  img[p] = (float)acc;
}

// One thread per (frequency, receiver): the DFT sum in double, the kernel
// e^{-i w n dt} advanced by rotation and reset exactly every 64 samples.
__global__ void k_ssf_data_dft(const float* __restrict__ x, int nt, int nrec,
                               double dt, int k0, double dw,
                               float* __restrict__ X) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= nrec) return;
  const double w = (double)(k0 + k) * dw;
  double rs, rc;
  sincos(-w * dt, &rs, &rc);
  double re = 0.0, im = 0.0;
  for (int n0 = 0; n0 < nt; n0 += 64) {
    double es, ec;
    sincos(-w * dt * n0, &es, &ec);
    const int n1 = n0 + 64 < nt ? n0 + 64 : nt;
    for (int n = n0; n < n1; ++n) {
      const double xv = x[(int64_t)n * nrec + r];
      re = fma(xv, ec, re);
      im = fma(xv, es, im);
      const double c2 = ec * rc - es * rs;
      es = ec * rs + es * rc;
      ec = c2;
    }
  }
  X[((int64_t)k * nrec + r) * 2] = (float)(re * dt);
  X[((int64_t)k * nrec + r) * 2 + 1] = (float)(im * dt);
}

}  // namespace

#define SSF_DISPATCH(L_, CALL)                                  \
  switch (L_) {                                                 \
    case 6: { constexpr int L = 6; CALL; break; }               \
    case 7: { constexpr int L = 7; CALL; break; }               \
    case 8: { constexpr int L = 8; CALL; break; }               \
    case 9: { constexpr int L = 9; CALL; break; }               \
    case 10: { constexpr int L = 10; CALL; break; }             \
    case 11: { constexpr int L = 11; CALL; break; }             \
    default: return hipErrorInvalidValue;                       \
  }

hipError_t launch_ssf_source(const SsfArgs& a, int slot, int xs,
                             hipStream_t st) {
  if (a.nw <= 0) return hipSuccess;
  SSF_DISPATCH(a.log2n,
               hipLaunchKernelGGL(k_ssf_source<L>, dim3(a.nw),
                                  dim3(Geo<L>::kBlock), 0, st, a, slot, xs));
  return hipGetLastError();
}

hipError_t launch_ssf_born(const SsfArgs& a, const float* m, float* d,
                           hipStream_t st) {
  const int items = a.nshots * a.nw;
  if (items <= 0) return hipSuccess;
  SSF_DISPATCH(a.log2n,
               hipLaunchKernelGGL(k_ssf_born<L>, dim3(items),
                                  dim3(Geo<L>::kBlock), 0, st, a, m, d));
  return hipGetLastError();
}

hipError_t launch_ssf_adjoint(const SsfArgs& a, const float* d, float* part,
                              hipStream_t st) {
  const int items = a.nshots * a.nw;
  if (items <= 0) return hipSuccess;
  SSF_DISPATCH(a.log2n,
               hipLaunchKernelGGL(k_ssf_adjoint<L>, dim3(items),
                                  dim3(Geo<L>::kBlock), 0, st, a, d, part));
  return hipGetLastError();
}

hipError_t launch_ssf_image_sum(const float* part, int items, int64_t npts,
                                float* img, hipStream_t st) {
  if (npts <= 0) return hipSuccess;
  const int blk = 256;
  hipLaunchKernelGGL(k_ssf_image_sum, dim3((npts + blk - 1) / blk), dim3(blk),
                     0, st, part, items, npts, img);
  return hipGetLastError();
}

hipError_t launch_ssf_data_dft(const float* x, int nt, int nrec, double dt,
                               int nw, int k0, double dw, float* X,
                               hipStream_t st) {
  if (nw <= 0 || nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ssf_data_dft, dim3((nrec + 63) / 64, nw), dim3(64), 0,
                     st, x, nt, nrec, dt, k0, dw, X);
  return hipGetLastError();
}

}  // namespace brls
