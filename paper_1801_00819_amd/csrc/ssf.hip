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
// buffers used alternately, addresses swizzled against bank conflicts).
// Twiddles depend only on the thread and the pass, so they sit in
// registers for the whole march.
//
// The phase factors depend on the frequency, the level and the column but
// not on the shot: they are tabulated once per context (k_ssf_tables) and
// the operator marches read them, with the Born weights, one level ahead
// of their use. Their angles (kz dz and w theta) are formed and reduced in
// double and only then rounded to float: the same rounded factor is
// applied at every level, so a float error in the angle would grow
// linearly with depth. The source march, which runs once per shot and
// whose Born weights every later application reuses, runs in double.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b mod 8),
// and each XCD has its own L2. Block b serves frequency
// k = (b mod 8) + 8 ((b / 8) / nshots) and shot (b / 8) mod nshots, so the
// shots of one frequency run back to back on one XCD and share that
// frequency's phase-table rows in its L2. Blocks past the last frequency
// exit at once. Returns false for those.
__device__ inline bool item_of(int b, int nshots, int nw, int* i, int* k) {
  const int idx = b >> 3;
  const int kk = idx / nshots;
  *i = idx - kk * nshots;
  *k = (b & 7) + 8 * kk;
  return *k < nw;
}
__host__ inline int item_blocks(int nshots, int nw) {
  return 8 * ((nw + 7) / 8) * nshots;
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

// LDS slot of FFT element p: the low four bits (sixteen complex numbers,
// 128 bytes) XORed with 5 * ((p >> 4) & 3). The Stockham passes write
// elements 4 apart (first pass) and groups of 4 elements 16 apart (second
// pass); with the swizzle every 16 consecutive lanes of those writes, and
// of the contiguous reads, touch 16 different 8-byte bank pairs.
__device__ inline int sw(int p) { return p ^ (((p >> 4) & 3) * 5); }

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
      y[sw(2 * t)] = cadd(v[0], v[2]);
      y[sw(2 * t + 1)] = csub(v[0], v[2]);
      y[sw(2 * t + 2 * Q)] = cadd(v[1], v[3]);
      y[sw(2 * t + 2 * Q + 1)] = csub(v[1], v[3]);
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = y[sw(t + r * Q)];
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
      for (int r = 0; r < 4; ++r) y[sw(base + r * Ns)] = v[r];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = y[sw(t + r * Q)];
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
// Threads beyond N/4 (only when N < 256) shadow column tx = t mod N/4 for
// their loads, so every load is in bounds without a branch; they store
// nothing.
template <int L, typename T>
struct March {
  using V = typename Cplx<T>::V;
  int t, tx;
  bool on;
  double w;        // angular frequency
  double kx2[4];   // squared wavenumbers of the thread's four q
  T tau[4];        // taper at the thread's four columns
  Twiddles<L, V> tw;
  int pb = 0;
};

template <int L, typename T>
__device__ void march_init(March<L, T>& s, const SsfArgs& a, int k,
                           const typename Cplx<T>::V* tw) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  s.t = threadIdx.x;
  s.tx = s.t & (Q - 1);
  s.on = s.t < Q;
  s.w = (double)(a.k0 + k) * a.dw;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = s.t + r * Q;
    const int qs = r < 2 ? q : q - N;
    const double kx = qs * a.kx_unit;
    s.kx2[r] = kx * kx;
    s.tau[r] = (T)a.tau[s.tx + r * Q];
  }
  load_twiddles<L>(s.tw, tw, s.t);
}

// The medium at one level, loaded ahead of the FFTs that precede its use.
struct Level {
  double s0;     // reference slowness
  double th[4];  // split-step times at the thread's columns
};

template <int L>
__device__ inline void load_level(Level& lv, const SsfArgs& a, int j,
                                  int tx) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  lv.s0 = a.s0[j];
  const double* th = a.theta + (int64_t)j * N;
#pragma unroll
  for (int r = 0; r < 4; ++r) lv.th[r] = th[tx + r * Q];
}

// One level's precomputed phase factors at the thread's four q and x.
struct Phases {
  float2 p[4];   // wavenumber-domain factor / N
  float2 ss[4];  // split-step factor times the taper
};

template <int L>
__device__ inline void load_phases(Phases& ph, const SsfArgs& a, int k,
                                   int j, int tx) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  const int64_t row = ((int64_t)k * a.nz + j) * N;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    ph.p[r] = a.ptab[row + tx + r * Q];
    ph.ss[r] = a.sstab[row + tx + r * Q];
  }
}

// v <- E_j v from the level's phase factors (float marches)
template <int L>
__device__ void step_down_tab(March<L, float>& s, const Phases& ph,
                              float2 v[4], float2* b0, float2* b1) {
  fft<L, float2>(v, b0, b1, s.tw, s.t, s.pb);
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = cmul(v[r], ph.p[r]);
  ifft<L, float2>(v, b0, b1, s.tw, s.t, s.pb);
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = cmul(v[r], ph.ss[r]);
}

// v <- E_j^H v from the level's phase factors
template <int L>
__device__ void step_up_adj_tab(March<L, float>& s, const Phases& ph,
                                float2 v[4], float2* b0, float2* b1) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float2 c = ph.ss[r];
    c.y = -c.y;
    v[r] = cmul(v[r], c);
  }
  fft<L, float2>(v, b0, b1, s.tw, s.t, s.pb);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float2 c = ph.p[r];
    c.y = -c.y;
    v[r] = cmul(v[r], c);
  }
  ifft<L, float2>(v, b0, b1, s.tw, s.t, s.pb);
}

// v <- E_j v, with lv the medium of level j
template <int L, typename T, typename V>
__device__ void step_down(March<L, T>& s, const SsfArgs& a, const Level& lv,
                          V v[4], V* b0, V* b1) {
  constexpr int N = Geo<L>::N;
  constexpr T kInvN = T(1) / N;
  fft<L, V>(v, b0, b1, s.tw, s.t, s.pb);
  const double ws0 = s.w * lv.s0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    v[r] = cscale(cmul(v[r], kz_phase<T>(ws0, s.kx2[r], a.dz)), kInvN);
  ifft<L, V>(v, b0, b1, s.tw, s.t, s.pb);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    v[r] = cscale(cmul(v[r], cis<T>(-s.w * lv.th[r])), s.tau[r]);
}

// --- source: Born weights W_j = -i (w dz/2) s_j S_j for one slot ---------
// The source field is marched in double (it runs once per shot and every
// later application of A and A^T reads its result); W is stored in float.
// One block per (pending shot, frequency).
template <int L>
__global__ __launch_bounds__(Geo<L>::kBlock) void k_ssf_source(
    SsfArgs a, const SsfShotDev* __restrict__ pend, int npend) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  __shared__ double2 b0[N], b1[N];
  int pi, k;
  if (!item_of(blockIdx.x, npend, a.nw, &pi, &k)) return;
  const int slot = pend[pi].slot, xs = pend[pi].xs;
  March<L, double> s;
  march_init<L, double>(s, a, k, a.tw64);
  double2 v[4];
  const double2 f = a.wav[(int64_t)slot * a.nw + k];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    v[r] = (s.on && s.t + r * Q == xs) ? f : czero<double2>();
  float2* Wb = a.W + ((int64_t)slot * a.nw + k) * a.nz * N;
  const double c = 0.5 * s.w * a.dz;
  Level cur;
  load_level<L>(cur, a, 0, s.tx);
  for (int j = 0; j < a.nz; ++j) {
    if (s.on) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = s.t + r * Q;
        const double cs = c * (cur.s0 + cur.th[r] / a.dz);  // (w dz/2) s_j
        Wb[(int64_t)j * N + x] =
            make_float2((float)(cs * v[r].y), (float)(-cs * v[r].x));
      }
    }
    if (j + 1 < a.nz) {
      Level nxt;
      load_level<L>(nxt, a, j + 1, s.tx);
      // level j's factors from the double tables (the values step_down
      // would evaluate), loaded before the forward FFT
      const int64_t row = ((int64_t)k * a.nz + j) * N;
      double2 pk[4], sx[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pk[r] = a.ptab64[row + s.tx + r * Q];
        sx[r] = a.sstab64[row + s.tx + r * Q];
      }
      fft<L, double2>(v, b0, b1, s.tw, s.t, s.pb);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        v[r] = cscale(cmul(v[r], pk[r]), 1.0 / N);
      ifft<L, double2>(v, b0, b1, s.tw, s.t, s.pb);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        v[r] = cscale(cmul(v[r], sx[r]), s.tau[r]);
      cur = nxt;
    }
  }
}

// --- A: upward recursion R_j = W_j m_j + E_j R_{j+1}, receivers of R_0 ---
template <int L>
__global__ __launch_bounds__(Geo<L>::kBlock) void k_ssf_born(
    SsfArgs a, const float* __restrict__ m, float* __restrict__ d) {
  constexpr int N = Geo<L>::N, Q = Geo<L>::Q;
  __shared__ float2 b0[N], b1[N];
  int i, k;
  if (!item_of(blockIdx.x, a.nshots, a.nw, &i, &k)) return;
  const SsfShotDev sh = a.tab[i];
  March<L, float> s;
  march_init<L, float>(s, a, k, a.tw);
  const float2* Wb = a.W + ((int64_t)sh.slot * a.nw + k) * a.nz * N;
  float2 v[4];
  {
    const int j = a.nz - 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = s.tx + r * Q;
      v[r] = cscale(Wb[(int64_t)j * N + x], m[(int64_t)j * N + x]);
    }
  }
  for (int j = a.nz - 2; j >= 0; --j) {
    // this level's operands, in flight while the FFTs run
    Phases ph;
    load_phases<L>(ph, a, k, j, s.tx);
    float2 wv[4];
    float mv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = s.tx + r * Q;
      wv[r] = Wb[(int64_t)j * N + x];
      mv[r] = m[(int64_t)j * N + x];
    }
    step_down_tab<L>(s, ph, v, b0, b1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[r].x = fmaf(wv[r].x, mv[r], v[r].x);
      v[r].y = fmaf(wv[r].y, mv[r], v[r].y);
    }
  }
  // gather the receivers' columns of R_0
  __syncthreads();
  if (s.on) {
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
  int i, k;
  if (!item_of(blockIdx.x, a.nshots, a.nw, &i, &k)) return;
  const int item = i * a.nw + k;  // this pair's image slice (adjoint)
  const SsfShotDev sh = a.tab[i];
  March<L, float> s;
  march_init<L, float>(s, a, k, a.tw);
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
      if (s.on) {
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
  // level j's phases and weights are loaded one level ahead
  Phases cur;
  load_phases<L>(cur, a, k, 0, s.tx);
  float2 wcur[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) wcur[r] = Wb[s.tx + r * Q];
  for (int j = 0; j < a.nz; ++j) {
    if (s.on) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        pb[(int64_t)j * N + s.t + r * Q] =
            fmaf(wcur[r].x, v[r].x, wcur[r].y * v[r].y);
    }
    if (j + 1 < a.nz) {
      Phases nxt;
      load_phases<L>(nxt, a, k, j + 1, s.tx);
      float2 wnxt[4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        wnxt[r] = Wb[(int64_t)(j + 1) * N + s.tx + r * Q];
      step_up_adj_tab<L>(s, cur, v, b0, b1);
      cur = nxt;
#pragma unroll
      for (int r = 0; r < 4; ++r) wcur[r] = wnxt[r];
    }
  }
}

// out[p] = sum over the window's shots and frequencies of |W(p)|^2, in
// double and in a fixed order (one thread per point).
__global__ __launch_bounds__(256) void k_ssf_illumination(SsfArgs a,
                                                          int64_t npts,
                                                          float* out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  double acc = 0.0;
  for (int i = 0; i < a.nshots; ++i) {
    const float2* Wb = a.W + (int64_t)a.tab[i].slot * a.nw * npts + p;
    for (int k = 0; k < a.nw; ++k) {
      const float2 v = Wb[(int64_t)k * npts];
      acc += (double)v.x * v.x + (double)v.y * v.y;
    }
  }
  out[p] = (float)acc;
}

// Phase tables of every (frequency, level, column): the wavenumber-domain
// factor divided by N, and the split-step factor times the taper, each
// formed from its angle in double and rounded once to float.
__global__ __launch_bounds__(256) void k_ssf_tables(SsfArgs a, int n,
                                                    float2* ptab,
                                                    float2* sstab,
                                                    double2* ptab64,
                                                    double2* sstab64) {
  const int64_t total = (int64_t)a.nw * a.nz * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(e % n);
    const int64_t kj = e / n;
    const int j = (int)(kj % a.nz);
    const int k = (int)(kj / a.nz);
    const double w = (double)(a.k0 + k) * a.dw;
    const int qs = q < n / 2 ? q : q - n;
    const double kx = qs * a.kx_unit;
    ptab[e] = cscale(kz_phase<float>(w * a.s0[j], kx * kx, a.dz),
                     1.0f / n);
    sstab[e] = cscale(cis<float>(-w * a.theta[(int64_t)j * n + q]),
                      a.tau[q]);
    ptab64[e] = kz_phase<double>(w * a.s0[j], kx * kx, a.dz);
    sstab64[e] = cis<double>(-w * a.theta[(int64_t)j * n + q]);
  }
}

// img = sum over items of part, in a fixed order: item groups of
// consecutive items summed into double partials (each thread four
// consecutive points), then the groups in order.
constexpr int kSumGroups = kSsfSumGroups;

__global__ __launch_bounds__(256) void k_ssf_sum_groups(
    const float* __restrict__ part, int items, int64_t npts,
    double* __restrict__ psum) {
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const int g = blockIdx.y;
  if (p >= npts) return;
  const int i0 = (int)((int64_t)items * g / kSumGroups);
  const int i1 = (int)((int64_t)items * (g + 1) / kSumGroups);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int i = i0; i < i1; ++i) {
    const float4 v = *reinterpret_cast<const float4*>(part + (int64_t)i * npts
                                                      + p);
    a0 += v.x;
    a1 += v.y;
    a2 += v.z;
    a3 += v.w;
  }
  double* o = psum + (int64_t)g * npts + p;
  o[0] = a0;
  o[1] = a1;
  o[2] = a2;
  o[3] = a3;
}

__global__ __launch_bounds__(256) void k_ssf_sum_final(
    const double* __restrict__ psum, int64_t npts, float* __restrict__ img) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  double acc = 0.0;
#pragma unroll
  for (int g = 0; g < kSumGroups; ++g) acc += psum[(int64_t)g * npts + p];
  img[p] = (float)acc;
}

// X[k][r] = sum_n x[n][r] e^{-i w_k n dt} dt for one shot. A block serves
// one frequency and 16 receivers; its 16 thread rows take 16 consecutive
// chunks of the time axis. Each thread sums its chunk in double, the kernel
// e^{-i w n dt} advanced by rotation from an exact start and reset exactly
// every 64 samples; the chunks are then added in order.
constexpr int kDftRecs = 16, kDftChunks = 16;

__global__ __launch_bounds__(kDftRecs * kDftChunks) void k_ssf_data_dft(
    const float* __restrict__ x, int nt, int nrec, double dt, int k0,
    double dw, float* __restrict__ X) {
  __shared__ double pre[kDftChunks][kDftRecs], pim[kDftChunks][kDftRecs];
  const int rr = threadIdx.x % kDftRecs, c = threadIdx.x / kDftRecs;
  const int r = blockIdx.x * kDftRecs + rr;
  const int k = blockIdx.y;
  const double w = (double)(k0 + k) * dw;
  const int len = (nt + kDftChunks - 1) / kDftChunks;
  const int na = c * len, nb = min(nt, na + len);
  double re = 0.0, im = 0.0;
  if (r < nrec) {
    double rs, rc;
    sincos(-w * dt, &rs, &rc);
    for (int n0 = na; n0 < nb; n0 += 64) {
      double es, ec;
      sincos(-w * dt * n0, &es, &ec);
      const int n1 = min(nb, n0 + 64);
      for (int n = n0; n < n1; ++n) {
        const double xv = x[(int64_t)n * nrec + r];
        re = fma(xv, ec, re);
        im = fma(xv, es, im);
        const double c2 = ec * rc - es * rs;
        es = ec * rs + es * rc;
        ec = c2;
      }
    }
  }
  pre[c][rr] = re;
  pim[c][rr] = im;
  __syncthreads();
  if (c == 0 && r < nrec) {
    double sre = 0.0, sim = 0.0;
    for (int q = 0; q < kDftChunks; ++q) {
      sre += pre[q][rr];
      sim += pim[q][rr];
    }
    X[((int64_t)k * nrec + r) * 2] = (float)(sre * dt);
    X[((int64_t)k * nrec + r) * 2 + 1] = (float)(sim * dt);
  }
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

hipError_t launch_ssf_source(const SsfArgs& a, const SsfShotDev* pend,
                             int npend, hipStream_t st) {
  if (a.nw <= 0 || npend <= 0) return hipSuccess;
  SSF_DISPATCH(a.log2n,
               hipLaunchKernelGGL(k_ssf_source<L>,
                                  dim3(item_blocks(npend, a.nw)),
                                  dim3(Geo<L>::kBlock), 0, st, a, pend,
                                  npend));
  return hipGetLastError();
}

hipError_t launch_ssf_born(const SsfArgs& a, const float* m, float* d,
                           hipStream_t st) {
  const int items = a.nshots * a.nw;
  if (items <= 0) return hipSuccess;
  SSF_DISPATCH(a.log2n,
               hipLaunchKernelGGL(k_ssf_born<L>,
                                  dim3(item_blocks(a.nshots, a.nw)),
                                  dim3(Geo<L>::kBlock), 0, st, a, m, d));
  return hipGetLastError();
}

hipError_t launch_ssf_adjoint(const SsfArgs& a, const float* d, float* part,
                              hipStream_t st) {
  const int items = a.nshots * a.nw;
  if (items <= 0) return hipSuccess;
  SSF_DISPATCH(a.log2n,
               hipLaunchKernelGGL(k_ssf_adjoint<L>,
                                  dim3(item_blocks(a.nshots, a.nw)),
                                  dim3(Geo<L>::kBlock), 0, st, a, d, part));
  return hipGetLastError();
}

hipError_t launch_ssf_tables(const SsfArgs& a, float2* ptab, float2* sstab,
                             double2* ptab64, double2* sstab64,
                             hipStream_t st) {
  const int n = 1 << a.log2n;
  const int64_t total = (int64_t)a.nw * a.nz * n;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(k_ssf_tables, dim3((unsigned)blocks), dim3(256), 0, st,
                     a, n, ptab, sstab, ptab64, sstab64);
  return hipGetLastError();
}

hipError_t launch_ssf_illumination(const SsfArgs& a, float* out,
                                   hipStream_t st) {
  const int64_t npts = (int64_t)a.nz << a.log2n;
  if (npts <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ssf_illumination, dim3((npts + 255) / 256), dim3(256),
                     0, st, a, npts, out);
  return hipGetLastError();
}

hipError_t launch_ssf_image_sum(const float* part, int items, int64_t npts,
                                float* img, double* psum, hipStream_t st) {
  if (npts <= 0) return hipSuccess;
  if (npts % 4) return hipErrorInvalidValue;
  const int blk = 256;
  hipLaunchKernelGGL(k_ssf_sum_groups,
                     dim3((npts / 4 + blk - 1) / blk, kSumGroups), dim3(blk),
                     0, st, part, items, npts, psum);
  hipLaunchKernelGGL(k_ssf_sum_final, dim3((npts + blk - 1) / blk), dim3(blk),
                     0, st, psum, npts, img);
  return hipGetLastError();
}

hipError_t launch_ssf_data_dft(const float* x, int nt, int nrec, double dt,
                               int nw, int k0, double dw, float* X,
                               hipStream_t st) {
  if (nw <= 0 || nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ssf_data_dft, dim3((nrec + kDftRecs - 1) / kDftRecs, nw),
                     dim3(kDftRecs * kDftChunks), 0, st, x, nt, nrec, dt, k0,
                     dw, X);
  return hipGetLastError();
}

}  // namespace brls
