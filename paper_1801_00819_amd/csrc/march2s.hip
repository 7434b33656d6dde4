// Two time steps per launch over tall segments of a strip (gfx950).
//
// The step of march2t.hip (a wavefront holds columns x0 - 4 .. x0 + 59 of
// a strip, computes the first step A on all 64 lanes and on rows widened
// by 4, and the second step B on the 56 inner columns, trailing A by four
// rows) with the wavefront marching a whole segment of SEG output rows
// instead of one 16-row chunk: the rows a chunk shares with the next one
// (8 rows of u for step A's stencil, 4 rows of step-A results for step
// B's) stay in registers instead of being loaded again by the wavefront
// that owns the next chunk. Per SEG output rows a wavefront loads SEG + 16
// rows of u and SEG + 8 rows of v and W, and computes step A on SEG + 8
// rows.
//
// The row loop runs 16 rows per trip with every per-row array a ring of 16
// registers indexed by the row modulo 16 (compile-time inside the unrolled
// trip), so the carried rows need no copies; the last trip stops at the
// segment's end.
//
// The segment height sets how many wavefronts a launch runs: the heights
// that give about one wavefront per resident slot (20 rows for Born and 24
// for the adjoint on the 592 x 1104 grid with 8 shots) keep every SIMD
// busy to the end of the launch instead of leaving a short second round.
//
// A block is P wavefronts marching the same segment for the P shots of one
// group (P = shots per work item). The adjoint's wavefronts write their
// shot's image contributions to their own LDS slice, one row when both
// steps have added to it; at the end of the segment the block adds the
// slices in shot order (float64) to the group's accumulator. Born's
// wavefronts share the medium and model rows through the caches.
//
// Modes: kBorn and kAdjoint take two steps (one where a shot has one left),
// kBackground one step (its Born-source frames written). Floating-point
// operations are those of march2t.hip, in the same order.
#include <hip/hip_runtime.h>

#include "devutil.h"
#include "kernels.h"
#include "layout.h"
#include "march_common.h"

namespace brls {

namespace {

using namespace dev;
using namespace march;

constexpr int kCore = kLanes - 2 * kRadius;  // output columns per strip
constexpr int kRing = 16;                    // rows per trip, ring size

// Local index r * 64 + lane of a receiver entry (r = padded row - (z0 - 4)
// in [0, seg + 8), lane = column - (x0 - 4)) on the segment's outputs.
__device__ __forceinline__ bool core_entry_s(int le, int seg) {
  const int r = le >> 6, l = le & (kLanes - 1);
  return r >= kRadius && r < seg + kRadius && l >= kRadius &&
         l < kLanes - kRadius;
}

// One shot over the segment of output rows z0 .. z0 + SEG - 1 of the strip
// whose lanes hold columns x0 - 4 .. x0 + 59. Adjoint: the shot's image
// contributions land in accl[SEG][64] (this wavefront's slice).
template <int SEG, int D, int MODE, bool INT>
__device__ __forceinline__ void march_segment(const StepArgs& a, int t,
                                              int s, int z0, int x0,
                                              float* inj, float* accl) {
  static_assert(SEG >= 8, "segment height");
  static_assert(D >= 1 && D + 9 <= kRing, "prefetch depth");
  constexpr bool BG = MODE == kBackground;
  constexpr bool BORN = MODE == kBorn;
  constexpr bool ADJ = MODE == kAdjoint;
  constexpr int NI = SEG + 8;  // step-A rows: padded z0 - 4 .. z0 + SEG + 3
  const Geo2D& g = a.g;
  const int lane = threadIdx.x & (kLanes - 1);
  const int xl = x0 - kRadius + lane;  // this lane's column
  const bool core_lane = lane >= kRadius && lane < kLanes - kRadius;
  const int pitch4 = g.pitch * 4;
  const int nx4 = g.nx * 4;
  const int mplane = g.nz * g.nx;
  const int s_top = ((z0 - 4) * g.pitch + x0 - kRadius + g.xoff) * 4;
  const int v_lane = lane * 4;
  const int v_fill =
      (lane < 4 ? lane : (lane >= 60 ? lane + 8 : lane + 4)) * 4;
  const int v_mod = max(xl - g.nb, 0) * 4;
  const bool okx = INT || (xl >= 0 && xl < g.px);
  const bool inx = INT || (xl >= g.nb && xl < g.nb + g.nx);
  const int dx = INT ? 0 : (okx ? sponge_depth(xl, g.nb, g.nx) : 0);
  const Rsrc Rw = rsrc(a.wp);
  const Rsrc Rp = rsrc(a.pm);

  // levels of this launch (see march2t.hip)
  const int nt = uni(a.tab[s].nt);
  int levA;
  bool two;
  if (ADJ) {
    const bool actA = a.n <= nt - 1;
    const bool actB = a.nsub == 2 && a.n - 1 <= nt - 1;
    if (!actA && !actB) {
      for (int o = 0; o < SEG; ++o) accl[o * kLanes + lane] = 0.f;
      return;
    }
    levA = actA ? a.n : a.n - 1;
    two = actA && actB;
  } else {
    if (!(a.n < nt - 1)) return;
    levA = a.n;
    two = !BG && a.nsub == 2 && a.n + 1 < nt - 1;
  }
  const int levB = ADJ ? levA - 1 : levA + 1;
  const ShotDev sd = shot(a.tab, s);
  const Rsrc Rui = rsrc(a.par ? sd.f[1] : sd.f[0]);
  const Rsrc Rvi = rsrc(a.par ? sd.f[3] : sd.f[2]);
  const Rsrc Ruo = rsrc(a.par ? sd.f[0] : sd.f[1]);
  const Rsrc Rvo = rsrc(a.par ? sd.f[2] : sd.f[3]);
  const int frA = (ADJ ? levA - 1 : levA) - a.d2_n0;
  const int frB = (ADJ ? levB - 1 : levB) - a.d2_n0;
  const Rsrc RdA = rsrc(sd.d2 + (int64_t)frA * mplane);
  const Rsrc RdB = rsrc(sd.d2 + (int64_t)max(frB, 0) * mplane);
  const float wav_n = BG ? sd.wav[levA] : 0.f;
  // receivers: eA walks every entry (step-A rows), eB the core entries
  // (step-B rows); erow* = local row of the next entry
  int eA = 0, eB = 0, e1 = 0, erowA = NI, erowB = NI;
  if (!BG) {
    eA = eB = uni(sd.rptr[t]);
    e1 = uni(sd.rptr[t + 1]);
    if (eA < e1) erowA = erowB = uni(sd.rent[eA].x) >> 6;
  }

  // rings, slot = row index mod 16: q by input row r (padded z0 - 8 + r);
  // the others by step-A row i (padded z0 - 4 + i); dB by trip row i (its
  // step-B row is padded z0 - 8 + i); acc by output row o = i - 4
  float q[kRing], hf[kRing], vi[kRing], Wr[kRing], Pr[kRing], dA[kRing],
      dB[kRing], uA[kRing], vA[kRing], acc[kRing];
  int s_q = s_top;
  int p_q = z0 - 8;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const bool there = INT || (p_q >= -kGhost && p_q < g.pz + kGhost);
    q[r] = there ? bload(Rui, v_lane, s_q) : 0.f;
    s_q = opaque(s_q + pitch4);
    p_q = opaque(p_q + 1);
  }
  int s_c = opaque(s_top + 4 * pitch4);  // storage of step-A row loaded next
  int m_c = opaque((z0 - 4 - g.nb) * nx4);
  int z_c = z0 - 4;
  int m_b = opaque((z0 - 8 - g.nb) * nx4);
  // loads of step-A row i (slot k = i mod 16) and of trip row i's step-B
  // Born-source frame
  auto load_row = [&](int i, const int k) {
    {
      const bool there = INT || (p_q >= -kGhost && p_q < g.pz + kGhost);
      q[(k + 8) & (kRing - 1)] = there ? bload(Rui, v_lane, s_q) : 0.f;
      s_q = opaque(s_q + pitch4);
      p_q = opaque(p_q + 1);
    }
    const int z = z_c;
    const bool okz = INT || (z >= 0 && z < g.pz);
    const bool inz = INT || (z >= g.nb && z < g.nb + g.nz);
    const bool coreA = i >= kRadius && i < SEG + kRadius;
    hf[k] = okz ? bload(Rui, v_fill, s_c - 16) : 0.f;
    vi[k] = okz ? bload(Rvi, v_lane, s_c) : 0.f;
    Wr[k] = (okx && okz) ? bload(Rw, v_lane, s_c) : 0.f;
    Pr[k] = (BORN && inx && inz) ? bload(Rp, v_mod, m_c) : 0.f;
    dA[k] = ((BORN || (ADJ && coreA)) && inx && inz)
                ? bload<kNT>(RdA, v_mod, m_c)
                : 0.f;
    const bool coreB = i >= 8;
    const bool inzB = INT || (z - 4 >= g.nb && z - 4 < g.nb + g.nz);
    dB[k] = (!BG && coreB && two && inx && inzB)
                ? bload<kNT>(RdB, v_mod, m_b)
                : 0.f;
    s_c = opaque(s_c + pitch4);
    m_c = opaque(m_c + nx4);
    m_b = opaque(m_b + nx4);
    z_c = opaque(z_c + 1);
  };
#pragma unroll
  for (int i = 0; i < D; ++i) load_row(i, i);

  int s_w = opaque(s_top + 4 * pitch4);  // storage of step-A row i
  int m_w = opaque((z0 - 4 - g.nb) * nx4);
  int z_w = z0 - 4;
  // iteration i: step A on padded row z0 - 4 + i, step B on z0 - 8 + i
  auto row = [&](int i, const int k) {
    __builtin_amdgcn_sched_barrier(0);
    if (i + D < NI) load_row(i + D, (k + D) & (kRing - 1));
    const int z = z_w;
    const int so = s_w, mo = m_w;
    s_w = opaque(s_w + pitch4);
    m_w = opaque(m_w + nx4);
    z_w = opaque(z_w + 1);
    const bool coreA = i >= kRadius && i < SEG + kRadius;
    const int ka = (k - 4) & (kRing - 1);  // output row i - 4
    // ---- step A on padded row z (all lanes) ----
    const bool okz = INT || (z >= 0 && z < g.pz);
    if (!okz) {
      uA[k] = 0.f;
      vA[k] = 0.f;
      if (ADJ) acc[ka] = 0.f;
    } else {
      const bool inz = INT || (z >= g.nb && z < g.nb + g.nz);
      const bool in = inx && inz;
      float C1 = 1.f, C2 = 1.f;
      if (!INT) {
        const int dz = sponge_depth(z, g.nb, g.nz);
        const float damp =
            okx ? g.eta_scale * (float)(dz * dz + dx * dx) : 0.f;
        C1 = __builtin_amdgcn_rcpf(1.f + damp);
        C2 = (1.f - damp) * C1;
      }
      const float c = q[(k + 4) & (kRing - 1)];
      float inj_v = 0.f;
      if (ADJ && erowA == i) {  // residual r^levA at this row's receivers
        for (;;) {
          const int e = eA + lane;
          int2 re = make_int2(0, 0);
          if (e < e1) re = sd.rent[e];
          const bool m = e < e1 && (re.x >> 6) == i;
          const int cnt = __popcll(__ballot(m));
          const float* res = a.dat + sd.dat_off + (int64_t)levA * sd.nrec;
          if (m) atomicAdd(&inj[re.x & (kLanes - 1)], res[re.y]);
          eA += cnt;
          if (cnt < kLanes || eA >= e1) break;
        }
        erowA = eA < e1 ? (uni(sd.rent[eA].x) >> 6) : NI;
        inj_v = inj[lane];
        inj[lane] = 0.f;
      }
      float src = 0.f;
      if (BG) src = (z == sd.src_z && xl == sd.src_x) ? wav_n : 0.f;
      Nb zn;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        zn.m[r] = q[(k + 3 - r) & (kRing - 1)];
        zn.p[r] = q[(k + 5 + r) & (kRing - 1)];
      }
      const float lap = lap8(g.w, c, zn, xnb(c, hf[k]));
      float inc;
      if (BORN) {
        inc = Wr[k] * lap;
        if (in) inc = fmaf(-Pr[k], dA[k], inc);
      } else if (ADJ) {
        inc = Wr[k] * (lap + inj_v);
      } else {
        inc = Wr[k] * (lap + src);
      }
      const float vn = INT ? vi[k] + inc : fmaf(C2, vi[k], C1 * inc);
      const float un = c + vn;
      uA[k] = okx ? un : 0.f;
      vA[k] = vn;
      if (BORN && erowA == i) {  // d^levA, d^(levA+1) at core receivers
        for (;;) {
          const int e = eA + lane;
          int2 re = make_int2(0, 0);
          if (e < e1) re = sd.rent[e];
          const bool m = e < e1 && (re.x >> 6) == i;
          const int cnt = __popcll(__ballot(m));
          const int src_lane = (re.x & (kLanes - 1)) << 2;
          const float d0 = __int_as_float(
              __builtin_amdgcn_ds_bpermute(src_lane, __float_as_int(c)));
          const float d1 = __int_as_float(
              __builtin_amdgcn_ds_bpermute(src_lane, __float_as_int(un)));
          if (m && core_entry_s(re.x, SEG)) {
            float* dat = a.dat + sd.dat_off + (int64_t)levA * sd.nrec;
            dat[re.y] = d0;
            dat[sd.nrec + re.y] = d1;
          }
          eA += cnt;
          if (cnt < kLanes || eA >= e1) break;
        }
        erowA = eA < e1 ? (uni(sd.rent[eA].x) >> 6) : NI;
      }
      if (ADJ) acc[ka] = (coreA && in) ? -dA[k] * un : 0.f;
      if (coreA) {
        if (BG && a.write_d2 && in && core_lane)
          bstore<kNT>(RdA, v_mod, mo, inc);
        if (!two && okx && core_lane) {  // one step: A's rows are output
          bstore(Rvo, v_lane, so, vn);
          bstore(Ruo, v_lane, so, un);
        }
      }
    }
    // ---- step B on padded row z - 4 (output lanes) ----
    if (i >= 8) {
      const int ib = (k - 4) & (kRing - 1);  // step-A slot of row z - 4
      const int ko = (k - 8) & (kRing - 1);  // output row i - 8
      if (two && (INT || z - 4 < g.pz)) {
        const int zb = z - 4;
        const bool inzB = INT || (zb >= g.nb && zb < g.nb + g.nz);
        const bool in = inx && inzB;
        float C1 = 1.f, C2 = 1.f;
        if (!INT) {
          const int dz = sponge_depth(zb, g.nb, g.nz);
          const float damp =
              okx ? g.eta_scale * (float)(dz * dz + dx * dx) : 0.f;
          C1 = __builtin_amdgcn_rcpf(1.f + damp);
          C2 = (1.f - damp) * C1;
        }
        const float c = uA[ib];
        float inj_v = 0.f;
        if (ADJ && erowB == i - 4) {  // residual r^levB at core receivers
          for (;;) {
            const int e = eB + lane;
            int2 re = make_int2(0, 0);
            if (e < e1) re = sd.rent[e];
            const bool m = e < e1 && (re.x >> 6) == i - 4;
            const int cnt = __popcll(__ballot(m));
            const float* res = a.dat + sd.dat_off + (int64_t)levB * sd.nrec;
            if (m && core_entry_s(re.x, SEG))
              atomicAdd(&inj[re.x & (kLanes - 1)], res[re.y]);
            eB += cnt;
            if (cnt < kLanes || eB >= e1) break;
          }
          erowB = eB < e1 ? (uni(sd.rent[eB].x) >> 6) : NI;
          inj_v = inj[lane];
          inj[lane] = 0.f;
        }
        Nb zn;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          zn.m[r] = uA[(k - 5 - r) & (kRing - 1)];
          zn.p[r] = uA[(k - 3 + r) & (kRing - 1)];
        }
        const float lap = lap8(g.w, c, zn, xnb_inner(c));
        float inc;
        if (BORN) {
          inc = Wr[ib] * lap;
          if (in) inc = fmaf(-Pr[ib], dB[k], inc);
        } else {
          inc = Wr[ib] * (lap + inj_v);
        }
        const float vn = INT ? vA[ib] + inc : fmaf(C2, vA[ib], C1 * inc);
        const float un = c + vn;
        const int sob = so - 4 * pitch4;
        if (okx && core_lane) {
          bstore(Rvo, v_lane, sob, vn);
          bstore(Ruo, v_lane, sob, un);
        }
        if (ADJ && in) acc[ko] = fmaf(-dB[k], un, acc[ko]);
      }
      if (ADJ) accl[(i - 8) * kLanes + lane] = acc[ko];
    }
    (void)mo;
  };

  constexpr int kFull = NI / kRing * kRing;  // rows in whole trips
#pragma unroll 1
  for (int base = 0; base < kFull; base += kRing) {
#pragma unroll
    for (int k = 0; k < kRing; ++k) row(base + k, k);
  }
#pragma unroll
  for (int k = 0; k < NI - kFull; ++k) row(kFull + k, k);
}

}  // namespace

// Block of P wavefronts: work item (segment of a strip, shot group), wave w
// marching shot group * per_block + w (waves past per_block idle).
// Adjoint: the group's image contributions summed over its shots in LDS and
// added to the group's accumulator once.
// The work items of one launch (segment of a strip, shot group) that this
// block owns, wave w marching shot group * per_block + w (waves past
// per_block idle). Adjoint: the group's image contributions summed over its
// shots in LDS and added to the group's accumulator once per item.
template <int SEG, int D, int MODE, int P>
__device__ __forceinline__ void segment_items(const StepArgs& a, float* inj,
                                              float* accs) {
  constexpr bool ADJ = MODE == kAdjoint;
  const int wv = (int)uni((uint32_t)threadIdx.x / kLanes);
  const int lane = threadIdx.x & (kLanes - 1);
  float* accl = accs + (ADJ ? wv * SEG * kLanes : 0);
  const Geo2D& g = a.g;
  const int mplane = g.nz * g.nx;
  const int items = g.ntiles * a.ngroups;
  int first, hi, stride;
  if (a.resident_grid & 2) {
    first = (int)blockIdx.x;
    hi = items;
    stride = (int)gridDim.x;
  } else {
    const int xcd = blockIdx.x & 7;
    const int q = items >> 3, r = items & 7;
    first = xcd * q + min(xcd, r) + (int)(blockIdx.x >> 3);
    hi = xcd * q + min(xcd, r) + q + (xcd < r ? 1 : 0);
    stride = (int)(gridDim.x >> 3);
  }
  // grid shape bit 2: strips vary fastest along the item index, so the
  // wavefronts that run together cover whole rows of the grid (DRAM pages
  // shared) instead of consecutive segments of one strip
  const bool xfast = (a.resident_grid & 4) != 0;
  for (int L = first; L < hi; L += stride) {
    const int grp = L % a.ngroups;
    const int tl = L / a.ngroups;
    const int tzi = xfast ? tl / g.ntx : tl % g.ntz;
    const int txi = xfast ? tl % g.ntx : tl / g.ntz;
    const int z0 = tzi * SEG;
    const int x0 = g.x_org + txi * kCore;
    const int t = tzi * g.ntx + txi;
    const bool interior = x0 - kRadius >= g.nb &&
                          x0 + kCore + kRadius <= g.nb + g.nx &&
                          z0 - kRadius >= g.nb &&
                          z0 + SEG + kRadius <= g.nb + g.nz;
    const int s = grp * a.per_block + wv;
    if (wv < a.per_block && s < a.nshots) {
      if (interior)
        march_segment<SEG, D, MODE, true>(a, t, s, z0, x0, inj, accl);
      else
        march_segment<SEG, D, MODE, false>(a, t, s, z0, x0, inj, accl);
    } else if (ADJ) {
      for (int o = 0; o < SEG; ++o) accl[o * kLanes + lane] = 0.f;
    }
    if (ADJ) {
      __syncthreads();
      for (int e = threadIdx.x; e < SEG * kLanes; e += P * kLanes) {
        const int j = e / kLanes, ln = e % kLanes;
        const int xl = x0 - kRadius + ln, z = z0 + j;
        if (ln >= kRadius && ln < kLanes - kRadius && xl >= g.nb &&
            xl < g.nb + g.nx && z >= g.nb && z < g.nb + g.nz) {
          double sum = 0.0;
#pragma unroll
          for (int w = 0; w < P; ++w)
            sum += (double)accs[w * SEG * kLanes + e];
          a.acc[(int64_t)grp * mplane + (int64_t)(z - g.nb) * g.nx +
                (xl - g.nb)] += sum;
        }
      }
      __syncthreads();
    }
  }
}

// Register budget: 4 wavefronts per SIMD (at most 128 VGPRs).
template <int SEG, int D, int MODE, int P>
__global__ void __launch_bounds__(kLanes* P)
    __attribute__((amdgpu_waves_per_eu(4))) k_march2s(StepArgs a) {
  constexpr bool ADJ = MODE == kAdjoint;
  __shared__ float inj_all[ADJ ? P * kLanes : 1];
  __shared__ float accs[ADJ ? P * SEG * kLanes : 1];
  const int wv = (int)uni((uint32_t)threadIdx.x / kLanes);
  float* inj = inj_all + (ADJ ? wv * kLanes : 0);
  if (ADJ) inj[threadIdx.x & (kLanes - 1)] = 0.f;
  segment_items<SEG, D, MODE, P>(a, inj, accs);
}

// Grid barrier of the persistent kernel: every block adds one arrival to
// the counter and waits for `target` arrivals. The wait is bounded: after
// spin_limit polls the block records a failure in *error and the call
// returns false (the kernel then ends; the blocks still waiting for it
// reach their own limit), so no launch can hang.
__device__ __forceinline__ bool grid_barrier(const PersistArgs& p,
                                             unsigned target) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(p.counter, 1u);
    int good = 1;
    for (int spins = 0;
         __hip_atomic_load(p.counter, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT) < target;
         ++spins) {
      if (spins >= p.spin_limit) {
        atomicOr(p.error, 1);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// One launch for a whole operator application: the grid (no larger than
// what is resident at once) runs the work items of every two-step launch
// in turn, a grid barrier between consecutive ones (a level's neighbouring
// segments must be complete before the next level reads them).
template <int SEG, int D, int MODE, int P>
__global__ void __launch_bounds__(kLanes* P)
    __attribute__((amdgpu_waves_per_eu(4)))
    k_march2s_persist(StepArgs a, PersistArgs p) {
  constexpr bool ADJ = MODE == kAdjoint;
  __shared__ float inj_all[ADJ ? P * kLanes : 1];
  __shared__ float accs[ADJ ? P * SEG * kLanes : 1];
  const int wv = (int)uni((uint32_t)threadIdx.x / kLanes);
  float* inj = inj_all + (ADJ ? wv * kLanes : 0);
  if (ADJ) inj[threadIdx.x & (kLanes - 1)] = 0.f;
  for (int j = 0; j < p.nlaunch; ++j) {
    StepArgs b = a;
    if (ADJ) {
      b.n = p.k_hi - 2 * j;
      b.nsub = min(2, b.n - p.k_lo + 1);
    } else {
      b.n = 2 * j;
      b.nsub = min(2, p.nt_max - 1 - b.n);
    }
    b.par = j & 1;
    segment_items<SEG, D, MODE, P>(b, inj, accs);
    if (j + 1 < p.nlaunch &&
        !grid_barrier(p, (unsigned)(j + 1) * gridDim.x))
      return;
  }
}

namespace {

template <int SEG, int D, int MODE, int P>
hipError_t launch_s(const StepArgs& a, hipStream_t st) {
  static const int cap = resident_blocks(
      reinterpret_cast<const void*>(&k_march2s<SEG, D, MODE, P>), kLanes * P);
  const int need = a.g.ntiles * a.ngroups;
  const int lim = (a.resident_grid & 1) ? cap : need;
  const int nblk = ((need < lim ? need : lim) + 7) / 8 * 8;
  hipLaunchKernelGGL((k_march2s<SEG, D, MODE, P>), dim3(nblk),
                     dim3(kLanes * P), 0, st, a);
  return hipGetLastError();
}

// Blocks of the smallest of 1, 2, 4, 8 wavefronts that holds per_block.
template <int SEG, int D, int MODE>
hipError_t launch_s_mode(const StepArgs& a, hipStream_t st) {
  if (a.per_block <= 1) return launch_s<SEG, D, MODE, 1>(a, st);
  if (a.per_block <= 2) return launch_s<SEG, D, MODE, 2>(a, st);
  if (a.per_block <= 4) return launch_s<SEG, D, MODE, 4>(a, st);
  if (a.per_block <= 8) return launch_s<SEG, D, MODE, 8>(a, st);
  return hipErrorInvalidValue;
}

template <int SEG, int D, int MODE, int P>
hipError_t launch_p(const StepArgs& a, const PersistArgs& p, hipStream_t st) {
  static const int cap = resident_blocks(
      reinterpret_cast<const void*>(&k_march2s_persist<SEG, D, MODE, P>),
      kLanes * P);
  // every block must be resident at once (grid barriers): the grid is the
  // resident capacity, in whole sets of 8 (the per-XCD dealing)
  const int need = a.g.ntiles * a.ngroups;
  int nblk = cap < need ? cap : need;
  nblk = nblk / 8 * 8;
  if (nblk < 8 || nblk > cap) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_march2s_persist<SEG, D, MODE, P>), dim3(nblk),
                     dim3(kLanes * P), 0, st, a, p);
  return hipGetLastError();
}

template <int SEG, int D, int MODE>
hipError_t launch_p_mode(const StepArgs& a, const PersistArgs& p,
                         hipStream_t st) {
  if (a.per_block <= 1) return launch_p<SEG, D, MODE, 1>(a, p, st);
  if (a.per_block <= 2) return launch_p<SEG, D, MODE, 2>(a, p, st);
  if (a.per_block <= 4) return launch_p<SEG, D, MODE, 4>(a, p, st);
  if (a.per_block <= 8) return launch_p<SEG, D, MODE, 8>(a, p, st);
  return hipErrorInvalidValue;
}

template <int SEG, int D>
hipError_t launch_p_shape(int mode, const StepArgs& a, const PersistArgs& p,
                          hipStream_t st) {
  switch (mode) {
    case kBorn: return launch_p_mode<SEG, D, kBorn>(a, p, st);
    case kAdjoint: return launch_p_mode<SEG, D, kAdjoint>(a, p, st);
  }
  return hipErrorInvalidValue;
}

template <int SEG, int D>
hipError_t launch_s_shape(int mode, const StepArgs& a, hipStream_t st) {
  switch (mode) {
    case kBackground: return launch_s_mode<SEG, D, kBackground>(a, st);
    case kBorn: return launch_s_mode<SEG, D, kBorn>(a, st);
    case kAdjoint: return launch_s_mode<SEG, D, kAdjoint>(a, st);
  }
  return hipErrorInvalidValue;  // no fused mode: needs stored sources
}

}  // namespace

hipError_t launch_march2s_persistent(int seg, int ahead, int mode,
                                     const StepArgs& a, const PersistArgs& p,
                                     hipStream_t st) {
  if (seg == 20 && ahead == 4) return launch_p_shape<20, 4>(mode, a, p, st);
  if (seg == 24 && ahead == 4) return launch_p_shape<24, 4>(mode, a, p, st);
  if (seg == 32 && ahead == 4) return launch_p_shape<32, 4>(mode, a, p, st);
  if (seg == 16 && ahead == 4) return launch_p_shape<16, 4>(mode, a, p, st);
  return hipErrorInvalidValue;
}

template <int SEG, int MODE>
static int capacity_of(int P) {
  switch (P) {
    case 1: return resident_blocks(reinterpret_cast<const void*>(
                &k_march2s_persist<SEG, 4, MODE, 1>), kLanes);
    case 2: return resident_blocks(reinterpret_cast<const void*>(
                &k_march2s_persist<SEG, 4, MODE, 2>), 2 * kLanes);
    case 4: return resident_blocks(reinterpret_cast<const void*>(
                &k_march2s_persist<SEG, 4, MODE, 4>), 4 * kLanes);
  }
  return resident_blocks(reinterpret_cast<const void*>(
      &k_march2s_persist<SEG, 4, MODE, 8>), 8 * kLanes);
}

template <int SEG>
static int capacity_seg(int mode, int P) {
  return mode == kBorn ? capacity_of<SEG, kBorn>(P)
                       : capacity_of<SEG, kAdjoint>(P);
}

int march2s_persistent_capacity(int seg, int ahead, int mode, int per_block) {
  (void)ahead;
  const int P = per_block <= 1 ? 1 : per_block <= 2 ? 2
              : per_block <= 4 ? 4 : 8;
  switch (seg) {
    case 20: return capacity_seg<20>(mode, P);
    case 24: return capacity_seg<24>(mode, P);
    case 32: return capacity_seg<32>(mode, P);
  }
  return capacity_seg<16>(mode, P);
}

hipError_t launch_march2s(int seg, int ahead, int mode, const StepArgs& a,
                          hipStream_t st) {
  if (seg == 20 && ahead == 4) return launch_s_shape<20, 4>(mode, a, st);
  if (seg == 24 && ahead == 4) return launch_s_shape<24, 4>(mode, a, st);
  if (seg == 32 && ahead == 4) return launch_s_shape<32, 4>(mode, a, st);
  if (seg == 16 && ahead == 4) return launch_s_shape<16, 4>(mode, a, st);
  return hipErrorInvalidValue;
}

}  // namespace brls
