// Two time steps per launch of the z-marching 2-D kernel (gfx950).
//
// Temporal blocking of the step in march2d.hip: a wavefront advances its
// strip by two time steps, so the wavefields are read and written once per
// two steps instead of once per step. The 64 lanes hold columns
// x0 - 4 .. x0 + 59; the first step (A) is computed on all 64 lanes and on
// the chunk's rows widened by 4 on each side, which is exactly the halo the
// second step (B) needs on its 56 output columns x0 .. x0 + 55 and CZ output
// rows. Step B trails step A by four rows, reading A's results from a
// register queue (z-stencil) and neighbouring lanes (x-stencil); nothing of
// step A goes to memory. Step A's values outside the padded grid are set to
// zero (the Dirichlet ring).
//
// Wavefield sets: a launch reads u, v from set `par` ({f0, f2} or {f1, f3})
// and writes both to the other set, so no wavefront overwrites values a
// neighbour still reads. Level L of a run that started at level 0 (Born,
// background) therefore sits in set ceil(L / 2) mod 2 when launches take two
// steps, set L mod 2 when they take one.
//
// Modes: kBorn and kAdjoint take two steps (or one, where a shot has only
// one left); kBackground takes one step per launch (its Born-source frames
// are written on the output rows). Floating-point operations are those of
// the one-step kernels, in the same order.
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

// Receivers of a tile, sorted by local index r * 64 + lane, r = padded row
// - (z0 - 4) in [0, CZ + 8), lane = column - (x0 - 4). Entries with r in
// [4, CZ + 4) and lane in [4, 60) lie on the tile's outputs ("core").
__device__ __forceinline__ bool core_entry(int le, int cz) {
  const int r = le >> 6, l = le & (kLanes - 1);
  return r >= kRadius && r < cz + kRadius && l >= kRadius &&
         l < kLanes - kRadius;
}

// COOP (adjoint, cooperative blocks): the item is one shot, coop_shot, and
// its image contributions accumulate in this wavefront's LDS slice `accl`
// ([CZ][64], each lane its own column) for the block to sum over its shots,
// instead of in registers flushed to the group's float64 accumulator (the
// CZ registers saved raise the occupancy from 3 to 4 wavefronts per SIMD).
template <int CZ, int AHEAD, int MODE, bool INT, bool COOP = false>
__device__ __forceinline__ void march2_item(const StepArgs& a, int t, int grp,
                                            int z0, int x0, float* inj,
                                            float* accl = nullptr,
                                            int coop_shot = 0) {
  constexpr bool BG = MODE == kBackground;
  constexpr bool BORN = MODE == kBorn;
  constexpr bool ADJ = MODE == kAdjoint;
  constexpr int D = AHEAD;
  constexpr int NI = CZ + 8;   // step-A rows: padded z0 - 4 .. z0 + CZ + 3
  constexpr int NQ = CZ + 16;  // input rows: padded z0 - 8 .. z0 + CZ + 7
  const Geo2D& g = a.g;
  const int lane = threadIdx.x & (kLanes - 1);
  const int xl = x0 - kRadius + lane;  // this lane's column
  const bool core_lane = lane >= kRadius && lane < kLanes - kRadius;
  const int pitch4 = g.pitch * 4;
  const int nx4 = g.nx * 4;
  const int mplane = g.nz * g.nx;
  // byte offset of padded row z0 - 8 (storage row z0 - 4) at column x0 - 4;
  // the fill load starts 4 columns further left (lanes 0..3 -> x0-8..x0-5,
  // lanes 60..63 -> x0+60..x0+63, the rest their own column)
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

  float acc[COOP ? 1 : CZ];
#pragma unroll
  for (int j = 0; j < (COOP ? 1 : CZ); ++j) acc[j] = 0.f;
  if constexpr (COOP) {
#pragma unroll
    for (int j = 0; j < CZ; ++j) accl[j * kLanes + lane] = 0.f;
  }
  bool any = false;

  const int s0 = COOP ? coop_shot : grp * a.per_block;
  const int s1 =
      COOP ? min(coop_shot + 1, a.nshots) : min(s0 + a.per_block, a.nshots);
  for (int s = s0; s < s1; ++s) {
    // the launch covers levels n and n + 1 (Born, background: input
    // levels) or k and k - 1 (adjoint: output levels), a.nsub of them
    const int nt = uni(a.tab[s].nt);
    int levA;
    bool two;
    if (ADJ) {
      const bool actA = a.n <= nt - 1;
      const bool actB = a.nsub == 2 && a.n - 1 <= nt - 1;
      if (!actA && !actB) continue;
      levA = actA ? a.n : a.n - 1;
      two = actA && actB;
    } else {
      if (!(a.n < nt - 1)) continue;
      levA = a.n;
      two = !BG && a.nsub == 2 && a.n + 1 < nt - 1;
    }
    any = true;
    const int levB = ADJ ? levA - 1 : levA + 1;
    const ShotDev sd = shot(a.tab, s);
    const Rsrc Rui = rsrc(a.par ? sd.f[1] : sd.f[0]);
    const Rsrc Rvi = rsrc(a.par ? sd.f[3] : sd.f[2]);
    const Rsrc Ruo = rsrc(a.par ? sd.f[0] : sd.f[1]);
    const Rsrc Rvo = rsrc(a.par ? sd.f[2] : sd.f[3]);
    // Born-source frames (Born: levels A and B; background: level A,
    // written) or image frames (adjoint: levels A - 1 and B - 1)
    const int frA = (ADJ ? levA - 1 : levA) - a.d2_n0;
    const int frB = (ADJ ? levB - 1 : levB) - a.d2_n0;
    const Rsrc RdA = rsrc(sd.d2 + (int64_t)frA * mplane);
    const Rsrc RdB = rsrc(sd.d2 + (int64_t)max(frB, 0) * mplane);
    const float wav_n = BG ? sd.wav[levA] : 0.f;
    // receivers: cursor eA walks every entry (step A rows), eB the core
    // entries (step B rows); erow* = row of the next entry
    int eA = 0, eB = 0, e1 = 0, erowA = NI, erowB = NI;
    if (!BG) {
      eA = eB = uni(sd.rptr[t]);
      e1 = uni(sd.rptr[t + 1]);
      if (eA < e1) erowA = erowB = uni(sd.rent[eA].x) >> 6;
    }

    float q[NQ];                       // u^n, padded rows z0 - 8 + r
    float hf[NI], vi[NI], Wr[NI], Pr[NI], dA[NI], dB[NI];
    float uA[NI], vA[NI];              // step A results
    // rolling offsets of the rows whose loads are issued next
    int s_q = s_top;
    int p_q = z0 - 8;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const bool there = INT || (p_q >= -kGhost && p_q < g.pz + kGhost);
      q[r] = there ? bload(Rui, v_lane, s_q) : 0.f;
      s_q = opaque(s_q + pitch4);
      p_q = opaque(p_q + 1);
    }
    int s_c = opaque(s_top + 4 * pitch4);       // step-A row i + D
    int m_c = opaque((z0 - 4 - g.nb) * nx4);
    int z_c = z0 - 4;
    int m_b = opaque((z0 - 8 - g.nb) * nx4);    // step-B row i + D
    auto load_row = [&](int i) {
      {  // input row for the queue (padded z0 + i)
        const bool there = INT || (p_q >= -kGhost && p_q < g.pz + kGhost);
        q[i + 8] = there ? bload(Rui, v_lane, s_q) : 0.f;
        s_q = opaque(s_q + pitch4);
        p_q = opaque(p_q + 1);
      }
      const int z = z_c;
      const bool okz = INT || (z >= 0 && z < g.pz);
      const bool inz = INT || (z >= g.nb && z < g.nb + g.nz);
      const bool coreA = i >= kRadius && i < CZ + kRadius;
      hf[i] = okz ? bload(Rui, v_fill, s_c - 16) : 0.f;
      vi[i] = okz ? bload(Rvi, v_lane, s_c) : 0.f;
      Wr[i] = (okx && okz) ? bload(Rw, v_lane, s_c) : 0.f;
      Pr[i] = (BORN && inx && inz) ? bload(Rp, v_mod, m_c) : 0.f;
      dA[i] = ((BORN || (ADJ && coreA)) && inx && inz)
                  ? bload<kNT>(RdA, v_mod, m_c)
                  : 0.f;
      // step-B row of iteration i: padded z0 - 8 + i
      const bool coreB = i >= 8;
      const bool inzB = INT || (z - 4 >= g.nb && z - 4 < g.nb + g.nz);
      dB[i] = (!BG && coreB && two && inx && inzB)
                  ? bload<kNT>(RdB, v_mod, m_b)
                  : 0.f;
      s_c = opaque(s_c + pitch4);
      m_c = opaque(m_c + nx4);
      m_b = opaque(m_b + nx4);
      z_c = opaque(z_c + 1);
    };
#pragma unroll
    for (int i = 0; i < D; ++i) load_row(i);

    int s_w = opaque(s_top + 4 * pitch4);  // storage of step-A row i
    int m_w = opaque((z0 - 4 - g.nb) * nx4);
    int z_w = z0 - 4;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      __builtin_amdgcn_sched_barrier(0);
      if (i + D < NI) load_row(i + D);
      const int z = z_w;
      const int so = s_w, mo = m_w;
      s_w = opaque(s_w + pitch4);
      m_w = opaque(m_w + nx4);
      z_w = opaque(z_w + 1);
      const bool coreA = i >= kRadius && i < CZ + kRadius;
      // ---- step A on padded row z (all lanes) ----
      const bool okz = INT || (z >= 0 && z < g.pz);
      if (!okz) {
        uA[i] = 0.f;
        vA[i] = 0.f;
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
        const float c = q[i + 4];
        float inj_v = 0.f;
        if (ADJ && erowA == i) {  // residual r^levA at this row's receivers
          for (;;) {
            const int k = eA + lane;
            int2 re = make_int2(0, 0);
            if (k < e1) re = sd.rent[k];
            const bool m = k < e1 && (re.x >> 6) == i;
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
        const float lap = lap8(g.w, c, znb(q, i + 4), xnb(c, hf[i]));
        float inc;
        if (BORN) {
          inc = Wr[i] * lap;
          if (in) inc = fmaf(-Pr[i], dA[i], inc);
        } else if (ADJ) {
          inc = Wr[i] * (lap + inj_v);
        } else {
          inc = Wr[i] * (lap + src);
        }
        const float vn = INT ? vi[i] + inc : fmaf(C2, vi[i], C1 * inc);
        const float un = c + vn;
        uA[i] = okx ? un : 0.f;
        vA[i] = vn;
        if (BORN && erowA == i) {  // d^levA, d^(levA+1) at core receivers
          for (;;) {
            const int k = eA + lane;
            int2 re = make_int2(0, 0);
            if (k < e1) re = sd.rent[k];
            const bool m = k < e1 && (re.x >> 6) == i;
            const int cnt = __popcll(__ballot(m));
            const int src_lane = (re.x & (kLanes - 1)) << 2;
            const float d0 = __int_as_float(
                __builtin_amdgcn_ds_bpermute(src_lane, __float_as_int(c)));
            const float d1 = __int_as_float(
                __builtin_amdgcn_ds_bpermute(src_lane, __float_as_int(un)));
            if (m && core_entry(re.x, CZ)) {
              float* dat = a.dat + sd.dat_off + (int64_t)levA * sd.nrec;
              dat[re.y] = d0;
              dat[sd.nrec + re.y] = d1;
            }
            eA += cnt;
            if (cnt < kLanes || eA >= e1) break;
          }
          erowA = eA < e1 ? (uni(sd.rent[eA].x) >> 6) : NI;
        }
        if (coreA) {
          if (BG && a.write_d2 && in && core_lane)
            bstore<kNT>(RdA, v_mod, mo, inc);
          if (ADJ && in) {
            if constexpr (COOP)
              accl[(i - kRadius) * kLanes + lane] =
                  fmaf(-dA[i], un, accl[(i - kRadius) * kLanes + lane]);
            else
              acc[i - kRadius] = fmaf(-dA[i], un, acc[i - kRadius]);
          }
          if (!two && okx && core_lane) {  // one step: A's rows are output
            bstore(Rvo, v_lane, so, vn);
            bstore(Ruo, v_lane, so, un);
          }
        }
      }
      // ---- step B on padded row z - 4 (output lanes) ----
      if (i >= 8 && two) {
        const int zb = z - 4;
        const int ib = i - 4;  // step-A index of row zb
        if (INT || zb < g.pz) {
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
          if (ADJ && erowB == ib) {  // residual r^levB at core receivers
            for (;;) {
              const int k = eB + lane;
              int2 re = make_int2(0, 0);
              if (k < e1) re = sd.rent[k];
              const bool m = k < e1 && (re.x >> 6) == ib;
              const int cnt = __popcll(__ballot(m));
              const float* res =
                  a.dat + sd.dat_off + (int64_t)levB * sd.nrec;
              if (m && core_entry(re.x, CZ))
                atomicAdd(&inj[re.x & (kLanes - 1)], res[re.y]);
              eB += cnt;
              if (cnt < kLanes || eB >= e1) break;
            }
            erowB = eB < e1 ? (uni(sd.rent[eB].x) >> 6) : NI;
            inj_v = inj[lane];
            inj[lane] = 0.f;
          }
          const float lap = lap8(g.w, c, znb(uA, ib), xnb_inner(c));
          float inc;
          if (BORN) {
            inc = Wr[ib] * lap;
            if (in) inc = fmaf(-Pr[ib], dB[i], inc);
          } else {
            inc = Wr[ib] * (lap + inj_v);
          }
          const float vn =
              INT ? vA[ib] + inc : fmaf(C2, vA[ib], C1 * inc);
          const float un = c + vn;
          const int sob = so - 4 * pitch4;
          if (okx && core_lane) {
            bstore(Rvo, v_lane, sob, vn);
            bstore(Ruo, v_lane, sob, un);
          }
          if (ADJ && in) {
            if constexpr (COOP)
              accl[(i - 8) * kLanes + lane] =
                  fmaf(-dB[i], un, accl[(i - 8) * kLanes + lane]);
            else
              acc[i - 8] = fmaf(-dB[i], un, acc[i - 8]);
          }
        }
      }
      (void)mo;
    }
  }
  if (!COOP && ADJ && any) {
    double* out = a.acc + (int64_t)grp * mplane +
                  (int64_t)(z0 - g.nb) * g.nx + (xl - g.nb);
    int mo = 0, z = z0;
#pragma unroll
    for (int j = 0; j < CZ; ++j) {
      if (core_lane && inx && (INT || (z >= g.nb && z < g.nb + g.nz)))
        out[mo] += (double)acc[j];
      mo = opaque(mo + g.nx);
      z = opaque(z + 1);
    }
  }
}

}  // namespace

template <int CZ, int AHEAD, int MODE>
__global__ void __launch_bounds__(kLanes* kWaves) k_march2t(StepArgs a) {
  __shared__ float inj_all[MODE == kAdjoint ? kWaves * kLanes : 1];
  const int wv = (int)uni((uint32_t)threadIdx.x / kLanes);
  float* inj = inj_all + (MODE == kAdjoint ? wv * kLanes : 0);
  if (MODE == kAdjoint) inj[threadIdx.x & (kLanes - 1)] = 0.f;
  const Geo2D& g = a.g;
  // work items (strip chunk, shot group) as in k_march2d
  const int items = g.ntiles * a.ngroups;
  int first, hi, stride;
  if (a.resident_grid & 2) {
    first = (int)blockIdx.x * kWaves + wv;
    hi = items;
    stride = (int)gridDim.x * kWaves;
  } else {
    const int xcd = blockIdx.x & 7;
    const int q = items >> 3, r = items & 7;
    first = xcd * q + min(xcd, r) + (int)(blockIdx.x >> 3) * kWaves + wv;
    hi = xcd * q + min(xcd, r) + q + (xcd < r ? 1 : 0);
    stride = (int)(gridDim.x >> 3) * kWaves;
  }
  const bool xfast = (a.resident_grid & 4) != 0;  // see k_march2s
  for (int L = first; L < hi; L += stride) {
    const int grp = L % a.ngroups;
    const int tl = L / a.ngroups;
    const int tzi = xfast ? tl / g.ntx : tl % g.ntz;
    const int txi = xfast ? tl % g.ntx : tl / g.ntz;
    const int z0 = tzi * CZ;
    const int x0 = g.x_org + txi * kCore;
    const int t = tzi * g.ntx + txi;
    const bool interior = x0 - kRadius >= g.nb &&
                          x0 + kCore + kRadius <= g.nb + g.nx &&
                          z0 - kRadius >= g.nb &&
                          z0 + CZ + kRadius <= g.nb + g.nz;
    if (interior)
      march2_item<CZ, AHEAD, MODE, true>(a, t, grp, z0, x0, inj);
    else
      march2_item<CZ, AHEAD, MODE, false>(a, t, grp, z0, x0, inj);
  }
}

// Adjoint with cooperative blocks: the P wavefronts of a block march the P
// shots of one group over the same tile, park their image accumulators in
// LDS and the block adds their sum over the shots (in shot order, float64)
// to the group's accumulator: one read-modify-write per point and launch
// for P shots instead of P.
template <int CZ, int AHEAD, int P>
__global__ void __launch_bounds__(kLanes* P) k_march2t_coop(StepArgs a) {
  __shared__ float inj_all[P * kLanes];
  __shared__ float accs[P * CZ * kLanes];
  const int wv = (int)uni((uint32_t)threadIdx.x / kLanes);
  const int lane = threadIdx.x & (kLanes - 1);
  float* inj = inj_all + wv * kLanes;
  inj[lane] = 0.f;
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
  const bool xfast = (a.resident_grid & 4) != 0;  // see k_march2s
  for (int L = first; L < hi; L += stride) {
    const int grp = L % a.ngroups;
    const int tl = L / a.ngroups;
    const int tzi = xfast ? tl / g.ntx : tl % g.ntz;
    const int txi = xfast ? tl % g.ntx : tl / g.ntz;
    const int z0 = tzi * CZ;
    const int x0 = g.x_org + txi * kCore;
    const int t = tzi * g.ntx + txi;
    const bool interior = x0 - kRadius >= g.nb &&
                          x0 + kCore + kRadius <= g.nb + g.nx &&
                          z0 - kRadius >= g.nb &&
                          z0 + CZ + kRadius <= g.nb + g.nz;
    float* accl = accs + wv * CZ * kLanes;
    const int my_shot = grp * P + wv;
    if (interior)
      march2_item<CZ, AHEAD, kAdjoint, true, true>(a, t, grp, z0, x0, inj,
                                                   accl, my_shot);
    else
      march2_item<CZ, AHEAD, kAdjoint, false, true>(a, t, grp, z0, x0, inj,
                                                    accl, my_shot);
    __syncthreads();
    for (int e = threadIdx.x; e < CZ * kLanes; e += P * kLanes) {
      const int j = e / kLanes, ln = e % kLanes;
      const int xl = x0 - kRadius + ln, z = z0 + j;
      if (ln >= kRadius && ln < kLanes - kRadius && xl >= g.nb &&
          xl < g.nb + g.nx && z >= g.nb && z < g.nb + g.nz) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < P; ++w) sum += (double)accs[w * CZ * kLanes + e];
        a.acc[(int64_t)grp * mplane + (int64_t)(z - g.nb) * g.nx +
              (xl - g.nb)] += sum;
      }
    }
    __syncthreads();
  }
}

template <int CZ, int AHEAD, int P>
static hipError_t launch_t2_coop(const StepArgs& a, hipStream_t st) {
  static const int cap = resident_blocks(
      reinterpret_cast<const void*>(&k_march2t_coop<CZ, AHEAD, P>),
      kLanes * P);
  const int need = a.g.ntiles * a.ngroups;
  const int lim = (a.resident_grid & 1) ? cap : need;
  const int nblk = ((need < lim ? need : lim) + 7) / 8 * 8;
  hipLaunchKernelGGL((k_march2t_coop<CZ, AHEAD, P>), dim3(nblk),
                     dim3(kLanes * P), 0, st, a);
  return hipGetLastError();
}

template <int CZ, int AHEAD, int MODE>
static hipError_t launch_t2_mode(const StepArgs& a, hipStream_t st) {
  if (MODE == kAdjoint && a.per_block == 4)
    return launch_t2_coop<CZ, AHEAD, 4>(a, st);
  if (MODE == kAdjoint && a.per_block == 8)
    return launch_t2_coop<CZ, AHEAD, 8>(a, st);
  static const int cap = resident_blocks(
      reinterpret_cast<const void*>(&k_march2t<CZ, AHEAD, MODE>),
      kLanes * kWaves);
  const int items = a.g.ntiles * a.ngroups;
  const int need = (items + kWaves - 1) / kWaves;
  const int lim = (a.resident_grid & 1) ? cap : need;
  const int nblk = ((need < lim ? need : lim) + 7) / 8 * 8;
  hipLaunchKernelGGL((k_march2t<CZ, AHEAD, MODE>), dim3(nblk),
                     dim3(kLanes * kWaves), 0, st, a);
  return hipGetLastError();
}

template <int CZ, int AHEAD>
static hipError_t launch_t2_shape(int mode, const StepArgs& a,
                                  hipStream_t st) {
  switch (mode) {
    case kBackground: return launch_t2_mode<CZ, AHEAD, kBackground>(a, st);
    case kBorn: return launch_t2_mode<CZ, AHEAD, kBorn>(a, st);
    case kAdjoint: return launch_t2_mode<CZ, AHEAD, kAdjoint>(a, st);
  }
  return hipErrorInvalidValue;  // no fused mode: needs stored sources
}

hipError_t launch_march2t(int cz, int ahead, int mode, const StepArgs& a,
                          hipStream_t st) {
  if (cz == 16 && ahead == 2) return launch_t2_shape<16, 2>(mode, a, st);
  if (cz == 16 && ahead == 4) return launch_t2_shape<16, 4>(mode, a, st);
  return hipErrorInvalidValue;
}

}  // namespace brls
