// z-marching form of the 2-D time step (gfx950).
//
// The same update as k_step2d (difference form, the four StepModes; see
// layout.h and stencil2d.hip), organised around a wavefront instead of a
// block. A work item is a 64-column strip of a chunk of CZ rows for a group
// of shots; one wavefront walks down the chunk a row at a time, lane i
// holding column x0 + i. The z-derivative comes from a queue of nine rows
// kept in registers; the x-derivative from lanes i -+ 1..4 through DPP wave
// shifts, the four columns past each edge of the strip entering as the
// shifts' fill values (one load per row brings all eight). Nothing is staged
// in LDS and no barrier is taken: wavefronts never wait for one another, and
// the loads of row j + AHEAD are issued before row j is computed. Accesses
// are buffer loads and stores whose row offset is a scalar register.
// Receivers are handled on the rows that hold them, up to 64 entries per
// pass (each tile's entries sorted by local index, so by row).
//
// The floating-point operations and their order are those of k_step2d
// (both forms agree to float32 rounding of contractions the compiler may
// form differently).
#include <hip/hip_runtime.h>

#include "devutil.h"
#include "kernels.h"
#include "layout.h"
#include "march_common.h"

namespace brls {

namespace {

using namespace dev;
using namespace march;

// One work item: strip [x0, x0 + 64) x rows [z0, z0 + CZ) for the shots of
// group grp; t is the tile's receiver bin. inj: this wavefront's 64 LDS
// words (all zero on entry and on exit). AHEAD: rows whose loads are in
// flight ahead of the row computed.
template <int CZ, int AHEAD, int MODE, bool INT>
__device__ __forceinline__ void march_item(const StepArgs& a, int t, int grp,
                                           int z0, int x0, float* inj) {
  constexpr bool BG = MODE == kBackground || MODE == kBornFused;
  constexpr bool FW = MODE != kBackground;
  constexpr bool SRC_D2 = MODE == kBorn || MODE == kAdjoint;
  constexpr bool PERT = MODE == kBorn || MODE == kBornFused;
  constexpr int D = AHEAD;
  const Geo2D& g = a.g;
  const int lane = threadIdx.x & (kLanes - 1);
  const int x = x0 + lane;
  const int pitch4 = g.pitch * 4;
  const int nx4 = g.nx * 4;
  const int mplane = g.nz * g.nx;
  // byte offsets. Storage arrays: uniform part = padded row z0 - 4
  // (storage row z0) at column x0, lane part = 4 * lane; the halo load
  // starts 4 columns left (its lane part: lanes 0..3 -> x0-4.., 60..63 ->
  // x0+64.., the rest their own column). Model arrays: lane part = column
  // x - nb (used only inside the model), uniform part = (z - nb) * nx.
  const int s_top = (z0 * g.pitch + x0 + g.xoff) * 4;
  const int v_lane = lane * 4;
  const int v_halo = (lane < 4 ? lane : (lane >= 60 ? lane + 8 : lane + 4)) * 4;
  // (clamped so that even a lane outside the model holds an in-bounds
  // offset; such lanes never access the model arrays)
  const int v_mod = max(x - g.nb, 0) * 4;
  const bool okx = INT || (x >= 0 && x < g.px);
  const bool inx = INT || (x >= g.nb && x < g.nb + g.nx);
  const int dx = INT ? 0 : (okx ? sponge_depth(x, g.nb, g.nx) : 0);
  const Rsrc Rw = rsrc(a.wp);
  const Rsrc Rp = rsrc(a.pm);

  float acc[CZ];
#pragma unroll
  for (int j = 0; j < CZ; ++j) acc[j] = 0.f;
  bool any = false;

  const int s0 = grp * a.per_block;
  const int s1 = min(s0 + a.per_block, a.nshots);
  for (int s = s0; s < s1; ++s) {
    if (!active(MODE, a.n, uni(a.tab[s].nt))) continue;
    any = true;
    const ShotDev sd = shot(a.tab, s);
    const int lin = (MODE == kAdjoint) ? a.n + 1 : a.n;
    const Rsrc Rfi = rsrc((lin & 1) ? sd.f[1] : sd.f[0]);
    const Rsrc Rfo = rsrc((lin & 1) ? sd.f[0] : sd.f[1]);
    const Rsrc Rfv = rsrc(sd.f[2]);
    const Rsrc Rbi = rsrc((a.n & 1) ? sd.b[1] : sd.b[0]);
    const Rsrc Rbo = rsrc((a.n & 1) ? sd.b[0] : sd.b[1]);
    const Rsrc Rbv = rsrc(sd.b[2]);
    const int fr = (MODE == kAdjoint ? a.n - 1 : a.n) - a.d2_n0;
    const Rsrc Rd = rsrc(sd.d2 + (int64_t)fr * mplane);
    const float wav_n = BG ? sd.wav[a.n] : 0.f;
    // receivers of this tile: next entry e of [e, e1) and its row
    int e = 0, e1 = 0, erow = CZ;
    if (FW) {
      e = uni(sd.rptr[t]);
      e1 = uni(sd.rptr[t + 1]);
      if (e < e1) erow = uni(sd.rent[e].x) >> 6;
    }

    // queues q[r] = field at padded row z0 - 4 + r; per-row values of row j
    float q[CZ + 8], bq[CZ + 8];
    float hh[CZ], bhh[CZ], vo[CZ], bvo[CZ], dv[CZ], Wr[CZ], Pr[CZ];
    // rolling offsets of the rows whose loads are issued next: queue row
    // (s_q), its value row 4 above (s_c) and that row's model row (m_c)
    int s_q = s_top;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (FW) q[r] = bload(Rfi, v_lane, s_q);
      if (BG) bq[r] = bload(Rbi, v_lane, s_q);
      s_q = opaque(s_q + pitch4);
    }
    int s_c = opaque(s_top + 4 * pitch4);
    int m_c = opaque((z0 - g.nb) * nx4);
    int z_l = z0;
    auto load_row = [&](int j) {
      const int z = z_l;
      const bool okz = INT || z < g.pz;
      const bool inz = INT || (z >= g.nb && z < g.nb + g.nz);
      if (FW) {
        q[j + 8] = bload(Rfi, v_lane, s_q);
        hh[j] = bload(Rfi, v_halo, s_c - 16);
        vo[j] = bload(Rfv, v_lane, s_c);
      }
      if (BG) {
        bq[j + 8] = bload(Rbi, v_lane, s_q);
        bhh[j] = bload(Rbi, v_halo, s_c - 16);
        bvo[j] = bload(Rbv, v_lane, s_c);
      }
      Wr[j] = (okx && okz) ? bload(Rw, v_lane, s_c) : 0.f;
      Pr[j] = (PERT && inx && inz) ? bload(Rp, v_mod, m_c) : 0.f;
      dv[j] = (SRC_D2 && inx && inz) ? bload<kNT>(Rd, v_mod, m_c) : 0.f;
      s_q = opaque(s_q + pitch4);
      s_c = opaque(s_c + pitch4);
      m_c = opaque(m_c + nx4);
      z_l = opaque(z_l + 1);
    };
#pragma unroll
    for (int j = 0; j < D; ++j) load_row(j);

    int s_w = opaque(s_top + 4 * pitch4);  // row j being computed
    int m_w = opaque((z0 - g.nb) * nx4);
    int z_w = z0;
#pragma unroll
    for (int j = 0; j < CZ; ++j) {
      // keep each row's work (and the loads it issues) in its own stretch
      // of the schedule, so the loads run AHEAD rows ahead, no further
      __builtin_amdgcn_sched_barrier(0);
      if (j + D < CZ) load_row(j + D);
      const int z = z_w;
      const int so = s_w, mo = m_w;
      s_w = opaque(s_w + pitch4);
      m_w = opaque(m_w + nx4);
      z_w = opaque(z_w + 1);
      if (!INT && z >= g.pz) continue;  // below the padded grid
      const bool inz = INT || (z >= g.nb && z < g.nb + g.nz);
      const bool ok = okx;
      const bool in = inx && inz;
      float C1 = 1.f, C2 = 1.f;
      if (!INT) {
        const int dz = sponge_depth(z, g.nb, g.nz);
        const float damp =
            ok ? g.eta_scale * (float)(dz * dz + dx * dx) : 0.f;
        C1 = __builtin_amdgcn_rcpf(1.f + damp);
        C2 = (1.f - damp) * C1;
      }
      float srcv = 0.f;  // Born source of this point (fused mode)
      if (BG) {
        const float c = bq[j + 4];
        const float src = (z == sd.src_z && x == sd.src_x) ? wav_n : 0.f;
        const float incb =
            Wr[j] * (lap8(g.w, c, znb(bq, j + 4), xnb(c, bhh[j])) + src);
        const float vb = INT ? bvo[j] + incb : fmaf(C2, bvo[j], C1 * incb);
        if (ok) {
          bstore(Rbv, v_lane, so, vb);
          bstore(Rbo, v_lane, so, c + vb);
        }
        srcv = incb;
        if (MODE == kBackground && a.write_d2 && in)
          bstore<kNT>(Rd, v_mod, mo, incb);
      }
      if (!FW) continue;
      const float c = q[j + 4];
      float injv = 0.f;
      if (erow == j) {  // receivers on this row (wave-uniform)
        for (;;) {
          const int k = e + lane;
          int2 re = make_int2(0, 0);
          if (k < e1) re = sd.rent[k];
          const bool m = k < e1 && (re.x >> 6) == j;
          const int cnt = __popcll(__ballot(m));
          if (MODE == kAdjoint) {
            const float* res = a.dat + sd.dat_off + (int64_t)a.n * sd.nrec;
            if (m) atomicAdd(&inj[re.x & (kLanes - 1)], res[re.y]);
          } else {  // d^n = du^n at the receivers
            float* dat = a.dat + sd.dat_off + (int64_t)a.n * sd.nrec;
            const float val = __int_as_float(__builtin_amdgcn_ds_bpermute(
                (re.x & (kLanes - 1)) << 2, __float_as_int(c)));
            if (m) dat[re.y] = val;
          }
          e += cnt;
          if (cnt < kLanes || e >= e1) break;
        }
        erow = e < e1 ? (uni(sd.rent[e].x) >> 6) : CZ;
        if (MODE == kAdjoint) {
          injv = inj[lane];
          inj[lane] = 0.f;
        }
      }
      const float lap = lap8(g.w, c, znb(q, j + 4), xnb(c, hh[j]));
      float inc;
      if (MODE == kBorn) {
        inc = Wr[j] * lap;
        if (in) inc = fmaf(-Pr[j], dv[j], inc);
      } else if (MODE == kBornFused) {
        inc = fmaf(-Pr[j], srcv, Wr[j] * lap);
      } else {
        inc = Wr[j] * (lap + injv);
      }
      const float vn = INT ? vo[j] + inc : fmaf(C2, vo[j], C1 * inc);
      const float un = c + vn;
      if (ok) {
        bstore(Rfv, v_lane, so, vn);
        bstore(Rfo, v_lane, so, un);
      }
      if (MODE == kAdjoint && in) acc[j] = fmaf(-dv[j], un, acc[j]);
    }
  }
  if (MODE == kAdjoint && any) {
    double* out =
        a.acc + (int64_t)grp * mplane + (int64_t)(z0 - g.nb) * g.nx + x - g.nb;
    int mo = 0, z = z0;
#pragma unroll
    for (int j = 0; j < CZ; ++j) {
      if (inx && (INT || (z >= g.nb && z < g.nb + g.nz)))
        out[mo] += (double)acc[j];
      mo = opaque(mo + g.nx);
      z = opaque(z + 1);
    }
  }
}

}  // namespace

template <int CZ, int AHEAD, int MODE>
__global__ void __launch_bounds__(kLanes* kWaves) k_march2d(StepArgs a) {
  __shared__ float inj_all[MODE == kAdjoint ? kWaves * kLanes : 1];
  const int wv = (int)uni((uint32_t)threadIdx.x / kLanes);
  float* inj = inj_all + (MODE == kAdjoint ? wv * kLanes : 0);
  if (MODE == kAdjoint) inj[threadIdx.x & (kLanes - 1)] = 0.f;
  const Geo2D& g = a.g;
  // Work items (strip chunk, shot group), shot groups innermost and chunks
  // of one strip next, are split into 8 contiguous ranges, one per XCD (the
  // hardware deals consecutive block ids to the 8 XCDs in turn; gridDim.x
  // is a multiple of 8); each wavefront loops over its XCD's range.
  // (Or, with bit 1 of resident_grid, in launch order.)
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
  for (int L = first; L < hi; L += stride) {
    const int grp = L % a.ngroups;
    const int tl = L / a.ngroups;
    const int tzi = tl % g.ntz, txi = tl / g.ntz;
    const int z0 = tzi * CZ;
    const int x0 = g.x_org + txi * kLanes;
    const int t = tzi * g.ntx + txi;
    const bool interior = x0 >= g.nb && x0 + kLanes <= g.nb + g.nx &&
                          z0 >= g.nb && z0 + CZ <= g.nb + g.nz;
    if (interior)
      march_item<CZ, AHEAD, MODE, true>(a, t, grp, z0, x0, inj);
    else
      march_item<CZ, AHEAD, MODE, false>(a, t, grp, z0, x0, inj);
  }
}

template <int CZ, int AHEAD, int MODE>
static hipError_t launch_march_mode(const StepArgs& a, hipStream_t st) {
  static const int cap = resident_blocks(
      reinterpret_cast<const void*>(&k_march2d<CZ, AHEAD, MODE>),
      kLanes * kWaves);
  const int items = a.g.ntiles * a.ngroups;
  const int need = (items + kWaves - 1) / kWaves;
  const int lim = (a.resident_grid & 1) ? cap : need;
  const int nblk = ((need < lim ? need : lim) + 7) / 8 * 8;
  hipLaunchKernelGGL((k_march2d<CZ, AHEAD, MODE>), dim3(nblk),
                     dim3(kLanes * kWaves), 0, st, a);
  return hipGetLastError();
}

template <int CZ, int AHEAD>
static hipError_t launch_march_shape(int mode, const StepArgs& a,
                                     hipStream_t st) {
  switch (mode) {
    case kBackground:
      return launch_march_mode<CZ, AHEAD, kBackground>(a, st);
    case kBorn: return launch_march_mode<CZ, AHEAD, kBorn>(a, st);
    case kBornFused: return launch_march_mode<CZ, AHEAD, kBornFused>(a, st);
    default: return launch_march_mode<CZ, AHEAD, kAdjoint>(a, st);
  }
}

hipError_t launch_march2d(int cz, int ahead, int mode, const StepArgs& a,
                          hipStream_t st) {
  if (cz == 8 && ahead == 2) return launch_march_shape<8, 2>(mode, a, st);
  if (cz == 8 && ahead == 4) return launch_march_shape<8, 4>(mode, a, st);
  if (cz == 12 && ahead == 2) return launch_march_shape<12, 2>(mode, a, st);
  if (cz == 12 && ahead == 4) return launch_march_shape<12, 4>(mode, a, st);
  if (cz == 16 && ahead == 2) return launch_march_shape<16, 2>(mode, a, st);
  if (cz == 16 && ahead == 4) return launch_march_shape<16, 4>(mode, a, st);
  if (cz == 32 && ahead == 2) return launch_march_shape<32, 2>(mode, a, st);
  if (cz == 32 && ahead == 4) return launch_march_shape<32, 4>(mode, a, st);
  return hipErrorInvalidValue;
}

}  // namespace brls
