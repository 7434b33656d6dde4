// 2-D time-step kernels of the Born operator pair (gfx950).
//
// One kernel template advances damped acoustic wavefields by one step of the
// 8th-order-in-space / second-order-in-time scheme, in difference form (see
// layout.h). Modes (StepMode):
//   kBackground  background field u0 of a shot; its increment on the model
//                region is the Born source D2u0^n = u0^{n+1} - 2u0^n +
//                u0^{n-1} (exactly: C1 = C2 = 1 there), optionally stored;
//   kBorn        Born field du with source -m D2u0^n, recording du^n at the
//                receivers (the de-migration operator A, eq. 1 of the paper);
//   kBornFused   background and Born field advanced together, the Born
//                source taken from the background's increment on the fly;
//   kAdjoint     adjoint field psi run backward in time with the data
//                residual injected at the receivers, accumulating the
//                cross-correlation image -D2u0^{k-1} psi^k (the migration
//                operator A^T, eq. 2).
//
// Work decomposition: a block owns a TZ x TX tile of the padded grid and runs
// it for up to `per_block` shots in turn, so the medium and the model vector
// are read once per tile and step for all of them. The tile plus a 4-cell
// halo is staged in LDS; each thread handles PZ = TZ/NTZ consecutive points
// of one column, taking the z-derivative from a register column and the
// x-derivative from LDS rows. Tiles wholly inside the model region (most of
// them) take a path with no predicates and no damping arithmetic. Blocks are
// renumbered so each of the 8 XCDs gets a contiguous range of tiles
// (neighbouring tiles share halos through that XCD's L2). Global accesses use
// 32-bit offsets from uniform bases; the Born-source stream is read and
// written with non-temporal hints (it is touched once per step).
#include <hip/hip_runtime.h>

#include "devutil.h"
#include "kernels.h"
#include "layout.h"

namespace brls {

namespace {

using namespace dev;

// L u * h^2 at one point on differences, smallest weights first. col: the
// thread's register column (centre at col[j+4]); rw: the point in LDS.
template <int NC>
__device__ __forceinline__ float lap_at(const StencilW& w, const float (&col)[NC],
                                        int j, const float* rw) {
  const float c = col[j + 4];
  float lap = w.c4 * (((col[j + 8] - c) + (col[j] - c)) +
                      ((rw[4] - c) + (rw[-4] - c)));
  lap = fmaf(w.c3, ((col[j + 7] - c) + (col[j + 1] - c)) +
                       ((rw[3] - c) + (rw[-3] - c)),
             lap);
  lap = fmaf(w.c2, ((col[j + 6] - c) + (col[j + 2] - c)) +
                       ((rw[2] - c) + (rw[-2] - c)),
             lap);
  lap = fmaf(w.c1, ((col[j + 5] - c) + (col[j + 3] - c)) +
                       ((rw[1] - c) + (rw[-1] - c)),
             lap);
  return lap;
}

// Staging of rows [z0-4, z0+TZ+4) x columns [x0-4, x0+TX+4) of a field into
// LDS, split in two so all global loads of a step can be in flight before the
// block synchronises: thread (tx, ty) owns rows ty, ty + NTZ, ... (column
// x0 + tx, plus one halo column for lanes tx < 8).
template <int TX, int NTZ, int LZ>
struct Stager {
  static constexpr int RPT = (LZ + NTZ - 1) / NTZ;
  float v[RPT], h[RPT];
  __device__ __forceinline__ void load(cgfloat* u, uint32_t base,
                                       uint32_t pitch, int tx, int ty) {
    const int c = tx < kRadius ? tx - kRadius : TX + tx - kRadius;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = ty + k * NTZ;
      if (r < LZ) {
        const uint32_t row = base + (uint32_t)r * pitch;
        v[k] = *at(u, row + tx);
        if (tx < 2 * kRadius) h[k] = *at(u, row + c);
      }
    }
  }
  __device__ __forceinline__ void store(float* tile, int tx, int ty) const {
    constexpr int LX = TX + 2 * kRadius;
    const int c = tx < kRadius ? tx - kRadius : TX + tx - kRadius;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = ty + k * NTZ;
      if (r < LZ) {
        tile[r * LX + kRadius + tx] = v[k];
        if (tx < 2 * kRadius) tile[r * LX + kRadius + c] = h[k];
      }
    }
  }
};

template <int TX, int TZ, int NTZ, int MODE, bool PIPE, bool INT>
__device__ __forceinline__ void step_body(const StepArgs& a, int t, int grp,
                                          int z0, int x0, float* tile,
                                          float* btile, float* inj) {
  constexpr int NT = TX * NTZ;
  constexpr int PZ = TZ / NTZ;
  constexpr int LX = TX + 2 * kRadius;
  constexpr int LZ = TZ + 2 * kRadius;
  constexpr int NC = PZ + 2 * kRadius;
  const Geo2D& g = a.g;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * TX + tx;
  const int x = x0 + tx;
  const int zb = z0 + ty * PZ;
  const uint32_t pitch = (uint32_t)g.pitch;
  const uint32_t mplane = (uint32_t)g.nz * (uint32_t)g.nx;
  // storage offset of this thread's first point and of the staged block
  const uint32_t so0 = (uint32_t)(zb + kGhost) * pitch + (uint32_t)(x + g.xoff);
  const uint32_t tbase = (uint32_t)z0 * pitch + (uint32_t)(x0 + g.xoff);
  const uint32_t mo0 =
      (uint32_t)(zb - g.nb) * (uint32_t)g.nx + (uint32_t)(x - g.nb);

  float W[PZ], C1[PZ], C2[PZ], P[PZ], acc[PZ];
  bool ok[PZ], in[PZ];
  cgfloat* wp = G(a.wp);
#pragma unroll
  for (int j = 0; j < PZ; ++j) {
    const int z = zb + j;
    if (INT) {
      ok[j] = in[j] = true;
      C1[j] = C2[j] = 1.f;
    } else {
      ok[j] = x >= 0 && x < g.px && z < g.pz;
      in[j] = x >= g.nb && x < g.nb + g.nx && z >= g.nb && z < g.nb + g.nz;
      const int dx = ok[j] ? sponge_depth(x, g.nb, g.nx) : 0;
      const int dz = ok[j] ? sponge_depth(z, g.nb, g.nz) : 0;
      const float damp = g.eta_scale * (float)(dz * dz + dx * dx);
      C1[j] = __builtin_amdgcn_rcpf(1.f + damp);
      C2[j] = (1.f - damp) * C1[j];
    }
    W[j] = ok[j] ? *at(wp, so0 + j * pitch) : 0.f;
    P[j] = ((MODE == kBorn || MODE == kBornFused) && in[j])
               ? *at(G(a.pm), mo0 + j * (uint32_t)g.nx)
               : 0.f;
    acc[j] = 0.f;
  }

  const int s0 = grp * a.per_block;
  const int s1 = min(s0 + a.per_block, a.nshots);
  // A shot takes part in this step while it has time steps left.
  auto next_active = [&](int from) {
    for (int k = from; k < s1; ++k) {
      const int nt = uni(a.tab[k].nt);
      if ((MODE == kAdjoint) ? (a.n <= nt - 1) : (a.n < nt - 1)) return k;
    }
    return s1;
  };
  // Global loads of one shot: the staged tiles and the per-point values.
  // The next shot's loads are issued before the current shot is computed,
  // so their latency overlaps the arithmetic.
  Stager<TX, NTZ, LZ> sf, sb;
  float nv[PZ], nbv[PZ], nd2[PZ];
  auto issue = [&](int k) {
    const ShotDev sd = shot(a.tab, k);
    const int lin = (MODE == kAdjoint) ? a.n + 1 : a.n;
    if (MODE != kBackground)
      sf.load(G((lin & 1) ? sd.f[1] : sd.f[0]), tbase, pitch, tx, ty);
    if (MODE == kBackground || MODE == kBornFused)
      sb.load(G((a.n & 1) ? sd.b[1] : sd.b[0]), tbase, pitch, tx, ty);
    const int fr = (MODE == kAdjoint ? a.n - 1 : a.n) - a.d2_n0;
    cgfloat* d2 = G(sd.d2) + (int64_t)fr * mplane;
#pragma unroll
    for (int j = 0; j < PZ; ++j) {
      const uint32_t so = so0 + j * pitch;
      nv[j] = (MODE != kBackground) ? *at(G(sd.f[2]), so) : 0.f;
      nbv[j] = (MODE == kBackground || MODE == kBornFused)
                   ? *at(G(sd.b[2]), so)
                   : 0.f;
      nd2[j] = ((MODE == kBorn || MODE == kAdjoint) && in[j])
                   ? __builtin_nontemporal_load(
                         at(d2, mo0 + j * (uint32_t)g.nx))
                   : 0.f;
    }
  };
  int prev = -1;
  int s = next_active(s0);
  if (PIPE && s < s1) issue(s);
  while (s < s1) {
    if (!PIPE) issue(s);
    const ShotDev sd = shot(a.tab, s);
    const int lin = (MODE == kAdjoint) ? a.n + 1 : a.n;
    gfloat* uout = G((lin & 1) ? sd.f[0] : sd.f[1]);
    gfloat* vv = G(sd.f[2]);
    gfloat* bvv = G(sd.b[2]);
    const int fr = (MODE == kAdjoint ? a.n - 1 : a.n) - a.d2_n0;
    gfloat* d2 = G(sd.d2) + (int64_t)fr * mplane;
    __syncthreads();  // previous shot done with the LDS arrays
    if (MODE == kAdjoint && prev >= 0) {
      const ShotDev pd = shot(a.tab, prev);
      for (int e = pd.rptr[t] + tid; e < pd.rptr[t + 1]; e += NT)
        inj[pd.rent[e].x] = 0.f;
    }
    if (MODE != kBackground) sf.store(tile, tx, ty);
    if (MODE == kBackground || MODE == kBornFused) sb.store(btile, tx, ty);
    __syncthreads();
    if (MODE == kBorn || MODE == kBornFused) {  // d^n = du^n at receivers
      gfloat* dat = G(a.dat) + sd.dat_off + (int64_t)a.n * sd.nrec;
      for (int e = sd.rptr[t] + tid; e < sd.rptr[t + 1]; e += NT) {
        const int2 re = sd.rent[e];
        const int lz = re.x / TX, lx = re.x - lz * TX;
        dat[re.y] = tile[(lz + kRadius) * LX + lx + kRadius];
      }
    }
    if (MODE == kAdjoint) {  // R^T r^k
      cgfloat* res = G(a.dat) + sd.dat_off + (int64_t)a.n * sd.nrec;
      for (int e = sd.rptr[t] + tid; e < sd.rptr[t + 1]; e += NT) {
        const int2 re = sd.rent[e];
        atomicAdd(&inj[re.x], res[re.y]);
      }
      __syncthreads();
    }
    float vold[PZ], bvold[PZ], d2v[PZ];
#pragma unroll
    for (int j = 0; j < PZ; ++j) {
      vold[j] = nv[j];
      bvold[j] = nbv[j];
      d2v[j] = nd2[j];
    }
    const int sn = next_active(s + 1);
    if (PIPE && sn < s1) issue(sn);
    float col[NC], bcol[NC];
    if (MODE != kBackground)
#pragma unroll
      for (int i = 0; i < NC; ++i)
        col[i] = tile[(ty * PZ + i) * LX + kRadius + tx];
    if (MODE == kBackground || MODE == kBornFused)
#pragma unroll
      for (int i = 0; i < NC; ++i)
        bcol[i] = btile[(ty * PZ + i) * LX + kRadius + tx];
#pragma unroll
    for (int j = 0; j < PZ; ++j) {
      const uint32_t so = so0 + j * pitch;
      const uint32_t mo = mo0 + j * (uint32_t)g.nx;
      float srcv = 0.f;  // Born source of this point
      if (MODE == kBackground || MODE == kBornFused) {
        const float* brw = &btile[(ty * PZ + j + kRadius) * LX + kRadius + tx];
        const float src =
            (zb + j == sd.src_z && x == sd.src_x) ? sd.wav[a.n] : 0.f;
        const float incb = W[j] * (lap_at(g.w, bcol, j, brw) + src);
        const float vb =
            INT ? bvold[j] + incb : fmaf(C2[j], bvold[j], C1[j] * incb);
        if (ok[j]) {
          *at(bvv, so) = vb;
          *at(G((a.n & 1) ? sd.b[0] : sd.b[1]), so) = bcol[j + kRadius] + vb;
        }
        srcv = incb;
        if (MODE == kBackground && a.write_d2 && in[j])
          __builtin_nontemporal_store(incb, at(d2, mo));
      }
      if (MODE == kBackground) continue;
      const float* rw = &tile[(ty * PZ + j + kRadius) * LX + kRadius + tx];
      const float c = col[j + kRadius];
      const float lap = lap_at(g.w, col, j, rw);
      float inc;
      if (MODE == kBorn) {
        inc = W[j] * lap;
        if (in[j]) inc = fmaf(-P[j], d2v[j], inc);
      } else if (MODE == kBornFused) {
        inc = fmaf(-P[j], srcv, W[j] * lap);
      } else {
        inc = W[j] * (lap + inj[(ty * PZ + j) * TX + tx]);
      }
      const float vn =
          INT ? vold[j] + inc : fmaf(C2[j], vold[j], C1[j] * inc);
      const float un = c + vn;
      if (ok[j]) {
        *at(vv, so) = vn;
        *at(uout, so) = un;
      }
      if (MODE == kAdjoint && in[j]) acc[j] = fmaf(-d2v[j], un, acc[j]);
    }
    prev = s;
    s = sn;
  }
  if (MODE == kAdjoint && prev >= 0) {
    double* out = a.acc + (int64_t)grp * mplane;
#pragma unroll
    for (int j = 0; j < PZ; ++j)
      if (in[j]) out[mo0 + j * (uint32_t)g.nx] += (double)acc[j];
    // leave inj[] all zero for the block's next work item
    __syncthreads();
    const ShotDev pd = shot(a.tab, prev);
    for (int e = pd.rptr[t] + tid; e < pd.rptr[t + 1]; e += NT)
      inj[pd.rent[e].x] = 0.f;
  }
}

}  // namespace

template <int TX, int TZ, int NTZ, int MODE, bool PIPE>
__global__ void __launch_bounds__(TX* NTZ) k_step2d(StepArgs a) {
  constexpr int LX = TX + 2 * kRadius;
  constexpr int LZ = TZ + 2 * kRadius;
  static_assert(TZ % NTZ == 0 && TX >= 2 * kRadius, "tile shape");
  __shared__ float tile[MODE == kBackground ? 1 : LZ * LX];
  __shared__ float btile[(MODE == kBackground || MODE == kBornFused) ? LZ * LX
                                                                     : 1];
  __shared__ float inj[MODE == kAdjoint ? TZ * TX : 1];
  const Geo2D& g = a.g;
  if (MODE == kAdjoint)
    for (int i = threadIdx.y * TX + threadIdx.x; i < TZ * TX; i += TX * NTZ)
      inj[i] = 0.f;
  // Work items (tile, shot group) are split into 8 contiguous ranges, one
  // per XCD (the hardware deals consecutive block ids to the 8 XCDs in
  // turn; gridDim.x is a multiple of 8), and each block loops over its
  // XCD's range with a stride of the number of blocks placed there.
  // (Or, with bit 1 of resident_grid, in launch order.)
  const int items = g.ntiles * a.ngroups;
  int first, hi, stride;
  if (a.resident_grid & 2) {
    first = blockIdx.x;
    hi = items;
    stride = gridDim.x;
  } else {
    const int xcd = blockIdx.x & 7;
    const int q = items >> 3, r = items & 7;
    first = xcd * q + min(xcd, r) + (int)(blockIdx.x >> 3);
    hi = xcd * q + min(xcd, r) + q + (xcd < r ? 1 : 0);
    stride = gridDim.x >> 3;
  }
  for (int L = first; L < hi; L += stride) {
    const int t = L % g.ntiles;
    const int grp = L / g.ntiles;
    const int tzi = t / g.ntx;
    const int txi = t - tzi * g.ntx;
    const int z0 = tzi * TZ;
    const int x0 = g.x_org + txi * TX;
    const bool interior = x0 >= g.nb && x0 + TX <= g.nb + g.nx &&
                          z0 >= g.nb && z0 + TZ <= g.nb + g.nz;
    if (interior)
      step_body<TX, TZ, NTZ, MODE, PIPE, true>(a, t, grp, z0, x0, tile, btile,
                                               inj);
    else
      step_body<TX, TZ, NTZ, MODE, PIPE, false>(a, t, grp, z0, x0, tile,
                                                btile, inj);
  }
}

// Last sample of the Born data, d^{nt-1} = du^{nt-1} at the receivers.
__global__ void k_born_last(const ShotDev* tab, int nshots, float* dat,
                            int two_step) {
  const int s = blockIdx.y;
  if (s >= nshots) return;
  const ShotDev sd = tab[s];
  const int lvl = sd.nt - 1;
  const int set = two_step ? ((lvl + 1) >> 1) & 1 : lvl & 1;
  const float* u = set ? sd.f[1] : sd.f[0];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < sd.nrec;
       j += gridDim.x * blockDim.x)
    dat[sd.dat_off + (int64_t)lvl * sd.nrec + j] = u[sd.rsidx[j]];
}

// Image = (sum over accumulators) / W' on the model region.
__global__ void k_adj_finalize(const double* acc, int ngroups, Geo2D g,
                               const float* wp, float* out, double* out64) {
  const int64_t mplane = (int64_t)g.nz * g.nx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mplane;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < ngroups; ++k) s += acc[(int64_t)k * mplane + i];
    const int z = (int)(i / g.nx), x = (int)(i - (int64_t)(i / g.nx) * g.nx);
    const double v = s / (double)wp[sidx2(g, z + g.nb, x + g.nb)];
    out[i] = (float)v;
    if (out64) out64[i] = v;
  }
}

// Save (restore = 0) or restore (restore = 1) the background state of every
// shot at level n0: u^{n0} (buffer n0 & 1) and v^{n0}, checkpoint `seg`.
__global__ void k_ckpt(const ShotDev* tab, int nshots, int n0, int seg,
                       int64_t fs, int restore) {
  const int s = blockIdx.y;
  if (s >= nshots) return;
  const ShotDev sd = tab[s];
  if (n0 >= sd.nt - 1) return;  // this shot ends before the segment
  float* ck = sd.ck + (int64_t)seg * 2 * fs;
  float* u = (n0 & 1) ? sd.b[1] : sd.b[0];
  float* v = sd.b[2];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < fs;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (restore) {
      u[i] = ck[i];
      v[i] = ck[fs + i];
    } else {
      ck[i] = u[i];
      ck[fs + i] = v[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
// Tile shapes the autotuner chooses from: (TX, TZ, thread rows, kind) with
// kind 0 = staged tile, shots in turn; 1 = staged tile, the next shot's
// loads issued before the current shot is computed; 2 = z-marching
// wavefronts (march2d.hip: 64-column strips of TZ-row chunks; the third
// number is then the rows of loads in flight ahead of the row computed);
// 3 = z-marching with two time steps per launch (march2t.hip: 56 output
// columns per strip).
static const TileShape kShapes[] = {
    {64, 16, 4, 0}, {64, 32, 4, 0}, {64, 8, 2, 0},  {32, 32, 8, 0},
    {64, 32, 8, 0}, {32, 16, 4, 0}, {64, 16, 4, 1}, {32, 32, 8, 1},
    {32, 16, 4, 1}, {64, 32, 8, 1}, {64, 8, 2, 1},  {64, 16, 2, 2},
    {64, 32, 2, 2}, {64, 16, 4, 2}, {64, 32, 4, 2}, {64, 8, 2, 2},
    {64, 8, 4, 2},  {56, 16, 2, 3}, {56, 16, 4, 3}, {64, 12, 2, 2},
    {64, 12, 4, 2},  {56, 20, 4, 4}, {56, 24, 4, 4}, {56, 32, 4, 4},
    {56, 16, 4, 4},
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int tile_shape_count() { return kNumShapes; }
TileShape tile_shape(int v) { return kShapes[v]; }

// Blocks of a kernel that fit on the device at once.
int resident_blocks(const void* kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads,
                                                   0) != hipSuccess ||
      per < 1)
    per = 1;
  return per * cus;
}

// Grid: one block per work item, capped at what fits on the device at once,
// rounded up to a multiple of 8 (the kernel's XCD split needs it).
template <int TX, int TZ, int NTZ, int MODE, bool PIPE>
static hipError_t launch_mode(const StepArgs& a, hipStream_t st) {
  static const int cap = resident_blocks(
      reinterpret_cast<const void*>(&k_step2d<TX, TZ, NTZ, MODE, PIPE>),
      TX * NTZ);
  const int items = a.g.ntiles * a.ngroups;
  const int lim = (a.resident_grid & 1) ? cap : items;
  const int nblk = ((items < lim ? items : lim) + 7) / 8 * 8;
  hipLaunchKernelGGL((k_step2d<TX, TZ, NTZ, MODE, PIPE>), dim3(nblk),
                     dim3(TX, NTZ), 0, st, a);
  return hipGetLastError();
}

template <int TX, int TZ, int NTZ, bool PIPE>
static hipError_t launch_shape(int mode, const StepArgs& a,
                               hipStream_t st) {
  switch (mode) {
    case kBackground:
      return launch_mode<TX, TZ, NTZ, kBackground, PIPE>(a, st);
    case kBorn: return launch_mode<TX, TZ, NTZ, kBorn, PIPE>(a, st);
    case kBornFused: return launch_mode<TX, TZ, NTZ, kBornFused, PIPE>(a, st);
    default: return launch_mode<TX, TZ, NTZ, kAdjoint, PIPE>(a, st);
  }
}

hipError_t launch_step2d(int variant, int mode, const StepArgs& a,
                         hipStream_t st) {
  switch (variant) {
    case 0: return launch_shape<64, 16, 4, false>(mode, a, st);
    case 1: return launch_shape<64, 32, 4, false>(mode, a, st);
    case 2: return launch_shape<64, 8, 2, false>(mode, a, st);
    case 3: return launch_shape<32, 32, 8, false>(mode, a, st);
    case 4: return launch_shape<64, 32, 8, false>(mode, a, st);
    case 5: return launch_shape<32, 16, 4, false>(mode, a, st);
    case 6: return launch_shape<64, 16, 4, true>(mode, a, st);
    case 7: return launch_shape<32, 32, 8, true>(mode, a, st);
    case 8: return launch_shape<32, 16, 4, true>(mode, a, st);
    case 9: return launch_shape<64, 32, 8, true>(mode, a, st);
    case 10: return launch_shape<64, 8, 2, true>(mode, a, st);
    case 11: return launch_march2d(16, 2, mode, a, st);
    case 12: return launch_march2d(32, 2, mode, a, st);
    case 13: return launch_march2d(16, 4, mode, a, st);
    case 14: return launch_march2d(32, 4, mode, a, st);
    case 15: return launch_march2d(8, 2, mode, a, st);
    case 16: return launch_march2d(8, 4, mode, a, st);
    case 17: return launch_march2t(16, 2, mode, a, st);
    case 18: return launch_march2t(16, 4, mode, a, st);
    case 19: return launch_march2d(12, 2, mode, a, st);
    case 20: return launch_march2d(12, 4, mode, a, st);
    case 21: return launch_march2s(20, 4, mode, a, st);
    case 22: return launch_march2s(24, 4, mode, a, st);
    case 23: return launch_march2s(32, 4, mode, a, st);
    case 24: return launch_march2s(16, 4, mode, a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_born_last(const ShotDev* tab, int nshots, int nrec_max,
                            float* dat, int two_step, hipStream_t st) {
  const dim3 grid((nrec_max + 255) / 256, nshots);
  hipLaunchKernelGGL(k_born_last, grid, dim3(256), 0, st, tab, nshots, dat,
                     two_step);
  return hipGetLastError();
}

hipError_t launch_adj_finalize(const double* acc, int ngroups,
                               const Geo2D& g, const float* wp, float* out,
                               double* out64, hipStream_t st) {
  const int64_t m = (int64_t)g.nz * g.nx;
  int blocks = (int)((m + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_adj_finalize, dim3(blocks), dim3(256), 0, st, acc,
                     ngroups, g, wp, out, out64);
  return hipGetLastError();
}

hipError_t launch_ckpt(const ShotDev* tab, int nshots, int n0, int seg,
                       int64_t fs, int restore, hipStream_t st) {
  int64_t b = (fs + 255) / 256;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_ckpt, dim3((int)b, nshots), dim3(256), 0, st, tab,
                     nshots, n0, seg, fs, restore);
  return hipGetLastError();
}

}  // namespace brls
