// 2-D time-step kernels of the Born operator pair (gfx950).
//
// One kernel template serves three uses, all advancing a damped acoustic
// wavefield by one step of the 8th-order / second-order scheme in difference
// form (see layout.h):
//   kBackground  background field u0 of a shot; writes the Born source
//                D2u0^n = u0^{n+1} - 2u0^n + u0^{n-1} (on the model region
//                this equals the step's increment W L u0^n + source exactly);
//   kBorn        Born field du with source -m D2u0^n, recording du^n at the
//                receivers (the de-migration operator A, eq. 1 of the paper);
//   kAdjoint     adjoint field psi run backward in time with the data residual
//                injected at the receivers, accumulating the cross-correlation
//                image -D2u0^{k-1} psi^k (the migration operator A^T, eq. 2).
//
// Work decomposition: a block owns a TZ x TX tile of the padded grid and runs
// it for up to `per_block` shots in turn, so the medium (W, sponge factors)
// and the model vector are read once per tile and step for all of them. The
// tile plus a 4-cell halo is staged in LDS; each thread handles PZ = TZ/NTZ
// consecutive points of one column, taking the z-derivative from a register
// column and the x-derivative from LDS rows. Blocks are renumbered so that
// each of the 8 XCDs receives a contiguous range of tiles (neighbouring tiles
// share halos through that XCD's L2).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "layout.h"

namespace brls {

// Hardware hands consecutive workgroup ids to the 8 XCDs round-robin; map
// them so each XCD works on a contiguous range of logical blocks.
__device__ __forceinline__ int xcd_chunk(int b, int n) {
  const int xcd = b & 7, k = b >> 3;
  const int q = n >> 3, r = n & 7;
  return xcd * q + min(xcd, r) + k;
}

__device__ __forceinline__ int sponge_depth(int i, int nb, int n) {
  return i < nb ? nb - i : (i >= nb + n ? i - (nb + n - 1) : 0);
}

template <int TX, int TZ, int NTZ, int MODE>
__global__ void __launch_bounds__(TX* NTZ) k_step2d(StepArgs a) {
  constexpr int NT = TX * NTZ;
  constexpr int PZ = TZ / NTZ;
  constexpr int LX = TX + 2 * kRadius;
  constexpr int LZ = TZ + 2 * kRadius;
  static_assert(TZ % NTZ == 0 && TX >= 2 * kRadius, "tile shape");
  __shared__ float tile[LZ * LX];
  __shared__ float inj[MODE == kAdjoint ? TZ * TX : 1];

  const Geo2D& g = a.g;
  const int L = xcd_chunk(blockIdx.x, g.ntiles * a.ngroups);
  const int t = L % g.ntiles;
  const int grp = L / g.ntiles;
  const int tzi = t / g.ntx;
  const int txi = t - tzi * g.ntx;
  const int z0 = tzi * TZ;
  const int x0 = g.x_org + txi * TX;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * TX + tx;
  const int x = x0 + tx;
  const int zb = z0 + ty * PZ;
  const bool colok = x >= 0 && x < g.px;
  const bool colint = x >= g.nb && x < g.nb + g.nx;
  const int dx = colok ? sponge_depth(x, g.nb, g.nx) : 0;
  const int64_t mplane = (int64_t)g.nz * g.nx;

  float W[PZ], C1[PZ], C2[PZ], P[PZ], acc[PZ];
  int64_t midx[PZ];
  bool ok[PZ], in[PZ];
#pragma unroll
  for (int j = 0; j < PZ; ++j) {
    const int z = zb + j;
    ok[j] = colok && z < g.pz;
    in[j] = colint && z >= g.nb && z < g.nb + g.nz;
    midx[j] = in[j] ? (int64_t)(z - g.nb) * g.nx + (x - g.nb) : 0;
    W[j] = ok[j] ? a.wp[sidx2(g, z, x)] : 0.f;
    const int dz = ok[j] ? sponge_depth(z, g.nb, g.nz) : 0;
    const float damp = g.eta_scale * (float)(dz * dz + dx * dx);
    C1[j] = 1.f / (1.f + damp);
    C2[j] = (1.f - damp) * C1[j];
    P[j] = (MODE == kBorn && in[j]) ? a.pm[midx[j]] : 0.f;
    acc[j] = 0.f;
  }
  if (MODE == kAdjoint)
    for (int i = tid; i < TZ * TX; i += NT) inj[i] = 0.f;

  const int s0 = grp * a.per_block;
  const int s1 = min(s0 + a.per_block, a.nshots);
  int prev = -1;
  for (int s = s0; s < s1; ++s) {
    const ShotDev sd = a.tab[s];
    const bool active =
        (MODE == kAdjoint) ? (a.n <= sd.nt - 1) : (a.n < sd.nt - 1);
    if (!active) continue;  // uniform across the block
    const int lin = (MODE == kAdjoint) ? a.n + 1 : a.n;
    const float* __restrict__ uin = (lin & 1) ? sd.u1 : sd.u0;
    float* __restrict__ uout = (lin & 1) ? sd.u0 : sd.u1;
    __syncthreads();  // previous shot done with tile[] and inj[]
    if (MODE == kAdjoint && prev >= 0) {
      const ShotDev pd = a.tab[prev];
      for (int e = pd.rptr[t] + tid; e < pd.rptr[t + 1]; e += NT)
        inj[pd.rent[e].x] = 0.f;
    }
    for (int r = ty; r < LZ; r += NTZ) {
      const float* row = uin + sidx2(g, z0 - kRadius + r, x0);
      tile[r * LX + kRadius + tx] = row[tx];
      if (tx < 2 * kRadius) {
        const int c = tx < kRadius ? tx - kRadius : TX + tx - kRadius;
        tile[r * LX + kRadius + c] = row[c];
      }
    }
    __syncthreads();
    if (MODE == kBorn) {  // d^n = du^n at the receivers of this tile
      for (int e = sd.rptr[t] + tid; e < sd.rptr[t + 1]; e += NT) {
        const int2 re = sd.rent[e];
        const int lz = re.x / TX, lx = re.x - (re.x / TX) * TX;
        a.dat[sd.dat_off + (int64_t)a.n * sd.nrec + re.y] =
            tile[(lz + kRadius) * LX + lx + kRadius];
      }
    }
    if (MODE == kAdjoint) {  // R^T r^k
      for (int e = sd.rptr[t] + tid; e < sd.rptr[t + 1]; e += NT) {
        const int2 re = sd.rent[e];
        atomicAdd(&inj[re.x],
                  a.dat[sd.dat_off + (int64_t)a.n * sd.nrec + re.y]);
      }
      __syncthreads();
    }
    float col[PZ + 2 * kRadius];
#pragma unroll
    for (int i = 0; i < PZ + 2 * kRadius; ++i)
      col[i] = tile[(ty * PZ + i) * LX + kRadius + tx];
#pragma unroll
    for (int j = 0; j < PZ; ++j) {
      if (!ok[j]) continue;
      const int z = zb + j;
      const float c = col[j + kRadius];
      const float* rw = &tile[(ty * PZ + j + kRadius) * LX + kRadius + tx];
      // L u on differences, smallest weights first
      float lap = g.w.c4 * (((col[j + 8] - c) + (col[j] - c)) +
                            ((rw[4] - c) + (rw[-4] - c)));
      lap = fmaf(g.w.c3, ((col[j + 7] - c) + (col[j + 1] - c)) +
                             ((rw[3] - c) + (rw[-3] - c)),
                 lap);
      lap = fmaf(g.w.c2, ((col[j + 6] - c) + (col[j + 2] - c)) +
                             ((rw[2] - c) + (rw[-2] - c)),
                 lap);
      lap = fmaf(g.w.c1, ((col[j + 5] - c) + (col[j + 3] - c)) +
                             ((rw[1] - c) + (rw[-1] - c)),
                 lap);
      float inc;
      if (MODE == kBackground) {
        const float src =
            (z == sd.src_z && x == sd.src_x) ? sd.wav[a.n] : 0.f;
        inc = W[j] * (lap + src);
        if (in[j]) sd.d2[(int64_t)a.n * mplane + midx[j]] = inc;
      } else if (MODE == kBorn) {
        inc = W[j] * lap;
        if (in[j])
          inc = fmaf(-P[j], sd.d2[(int64_t)a.n * mplane + midx[j]], inc);
      } else {
        inc = W[j] * (lap + inj[(ty * PZ + j) * TX + tx]);
      }
      const int64_t si = sidx2(g, z, x);
      const float vn = fmaf(C2[j], sd.v[si], C1[j] * inc);
      sd.v[si] = vn;
      const float un = c + vn;
      uout[si] = un;
      if (MODE == kAdjoint && in[j])
        acc[j] = fmaf(-sd.d2[(int64_t)(a.n - 1) * mplane + midx[j]], un,
                      acc[j]);
    }
    prev = s;
  }
  if (MODE == kAdjoint && prev >= 0) {
    double* out = a.acc + (int64_t)grp * mplane;
#pragma unroll
    for (int j = 0; j < PZ; ++j)
      if (in[j]) out[midx[j]] += (double)acc[j];
  }
}

// Last sample of the Born data, d^{nt-1} = du^{nt-1} at the receivers.
__global__ void k_born_last(const ShotDev* tab, int nshots, float* dat) {
  const int s = blockIdx.y;
  if (s >= nshots) return;
  const ShotDev sd = tab[s];
  const int lvl = sd.nt - 1;
  const float* u = (lvl & 1) ? sd.u1 : sd.u0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < sd.nrec;
       j += gridDim.x * blockDim.x)
    dat[sd.dat_off + (int64_t)lvl * sd.nrec + j] = u[sd.rsidx[j]];
}

// Image = (sum over accumulators) / W' on the model region.
__global__ void k_adj_finalize(const double* acc, int ngroups, Geo2D g,
                               const float* wp, float* out) {
  const int64_t mplane = (int64_t)g.nz * g.nx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mplane;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < ngroups; ++k) s += acc[(int64_t)k * mplane + i];
    const int z = (int)(i / g.nx), x = (int)(i - (int64_t)(i / g.nx) * g.nx);
    out[i] = (float)(s / (double)wp[sidx2(g, z + g.nb, x + g.nb)]);
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static const TileShape kShapes[] = {
    {64, 16, 4}, {64, 32, 4}, {64, 8, 2}, {128, 16, 2}, {32, 32, 8},
    {64, 32, 8},
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int tile_shape_count() { return kNumShapes; }
TileShape tile_shape(int v) { return kShapes[v]; }

template <int TX, int TZ, int NTZ>
static hipError_t launch_shape(int mode, const StepArgs& a,
                               hipStream_t st) {
  const dim3 block(TX, NTZ);
  const dim3 grid(a.g.ntiles * a.ngroups);
  switch (mode) {
    case kBackground:
      hipLaunchKernelGGL((k_step2d<TX, TZ, NTZ, kBackground>), grid, block, 0,
                         st, a);
      break;
    case kBorn:
      hipLaunchKernelGGL((k_step2d<TX, TZ, NTZ, kBorn>), grid, block, 0, st,
                         a);
      break;
    default:
      hipLaunchKernelGGL((k_step2d<TX, TZ, NTZ, kAdjoint>), grid, block, 0,
                         st, a);
  }
  return hipGetLastError();
}

hipError_t launch_step2d(int variant, int mode, const StepArgs& a,
                         hipStream_t st) {
  switch (variant) {
    case 0: return launch_shape<64, 16, 4>(mode, a, st);
    case 1: return launch_shape<64, 32, 4>(mode, a, st);
    case 2: return launch_shape<64, 8, 2>(mode, a, st);
    case 3: return launch_shape<128, 16, 2>(mode, a, st);
    case 4: return launch_shape<32, 32, 8>(mode, a, st);
    case 5: return launch_shape<64, 32, 8>(mode, a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_born_last(const ShotDev* tab, int nshots, int nrec_max,
                            float* dat, hipStream_t st) {
  const dim3 grid((nrec_max + 255) / 256, nshots);
  hipLaunchKernelGGL(k_born_last, grid, dim3(256), 0, st, tab, nshots, dat);
  return hipGetLastError();
}

hipError_t launch_adj_finalize(const double* acc, int ngroups,
                               const Geo2D& g, const float* wp, float* out,
                               hipStream_t st) {
  const int64_t m = (int64_t)g.nz * g.nx;
  int blocks = (int)((m + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_adj_finalize, dim3(blocks), dim3(256), 0, st, acc,
                     ngroups, g, wp, out);
  return hipGetLastError();
}

}  // namespace brls
