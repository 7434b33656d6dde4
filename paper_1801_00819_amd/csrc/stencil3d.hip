// 3-D time-step kernels of the Born operator pair (gfx950).
//
// Same scheme and modes as the 2-D kernels (see stencil2d.hip and
// layout.h): 8th-order Laplacian on differences, difference-form time
// update, sponge damping, Born source from the background's increment.
//
// Work decomposition: a work item is an XY tile of TX x TY columns, a chunk
// of consecutive z planes, and a group of SB shots. The block marches up the
// chunk plane by plane. Each thread keeps, per shot, a register queue of the
// 9 values of its column around the current plane (the z-derivative), and
// the current plane of every shot in the group is staged in LDS with a 4-cell
// ring (the x- and y-derivatives), so one pair of barriers serves all SB
// shots of a plane. The medium and the model vector are read once per point
// for the whole group, and the adjoint sums the group's image contributions
// in registers before one update of the float64 accumulator. Work items are
// dealt to the 8 XCDs in contiguous ranges (neighbouring tiles share halos
// through an XCD's L2).
//
// Receivers: per shot, a CSR list over (XY tile, padded z plane), entries
// (local index ly * TX + lx, receiver index).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "layout.h"

#define GLOBAL __attribute__((address_space(1)))

namespace brls {

namespace {

typedef GLOBAL float gfloat;
typedef const GLOBAL float cgfloat;

__device__ __forceinline__ gfloat* G(float* p) { return (gfloat*)p; }
__device__ __forceinline__ cgfloat* G(const float* p) { return (cgfloat*)p; }
__device__ __forceinline__ cgfloat* at(cgfloat* base, uint32_t i) {
  return (cgfloat*)((const GLOBAL char*)base + (i << 2));
}
__device__ __forceinline__ gfloat* at(gfloat* base, uint32_t i) {
  return (gfloat*)((GLOBAL char*)base + (i << 2));
}
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int uni(int v) {
  return (int)__builtin_amdgcn_readfirstlane((uint32_t)v);
}
__device__ __forceinline__ uint64_t uni(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
template <class T>
__device__ __forceinline__ T* uni(T* p) {
  return (T*)(uintptr_t)uni((uint64_t)(uintptr_t)p);
}
__device__ __forceinline__ int sponge_depth(int i, int nb, int n) {
  return i < nb ? nb - i : (i >= nb + n ? i - (nb + n - 1) : 0);
}

// Uniform per-shot values a 3-D step needs, held in scalar registers.
struct Shot3 {
  cgfloat* uin;   // level being read
  gfloat* uout;   // level being written
  gfloat* v;
  cgfloat* bin;   // background, level n
  gfloat* bout;   // background, level n + 1
  gfloat* bv;
  gfloat* d2;     // frame of this step
  const int* rptr;
  const int2* rent;
  const float* wav;
  int64_t dat_off;
  int nrec;
  int sz, sy, sx;
  int active;
};

template <int MODE>
__device__ __forceinline__ Shot3 load_shot(const StepArgs& a, int s,
                                           uint32_t mplane) {
  Shot3 r{};
  if (s >= a.nshots) {
    r.active = 0;
    return r;
  }
  const ShotDev d = a.tab[s];
  const int nt = uni(d.nt);
  r.active = (MODE == kAdjoint) ? (a.n <= nt - 1) : (a.n < nt - 1);
  const int lin = (MODE == kAdjoint) ? a.n + 1 : a.n;
  r.uin = G(uni((lin & 1) ? d.f[1] : d.f[0]));
  r.uout = G(uni((lin & 1) ? d.f[0] : d.f[1]));
  r.v = G(uni(d.f[2]));
  r.bin = G(uni((a.n & 1) ? d.b[1] : d.b[0]));
  r.bout = G(uni((a.n & 1) ? d.b[0] : d.b[1]));
  r.bv = G(uni(d.b[2]));
  const int fr = (MODE == kAdjoint ? a.n - 1 : a.n) - a.d2_n0;
  r.d2 = G(uni(d.d2)) + (int64_t)fr * mplane;
  r.rptr = uni(d.rptr);
  r.rent = uni(d.rent);
  r.wav = uni(d.wav);
  r.dat_off = (int64_t)uni((uint64_t)d.dat_off);
  r.nrec = uni(d.nrec);
  r.sz = uni(d.src_z);
  r.sy = uni(d.src_y);
  r.sx = uni(d.src_x);
  return r;
}

// Halo ring of one plane (no corners: the stencil is axis-aligned): 4 rows
// above and below the tile (TX wide) and 4 columns left and right (TY high).
template <int TX, int TY>
__device__ __forceinline__ void halo_cell(int h, int& ly, int& lx) {
  if (h < 4 * TX) {
    ly = h / TX - 4;
    lx = h % TX;
  } else if (h < 8 * TX) {
    ly = TY + (h - 4 * TX) / TX;
    lx = (h - 4 * TX) % TX;
  } else if (h < 8 * TX + 4 * TY) {
    ly = (h - 8 * TX) / 4;
    lx = (h - 8 * TX) % 4 - 4;
  } else {
    ly = (h - 8 * TX - 4 * TY) / 4;
    lx = TX + (h - 8 * TX - 4 * TY) % 4;
  }
}

// x + y part of h^2 L at the thread's point (centre c) from an LDS plane.
template <int LX>
__device__ __forceinline__ float lap_xy(const StencilW& w, const float* p,
                                        float c) {
  float l = w.c4 * (((p[4] - c) + (p[-4] - c)) +
                    ((p[4 * LX] - c) + (p[-4 * LX] - c)));
  l = fmaf(w.c3, ((p[3] - c) + (p[-3] - c)) +
                     ((p[3 * LX] - c) + (p[-3 * LX] - c)),
           l);
  l = fmaf(w.c2, ((p[2] - c) + (p[-2] - c)) +
                     ((p[2 * LX] - c) + (p[-2 * LX] - c)),
           l);
  l = fmaf(w.c1, ((p[1] - c) + (p[-1] - c)) + ((p[LX] - c) + (p[-LX] - c)),
           l);
  return l;
}

// z part of h^2 L from the register queue (centre at q[4]).
__device__ __forceinline__ float lap_z(const StencilW& w, const float (&q)[9]) {
  const float c = q[4];
  float l = w.c4 * ((q[8] - c) + (q[0] - c));
  l = fmaf(w.c3, (q[7] - c) + (q[1] - c), l);
  l = fmaf(w.c2, (q[6] - c) + (q[2] - c), l);
  l = fmaf(w.c1, (q[5] - c) + (q[3] - c), l);
  return l;
}

template <int TX, int TY, int SB, int MODE, bool INT>
__device__ __forceinline__ void march(const StepArgs& a, int txy, int zc,
                                      int grp, float* pl, float* bpl,
                                      float* inj) {
  constexpr int NT = TX * TY;
  constexpr int LX = TX + 2 * kRadius;
  constexpr int LY = TY + 2 * kRadius;
  constexpr int PL = LX * LY;
  constexpr int H = 8 * TX + 8 * TY;
  constexpr int HR = (H + NT - 1) / NT;
  constexpr bool BG = (MODE == kBackground || MODE == kBornFused);
  constexpr bool FF = (MODE != kBackground);
  const Geo3D& g = a.g3;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int tyi = txy / g.ntx, txi = txy - tyi * g.ntx;
  const int x0 = g.x_org + txi * TX, y0 = tyi * TY;
  const int x = x0 + tx, y = y0 + ty;
  const int z0 = zc * g.tzc, z1 = min(z0 + g.tzc, g.pz);
  const uint32_t plane = (uint32_t)g.plane, pitch = (uint32_t)g.pitch;
  const uint32_t mplane = (uint32_t)g.nz * g.ny * g.nx;
  const uint32_t mrow = (uint32_t)g.nx, mpl = (uint32_t)g.ny * g.nx;
  const bool colok = x >= 0 && x < g.px && y < g.py;
  const bool colint = x >= g.nb && x < g.nb + g.nx && y >= g.nb &&
                      y < g.nb + g.ny;
  const int dxy = colok ? sponge_depth(x, g.nb, g.nx) * sponge_depth(x, g.nb, g.nx) +
                              sponge_depth(y, g.nb, g.ny) * sponge_depth(y, g.nb, g.ny)
                        : 0;
  // storage offset of (z, y, x) = so_col + (z + 4) * plane
  const uint32_t so_col = (uint32_t)(y + kGhost) * pitch + (uint32_t)(x + g.xoff);
  const uint32_t mo_col = (uint32_t)(y - g.nb) * mrow + (uint32_t)(x - g.nb);
  // halo cells this thread stages, as offsets within a plane
  uint32_t hso[HR];
  int hlds[HR];
  bool hv[HR];
#pragma unroll
  for (int k = 0; k < HR; ++k) {
    const int h = tid + k * NT;
    int ly = 0, lx = 0;
    hv[k] = h < H;
    if (hv[k]) halo_cell<TX, TY>(h, ly, lx);
    hso[k] = (uint32_t)(y0 + ly + kGhost) * pitch + (uint32_t)(x0 + lx + g.xoff);
    hlds[k] = (ly + kRadius) * LX + lx + kRadius;
  }
  const int cl = (ty + kRadius) * LX + tx + kRadius;  // my LDS cell

  Shot3 sh[SB];
  bool any = false;
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    sh[j] = load_shot<MODE>(a, grp * SB + j, mplane);
    any |= (bool)sh[j].active;
  }
  if (!any) return;  // uniform

  float q[SB][9], qb[SB][9];
#pragma unroll
  for (int j = 0; j < SB; ++j)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t so = so_col + (uint32_t)(z0 - kRadius + i + kGhost) * plane;
      q[j][i] = (FF && sh[j].active) ? *at(sh[j].uin, so) : 0.f;
      qb[j][i] = (BG && sh[j].active) ? *at(sh[j].bin, so) : 0.f;
    }
  for (int z = z0; z < z1; ++z) {
    const uint32_t so = so_col + (uint32_t)(z + kGhost) * plane;
    const uint32_t mo = mo_col + (uint32_t)(z - g.nb) * mpl;
    const bool ok = INT || (colok && z < g.pz);
    const bool in = INT || (colint && z >= g.nb && z < g.nb + g.nz);
    // --- global loads of this plane, issued together ---
    float vold[SB], bvold[SB], d2v[SB], hval[SB][HR], hbval[SB][HR];
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      const uint32_t so4 = so + 4 * plane;
      q[j][8] = (FF && sh[j].active) ? *at(sh[j].uin, so4) : 0.f;
      qb[j][8] = (BG && sh[j].active) ? *at(sh[j].bin, so4) : 0.f;
      vold[j] = (FF && sh[j].active) ? *at(sh[j].v, so) : 0.f;
      bvold[j] = (BG && sh[j].active) ? *at(sh[j].bv, so) : 0.f;
      d2v[j] = ((MODE == kBorn || MODE == kAdjoint) && sh[j].active && in)
                   ? __builtin_nontemporal_load(at(sh[j].d2, mo))
                   : 0.f;
      const uint32_t zoff = (uint32_t)(z + kGhost) * plane;
#pragma unroll
      for (int k = 0; k < HR; ++k) {
        hval[j][k] = (FF && sh[j].active && hv[k]) ? *at(sh[j].uin, zoff + hso[k])
                                                   : 0.f;
        hbval[j][k] = (BG && sh[j].active && hv[k])
                          ? *at(sh[j].bin, zoff + hso[k])
                          : 0.f;
      }
    }
    float W = 0.f, C1 = 1.f, C2 = 1.f, P = 0.f;
    W = ok ? *at(G(a.wp), so) : 0.f;
    if (!INT) {
      const int dz = ok ? sponge_depth(z, g.nb, g.nz) : 0;
      const float damp = g.eta_scale * (float)(dz * dz + dxy);
      C1 = __builtin_amdgcn_rcpf(1.f + damp);
      C2 = (1.f - damp) * C1;
    }
    if ((MODE == kBorn || MODE == kBornFused) && in) P = *at(G(a.pm), mo);
    __syncthreads();  // previous plane done with the LDS arrays
    if (MODE == kAdjoint && z > z0) {  // clear the previous plane's injections
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        if (!sh[j].active) continue;
        const int r0 = sh[j].rptr[txy * g.pz + z - 1];
        const int r1 = sh[j].rptr[txy * g.pz + z];
        for (int e = r0 + tid; e < r1; e += NT) inj[j * TX * TY + sh[j].rent[e].x] = 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      if (FF) {
        pl[j * PL + cl] = q[j][4];
#pragma unroll
        for (int k = 0; k < HR; ++k)
          if (hv[k]) pl[j * PL + hlds[k]] = hval[j][k];
      }
      if (BG) {
        bpl[j * PL + cl] = qb[j][4];
#pragma unroll
        for (int k = 0; k < HR; ++k)
          if (hv[k]) bpl[j * PL + hlds[k]] = hbval[j][k];
      }
    }
    __syncthreads();
    if (MODE == kBorn || MODE == kBornFused || MODE == kAdjoint) {
      bool inj_any = false;
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        if (!sh[j].active) continue;
        const int r0 = sh[j].rptr[txy * g.pz + z];
        const int r1 = sh[j].rptr[txy * g.pz + z + 1];
        if (r1 > r0) inj_any = true;
        for (int e = r0 + tid; e < r1; e += NT) {
          const int2 re = sh[j].rent[e];
          const int ly = re.x / TX, lx = re.x - ly * TX;
          if (MODE == kAdjoint) {
            cgfloat* res = G(a.dat) + sh[j].dat_off + (int64_t)a.n * sh[j].nrec;
            atomicAdd(&inj[j * TX * TY + re.x], res[re.y]);
          } else {
            gfloat* dat = G(a.dat) + sh[j].dat_off + (int64_t)a.n * sh[j].nrec;
            dat[re.y] = pl[j * PL + (ly + kRadius) * LX + lx + kRadius];
          }
        }
      }
      if (MODE == kAdjoint && inj_any) __syncthreads();
    }
    // --- compute ---
    float accs = 0.f;
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      if (!sh[j].active) continue;
      float srcv = 0.f;
      if (BG) {
        const float src = (z == sh[j].sz && y == sh[j].sy && x == sh[j].sx)
                              ? sh[j].wav[a.n]
                              : 0.f;
        const float lb = lap_z(g.w, qb[j]) + lap_xy<LX>(g.w, &bpl[j * PL + cl], qb[j][4]);
        const float incb = W * (lb + src);
        const float vb = INT ? bvold[j] + incb : fmaf(C2, bvold[j], C1 * incb);
        if (ok) {
          *at(sh[j].bv, so) = vb;
          *at(sh[j].bout, so) = qb[j][4] + vb;
        }
        srcv = incb;
        if (MODE == kBackground && a.write_d2 && in)
          __builtin_nontemporal_store(incb, at(sh[j].d2, mo));
      }
      if (MODE == kBackground) continue;
      const float lap = lap_z(g.w, q[j]) + lap_xy<LX>(g.w, &pl[j * PL + cl], q[j][4]);
      float inc;
      if (MODE == kBorn) {
        inc = W * lap;
        if (in) inc = fmaf(-P, d2v[j], inc);
      } else if (MODE == kBornFused) {
        inc = fmaf(-P, srcv, W * lap);
      } else {
        inc = W * (lap + inj[j * TX * TY + ty * TX + tx]);
      }
      const float vn = INT ? vold[j] + inc : fmaf(C2, vold[j], C1 * inc);
      const float un = q[j][4] + vn;
      if (ok) {
        *at(sh[j].v, so) = vn;
        *at(sh[j].uout, so) = un;
      }
      if (MODE == kAdjoint) accs = fmaf(-d2v[j], un, accs);
    }
    if (MODE == kAdjoint && in)
      a.acc[(int64_t)grp * mplane + mo] += (double)accs;
    // advance the queues
#pragma unroll
    for (int j = 0; j < SB; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        q[j][i] = q[j][i + 1];
        qb[j][i] = qb[j][i + 1];
      }
  }
  if (MODE == kAdjoint) {  // clear the last plane's injections
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      if (!sh[j].active) continue;
      const int r0 = sh[j].rptr[txy * g.pz + z1 - 1];
      const int r1 = sh[j].rptr[txy * g.pz + z1];
      for (int e = r0 + tid; e < r1; e += NT) inj[j * TX * TY + sh[j].rent[e].x] = 0.f;
    }
  }
}

}  // namespace

template <int TX, int TY, int SB, int MODE>
__global__ void __launch_bounds__(TX* TY) k_step3d(StepArgs a) {
  constexpr int PL = (TX + 2 * kRadius) * (TY + 2 * kRadius);
  constexpr bool BG = (MODE == kBackground || MODE == kBornFused);
  __shared__ float pl[MODE == kBackground ? 1 : SB * PL];
  __shared__ float bpl[BG ? SB * PL : 1];
  __shared__ float inj[MODE == kAdjoint ? SB * TX * TY : 1];
  const Geo3D& g = a.g3;
  if (MODE == kAdjoint)
    for (int i = threadIdx.y * TX + threadIdx.x; i < SB * TX * TY; i += TX * TY)
      inj[i] = 0.f;
  const int ntxy = g.ntx * g.nty;
  const int items = g.ntiles * a.ngroups;
  const int xcd = blockIdx.x & 7;
  const int nbx = gridDim.x >> 3;
  const int q = items >> 3, r = items & 7;
  const int lo = xcd * q + min(xcd, r);
  const int hi = lo + q + (xcd < r ? 1 : 0);
  for (int L = lo + (int)(blockIdx.x >> 3); L < hi; L += nbx) {
    const int grp = L / g.ntiles;
    const int rem = L - grp * g.ntiles;
    const int zc = rem / ntxy;
    const int txy = rem - zc * ntxy;
    const int tyi = txy / g.ntx, txi = txy - tyi * g.ntx;
    const int x0 = g.x_org + txi * TX, y0 = tyi * TY, z0 = zc * g.tzc;
    const bool interior = x0 >= g.nb && x0 + TX <= g.nb + g.nx &&
                          y0 >= g.nb && y0 + TY <= g.nb + g.ny &&
                          z0 >= g.nb && z0 + g.tzc <= g.nb + g.nz;
    if (interior)
      march<TX, TY, SB, MODE, true>(a, txy, zc, grp, pl, bpl, inj);
    else
      march<TX, TY, SB, MODE, false>(a, txy, zc, grp, pl, bpl, inj);
  }
}

// Image = (sum over accumulators) / W' on the model region (3-D).
__global__ void k_adj_finalize3(const double* acc, int ngroups, Geo3D g,
                                const float* wp, float* out, double* out64) {
  const int64_t m = (int64_t)g.nz * g.ny * g.nx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < ngroups; ++k) s += acc[(int64_t)k * m + i];
    const int z = (int)(i / ((int64_t)g.ny * g.nx));
    const int rem = (int)(i - (int64_t)z * g.ny * g.nx);
    const int y = rem / g.nx, x = rem - (rem / g.nx) * g.nx;
    const double v = s / (double)wp[sidx3(g, z + g.nb, y + g.nb, x + g.nb)];
    out[i] = (float)v;
    if (out64) out64[i] = v;
  }
}

static const TileShape3 kShapes3[] = {
    {32, 8, 1}, {32, 8, 2}, {32, 8, 4}, {64, 4, 2},
    {64, 4, 4}, {32, 4, 4}, {64, 8, 1}, {64, 8, 2},
};
constexpr int kNumShapes3 = sizeof(kShapes3) / sizeof(kShapes3[0]);

int tile_shape3_count() { return kNumShapes3; }
TileShape3 tile_shape3(int v) { return kShapes3[v]; }

static int resident_blocks3(const void* kernel, int threads) {
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

template <int TX, int TY, int SB, int MODE>
static hipError_t launch3_mode(const StepArgs& a, hipStream_t st) {
  static const int cap = resident_blocks3(
      reinterpret_cast<const void*>(&k_step3d<TX, TY, SB, MODE>), TX * TY);
  const int items = a.g3.ntiles * a.ngroups;
  const int lim = (a.resident_grid & 1) ? cap : items;
  const int nblk = ((items < lim ? items : lim) + 7) / 8 * 8;
  hipLaunchKernelGGL((k_step3d<TX, TY, SB, MODE>), dim3(nblk), dim3(TX, TY),
                     0, st, a);
  return hipGetLastError();
}

template <int TX, int TY, int SB>
static hipError_t launch3_shape(int mode, const StepArgs& a, hipStream_t st) {
  switch (mode) {
    case kBackground: return launch3_mode<TX, TY, SB, kBackground>(a, st);
    case kBorn: return launch3_mode<TX, TY, SB, kBorn>(a, st);
    case kBornFused: return launch3_mode<TX, TY, SB, kBornFused>(a, st);
    default: return launch3_mode<TX, TY, SB, kAdjoint>(a, st);
  }
}

hipError_t launch_step3d(int variant, int mode, const StepArgs& a,
                         hipStream_t st) {
  switch (variant) {
    case 0: return launch3_shape<32, 8, 1>(mode, a, st);
    case 1: return launch3_shape<32, 8, 2>(mode, a, st);
    case 2: return launch3_shape<32, 8, 4>(mode, a, st);
    case 3: return launch3_shape<64, 4, 2>(mode, a, st);
    case 4: return launch3_shape<64, 4, 4>(mode, a, st);
    case 5: return launch3_shape<32, 4, 4>(mode, a, st);
    case 6: return launch3_shape<64, 8, 1>(mode, a, st);
    case 7: return launch3_shape<64, 8, 2>(mode, a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj_finalize3(const double* acc, int ngroups,
                                const Geo3D& g, const float* wp, float* out,
                                double* out64, hipStream_t st) {
  const int64_t m = (int64_t)g.nz * g.ny * g.nx;
  int blocks = (int)((m + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_adj_finalize3, dim3(blocks), dim3(256), 0, st, acc,
                     ngroups, g, wp, out, out64);
  return hipGetLastError();
}

}  // namespace brls
