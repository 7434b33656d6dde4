// Device-side data layout shared by the stencil kernels and the host engine.
//
// Wavefields live on the padded grid (model + nb absorbing cells per face)
// stored with a 4-cell ring of zeros around it, so the radius-4 stencil never
// needs a bounds test: padded point (z, x) sits at
//     (z + 4) * pitch + x + xoff
// where xoff puts the first model column (x = nb) on a 128-byte boundary and
// pitch is a multiple of 32 floats. The ring (and everything outside the
// padded grid) is never written, so it stays zero: the stencil sees u = 0
// outside the padded grid.
//
// Each field is advanced in "difference form": besides u^n the kernels keep
// v^n = u^n - u^{n-1}. The leapfrog update of a damped wave equation
//     u^{n+1} = C1 (2u^n + W L u^n + s^n) - C2 u^{n-1}
// is, exactly, v^{n+1} = C2 v^n + C1 (W L u^n + s^n), u^{n+1} = u^n + v^{n+1}.
// Carrying v instead of u^{n-1}, and evaluating L on differences
// (u[i+k] - u[i]), keeps float32 rounding from being amplified by the small
// (omega dt)^2 of well-sampled waves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace brls {

constexpr int kRadius = 4;
constexpr int kGhost = 4;  // zero ring around the padded grid

// 8th-order central second-derivative weights for offsets 1..4 (the centre
// weight is implied: the difference form needs only these).
struct StencilW {
  float c1, c2, c3, c4;
};

// Per-shot state of a window slot, read by the kernels through a device
// table in window order.
struct ShotDev {
  float* f[4];       // propagated field: u (even levels), u (odd levels), v;
                     // two-step kernels: u and v in sets {f0, f2} and
                     // {f1, f3}, alternating between launches (f3 is null
                     // where the context keeps three fields)
  float* b[3];       // background field (same layout); may alias f
  float* d2;         // Born-source frames [..][model]; frame index n - d2_n0
  float* ck;         // background checkpoints [seg][u | v][field] or null
  const int* rptr;   // receivers per tile: CSR offsets [ntiles + 1]
  const int2* rent;  // (local index lz*TX + lx, receiver index)
  const int* rsidx;  // storage index of each receiver
  const float* wav;  // h^2 * source wavelet [nt]
  int64_t dat_off;   // offset of this shot's [nt][nrec] segment in data vectors
  int nt;
  int nrec;
  int src_z, src_x;  // padded grid position of the source
  int src_y;         // (3-D)
};

struct Geo2D {
  int pz, px;        // padded grid
  int nz, nx, nb;    // model grid, sponge width
  int pitch;         // storage row pitch (floats)
  int xoff;          // storage column of padded x = 0
  int x_org;         // padded x of the first tile column (<= 0)
  int ntx, ntz, ntiles;
  float eta_scale;   // eta_max * dt / 2 / nb^2
  StencilW w;
};

// 3-D grid: padded point (z, y, x) sits at
//     (z + 4) * plane + (y + 4) * pitch + x + xoff
// with the same zero ring of 4 cells on every face.
struct Geo3D {
  int pz, py, px;      // padded grid
  int nz, ny, nx, nb;  // model grid, sponge width
  int pitch;           // storage row pitch (floats)
  int plane;           // storage floats per z-plane
  int xoff;            // storage column of padded x = 0
  int x_org;           // padded x of the first tile column (<= 0)
  int ntx, nty, ntz;   // tiles in x, y; z chunks
  int tzc;             // planes per z chunk
  int ntiles;          // ntx * nty * ntz
  float eta_scale;     // eta_max * dt / 2 / nb^2
  StencilW w;
};

// kBackground: advance the background field b with the source; optionally
//              store its Born source (the increment) as frame n.
// kBorn:       advance f with source -m * frame n.
// kBornFused:  advance b and f together, the Born source taken from b's
//              increment on the fly (no stored frames).
// kAdjoint:    advance f backward (output level n) with the residual
//              injected at the receivers; image += -frame(n-1) * f^n.
enum StepMode { kBackground = 0, kBorn = 1, kAdjoint = 2, kBornFused = 3 };

struct StepArgs {
  Geo2D g;
  Geo3D g3;            // 3-D launches
  const ShotDev* tab;  // shots of this launch
  int nshots;          // shots in tab
  int per_block;       // shots handled by one block (sequentially)
  int ngroups;         // ceil(nshots / per_block)
  int n;               // time level: input level (background, Born) or
                       // output level k (adjoint)
  int d2_n0;           // time level of stored frame 0
  int write_d2;        // background: store frames
  int nsub;            // two-step kernels: time steps in this launch (1, 2)
  int par;             // two-step kernels: field set read (0, 1); the other
                       // is written
  int resident_grid;   // bit 0: launch only as many blocks as fit at once
                       // (each loops over work items), else one block per
                       // item; bit 1: deal work items to blocks in launch
                       // order, else in 8 contiguous per-XCD ranges
  const float* wp;     // W' = v^2 dt^2 / h^2, storage layout
  const float* pm;     // Born: model perturbation [nz][nx]
  float* dat;          // Born: output data base; adjoint: input residual base
  double* acc;         // adjoint: image accumulators [ngroups][nz][nx]
};

__host__ __device__ inline int64_t sidx2(const Geo2D& g, int z, int x) {
  return (int64_t)(z + kGhost) * g.pitch + x + g.xoff;
}

__host__ __device__ inline int64_t sidx3(const Geo3D& g, int z, int y, int x) {
  return (int64_t)(z + kGhost) * g.plane + (int64_t)(y + kGhost) * g.pitch +
         x + g.xoff;
}

}  // namespace brls
