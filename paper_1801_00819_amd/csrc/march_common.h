// Building blocks of the z-marching 2-D kernels (march2d.hip, march2t.hip):
// DPP lane shifts for the x-stencil, the radius-4 Laplacian on differences,
// buffer accesses with scalar row offsets, and an optimisation barrier for
// rolling row offsets.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace brls {
namespace march {

constexpr int kLanes = 64;
constexpr int kWaves = 4;  // independent wavefronts per block

// DPP controls (GFX9 encodings): wave_shr:1 / wave_shl:1 move a value one
// lane up / down the wavefront; quad_perm picks within groups of 4 lanes.
constexpr int kWaveShr1 = 0x138;
constexpr int kWaveShl1 = 0x130;
constexpr int quad_perm(int a, int b, int c, int d) {
  return a | (b << 2) | (c << 4) | (d << 6);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v, float fill) {
  return __int_as_float(__builtin_amdgcn_update_dpp(
      __float_as_int(fill), __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Neighbours of a point at offsets -1..-4 (m) and +1..+4 (p) along one axis.
struct Nb {
  float m[4], p[4];
};

// x-neighbours of every lane's value c. h holds, in lanes 0..3, the four
// columns left of the strip (x0-4 .. x0-1) and, in lanes 60..63, the four
// right of it (x0+64 .. x0+67). A shift's vacated lane (0 for shr, 63 for
// shl) takes the fill value; the k-th fill needs h[4-k] in lane 0 and
// h[59+k] in lane 63, i.e. quad positions (4-k, k-1), which one quad
// permutation delivers for both edges at once.
__device__ __forceinline__ Nb xnb(float c, float h) {
  const float f1 = dpp<quad_perm(3, 1, 2, 0)>(h, h);
  const float f2 = dpp<quad_perm(2, 1, 2, 1)>(h, h);
  const float f3 = dpp<quad_perm(1, 1, 2, 2)>(h, h);
  const float f4 = h;
  Nb n;
  n.m[0] = dpp<kWaveShr1>(c, f1);
  n.m[1] = dpp<kWaveShr1>(n.m[0], f2);
  n.m[2] = dpp<kWaveShr1>(n.m[1], f3);
  n.m[3] = dpp<kWaveShr1>(n.m[2], f4);
  n.p[0] = dpp<kWaveShl1>(c, f1);
  n.p[1] = dpp<kWaveShl1>(n.p[0], f2);
  n.p[2] = dpp<kWaveShl1>(n.p[1], f3);
  n.p[3] = dpp<kWaveShl1>(n.p[2], f4);
  return n;
}

// A shift whose vacated lane reads zero (bound_ctrl): no old value to copy
// into the destination first.
template <int CTRL>
__device__ __forceinline__ float dpp0(float v) {
  return __int_as_float(
      __builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// x-neighbours for the second step of a two-step kernel, whose results at
// the four lanes on each edge are discarded: plain shifts, no fill values.
__device__ __forceinline__ Nb xnb_inner(float c) {
  Nb n;
  n.m[0] = dpp0<kWaveShr1>(c);
  n.m[1] = dpp0<kWaveShr1>(n.m[0]);
  n.m[2] = dpp0<kWaveShr1>(n.m[1]);
  n.m[3] = dpp0<kWaveShr1>(n.m[2]);
  n.p[0] = dpp0<kWaveShl1>(c);
  n.p[1] = dpp0<kWaveShl1>(n.p[0]);
  n.p[2] = dpp0<kWaveShl1>(n.p[1]);
  n.p[3] = dpp0<kWaveShl1>(n.p[2]);
  return n;
}

// z-neighbours of queue entry q[r] (r compile-time after unrolling).
template <int N>
__device__ __forceinline__ Nb znb(const float (&q)[N], int r) {
  Nb n;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    n.m[k] = q[r - 1 - k];
    n.p[k] = q[r + 1 + k];
  }
  return n;
}

// L u * h^2 on differences, in the order k_step2d uses (largest offset
// first, z pair before x pair).
__device__ __forceinline__ float lap8(const StencilW& w, float c, const Nb& z,
                                      const Nb& x) {
  float lap = w.c4 * (((z.p[3] - c) + (z.m[3] - c)) +
                      ((x.p[3] - c) + (x.m[3] - c)));
  lap = fmaf(w.c3, ((z.p[2] - c) + (z.m[2] - c)) +
                       ((x.p[2] - c) + (x.m[2] - c)),
             lap);
  lap = fmaf(w.c2, ((z.p[1] - c) + (z.m[1] - c)) +
                       ((x.p[1] - c) + (x.m[1] - c)),
             lap);
  lap = fmaf(w.c1, ((z.p[0] - c) + (z.m[0] - c)) +
                       ((x.p[0] - c) + (x.m[0] - c)),
             lap);
  return lap;
}

// Buffer accesses: a resource over an array (base in scalar registers), a
// per-lane byte offset fixed for the item and a wave-uniform byte offset
// that walks the rows, so a row costs one scalar add per stream. No range
// limit is set (every access is in bounds by construction).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, GFX9
constexpr int kNT = 2;                  // non-temporal cache policy
__device__ __forceinline__ Rsrc rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                           -1, kRsrcWord3);
}
template <int AUX = 0>
__device__ __forceinline__ float bload(Rsrc r, int voff, int soff) {
  return __int_as_float(
      __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ void bstore(Rsrc r, int voff, int soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, voff, soff,
                                        AUX);
}

// A wave-uniform value the optimiser must treat as formed here (no
// instruction is emitted): rolling row offsets pass through it so each row's
// offset is made inside the row loop instead of being hoisted out of the
// shot loop as one register per row.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

}  // namespace march
}  // namespace brls
