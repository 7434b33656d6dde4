// Device helpers shared by the 2-D step kernels: global-address-space
// pointers, scalar (wave-uniform) copies of table values, 32-bit element
// offsets, and the sponge depth of a padded index.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

#define GLOBAL __attribute__((address_space(1)))

namespace brls {
namespace dev {

typedef GLOBAL float gfloat;
typedef const GLOBAL float cgfloat;

__device__ __forceinline__ gfloat* G(float* p) { return (gfloat*)p; }
__device__ __forceinline__ cgfloat* G(const float* p) { return (cgfloat*)p; }

// Every value of a shot's table entry is uniform across the block; moving
// them to scalar registers lets global accesses use a scalar base plus a
// 32-bit vector offset instead of 64-bit vector address arithmetic.
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
__device__ __forceinline__ ShotDev shot(const ShotDev* tab, int s) {
  ShotDev d = tab[s];
  for (int k = 0; k < 3; ++k) {
    d.f[k] = uni(d.f[k]);
    d.b[k] = uni(d.b[k]);
  }
  d.f[3] = uni(d.f[3]);
  d.d2 = uni(d.d2);
  d.ck = uni(d.ck);
  d.rptr = uni(d.rptr);
  d.rent = uni(d.rent);
  d.rsidx = uni(d.rsidx);
  d.wav = uni(d.wav);
  d.dat_off = (int64_t)uni((uint64_t)d.dat_off);
  d.nt = uni(d.nt);
  d.nrec = uni(d.nrec);
  d.src_z = uni(d.src_z);
  d.src_x = uni(d.src_x);
  return d;
}

// Element i of a global array, the byte offset formed in 32 bits so the
// access can use a scalar base plus a 32-bit vector offset (every array the
// kernels index this way is below 2^30 elements).
__device__ __forceinline__ cgfloat* at(cgfloat* base, uint32_t i) {
  return (cgfloat*)((const GLOBAL char*)base + (i << 2));
}
__device__ __forceinline__ gfloat* at(gfloat* base, uint32_t i) {
  return (gfloat*)((GLOBAL char*)base + (i << 2));
}

// Cells between padded index i and the model region [nb, nb + n).
__device__ __forceinline__ int sponge_depth(int i, int nb, int n) {
  return i < nb ? nb - i : (i >= nb + n ? i - (nb + n - 1) : 0);
}

// Whether shot s takes part in the step of level n (adjoint: output level).
__device__ __forceinline__ bool active(int mode, int n, int nt) {
  return mode == kAdjoint ? n <= nt - 1 : n < nt - 1;
}

}  // namespace dev
}  // namespace brls
