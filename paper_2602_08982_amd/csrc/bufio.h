// Vector-memory buffer loads / stores with a wave-uniform base (buffer
// resource in SGPRs), a wave-uniform byte offset (SGPR) and one per-lane
// byte offset (VGPR).  A line of a state is then addressed by the lane's
// column offset plus a scalar row offset, instead of one 64-bit VGPR
// address per element, which keeps the in-register transforms from
// spilling.  Accesses beyond the resource size return zero (loads) or are
// dropped (stores) by the hardware range check.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "fft.h"

namespace tdslda {

typedef int bi32x4 __attribute__((ext_vector_type(4)));
typedef int bi32x2 __attribute__((ext_vector_type(2)));

__device__ bi32x4 tds_raw_load_b128(bi32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.v4i32");
__device__ bi32x2 tds_raw_load_b64(bi32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.v2i32");
__device__ int tds_raw_load_b32(bi32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.load.i32");
__device__ void tds_raw_store_b128(bi32x4 v, bi32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.store.v4i32");
__device__ void tds_raw_store_b64(bi32x2 v, bi32x4 rsrc, int voff, int soff, int aux) __asm("llvm.amdgcn.raw.buffer.store.v2i32");

// Cache-policy operand of a streaming access (data read or written once per
// pass): the non-temporal hint, so that lines that are re-read within the
// pass (phi re-read at the end of the fused pass, the per-site fields read
// by every state) keep their place in L2 and the last-level cache.
#ifndef TDSLDA_NT_AUX
#define TDSLDA_NT_AUX 2
#endif
constexpr int kStream = TDSLDA_NT_AUX;

// Buffer resource over [p, p + bytes); p must be wave-uniform.
__device__ __forceinline__ bi32x4 make_rsrc(const void* p, uint32_t bytes) {
  const uint64_t a = (uint64_t)p;
  bi32x4 r;
  r.x = __builtin_amdgcn_readfirstlane((int)(a & 0xffffffffu));
  r.y = __builtin_amdgcn_readfirstlane((int)(a >> 32));  // stride 0
  r.z = (int)bytes;                                       // range in bytes
  r.w = 0x00020000;                                       // raw 32-bit data format
  return r;
}

template <typename R, int AUX = 0>
__device__ __forceinline__ cpx<R> bload(bi32x4 rs, int voff, int soff) {
  cpx<R> c;
  if constexpr (sizeof(R) == 8) {
    bi32x4 v = tds_raw_load_b128(rs, voff, soff, AUX);
    __builtin_memcpy(&c, &v, 16);
  } else {
    bi32x2 v = tds_raw_load_b64(rs, voff, soff, AUX);
    __builtin_memcpy(&c, &v, 8);
  }
  return c;
}

// Stores take the scalar offset through the lane offset and pass a zero
// soffset: a 128-bit store whose soffset is an SGPR is not protected by the
// compiler's store-data hazard handling (a VALU write of the data VGPRs right
// after the store), and on gfx950 such stores have been seen to commit the
// overwritten value for some lanes.  With an immediate soffset the compiler
// inserts the required wait state.
template <typename R, int AUX = 0>
__device__ __forceinline__ void bstore(cpx<R> c, bi32x4 rs, int voff, int soff) {
  if constexpr (sizeof(R) == 8) {
    bi32x4 v;
    __builtin_memcpy(&v, &c, 16);
    tds_raw_store_b128(v, rs, voff + soff, 0, AUX);
  } else {
    bi32x2 v;
    __builtin_memcpy(&v, &c, 8);
    tds_raw_store_b64(v, rs, voff + soff, 0, AUX);
  }
}

// real scalar of R
template <typename R>
__device__ __forceinline__ cpx<R> bload_nt(bi32x4 rs, int voff, int soff) {
  return bload<R, kStream>(rs, voff, soff);
}
template <typename R>
__device__ __forceinline__ void bstore_nt(cpx<R> c, bi32x4 rs, int voff, int soff) {
  bstore<R, kStream>(c, rs, voff, soff);
}

// streaming load through a plain pointer
template <typename R>
__device__ __forceinline__ cpx<R> ld_stream(const cpx<R>* p) {
  if constexpr (kStream == 0) {
    return *p;
  } else if constexpr (sizeof(R) == 8) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return cpx<R>{v.x, v.y};
  } else {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return cpx<R>{v.x, v.y};
  }
}

template <typename R>
__device__ __forceinline__ R bload_real(bi32x4 rs, int voff, int soff) {
  R r;
  if constexpr (sizeof(R) == 8) {
    bi32x2 v = tds_raw_load_b64(rs, voff, soff, 0);
    __builtin_memcpy(&r, &v, 8);
  } else {
    int v = tds_raw_load_b32(rs, voff, soff, 0);
    __builtin_memcpy(&r, &v, 4);
  }
  return r;
}

}  // namespace tdslda
