// Workgroup-uniform base pointers with 32-bit per-thread byte offsets.
//
// A load p[off] whose base p is the same for the whole workgroup and whose
// offset is a 32-bit byte count can use the global-memory form with the base
// in scalar registers and only the offset in a vector register.  The compiler
// otherwise folds uniform level offsets and per-thread offsets into one
// 64-bit per-thread address, which costs a 64-bit vector add per access.
// uniform_ptr() hides the base from that folding (readfirstlane of a value
// that is already uniform is a scalar move); at() indexes it by bytes.
// Callers guarantee that every offset they pass fits in 32 bits (fields of
// fewer than 2^32 bytes).
#pragma once

namespace oc {

template <class T>
using global_ptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ inline global_ptr<T> uniform_ptr(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (global_ptr<T>)(((unsigned long long)hi << 32) | lo);
}

template <class T>
__device__ inline __attribute__((address_space(1))) T& at(global_ptr<T> p, unsigned off) {
  return *(global_ptr<T>)((__attribute__((address_space(1))) char*)p + off);
}

}  // namespace oc
