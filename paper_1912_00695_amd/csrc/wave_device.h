// wave_device.h -- device helpers shared by the HIP kernels (element access per
// storage kind, range-checked buffer loads, XCD-aware block order, reductions).
#pragma once
#include "wave_internal.h"

namespace wave {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));

// Global-memory view of a pointer. Every array the kernels address is device
// global memory, but a pointer read from memory (the serving engine's shot
// descriptors) is not known to be, and accesses through it compile to flat
// instructions, which the compiler also has to count as possible LDS traffic:
// each wait for an LDS read then waits for them too (a flat store per plane made
// the batched kernel 13 % slower than the single-shot one on the same tiles).
// (The host pass of the compilation sees these bodies too; there the qualifier
// has no meaning and the view is the plain pointer.)
#if defined(__HIP_DEVICE_COMPILE__)
#define WAVE_GLOBAL_AS __attribute__((address_space(1)))
#else
#define WAVE_GLOBAL_AS
#endif
template <class T>
__device__ __forceinline__ WAVE_GLOBAL_AS T* gmem(T* p) {
  return (WAVE_GLOBAL_AS T*)p;
}

__device__ __forceinline__ float4 ld4(const float* p) {
  const f4v v = *gmem(reinterpret_cast<const f4v*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(float* p, const float4& v) {
  const f4v w = {v.x, v.y, v.z, v.w};
  *gmem(reinterpret_cast<f4v*>(p)) = w;
}
__device__ __forceinline__ float comp(const float4& v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
__device__ __forceinline__ void set_comp(float4& v, int i, float s) {
  if (i == 0) v.x = s; else if (i == 1) v.y = s; else if (i == 2) v.z = s; else v.w = s;
}


// Block id -> logical tile id. Workgroups are dealt round-robin to the 8 XCDs;
// remapping gives each XCD a contiguous run of logical tiles (whole xy-planes
// of consecutive z-chunks), so tiles that exchange halos share one L2.
__device__ __forceinline__ int remap_tile(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7;
  const int xcd = b & 7, k = b >> 3;
  const int base = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
  return base + k;
}

// Element access per storage kind: 4 consecutive values (16- or 8-byte aligned)
// or 1 value, widened to / narrowed from FP32 (round to nearest even). NT selects
// non-temporal loads/stores (streamed once per step, not kept in the caches).
template <bool NT, class V>
__device__ __forceinline__ V vload(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(gmem(p)); else return *gmem(p);
}
template <bool NT, class V>
__device__ __forceinline__ void vstore(V* p, const V& v) {
  if constexpr (NT) __builtin_nontemporal_store(v, gmem(p)); else *gmem(p) = v;
}
// Range-checked buffer loads (the CDNA buffer resource): a lane whose byte offset
// is kOOB, or every lane of a resource with zero records, reads zeros without a
// memory access, so predicated loads need no branch. Each resource is based at
// one plane of one array (offsets stay below 2^31; the host bounds plane bytes).
constexpr unsigned kOOB = 0x80000000u;
constexpr int kBufWord3 = 0x00020000;  // resource word 3 for gfx9-family raw buffers
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int64_t byte_off,
                                                             int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(static_cast<const char*>(base)) + byte_off, (short)0, bytes, kBufWord3);
}
template <bool NT>
__device__ __forceinline__ i4v bload16(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, NT ? 2 : 0);  // aux bit 1: nt
}
template <bool NT>
__device__ __forceinline__ i2v bload8(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, NT ? 2 : 0);
}

// Buffer stores through the same resources: a lane whose offset is kOOB (or any
// lane of a resource with zero records) writes nothing. A store issued on every
// path keeps the compiler's count of outstanding memory operations exact (after a
// store that may have been skipped, a wait for an older load has to assume the
// store was not issued and then also covers loads issued after it). The two-step
// kernel uses them; in the one-step kernel predicated global stores measured ~2 %
// faster on MI355X.
template <bool NT>
__device__ __forceinline__ void bstore16(__amdgpu_buffer_rsrc_t r, unsigned off, const i4v& v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, NT ? 2 : 0);
}
template <bool NT>
__device__ __forceinline__ void bstore8(__amdgpu_buffer_rsrc_t r, unsigned off, const i2v& v) {
  __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, NT ? 2 : 0);
}

template <int ST> struct Store;
// Each kind also exposes its raw 4-value vector (Raw), a raw load (ldr) and the
// widening to FP32 (widen), so that loads issued ahead of their use are not
// followed at once by a conversion that would wait for them.
template <> struct Store<ST_F32> {
  using Raw = f4v;
  __device__ static Raw zero() { return Raw{0.f, 0.f, 0.f, 0.f}; }
  template <bool NT = false>
  __device__ static Raw ldr(const void* b, int64_t i) {
    return vload<NT>(reinterpret_cast<const f4v*>(static_cast<const float*>(b) + i));
  }
  static constexpr int kBytes = 4;
  template <bool NT = false>
  __device__ static Raw ldb(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(Raw, bload16<NT>(r, off));
  }
  template <bool NT = false>
  __device__ static void stb(__amdgpu_buffer_rsrc_t r, unsigned off, const float4& v) {
    const f4v w = {v.x, v.y, v.z, v.w};
    bstore16<NT>(r, off, __builtin_bit_cast(i4v, w));
  }
  __device__ static float4 widen(const Raw& v) { return make_float4(v.x, v.y, v.z, v.w); }
  template <bool NT = false>
  __device__ static float4 ld(const void* b, int64_t i) { return widen(ldr<NT>(b, i)); }
  __device__ static float ld1(const void* b, int64_t i) { return gmem(static_cast<const float*>(b))[i]; }
  template <bool NT = false>
  __device__ static void st(void* b, int64_t i, const float4& v) {
    f4v w;
    w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
    vstore<NT>(reinterpret_cast<f4v*>(static_cast<float*>(b) + i), w);
  }
};
template <> struct Store<ST_F16> {
  using Raw = h4v;
  __device__ static Raw zero() { return Raw{0, 0, 0, 0}; }
  template <bool NT = false>
  __device__ static Raw ldr(const void* b, int64_t i) {
    return vload<NT>(reinterpret_cast<const h4v*>(static_cast<const _Float16*>(b) + i));
  }
  static constexpr int kBytes = 2;
  template <bool NT = false>
  __device__ static Raw ldb(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(Raw, bload8<NT>(r, off));
  }
  template <bool NT = false>
  __device__ static void stb(__amdgpu_buffer_rsrc_t r, unsigned off, const float4& v) {
    h4v h;
    h.x = (_Float16)v.x; h.y = (_Float16)v.y; h.z = (_Float16)v.z; h.w = (_Float16)v.w;
    bstore8<NT>(r, off, __builtin_bit_cast(i2v, h));
  }
  __device__ static float4 widen(const Raw& h) {
    return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
  }
  template <bool NT = false>
  __device__ static float4 ld(const void* b, int64_t i) { return widen(ldr<NT>(b, i)); }
  __device__ static float ld1(const void* b, int64_t i) {
    return (float)gmem(static_cast<const _Float16*>(b))[i];
  }
  template <bool NT = false>
  __device__ static void st(void* b, int64_t i, const float4& v) {
    h4v h;
    h.x = (_Float16)v.x; h.y = (_Float16)v.y; h.z = (_Float16)v.z; h.w = (_Float16)v.w;
    vstore<NT>(reinterpret_cast<h4v*>(static_cast<_Float16*>(b) + i), h);
  }
};
__device__ __forceinline__ unsigned bf16_rne(float f) {
  const unsigned u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
template <> struct Store<ST_BF16> {
  using Raw = u2v;
  __device__ static Raw zero() { return Raw{0u, 0u}; }
  template <bool NT = false>
  __device__ static Raw ldr(const void* b, int64_t i) {
    return vload<NT>(reinterpret_cast<const u2v*>(static_cast<const unsigned short*>(b) + i));
  }
  static constexpr int kBytes = 2;
  template <bool NT = false>
  __device__ static Raw ldb(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(Raw, bload8<NT>(r, off));
  }
  template <bool NT = false>
  __device__ static void stb(__amdgpu_buffer_rsrc_t r, unsigned off, const float4& v) {
    u2v w;
    w.x = bf16_rne(v.x) | (bf16_rne(v.y) << 16);
    w.y = bf16_rne(v.z) | (bf16_rne(v.w) << 16);
    bstore8<NT>(r, off, __builtin_bit_cast(i2v, w));
  }
  __device__ static float4 widen(const Raw& r) {
    return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                       __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
  }
  template <bool NT = false>
  __device__ static float4 ld(const void* b, int64_t i) { return widen(ldr<NT>(b, i)); }
  __device__ static float ld1(const void* b, int64_t i) {
    return __uint_as_float((unsigned)gmem(static_cast<const unsigned short*>(b))[i] << 16);
  }
  template <bool NT = false>
  __device__ static void st(void* b, int64_t i, const float4& v) {
    u2v r;
    r.x = bf16_rne(v.x) | (bf16_rne(v.y) << 16);
    r.y = bf16_rne(v.z) | (bf16_rne(v.w) << 16);
    vstore<NT>(reinterpret_cast<u2v*>(static_cast<unsigned short*>(b) + i), r);
  }
};

__device__ __forceinline__ float4 mul4(const float4& v, float s) {
  return make_float4(v.x * s, v.y * s, v.z * s, v.w * s);
}

// Scale exponent e for a level whose magnitudes are bounded by b: b * 2^e stays
// below 2^kScaleTarget (16x below the FP16 maximum).
__device__ __forceinline__ int scale_exp(float b) {
  int e = -126;
  if (b > 0.f && b <= 3.0e38f) {
    int ex;
    frexpf(b, &ex);  // b < 2^ex
    e = ex;
  }
  return min(max(kScaleTarget - e, -120), 120);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Weighted sum over up to 8 trilinear corners (unused corners carry weight 0
// and index 0) of a stored level, decoded with factor dec.
template <int ST>
__device__ __forceinline__ float sample_point(const void* f, float dec, const int* idx,
                                              const float* w, int r) {
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c)
    acc = fmaf(gmem(w)[8 * r + c], Store<ST>::ld1(f, gmem(idx)[8 * r + c]) * dec, acc);
  return acc;
}
}  // namespace
}  // namespace wave
