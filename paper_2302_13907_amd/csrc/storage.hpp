// Field storage policies of the step kernels: load a physical value (a
// stored value times its field's scale s) and store one (times 1/s), one
// value at a time or four consecutive ones with a single wide access.
// Arithmetic is float32 for every policy.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace cw {

struct StF32 {
  static constexpr bool scaled = false;
  __device__ static float ld(const float *f, size_t p, float) { return f[p]; }
  __device__ static void st(float *f, size_t p, float v, float) { f[p] = v; }
  template <int V>
  __device__ static void ldv(float (&o)[V], const float *f, size_t p, float)
  {
    static_assert(V == 4, "four values per access");
    const float4 v = *reinterpret_cast<const float4 *>(f + p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  template <int V>
  __device__ static void stv(float *f, size_t p, const float (&v)[V], float)
  {
    static_assert(V == 4, "four values per access");
    *reinterpret_cast<float4 *>(f + p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};

// float16 with a per-field power-of-two scale; conversion rounds to nearest even
struct StF16 {
  static constexpr bool scaled = true;
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  __device__ static float ld(const float *f, size_t p, float s)
  {
    return (float)reinterpret_cast<const _Float16 *>(f)[p] * s;
  }
  __device__ static void st(float *f, size_t p, float v, float is)
  {
    reinterpret_cast<_Float16 *>(f)[p] = (_Float16)(v * is);
  }
  template <int V>
  __device__ static void ldv(float (&o)[V], const float *f, size_t p, float s)
  {
    static_assert(V == 4, "four values per access");
    const h4 v = *reinterpret_cast<const h4 *>(reinterpret_cast<const _Float16 *>(f) + p);
    o[0] = (float)v[0] * s; o[1] = (float)v[1] * s; o[2] = (float)v[2] * s; o[3] = (float)v[3] * s;
  }
  template <int V>
  __device__ static void stv(float *f, size_t p, const float (&v)[V], float is)
  {
    static_assert(V == 4, "four values per access");
    h4 h;
    h[0] = (_Float16)(v[0] * is); h[1] = (_Float16)(v[1] * is);
    h[2] = (_Float16)(v[2] * is); h[3] = (_Float16)(v[3] * is);
    *reinterpret_cast<h4 *>(reinterpret_cast<_Float16 *>(f) + p) = h;
  }
};

// bfloat16: the upper half of a float32 (same exponent range, no scale);
// conversion rounds to nearest even on the dropped bits (fields stay finite)
struct StBF16 {
  static constexpr bool scaled = false;
  __device__ static unsigned short pack(float v)
  {
    unsigned u = __builtin_bit_cast(unsigned, v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
  }
  __device__ static float unpack(unsigned short h) { return __builtin_bit_cast(float, (unsigned)h << 16); }
  __device__ static float ld(const float *f, size_t p, float)
  {
    return unpack(reinterpret_cast<const unsigned short *>(f)[p]);
  }
  __device__ static void st(float *f, size_t p, float v, float)
  {
    reinterpret_cast<unsigned short *>(f)[p] = pack(v);
  }
  template <int V>
  __device__ static void ldv(float (&o)[V], const float *f, size_t p, float)
  {
    static_assert(V == 4, "four values per access");
    const uint2 u = *reinterpret_cast<const uint2 *>(reinterpret_cast<const unsigned short *>(f) + p);
    o[0] = __builtin_bit_cast(float, u.x << 16); o[1] = __builtin_bit_cast(float, u.x & 0xffff0000u);
    o[2] = __builtin_bit_cast(float, u.y << 16); o[3] = __builtin_bit_cast(float, u.y & 0xffff0000u);
  }
  template <int V>
  __device__ static void stv(float *f, size_t p, const float (&v)[V], float)
  {
    static_assert(V == 4, "four values per access");
    uint2 u;
    u.x = (unsigned)pack(v[0]) | ((unsigned)pack(v[1]) << 16);
    u.y = (unsigned)pack(v[2]) | ((unsigned)pack(v[3]) << 16);
    *reinterpret_cast<uint2 *>(reinterpret_cast<unsigned short *>(f) + p) = u;
  }
};

}  // namespace cw
