// Field storage policies of the step kernels: load a physical value (a
// stored value times its field's scale s) and store one (times 1/s), one
// value at a time or four consecutive ones with a single wide access.
// Arithmetic is float32 for every policy.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

#include "cwell_internal.hpp"

namespace cw {

// Buffer accesses: a wavefront-uniform resource (base address and size in
// scalar registers), a per-lane byte offset and a uniform byte offset.
// Raw buffer reads beyond the resource's size return zero.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
// Cache policy of the field streams (bit 1 = non-temporal: the line is not
// kept for reuse).  Every field value a launch writes is read only by a
// later launch, long after it would have left the caches, so the stores are
// non-temporal.  Measured on MI355X at 256 x 128 x 8192: 3 % faster in
// float32 and bfloat16, 5 % fewer L2 fetches.  Loads of the arrays that
// neighbouring columns re-read stay cached (non-temporal there: 7-16 %
// slower); loads that only the lane's own update reads (the old values of
// the updated fields, the layer memory) are non-temporal, which leaves the
// caches to the re-read arrays: 2 % faster in every storage.
#ifndef CW_NT_LOAD
#define CW_NT_LOAD 0
#endif
#ifndef CW_NT_STORE
#define CW_NT_STORE 1
#endif
#ifndef CW_NT_OWN
#define CW_NT_OWN 1
#endif
constexpr int kFieldLoadAux = CW_NT_LOAD ? 2 : 0;
constexpr int kFieldStoreAux = CW_NT_STORE ? 2 : 0;
// loads of values only the lane's own update reads (no neighbour re-reads them)
constexpr int kOwnLoadAux = CW_NT_OWN ? 2 : 0;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, unsigned nbytes)
{
  // word 3: 32-bit data format, which untyped loads and stores require on this family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nbytes, 0x00020000);
}
template <int AUX = 0>
__device__ __forceinline__ void ldb4(float (&o)[4], rsrc_t r, unsigned voff, unsigned soff)
{
  const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX);
  // copy the elements out first: a bit cast of a vector-element lvalue reads element 0
  const unsigned x = u.x, y = u.y, z = u.z, w = u.w;
  o[0] = __builtin_bit_cast(float, x); o[1] = __builtin_bit_cast(float, y);
  o[2] = __builtin_bit_cast(float, z); o[3] = __builtin_bit_cast(float, w);
}
template <int AUX = 0>
__device__ __forceinline__ void stb4(rsrc_t r, unsigned voff, unsigned soff, const float (&v)[4])
{
  u32x4 u;
  u.x = __builtin_bit_cast(unsigned, v[0]); u.y = __builtin_bit_cast(unsigned, v[1]);
  u.z = __builtin_bit_cast(unsigned, v[2]); u.w = __builtin_bit_cast(unsigned, v[3]);
  __builtin_amdgcn_raw_buffer_store_b128(u, r, voff, soff, AUX);
}
__device__ __forceinline__ float ldb1(rsrc_t r, unsigned voff, unsigned soff)
{
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// A 32-bit integer hash (two multiply and three xor-shift rounds; the
// "lowbias32" constants of C. Wellons' hash-prospector): the counter-based
// random bits of stochastic rounding, from a cell, a field and a step.
__device__ __forceinline__ unsigned hash32(unsigned x)
{
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

struct StF32 {
  static constexpr bool scaled = false;
  static constexpr unsigned bytes = 4;   // bytes per stored value
  // f advanced by p stored values
  __device__ static const float *adv(const float *f, ptrdiff_t p) { return f + p; }
  __device__ static float *adv(float *f, ptrdiff_t p) { return f + p; }
  __device__ static float ld(const float *f, size_t p, float) { return f[p]; }
  __device__ static void ldb(float (&o)[4], rsrc_t r, unsigned voff, unsigned soff, float)
  {
    ldb4<kFieldLoadAux>(o, r, voff, soff);
  }
  __device__ static void ldbu(float (&o)[4], rsrc_t r, unsigned voff, unsigned soff, float)
  {
    ldb4<kOwnLoadAux>(o, r, voff, soff);
  }
  __device__ static float ldb1(rsrc_t r, unsigned voff, unsigned soff, float) { return cw::ldb1(r, voff, soff); }
  static constexpr bool stochastic = false;   // float32 stores are exact: no rounding mode
  __device__ static void stb(rsrc_t r, unsigned voff, unsigned soff, const float (&v)[4], float, unsigned = 0u,
                             bool = false)
  {
    stb4<kFieldStoreAux>(r, voff, soff, v);
  }
  __device__ static void st(float *f, size_t p, float v, float) { f[p] = v; }
  // one value that only the thread's own update reads / one field value written
  __device__ static float ldn(const float *f, size_t p, float)
  {
    return CW_NT_OWN ? __builtin_nontemporal_load(f + p) : f[p];
  }
  __device__ static void stn(float *f, size_t p, float v, float, unsigned = 0u, bool = false)
  {
    if (CW_NT_STORE) __builtin_nontemporal_store(v, f + p);
    else f[p] = v;
  }
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
  static constexpr unsigned bytes = 2;
  __device__ static const float *adv(const float *f, ptrdiff_t p)
  {
    return reinterpret_cast<const float *>(reinterpret_cast<const unsigned short *>(f) + p);
  }
  __device__ static float *adv(float *f, ptrdiff_t p)
  {
    return reinterpret_cast<float *>(reinterpret_cast<unsigned short *>(f) + p);
  }
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  __device__ static float ld(const float *f, size_t p, float s)
  {
    return (float)reinterpret_cast<const _Float16 *>(f)[p] * s;
  }
  template <int AUX = kFieldLoadAux>
  __device__ static void ldb(float (&o)[4], rsrc_t r, unsigned voff, unsigned soff, float s)
  {
    const h4 v = __builtin_bit_cast(h4, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
    o[0] = (float)v[0] * s; o[1] = (float)v[1] * s; o[2] = (float)v[2] * s; o[3] = (float)v[3] * s;
  }
  __device__ static void ldbu(float (&o)[4], rsrc_t r, unsigned voff, unsigned soff, float s)
  {
    ldb<kOwnLoadAux>(o, r, voff, soff, s);
  }
  __device__ static float ldb1(rsrc_t r, unsigned voff, unsigned soff, float s)
  {
    return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)) * s;
  }
  static constexpr bool stochastic = false;   // float16 stores round to nearest even
  __device__ static void stb(rsrc_t r, unsigned voff, unsigned soff, const float (&v)[4], float is, unsigned = 0u,
                             bool = false)
  {
    h4 h;
    h[0] = (_Float16)(v[0] * is); h[1] = (_Float16)(v[1] * is);
    h[2] = (_Float16)(v[2] * is); h[3] = (_Float16)(v[3] * is);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, h), r, voff, soff, kFieldStoreAux);
  }
  __device__ static void st(float *f, size_t p, float v, float is)
  {
    reinterpret_cast<_Float16 *>(f)[p] = (_Float16)(v * is);
  }
  __device__ static float ldn(const float *f, size_t p, float s)
  {
    const _Float16 *h = reinterpret_cast<const _Float16 *>(f) + p;
    return (float)(CW_NT_OWN ? __builtin_nontemporal_load(h) : *h) * s;
  }
  __device__ static void stn(float *f, size_t p, float v, float is, unsigned = 0u, bool = false)
  {
    _Float16 *h = reinterpret_cast<_Float16 *>(f) + p;
    const _Float16 x = (_Float16)(v * is);
    if (CW_NT_STORE) __builtin_nontemporal_store(x, h);
    else *h = x;
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
  static constexpr unsigned bytes = 2;
  __device__ static const float *adv(const float *f, ptrdiff_t p)
  {
    return reinterpret_cast<const float *>(reinterpret_cast<const unsigned short *>(f) + p);
  }
  __device__ static float *adv(float *f, ptrdiff_t p)
  {
    return reinterpret_cast<float *>(reinterpret_cast<unsigned short *>(f) + p);
  }
  // round to nearest even (the hardware conversion, two values per instruction)
  __device__ static unsigned short pack(float v) { return __builtin_bit_cast(unsigned short, (__bf16)v); }
  __device__ static unsigned pack2(float a, float b)
  {
    bf2 h;
    h[0] = (__bf16)a;
    h[1] = (__bf16)b;
    return __builtin_bit_cast(unsigned, h);
  }
  __device__ static float unpack(unsigned short h) { return __builtin_bit_cast(float, (unsigned)h << 16); }
  __device__ static float ld(const float *f, size_t p, float)
  {
    return unpack(reinterpret_cast<const unsigned short *>(f)[p]);
  }
  template <int AUX = kFieldLoadAux>
  __device__ static void ldb(float (&o)[4], rsrc_t r, unsigned voff, unsigned soff, float)
  {
    const u32x2 u = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
    o[0] = __builtin_bit_cast(float, u.x << 16); o[1] = __builtin_bit_cast(float, u.x & 0xffff0000u);
    o[2] = __builtin_bit_cast(float, u.y << 16); o[3] = __builtin_bit_cast(float, u.y & 0xffff0000u);
  }
  __device__ static void ldbu(float (&o)[4], rsrc_t r, unsigned voff, unsigned soff, float s)
  {
    ldb<kOwnLoadAux>(o, r, voff, soff, s);
  }
  __device__ static float ldb1(rsrc_t r, unsigned voff, unsigned soff, float)
  {
    return unpack(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  }
  // Stochastic rounding (gfx950 v_cvt_sr_bf16_f32): the value is rounded up
  // with probability equal to the fraction of a unit in the last place that
  // rounding down would drop, so the rounding error has mean zero and the
  // small per-step increments of a slowly varying field are kept on
  // average instead of being lost below half a unit.  The instruction takes
  // its 16 random bits from bits 31..16 of its random operand, so one
  // 32-bit random word serves two values (the word, and the word shifted
  // left by 16).
  static constexpr bool stochastic = true;
  __device__ static unsigned pack2_sr(float a, unsigned ra, float b, unsigned rb)
  {
    bf2 h = {};
    h = __builtin_amdgcn_cvt_sr_bf16_f32(h, a, ra, false);
    h = __builtin_amdgcn_cvt_sr_bf16_f32(h, b, rb, true);
    return __builtin_bit_cast(unsigned, h);
  }
  // sr: stochastic rounding with the random bits hash32(key) (a second word
  // for the last two values is derived by an odd multiplier); else nearest
  // even
  __device__ static void stb(rsrc_t r, unsigned voff, unsigned soff, const float (&v)[4], float, unsigned key = 0u,
                             bool sr = false)
  {
    u32x2 u;
    if (sr) {
      const unsigned rnd = hash32(key), rnd2 = rnd * 0x9e3779b1u;
      u.x = pack2_sr(v[0], rnd, v[1], rnd << 16);
      u.y = pack2_sr(v[2], rnd2, v[3], rnd2 << 16);
    } else {
      u.x = pack2(v[0], v[1]);
      u.y = pack2(v[2], v[3]);
    }
    __builtin_amdgcn_raw_buffer_store_b64(u, r, voff, soff, kFieldStoreAux);
  }
  __device__ static void st(float *f, size_t p, float v, float)
  {
    reinterpret_cast<unsigned short *>(f)[p] = pack(v);
  }
  __device__ static float ldn(const float *f, size_t p, float)
  {
    const unsigned short *h = reinterpret_cast<const unsigned short *>(f) + p;
    return unpack(CW_NT_OWN ? __builtin_nontemporal_load(h) : *h);
  }
  __device__ static void stn(float *f, size_t p, float v, float, unsigned key = 0u, bool sr = false)
  {
    unsigned short *h = reinterpret_cast<unsigned short *>(f) + p;
    const unsigned short x = sr ? (unsigned short)pack2_sr(v, hash32(key), 0.0f, 0u) : pack(v);
    if (CW_NT_STORE) __builtin_nontemporal_store(x, h);
    else *h = x;
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
    u.x = pack2(v[0], v[1]);
    u.y = pack2(v[2], v[3]);
    *reinterpret_cast<uint2 *>(reinterpret_cast<unsigned short *>(f) + p) = u;
  }
};

// Stochastic rounding of a step's stores (storages that have it, when
// asked for).  The random bits of field q's value(s) at linear cell index c
// (the first cell of a group) are hash32 of the key c ^ (q << 28) ^ h(step),
// formed by the store only when it rounds stochastically: cells below 2^28
// and fields below 16 never share a key within a step.
template <class S>
__device__ __forceinline__ bool sr_on(const StepArgs &a) { return S::stochastic && a.sr != 0; }
// c ^ h(step) for the lane's cell (0 when the stores round to nearest)
template <class S>
__device__ __forceinline__ unsigned sr_base(const StepArgs &a, size_t c)
{
  return sr_on<S>(a) ? (unsigned)c ^ hash32((unsigned)*a.step * 0x9e3779b9u + 0x632be5abu) : 0u;
}
__device__ __forceinline__ unsigned sr_key(unsigned base, int q) { return base ^ ((unsigned)q << 28); }

}  // namespace cw
