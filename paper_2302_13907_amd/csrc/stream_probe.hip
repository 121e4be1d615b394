// Bandwidth reference for the roofline: a kernel that only streams.  Each
// thread reads one group (16 bytes, or 4) from each of R arrays and writes
// one to each of W arrays (their sum, so no read can be dropped), which is
// the access pattern of the step kernels with the stencil taken out.  The
// rate it reaches for a kernel's mix of read and write streams is what HBM
// delivers for that pattern on the device at hand; the 4-byte form has four
// times as many threads resident for the same bytes.
#include "cwell_internal.hpp"

namespace cw {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
// non-temporal load and store of one group
__device__ __forceinline__ float ldnt(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float4 ldnt(const float4 *p)
{
  const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stnt(float v, float *p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void stnt(float4 v, float4 *p)
{
  f4v u;
  u.x = v.x; u.y = v.y; u.z = v.z; u.w = v.w;
  __builtin_nontemporal_store(u, reinterpret_cast<f4v *>(p));
}

__device__ __forceinline__ void acc(float4 &s, const float4 &v) { s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w; }
__device__ __forceinline__ void acc(float &s, float v) { s += v; }
__device__ __forceinline__ float4 bump(float4 s, int q) { s.x += (float)q; return s; }
__device__ __forceinline__ float bump(float s, int q) { return s + (float)q; }

// NT: every load and store non-temporal (the lines are not kept), the rate
// a stream reaches when nothing it reads is read again
template <class T, int R, int W, bool NT>
__global__ void __launch_bounds__(256) k_stream(const T *base, size_t ng)
{
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= ng) return;
  T s{};
#pragma unroll
  for (int q = 0; q < R; q++) {
    const T *p = base + (size_t)q * ng + t;
    acc(s, NT ? ldnt(p) : *p);
  }
  T *out = const_cast<T *>(base) + (size_t)R * ng;
#pragma unroll
  for (int q = 0; q < W; q++) {
    if (NT) stnt(bump(s, q), out + (size_t)q * ng + t);
    else out[(size_t)q * ng + t] = bump(s, q);
  }
}

template <class T, int R, int W>
hipError_t launch(const void *base, size_t bytes_per_array, bool nt, hipStream_t stream)
{
  const size_t ng = bytes_per_array / sizeof(T);
  const size_t g = (ng + 255) / 256;
  if (g > 0x7fffffffu) return hipErrorInvalidConfiguration;
  if (nt) hipLaunchKernelGGL((k_stream<T, R, W, true>), dim3((unsigned)g), dim3(256), 0, stream, static_cast<const T *>(base), ng);
  else hipLaunchKernelGGL((k_stream<T, R, W, false>), dim3((unsigned)g), dim3(256), 0, stream, static_cast<const T *>(base), ng);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mix(const void *b, size_t bytes, int r, int w, bool nt, hipStream_t stream)
{
  if (r == 1 && w == 1) return launch<T, 1, 1>(b, bytes, nt, stream);
  if (r == 9 && w == 3) return launch<T, 9, 3>(b, bytes, nt, stream);
  if (r == 10 && w == 3) return launch<T, 10, 3>(b, bytes, nt, stream);
  if (r == 9 && w == 6) return launch<T, 9, 6>(b, bytes, nt, stream);
  if (r == 11 && w == 6) return launch<T, 11, 6>(b, bytes, nt, stream);
  if (r == 9 && w == 9) return launch<T, 9, 9>(b, bytes, nt, stream);
  if (r == 12 && w == 9) return launch<T, 12, 9>(b, bytes, nt, stream);
  return hipErrorInvalidValue;
}

}  // namespace

// the stream mixes of the step kernels (velocity, stress, single pass; with and
// without the medium arrays) and a copy
bool stream_mix_supported(int r, int w)
{
  static const int mixes[][2] = {{1, 1}, {9, 3}, {10, 3}, {9, 6}, {11, 6}, {9, 9}, {12, 9}};
  for (const auto &m : mixes)
    if (m[0] == r && m[1] == w) return true;
  return false;
}

hipError_t launch_stream(const void *base, size_t bytes_per_array, int lane_bytes, bool nt, int r, int w,
                         hipStream_t stream)
{
  if (lane_bytes == 16) return launch_mix<float4>(base, bytes_per_array, r, w, nt, stream);
  if (lane_bytes == 4) return launch_mix<float>(base, bytes_per_array, r, w, nt, stream);
  return hipErrorInvalidValue;
}

}  // namespace cw
