// Bandwidth reference for the roofline: a kernel that only streams.  Each
// thread reads one 16-byte group from each of R arrays and writes one to
// each of W arrays (their sum, so no read can be dropped), which is the
// access pattern of the step kernels with the stencil taken out.  The rate
// it reaches for a kernel's mix of read and write streams is what HBM
// delivers for that pattern on the device at hand.
#include "cwell_internal.hpp"

namespace cw {

namespace {

template <int R, int W>
__global__ void __launch_bounds__(256) k_stream(const float4 *base, size_t n4)
{
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n4) return;
  float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int q = 0; q < R; q++) {
    const float4 v = base[(size_t)q * n4 + t];
    s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
  }
  float4 *out = const_cast<float4 *>(base) + (size_t)R * n4;
#pragma unroll
  for (int q = 0; q < W; q++) out[(size_t)q * n4 + t] = make_float4(s.x + q, s.y, s.z, s.w);
}

template <int R, int W>
hipError_t launch(const float4 *base, size_t n4, hipStream_t stream)
{
  const size_t g = (n4 + 255) / 256;
  hipLaunchKernelGGL((k_stream<R, W>), dim3((unsigned)g), dim3(256), 0, stream, base, n4);
  return hipGetLastError();
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

hipError_t launch_stream(const void *base, size_t n4, int r, int w, hipStream_t stream)
{
  const float4 *b = static_cast<const float4 *>(base);
  if ((size_t)((n4 + 255) / 256) > 0x7fffffffu) return hipErrorInvalidConfiguration;
  if (r == 1 && w == 1) return launch<1, 1>(b, n4, stream);
  if (r == 9 && w == 3) return launch<9, 3>(b, n4, stream);
  if (r == 10 && w == 3) return launch<10, 3>(b, n4, stream);
  if (r == 9 && w == 6) return launch<9, 6>(b, n4, stream);
  if (r == 11 && w == 6) return launch<11, 6>(b, n4, stream);
  if (r == 9 && w == 9) return launch<9, 9>(b, n4, stream);
  if (r == 12 && w == 9) return launch<12, 9>(b, n4, stream);
  return hipErrorInvalidValue;
}

}  // namespace cw
