// Azimuthal refinement (Sec. 3): the values the stencils of one zone need
// from the edge ring of the neighbouring zone, on the zone's own azimuthal
// grid.  A transfer maps one source ring [ns][nz] to one ghost ring
// [nd][nz] through a dense matrix M [nd][ns] (the Fourier interpolation or
// its transpose, written out on the host): out[r][k] = sum_j M[r][j] in[j][k].
//
// A workgroup stages a tile of KT depth columns of the source ring in LDS,
// so every source value is read from memory once; its four wavefronts
// produce the destination rows r = w, w + 4, ...: the matrix row is the
// same for a whole wavefront and the LDS reads are consecutive across lanes.
#include "cwell_internal.hpp"

namespace cw {

namespace {

constexpr int KT = 64;   // depth columns per workgroup (one per lane)

__global__ void __launch_bounds__(256) k_interp(const Transfer *__restrict__ T, int nz)
{
  extern __shared__ float tile[];                  // [ns][KT]
  const Transfer t = T[blockIdx.y];
  const int k0 = blockIdx.x * KT;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kw = nz - k0 < KT ? nz - k0 : KT;      // columns of this tile inside the grid
  for (int c = threadIdx.x; c < t.ns * KT; c += 256) {
    const int j = c / KT, kk = c - j * KT;
    tile[c] = kk < kw ? t.src[(size_t)j * nz + k0 + kk] : 0.0f;
  }
  __syncthreads();
  if (lane >= kw) return;                          // no barrier below
  for (int r = w; r < t.nd; r += 4) {
    const float *m = t.M + (size_t)r * t.ns;
    float acc = 0.0f;
    for (int j = 0; j < t.ns; j++) acc += m[j] * tile[j * KT + lane];
    t.dst[(size_t)r * nz + k0 + lane] = acc;
  }
}

}  // namespace

size_t interp_lds_bytes(int max_ns) { return (size_t)max_ns * KT * sizeof(float); }

hipError_t launch_interp(const Transfer *dev, int count, int nz, int max_ns, hipStream_t stream)
{
  if (count == 0) return hipSuccess;
  if (interp_lds_bytes(max_ns) > 160 * 1024) return hipErrorInvalidConfiguration;
  const unsigned gx = (unsigned)((nz + KT - 1) / KT);
  hipLaunchKernelGGL(k_interp, dim3(gx, (unsigned)count), dim3(256), interp_lds_bytes(max_ns), stream, dev, nz);
  return hipGetLastError();
}

}  // namespace cw
