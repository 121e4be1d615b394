// Azimuthal refinement (Sec. 3): the values the stencils of one zone need
// from the edge ring of the neighbouring zone, on the zone's own azimuthal
// grid.  A transfer maps one source ring [ns][nz] to one ghost ring
// [nd][nz] through a dense matrix M [nd][ns] (the Fourier interpolation or
// its transpose, written out on the host): out[r][k] = sum_j M[r][j] in[j][k].
//
// A workgroup stages the matrix and a tile of KT depth columns of the
// source ring in LDS, so every source value is read from memory once and the
// matrix entries are LDS broadcasts; each lane (one depth column) produces
// four destination rows per pass over the source rows, rows w, w + 4, ...
// going to wavefront w.
#include "cwell_internal.hpp"

namespace cw {

namespace {

constexpr int KT = 64;   // depth columns per workgroup (one per lane)

__global__ void __launch_bounds__(256) k_interp(const Transfer *__restrict__ T, int nz)
{
  extern __shared__ float lds[];                   // tile [ns][KT], then M [nd][ns]
  const Transfer t = T[blockIdx.y];
  const int ns = t.ns, nd = t.nd;
  float *tile = lds, *M = lds + ns * KT;
  const int k0 = blockIdx.x * KT;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kw = nz - k0 < KT ? nz - k0 : KT;      // columns of this tile inside the grid
  for (int c = threadIdx.x; c < ns * KT; c += 256) {
    const int j = c / KT, kk = c - j * KT;
    tile[c] = kk < kw ? t.src[(size_t)j * nz + k0 + kk] : 0.0f;
  }
  for (int c = threadIdx.x; c < nd * ns; c += 256) M[c] = t.M[c];
  __syncthreads();
  if (lane >= kw) return;                          // no barrier below
  for (int r0 = w; r0 < nd; r0 += 16) {            // rows r0, r0 + 4, r0 + 8, r0 + 12
    const int nrow = r0 + 12 < nd ? 4 : (nd - r0 + 3) / 4;
    const float *m0 = M + r0 * ns;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (nrow == 4) {
      for (int j = 0; j < ns; j++) {
        const float x = tile[j * KT + lane];
        a0 += m0[j] * x;
        a1 += m0[4 * ns + j] * x;
        a2 += m0[8 * ns + j] * x;
        a3 += m0[12 * ns + j] * x;
      }
    } else {
      for (int j = 0; j < ns; j++) {
        const float x = tile[j * KT + lane];
        a0 += m0[j] * x;
        if (nrow > 1) a1 += m0[4 * ns + j] * x;
        if (nrow > 2) a2 += m0[8 * ns + j] * x;
      }
    }
    float *d = t.dst + (size_t)r0 * nz + k0 + lane;
    d[0] = a0;
    if (nrow > 1) d[(size_t)4 * nz] = a1;
    if (nrow > 2) d[(size_t)8 * nz] = a2;
    if (nrow > 3) d[(size_t)12 * nz] = a3;
  }
}

}  // namespace

// LDS of one workgroup: the source tile and the matrix (at most 2 max_ns x max_ns / 2 values)
size_t interp_lds_bytes(int max_ns) { return ((size_t)max_ns * KT + (size_t)max_ns * max_ns / 2) * sizeof(float); }

hipError_t launch_interp(const Transfer *dev, int count, int nz, int max_ns, hipStream_t stream)
{
  if (count == 0) return hipSuccess;
  if (interp_lds_bytes(max_ns) > 160 * 1024) return hipErrorInvalidConfiguration;
  const unsigned gx = (unsigned)((nz + KT - 1) / KT);
  hipLaunchKernelGGL(k_interp, dim3(gx, (unsigned)count), dim3(256), interp_lds_bytes(max_ns), stream, dev, nz);
  return hipGetLastError();
}

}  // namespace cw
