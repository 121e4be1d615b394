// Device helpers shared by the depth-vectorized step kernels (solo and
// batched column forms): VW consecutive depth cells per thread, zero ghosts
// outside the grid, layer memory updates, float16 scale tracking.
#pragma once
#include "cwell_internal.hpp"
#include "storage.hpp"

namespace cw {
namespace vec {

constexpr int VW = 4;

__device__ __forceinline__ size_t at(const StepArgs &a, int i, int j, int k)
{
  return (size_t)i * a.rs + (size_t)j * a.nz + k;
}

// index of cell (i, j, k) in the medium arrays
__device__ __forceinline__ size_t mat(const StepArgs &a, int i, int j, int k)
{
  return (size_t)i * a.m_ring + (size_t)j * a.m_row + k;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int zrow(const StepArgs &a, int k)
{
  if (a.npz == 0) return -1;
  if (k < a.npz) return k;
  const int lo = a.nz - 1 - a.npz;
  return k >= lo ? k - lo + a.npz : -1;
}

// VW physical values of field f at (i, j, k0..k0+VW-1); zero for a ring
// outside [0, nr)
template <class S>
__device__ __forceinline__ void ldv(float (&o)[VW], const float *f, float s, const StepArgs &a, int i, int j, int k0)
{
  if (i < 0 || i >= a.nr) {
#pragma unroll
    for (int e = 0; e < VW; e++) o[e] = 0.0f;
    return;
  }
  S::template ldv<VW>(o, f, at(a, i, j, k0), s);
}

// one value at (i, j, k), zero for k outside [0, nz)
template <class S>
__device__ __forceinline__ float ld1(const float *f, float s, const StepArgs &a, int i, int j, int k)
{
  const int kc = k < 0 ? 0 : (k >= a.nz ? a.nz - 1 : k);
  const float v = S::ld(f, at(a, i, j, kc), s);
  return (k >= 0 && k < a.nz) ? v : 0.0f;
}

__device__ __forceinline__ float cpml1(float *psi, size_t q, float ca, float cb, float X)
{
  const float v = cb * psi[q] + ca * X;
  psi[q] = v;
  return X + v;
}

// Depth-layer memory of the lane's VW cells for three slab arrays p0..p2
// (hN: array N takes the half-node coefficients): psi <- b psi + a X,
// X += psi for the cells inside the layer.  The arrays and the table are
// declared not to overlap, so a cell's three slab reads and its coefficients
// go out together instead of each waiting for the previous array's store:
// four memory round trips per lane in the layer instead of twelve.  The
// 16-bit forms use it (256 x 128 x 8192: float16 step 4.06 -> 3.90 ms,
// bfloat16 3.88 -> 3.84; float16 on 192 x 96 x 4096 61.8 -> 64.3
// Gcell/s).  In float32 the four-cell stress update then spilled registers
// and was 8 % slower, so float32 keeps the arrays one after the other; the
// same treatment of the radial block cost bfloat16 8 % (spills) for 0.3 %
// in float16.
__device__ __forceinline__ void cpml_z3(const StepArgs &a, int i, int j, int kb, float *__restrict__ p0,
                                        float *__restrict__ p1, float *__restrict__ p2, const float *__restrict__ T,
                                        bool h0, bool h1, bool h2, float (&X0)[VW], float (&X1)[VW],
                                        float (&X2)[VW])
{
#pragma unroll
  for (int e = 0; e < VW; e++) {
    const int k = kb + e, kz = zrow(a, k);
    if (kz < 0) continue;
    const size_t q = ((size_t)i * a.nt + j) * a.nzs + kz;
    const float ac = T[AZ_C * a.nz + k], bc = T[BZ_C * a.nz + k], ah = T[AZ_H * a.nz + k], bh = T[BZ_H * a.nz + k];
    const float v0 = (h0 ? bh : bc) * p0[q] + (h0 ? ah : ac) * X0[e];
    p0[q] = v0;
    X0[e] = X0[e] + v0;
    const float v1 = (h1 ? bh : bc) * p1[q] + (h1 ? ah : ac) * X1[e];
    p1[q] = v1;
    X1[e] = X1[e] + v1;
    const float v2 = (h2 ? bh : bc) * p2[q] + (h2 ? ah : ac) * X2[e];
    p2[q] = v2;
    X2[e] = X2[e] + v2;
  }
}

// largest |x| of the wavefront into one of 64 slots of a field (spreads
// the atomics of a launch over 64 addresses)
__device__ __forceinline__ void track_max(unsigned *slots, float m)
{
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0f)
    atomicMax(&slots[(blockIdx.x + (threadIdx.x >> 6)) & (kMaxSlots - 1)], __builtin_bit_cast(unsigned, m));
}

// Addressing of one wavefront.  Every access goes through a buffer
// resource spanning one ring of one array (base and size in scalar
// registers); the theta row is a uniform byte offset and the lane's depth
// position a per-lane byte offset, the same for every array of a width.
template <class S>
struct Lanes {
  unsigned v0, vb, va;      // field bytes: the lane's group, the cell before it, the cell after it
  unsigned m0, ma;          // float32 bytes: the lane's group, the clamped cell after it
  bool has_b, has_a;        // the cell before / after the group is inside the grid
  unsigned sj, sjm, sjp;    // field bytes of rows j, j - 1, j + 1 within a ring
  unsigned tj, tjm, tjp;    // float32 bytes of the same rows (layer memory)
  unsigned mj, mjp;         // medium bytes of rows j, j + 1 (0 when the medium does not vary along theta)
  size_t ring, pring;       // ring strides (values): fields (padded), layer memory (nt x nz)
  unsigned ringb, ringm;    // bytes of one ring's cells: fields, float32 arrays
  size_t mring;             // medium values per ring
  unsigned mringb;

  __device__ Lanes(const StepArgs &a, int kb, int j, int jm, int jp)
  {
    ring = a.rs;
    pring = (size_t)a.nt * a.nz;
    ringb = (unsigned)(pring * S::bytes);
    ringm = (unsigned)(pring * 4);
    has_b = kb > 0;
    has_a = kb + VW < a.nz;
    v0 = (unsigned)kb * S::bytes;
    vb = has_b ? v0 - S::bytes : v0;
    va = has_a ? v0 + VW * S::bytes : v0;
    m0 = (unsigned)kb * 4u;
    ma = has_a ? m0 + VW * 4u : (unsigned)(a.nz - 1) * 4u;
    sj = (unsigned)j * a.nz * S::bytes; sjm = (unsigned)jm * a.nz * S::bytes; sjp = (unsigned)jp * a.nz * S::bytes;
    tj = (unsigned)j * a.nz * 4u; tjm = (unsigned)jm * a.nz * 4u; tjp = (unsigned)jp * a.nz * 4u;
    mj = (unsigned)j * a.m_row * 4u; mjp = (unsigned)jp * a.m_row * 4u;
    mring = a.m_ring;
    mringb = (unsigned)(mring * 4);
  }
  // resource of ring i of a field array / a float32 array
  // (i may be -1: a ghost ring before ring 0)
  __device__ rsrc_t field(const float *f, int i) const { return make_rsrc(S::adv(f, (ptrdiff_t)i * (ptrdiff_t)ring), ringb); }
  __device__ rsrc_t fieldw(float *f, int i) const { return make_rsrc(S::adv(f, (ptrdiff_t)i * (ptrdiff_t)ring), ringb); }
  __device__ rsrc_t f32(const float *f, int i) const { return make_rsrc(f + (size_t)i * pring, ringm); }
  __device__ rsrc_t med(const float *f, int i) const { return make_rsrc(f + (size_t)i * mring, mringb); }
};

// VW values of a field at ring i, row offset soff: zero for a ring outside
// [0, nr) unless a ghost ring stands there.
// In 16-bit storage such a ring is read through an empty resource (size 0:
// every read is out of range and returns zero) rather than skipped by a
// branch: those forms convert a value where it is loaded, so a load inside
// a branch waits there for every load in flight, and the six guarded
// neighbour reads of a column cost six memory round trips one after the
// other (measured at 256 x 128 x 8192: bfloat16 4.01 -> 3.87 ms per step,
// float16 4.55 -> 4.30).  Float32 keeps the branch, which waits for nothing:
// read unconditionally, the batched launches were 2 % slower.
template <class S>
__device__ __forceinline__ void ldf(float (&o)[VW], const Lanes<S> &L, const StepArgs &a, const float *f, float s,
                                    int i, unsigned soff)
{
  const bool out = (i < 0 && !a.ghost_in) || (i >= a.nr && !a.ghost_out);
  if (S::bytes == 2) {
    const rsrc_t r = make_rsrc(S::adv(f, (ptrdiff_t)(out ? 0 : i) * (ptrdiff_t)L.ring), out ? 0u : L.ringb);
    S::ldb(o, r, L.v0, soff, s);
    return;
  }
  if (out) {
#pragma unroll
    for (int e = 0; e < VW; e++) o[e] = 0.0f;
    return;
  }
  S::ldb(o, L.field(f, i), L.v0, soff, s);
}

// one depth neighbour of the lane's group (offset voff, clamped to a valid
// cell when there is none), zero when there is none; in 16-bit storage read
// unconditionally and selected, for the reason given at ldf
template <class S>
__device__ __forceinline__ float ldz(bool has, rsrc_t r, unsigned voff, unsigned soff, float s)
{
  if (S::bytes == 2) {
    const float x = S::ldb1(r, voff, soff, s);
    return has ? x : 0.0f;
  }
  return has ? S::ldb1(r, voff, soff, s) : 0.0f;
}

// layer memory update of the lane's VW values of one radial-slab array: psi <- b psi + a X, X += psi.
// The arrays of a layer block are updated one after the other, each read
// waiting for the previous store.  Reading them two at a time before writing
// (as the one-cell kernels read all six) held more registers and made the
// four-cell forms slower at 256 x 128 x 8192: bfloat16 4.22 against 3.87 ms
// per step, float16 4.66 against 4.31.
__device__ __forceinline__ void cpml_b(rsrc_t r, unsigned voff, unsigned soff, float ca, float cb, float (&X)[VW])
{
  float p[VW];
  ldb4<kOwnLoadAux>(p, r, voff, soff);
#pragma unroll
  for (int e = 0; e < VW; e++) {
    p[e] = cb * p[e] + ca * X[e];
    X[e] += p[e];
  }
  stb4<kFieldStoreAux>(r, voff, soff, p);      // read again only by the next step
}

// 1 / s for a power-of-two scale s, exactly
__device__ __forceinline__ float inv_pow2(float s)
{
  return __builtin_amdgcn_ldexpf(1.0f, 1 - __builtin_amdgcn_frexp_expf(s));
}

}  // namespace vec
}  // namespace cw
