// Adjoint of the two-pass time step and the gradient of a receiver loss
// with respect to the moduli of a parameter region.
//
// The step (Eq. (1) in staggered form, with the absorbing layer's memory
// recursions) is linear in the state (v^{n-1/2}, sigma^n, psi^n); its
// transpose runs the two half-steps backwards.  Each half-step is split
// into a "terms" kernel, which turns the adjoints of the updated fields into
// the adjoints of the nine derivative / bracket terms the update summed
// (through the transposed layer recursion psi' = b psi + a X, X + psi'),
// and a "gather" kernel, which adds to every field adjoint the terms that
// read that field, with the transposed stencil coefficients.  Gathering
// (rather than scattering) keeps every sum in a fixed order without atomics.
//
// Gradient: sigma^{n+1} = sigma^n + dt C(lambda, mu) Z^{n+1/2}, Z the strain
// rates, so dL/dlambda and dL/dmu of a cell collect dt Z * (stress adjoint)
// over the steps; a shear node's modulus is the harmonic mean of four cells
// and passes its share to each through d HM4 / d mu.  The strain rates of the
// region come from a forward recomputation of each checkpoint segment.
#include "cwell_internal.hpp"

namespace cw {

namespace {

__device__ __forceinline__ size_t at(const AdjArgs &a, int i, int j, int k)
{
  return (size_t)i * a.rs + (size_t)j * a.nz + k;
}
__device__ __forceinline__ size_t mat(const AdjArgs &a, int i, int j, int k)
{
  return (size_t)i * a.m_ring + (size_t)j * a.m_row + k;
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ int zrow(const AdjArgs &a, int k)
{
  if (a.npz == 0) return -1;
  if (k < a.npz) return k;
  const int lo = a.nz - 1 - a.npz;
  return k >= lo ? k - lo + a.npz : -1;
}
// harmonic mean of four moduli, zero when one is zero (as the forward kernels form it)
__device__ __forceinline__ float hm4(float p, float q, float r, float s)
{
  return 4.0f * rcp(rcp(p) + rcp(q) + rcp(r) + rcp(s));
}
// transposed layer recursion: forward psi' = b psi + a X, out = X + psi';
// from out's adjoint and psi''s adjoint (old, read from *pb) returns X's
// adjoint and leaves psi's adjoint in *pb.  A cell's layer block reads
// every old value and coefficient before it writes any: a store could
// alias a later read, so one array after the other would cost the cell a
// memory round trip per array.
__device__ __forceinline__ float sadj(float *pb, float old, float ca, float cb, float outb)
{
  const float t = old + outb;
  *pb = cb * t;
  return outb + ca * t;
}

__device__ __forceinline__ bool cell(const AdjArgs &a, int &i, int &j, int &k)
{
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (size_t)a.nr * a.nt * a.nz) return false;
  k = (int)(c % a.nz);
  const size_t ij = c / a.nz;
  j = (int)(ij % a.nt);
  i = (int)(ij / a.nt);
  return true;
}

// cells of the absorbing-layer slabs, one per thread: the radial slab
// (rings [nr - npr, nr), every depth) first, then the two depth slabs of the
// remaining rings (rows [0, npz) and [nz - 1 - npz, nz)); each cell once
__device__ __forceinline__ bool slab_cell(const AdjArgs &a, int &i, int &j, int &k)
{
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nrs = (size_t)a.npr * a.nt * a.nz;
  if (c < nrs) {
    k = (int)(c % a.nz);
    const size_t ij = c / a.nz;
    j = (int)(ij % a.nt);
    i = a.nr - a.npr + (int)(ij / a.nt);
    return true;
  }
  const int zr = a.npz > 0 ? 2 * a.npz + 1 : 0;
  const size_t cz = c - nrs;
  if (cz >= (size_t)(a.nr - a.npr) * a.nt * zr) return false;
  const int kz = (int)(cz % zr);
  const size_t ij = cz / zr;
  j = (int)(ij % a.nt);
  i = (int)(ij / a.nt);
  k = kz < a.npz ? kz : a.nz - 1 - a.npz + (kz - a.npz);
  return true;
}
size_t slab_cells(const AdjArgs &a)
{
  return (size_t)a.npr * a.nt * a.nz + (size_t)(a.nr - a.npr) * a.nt * (a.npz > 0 ? 2 * a.npz + 1 : 0);
}
// the cell carries layer memory (its terms depend on state, not only on the fields)
__device__ __forceinline__ bool in_slab(const AdjArgs &a, int i, int k)
{
  return i >= a.nr - a.npr || zrow(a, k) >= 0;
}

// stress half-step, terms: T = (e_rr, e_tt bracket, e_zz, rt_dr, rt_b, rz_dr, rz_dz, tz_b, tz_dz) adjoints
__device__ __forceinline__ void stress_terms_cell(const AdjArgs &a, int i, int j, int k)
{
  const size_t p = at(a, i, j, k);
  const int i1 = i + 1 < a.nr ? i + 1 : a.nr - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const int k1 = k + 1 < a.nz ? k + 1 : a.nz - 1;
  const float mu = a.mu[mat(a, i, j, k)], lam = a.lam[mat(a, i, j, k)];
  const float m_i1 = a.mu[mat(a, i1, j, k)], m_jp = a.mu[mat(a, i, jp, k)], m_k1 = a.mu[mat(a, i, j, k1)];
  const float mu_rt = hm4(mu, m_i1, m_jp, a.mu[mat(a, i1, jp, k)]);
  const float mu_rz = hm4(mu, m_i1, m_k1, a.mu[mat(a, i1, j, k1)]);
  const float mu_tz = hm4(mu, m_jp, m_k1, a.mu[mat(a, i, jp, k1)]);
  const float grr = a.fb[SRR][p], gtt = a.fb[STT][p], gzz = a.fb[SZZ][p];
  const float gs = grr + gtt + gzz;
  float err = a.dt * (lam * gs + 2.0f * mu * grr);
  float ett = a.dt * (lam * gs + 2.0f * mu * gtt);
  float ezz = a.dt * (lam * gs + 2.0f * mu * gzz);
  const float zrt = a.dt * mu_rt * a.fb[SRT][p], zrz = a.dt * mu_rz * a.fb[SRZ][p];
  const float ztz = a.dt * mu_tz * a.fb[STZ][p];
  float rt_dr = zrt, rt_b = zrt, rz_dr = zrz, rz_dz = zrz, tz_b = ztz, tz_dz = ztz;
  const int ir = i - (a.nr - a.npr);
  if (ir >= 0) {
    const size_t q = ((size_t)ir * a.nt + j) * a.nz + k;
    const float *T = a.tab_r;
    float *const *P = a.pr;
    const float ar_c = T[AR_C * a.nr + i], br_c = T[BR_C * a.nr + i], at_c = T[AT_C * a.nr + i], bt_c = T[BT_C * a.nr + i];
    const float ar_f = T[AR_F * a.nr + i], br_f = T[BR_F * a.nr + i], at_f = T[AT_F * a.nr + i], bt_f = T[BT_F * a.nr + i];
    const float m0 = P[R_N_DR][q], m1 = P[R_N_B][q], m2 = P[R_RT_DR][q];
    const float m3 = P[R_RT_B][q], m4 = P[R_RZ_DR][q], m5 = P[R_TZ_B][q];
    err = sadj(&P[R_N_DR][q], m0, ar_c, br_c, err);
    ett = sadj(&P[R_N_B][q], m1, at_c, bt_c, ett);
    rt_dr = sadj(&P[R_RT_DR][q], m2, ar_f, br_f, zrt);
    rt_b = sadj(&P[R_RT_B][q], m3, at_f, bt_f, zrt);
    rz_dr = sadj(&P[R_RZ_DR][q], m4, ar_f, br_f, zrz);
    tz_b = sadj(&P[R_TZ_B][q], m5, at_c, bt_c, ztz);
  }
  const int kz = zrow(a, k);
  if (kz >= 0) {
    const size_t q = ((size_t)i * a.nt + j) * a.nzs + kz;
    const float *T = a.tab_z;
    float *const *P = a.pz;
    const float az_c = T[AZ_C * a.nz + k], bz_c = T[BZ_C * a.nz + k], az_h = T[AZ_H * a.nz + k], bz_h = T[BZ_H * a.nz + k];
    const float m0 = P[Z_N_DZ][q], m1 = P[Z_RZ_DZ][q], m2 = P[Z_TZ_DZ][q];
    ezz = sadj(&P[Z_N_DZ][q], m0, az_c, bz_c, ezz);
    rz_dz = sadj(&P[Z_RZ_DZ][q], m1, az_h, bz_h, zrz);
    tz_dz = sadj(&P[Z_TZ_DZ][q], m2, az_h, bz_h, ztz);
  }
  a.T[0][p] = err; a.T[1][p] = ett; a.T[2][p] = ezz;
  a.T[3][p] = rt_dr; a.T[4][p] = rt_b; a.T[5][p] = rz_dr;
  a.T[6][p] = rz_dz; a.T[7][p] = tz_b; a.T[8][p] = tz_dz;
}
__global__ void __launch_bounds__(256) k_adj_stress_terms(AdjArgs a)
{
  int i, j, k;
  if (cell(a, i, j, k)) stress_terms_cell(a, i, j, k);
}
__global__ void __launch_bounds__(256) k_adj_stress_terms_slab(AdjArgs a)
{
  int i, j, k;
  if (slab_cell(a, i, j, k)) stress_terms_cell(a, i, j, k);
}

// stress half-step, gather: velocity adjoints += (strain operator)^T T
__global__ void __launch_bounds__(256) k_adj_stress_gather(AdjArgs a)
{
  int i, j, k;
  if (!cell(a, i, j, k)) return;
  const size_t p = at(a, i, j, k);
  const int jm = j == 0 ? a.nt - 1 : j - 1, jp = j == a.nt - 1 ? 0 : j + 1;
  const float ci = a.inv_rc[i], fi = a.inv_rf[i];
  float *const *T = a.T;
  const size_t pjm = at(a, i, jm, k), pjp = at(a, i, jp, k);
  // v_r: e_rr and the e_tt bracket of cells i and i+1, rt_b of rows j-1 and j, rz_dz of depths k-1 and k
  float gr = T[0][p] * a.inv_dr + 0.5f * ci * T[1][p];
  if (i + 1 < a.nr) {
    const size_t q = at(a, i + 1, j, k);
    gr += -T[0][q] * a.inv_dr + 0.5f * a.inv_rc[i + 1] * T[1][q];
  }
  gr += fi * (T[4][pjm] - T[4][p]) * a.inv_dth;
  gr -= T[6][p] * a.inv_dz;
  if (k >= 1) gr += T[6][p - 1] * a.inv_dz;
  // v_t: the e_tt bracket of rows j and j+1, rt_dr and rt_b of rings i-1 and i, tz_dz of depths k-1 and k
  float gt = ci * (T[1][p] - T[1][pjp]) * a.inv_dth;
  gt += -T[3][p] * a.inv_dr - 0.5f * fi * T[4][p];
  if (i >= 1) {
    const size_t q = at(a, i - 1, j, k);
    gt += T[3][q] * a.inv_dr - 0.5f * a.inv_rf[i - 1] * T[4][q];
  }
  gt -= T[8][p] * a.inv_dz;
  if (k >= 1) gt += T[8][p - 1] * a.inv_dz;
  // v_z: e_zz of depths k and k+1, rz_dr of rings i-1 and i, tz_b of rows j-1 and j
  float gz = T[2][p] * a.inv_dz;
  if (k + 1 < a.nz) gz -= T[2][p + 1] * a.inv_dz;
  gz -= T[5][p] * a.inv_dr;
  if (i >= 1) gz += T[5][at(a, i - 1, j, k)] * a.inv_dr;
  gz += ci * (T[7][pjm] - T[7][p]) * a.inv_dth;
  a.fb[VR][p] += gr;
  a.fb[VT][p] += gt;
  a.fb[VZ][p] += gz;
}

// velocity half-step, terms: T = (r_dr, r_b, r_dz, t_dr, t_b, t_dz, z_dr, z_b, z_dz) adjoints
__device__ __forceinline__ void velocity_terms_cell(const AdjArgs &a, int i, int j, int k)
{
  const size_t p = at(a, i, j, k);
  const int i1 = i + 1 < a.nr ? i + 1 : a.nr - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const int k1 = k + 1 < a.nz ? k + 1 : a.nz - 1;
  const float rho0 = a.rho[mat(a, i, j, k)];
  const float b_r = 2.0f * rcp(rho0 + a.rho[mat(a, i1, j, k)]);
  const float b_t = 2.0f * rcp(rho0 + a.rho[mat(a, i, jp, k)]);
  const float b_z = 2.0f * rcp(rho0 + a.rho[mat(a, i, j, k1)]);
  const float wr = a.dt * b_r * a.fb[VR][p], wt = a.dt * b_t * a.fb[VT][p], wz = a.dt * b_z * a.fb[VZ][p];
  float r_dr = wr, r_b = wr, r_dz = wr, t_dr = wt, t_b = wt, t_dz = wt, z_dr = wz, z_b = wz, z_dz = wz;
  const int ir = i - (a.nr - a.npr);
  if (ir >= 0) {
    const size_t q = ((size_t)ir * a.nt + j) * a.nz + k;
    const float *T = a.tab_r;
    float *const *P = a.pr;
    const float ar_f = T[AR_F * a.nr + i], br_f = T[BR_F * a.nr + i], at_f = T[AT_F * a.nr + i], bt_f = T[BT_F * a.nr + i];
    const float ar_c = T[AR_C * a.nr + i], br_c = T[BR_C * a.nr + i], at_c = T[AT_C * a.nr + i], bt_c = T[BT_C * a.nr + i];
    const float m0 = P[R_VR_DR][q], m1 = P[R_VR_B][q], m2 = P[R_VT_DR][q];
    const float m3 = P[R_VT_B][q], m4 = P[R_VZ_DR][q], m5 = P[R_VZ_B][q];
    r_dr = sadj(&P[R_VR_DR][q], m0, ar_f, br_f, wr);
    r_b = sadj(&P[R_VR_B][q], m1, at_f, bt_f, wr);
    t_dr = sadj(&P[R_VT_DR][q], m2, ar_c, br_c, wt);
    t_b = sadj(&P[R_VT_B][q], m3, at_c, bt_c, wt);
    z_dr = sadj(&P[R_VZ_DR][q], m4, ar_c, br_c, wz);
    z_b = sadj(&P[R_VZ_B][q], m5, at_c, bt_c, wz);
  }
  const int kz = zrow(a, k);
  if (kz >= 0) {
    const size_t q = ((size_t)i * a.nt + j) * a.nzs + kz;
    const float *T = a.tab_z;
    float *const *P = a.pz;
    const float az_c = T[AZ_C * a.nz + k], bz_c = T[BZ_C * a.nz + k], az_h = T[AZ_H * a.nz + k], bz_h = T[BZ_H * a.nz + k];
    const float m0 = P[Z_VR_DZ][q], m1 = P[Z_VT_DZ][q], m2 = P[Z_VZ_DZ][q];
    r_dz = sadj(&P[Z_VR_DZ][q], m0, az_c, bz_c, wr);
    t_dz = sadj(&P[Z_VT_DZ][q], m1, az_c, bz_c, wt);
    z_dz = sadj(&P[Z_VZ_DZ][q], m2, az_h, bz_h, wz);
  }
  a.T[0][p] = r_dr; a.T[1][p] = r_b; a.T[2][p] = r_dz;
  a.T[3][p] = t_dr; a.T[4][p] = t_b; a.T[5][p] = t_dz;
  a.T[6][p] = z_dr; a.T[7][p] = z_b; a.T[8][p] = z_dz;
}
__global__ void __launch_bounds__(256) k_adj_velocity_terms(AdjArgs a)
{
  int i, j, k;
  if (cell(a, i, j, k)) velocity_terms_cell(a, i, j, k);
}
__global__ void __launch_bounds__(256) k_adj_velocity_terms_slab(AdjArgs a)
{
  int i, j, k;
  if (slab_cell(a, i, j, k)) velocity_terms_cell(a, i, j, k);
}

// velocity half-step, gather: stress adjoints += (divergence operator)^T T
__global__ void __launch_bounds__(256) k_adj_velocity_gather(AdjArgs a)
{
  int i, j, k;
  if (!cell(a, i, j, k)) return;
  const size_t p = at(a, i, j, k);
  const int jm = j == 0 ? a.nt - 1 : j - 1, jp = j == a.nt - 1 ? 0 : j + 1;
  const float ci = a.inv_rc[i], fi = a.inv_rf[i];
  float *const *T = a.T;
  const size_t pjm = at(a, i, jm, k), pjp = at(a, i, jp, k);
  const bool has_im = i >= 1, has_ip = i + 1 < a.nr;
  const size_t pim = has_im ? at(a, i - 1, j, k) : p, pip = has_ip ? at(a, i + 1, j, k) : p;
  const float fim = has_im ? a.inv_rf[i - 1] : 0.0f, cip = has_ip ? a.inv_rc[i + 1] : 0.0f;
  // sigma_rr: r_dr and r_b of the v_r faces i-1 and i
  float grr = -T[0][p] * a.inv_dr + 0.5f * fi * T[1][p];
  if (has_im) grr += T[0][pim] * a.inv_dr + 0.5f * fim * T[1][pim];
  // sigma_tt: r_b of faces i-1 and i, t_b of rows j-1 and j
  float gtt = -0.5f * fi * T[1][p] + ci * (T[4][pjm] - T[4][p]) * a.inv_dth;
  if (has_im) gtt -= 0.5f * fim * T[1][pim];
  // sigma_zz: z_dz of the v_z nodes k-1 and k
  float gzz = -T[8][p] * a.inv_dz;
  if (k >= 1) gzz += T[8][p - 1] * a.inv_dz;
  // sigma_rt: r_b of rows j and j+1, t_dr and t_b of rings i and i+1
  float grt = fi * (T[1][p] - T[1][pjp]) * a.inv_dth + T[3][p] * a.inv_dr + ci * T[4][p];
  if (has_ip) grt += -T[3][pip] * a.inv_dr + cip * T[4][pip];
  // sigma_rz: r_dz of depths k and k+1, z_dr and z_b of rings i and i+1
  float grz = T[2][p] * a.inv_dz + T[6][p] * a.inv_dr + 0.5f * ci * T[7][p];
  if (k + 1 < a.nz) grz -= T[2][p + 1] * a.inv_dz;
  if (has_ip) grz += -T[6][pip] * a.inv_dr + 0.5f * cip * T[7][pip];
  // sigma_tz: t_dz of depths k and k+1, z_b of rows j and j+1
  float gtz = T[5][p] * a.inv_dz + ci * (T[7][p] - T[7][pjp]) * a.inv_dth;
  if (k + 1 < a.nz) gtz -= T[5][p + 1] * a.inv_dz;
  a.fb[SRR][p] += grr; a.fb[STT][p] += gtt; a.fb[SZZ][p] += gzz;
  a.fb[SRT][p] += grt; a.fb[SRZ][p] += grz; a.fb[STZ][p] += gtz;
}

// ---- depth-vectorized gathers (nz a multiple of 4): one workgroup per
// (ring, theta row, 1024 depth cells), four consecutive depth cells per
// thread, 16-byte accesses; the depth neighbours of a thread's group come
// from its own registers except at the group's two ends.  Each cell's
// arithmetic is that of the one-cell gathers above, in the same order.
// Measured on MI355X at 128 x 64 x 2048 (one adjoint step): terms kernels
// over every cell plus four-cell gathers reading the nine stored terms,
// 0.90 ms; gathers forming the terms themselves, 0.67 ms.
constexpr int AW = 4;

struct Col {
  int i, j, jm, jp, kb;
  bool live;
  size_t p, pjm, pjp;       // cell offsets of the group in rows j, j-1, j+1 of ring i
  size_t ring;              // values per ring
};

__device__ __forceinline__ bool col(const AdjArgs &a, Col &c)
{
  const int nbx = (a.nz / AW + 255) / 256;
  const int bx = blockIdx.x % nbx, cc = blockIdx.x / nbx;
  c.i = cc / a.nt;
  c.j = cc - c.i * a.nt;
  if (c.i >= a.nr) return false;
  const int k0 = (bx * 256 + (int)threadIdx.x) * AW;
  c.live = k0 < a.nz;
  c.kb = c.live ? k0 : a.nz - AW;                  // dead lanes compute on a valid group, store nothing
  c.jm = c.j == 0 ? a.nt - 1 : c.j - 1;
  c.jp = c.j == a.nt - 1 ? 0 : c.j + 1;
  c.ring = a.rs;
  c.p = at(a, c.i, c.j, c.kb);
  c.pjm = at(a, c.i, c.jm, c.kb);
  c.pjp = at(a, c.i, c.jp, c.kb);
  return true;
}

__device__ __forceinline__ void ld4(float (&o)[AW], const float *f, size_t q)
{
  const float4 v = *reinterpret_cast<const float4 *>(f + q);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void st4(float *f, size_t q, const float (&v)[AW])
{
  *reinterpret_cast<float4 *>(f + q) = make_float4(v[0], v[1], v[2], v[3]);
}
#ifndef CW_ADJ_NT
#define CW_ADJ_NT 1
#endif
typedef float f4v __attribute__((ext_vector_type(4)));
// f[m][q..q+3] += v[m] for the N arrays f[0..N-1]: the gathers' own
// updates, which no other lane of the launch reads, load and store
// non-temporally (the caches stay with the arrays that neighbouring columns
// re-read).  Every old value is read before any sum is stored: a store could
// alias a later read, so one array after the other would cost the lane a
// memory round trip per array.
template <int N>
__device__ __forceinline__ void add4n(float *const *f, size_t q, const float (&v)[N][AW])
{
  f4v o[N];
#pragma unroll
  for (int m = 0; m < N; m++) {
    f4v *p = reinterpret_cast<f4v *>(f[m] + q);
    o[m] = CW_ADJ_NT ? __builtin_nontemporal_load(p) : *p;
  }
#pragma unroll
  for (int m = 0; m < N; m++) {
    f4v *p = reinterpret_cast<f4v *>(f[m] + q);
    o[m].x += v[m][0]; o[m].y += v[m][1]; o[m].z += v[m][2]; o[m].w += v[m][3];
    if (CW_ADJ_NT) __builtin_nontemporal_store(o[m], p);
    else *p = o[m];
  }
}
// ---- fused gathers (nz a multiple of 4).  Outside the layer slabs a
// term is a pointwise function of the field adjoints and the medium, so
// the gathers form the terms they need, at the group and at its
// neighbours, from the fields themselves instead of reading nine stored
// term arrays; inside the slabs, where the transposed memory recursion
// carries state, a terms pass over the slab cells alone stores them and the
// gathers read them there.  Each term is the expression of the terms
// kernels above, with dt times the harmonic-mean moduli and the face
// buoyancies read from arrays formed once per gradient (k_adj_coefs).

// Minimum wavefronts per SIMD of the fused gathers (1: no constraint).  On
// MI355X at 128 x 64 x 2048, 4 changes nothing and 5 or 6 spill and slow.
#ifndef CW_ADJ_WAVES
#define CW_ADJ_WAVES 1
#endif
// dt mu_rt, dt mu_rz, dt mu_tz, dt b_r, dt b_t, dt b_z of every medium cell
// (one per thread, the medium's own layout), as the terms kernels form them
__global__ void __launch_bounds__(256) k_adj_coefs(AdjArgs a)
{
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (size_t)a.nr * a.m_ring) return;
  const int i = (int)(c / a.m_ring);
  const size_t rem = c - (size_t)i * a.m_ring;
  const int j = a.m_row ? (int)(rem / a.m_row) : 0;
  const int k = a.m_row ? (int)(rem % a.m_row) : (int)rem;
  const int i1 = i + 1 < a.nr ? i + 1 : a.nr - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const int k1 = k + 1 < a.nz ? k + 1 : a.nz - 1;
  const float mu = a.mu[mat(a, i, j, k)];
  const float m_i1 = a.mu[mat(a, i1, j, k)], m_jp = a.mu[mat(a, i, jp, k)], m_k1 = a.mu[mat(a, i, j, k1)];
  a.C[C_RT][c] = a.dt * hm4(mu, m_i1, m_jp, a.mu[mat(a, i1, jp, k)]);
  a.C[C_RZ][c] = a.dt * hm4(mu, m_i1, m_k1, a.mu[mat(a, i1, j, k1)]);
  a.C[C_TZ][c] = a.dt * hm4(mu, m_jp, m_k1, a.mu[mat(a, i, jp, k1)]);
  const float rho0 = a.rho[mat(a, i, j, k)];
  a.C[C_BR][c] = a.dt * (2.0f * rcp(rho0 + a.rho[mat(a, i1, j, k)]));
  a.C[C_BT][c] = a.dt * (2.0f * rcp(rho0 + a.rho[mat(a, i, jp, k)]));
  a.C[C_BZ][c] = a.dt * (2.0f * rcp(rho0 + a.rho[mat(a, i, j, k1)]));
}

// medium index of (i, j, k); AXI: the medium does not vary along theta
// (one row per ring), which lets the compiler share the rows' loads
template <bool AXI>
__device__ __forceinline__ size_t matx(const AdjArgs &a, int i, int j, int k)
{
  return AXI ? (size_t)i * a.m_ring + k : mat(a, i, j, k);
}

// stress-half terms of the four cells (i, j, kb..kb+3)
template <bool AXI>
__device__ __forceinline__ void stress_terms4(const AdjArgs &a, int i, int j, int kb, float (&T)[9][AW])
{
  const size_t p = at(a, i, j, kb), m = matx<AXI>(a, i, j, kb);
  float mu[AW], lam[AW], crt[AW], crz[AW], ctz[AW];
  ld4(mu, a.mu, m); ld4(lam, a.lam, m);
  ld4(crt, a.C[C_RT], m); ld4(crz, a.C[C_RZ], m); ld4(ctz, a.C[C_TZ], m);
  float grr[AW], gtt[AW], gzz[AW], srt[AW], srz[AW], stz[AW];
  ld4(grr, a.fb[SRR], p); ld4(gtt, a.fb[STT], p); ld4(gzz, a.fb[SZZ], p);
  ld4(srt, a.fb[SRT], p); ld4(srz, a.fb[SRZ], p); ld4(stz, a.fb[STZ], p);
  for (int e = 0; e < AW; e++) {
    const float gs = grr[e] + gtt[e] + gzz[e];
    T[0][e] = a.dt * (lam[e] * gs + 2.0f * mu[e] * grr[e]);
    T[1][e] = a.dt * (lam[e] * gs + 2.0f * mu[e] * gtt[e]);
    T[2][e] = a.dt * (lam[e] * gs + 2.0f * mu[e] * gzz[e]);
    T[3][e] = T[4][e] = crt[e] * srt[e];
    T[5][e] = T[6][e] = crz[e] * srz[e];
    T[7][e] = T[8][e] = ctz[e] * stz[e];
  }
}

// stress-half terms of the one cell (i, j, k)
template <bool AXI>
__device__ __forceinline__ void stress_terms1(const AdjArgs &a, int i, int j, int k, float (&T)[9])
{
  const size_t p = at(a, i, j, k);
  const size_t m = matx<AXI>(a, i, j, k);
  const float mu = a.mu[m], lam = a.lam[m];
  const float grr = a.fb[SRR][p], gtt = a.fb[STT][p], gzz = a.fb[SZZ][p];
  const float gs = grr + gtt + gzz;
  T[0] = a.dt * (lam * gs + 2.0f * mu * grr);
  T[1] = a.dt * (lam * gs + 2.0f * mu * gtt);
  T[2] = a.dt * (lam * gs + 2.0f * mu * gzz);
  T[3] = T[4] = a.C[C_RT][m] * a.fb[SRT][p];
  T[5] = T[6] = a.C[C_RZ][m] * a.fb[SRZ][p];
  T[7] = T[8] = a.C[C_TZ][m] * a.fb[STZ][p];
}

// velocity-half terms of the four cells (i, j, kb..kb+3)
template <bool AXI>
__device__ __forceinline__ void velocity_terms4(const AdjArgs &a, int i, int j, int kb, float (&T)[9][AW])
{
  const size_t p = at(a, i, j, kb), m = matx<AXI>(a, i, j, kb);
  float br[AW], bt[AW], bz[AW];
  ld4(br, a.C[C_BR], m); ld4(bt, a.C[C_BT], m); ld4(bz, a.C[C_BZ], m);
  float vr[AW], vt[AW], vz[AW];
  ld4(vr, a.fb[VR], p); ld4(vt, a.fb[VT], p); ld4(vz, a.fb[VZ], p);
  for (int e = 0; e < AW; e++) {
    T[0][e] = T[1][e] = T[2][e] = br[e] * vr[e];
    T[3][e] = T[4][e] = T[5][e] = bt[e] * vt[e];
    T[6][e] = T[7][e] = T[8][e] = bz[e] * vz[e];
  }
}

// velocity-half terms of the one cell (i, j, k)
template <bool AXI>
__device__ __forceinline__ void velocity_terms1(const AdjArgs &a, int i, int j, int k, float (&T)[9])
{
  const size_t p = at(a, i, j, k);
  const size_t m = matx<AXI>(a, i, j, k);
  T[0] = T[1] = T[2] = a.C[C_BR][m] * a.fb[VR][p];
  T[3] = T[4] = T[5] = a.C[C_BT][m] * a.fb[VT][p];
  T[6] = T[7] = T[8] = a.C[C_BZ][m] * a.fb[VZ][p];
}

// inside the slabs the stored terms replace the formed ones
__device__ __forceinline__ void slab_terms4(const AdjArgs &a, int i, int j, int kb, float (&T)[9][AW])
{
  const bool rs = i >= a.nr - a.npr;
  bool zs[AW], any = rs;
  for (int e = 0; e < AW; e++) { zs[e] = zrow(a, kb + e) >= 0; any |= zs[e]; }
  if (!any) return;
  const size_t p = at(a, i, j, kb);
  for (int t = 0; t < 9; t++) {
    float v[AW];
    ld4(v, a.T[t], p);
    for (int e = 0; e < AW; e++)
      if (rs || zs[e]) T[t][e] = v[e];
  }
}
__device__ __forceinline__ void slab_terms1(const AdjArgs &a, int i, int j, int k, float (&T)[9])
{
  if (!in_slab(a, i, k)) return;
  const size_t p = at(a, i, j, k);
  for (int t = 0; t < 9; t++) T[t] = a.T[t][p];
}

// Both fused gathers form the terms of every position they read without
// branches (a missing ring or depth neighbour is formed on a clamped valid
// index and its contribution dropped), so all loads issue together; a group
// whose positions reach a slab then swaps in the stored terms.
template <bool AXI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CW_ADJ_WAVES))) k_adj_stress_gather_f(AdjArgs a)
{
  Col c;
  if (!col(a, c) || !c.live) return;
  const int i = c.i, j = c.j, kb = c.kb;
  const float ci = a.inv_rc[i], fi = a.inv_rf[i];
  const bool has_ip = i + 1 < a.nr, has_im = i >= 1;
  const float cip = has_ip ? a.inv_rc[i + 1] : 0.0f, fim = has_im ? a.inv_rf[i - 1] : 0.0f;
  const int ip = has_ip ? i + 1 : i, im = has_im ? i - 1 : i;
  const int kbm = kb >= 1 ? kb - 1 : kb, kba = kb + AW < a.nz ? kb + AW : a.nz - 1;
  float T[9][AW], Tip[9][AW], Tim[9][AW], Tjp[9][AW], Tjm[9][AW], Tb[9], Ta[9];
  stress_terms4<AXI>(a, i, j, kb, T);
  stress_terms4<AXI>(a, i, c.jp, kb, Tjp);
  stress_terms4<AXI>(a, i, c.jm, kb, Tjm);
  stress_terms4<AXI>(a, ip, j, kb, Tip);
  stress_terms4<AXI>(a, im, j, kb, Tim);
  stress_terms1<AXI>(a, i, j, kbm, Tb);
  stress_terms1<AXI>(a, i, j, kba, Ta);
  if (ip >= a.nr - a.npr || zrow(a, kbm) >= 0 || zrow(a, kba) >= 0) {
    slab_terms4(a, i, j, kb, T);
    slab_terms4(a, i, c.jp, kb, Tjp);
    slab_terms4(a, i, c.jm, kb, Tjm);
    slab_terms4(a, ip, j, kb, Tip);
    slab_terms4(a, im, j, kb, Tim);
    slab_terms1(a, i, j, kbm, Tb);
    slab_terms1(a, i, j, kba, Ta);
  }
  float g[3][AW];
  for (int e = 0; e < AW; e++) {
    const int k = kb + e;
    float r = T[0][e] * a.inv_dr + 0.5f * ci * T[1][e];
    if (has_ip) r += -Tip[0][e] * a.inv_dr + 0.5f * cip * Tip[1][e];
    r += fi * (Tjm[4][e] - T[4][e]) * a.inv_dth;
    r -= T[6][e] * a.inv_dz;
    if (k >= 1) r += (e ? T[6][e - 1] : Tb[6]) * a.inv_dz;
    float t = ci * (T[1][e] - Tjp[1][e]) * a.inv_dth;
    t += -T[3][e] * a.inv_dr - 0.5f * fi * T[4][e];
    if (has_im) t += Tim[3][e] * a.inv_dr - 0.5f * fim * Tim[4][e];
    t -= T[8][e] * a.inv_dz;
    if (k >= 1) t += (e ? T[8][e - 1] : Tb[8]) * a.inv_dz;
    float z = T[2][e] * a.inv_dz;
    if (k + 1 < a.nz) z -= (e + 1 < AW ? T[2][e + 1] : Ta[2]) * a.inv_dz;
    z -= T[5][e] * a.inv_dr;
    if (has_im) z += Tim[5][e] * a.inv_dr;
    z += ci * (Tjm[7][e] - T[7][e]) * a.inv_dth;
    g[0][e] = r; g[1][e] = t; g[2][e] = z;
  }
  add4n<3>(a.fb + VR, c.p, g);
}

template <bool AXI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CW_ADJ_WAVES))) k_adj_velocity_gather_f(AdjArgs a)
{
  Col c;
  if (!col(a, c) || !c.live) return;
  const int i = c.i, j = c.j, kb = c.kb;
  const float ci = a.inv_rc[i], fi = a.inv_rf[i];
  const bool has_im = i >= 1, has_ip = i + 1 < a.nr;
  const float fim = has_im ? a.inv_rf[i - 1] : 0.0f, cip = has_ip ? a.inv_rc[i + 1] : 0.0f;
  const int ip = has_ip ? i + 1 : i, im = has_im ? i - 1 : i;
  const int kbm = kb >= 1 ? kb - 1 : kb, kba = kb + AW < a.nz ? kb + AW : a.nz - 1;
  float T[9][AW], Tim[9][AW], Tip[9][AW], Tjp[9][AW], Tjm[9][AW], Tb[9], Ta[9];
  velocity_terms4<AXI>(a, i, j, kb, T);
  velocity_terms4<AXI>(a, i, c.jp, kb, Tjp);
  velocity_terms4<AXI>(a, i, c.jm, kb, Tjm);
  velocity_terms4<AXI>(a, im, j, kb, Tim);
  velocity_terms4<AXI>(a, ip, j, kb, Tip);
  velocity_terms1<AXI>(a, i, j, kbm, Tb);
  velocity_terms1<AXI>(a, i, j, kba, Ta);
  if (ip >= a.nr - a.npr || zrow(a, kbm) >= 0 || zrow(a, kba) >= 0) {
    slab_terms4(a, i, j, kb, T);
    slab_terms4(a, i, c.jp, kb, Tjp);
    slab_terms4(a, i, c.jm, kb, Tjm);
    slab_terms4(a, im, j, kb, Tim);
    slab_terms4(a, ip, j, kb, Tip);
    slab_terms1(a, i, j, kbm, Tb);
    slab_terms1(a, i, j, kba, Ta);
  }
  float g[6][AW];
  for (int e = 0; e < AW; e++) {
    const int k = kb + e;
    float rr = -T[0][e] * a.inv_dr + 0.5f * fi * T[1][e];
    if (has_im) rr += Tim[0][e] * a.inv_dr + 0.5f * fim * Tim[1][e];
    float tt = -0.5f * fi * T[1][e] + ci * (Tjm[4][e] - T[4][e]) * a.inv_dth;
    if (has_im) tt -= 0.5f * fim * Tim[1][e];
    float zz = -T[8][e] * a.inv_dz;
    if (k >= 1) zz += (e ? T[8][e - 1] : Tb[8]) * a.inv_dz;
    float rt = fi * (T[1][e] - Tjp[1][e]) * a.inv_dth + T[3][e] * a.inv_dr + ci * T[4][e];
    if (has_ip) rt += -Tip[3][e] * a.inv_dr + cip * Tip[4][e];
    float rz = T[2][e] * a.inv_dz + T[6][e] * a.inv_dr + 0.5f * ci * T[7][e];
    if (k + 1 < a.nz) rz -= (e + 1 < AW ? T[2][e + 1] : Ta[2]) * a.inv_dz;
    if (has_ip) rz += -Tip[6][e] * a.inv_dr + 0.5f * cip * Tip[7][e];
    float tz = T[5][e] * a.inv_dz + ci * (T[7][e] - Tjp[7][e]) * a.inv_dth;
    if (k + 1 < a.nz) tz -= (e + 1 < AW ? T[5][e + 1] : Ta[5]) * a.inv_dz;
    g[0][e] = rr; g[1][e] = tt; g[2][e] = zz; g[3][e] = rt; g[4][e] = rz; g[5][e] = tz;
  }
  add4n<6>(a.fb + SRR, c.p, g);
}

// receivers: the loss's derivative with respect to sigma^{n+1}; weights
// w[m] = 2 p_m(t_{n+1}) * (-1 / (3 cells of the receiver)); one block, the
// receivers in order (two on one cell add in a fixed order)
__global__ void __launch_bounds__(256) k_adj_receivers(AdjArgs a, const Receiver *rec, int nrec, const float *w)
{
  for (int m = 0; m < nrec; m++) {
    const Receiver r = rec[m];
    if (r.kind == 0 && w[m] != 0.0f) {
      const int j0 = r.j < 0 ? 0 : r.j, j1 = r.j < 0 ? a.nt : r.j + 1;
      for (int j = j0 + (int)threadIdx.x; j < j1; j += blockDim.x) {
        const size_t p = at(a, r.i, j, r.k);
        a.fb[SRR][p] += w[m]; a.fb[STT][p] += w[m]; a.fb[SZZ][p] += w[m];
      }
    }
    __syncthreads();
  }
}

// d HM4 / d p at (p, q, r, s); the one-sided limit 4 when p alone is zero
__device__ __forceinline__ double dhm4(double p, double q, double r, double s)
{
  if (q == 0.0 || r == 0.0 || s == 0.0) return 0.0;
  if (p == 0.0) return 4.0;
  const double h = 4.0 / (1.0 / p + 1.0 / q + 1.0 / r + 1.0 / s);
  return h * h / (4.0 * p * p);
}

// Gradient of one step for the region's cells (one thread per cell; sums
// in float64, no atomics).  Z holds this step's strain rates of the region's
// nodes [6][ea..eb) x nt x [za..zb): e_rr, e_tt, e_zz, g_rt, g_rz, g_tz.
__global__ void __launch_bounds__(256) k_adj_gradient(AdjArgs a, AdjRegion g, const float *Z, double *glam,
                                                      double *gmu)
{
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ni = g.i1 - g.i0, nk = g.k1 - g.k0;
  if (c >= (size_t)ni * a.nt * nk) return;
  const int k = g.k0 + (int)(c % nk);
  const int j = (int)((c / nk) % a.nt);
  const int i = g.i0 + (int)(c / ((size_t)nk * a.nt));
  const int ne_i = g.eb - g.ea, ne_k = g.zb - g.za;
  const size_t nreg = (size_t)ne_i * a.nt * ne_k;
  auto zi = [&](int ii, int jj, int kk) { return ((size_t)(ii - g.ea) * a.nt + jj) * ne_k + (kk - g.za); };
  const double dt = a.dt;
  const size_t p = at(a, i, j, k), zc = zi(i, j, k);
  const double srr = a.fb[SRR][p], stt = a.fb[STT][p], szz = a.fb[SZZ][p];
  const double z0 = Z[zc], z1 = Z[nreg + zc], z2 = Z[2 * nreg + zc];
  double dl = dt * (z0 + z1 + z2) * (srr + stt + szz);
  double dm = 2.0 * dt * (z0 * srr + z1 * stt + z2 * szz);
  auto mu = [&](int ii, int jj, int kk) { return (double)a.mu[mat(a, ii, jj, kk)]; };
  const int nr1 = a.nr - 1, nz1 = a.nz - 1;
  for (int di = -1; di <= 0; di++)
    for (int dj = -1; dj <= 0; dj++) {
      // r-theta node (i+di, j+dj): cells (in, jn), (in+1, jn), (in, jn+1), (in+1, jn+1)
      const int in = i + di, jn = (j + dj + a.nt) % a.nt;
      const int ia = in + 1 < a.nr ? in + 1 : nr1, ja = (jn + 1) % a.nt;
      const size_t q = at(a, in, jn, k);
      const double gq = dt * (double)Z[3 * nreg + zi(in, jn, k)] * (double)a.fb[SRT][q];
      const double m4[4] = {mu(in, jn, k), mu(ia, jn, k), mu(in, ja, k), mu(ia, ja, k)};
      const int w = (di == 0 ? 0 : 1) + (dj == 0 ? 0 : 2);      // this cell's place among the four
      dm += gq * dhm4(m4[w], m4[(w + 1) & 3], m4[(w + 2) & 3], m4[(w + 3) & 3]);
    }
  for (int di = -1; di <= 0; di++)
    for (int dk = -1; dk <= 0; dk++) {
      // r-z node (i+di, k+dk): cells (in, kn), (in+1, kn), (in, kn+1), (in+1, kn+1)
      const int in = i + di, kn = k + dk;
      const int ia = in + 1 < a.nr ? in + 1 : nr1, ka = kn + 1 < a.nz ? kn + 1 : nz1;
      const size_t q = at(a, in, j, kn);
      const double gq = dt * (double)Z[4 * nreg + zi(in, j, kn)] * (double)a.fb[SRZ][q];
      const double m4[4] = {mu(in, j, kn), mu(ia, j, kn), mu(in, j, ka), mu(ia, j, ka)};
      const int w = (di == 0 ? 0 : 1) + (dk == 0 ? 0 : 2);
      dm += gq * dhm4(m4[w], m4[(w + 1) & 3], m4[(w + 2) & 3], m4[(w + 3) & 3]);
    }
  for (int dj = -1; dj <= 0; dj++)
    for (int dk = -1; dk <= 0; dk++) {
      // theta-z node (j+dj, k+dk): cells (jn, kn), (jn+1, kn), (jn, kn+1), (jn+1, kn+1)
      const int jn = (j + dj + a.nt) % a.nt, kn = k + dk;
      const int ja = (jn + 1) % a.nt, ka = kn + 1 < a.nz ? kn + 1 : nz1;
      const size_t q = at(a, i, jn, kn);
      const double gq = dt * (double)Z[5 * nreg + zi(i, jn, kn)] * (double)a.fb[STZ][q];
      const double m4[4] = {mu(i, jn, kn), mu(i, ja, kn), mu(i, jn, ka), mu(i, ja, ka)};
      const int w = (dj == 0 ? 0 : 1) + (dk == 0 ? 0 : 2);
      dm += gq * dhm4(m4[w], m4[(w + 1) & 3], m4[(w + 2) & 3], m4[(w + 3) & 3]);
    }
  glam[c] += dl;
  gmu[c] += dm;
}

// strain rates of the region's nodes from v^{n+1/2} (the fields in `v`)
__global__ void __launch_bounds__(256) k_adj_capture(AdjArgs a, AdjRegion g, const float *vr_, const float *vt_,
                                                     const float *vz_, float *Z)
{
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ne_i = g.eb - g.ea, ne_k = g.zb - g.za;
  const size_t nreg = (size_t)ne_i * a.nt * ne_k;
  if (c >= nreg) return;
  const int k = g.za + (int)(c % ne_k);
  const int j = (int)((c / ne_k) % a.nt);
  const int i = g.ea + (int)(c / ((size_t)ne_k * a.nt));
  auto v = [&](const float *f, int ii, int jj, int kk) -> float {
    if (ii < 0 || ii >= a.nr || kk < 0 || kk >= a.nz) return 0.0f;
    jj = (jj + a.nt) % a.nt;
    return f[at(a, ii, jj, kk)];
  };
  const float ci = a.inv_rc[i], fi = a.inv_rf[i];
  const float vr0 = v(vr_, i, j, k), vt0 = v(vt_, i, j, k), vz0 = v(vz_, i, j, k);
  const float vr_im = v(vr_, i - 1, j, k);
  Z[c] = (vr0 - vr_im) * a.inv_dr;
  Z[nreg + c] = ci * ((vt0 - v(vt_, i, j - 1, k)) * a.inv_dth + 0.5f * (vr0 + vr_im));
  Z[2 * nreg + c] = (vz0 - v(vz_, i, j, k - 1)) * a.inv_dz;
  const float vt_ip = v(vt_, i + 1, j, k);
  Z[3 * nreg + c] = (vt_ip - vt0) * a.inv_dr + fi * ((v(vr_, i, j + 1, k) - vr0) * a.inv_dth - 0.5f * (vt_ip + vt0));
  Z[4 * nreg + c] = (v(vz_, i + 1, j, k) - vz0) * a.inv_dr + (v(vr_, i, j, k + 1) - vr0) * a.inv_dz;
  Z[5 * nreg + c] = ci * (v(vz_, i, j + 1, k) - vz0) * a.inv_dth + (v(vt_, i, j, k + 1) - vt0) * a.inv_dz;
}

__global__ void k_set_step(int64_t *step, int64_t value)
{
  if (threadIdx.x == 0) *step = value;
}

dim3 grid_of(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_adjoint_step(const AdjArgs &a, const Receiver *rec, int nrec, const float *w, const AdjRegion &g,
                               const float *Z, double *glam, double *gmu, hipStream_t stream)
{
  const size_t n = (size_t)a.nr * a.nt * a.nz;
  if ((n + 255) / 256 > 0x7fffffffu) return hipErrorInvalidConfiguration;
  if (nrec > 0 && w) hipLaunchKernelGGL(k_adj_receivers, dim3(1), dim3(256), 0, stream, a, rec, nrec, w);
  const size_t nc = (size_t)(g.i1 - g.i0) * a.nt * (g.k1 - g.k0);
  if (nc) hipLaunchKernelGGL(k_adj_gradient, grid_of(nc), dim3(256), 0, stream, a, g, Z, glam, gmu);
  if (a.nz % AW == 0) {
    const size_t nb = (size_t)((a.nz / AW + 255) / 256) * a.nt * a.nr;
    if (nb > 0x7fffffffu) return hipErrorInvalidConfiguration;
    const dim3 gv((unsigned)nb);
    // terms stored only for the slab cells (one per thread), gathers four
    // cells per thread forming the other terms in place
    const size_t ns = slab_cells(a);
    const bool axi = a.m_row == 0;
    if (ns) hipLaunchKernelGGL(k_adj_stress_terms_slab, grid_of(ns), dim3(256), 0, stream, a);
    if (axi) hipLaunchKernelGGL(k_adj_stress_gather_f<true>, gv, dim3(256), 0, stream, a);
    else hipLaunchKernelGGL(k_adj_stress_gather_f<false>, gv, dim3(256), 0, stream, a);
    if (ns) hipLaunchKernelGGL(k_adj_velocity_terms_slab, grid_of(ns), dim3(256), 0, stream, a);
    if (axi) hipLaunchKernelGGL(k_adj_velocity_gather_f<true>, gv, dim3(256), 0, stream, a);
    else hipLaunchKernelGGL(k_adj_velocity_gather_f<false>, gv, dim3(256), 0, stream, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_adj_stress_terms, grid_of(n), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_adj_stress_gather, grid_of(n), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_adj_velocity_terms, grid_of(n), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_adj_velocity_gather, grid_of(n), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_adjoint_coefs(const AdjArgs &a, hipStream_t stream)
{
  const size_t n = (size_t)a.nr * a.m_ring;
  if ((n + 255) / 256 > 0x7fffffffu) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_adj_coefs, grid_of(n), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_adjoint_capture(const AdjArgs &a, const AdjRegion &g, const float *vr, const float *vt,
                                  const float *vz, float *Z, hipStream_t stream)
{
  const size_t nreg = (size_t)(g.eb - g.ea) * a.nt * (g.zb - g.za);
  hipLaunchKernelGGL(k_adj_capture, grid_of(nreg), dim3(256), 0, stream, a, g, vr, vt, vz, Z);
  return hipGetLastError();
}

hipError_t launch_set_step(int64_t *step, int64_t value, hipStream_t stream)
{
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, stream, step, value);
  return hipGetLastError();
}

}  // namespace cw
