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
  return ((size_t)i * a.nt + j) * a.nz + k;
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
// from out's adjoint and psi''s adjoint (in *pb) returns X's adjoint and
// leaves psi's adjoint in *pb
__device__ __forceinline__ float sadj(float *pb, float ca, float cb, float outb)
{
  const float t = *pb + outb;
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

// stress half-step, terms: T = (e_rr, e_tt bracket, e_zz, rt_dr, rt_b, rz_dr, rz_dz, tz_b, tz_dz) adjoints
__global__ void __launch_bounds__(256) k_adj_stress_terms(AdjArgs a)
{
  int i, j, k;
  if (!cell(a, i, j, k)) return;
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
    err = sadj(&a.pr[R_N_DR][q], T[AR_C * a.nr + i], T[BR_C * a.nr + i], err);
    ett = sadj(&a.pr[R_N_B][q], T[AT_C * a.nr + i], T[BT_C * a.nr + i], ett);
    rt_dr = sadj(&a.pr[R_RT_DR][q], T[AR_F * a.nr + i], T[BR_F * a.nr + i], zrt);
    rt_b = sadj(&a.pr[R_RT_B][q], T[AT_F * a.nr + i], T[BT_F * a.nr + i], zrt);
    rz_dr = sadj(&a.pr[R_RZ_DR][q], T[AR_F * a.nr + i], T[BR_F * a.nr + i], zrz);
    tz_b = sadj(&a.pr[R_TZ_B][q], T[AT_C * a.nr + i], T[BT_C * a.nr + i], ztz);
  }
  const int kz = zrow(a, k);
  if (kz >= 0) {
    const size_t q = ((size_t)i * a.nt + j) * a.nzs + kz;
    const float *T = a.tab_z;
    ezz = sadj(&a.pz[Z_N_DZ][q], T[AZ_C * a.nz + k], T[BZ_C * a.nz + k], ezz);
    rz_dz = sadj(&a.pz[Z_RZ_DZ][q], T[AZ_H * a.nz + k], T[BZ_H * a.nz + k], zrz);
    tz_dz = sadj(&a.pz[Z_TZ_DZ][q], T[AZ_H * a.nz + k], T[BZ_H * a.nz + k], ztz);
  }
  a.T[0][p] = err; a.T[1][p] = ett; a.T[2][p] = ezz;
  a.T[3][p] = rt_dr; a.T[4][p] = rt_b; a.T[5][p] = rz_dr;
  a.T[6][p] = rz_dz; a.T[7][p] = tz_b; a.T[8][p] = tz_dz;
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
__global__ void __launch_bounds__(256) k_adj_velocity_terms(AdjArgs a)
{
  int i, j, k;
  if (!cell(a, i, j, k)) return;
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
    r_dr = sadj(&a.pr[R_VR_DR][q], T[AR_F * a.nr + i], T[BR_F * a.nr + i], wr);
    r_b = sadj(&a.pr[R_VR_B][q], T[AT_F * a.nr + i], T[BT_F * a.nr + i], wr);
    t_dr = sadj(&a.pr[R_VT_DR][q], T[AR_C * a.nr + i], T[BR_C * a.nr + i], wt);
    t_b = sadj(&a.pr[R_VT_B][q], T[AT_C * a.nr + i], T[BT_C * a.nr + i], wt);
    z_dr = sadj(&a.pr[R_VZ_DR][q], T[AR_C * a.nr + i], T[BR_C * a.nr + i], wz);
    z_b = sadj(&a.pr[R_VZ_B][q], T[AT_C * a.nr + i], T[BT_C * a.nr + i], wz);
  }
  const int kz = zrow(a, k);
  if (kz >= 0) {
    const size_t q = ((size_t)i * a.nt + j) * a.nzs + kz;
    const float *T = a.tab_z;
    r_dz = sadj(&a.pz[Z_VR_DZ][q], T[AZ_C * a.nz + k], T[BZ_C * a.nz + k], wr);
    t_dz = sadj(&a.pz[Z_VT_DZ][q], T[AZ_C * a.nz + k], T[BZ_C * a.nz + k], wt);
    z_dz = sadj(&a.pz[Z_VZ_DZ][q], T[AZ_H * a.nz + k], T[BZ_H * a.nz + k], wz);
  }
  a.T[0][p] = r_dr; a.T[1][p] = r_b; a.T[2][p] = r_dz;
  a.T[3][p] = t_dr; a.T[4][p] = t_b; a.T[5][p] = t_dz;
  a.T[6][p] = z_dr; a.T[7][p] = z_b; a.T[8][p] = z_dz;
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
  c.ring = (size_t)a.nt * a.nz;
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
__device__ __forceinline__ void add4(float *f, size_t q, const float (&v)[AW])
{
  float o[AW];
  ld4(o, f, q);
  for (int e = 0; e < AW; e++) o[e] += v[e];
  st4(f, q, o);
}
__global__ void __launch_bounds__(256) k_adj_stress_gather_v(AdjArgs a)
{
  Col c;
  if (!col(a, c) || !c.live) return;               // a write-only pass: dead lanes have nothing to do
  const int i = c.i, kb = c.kb;
  const float ci = a.inv_rc[i], fi = a.inv_rf[i];
  float *const *T = a.T;
  const bool has_ip = i + 1 < a.nr, has_im = i >= 1;
  const size_t pip = c.p + c.ring, pim = c.p - c.ring;
  const float cip = has_ip ? a.inv_rc[i + 1] : 0.0f, fim = has_im ? a.inv_rf[i - 1] : 0.0f;
  float t0[AW], t0i[AW], t1[AW], t1i[AW], t1jp[AW], t4[AW], t4jm[AW], t4m[AW], t6[AW], t3[AW], t3m[AW], t8[AW];
  float t2[AW], t5[AW], t5m[AW], t7[AW], t7jm[AW];
  ld4(t0, T[0], c.p); ld4(t1, T[1], c.p); ld4(t1jp, T[1], c.pjp);
  ld4(t4, T[4], c.p); ld4(t4jm, T[4], c.pjm); ld4(t6, T[6], c.p);
  ld4(t3, T[3], c.p); ld4(t8, T[8], c.p); ld4(t2, T[2], c.p); ld4(t5, T[5], c.p);
  ld4(t7, T[7], c.p); ld4(t7jm, T[7], c.pjm);
  if (has_ip) { ld4(t0i, T[0], pip); ld4(t1i, T[1], pip); }
  if (has_im) { ld4(t4m, T[4], pim); ld4(t3m, T[3], pim); ld4(t5m, T[5], pim); }
  const float t6b = kb >= 1 ? T[6][c.p - 1] : 0.0f, t8b = kb >= 1 ? T[8][c.p - 1] : 0.0f;
  const float t2a = kb + AW < a.nz ? T[2][c.p + AW] : 0.0f;
  float gr[AW], gt[AW], gz[AW];
  for (int e = 0; e < AW; e++) {
    const int k = kb + e;
    float r = t0[e] * a.inv_dr + 0.5f * ci * t1[e];
    if (has_ip) r += -t0i[e] * a.inv_dr + 0.5f * cip * t1i[e];
    r += fi * (t4jm[e] - t4[e]) * a.inv_dth;
    r -= t6[e] * a.inv_dz;
    if (k >= 1) r += (e ? t6[e - 1] : t6b) * a.inv_dz;
    float t = ci * (t1[e] - t1jp[e]) * a.inv_dth;
    t += -t3[e] * a.inv_dr - 0.5f * fi * t4[e];
    if (has_im) t += t3m[e] * a.inv_dr - 0.5f * fim * t4m[e];
    t -= t8[e] * a.inv_dz;
    if (k >= 1) t += (e ? t8[e - 1] : t8b) * a.inv_dz;
    float z = t2[e] * a.inv_dz;
    if (k + 1 < a.nz) z -= (e + 1 < AW ? t2[e + 1] : t2a) * a.inv_dz;
    z -= t5[e] * a.inv_dr;
    if (has_im) z += t5m[e] * a.inv_dr;
    z += ci * (t7jm[e] - t7[e]) * a.inv_dth;
    gr[e] = r; gt[e] = t; gz[e] = z;
  }
  add4(a.fb[VR], c.p, gr);
  add4(a.fb[VT], c.p, gt);
  add4(a.fb[VZ], c.p, gz);
}

__global__ void __launch_bounds__(256) k_adj_velocity_gather_v(AdjArgs a)
{
  Col c;
  if (!col(a, c) || !c.live) return;
  const int i = c.i, kb = c.kb;
  const float ci = a.inv_rc[i], fi = a.inv_rf[i];
  float *const *T = a.T;
  const bool has_im = i >= 1, has_ip = i + 1 < a.nr;
  const size_t pim = c.p - c.ring, pip = c.p + c.ring;
  const float fim = has_im ? a.inv_rf[i - 1] : 0.0f, cip = has_ip ? a.inv_rc[i + 1] : 0.0f;
  float t0[AW], t0m[AW], t1[AW], t1m[AW], t1jp[AW], t4[AW], t4jm[AW], t4p[AW], t8[AW], t3[AW], t3p[AW];
  float t2[AW], t6[AW], t6p[AW], t7[AW], t7p[AW], t7jp[AW], t5[AW];
  ld4(t0, T[0], c.p); ld4(t1, T[1], c.p); ld4(t1jp, T[1], c.pjp);
  ld4(t4, T[4], c.p); ld4(t4jm, T[4], c.pjm); ld4(t8, T[8], c.p);
  ld4(t3, T[3], c.p); ld4(t2, T[2], c.p); ld4(t6, T[6], c.p);
  ld4(t7, T[7], c.p); ld4(t7jp, T[7], c.pjp); ld4(t5, T[5], c.p);
  if (has_im) { ld4(t0m, T[0], pim); ld4(t1m, T[1], pim); }
  if (has_ip) { ld4(t3p, T[3], pip); ld4(t4p, T[4], pip); ld4(t6p, T[6], pip); ld4(t7p, T[7], pip); }
  const float t8b = kb >= 1 ? T[8][c.p - 1] : 0.0f;
  const bool in_a = kb + AW < a.nz;
  const float t2a = in_a ? T[2][c.p + AW] : 0.0f, t5a = in_a ? T[5][c.p + AW] : 0.0f;
  float g[6][AW];
  for (int e = 0; e < AW; e++) {
    const int k = kb + e;
    float rr = -t0[e] * a.inv_dr + 0.5f * fi * t1[e];
    if (has_im) rr += t0m[e] * a.inv_dr + 0.5f * fim * t1m[e];
    float tt = -0.5f * fi * t1[e] + ci * (t4jm[e] - t4[e]) * a.inv_dth;
    if (has_im) tt -= 0.5f * fim * t1m[e];
    float zz = -t8[e] * a.inv_dz;
    if (k >= 1) zz += (e ? t8[e - 1] : t8b) * a.inv_dz;
    float rt = fi * (t1[e] - t1jp[e]) * a.inv_dth + t3[e] * a.inv_dr + ci * t4[e];
    if (has_ip) rt += -t3p[e] * a.inv_dr + cip * t4p[e];
    float rz = t2[e] * a.inv_dz + t6[e] * a.inv_dr + 0.5f * ci * t7[e];
    if (k + 1 < a.nz) rz -= (e + 1 < AW ? t2[e + 1] : t2a) * a.inv_dz;
    if (has_ip) rz += -t6p[e] * a.inv_dr + 0.5f * cip * t7p[e];
    float tz = t5[e] * a.inv_dz + ci * (t7[e] - t7jp[e]) * a.inv_dth;
    if (k + 1 < a.nz) tz -= (e + 1 < AW ? t5[e + 1] : t5a) * a.inv_dz;
    g[0][e] = rr; g[1][e] = tt; g[2][e] = zz; g[3][e] = rt; g[4][e] = rz; g[5][e] = tz;
  }
  for (int q = 0; q < 6; q++) add4(a.fb[SRR + q], c.p, g[q]);
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
    // terms one cell per thread (pointwise: measured on MI355X at 128 x 64 x 2048,
    // a four-cells-per-thread form was slower, 268 vs 211 us and 224 vs 175 us),
    // gathers four cells per thread (their depth neighbours come from registers:
    // 210 vs 316 us and 285 vs 434 us)
    hipLaunchKernelGGL(k_adj_stress_terms, grid_of(n), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_adj_stress_gather_v, gv, dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_adj_velocity_terms, grid_of(n), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_adj_velocity_gather_v, gv, dim3(256), 0, stream, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_adj_stress_terms, grid_of(n), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_adj_stress_gather, grid_of(n), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_adj_velocity_terms, grid_of(n), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(k_adj_velocity_gather, grid_of(n), dim3(256), 0, stream, a);
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
