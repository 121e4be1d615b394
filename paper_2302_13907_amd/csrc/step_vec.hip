// Two-pass time step, vectorized along depth: each thread updates VW = 4
// consecutive cells of one (ring, theta row) column with one wide load per
// array (16 B per lane in float32, 8 B in 16-bit storage) instead of VW
// single loads -- on MI355X the memory pipeline is limited by the number of
// load instructions as much as by bytes, and 2-byte loads would cost as
// much as 4-byte ones.  The depth neighbours inside a group come from the
// group itself; the one before and the one after the group are single
// loads.  Used when nz is a multiple of VW; the operators, the storage
// policies and the float16 scale tracking are those of the scalar kernels.
#include "vec_common.hpp"

namespace cw {

namespace {

using namespace vec;

template <class S>
__global__ void __launch_bounds__(256) k_velocity_vec(StepArgs a, int nbx)
{
  const int bx = blockIdx.x % nbx;
  const int k0 = (bx * 256 + threadIdx.x) * VW;
  int i, j;
  strip_column(blockIdx.x / nbx, a.nr, a.nt, i, j);
  const bool live = k0 < a.nz;
  const int kb = live ? k0 : a.nz - VW;            // dead lanes compute on a valid group, store nothing
  const int jm = j == 0 ? a.nt - 1 : j - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const float *c = a.scl_in;
  float srr0[VW], srr1[VW], stt0[VW], stt1[VW], stt_jp[VW], srt0[VW], srt_jm[VW], srt_im[VW];
  float srz0[VW], srz_im[VW], stz0[VW], stz_jm[VW], szz0[VW];
  ldv<S>(srr0, a.in[SRR], c[SRR], a, i, j, kb);
  ldv<S>(srr1, a.in[SRR], c[SRR], a, i + 1, j, kb);
  ldv<S>(stt0, a.in[STT], c[STT], a, i, j, kb);
  ldv<S>(stt1, a.in[STT], c[STT], a, i + 1, j, kb);
  ldv<S>(stt_jp, a.in[STT], c[STT], a, i, jp, kb);
  ldv<S>(srt0, a.in[SRT], c[SRT], a, i, j, kb);
  ldv<S>(srt_jm, a.in[SRT], c[SRT], a, i, jm, kb);
  ldv<S>(srt_im, a.in[SRT], c[SRT], a, i - 1, j, kb);
  ldv<S>(srz0, a.in[SRZ], c[SRZ], a, i, j, kb);
  ldv<S>(srz_im, a.in[SRZ], c[SRZ], a, i - 1, j, kb);
  ldv<S>(stz0, a.in[STZ], c[STZ], a, i, j, kb);
  ldv<S>(stz_jm, a.in[STZ], c[STZ], a, i, jm, kb);
  ldv<S>(szz0, a.in[SZZ], c[SZZ], a, i, j, kb);
  const float srz_b = ld1<S>(a.in[SRZ], c[SRZ], a, i, j, kb - 1);     // depth neighbours of the group
  const float stz_b = ld1<S>(a.in[STZ], c[STZ], a, i, j, kb - 1);
  const float szz_a = ld1<S>(a.in[SZZ], c[SZZ], a, i, j, kb + VW);
  const int i1 = i + 1 < a.nr ? i + 1 : a.nr - 1;
  float rho0[VW], rho_i1[VW], rho_jp[VW];
  ldv4(rho0, a.rho, mat(a, i, j, kb));
  ldv4(rho_i1, a.rho, mat(a, i1, j, kb));
  ldv4(rho_jp, a.rho, mat(a, i, jp, kb));
  const float rho_a = a.rho[mat(a, i, j, kb + VW < a.nz ? kb + VW : a.nz - 1)];

  const float irc = a.inv_rc[i], irf = a.inv_rf[i];
  float r_dr[VW], r_b[VW], r_dz[VW], t_dr[VW], t_b[VW], t_dz[VW], z_dr[VW], z_b[VW], z_dz[VW];
#pragma unroll
  for (int e = 0; e < VW; e++) {
    const float srz_km = e == 0 ? srz_b : srz0[e - 1];
    const float stz_km = e == 0 ? stz_b : stz0[e - 1];
    const float szz_kp = e == VW - 1 ? szz_a : szz0[e + 1];
    r_dr[e] = (srr1[e] - srr0[e]) * a.inv_dr;
    r_b[e] = irf * ((srt0[e] - srt_jm[e]) * a.inv_dth + 0.5f * (srr1[e] + srr0[e]) - 0.5f * (stt1[e] + stt0[e]));
    r_dz[e] = (srz0[e] - srz_km) * a.inv_dz;
    t_dr[e] = (srt0[e] - srt_im[e]) * a.inv_dr;
    t_b[e] = irc * ((stt_jp[e] - stt0[e]) * a.inv_dth + (srt0[e] + srt_im[e]));
    t_dz[e] = (stz0[e] - stz_km) * a.inv_dz;
    z_dr[e] = (srz0[e] - srz_im[e]) * a.inv_dr;
    z_b[e] = irc * ((stz0[e] - stz_jm[e]) * a.inv_dth + 0.5f * (srz0[e] + srz_im[e]));
    z_dz[e] = (szz_kp - szz0[e]) * a.inv_dz;
  }
  const int ir = i - (a.nr - a.npr);
  if (ir >= 0 && live) {
    const size_t q = ((size_t)ir * a.nt + j) * a.nz + kb;
    const float *T = a.tab_r;
    cpml_v(a.psi_r[R_VR_DR], q, T[AR_F * a.nr + i], T[BR_F * a.nr + i], r_dr);
    cpml_v(a.psi_r[R_VR_B], q, T[AT_F * a.nr + i], T[BT_F * a.nr + i], r_b);
    cpml_v(a.psi_r[R_VT_DR], q, T[AR_C * a.nr + i], T[BR_C * a.nr + i], t_dr);
    cpml_v(a.psi_r[R_VT_B], q, T[AT_C * a.nr + i], T[BT_C * a.nr + i], t_b);
    cpml_v(a.psi_r[R_VZ_DR], q, T[AR_C * a.nr + i], T[BR_C * a.nr + i], z_dr);
    cpml_v(a.psi_r[R_VZ_B], q, T[AT_C * a.nr + i], T[BT_C * a.nr + i], z_b);
  }
  if (live && a.npz > 0 && (kb < a.npz || kb + VW - 1 >= a.nz - 1 - a.npz)) {
    const float *T = a.tab_z;
#pragma unroll
    for (int e = 0; e < VW; e++) {
      const int k = kb + e, kz = zrow(a, k);
      if (kz < 0) continue;
      const size_t q = ((size_t)i * a.nt + j) * a.nzs + kz;
      r_dz[e] = cpml1(a.psi_z[Z_VR_DZ], q, T[AZ_C * a.nz + k], T[BZ_C * a.nz + k], r_dz[e]);
      t_dz[e] = cpml1(a.psi_z[Z_VT_DZ], q, T[AZ_C * a.nz + k], T[BZ_C * a.nz + k], t_dz[e]);
      z_dz[e] = cpml1(a.psi_z[Z_VZ_DZ], q, T[AZ_H * a.nz + k], T[BZ_H * a.nz + k], z_dz[e]);
    }
  }
  const size_t p = at(a, i, j, kb);
  float vr[VW], vt[VW], vz[VW];
  S::template ldv<VW>(vr, a.in[VR], p, c[VR]);
  S::template ldv<VW>(vt, a.in[VT], p, c[VT]);
  S::template ldv<VW>(vz, a.in[VZ], p, c[VZ]);
  float mr = 0.0f, mt = 0.0f, mz = 0.0f;
#pragma unroll
  for (int e = 0; e < VW; e++) {
    const float rho_kp = e == VW - 1 ? rho_a : rho0[e + 1];
    const float b_r = 2.0f * rcp(rho0[e] + rho_i1[e]);
    const float b_t = 2.0f * rcp(rho0[e] + rho_jp[e]);
    const float b_z = 2.0f * rcp(rho0[e] + rho_kp);
    vr[e] += a.dt * b_r * (r_dr[e] + r_b[e] + r_dz[e]);
    vt[e] += a.dt * b_t * (t_dr[e] + t_b[e] + t_dz[e]);
    vz[e] += a.dt * b_z * (z_dr[e] + z_b[e] + z_dz[e]);
    mr = fmaxf(mr, fabsf(vr[e])); mt = fmaxf(mt, fabsf(vt[e])); mz = fmaxf(mz, fabsf(vz[e]));
  }
  if (live) {
    const float *o = a.scl_out;
    S::template stv<VW>(a.out[VR], p, vr, 1.0f / o[VR]);
    S::template stv<VW>(a.out[VT], p, vt, 1.0f / o[VT]);
    S::template stv<VW>(a.out[VZ], p, vz, 1.0f / o[VZ]);
  }
  if (S::scaled) {
    track_max(a.maxabs + VR * kMaxSlots, live ? mr : 0.0f);
    track_max(a.maxabs + VT * kMaxSlots, live ? mt : 0.0f);
    track_max(a.maxabs + VZ * kMaxSlots, live ? mz : 0.0f);
  }
}

template <class S>
__global__ void __launch_bounds__(256) k_stress_vec(StepArgs a, int nbx)
{
  const int bx = blockIdx.x % nbx;
  const int k0 = (bx * 256 + threadIdx.x) * VW;
  int i, j;
  strip_column(blockIdx.x / nbx, a.nr, a.nt, i, j);
  const bool live = k0 < a.nz;
  const int kb = live ? k0 : a.nz - VW;
  const int jm = j == 0 ? a.nt - 1 : j - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const float *o = a.scl_out;                      // velocities at level n+1/2 (output buffer)
  const float *vR = a.out[VR], *vT = a.out[VT], *vZ = a.out[VZ];
  float vr0[VW], vr_im[VW], vr_jp[VW], vt0[VW], vt_jm[VW], vt_ip[VW], vz0[VW], vz_ip[VW], vz_jp[VW];
  ldv<S>(vr0, vR, o[VR], a, i, j, kb);
  ldv<S>(vr_im, vR, o[VR], a, i - 1, j, kb);
  ldv<S>(vr_jp, vR, o[VR], a, i, jp, kb);
  ldv<S>(vt0, vT, o[VT], a, i, j, kb);
  ldv<S>(vt_jm, vT, o[VT], a, i, jm, kb);
  ldv<S>(vt_ip, vT, o[VT], a, i + 1, j, kb);
  ldv<S>(vz0, vZ, o[VZ], a, i, j, kb);
  ldv<S>(vz_ip, vZ, o[VZ], a, i + 1, j, kb);
  ldv<S>(vz_jp, vZ, o[VZ], a, i, jp, kb);
  const float vr_a = ld1<S>(vR, o[VR], a, i, j, kb + VW);
  const float vt_a = ld1<S>(vT, o[VT], a, i, j, kb + VW);
  const float vz_b = ld1<S>(vZ, o[VZ], a, i, j, kb - 1);

  const float irc = a.inv_rc[i], irf = a.inv_rf[i];
  float err[VW], ett[VW], ezz[VW], rt_dr[VW], rt_b[VW], rz_dr[VW], rz_dz[VW], tz_b[VW], tz_dz[VW];
#pragma unroll
  for (int e = 0; e < VW; e++) {
    const float vr_kp = e == VW - 1 ? vr_a : vr0[e + 1];
    const float vt_kp = e == VW - 1 ? vt_a : vt0[e + 1];
    const float vz_km = e == 0 ? vz_b : vz0[e - 1];
    err[e] = (vr0[e] - vr_im[e]) * a.inv_dr;
    ett[e] = irc * ((vt0[e] - vt_jm[e]) * a.inv_dth + 0.5f * (vr0[e] + vr_im[e]));
    ezz[e] = (vz0[e] - vz_km) * a.inv_dz;
    rt_dr[e] = (vt_ip[e] - vt0[e]) * a.inv_dr;
    rt_b[e] = irf * ((vr_jp[e] - vr0[e]) * a.inv_dth - 0.5f * (vt_ip[e] + vt0[e]));
    rz_dr[e] = (vz_ip[e] - vz0[e]) * a.inv_dr;
    rz_dz[e] = (vr_kp - vr0[e]) * a.inv_dz;
    tz_b[e] = irc * (vz_jp[e] - vz0[e]) * a.inv_dth;
    tz_dz[e] = (vt_kp - vt0[e]) * a.inv_dz;
  }
  const int ir = i - (a.nr - a.npr);
  if (ir >= 0 && live) {
    const size_t q = ((size_t)ir * a.nt + j) * a.nz + kb;
    const float *T = a.tab_r;
    cpml_v(a.psi_r[R_N_DR], q, T[AR_C * a.nr + i], T[BR_C * a.nr + i], err);
    cpml_v(a.psi_r[R_N_B], q, T[AT_C * a.nr + i], T[BT_C * a.nr + i], ett);
    cpml_v(a.psi_r[R_RT_DR], q, T[AR_F * a.nr + i], T[BR_F * a.nr + i], rt_dr);
    cpml_v(a.psi_r[R_RT_B], q, T[AT_F * a.nr + i], T[BT_F * a.nr + i], rt_b);
    cpml_v(a.psi_r[R_RZ_DR], q, T[AR_F * a.nr + i], T[BR_F * a.nr + i], rz_dr);
    cpml_v(a.psi_r[R_TZ_B], q, T[AT_C * a.nr + i], T[BT_C * a.nr + i], tz_b);
  }
  if (live && a.npz > 0 && (kb < a.npz || kb + VW - 1 >= a.nz - 1 - a.npz)) {
    const float *T = a.tab_z;
#pragma unroll
    for (int e = 0; e < VW; e++) {
      const int k = kb + e, kz = zrow(a, k);
      if (kz < 0) continue;
      const size_t q = ((size_t)i * a.nt + j) * a.nzs + kz;
      ezz[e] = cpml1(a.psi_z[Z_N_DZ], q, T[AZ_C * a.nz + k], T[BZ_C * a.nz + k], ezz[e]);
      rz_dz[e] = cpml1(a.psi_z[Z_RZ_DZ], q, T[AZ_H * a.nz + k], T[BZ_H * a.nz + k], rz_dz[e]);
      tz_dz[e] = cpml1(a.psi_z[Z_TZ_DZ], q, T[AZ_H * a.nz + k], T[BZ_H * a.nz + k], tz_dz[e]);
    }
  }
  // moduli: reciprocals of mu at the cell and its neighbours (r, theta, depth)
  const int i1 = i + 1 < a.nr ? i + 1 : a.nr - 1;
  const int ka = kb + VW < a.nz ? kb + VW : a.nz - 1;   // depth neighbour of the group, clamped
  float lam[VW], mu[VW], m_i1[VW], m_jp[VW], m_i1jp[VW];
  ldv4(lam, a.lam, mat(a, i, j, kb));
  ldv4(mu, a.mu, mat(a, i, j, kb));
  ldv4(m_i1, a.mu, mat(a, i1, j, kb));
  ldv4(m_jp, a.mu, mat(a, i, jp, kb));
  ldv4(m_i1jp, a.mu, mat(a, i1, jp, kb));
  const float ia = rcp(a.mu[mat(a, i, j, ka)]), ia_i1 = rcp(a.mu[mat(a, i1, j, ka)]);
  const float ia_jp = rcp(a.mu[mat(a, i, jp, ka)]);
  float im[VW], im_i1[VW], im_jp[VW];
#pragma unroll
  for (int e = 0; e < VW; e++) { im[e] = rcp(mu[e]); im_i1[e] = rcp(m_i1[e]); im_jp[e] = rcp(m_jp[e]); }

  const size_t p = at(a, i, j, kb);
  const float *c = a.scl_in;
  float srr[VW], stt[VW], szz[VW], srt[VW], srz[VW], stz[VW];
  S::template ldv<VW>(srr, a.in[SRR], p, c[SRR]);
  S::template ldv<VW>(stt, a.in[STT], p, c[STT]);
  S::template ldv<VW>(szz, a.in[SZZ], p, c[SZZ]);
  S::template ldv<VW>(srt, a.in[SRT], p, c[SRT]);
  S::template ldv<VW>(srz, a.in[SRZ], p, c[SRZ]);
  S::template ldv<VW>(stz, a.in[STZ], p, c[STZ]);
  float mx[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < VW; e++) {
    const float ik = e == VW - 1 ? ia : im[e + 1];            // 1/mu at k+1
    const float ik_i1 = e == VW - 1 ? ia_i1 : im_i1[e + 1];
    const float ik_jp = e == VW - 1 ? ia_jp : im_jp[e + 1];
    // harmonic means, terms summed in the order of the definition
    const float mu_rt = 4.0f * rcp(im[e] + im_i1[e] + im_jp[e] + rcp(m_i1jp[e]));
    const float mu_rz = 4.0f * rcp(im[e] + im_i1[e] + ik + ik_i1);
    const float mu_tz = 4.0f * rcp(im[e] + im_jp[e] + ik + ik_jp);
    const float tr = err[e] + ett[e] + ezz[e];
    const float lt = lam[e] * tr, m2 = 2.0f * mu[e];
    srr[e] += a.dt * (lt + m2 * err[e]);
    stt[e] += a.dt * (lt + m2 * ett[e]);
    szz[e] += a.dt * (lt + m2 * ezz[e]);
    srt[e] += a.dt * mu_rt * (rt_dr[e] + rt_b[e]);
    srz[e] += a.dt * mu_rz * (rz_dr[e] + rz_dz[e]);
    stz[e] += a.dt * mu_tz * (tz_b[e] + tz_dz[e]);
    mx[0] = fmaxf(mx[0], fabsf(srr[e])); mx[1] = fmaxf(mx[1], fabsf(stt[e]));
    mx[2] = fmaxf(mx[2], fabsf(szz[e])); mx[3] = fmaxf(mx[3], fabsf(srt[e]));
    mx[4] = fmaxf(mx[4], fabsf(srz[e])); mx[5] = fmaxf(mx[5], fabsf(stz[e]));
  }
  if (live) {
    S::template stv<VW>(a.out[SRR], p, srr, 1.0f / o[SRR]);
    S::template stv<VW>(a.out[STT], p, stt, 1.0f / o[STT]);
    S::template stv<VW>(a.out[SZZ], p, szz, 1.0f / o[SZZ]);
    S::template stv<VW>(a.out[SRT], p, srt, 1.0f / o[SRT]);
    S::template stv<VW>(a.out[SRZ], p, srz, 1.0f / o[SRZ]);
    S::template stv<VW>(a.out[STZ], p, stz, 1.0f / o[STZ]);
  }
  if (S::scaled) {
#pragma unroll
    for (int q = 0; q < 6; q++) track_max(a.maxabs + (SRR + q) * kMaxSlots, live ? mx[q] : 0.0f);
  }
}

template <class F>
hipError_t dispatch(int storage, F &&f)
{
  switch (storage) {
  case ST_F32: return f(StF32{});
  case ST_F16: return f(StF16{});
  case ST_BF16: return f(StBF16{});
  default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool vec_applies(int nz) { return nz % VW == 0 && nz >= VW; }

hipError_t launch_velocity_vec(const StepArgs &a, int storage, hipStream_t stream)
{
  const int nbx = (a.nz / VW + 255) / 256;
  const long g = (long)nbx * a.nt * a.nr;
  if (g > 0x7fffffff || !vec_applies(a.nz)) return hipErrorInvalidConfiguration;
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_velocity_vec<decltype(s)>, dim3((unsigned)g), dim3(256), 0, stream, a, nbx);
    return hipGetLastError();
  });
}

hipError_t launch_stress_vec(const StepArgs &a, int storage, hipStream_t stream)
{
  const int nbx = (a.nz / VW + 255) / 256;
  const long g = (long)nbx * a.nt * a.nr;
  if (g > 0x7fffffff || !vec_applies(a.nz)) return hipErrorInvalidConfiguration;
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_stress_vec<decltype(s)>, dim3((unsigned)g), dim3(256), 0, stream, a, nbx);
    return hipGetLastError();
  });
}

}  // namespace cw
