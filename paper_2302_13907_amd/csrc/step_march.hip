// Two-pass time step, radial-march form.  Each wavefront owns one theta row
// j and a depth range of 64 x VW cells (VW consecutive cells per lane) and
// walks outward through a range of rings, updating ring i before ring i+1.
// The radial neighbours a cell needs (ring i+1 for the velocity update,
// ring i-1 and ring i+1 for the stress update) stay in registers from one
// ring to the next, so every array is fetched from memory once per step;
// the theta neighbours (rows j-1 and j+1, owned by the neighbouring
// wavefronts, which walk the same rings at the same time) are read again
// and come from the L2 cache.  No LDS and no barriers: wavefronts are
// independent.  All workgroups start on the same ring, so at any moment the
// chip streams through a few rings of each array -- compact address ranges.
//
// Operators, storage policies and float16 scale tracking are those of the
// column kernels, expression for expression (results agree to float32
// rounding: the compiler may contract the two differently).
#include "vec_common.hpp"

namespace cw {

namespace {

using namespace vec;

#ifndef CW_MARCH_TJ
#define CW_MARCH_TJ 4
#endif
#ifndef CW_MARCH_WAVES
#define CW_MARCH_WAVES 4                        // wavefronts per SIMD the register budget is sized for
#endif
#ifndef CW_MARCH_BLOCKS
#define CW_MARCH_BLOCKS 1024
#endif
constexpr int TJ = CW_MARCH_TJ;                // wavefronts (theta rows) per workgroup
constexpr int kTargetBlocks = CW_MARCH_BLOCKS; // radial segments are added until the grid has this many workgroups
constexpr int kMinRings = 8;                   // shortest radial segment

struct MarchGrid {
  int nzb;     // depth groups of 64 x VW cells
  int njt;     // theta tiles of TJ rows
  int rseg;    // rings per radial segment
  long blocks;
};

// Workgroup b: depth group b % nzb (fastest), theta tile, then radial
// segment.  Consecutive workgroups go to different XCDs; the workgroups of
// one theta tile's depth groups that share an XCD are nzb apart.
__device__ __forceinline__ void march_decode(const StepArgs &a, int nzb, int njt, int rseg, int &kb, bool &live,
                                             int &j, int &i0, int &i1)
{
  const int zc = blockIdx.x % nzb;
  const int rest = blockIdx.x / nzb;
  const int jt = rest % njt, rs = rest / njt;
  j = __builtin_amdgcn_readfirstlane(jt * TJ + (threadIdx.x >> 6));   // one row per wavefront
  const int k0 = (zc * 64 + (threadIdx.x & 63)) * VW;
  live = k0 < a.nz;
  kb = live ? k0 : a.nz - VW;                    // dead lanes compute on a valid group, store nothing
  i0 = rs * rseg;
  i1 = i0 + rseg < a.nr ? i0 + rseg : a.nr;
}

template <class S>
__global__ void __launch_bounds__(TJ * 64) __attribute__((amdgpu_waves_per_eu(CW_MARCH_WAVES)))
k_velocity_march(StepArgs a, int nzb, int njt, int rseg)
{
  int kb, j, i0, i1;
  bool live;
  march_decode(a, nzb, njt, rseg, kb, live, j, i0, i1);
  if (j >= a.nt) return;                         // whole wavefront: no barriers in this kernel
  const int jm = j == 0 ? a.nt - 1 : j - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const Lanes<S> L(a, kb, j, jm, jp);
  const float *c = a.scl_in;

  // ring i values carried from the previous ring (as its "i + 1" values)
  float srr0[VW], stt0[VW], stt0_jp[VW], rho0[VW], rho0_jp[VW];
  // ring i - 1 values carried from the previous ring (as its own values)
  float srt_im[VW], srz_im[VW];
  ldf<S>(srr0, L, a, a.in[SRR], c[SRR], i0, L.sj);
  ldf<S>(stt0, L, a, a.in[STT], c[STT], i0, L.sj);
  ldf<S>(stt0_jp, L, a, a.in[STT], c[STT], i0, L.sjp);
  ldb4(rho0, L.med(a.rho, i0), L.m0, L.mj);
  ldb4(rho0_jp, L.med(a.rho, i0), L.m0, L.mjp);
  ldf<S>(srt_im, L, a, a.in[SRT], c[SRT], i0 - 1, L.sj);
  ldf<S>(srz_im, L, a, a.in[SRZ], c[SRZ], i0 - 1, L.sj);
  float mr = 0.0f, mt = 0.0f, mz = 0.0f;

  for (int i = i0; i < i1; i++) {
    const int i1c = i + 1 < a.nr ? i + 1 : a.nr - 1;
    float srr1[VW], stt1[VW], stt1_jp[VW], rho1[VW], rho1_jp[VW];
    ldf<S>(srr1, L, a, a.in[SRR], c[SRR], i + 1, L.sj);    // zero beyond the last ring
    ldf<S>(stt1, L, a, a.in[STT], c[STT], i + 1, L.sj);
    ldf<S>(stt1_jp, L, a, a.in[STT], c[STT], i + 1, L.sjp);
    const rsrc_t rho_n = L.med(a.rho, i1c);                // medium index clamped at the edge
    ldb4(rho1, rho_n, L.m0, L.mj);
    ldb4(rho1_jp, rho_n, L.m0, L.mjp);
    const rsrc_t R_srt = L.field(a.in[SRT], i), R_srz = L.field(a.in[SRZ], i);
    const rsrc_t R_stz = L.field(a.in[STZ], i), R_szz = L.field(a.in[SZZ], i);
    float srt0[VW], srt_jm[VW], srz0[VW], stz0[VW], stz_jm[VW], szz0[VW];
    S::ldb(srt0, R_srt, L.v0, L.sj, c[SRT]);
    S::ldb(srt_jm, R_srt, L.v0, L.sjm, c[SRT]);
    S::ldb(srz0, R_srz, L.v0, L.sj, c[SRZ]);
    S::ldb(stz0, R_stz, L.v0, L.sj, c[STZ]);
    S::ldb(stz_jm, R_stz, L.v0, L.sjm, c[STZ]);
    S::ldb(szz0, R_szz, L.v0, L.sj, c[SZZ]);
    // depth neighbours of the group (zero outside the grid)
    const float srz_b = L.has_b ? S::ldb1(R_srz, L.vb, L.sj, c[SRZ]) : 0.0f;
    const float stz_b = L.has_b ? S::ldb1(R_stz, L.vb, L.sj, c[STZ]) : 0.0f;
    const float szz_a = L.has_a ? S::ldb1(R_szz, L.va, L.sj, c[SZZ]) : 0.0f;
    const float rho_a = ldb1(L.med(a.rho, i), L.ma, L.mj);
    const rsrc_t R_vr = L.field(a.in[VR], i), R_vt = L.field(a.in[VT], i), R_vz = L.field(a.in[VZ], i);
    float vr[VW], vt[VW], vz[VW];
    S::ldbu(vr, R_vr, L.v0, L.sj, c[VR]);
    S::ldbu(vt, R_vt, L.v0, L.sj, c[VT]);
    S::ldbu(vz, R_vz, L.v0, L.sj, c[VZ]);

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
      t_b[e] = irc * ((stt0_jp[e] - stt0[e]) * a.inv_dth + (srt0[e] + srt_im[e]));
      t_dz[e] = (stz0[e] - stz_km) * a.inv_dz;
      z_dr[e] = (srz0[e] - srz_im[e]) * a.inv_dr;
      z_b[e] = irc * ((stz0[e] - stz_jm[e]) * a.inv_dth + 0.5f * (srz0[e] + srz_im[e]));
      z_dz[e] = (szz_kp - szz0[e]) * a.inv_dz;
    }
    const int ir = i - (a.nr - a.npr);
    if (ir >= 0 && live) {
      const float *T = a.tab_r;
      cpml_b(L.f32(a.psi_r[R_VR_DR], ir), L.m0, L.tj, T[AR_F * a.nr + i], T[BR_F * a.nr + i], r_dr);
      cpml_b(L.f32(a.psi_r[R_VR_B], ir), L.m0, L.tj, T[AT_F * a.nr + i], T[BT_F * a.nr + i], r_b);
      cpml_b(L.f32(a.psi_r[R_VT_DR], ir), L.m0, L.tj, T[AR_C * a.nr + i], T[BR_C * a.nr + i], t_dr);
      cpml_b(L.f32(a.psi_r[R_VT_B], ir), L.m0, L.tj, T[AT_C * a.nr + i], T[BT_C * a.nr + i], t_b);
      cpml_b(L.f32(a.psi_r[R_VZ_DR], ir), L.m0, L.tj, T[AR_C * a.nr + i], T[BR_C * a.nr + i], z_dr);
      cpml_b(L.f32(a.psi_r[R_VZ_B], ir), L.m0, L.tj, T[AT_C * a.nr + i], T[BT_C * a.nr + i], z_b);
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
#pragma unroll
    for (int e = 0; e < VW; e++) {
      const float rho_kp = e == VW - 1 ? rho_a : rho0[e + 1];
      const float b_r = 2.0f * rcp(rho0[e] + rho1[e]);
      const float b_t = 2.0f * rcp(rho0[e] + rho0_jp[e]);
      const float b_z = 2.0f * rcp(rho0[e] + rho_kp);
      vr[e] += a.dt * b_r * (r_dr[e] + r_b[e] + r_dz[e]);
      vt[e] += a.dt * b_t * (t_dr[e] + t_b[e] + t_dz[e]);
      vz[e] += a.dt * b_z * (z_dr[e] + z_b[e] + z_dz[e]);
      mr = fmaxf(mr, fabsf(vr[e])); mt = fmaxf(mt, fabsf(vt[e])); mz = fmaxf(mz, fabsf(vz[e]));
    }
    if (live) {
      const float *o = a.scl_out;
      S::stb(L.fieldw(a.out[VR], i), L.v0, L.sj, vr, 1.0f / o[VR]);
      S::stb(L.fieldw(a.out[VT], i), L.v0, L.sj, vt, 1.0f / o[VT]);
      S::stb(L.fieldw(a.out[VZ], i), L.v0, L.sj, vz, 1.0f / o[VZ]);
    }
#pragma unroll
    for (int e = 0; e < VW; e++) {
      srr0[e] = srr1[e]; stt0[e] = stt1[e]; stt0_jp[e] = stt1_jp[e];
      rho0[e] = rho1[e]; rho0_jp[e] = rho1_jp[e];
      srt_im[e] = srt0[e]; srz_im[e] = srz0[e];
    }
  }
  if (S::scaled) {
    track_max(a.maxabs + VR * kMaxSlots, live ? mr : 0.0f);
    track_max(a.maxabs + VT * kMaxSlots, live ? mt : 0.0f);
    track_max(a.maxabs + VZ * kMaxSlots, live ? mz : 0.0f);
  }
}

template <class S>
__global__ void __launch_bounds__(TJ * 64) __attribute__((amdgpu_waves_per_eu(CW_MARCH_WAVES)))
k_stress_march(StepArgs a, int nzb, int njt, int rseg)
{
  int kb, j, i0, i1;
  bool live;
  march_decode(a, nzb, njt, rseg, kb, live, j, i0, i1);
  if (j >= a.nt) return;
  const int jm = j == 0 ? a.nt - 1 : j - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const Lanes<S> L(a, kb, j, jm, jp);
  const float *o = a.scl_out;                      // velocities at level n+1/2 (output buffer)
  const float *vR = a.out[VR], *vT = a.out[VT], *vZ = a.out[VZ];

  // carried: v_r of ring i - 1; v_t, v_z, mu of ring i (rows j and j + 1), 1/mu after the group
  float vr_im[VW], vt0[VW], vz0[VW], mu0[VW], mu0_jp[VW];
  ldf<S>(vr_im, L, a, vR, o[VR], i0 - 1, L.sj);
  ldf<S>(vt0, L, a, vT, o[VT], i0, L.sj);
  ldf<S>(vz0, L, a, vZ, o[VZ], i0, L.sj);
  {
    const rsrc_t m = L.med(a.mu, i0);
    ldb4(mu0, m, L.m0, L.mj);
    ldb4(mu0_jp, m, L.m0, L.mjp);
  }
  float ia0 = rcp(ldb1(L.med(a.mu, i0), L.ma, L.mj)), ia0_jp = rcp(ldb1(L.med(a.mu, i0), L.ma, L.mjp));
  float mx[6] = {0, 0, 0, 0, 0, 0};

  for (int i = i0; i < i1; i++) {
    const int i1c = i + 1 < a.nr ? i + 1 : a.nr - 1;
    const rsrc_t R_vr = L.field(vR, i), R_vt = L.field(vT, i), R_vz = L.field(vZ, i);
    float vr0[VW], vr_jp[VW], vt_jm[VW], vt_ip[VW], vz_ip[VW], vz_jp[VW];
    S::ldb(vr0, R_vr, L.v0, L.sj, o[VR]);
    S::ldb(vr_jp, R_vr, L.v0, L.sjp, o[VR]);
    S::ldb(vt_jm, R_vt, L.v0, L.sjm, o[VT]);
    ldf<S>(vt_ip, L, a, vT, o[VT], i + 1, L.sj);          // zero beyond the last ring
    ldf<S>(vz_ip, L, a, vZ, o[VZ], i + 1, L.sj);
    S::ldb(vz_jp, R_vz, L.v0, L.sjp, o[VZ]);
    const float vr_a = L.has_a ? S::ldb1(R_vr, L.va, L.sj, o[VR]) : 0.0f;
    const float vt_a = L.has_a ? S::ldb1(R_vt, L.va, L.sj, o[VT]) : 0.0f;
    const float vz_b = L.has_b ? S::ldb1(R_vz, L.vb, L.sj, o[VZ]) : 0.0f;
    float lam[VW], mu1[VW], mu1_jp[VW];
    ldb4(lam, L.med(a.lam, i), L.m0, L.mj);
    const rsrc_t R_mu1 = L.med(a.mu, i1c);                // medium index clamped at the edge
    ldb4(mu1, R_mu1, L.m0, L.mj);
    ldb4(mu1_jp, R_mu1, L.m0, L.mjp);
    const float ia1 = rcp(ldb1(R_mu1, L.ma, L.mj)), ia1_jp = rcp(ldb1(R_mu1, L.ma, L.mjp));
    const float *c = a.scl_in;
    float srr[VW], stt[VW], szz[VW], srt[VW], srz[VW], stz[VW];
    S::ldbu(srr, L.field(a.in[SRR], i), L.v0, L.sj, c[SRR]);
    S::ldbu(stt, L.field(a.in[STT], i), L.v0, L.sj, c[STT]);
    S::ldbu(szz, L.field(a.in[SZZ], i), L.v0, L.sj, c[SZZ]);
    S::ldbu(srt, L.field(a.in[SRT], i), L.v0, L.sj, c[SRT]);
    S::ldbu(srz, L.field(a.in[SRZ], i), L.v0, L.sj, c[SRZ]);
    S::ldbu(stz, L.field(a.in[STZ], i), L.v0, L.sj, c[STZ]);

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
      const float *T = a.tab_r;
      cpml_b(L.f32(a.psi_r[R_N_DR], ir), L.m0, L.tj, T[AR_C * a.nr + i], T[BR_C * a.nr + i], err);
      cpml_b(L.f32(a.psi_r[R_N_B], ir), L.m0, L.tj, T[AT_C * a.nr + i], T[BT_C * a.nr + i], ett);
      cpml_b(L.f32(a.psi_r[R_RT_DR], ir), L.m0, L.tj, T[AR_F * a.nr + i], T[BR_F * a.nr + i], rt_dr);
      cpml_b(L.f32(a.psi_r[R_RT_B], ir), L.m0, L.tj, T[AT_F * a.nr + i], T[BT_F * a.nr + i], rt_b);
      cpml_b(L.f32(a.psi_r[R_RZ_DR], ir), L.m0, L.tj, T[AR_F * a.nr + i], T[BR_F * a.nr + i], rz_dr);
      cpml_b(L.f32(a.psi_r[R_TZ_B], ir), L.m0, L.tj, T[AT_C * a.nr + i], T[BT_C * a.nr + i], tz_b);
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
    float im[VW], im_i1[VW], im_jp[VW];
#pragma unroll
    for (int e = 0; e < VW; e++) { im[e] = rcp(mu0[e]); im_i1[e] = rcp(mu1[e]); im_jp[e] = rcp(mu0_jp[e]); }
#pragma unroll
    for (int e = 0; e < VW; e++) {
      const float ik = e == VW - 1 ? ia0 : im[e + 1];            // 1/mu at k+1
      const float ik_i1 = e == VW - 1 ? ia1 : im_i1[e + 1];
      const float ik_jp = e == VW - 1 ? ia0_jp : im_jp[e + 1];
      // harmonic means, terms summed in the order of the definition
      const float mu_rt = 4.0f * rcp(im[e] + im_i1[e] + im_jp[e] + rcp(mu1_jp[e]));
      const float mu_rz = 4.0f * rcp(im[e] + im_i1[e] + ik + ik_i1);
      const float mu_tz = 4.0f * rcp(im[e] + im_jp[e] + ik + ik_jp);
      const float tr = err[e] + ett[e] + ezz[e];
      const float lt = lam[e] * tr, m2 = 2.0f * mu0[e];
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
      S::stb(L.fieldw(a.out[SRR], i), L.v0, L.sj, srr, 1.0f / o[SRR]);
      S::stb(L.fieldw(a.out[STT], i), L.v0, L.sj, stt, 1.0f / o[STT]);
      S::stb(L.fieldw(a.out[SZZ], i), L.v0, L.sj, szz, 1.0f / o[SZZ]);
      S::stb(L.fieldw(a.out[SRT], i), L.v0, L.sj, srt, 1.0f / o[SRT]);
      S::stb(L.fieldw(a.out[SRZ], i), L.v0, L.sj, srz, 1.0f / o[SRZ]);
      S::stb(L.fieldw(a.out[STZ], i), L.v0, L.sj, stz, 1.0f / o[STZ]);
    }
#pragma unroll
    for (int e = 0; e < VW; e++) {
      vr_im[e] = vr0[e]; vt0[e] = vt_ip[e]; vz0[e] = vz_ip[e];
      mu0[e] = mu1[e]; mu0_jp[e] = mu1_jp[e];
    }
    ia0 = ia1; ia0_jp = ia1_jp;
  }
  if (S::scaled) {
#pragma unroll
    for (int q = 0; q < 6; q++) track_max(a.maxabs + (SRR + q) * kMaxSlots, live ? mx[q] : 0.0f);
  }
}

MarchGrid march_grid(const StepArgs &a)
{
  MarchGrid g;
  g.nzb = (a.nz / VW + 63) / 64;
  g.njt = (a.nt + TJ - 1) / TJ;
  const long cols = (long)g.nzb * g.njt;
  long nseg = (kTargetBlocks + cols - 1) / cols;
  const long max_seg = a.nr / kMinRings > 1 ? a.nr / kMinRings : 1;
  if (nseg > max_seg) nseg = max_seg;
  if (nseg < 1) nseg = 1;
  g.rseg = (int)((a.nr + nseg - 1) / nseg);
  nseg = (a.nr + g.rseg - 1) / g.rseg;
  g.blocks = cols * nseg;
  return g;
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

// a ring of one float32 array must fit a buffer resource (byte offsets below 2^31)
bool march_applies(int nt, int nz) { return vec_applies(nt, nz) && (uint64_t)nt * nz * 4 <= 0x7fffffffull; }

hipError_t launch_velocity_march(const StepArgs &a, int storage, hipStream_t stream)
{
  const MarchGrid g = march_grid(a);
  if (g.blocks > 0x7fffffff || !march_applies(a.nt, a.nz)) return hipErrorInvalidConfiguration;
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_velocity_march<decltype(s)>, dim3((unsigned)g.blocks), dim3(TJ * 64), 0, stream, a,
                       g.nzb, g.njt, g.rseg);
    return hipGetLastError();
  });
}

hipError_t launch_stress_march(const StepArgs &a, int storage, hipStream_t stream)
{
  const MarchGrid g = march_grid(a);
  if (g.blocks > 0x7fffffff || !march_applies(a.nt, a.nz)) return hipErrorInvalidConfiguration;
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_stress_march<decltype(s)>, dim3((unsigned)g.blocks), dim3(TJ * 64), 0, stream, a,
                       g.nzb, g.njt, g.rseg);
    return hipGetLastError();
  });
}

}  // namespace cw
