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

// Theta rows per workgroup.  Measured on MI355X: 2 to 8 rows done one after
// the other by the same wavefronts (set-up paid once) are 10-55 % slower
// than one row, as the compiler then keeps two rows' loads in flight and
// the register growth costs more occupancy than it saves.
#ifndef CW_VEC_ROWS
#define CW_VEC_ROWS 1
#endif
constexpr int kRows = CW_VEC_ROWS;
// Minimum wavefronts per SIMD the compiler sizes each kernel's registers
// for (1: no constraint).  Measured on MI355X at 256 x 128 x 8192 (ms per
// launch, velocity / stress):
//   float32:  stress 8 -> 3.455 against 3.489 unconstrained (64 registers, a
//             few scalar values kept in vector lanes); velocity 6 or 7 change
//             nothing;
//   bfloat16: 7 / 7 -> 1.815 / 2.209, against 1.904 / 2.340 at 6 / 6 and
//             2.369 / 2.759 at 8 / 8;
//   float16:  5 / 7 -> 2.097 / 2.375, against 2.129 / 2.617 at 6 / none;
//             8 spills.
// The stochastically rounding bfloat16 kernels need a few more registers
// (the random bits): their stress update asks for 6 waves per SIMD (at 7 it
// spills 36 bytes per lane).
#ifndef CW_SR_STRESS_WAVES
#define CW_SR_STRESS_WAVES 6
#endif
#ifndef CW_VEC_WAVES
template <class S> struct Occupancy { static constexpr int vel = 1, str = 8, vel_sr = 1, str_sr = 8; };
template <> struct Occupancy<StF16> { static constexpr int vel = 5, str = 7, vel_sr = 5, str_sr = 7; };
template <> struct Occupancy<StBF16> { static constexpr int vel = 7, str = 7, vel_sr = 7, str_sr = CW_SR_STRESS_WAVES; };
#else
template <class S> struct Occupancy {
  static constexpr int vel = CW_VEC_WAVES, str = CW_VEC_WAVES, vel_sr = CW_VEC_WAVES, str_sr = CW_VEC_WAVES;
};
#endif

// velocity update of the lane's VW cells of column (i, j); mr, mt, mz collect |v| maxima.
// kSR: the field stores round stochastically (a separate instantiation: the
// extra registers of the random bits would make the default form spill)
template <class S, bool kSR = false>
__device__ __forceinline__ void velocity_column(const StepArgs &a, int i, int j, int kb, bool live, float &mr,
                                                float &mt, float &mz)
{
  const int jm = j == 0 ? a.nt - 1 : j - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const Lanes<S> L(a, kb, j, jm, jp);
  const float *c = a.scl_in;
  const int i1 = i + 1 <= a.m_last ? i + 1 : a.m_last;   // medium ring index, clamped at the edge
  // densities first: issued after the stresses, the compiler held them
  // back until most stress reads had returned, a second round trip.
  // Measured: bfloat16 velocity update at 256 x 128 x 8192 1.699 -> 1.682
  // ms per launch (three runs on one box); refined grid 37.5-37.7 against
  // 37.5-38.9 Gcell/s (run-to-run spread).
  float rho0[VW], rho_i1[VW], rho_jp[VW];
  const rsrc_t R_rho = L.med(a.rho, i);
  ldb4(rho0, R_rho, L.m0, L.mj);
  ldb4(rho_i1, L.med(a.rho, i1), L.m0, L.mj);              // medium index clamped at the edge
  ldb4(rho_jp, R_rho, L.m0, L.mjp);
  const float rho_a = ldb1(R_rho, L.ma, L.mj);
  float srr0[VW], srr1[VW], stt0[VW], stt1[VW], stt_jp[VW], srt0[VW], srt_jm[VW], srt_im[VW];
  float srz0[VW], srz_im[VW], stz0[VW], stz_jm[VW], szz0[VW];
  const rsrc_t R_srr = L.field(a.in[SRR], i), R_stt = L.field(a.in[STT], i), R_srt = L.field(a.in[SRT], i);
  const rsrc_t R_srz = L.field(a.in[SRZ], i), R_stz = L.field(a.in[STZ], i), R_szz = L.field(a.in[SZZ], i);
  S::ldb(srr0, R_srr, L.v0, L.sj, c[SRR]);
  ldf<S>(srr1, L, a, a.in[SRR], c[SRR], i + 1, L.sj);      // zero beyond the last ring
  S::ldb(stt0, R_stt, L.v0, L.sj, c[STT]);
  ldf<S>(stt1, L, a, a.in[STT], c[STT], i + 1, L.sj);
  S::ldb(stt_jp, R_stt, L.v0, L.sjp, c[STT]);
  S::ldb(srt0, R_srt, L.v0, L.sj, c[SRT]);
  S::ldb(srt_jm, R_srt, L.v0, L.sjm, c[SRT]);
  ldf<S>(srt_im, L, a, a.in[SRT], c[SRT], i - 1, L.sj);    // zero on the axis side of ring 0
  S::ldb(srz0, R_srz, L.v0, L.sj, c[SRZ]);
  ldf<S>(srz_im, L, a, a.in[SRZ], c[SRZ], i - 1, L.sj);
  S::ldb(stz0, R_stz, L.v0, L.sj, c[STZ]);
  S::ldb(stz_jm, R_stz, L.v0, L.sjm, c[STZ]);
  S::ldb(szz0, R_szz, L.v0, L.sj, c[SZZ]);
  // depth neighbours of the group (zero outside the grid)
  const float srz_b = ldz<S>(L.has_b, R_srz, L.vb, L.sj, c[SRZ]);
  const float stz_b = ldz<S>(L.has_b, R_stz, L.vb, L.sj, c[STZ]);
  const float szz_a = ldz<S>(L.has_a, R_szz, L.va, L.sj, c[SZZ]);

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
    const float *T = a.tab_r;
    cpml_b(L.f32(a.psi_r[R_VR_DR], ir), L.m0, L.tj, T[AR_F * a.nr + i], T[BR_F * a.nr + i], r_dr);
    cpml_b(L.f32(a.psi_r[R_VR_B], ir), L.m0, L.tj, T[AT_F * a.nr + i], T[BT_F * a.nr + i], r_b);
    cpml_b(L.f32(a.psi_r[R_VT_DR], ir), L.m0, L.tj, T[AR_C * a.nr + i], T[BR_C * a.nr + i], t_dr);
    cpml_b(L.f32(a.psi_r[R_VT_B], ir), L.m0, L.tj, T[AT_C * a.nr + i], T[BT_C * a.nr + i], t_b);
    cpml_b(L.f32(a.psi_r[R_VZ_DR], ir), L.m0, L.tj, T[AR_C * a.nr + i], T[BR_C * a.nr + i], z_dr);
    cpml_b(L.f32(a.psi_r[R_VZ_B], ir), L.m0, L.tj, T[AT_C * a.nr + i], T[BT_C * a.nr + i], z_b);
  }
  if (live && a.npz > 0 && (kb < a.npz || kb + VW - 1 >= a.nz - 1 - a.npz)) {
    if (S::bytes == 2) {
      cpml_z3(a, i, j, kb, a.psi_z[Z_VR_DZ], a.psi_z[Z_VT_DZ], a.psi_z[Z_VZ_DZ], a.tab_z, false, false, true, r_dz,
              t_dz, z_dz);
    } else {
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
  }
  const rsrc_t R_vr = L.field(a.in[VR], i), R_vt = L.field(a.in[VT], i), R_vz = L.field(a.in[VZ], i);
  float vr[VW], vt[VW], vz[VW];
  S::ldbu(vr, R_vr, L.v0, L.sj, c[VR]);
  S::ldbu(vt, R_vt, L.v0, L.sj, c[VT]);
  S::ldbu(vz, R_vz, L.v0, L.sj, c[VZ]);
#pragma unroll
  for (int e = 0; e < VW; e++) {
    const float rho_kp = e == VW - 1 ? rho_a : rho0[e + 1];
    const float b_r = 2.0f * rcp(rho0[e] + rho_i1[e]);
    const float b_t = 2.0f * rcp(rho0[e] + rho_jp[e]);
    const float b_z = 2.0f * rcp(rho0[e] + rho_kp);
    vr[e] += a.dt * b_r * (r_dr[e] + r_b[e] + r_dz[e]);
    vt[e] += a.dt * b_t * (t_dr[e] + t_b[e] + t_dz[e]);
    vz[e] += a.dt * b_z * (z_dr[e] + z_b[e] + z_dz[e]);
  }
#pragma unroll
  for (int e = 0; e < VW; e++) {
    mr = fmaxf(mr, fabsf(vr[e])); mt = fmaxf(mt, fabsf(vt[e])); mz = fmaxf(mz, fabsf(vz[e]));
  }
  if (live) {
    const float *o = a.scl_out;
    constexpr bool sr = kSR && S::stochastic;
    const unsigned sb = sr ? sr_base<S>(a, at(a, i, j, kb)) : 0u;
    S::stb(L.fieldw(a.out[VR], i), L.v0, L.sj, vr, S::scaled ? inv_pow2(o[VR]) : 1.0f, sr_key(sb, VR), sr);
    S::stb(L.fieldw(a.out[VT], i), L.v0, L.sj, vt, S::scaled ? inv_pow2(o[VT]) : 1.0f, sr_key(sb, VT), sr);
    S::stb(L.fieldw(a.out[VZ], i), L.v0, L.sj, vz, S::scaled ? inv_pow2(o[VZ]) : 1.0f, sr_key(sb, VZ), sr);
  }
}

// One workgroup per (ring, CW_VEC_ROWS theta rows, depth segment of 1024
// cells): the rows are done one after the other, so each wavefront lives
// several column segments long and its set-up is paid once.
template <class S, bool kSR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kSR ? Occupancy<S>::vel_sr : Occupancy<S>::vel)))
k_velocity_vec(StepArgs a, int nbx)
{
  const int bx = blockIdx.x % nbx;
  const int k0 = (bx * 256 + threadIdx.x) * VW;
  const int njt = (a.nt + kRows - 1) / kRows;
  const int c = blockIdx.x / nbx, i = c / njt, j0 = (c - i * njt) * kRows;
  const int j1 = j0 + kRows < a.nt ? j0 + kRows : a.nt;
  const bool live = k0 < a.nz;
  const int kb = live ? k0 : a.nz - VW;            // dead lanes compute on a valid group, store nothing
  float mr = 0.0f, mt = 0.0f, mz = 0.0f;
  for (int j = j0; j < j1; j++) velocity_column<S, kSR>(a, i, j, kb, live, mr, mt, mz);
  if (S::scaled) {
    track_max(a.maxabs + VR * kMaxSlots, live ? mr : 0.0f);
    track_max(a.maxabs + VT * kMaxSlots, live ? mt : 0.0f);
    track_max(a.maxabs + VZ * kMaxSlots, live ? mz : 0.0f);
  }
}

// stress update of the lane's VW cells of column (i, j); mx collects |sigma| maxima
template <class S, bool kSR = false>
__device__ __forceinline__ void stress_column(const StepArgs &a, int i, int j, int kb, bool live, float (&mx)[6])
{
  const int jm = j == 0 ? a.nt - 1 : j - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const Lanes<S> L(a, kb, j, jm, jp);
  const float *o = a.scl_out;                      // velocities at level n+1/2 (output buffer)
  const float *vR = a.out[VR], *vT = a.out[VT], *vZ = a.out[VZ];
  const rsrc_t R_vr = L.field(vR, i), R_vt = L.field(vT, i), R_vz = L.field(vZ, i);
  float vr0[VW], vr_im[VW], vr_jp[VW], vt0[VW], vt_jm[VW], vt_ip[VW], vz0[VW], vz_ip[VW], vz_jp[VW];
  S::ldb(vr0, R_vr, L.v0, L.sj, o[VR]);
  ldf<S>(vr_im, L, a, vR, o[VR], i - 1, L.sj);              // zero on the axis side of ring 0
  S::ldb(vr_jp, R_vr, L.v0, L.sjp, o[VR]);
  S::ldb(vt0, R_vt, L.v0, L.sj, o[VT]);
  S::ldb(vt_jm, R_vt, L.v0, L.sjm, o[VT]);
  ldf<S>(vt_ip, L, a, vT, o[VT], i + 1, L.sj);              // zero beyond the last ring
  S::ldb(vz0, R_vz, L.v0, L.sj, o[VZ]);
  ldf<S>(vz_ip, L, a, vZ, o[VZ], i + 1, L.sj);
  S::ldb(vz_jp, R_vz, L.v0, L.sjp, o[VZ]);
  const float vr_a = ldz<S>(L.has_a, R_vr, L.va, L.sj, o[VR]);
  const float vt_a = ldz<S>(L.has_a, R_vt, L.va, L.sj, o[VT]);
  const float vz_b = ldz<S>(L.has_b, R_vz, L.vb, L.sj, o[VZ]);

  // The old stresses: float16 reads them here, with the velocities and
  // before the layer block, whose stores could alias them (read after it
  // they take a second memory round trip); the other storages read them
  // after it (below), where they hold fewer registers across the block.
  // Measured at 256 x 128 x 8192, ms per stress launch, read here against
  // after the block: float16 2.20 against 2.30-2.38; bfloat16 2.14 against
  // 2.04-2.12; float32 (8 waves per SIMD) spilled and slowed the solo
  // four-cell step by 28 %.
  float old[6][VW];
  if constexpr (S::scaled) {
#pragma unroll
    for (int q = 0; q < 6; q++) S::ldbu(old[q], L.field(a.in[SRR + q], i), L.v0, L.sj, a.scl_in[SRR + q]);
  }
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
    if (S::bytes == 2) {
      cpml_z3(a, i, j, kb, a.psi_z[Z_N_DZ], a.psi_z[Z_RZ_DZ], a.psi_z[Z_TZ_DZ], a.tab_z, false, true, true, ezz,
              rz_dz, tz_dz);
    } else {
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
  }
  // moduli: reciprocals of mu at the cell and its neighbours (r, theta, depth)
  const int i1 = i + 1 <= a.m_last ? i + 1 : a.m_last;
  const rsrc_t R_mu = L.med(a.mu, i), R_mu1 = L.med(a.mu, i1);   // medium index clamped at the edge
  float lam[VW], mu[VW], m_i1[VW], m_jp[VW], m_i1jp[VW];
  ldb4(lam, L.med(a.lam, i), L.m0, L.mj);
  ldb4(mu, R_mu, L.m0, L.mj);
  ldb4(m_i1, R_mu1, L.m0, L.mj);
  ldb4(m_jp, R_mu, L.m0, L.mjp);
  ldb4(m_i1jp, R_mu1, L.m0, L.mjp);
  const float ia = rcp(ldb1(R_mu, L.ma, L.mj)), ia_i1 = rcp(ldb1(R_mu1, L.ma, L.mj));
  const float ia_jp = rcp(ldb1(R_mu, L.ma, L.mjp));
  float im[VW], im_i1[VW], im_jp[VW];
#pragma unroll
  for (int e = 0; e < VW; e++) { im[e] = rcp(mu[e]); im_i1[e] = rcp(m_i1[e]); im_jp[e] = rcp(m_jp[e]); }

  const float *c = a.scl_in;
  const rsrc_t R_srr = L.field(a.in[SRR], i), R_stt = L.field(a.in[STT], i), R_szz = L.field(a.in[SZZ], i);
  const rsrc_t R_srt = L.field(a.in[SRT], i), R_srz = L.field(a.in[SRZ], i), R_stz = L.field(a.in[STZ], i);
  float srr[VW], stt[VW], szz[VW], srt[VW], srz[VW], stz[VW];
  if constexpr (S::scaled) {
#pragma unroll
    for (int e = 0; e < VW; e++) {
      srr[e] = old[0][e]; stt[e] = old[1][e]; szz[e] = old[2][e];
      srt[e] = old[3][e]; srz[e] = old[4][e]; stz[e] = old[5][e];
    }
  } else {
    S::ldbu(srr, R_srr, L.v0, L.sj, c[SRR]);
    S::ldbu(stt, R_stt, L.v0, L.sj, c[STT]);
    S::ldbu(szz, R_szz, L.v0, L.sj, c[SZZ]);
    S::ldbu(srt, R_srt, L.v0, L.sj, c[SRT]);
    S::ldbu(srz, R_srz, L.v0, L.sj, c[SRZ]);
    S::ldbu(stz, R_stz, L.v0, L.sj, c[STZ]);
  }
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
  }
#pragma unroll
  for (int e = 0; e < VW; e++) {
    mx[0] = fmaxf(mx[0], fabsf(srr[e])); mx[1] = fmaxf(mx[1], fabsf(stt[e]));
    mx[2] = fmaxf(mx[2], fabsf(szz[e])); mx[3] = fmaxf(mx[3], fabsf(srt[e]));
    mx[4] = fmaxf(mx[4], fabsf(srz[e])); mx[5] = fmaxf(mx[5], fabsf(stz[e]));
  }
  if (live) {
    constexpr bool sr = kSR && S::stochastic;
    const unsigned sb = sr ? sr_base<S>(a, at(a, i, j, kb)) : 0u;
    S::stb(L.fieldw(a.out[SRR], i), L.v0, L.sj, srr, S::scaled ? inv_pow2(o[SRR]) : 1.0f, sr_key(sb, SRR), sr);
    S::stb(L.fieldw(a.out[STT], i), L.v0, L.sj, stt, S::scaled ? inv_pow2(o[STT]) : 1.0f, sr_key(sb, STT), sr);
    S::stb(L.fieldw(a.out[SZZ], i), L.v0, L.sj, szz, S::scaled ? inv_pow2(o[SZZ]) : 1.0f, sr_key(sb, SZZ), sr);
    S::stb(L.fieldw(a.out[SRT], i), L.v0, L.sj, srt, S::scaled ? inv_pow2(o[SRT]) : 1.0f, sr_key(sb, SRT), sr);
    S::stb(L.fieldw(a.out[SRZ], i), L.v0, L.sj, srz, S::scaled ? inv_pow2(o[SRZ]) : 1.0f, sr_key(sb, SRZ), sr);
    S::stb(L.fieldw(a.out[STZ], i), L.v0, L.sj, stz, S::scaled ? inv_pow2(o[STZ]) : 1.0f, sr_key(sb, STZ), sr);
  }
}

template <class S, bool kSR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kSR ? Occupancy<S>::str_sr : Occupancy<S>::str)))
k_stress_vec(StepArgs a, int nbx)
{
  const int bx = blockIdx.x % nbx;
  const int k0 = (bx * 256 + threadIdx.x) * VW;
  const int njt = (a.nt + kRows - 1) / kRows;
  const int c = blockIdx.x / nbx, i = c / njt, j0 = (c - i * njt) * kRows;
  const int j1 = j0 + kRows < a.nt ? j0 + kRows : a.nt;
  const bool live = k0 < a.nz;
  const int kb = live ? k0 : a.nz - VW;
  float mx[6] = {0, 0, 0, 0, 0, 0};
  for (int j = j0; j < j1; j++) stress_column<S, kSR>(a, i, j, kb, live, mx);
  if (S::scaled) {
#pragma unroll
    for (int q = 0; q < 6; q++) track_max(a.maxabs + (SRR + q) * kMaxSlots, live ? mx[q] : 0.0f);
  }
}

// Batched form: one workgroup grid over the tiles of every instance; the
// instance is found by a binary search of the tiles' first indices (a small
// array the scalar cache keeps), then the column code runs as above.
__device__ __forceinline__ int batch_instance(const long *tile0, int count, long t)
{
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile0[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// this wavefront's (ring, theta row, depth group) in tile t of instance I; false if the row is past nt
// (32-bit index arithmetic: a batched grid has fewer than 2^31 workgroups)
__device__ __forceinline__ bool batch_cell(const BatchInst &I, const StepArgs &a, long t, int &i, int &j, int &kb,
                                           bool &live)
{
  const int w = I.tz_waves, rows = 4 / w;
  const int wv = threadIdx.x >> 6, dz = wv % w, dr = wv / w;
  const unsigned local = (unsigned)(t - I.tile0), nseg = (unsigned)I.nseg;
  const unsigned seg = local % nseg, rest = local / nseg;
  const unsigned njt = (unsigned)((a.nt + rows - 1) / rows);
  j = (int)(rest % njt) * rows + dr;
  i = (int)(rest / njt);
  if (j >= a.nt) return false;
  const int k0 = (int)seg * w * 256 + dz * 256 + (int)(threadIdx.x & 63) * 4;
  live = k0 < a.nz;
  kb = live ? k0 : a.nz - VW;
  return true;
}

// WPE: the minimum wavefronts per SIMD the registers are sized for (1: no
// constraint); the batch's tuner picks it with the tile shapes.
template <int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
k_velocity_batch(const BatchInst *__restrict__ B, const long *__restrict__ tile0, int count, int parity)
{
  const BatchInst &I = B[batch_instance(tile0, count, blockIdx.x)];
  const StepArgs a = I.a[parity];     // a private copy: the field stores cannot alias it
  int i, j, kb;
  bool live;
  if (!batch_cell(I, a, blockIdx.x, i, j, kb, live)) return;   // whole wavefront; no barriers here
  float mr = 0.0f, mt = 0.0f, mz = 0.0f;
  velocity_column<StF32>(a, i, j, kb, live, mr, mt, mz);
}

template <int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
k_stress_batch(const BatchInst *__restrict__ B, const long *__restrict__ tile0, int count, int parity)
{
  const BatchInst &I = B[batch_instance(tile0, count, blockIdx.x)];
  const StepArgs a = I.a[parity];
  int i, j, kb;
  bool live;
  if (!batch_cell(I, a, blockIdx.x, i, j, kb, live)) return;
  float mx[6] = {0, 0, 0, 0, 0, 0};
  stress_column<StF32>(a, i, j, kb, live, mx);
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

bool vec_applies(int nt, int nz) { return nz % VW == 0 && nz >= VW && (uint64_t)nt * nz * 4 < (1ull << 32); }

hipError_t launch_velocity_vec(const StepArgs &a, int storage, hipStream_t stream)
{
  const int nbx = (a.nz / VW + 255) / 256;
  const long g = (long)nbx * ((a.nt + kRows - 1) / kRows) * a.nr;
  if (g > 0x7fffffff || !vec_applies(a.nt, a.nz)) return hipErrorInvalidConfiguration;
  if (a.sr && storage == ST_BF16) {
    hipLaunchKernelGGL((k_velocity_vec<StBF16, true>), dim3((unsigned)g), dim3(256), 0, stream, a, nbx);
    return hipGetLastError();
  }
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL((k_velocity_vec<decltype(s), false>), dim3((unsigned)g), dim3(256), 0, stream, a, nbx);
    return hipGetLastError();
  });
}

hipError_t launch_stress_vec(const StepArgs &a, int storage, hipStream_t stream)
{
  const int nbx = (a.nz / VW + 255) / 256;
  const long g = (long)nbx * ((a.nt + kRows - 1) / kRows) * a.nr;
  if (g > 0x7fffffff || !vec_applies(a.nt, a.nz)) return hipErrorInvalidConfiguration;
  if (a.sr && storage == ST_BF16) {
    hipLaunchKernelGGL((k_stress_vec<StBF16, true>), dim3((unsigned)g), dim3(256), 0, stream, a, nbx);
    return hipGetLastError();
  }
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL((k_stress_vec<decltype(s), false>), dim3((unsigned)g), dim3(256), 0, stream, a, nbx);
    return hipGetLastError();
  });
}

bool batch_occupancy_supported(int wpe) { return wpe == 0 || wpe == 7 || wpe == 8; }

template <template <int> class K>
static hipError_t launch_batch(int wpe, const BatchInst *dev, const long *tile0, int count, long tiles, int parity,
                               hipStream_t stream)
{
  if (tiles < 1 || tiles > 0x7fffffff) return hipErrorInvalidConfiguration;
  const dim3 g((unsigned)tiles), b(256);
  switch (wpe) {
  case 0: hipLaunchKernelGGL(K<1>::f, g, b, 0, stream, dev, tile0, count, parity); break;
  case 7: hipLaunchKernelGGL(K<7>::f, g, b, 0, stream, dev, tile0, count, parity); break;
  case 8: hipLaunchKernelGGL(K<8>::f, g, b, 0, stream, dev, tile0, count, parity); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <int W> struct VelBatch { static constexpr auto f = k_velocity_batch<W>; };
template <int W> struct StrBatch { static constexpr auto f = k_stress_batch<W>; };

hipError_t launch_velocity_batch(const BatchInst *dev, const long *tile0, int count, long tiles, int parity, int wpe,
                                 hipStream_t stream)
{
  return launch_batch<VelBatch>(wpe, dev, tile0, count, tiles, parity, stream);
}

hipError_t launch_stress_batch(const BatchInst *dev, const long *tile0, int count, long tiles, int parity, int wpe,
                               hipStream_t stream)
{
  return launch_batch<StrBatch>(wpe, dev, tile0, count, tiles, parity, stream);
}

}  // namespace cw
