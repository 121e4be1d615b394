// Fused time step: one launch advances v^{n-1/2} -> v^{n+1/2} and
// sigma^n -> sigma^{n+1}, the absorbing layer's memory variables and the
// sources, reading the state, the medium and the layer memory once and
// writing them once.
//
// Mapping.  A workgroup of TJ wavefronts owns a tile of (TJ - 2) theta rows
// x 62 depth cells and marches outward through all nr rings.  Wavefront w
// holds theta row j0 - 1 + w; lane l holds depth k0 - 1 + l, so every load
// and store of a wavefront is one contiguous run along z.  The first and
// last rows and lanes are halo: they compute the velocities their neighbours
// need and store nothing.  Each lane keeps a sliding window of rings in
// registers (the r-neighbours); depth neighbours come from the adjacent
// lanes by a wavefront-wide DPP shift; theta neighbours come from the
// adjacent wavefronts through a double-buffered LDS exchange, one barrier
// per ring.  Ring m of the march updates the velocities of ring m and the
// stresses of ring m-1 (which need the new velocities of rings m-2..m).
//
// Addressing: every array access is (uniform base of a ring) + (this
// lane's 32-bit byte offset in the ring, fixed for the whole march).
//
// Values with k outside [0, nz) or i outside [0, nr) are zero (the axis and
// outer closures); medium indices are clamped at the edges.  The discrete
// operators are those of the two-pass kernels (staggered form of Eq. (1)).
// Reciprocals use the hardware v_rcp_f32 (1 ulp): 1/mu is formed once per
// cell and exchanged instead of mu, so each harmonic mean costs three adds
// and one reciprocal; a zero modulus gives an infinite reciprocal and a zero
// mean, exactly as the definition requires.
#include "cwell_internal.hpp"

namespace cw {

namespace {

#ifndef FUSED_PREFETCH_DEPTH
#define FUSED_PREFETCH_DEPTH 1
#endif
#ifndef FUSED_TJ
#define FUSED_TJ 10
#endif
constexpr int TJ = FUSED_TJ;    // wavefronts (theta rows) per workgroup, 2 of them halo
constexpr int ZT = 62;          // depth cells owned per wavefront (64 lanes - 2 halo)
constexpr int NX = 8;           // floats exchanged per lane and ring through LDS
constexpr int DEPTH = FUSED_PREFETCH_DEPTH;   // rings loaded ahead of use

// lane l receives lane l-1's value (lane 0 receives 0)
__device__ __forceinline__ float from_below(float x)
{
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, false));
}
// lane l receives lane l+1's value (lane 63 receives 0)
__device__ __forceinline__ float from_above(float x)
{
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// base (uniform) + byte offset (per lane, 32-bit)
__device__ __forceinline__ float ldo(const float *base, uint32_t off)
{
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off);
}
__device__ __forceinline__ void sto(float *base, uint32_t off, float v)
{
  *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + off) = v;
}

struct Six { float rr, tt, zz, rt, rz, tz; };
struct Three { float r, t, z; };
// What one lane loads ahead for a future ring of the march: the stresses and
// medium of ring p+1 and the old velocities and lambda of ring p, p being
// the ring whose velocities the march updates when this entry is used.
struct Ahead { Six S; Three v; float rho, mu, lam; };

// LDS slots
enum { X_VR = 0, X_VT, X_VZ, X_SRT, X_STT, X_STZ, X_RHO, X_IMU };

// Per-ring constants staged in LDS once per workgroup: 1/r_i, 1/R_i and the
// eight radial layer coefficients.  (Fetching them from global memory inside
// the march would make every ring wait for the whole prefetch queue, since
// vector-memory completions are counted in order.)
constexpr int NRT = 2 + NTAB_R;

__global__ void __launch_bounds__(TJ * 64) k_step_fused(FusedArgs F)
{
  __shared__ float xch[2][NX][TJ][64];
  extern __shared__ float rtab[];                  // [NRT][nr]
  const int nr = F.nr, nt = F.nt, nz = F.nz;
  for (int c = threadIdx.x; c < nr; c += TJ * 64) {
    rtab[c] = F.inv_rc[c];
    rtab[nr + c] = F.inv_rf[c];
  }
  for (int c = threadIdx.x; c < NTAB_R * nr; c += TJ * 64) rtab[2 * nr + c] = F.tab_r[c];
  const float *RT = rtab + 2 * nr;                 // layer table rows, as in tab_r

  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  // XCD-aware tile order: consecutive workgroups of one XCD take consecutive tiles
#ifndef FUSED_XCD_REMAP
#define FUSED_XCD_REMAP 0
#endif
  const int t = FUSED_XCD_REMAP ? xcd_tile_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  // theta tiles of one depth range are consecutive (measured faster on
  // MI355X than depth-fastest order: the theta-halo rows are other resident
  // workgroups' own rows)
  const int ntile_t = (nt + F.own_rows - 1) / F.own_rows;
  const int tt = t % ntile_t, tz = t / ntile_t;
  const int j0 = tt * F.own_rows;
  const int jr = j0 - 1 + w;                       // unwrapped row
  const int j = ((jr % nt) + nt) % nt;
  const int k = tz * ZT - 1 + l;
  const bool kin = k >= 0 && k < nz;
  const bool own = kin && l >= 1 && l <= ZT && w >= 1 && w <= F.own_rows && jr < nt;
  const int kc = k < 0 ? 0 : (k >= nz ? nz - 1 : k);   // clamped (medium, safe addresses)
  const int wm = w > 0 ? w - 1 : 0, wp = w < TJ - 1 ? w + 1 : TJ - 1;

  const size_t plane = (size_t)nt * nz, fplane = F.rs;   // ring strides: layer memory, fields
  const uint32_t off0 = (uint32_t)(j * nz + kc) * 4u;  // byte offset of this lane's cell in a ring
  const float *fin = F.in, *med = F.med;
  float *fout = F.out;
  const size_t n = F.n;
  auto fld = [&](int q, int i, uint32_t o) -> float {   // input field q at ring i (0 outside)
    const float v = ldo(fin + q * n + (size_t)(i < nr ? i : nr - 1) * fplane, o);
    return (kin && i < nr) ? v : 0.0f;
  };
  // byte offset of this lane's cell in a ring of the medium (no theta term when the
  // medium does not vary along theta)
  const uint32_t moff0 = (uint32_t)(j * F.m_row + kc) * 4u;
  auto mat = [&](int q, int i, uint32_t) -> float {   // medium q (0 rho, 1 lambda, 2 mu) at ring min(i, nr-1)
    return ldo(med + q * F.m_n + (size_t)(i < nr ? i : nr - 1) * F.m_ring, moff0);
  };
  auto six = [&](int i, uint32_t o) -> Six {
    return Six{fld(SRR, i, o), fld(STT, i, o), fld(SZZ, i, o), fld(SRT, i, o), fld(SRZ, i, o), fld(STZ, i, o)};
  };
  auto ahead = [&](int p, uint32_t o) -> Ahead {   // entry used when the march reaches ring p
    return Ahead{six(p + 1, o), Three{fld(VR, p, o), fld(VT, p, o), fld(VZ, p, o)},
                 mat(0, p + 1, o), mat(2, p + 1, o), mat(1, p, o)};
  };

  const int kz = (F.npz > 0 && kin) ? (k < F.npz ? k : (k >= nz - 1 - F.npz ? k - (nz - 1 - F.npz) + F.npz : -1)) : -1;
  const int r0 = nr - F.npr;                       // first ring of the radial layer
  const uint32_t offz0 = (uint32_t)(j * F.nzs + (kz < 0 ? 0 : kz)) * 4u;  // byte offset in a z-slab ring
  const size_t planez = (size_t)nt * F.nzs;
  // this lane's z layer coefficients (zero outside the z slabs)
  float azc = 0.0f, bzc = 0.0f, azh = 0.0f, bzh = 0.0f;
  if (kz >= 0) {
    azc = F.tab_z[AZ_C * nz + k]; bzc = F.tab_z[BZ_C * nz + k];
    azh = F.tab_z[AZ_H * nz + k]; bzh = F.tab_z[BZ_H * nz + k];
  }

  // ---- prologue: rings 0 and 1 in registers, theta neighbours of ring 0
  Six Sp{0, 0, 0, 0, 0, 0};
  Six Sc = six(0, off0);
  Six Sn = six(1, off0);
  Three vo = {fld(VR, 0, off0), fld(VT, 0, off0), fld(VZ, 0, off0)};
  float rho_c = mat(0, 0, off0), rho_n = mat(0, 1, off0);
  float mu_p = 0.0f, mu_c = mat(2, 0, off0), mu_n = mat(2, 1, off0);
  float imu_p = 0.0f, imu_c = rcp(mu_c);
  float lam_p = 0.0f, lam_c = mat(1, 0, off0);
  Ahead Q[DEPTH];
#pragma unroll
  for (int d = 0; d < DEPTH; d++) Q[d] = ahead(1 + d, off0);
  __syncthreads();                                 // the ring tables are in LDS
  xch[1][X_SRT][w][l] = Sc.rt; xch[1][X_STT][w][l] = Sc.tt; xch[1][X_STZ][w][l] = Sc.tz;
  xch[1][X_RHO][w][l] = rho_c; xch[1][X_IMU][w][l] = imu_c;
  __syncthreads();
  float nb_rt = xch[1][X_SRT][wm][l], nb_tt = xch[1][X_STT][wp][l], nb_tz = xch[1][X_STZ][wm][l];
  float nb_rho = xch[1][X_RHO][wp][l];
  float imuJ_p = 0.0f, imuJ_c = xch[1][X_IMU][wp][l];
  Three vp = {0, 0, 0}, vpN = {0, 0, 0};           // v^{n+1/2} of ring m-1 and its theta neighbours
  float vr_pp = 0.0f;                              // v_r^{n+1/2} of ring m-2

  for (int m = 0; m <= nr; ++m) {
    const uint32_t off = off0, offz = offz0;
    // ---- layer memory of the velocity update of ring m (its latency is
    //      exposed: only rings of the layer slabs pay it)
    const bool lr_v = m >= r0 && m < nr && kin, lr_s = m - 1 >= r0 && m >= 1 && kin;
    const bool lz_v = kz >= 0 && m < nr, lz_s = kz >= 0 && m >= 1;
    float pv[6], ps[6], pzv[3], pzs[3];
    if (lr_v) {
      const float *b0 = F.psi_r_in + (size_t)(m - r0) * plane;
#pragma unroll
      for (int c = 0; c < 6; c++) pv[c] = ldo(b0 + (size_t)(R_VR_DR + c) * F.slab_r, off);
    }
    if (lz_v) {
      const float *b0 = F.psi_z_in + (size_t)m * planez;
#pragma unroll
      for (int c = 0; c < 3; c++) pzv[c] = ldo(b0 + (size_t)(Z_VR_DZ + c) * F.slab_z, offz);
    }

    // ---- velocities of ring m
    Three vn = {0, 0, 0};
    if (m < nr) {
      const float irc = rtab[m], irf = rtab[nr + m];
      const float srz_km = from_below(Sc.rz), stz_km = from_below(Sc.tz), szz_kp = from_above(Sc.zz);
      float r_dr = (Sn.rr - Sc.rr) * F.inv_dr;
      float r_b = irf * ((Sc.rt - nb_rt) * F.inv_dth + 0.5f * (Sn.rr + Sc.rr) - 0.5f * (Sn.tt + Sc.tt));
      float r_dz = (Sc.rz - srz_km) * F.inv_dz;
      float t_dr = (Sc.rt - Sp.rt) * F.inv_dr;
      float t_b = irc * ((nb_tt - Sc.tt) * F.inv_dth + (Sc.rt + Sp.rt));
      float t_dz = (Sc.tz - stz_km) * F.inv_dz;
      float z_dr = (Sc.rz - Sp.rz) * F.inv_dr;
      float z_b = irc * ((Sc.tz - nb_tz) * F.inv_dth + 0.5f * (Sc.rz + Sp.rz));
      float z_dz = (szz_kp - Sc.zz) * F.inv_dz;
      if (lr_v) {
        const float arf = RT[AR_F * nr + m], brf = RT[BR_F * nr + m];
        const float atf = RT[AT_F * nr + m], btf = RT[BT_F * nr + m];
        const float arc = RT[AR_C * nr + m], brc = RT[BR_C * nr + m];
        const float atc = RT[AT_C * nr + m], btc = RT[BT_C * nr + m];
        const float p0 = brf * pv[0] + arf * r_dr;
        const float p1 = btf * pv[1] + atf * r_b;
        const float p2 = brc * pv[2] + arc * t_dr;
        const float p3 = btc * pv[3] + atc * t_b;
        const float p4 = brc * pv[4] + arc * z_dr;
        const float p5 = btc * pv[5] + atc * z_b;
        if (own) {
          float *o = F.psi_r_out + (size_t)(m - r0) * plane;
          sto(o + (size_t)R_VR_DR * F.slab_r, off, p0); sto(o + (size_t)R_VR_B * F.slab_r, off, p1);
          sto(o + (size_t)R_VT_DR * F.slab_r, off, p2); sto(o + (size_t)R_VT_B * F.slab_r, off, p3);
          sto(o + (size_t)R_VZ_DR * F.slab_r, off, p4); sto(o + (size_t)R_VZ_B * F.slab_r, off, p5);
        }
        r_dr += p0; r_b += p1; t_dr += p2; t_b += p3; z_dr += p4; z_b += p5;
      }
      if (lz_v) {
        const float p0 = bzc * pzv[0] + azc * r_dz;
        const float p1 = bzc * pzv[1] + azc * t_dz;
        const float p2 = bzh * pzv[2] + azh * z_dz;
        if (own) {
          float *o = F.psi_z_out + (size_t)m * planez;
          sto(o + (size_t)Z_VR_DZ * F.slab_z, offz, p0); sto(o + (size_t)Z_VT_DZ * F.slab_z, offz, p1);
          sto(o + (size_t)Z_VZ_DZ * F.slab_z, offz, p2);
        }
        r_dz += p0; t_dz += p1; z_dz += p2;
      }
      const float b_r = 2.0f * rcp(rho_c + rho_n);
      const float b_t = 2.0f * rcp(rho_c + nb_rho);
      const float b_z = 2.0f * rcp(rho_c + from_above(rho_c));
      vn.r = vo.r + F.dt * b_r * (r_dr + r_b + r_dz);
      vn.t = vo.t + F.dt * b_t * (t_dr + t_b + t_dz);
      vn.z = vo.z + F.dt * b_z * (z_dr + z_b + z_dz);
      for (int e = 0; e < F.ninj; e++) {
        const InjectStep &s = F.inj[e];
        if (s.phase == 0 && s.i == m && s.k == k && (s.j < 0 || s.j == j)) {
          if (s.field == VR) vn.r += s.amp;
          else if (s.field == VT) vn.t += s.amp;
          else if (s.field == VZ) vn.z += s.amp;
        }
      }
      if (!kin) vn = Three{0, 0, 0};
      if (own) {
        float *o = fout + (size_t)m * fplane;
        sto(o + VR * n, off, vn.r); sto(o + VT * n, off, vn.t); sto(o + VZ * n, off, vn.z);
      }
    }

    // ---- layer memory of the stress update of ring m-1, issued before the
    //      prefetch so that waiting for it does not wait for the prefetch
    if (lr_s) {
      const float *b0 = F.psi_r_in + (size_t)(m - 1 - r0) * plane;
#pragma unroll
      for (int c = 0; c < 6; c++) ps[c] = ldo(b0 + (size_t)(R_N_DR + c) * F.slab_r, off);
    }
    if (lz_s) {
      const float *b0 = F.psi_z_in + (size_t)(m - 1) * planez;
#pragma unroll
      for (int c = 0; c < 3; c++) pzs[c] = ldo(b0 + (size_t)(Z_N_DZ + c) * F.slab_z, offz);
    }

    // ---- prefetch the entry for ring m + 1 + DEPTH
    const Ahead Qn = ahead(m + 1 + DEPTH, off);

    // ---- exchange: new velocities of ring m; stresses and medium of ring m+1
    const float imu_n = rcp(mu_n);
    const int bf = m & 1;
    xch[bf][X_VR][w][l] = vn.r; xch[bf][X_VT][w][l] = vn.t; xch[bf][X_VZ][w][l] = vn.z;
    xch[bf][X_SRT][w][l] = Sn.rt; xch[bf][X_STT][w][l] = Sn.tt; xch[bf][X_STZ][w][l] = Sn.tz;
    xch[bf][X_RHO][w][l] = rho_n; xch[bf][X_IMU][w][l] = imu_n;
    __syncthreads();
    const Three vN = {xch[bf][X_VR][wp][l], xch[bf][X_VT][wm][l], xch[bf][X_VZ][wp][l]};
    const float nbn_rt = xch[bf][X_SRT][wm][l], nbn_tt = xch[bf][X_STT][wp][l];
    const float nbn_tz = xch[bf][X_STZ][wm][l], nbn_rho = xch[bf][X_RHO][wp][l];
    const float imuJ_n = xch[bf][X_IMU][wp][l];

    // ---- stresses of ring q = m-1
    if (m >= 1) {
      const int q = m - 1;
      const float irc = rtab[q], irf = rtab[nr + q];
      const float vr_kp = from_above(vp.r), vt_kp = from_above(vp.t), vz_km = from_below(vp.z);
      float err = (vp.r - vr_pp) * F.inv_dr;
      float ett = irc * ((vp.t - vpN.t) * F.inv_dth + 0.5f * (vp.r + vr_pp));
      float ezz = (vp.z - vz_km) * F.inv_dz;
      float rt_dr = (vn.t - vp.t) * F.inv_dr;
      float rt_b = irf * ((vpN.r - vp.r) * F.inv_dth - 0.5f * (vn.t + vp.t));
      float rz_dr = (vn.z - vp.z) * F.inv_dr;
      float rz_dz = (vr_kp - vp.r) * F.inv_dz;
      float tz_b = irc * (vpN.z - vp.z) * F.inv_dth;
      float tz_dz = (vt_kp - vp.t) * F.inv_dz;
      if (lr_s) {
        const float arf = RT[AR_F * nr + q], brf = RT[BR_F * nr + q];
        const float atf = RT[AT_F * nr + q], btf = RT[BT_F * nr + q];
        const float arc = RT[AR_C * nr + q], brc = RT[BR_C * nr + q];
        const float atc = RT[AT_C * nr + q], btc = RT[BT_C * nr + q];
        const float p0 = brc * ps[0] + arc * err;
        const float p1 = btc * ps[1] + atc * ett;
        const float p2 = brf * ps[2] + arf * rt_dr;
        const float p3 = btf * ps[3] + atf * rt_b;
        const float p4 = brf * ps[4] + arf * rz_dr;
        const float p5 = btc * ps[5] + atc * tz_b;
        if (own) {
          float *o = F.psi_r_out + (size_t)(q - r0) * plane;
          sto(o + (size_t)R_N_DR * F.slab_r, off, p0); sto(o + (size_t)R_N_B * F.slab_r, off, p1);
          sto(o + (size_t)R_RT_DR * F.slab_r, off, p2); sto(o + (size_t)R_RT_B * F.slab_r, off, p3);
          sto(o + (size_t)R_RZ_DR * F.slab_r, off, p4); sto(o + (size_t)R_TZ_B * F.slab_r, off, p5);
        }
        err += p0; ett += p1; rt_dr += p2; rt_b += p3; rz_dr += p4; tz_b += p5;
      }
      if (lz_s) {
        const float p0 = bzc * pzs[0] + azc * ezz;
        const float p1 = bzh * pzs[1] + azh * rz_dz;
        const float p2 = bzh * pzs[2] + azh * tz_dz;
        if (own) {
          float *o = F.psi_z_out + (size_t)q * planez;
          sto(o + (size_t)Z_N_DZ * F.slab_z, offz, p0); sto(o + (size_t)Z_RZ_DZ * F.slab_z, offz, p1);
          sto(o + (size_t)Z_TZ_DZ * F.slab_z, offz, p2);
        }
        ezz += p0; rz_dz += p1; tz_dz += p2;
      }
      // harmonic means from the exchanged reciprocals (order as in the definition)
      const float ipk = from_above(imu_p), ick = from_above(imu_c), ijpk = from_above(imuJ_p);
      const float mu_rt = 4.0f * rcp(imu_p + imu_c + imuJ_p + imuJ_c);
      const float mu_rz = 4.0f * rcp(imu_p + imu_c + ipk + ick);
      const float mu_tz = 4.0f * rcp(imu_p + imuJ_p + ipk + ijpk);
      const float tr = err + ett + ezz;
      const float lt = lam_p * tr, m2 = 2.0f * mu_p;
      Six sn;
      sn.rr = Sp.rr + F.dt * (lt + m2 * err);
      sn.tt = Sp.tt + F.dt * (lt + m2 * ett);
      sn.zz = Sp.zz + F.dt * (lt + m2 * ezz);
      sn.rt = Sp.rt + F.dt * mu_rt * (rt_dr + rt_b);
      sn.rz = Sp.rz + F.dt * mu_rz * (rz_dr + rz_dz);
      sn.tz = Sp.tz + F.dt * mu_tz * (tz_b + tz_dz);
      for (int e = 0; e < F.ninj; e++) {
        const InjectStep &s = F.inj[e];
        if (s.phase == 1 && s.i == q && s.k == k && (s.j < 0 || s.j == j)) {
          switch (s.field) {
          case SRR: sn.rr += s.amp; break;
          case STT: sn.tt += s.amp; break;
          case SZZ: sn.zz += s.amp; break;
          case SRT: sn.rt += s.amp; break;
          case SRZ: sn.rz += s.amp; break;
          case STZ: sn.tz += s.amp; break;
          default: break;
          }
        }
      }
      if (own) {
        float *o = fout + (size_t)q * fplane;
        sto(o + SRR * n, off, sn.rr); sto(o + STT * n, off, sn.tt); sto(o + SZZ * n, off, sn.zz);
        sto(o + SRT * n, off, sn.rt); sto(o + SRZ * n, off, sn.rz); sto(o + STZ * n, off, sn.tz);
      }
    }

    // ---- rotate the window
    vr_pp = vp.r;
    vp = vn;
    vpN = vN;
    Sp = Sc; Sc = Sn; Sn = Q[0].S;
    vo = Q[0].v;
    rho_c = rho_n; rho_n = Q[0].rho;
    mu_p = mu_c; mu_c = mu_n; mu_n = Q[0].mu;
    imu_p = imu_c; imu_c = imu_n;
    lam_p = lam_c; lam_c = Q[0].lam;
#pragma unroll
    for (int d = 0; d + 1 < DEPTH; d++) Q[d] = Q[d + 1];
    Q[DEPTH - 1] = Qn;
    nb_rt = nbn_rt; nb_tt = nbn_tt; nb_tz = nbn_tz; nb_rho = nbn_rho;
    imuJ_p = imuJ_c; imuJ_c = imuJ_n;
  }
}

}  // namespace

int fused_tiles(int nt, int nz, int *own_rows, int *ntile_z)
{
  *own_rows = nt < TJ - 2 ? nt : TJ - 2;
  *ntile_z = (nz + ZT - 1) / ZT;
  const int ntile_t = (nt + *own_rows - 1) / *own_rows;
  return ntile_t * *ntile_z;
}

size_t fused_lds_bytes(int nr) { return (size_t)NRT * nr * sizeof(float); }

hipError_t launch_fused(const FusedArgs &f, hipStream_t stream)
{
  const int tiles = (f.nt + f.own_rows - 1) / f.own_rows * f.ntile_z;
  hipLaunchKernelGGL(k_step_fused, dim3(tiles), dim3(TJ * 64), fused_lds_bytes(f.nr), stream, f);
  return hipGetLastError();
}

}  // namespace cw
