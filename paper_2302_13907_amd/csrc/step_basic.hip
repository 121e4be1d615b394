// Two-pass time step: one thread per cell, k (depth) across the lanes so
// every load of a wavefront is one contiguous run.  The velocity and stress
// updates are separate launches; the one-cell stress update adds the step's
// stress sources itself (the other forms take a small source launch, as do
// force sources after the velocity update); a last launch samples the
// receivers, sets the float16 scales and advances the step counter (with
// float32 storage only after the last step of a run of steps: the velocity
// launch of the next step does that work for the step before it).  The
// energy and the batched source and receiver kernels live here too.  The fields may be stored in float32, float16
// (with a power-of-two scale per field, chosen on the device from the
// largest magnitude written in the previous step) or bfloat16; every
// arithmetic operation is float32.
//
// The discrete operators are the staggered-grid form (Sec. 3) of Eq. (1):
//   rho dv_r/dt = ds_rr/dr + (1/r)(ds_rt/dth + s_rr - s_tt) + ds_rz/dz
//   rho dv_t/dt = ds_rt/dr + (1/r)(ds_tt/dth + 2 s_rt)      + ds_tz/dz
//   rho dv_z/dt = ds_rz/dr + (1/r)(ds_tz/dth + s_rz)        + ds_zz/dz
//   ds_qq/dt = lam tr(e) + 2 mu e_qq, e_rr = dv_r/dr,
//              e_tt = (1/r)(dv_t/dth + v_r), e_zz = dv_z/dz
//   ds_rt/dt = mu (dv_t/dr + (1/r)(dv_r/dth - v_t))
//   ds_rz/dt = mu (dv_z/dr + dv_r/dz),  ds_tz/dt = mu ((1/r) dv_z/dth + dv_t/dz)
// with the curvature terms averaged onto each node, zero values beyond the
// axis and the outer faces, and every r- or z-derivative term and 1/r
// bracket passed through the absorbing layer's recursive convolution.
#include "cwell_internal.hpp"
#include "storage.hpp"

namespace cw {

namespace {

__device__ __forceinline__ size_t at(const StepArgs &a, int i, int j, int k)
{
  return (size_t)i * a.rs + (size_t)j * a.nz + k;
}

// index of cell (i, j, k) in the medium arrays
__device__ __forceinline__ size_t mat(const StepArgs &a, int i, int j, int k)
{
  return (size_t)i * a.m_ring + (size_t)j * a.m_row + k;
}

// Element offsets of the columns one cell update reads, formed once per
// workgroup in scalar registers: the field columns (i, j), (i +- 1, j) and
// (i, j +- 1) (azimuth periodic), and the medium columns (i, j), (i1, j),
// (i, j + 1), (i1, j + 1) with i1 = min(i + 1, m_last).  A radial neighbour
// beyond the axis or the outer face reads zero; its offset then names the
// cell's own column, so that every load stays inside the arrays and no load
// needs a branch.  (A bounds-checked load per (i, j, k) made the compiler
// redo the 64-bit column product and an exec-mask branch for each load: about
// 500 scalar instructions per wavefront in the velocity update, nearly all
// the issue slots of the CU's one scalar unit; with the offsets the launch
// takes 2.68 ms instead of 3.68 at 256 x 128 x 8192 in float32.)
struct Cols {
  size_t c, ip, im, jp, jm;
  size_t m, m_i1, m_jp, m_i1jp;
  bool ip_in, im_in;
};

__device__ __forceinline__ Cols cols(const StepArgs &a, int i, int j)
{
  const int jm = j == 0 ? a.nt - 1 : j - 1;
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const int i1 = i + 1 <= a.m_last ? i + 1 : a.m_last;
  const size_t nz = (size_t)a.nz, base = (size_t)i * a.rs, ring = a.rs;
  Cols q;
  q.c = base + (size_t)j * nz;
  q.jp = base + (size_t)jp * nz;
  q.jm = base + (size_t)jm * nz;
  q.ip_in = i + 1 < a.nr;
  q.im_in = i > 0;
  q.ip = q.ip_in ? q.c + ring : q.c;
  q.im = q.im_in ? q.c - ring : q.c;
  q.m = (size_t)i * a.m_ring + (size_t)j * a.m_row;
  q.m_i1 = (size_t)i1 * a.m_ring + (size_t)j * a.m_row;
  q.m_jp = (size_t)i * a.m_ring + (size_t)jp * a.m_row;
  q.m_i1jp = (size_t)i1 * a.m_ring + (size_t)jp * a.m_row;
  return q;
}

// Value at (i, j, k) read with bounds checks: zero beyond the axis, the
// outer face and the top and bottom faces.  The stress update reads its
// depth neighbours this way: measured on MI355X at 256 x 128 x 8192
// (float32), 3.19 ms per launch against 3.27 with the clamped loads of ldz
// below and 3.20 with a branch on k over the column offset.
template <class S>
__device__ __forceinline__ float ld(const float *f, float s, const StepArgs &a, int i, int j, int k)
{
  if (i < 0 || i >= a.nr || k < 0 || k >= a.nz) return 0.0f;
  return S::ld(f, at(a, i, j, k), s);
}

// depth k of column col
template <class S>
__device__ __forceinline__ float ldc(const float *f, float s, size_t col, int k) { return S::ld(f, col + k, s); }

// depth k of a radial neighbour column; zero when it lies outside the grid
template <class S>
__device__ __forceinline__ float ldr(const float *f, float s, bool in, size_t col, int k)
{
  const float v = S::ld(f, col + k, s);
  return in ? v : 0.0f;
}

// The same reads, non-temporal: for the last read of a value in the
// launch's dispatch order (ring by ring, then azimuth, then depth), after
// which no other column needs the line; the first and middle reads stay
// cached for the neighbours that follow.  Measured at 256 x 128 x 8192:
// velocity launch 2.652 -> 2.603 ms with its five last reads (own sigma_rr
// and sigma_tt, sigma_rt and sigma_rz of the ring before, sigma_tz of the
// row before) non-temporal, stress launch 3.165 -> 3.160 with v_r of the
// ring before; the stress update's own v_z, which the next depth cell of
// the same wavefront reads again, took 3.214.
template <class S>
__device__ __forceinline__ float ldcn(const float *f, float s, size_t col, int k) { return S::ldn(f, col + k, s); }
template <class S>
__device__ __forceinline__ float ldrn(const float *f, float s, bool in, size_t col, int k)
{
  const float v = S::ldn(f, col + k, s);
  return in ? v : 0.0f;
}

// depth neighbour k (the lane's depth +- 1) of column col; zero beyond the
// top and bottom faces, where the load itself is clamped into the column
template <class S>
__device__ __forceinline__ float ldz(const float *f, float s, const StepArgs &a, size_t col, int k)
{
  const int kc = k < 0 ? 0 : (k >= a.nz ? a.nz - 1 : k);
  const float v = S::ld(f, col + kc, s);
  return k < 0 || k >= a.nz ? 0.0f : v;
}

// Reciprocal: the hardware v_rcp_f32 (1 ulp).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Harmonic mean of four moduli: 4 / (1/a + 1/b + 1/c + 1/d).  A zero
// argument makes its reciprocal +inf and the mean exactly zero.
__device__ __forceinline__ float hm4(float p, float q, float r, float s)
{
  return 4.0f * rcp(rcp(p) + rcp(q) + rcp(r) + rcp(s));
}

// z-slab row of depth index k, or -1 outside the slabs.
__device__ __forceinline__ int zrow(const StepArgs &a, int k)
{
  if (a.npz == 0) return -1;
  if (k < a.npz) return k;
  int lo = a.nz - 1 - a.npz;
  if (k >= lo) return k - lo + a.npz;
  return -1;
}

// Layer memory of one cell (read and written only by that cell:
// non-temporal).  A layer block reads every coefficient and memory value it
// needs (ldpsi) before it writes any (cpml): a store could alias a later
// read, so one array after the other would cost the cell a memory round
// trip per array, six in a radial layer.
__device__ __forceinline__ float ldpsi(const float *psi, size_t p)
{
  return CW_NT_OWN ? __builtin_nontemporal_load(psi + p) : psi[p];
}
// psi <- b psi + a X from the value old read at p; returns X + psi
__device__ __forceinline__ float cpml(float *psi, size_t p, float old, float ca, float cb, float X)
{
  const float v = cb * old + ca * X;
  if (CW_NT_STORE) __builtin_nontemporal_store(v, psi + p);
  else psi[p] = v;
  return X + v;
}

// largest |x| over the wavefront into one of the field's slots: one
// atomic per wavefront, spread over kMaxSlots addresses (float bits of a
// non-negative float order like unsigned integers)
__device__ __forceinline__ void track_max(unsigned *slots, float x)
{
  float m = fabsf(x);
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0f)
    atomicMax(&slots[(blockIdx.x + (threadIdx.x >> 6)) & (kMaxSlots - 1)], __builtin_bit_cast(unsigned, m));
}

// One wavefront per receiver; float64 sum over the ring in a fixed order.
// Samples the level-(n+1) buffer a.out, or with kIn the level-n buffer a.in
// (the previous step's result).
template <class S, bool kIn = false>
__device__ void record_one(const Receiver &r, int m, int64_t step, int64_t cap, const StepArgs &a, double *traces)
{
  const int lane = threadIdx.x & 63;
  const int j0 = r.j < 0 ? 0 : r.j, j1 = r.j < 0 ? a.nt : r.j + 1;
  const float *o = kIn ? a.scl_in : a.scl_out;
  const float *const *F = kIn ? a.in : a.out;
  double acc = 0.0;
  for (int j = j0 + lane; j < j1; j += 64) {
    const size_t p = at(a, r.i, j, r.k);
    if (r.kind == 0)
      acc += (double)S::ld(F[SRR], p, o[SRR]) + (double)S::ld(F[STT], p, o[STT]) +
             (double)S::ld(F[SZZ], p, o[SZZ]);
    else
      acc += (double)S::ld(F[r.field], p, o[r.field]);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    const double cnt = (double)(j1 - j0);
    traces[(size_t)m * cap + step] = r.kind == 0 ? -acc / (3.0 * cnt) : acc / cnt;
  }
}


// The receivers and the step counter of the previous step, done by T.blocks
// extra workgroups of the velocity launch that follows it instead of by a
// launch of their own: workgroup b samples receivers 4b .. 4b+3 (one
// wavefront each) from the buffer this step reads (the previous step's
// result, which no launch of this step writes); the last of these
// workgroups to finish, once every one of them has read the counter,
// advances it.  T.done is a zeroed counter of finished workgroups, left at
// zero.  No other workgroup of the launch reads the step counter.
template <class S>
__device__ void previous_step_tail(const TailArgs &T, const StepArgs &a)
{
  const int m = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (m < T.nrec) record_one<S, true>(T.rec[m], m, *T.step, T.cap, a, T.traces);
  __shared__ unsigned ticket;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    ticket = atomicAdd(T.done, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0 && ticket == (unsigned)T.blocks - 1) {
    __threadfence();
    *T.done = 0u;
    *T.step += 1;
  }
}

// kTail: T.blocks extra workgroups at the front of the grid finish the
// previous step (previous_step_tail) and update no cells; the others take
// the column segments in the same order as without them
template <class S, bool kTail>
__global__ void __launch_bounds__(256) k_velocity_basic(StepArgs a, int nbx, TailArgs T)
{
  if (kTail && (int)blockIdx.x < T.blocks) {
    previous_step_tail<S>(T, a);
    return;
  }
  const int t = kTail ? (int)blockIdx.x - T.blocks : xcd_tile(blockIdx.x, gridDim.x);
  const int bx = t % nbx;
  const int k = bx * 256 + threadIdx.x;
  int i, j;
  strip_column(t / nbx, a.nr, a.nt, i, j);
  const bool live = k < a.nz;
  const int kk = live ? k : a.nz - 1;              // dead lanes compute on a valid cell, store nothing
  const Cols col = cols(a, i, j);
  const float *sRR = a.in[SRR], *sTT = a.in[STT], *sZZ = a.in[SZZ];
  const float *sRT = a.in[SRT], *sRZ = a.in[SRZ], *sTZ = a.in[STZ];
  const float *c = a.scl_in;

  const float srr0 = ldcn<S>(sRR, c[SRR], col.c, kk), srr1 = ldr<S>(sRR, c[SRR], col.ip_in, col.ip, kk);
  const float stt0 = ldcn<S>(sTT, c[STT], col.c, kk), stt1 = ldr<S>(sTT, c[STT], col.ip_in, col.ip, kk);
  const float stt_jp = ldc<S>(sTT, c[STT], col.jp, kk);
  const float srt0 = ldc<S>(sRT, c[SRT], col.c, kk), srt_jm = ldc<S>(sRT, c[SRT], col.jm, kk);
  const float srt_im = ldrn<S>(sRT, c[SRT], col.im_in, col.im, kk);
  const float srz0 = ldc<S>(sRZ, c[SRZ], col.c, kk), srz_km = ldz<S>(sRZ, c[SRZ], a, col.c, kk - 1);
  const float srz_im = ldrn<S>(sRZ, c[SRZ], col.im_in, col.im, kk);
  const float stz0 = ldc<S>(sTZ, c[STZ], col.c, kk), stz_jm = ldcn<S>(sTZ, c[STZ], col.jm, kk);
  const float stz_km = ldz<S>(sTZ, c[STZ], a, col.c, kk - 1);
  const float szz0 = ldc<S>(sZZ, c[SZZ], col.c, kk), szz_kp = ldz<S>(sZZ, c[SZZ], a, col.c, kk + 1);

  const float irc = a.inv_rc[i], irf = a.inv_rf[i];
  // v_r at (R_i, th_j, z_k)
  float r_dr = (srr1 - srr0) * a.inv_dr;
  float r_b = irf * ((srt0 - srt_jm) * a.inv_dth + 0.5f * (srr1 + srr0) - 0.5f * (stt1 + stt0));
  float r_dz = (srz0 - srz_km) * a.inv_dz;
  // v_t at (r_i, th_j+1/2, z_k)
  float t_dr = (srt0 - srt_im) * a.inv_dr;
  float t_b = irc * ((stt_jp - stt0) * a.inv_dth + (srt0 + srt_im));
  float t_dz = (stz0 - stz_km) * a.inv_dz;
  // v_z at (r_i, th_j, z_k+1/2)
  float z_dr = (srz0 - srz_im) * a.inv_dr;
  float z_b = irc * ((stz0 - stz_jm) * a.inv_dth + 0.5f * (srz0 + srz_im));
  float z_dz = (szz_kp - szz0) * a.inv_dz;

  // buoyancies (arithmetic mean of the two adjacent densities, clamped at
  // the edges) and the old velocities, read before the layer block: its
  // stores could alias them, so read after it they would cost the cell a
  // second memory round trip (measured at 256 x 128 x 8192: 2.676 against
  // 2.693 ms per launch)
  const int k1 = kk + 1 < a.nz ? kk + 1 : a.nz - 1;
  const size_t p = col.c + kk;
  const float rho0 = a.rho[col.m + kk];
  const float b_r = 2.0f * rcp(rho0 + a.rho[col.m_i1 + kk]);
  const float b_t = 2.0f * rcp(rho0 + a.rho[col.m_jp + kk]);
  const float b_z = 2.0f * rcp(rho0 + a.rho[col.m + k1]);
  const float vr_old = S::ldn(a.in[VR], p, c[VR]), vt_old = S::ldn(a.in[VT], p, c[VT]);
  const float vz_old = S::ldn(a.in[VZ], p, c[VZ]);

  // The radial and the depth layer blocks read their memory and coefficients
  // before either block writes: a store could alias a later read, so the
  // depth block's reads would otherwise wait for the radial block's stores,
  // a second memory round trip for the cells in both layers (which set the
  // launch's length on small grids: 48 x 32 x 192, 16.5 -> 15.8 us per step
  // with the stress update read the same way; 256 x 128 x 8192 unchanged).
  const int ir = i - (a.nr - a.npr);
  const bool lr = ir >= 0 && live;
  const int kz = live ? zrow(a, k) : -1;
  const bool lz = kz >= 0;
  const size_t qr = lr ? ((size_t)ir * a.nt + j) * a.nz + k : 0;
  const size_t qz = lz ? ((size_t)i * a.nt + j) * a.nzs + kz : 0;
  float *const *P = a.psi_r;
  float *const *Z = a.psi_z;
  float arf = 0, brf = 0, atf = 0, btf = 0, arc = 0, brc = 0, atc = 0, btc = 0;
  float m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0;
  float azc = 0, bzc = 0, azh = 0, bzh = 0, n0 = 0, n1 = 0, n2 = 0;
  if (lr) {
    const float *T = a.tab_r;
    arf = T[AR_F * a.nr + i]; brf = T[BR_F * a.nr + i]; atf = T[AT_F * a.nr + i]; btf = T[BT_F * a.nr + i];
    arc = T[AR_C * a.nr + i]; brc = T[BR_C * a.nr + i]; atc = T[AT_C * a.nr + i]; btc = T[BT_C * a.nr + i];
    m0 = ldpsi(P[R_VR_DR], qr); m1 = ldpsi(P[R_VR_B], qr); m2 = ldpsi(P[R_VT_DR], qr);
    m3 = ldpsi(P[R_VT_B], qr); m4 = ldpsi(P[R_VZ_DR], qr); m5 = ldpsi(P[R_VZ_B], qr);
  }
  if (lz) {
    const float *T = a.tab_z;
    azc = T[AZ_C * a.nz + k]; bzc = T[BZ_C * a.nz + k]; azh = T[AZ_H * a.nz + k]; bzh = T[BZ_H * a.nz + k];
    n0 = ldpsi(Z[Z_VR_DZ], qz); n1 = ldpsi(Z[Z_VT_DZ], qz); n2 = ldpsi(Z[Z_VZ_DZ], qz);
  }
  if (lr) {
    r_dr = cpml(P[R_VR_DR], qr, m0, arf, brf, r_dr);
    r_b = cpml(P[R_VR_B], qr, m1, atf, btf, r_b);
    t_dr = cpml(P[R_VT_DR], qr, m2, arc, brc, t_dr);
    t_b = cpml(P[R_VT_B], qr, m3, atc, btc, t_b);
    z_dr = cpml(P[R_VZ_DR], qr, m4, arc, brc, z_dr);
    z_b = cpml(P[R_VZ_B], qr, m5, atc, btc, z_b);
  }
  if (lz) {
    r_dz = cpml(Z[Z_VR_DZ], qz, n0, azc, bzc, r_dz);
    t_dz = cpml(Z[Z_VT_DZ], qz, n1, azc, bzc, t_dz);
    z_dz = cpml(Z[Z_VZ_DZ], qz, n2, azh, bzh, z_dz);
  }

  const float vr = vr_old + a.dt * b_r * (r_dr + r_b + r_dz);
  const float vt = vt_old + a.dt * b_t * (t_dr + t_b + t_dz);
  const float vz = vz_old + a.dt * b_z * (z_dr + z_b + z_dz);
  if (live) {
    const float *o = a.scl_out;
    const bool sr = sr_on<S>(a);
    const unsigned sb = sr_base<S>(a, p);
    S::stn(a.out[VR], p, vr, 1.0f / o[VR], sr_key(sb, VR), sr);
    S::stn(a.out[VT], p, vt, 1.0f / o[VT], sr_key(sb, VT), sr);
    S::stn(a.out[VZ], p, vz, 1.0f / o[VZ], sr_key(sb, VZ), sr);
  }
  if (S::scaled) {
    track_max(a.maxabs + VR * kMaxSlots, live ? vr : 0.0f);
    track_max(a.maxabs + VT * kMaxSlots, live ? vt : 0.0f);
    track_max(a.maxabs + VZ * kMaxSlots, live ? vz : 0.0f);
  }
}

// stress update of the thread's cell (i, j, k); mx collects |sigma| maxima
template <class S>
__device__ __forceinline__ void stress_cell(const StepArgs &a, int i, int j, int k, float (&mx)[6])
{
  const bool live = k < a.nz;
  const int kk = live ? k : a.nz - 1;              // dead lanes compute on a valid cell, store nothing
  const Cols col = cols(a, i, j);
  // velocities at level n+1/2 are in the output buffer
  const float *vR = a.out[VR], *vT = a.out[VT], *vZ = a.out[VZ];
  const float *o = a.scl_out;

  const float vr0 = ldc<S>(vR, o[VR], col.c, kk), vr_im = ldrn<S>(vR, o[VR], col.im_in, col.im, kk);
  const float vr_jp = ldc<S>(vR, o[VR], col.jp, kk), vr_kp = ld<S>(vR, o[VR], a, i, j, kk + 1);
  const float vt0 = ldc<S>(vT, o[VT], col.c, kk), vt_jm = ldc<S>(vT, o[VT], col.jm, kk);
  const float vt_ip = ldr<S>(vT, o[VT], col.ip_in, col.ip, kk), vt_kp = ld<S>(vT, o[VT], a, i, j, kk + 1);
  const float vz0 = ldc<S>(vZ, o[VZ], col.c, kk), vz_km = ld<S>(vZ, o[VZ], a, i, j, kk - 1);
  const float vz_ip = ldr<S>(vZ, o[VZ], col.ip_in, col.ip, kk), vz_jp = ldc<S>(vZ, o[VZ], col.jp, kk);

  const float irc = a.inv_rc[i], irf = a.inv_rf[i];
  float err = (vr0 - vr_im) * a.inv_dr;
  float ett = irc * ((vt0 - vt_jm) * a.inv_dth + 0.5f * (vr0 + vr_im));
  float ezz = (vz0 - vz_km) * a.inv_dz;
  float rt_dr = (vt_ip - vt0) * a.inv_dr;
  float rt_b = irf * ((vr_jp - vr0) * a.inv_dth - 0.5f * (vt_ip + vt0));
  float rz_dr = (vz_ip - vz0) * a.inv_dr;
  float rz_dz = (vr_kp - vr0) * a.inv_dz;
  float tz_b = irc * (vz_jp - vz0) * a.inv_dth;
  float tz_dz = (vt_kp - vt0) * a.inv_dz;

  // Everything the cell reads from memory is read before the first layer
  // store, which could alias a later read and make it wait: the old
  // stresses, both layer blocks' memory and coefficients, then the moduli.
  // At 256 x 128 x 8192 the launch takes 3.16 ms in this order as in the
  // earlier one (layer blocks one after the other, moduli after them); at
  // 48 x 32 x 192, where the cells of both layers set the launch's length,
  // the step drops from 16.5 to 15.8 us with the velocity update read the
  // same way.  (With the blocks apart, reading the moduli before them cost
  // 3.182 ms against 3.160.)
  const int k1 = kk + 1 < a.nz ? kk + 1 : a.nz - 1;
  const size_t p = col.c + kk;
  const size_t pm = col.m + kk;
  const float *c = a.scl_in;
  const float so_rr = S::ldn(a.in[SRR], p, c[SRR]), so_tt = S::ldn(a.in[STT], p, c[STT]);
  const float so_zz = S::ldn(a.in[SZZ], p, c[SZZ]), so_rt = S::ldn(a.in[SRT], p, c[SRT]);
  const float so_rz = S::ldn(a.in[SRZ], p, c[SRZ]), so_tz = S::ldn(a.in[STZ], p, c[STZ]);
  const int ir = i - (a.nr - a.npr);
  const bool lr = ir >= 0 && live;
  const int kz = live ? zrow(a, k) : -1;
  const bool lz = kz >= 0;
  const size_t qr = lr ? ((size_t)ir * a.nt + j) * a.nz + k : 0;
  const size_t qz = lz ? ((size_t)i * a.nt + j) * a.nzs + kz : 0;
  float *const *P = a.psi_r;
  float *const *Z = a.psi_z;
  float arf = 0, brf = 0, atf = 0, btf = 0, arc = 0, brc = 0, atc = 0, btc = 0;
  float g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
  float azc = 0, bzc = 0, azh = 0, bzh = 0, n0 = 0, n1 = 0, n2 = 0;
  if (lr) {
    const float *T = a.tab_r;
    arf = T[AR_F * a.nr + i]; brf = T[BR_F * a.nr + i]; atf = T[AT_F * a.nr + i]; btf = T[BT_F * a.nr + i];
    arc = T[AR_C * a.nr + i]; brc = T[BR_C * a.nr + i]; atc = T[AT_C * a.nr + i]; btc = T[BT_C * a.nr + i];
    g0 = ldpsi(P[R_N_DR], qr); g1 = ldpsi(P[R_N_B], qr); g2 = ldpsi(P[R_RT_DR], qr);
    g3 = ldpsi(P[R_RT_B], qr); g4 = ldpsi(P[R_RZ_DR], qr); g5 = ldpsi(P[R_TZ_B], qr);
  }
  if (lz) {
    const float *T = a.tab_z;
    azc = T[AZ_C * a.nz + k]; bzc = T[BZ_C * a.nz + k]; azh = T[AZ_H * a.nz + k]; bzh = T[BZ_H * a.nz + k];
    n0 = ldpsi(Z[Z_N_DZ], qz); n1 = ldpsi(Z[Z_RZ_DZ], qz); n2 = ldpsi(Z[Z_TZ_DZ], qz);
  }
  const float lam = a.lam[pm], mu = a.mu[pm];
  const float mu_i1 = a.mu[col.m_i1 + kk], mu_jp = a.mu[col.m_jp + kk];
  const float mu_k1 = a.mu[col.m + k1];
  const float mu_i1jp = a.mu[col.m_i1jp + kk], mu_i1k1 = a.mu[col.m_i1 + k1], mu_jpk1 = a.mu[col.m_jp + k1];
  if (lr) {
    err = cpml(P[R_N_DR], qr, g0, arc, brc, err);
    ett = cpml(P[R_N_B], qr, g1, atc, btc, ett);
    rt_dr = cpml(P[R_RT_DR], qr, g2, arf, brf, rt_dr);
    rt_b = cpml(P[R_RT_B], qr, g3, atf, btf, rt_b);
    rz_dr = cpml(P[R_RZ_DR], qr, g4, arf, brf, rz_dr);
    tz_b = cpml(P[R_TZ_B], qr, g5, atc, btc, tz_b);
  }
  if (lz) {
    ezz = cpml(Z[Z_N_DZ], qz, n0, azc, bzc, ezz);
    rz_dz = cpml(Z[Z_RZ_DZ], qz, n1, azh, bzh, rz_dz);
    tz_dz = cpml(Z[Z_TZ_DZ], qz, n2, azh, bzh, tz_dz);
  }
  const float mu_rt = hm4(mu, mu_i1, mu_jp, mu_i1jp);
  const float mu_rz = hm4(mu, mu_i1, mu_k1, mu_i1k1);
  const float mu_tz = hm4(mu, mu_jp, mu_k1, mu_jpk1);

  const float tr = err + ett + ezz;
  const float lt = lam * tr, m2 = 2.0f * mu;
  float s_rr = so_rr + a.dt * (lt + m2 * err);
  float s_tt = so_tt + a.dt * (lt + m2 * ett);
  float s_zz = so_zz + a.dt * (lt + m2 * ezz);
  float s_rt = so_rt + a.dt * mu_rt * (rt_dr + rt_b);
  float s_rz = so_rz + a.dt * mu_rz * (rz_dr + rz_dz);
  float s_tz = so_tz + a.dt * mu_tz * (tz_b + tz_dz);
  // this step's stress sources at the cell, in the order they were added
  // (only workgroups of the rings the sources touch look at the list: the
  // scalar unit is this kernel's busiest)
  if (a.inj && live && i >= a.inj_i0 && i <= a.inj_i1) {
    const int64_t n = *a.step;
    for (int m = 0; m < a.ninj; m++) {
      const Inject s = a.inj[m];
      if (s.phase != 1 || s.i != i || (s.j >= 0 && s.j != j) || s.k != k || n >= s.nsamp) continue;
      const float amp = s.scale * s.amp[n];
      switch (s.field) {
      case SRR: s_rr += amp; break;
      case STT: s_tt += amp; break;
      case SZZ: s_zz += amp; break;
      case SRT: s_rt += amp; break;
      case SRZ: s_rz += amp; break;
      case STZ: s_tz += amp; break;
      default: break;
      }
    }
  }
  if (live) {
    const bool sr = sr_on<S>(a);
    const unsigned sb = sr_base<S>(a, p);
    S::stn(a.out[SRR], p, s_rr, 1.0f / o[SRR], sr_key(sb, SRR), sr);
    S::stn(a.out[STT], p, s_tt, 1.0f / o[STT], sr_key(sb, STT), sr);
    S::stn(a.out[SZZ], p, s_zz, 1.0f / o[SZZ], sr_key(sb, SZZ), sr);
    S::stn(a.out[SRT], p, s_rt, 1.0f / o[SRT], sr_key(sb, SRT), sr);
    S::stn(a.out[SRZ], p, s_rz, 1.0f / o[SRZ], sr_key(sb, SRZ), sr);
    S::stn(a.out[STZ], p, s_tz, 1.0f / o[STZ], sr_key(sb, STZ), sr);
  }
  if (S::scaled && live) {
    mx[0] = fmaxf(mx[0], fabsf(s_rr)); mx[1] = fmaxf(mx[1], fabsf(s_tt)); mx[2] = fmaxf(mx[2], fabsf(s_zz));
    mx[3] = fmaxf(mx[3], fabsf(s_rt)); mx[4] = fmaxf(mx[4], fabsf(s_rz)); mx[5] = fmaxf(mx[5], fabsf(s_tz));
  }
}

// Depth segments of 256 cells a workgroup takes one after the other: the
// (ring, row) set-up -- scalar base addresses of every array and row -- is
// paid once per kOneSegs segments.  Measured on MI355X at 256 x 128 x 8192
// (float32): 2, 4 and 8 segments 3.42, 3.36 and 3.48 ms against 3.28 for
// one, so one it is.
#ifndef CW_ONE_SEGS
#define CW_ONE_SEGS 1
#endif
constexpr int kOneSegs = CW_ONE_SEGS;

template <class S>
__global__ void __launch_bounds__(256) k_stress_basic(StepArgs a, int nbx)
{
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int bx = t % nbx;
  int i, j;
  strip_column(t / nbx, a.nr, a.nt, i, j);
  float mx[6] = {0, 0, 0, 0, 0, 0};
  for (int q = 0; q < kOneSegs; q++) {
    const int k0 = (bx * kOneSegs + q) * 256;
    if (k0 >= a.nz) break;                         // the whole workgroup
    stress_cell<S>(a, i, j, k0 + (int)threadIdx.x, mx);
  }
  if (S::scaled)
    for (int q = 0; q < 6; q++) track_max(a.maxabs + (SRR + q) * kMaxSlots, mx[q]);
}

// One block applies every injection of the phase in list order, so two
// sources hitting the same node add in a fixed order.
template <class S>
__device__ void inject_all(const Inject *list, int ninj, int phase, int64_t step, const StepArgs &a)
{
  for (int m = 0; m < ninj; m++) {
    const Inject e = list[m];
    if (e.phase == phase && step < e.nsamp) {
      const float amp = e.scale * e.amp[step];
      float *f = a.out[e.field];
      const float s = a.scl_out[e.field];
      const int j0 = e.j >= 0 ? e.j : 0, j1 = e.j >= 0 ? e.j + 1 : a.nt;
      for (int j = j0 + (int)threadIdx.x; j < j1; j += blockDim.x) {
        const size_t p = at(a, e.i, j, e.k);
        const float v = S::ld(f, p, s) + amp;
        S::st(f, p, v, 1.0f / s);
        if (S::scaled) atomicMax(&a.maxabs[e.field * kMaxSlots], __builtin_bit_cast(unsigned, fabsf(v)));
      }
    }
    __syncthreads();
  }
}

// the sources of one phase of a solo step: forces (phase 0) after the
// velocity update, stresses (phase 1) after the four-cell stress update
template <class S>
__global__ void __launch_bounds__(256) k_inject(StepArgs a, int phase)
{
  inject_all<S>(a.inj, a.ninj, phase, *a.step, a);
}

__global__ void __launch_bounds__(256) k_inject_batch(const BatchInst *B, int phase, int parity)
{
  const BatchInst &I = B[blockIdx.x];
  inject_all<StF32>(I.inject, I.ninj, phase, *I.step, I.a[parity]);
}

// New float16 scale of field q: 2^(e - target) with max|v| = f 2^e,
// f in [0.5, 1); unchanged while the field is still identically zero.  The
// maxima slots are cleared for the next step.  The maxima are of the
// float32 values before their conversion, so a maximum of 65520 or more
// times the scale they were stored with means that a value outran the
// scale's headroom (2^16 / 2^target) in one step and was stored as
// infinity (65520 is the least value that float16 rounds to infinity), and
// a NaN maximum that a NaN was written: the field's bit is set in the
// overflow word, which stays set until the state is reset.
__device__ void rescale_field(int q, float *scl_written, float *scl_next, unsigned *maxabs)
{
  const float used = scl_next[q];
  scl_written[q] = used;
  unsigned mb = 0u;
  for (int c = 0; c < kMaxSlots; c++) {
    mb = max(mb, maxabs[q * kMaxSlots + c]);
    maxabs[q * kMaxSlots + c] = 0u;
  }
  const float m = __builtin_bit_cast(float, mb);
  if (m != m || m >= 65520.0f * used) {
    atomicOr(&maxabs[kOverflowWord], 1u << q);
  } else if (m > 0.0f) {
    int e;
    frexpf(m, &e);
    scl_next[q] = ldexpf(1.0f, e - kF16TargetExp);
  }
}

// The last launch of a solo step: one workgroup per receiver, then -- in the
// workgroup that finishes last, once every other one has read the step
// counter and the scales -- the float16 scales and the step counter.  The
// finish counter is left at zero for the next step.
template <class S>
__global__ void __launch_bounds__(64) k_step_tail(const Receiver *rec, int nrec, int64_t *stepp, int64_t cap,
                                                  StepArgs a, double *traces, unsigned *done, float *scl_written,
                                                  float *scl_next, unsigned *maxabs)
{
  if ((int)blockIdx.x < nrec) record_one<S>(rec[blockIdx.x], blockIdx.x, *stepp, cap, a, traces);
  __shared__ unsigned ticket;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    ticket = atomicAdd(done, 1u);
  }
  __syncthreads();
  if (ticket != gridDim.x - 1) return;
  __threadfence();
  if (S::scaled && threadIdx.x < NF) rescale_field(threadIdx.x, scl_written, scl_next, maxabs);
  if (threadIdx.x == 0) {
    *done = 0u;
    *stepp += 1;
  }
}

// grid (receivers of the largest instance, instances)
__global__ void __launch_bounds__(64) k_record_batch(const BatchInst *B, int parity)
{
  const BatchInst &I = B[blockIdx.y];
  if ((int)blockIdx.x >= I.nrec) return;
  record_one<StF32>(I.rec[blockIdx.x], blockIdx.x, *I.step, I.cap, I.a[parity], I.traces);
}

__global__ void k_step_done_batch(const BatchInst *B, int count)
{
  const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (q < count) *B[q].step += 1;
}

// Energy density of one cell in float64; a.in = level n, a.out = level n+1.
template <class S>
__device__ double cell_energy(const StepArgs &a, int i, int j, int k)
{
  const int jp = j == a.nt - 1 ? 0 : j + 1;
  const int i1 = i + 1 <= a.m_last ? i + 1 : a.m_last;
  const int k1 = k + 1 < a.nz ? k + 1 : a.nz - 1;
  const size_t p = at(a, i, j, k);
  const float *ci = a.scl_in, *co = a.scl_out;
  const double ri = (double)(a.ring0 + i + 0.5), Ri = (double)(a.ring0 + i + 1);   // radii in units of dr
  const size_t pm = mat(a, i, j, k);
  const double rho0 = a.rho[pm];
  const double rr = 0.5 * (rho0 + a.rho[mat(a, i1, j, k)]);
  const double rt = 0.5 * (rho0 + a.rho[mat(a, i, jp, k)]);
  const double rz = 0.5 * (rho0 + a.rho[mat(a, i, j, k1)]);
  const double vr = S::ld(a.out[VR], p, co[VR]), vt = S::ld(a.out[VT], p, co[VT]);
  const double vz = S::ld(a.out[VZ], p, co[VZ]);
  double E = 0.5 * (Ri * rr * vr * vr + ri * rt * vt * vt + ri * rz * vz * vz);
  const double lam = a.lam[pm], mu = a.mu[pm];
  const double K = lam + 2.0 * mu / 3.0;
  const double n1[3] = {S::ld(a.out[SRR], p, co[SRR]), S::ld(a.out[STT], p, co[STT]), S::ld(a.out[SZZ], p, co[SZZ])};
  const double n0[3] = {S::ld(a.in[SRR], p, ci[SRR]), S::ld(a.in[STT], p, ci[STT]), S::ld(a.in[SZZ], p, ci[SZZ])};
  const double t1 = n1[0] + n1[1] + n1[2], t0 = n0[0] + n0[1] + n0[2];
  E += 0.5 * ri * t1 * t0 / (9.0 * K);
  if (mu > 0.0) {
    double d = 0.0;
    for (int q = 0; q < 3; q++) d += (n1[q] - t1 / 3.0) * (n0[q] - t0 / 3.0);
    E += 0.5 * ri * d / (2.0 * mu);
  }
  const double m_i1 = a.mu[mat(a, i1, j, k)], m_jp = a.mu[mat(a, i, jp, k)], m_k1 = a.mu[mat(a, i, j, k1)];
  auto hm = [](double w, double x, double y, double z) {
    return (w == 0.0 || x == 0.0 || y == 0.0 || z == 0.0) ? 0.0 : 4.0 / (1.0 / w + 1.0 / x + 1.0 / y + 1.0 / z);
  };
  const double mrt = hm(mu, m_i1, m_jp, a.mu[mat(a, i1, jp, k)]);
  const double mrz = hm(mu, m_i1, m_k1, a.mu[mat(a, i1, j, k1)]);
  const double mtz = hm(mu, m_jp, m_k1, a.mu[mat(a, i, jp, k1)]);
  if (mrt > 0.0) E += 0.5 * Ri * (double)S::ld(a.out[SRT], p, co[SRT]) * (double)S::ld(a.in[SRT], p, ci[SRT]) / mrt;
  if (mrz > 0.0) E += 0.5 * Ri * (double)S::ld(a.out[SRZ], p, co[SRZ]) * (double)S::ld(a.in[SRZ], p, ci[SRZ]) / mrz;
  if (mtz > 0.0) E += 0.5 * ri * (double)S::ld(a.out[STZ], p, co[STZ]) * (double)S::ld(a.in[STZ], p, ci[STZ]) / mtz;
  return E;
}

template <class S>
__global__ void __launch_bounds__(256) k_energy_partial(StepArgs a, double *partials)
{
  __shared__ double red[256];
  const size_t n = (size_t)a.nr * a.nt * a.nz;
  double acc = 0.0;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (size_t)gridDim.x * 256) {
    const int k = (int)(c % a.nz);
    const size_t ij = c / a.nz;
    const int j = (int)(ij % a.nt), i = (int)(ij / a.nt);
    acc += cell_energy<S>(a, i, j, k);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_energy_final(const double *partials, int n, double scale,
                                                      double *result)
{
  __shared__ double red[256];
  double acc = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) acc += partials[c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *result = red[0] * scale;
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

hipError_t launch_velocity_basic(const StepArgs &a, int storage, hipStream_t stream, const TailArgs *tail)
{
  const int nbx = (a.nz + 255) / 256;
  const long g = (long)nbx * a.nt * a.nr;
  if (g > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (tail) {
    if (storage != ST_F32 || tail->blocks < 1 || g + tail->blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_velocity_basic<StF32, true>), dim3((unsigned)(g + tail->blocks)), dim3(256), 0, stream, a,
                       nbx, *tail);
    return hipGetLastError();
  }
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL((k_velocity_basic<decltype(s), false>), dim3((unsigned)g), dim3(256), 0, stream, a, nbx,
                       TailArgs{});
    return hipGetLastError();
  });
}

hipError_t launch_stress_basic(const StepArgs &a, int storage, hipStream_t stream)
{
  const int nbx = (a.nz + 256 * kOneSegs - 1) / (256 * kOneSegs);
  const long g = (long)nbx * a.nt * a.nr;
  if (g > 0x7fffffff) return hipErrorInvalidConfiguration;
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_stress_basic<decltype(s)>, dim3((unsigned)g), dim3(256), 0, stream, a, nbx);
    return hipGetLastError();
  });
}

hipError_t launch_sources(const StepArgs &a, int phase, int storage, hipStream_t stream)
{
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_inject<decltype(s)>, dim3(1), dim3(256), 0, stream, a, phase);
    return hipGetLastError();
  });
}

hipError_t launch_step_tail(const Receiver *dev_rec, int nrec, int64_t *step, int64_t cap, const StepArgs &a,
                            int storage, double *traces, unsigned *done, float *scl_written, float *scl_next,
                            unsigned *maxabs, hipStream_t stream)
{
  const unsigned g = nrec > 0 ? (unsigned)nrec : 1u;
  return dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_step_tail<decltype(s)>, dim3(g), dim3(64), 0, stream, dev_rec, nrec, step, cap, a, traces,
                       done, scl_written, scl_next, maxabs);
    return hipGetLastError();
  });
}

hipError_t launch_energy(const StepArgs &a, int storage, double *partials, int nblocks, double scale,
                         double *result, hipStream_t stream)
{
  hipError_t e = dispatch(storage, [&](auto s) {
    hipLaunchKernelGGL(k_energy_partial<decltype(s)>, dim3(nblocks), dim3(256), 0, stream, a, partials);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, stream, partials, nblocks, scale, result);
  return hipGetLastError();
}

hipError_t launch_inject_batch(const BatchInst *dev, int count, int phase, int parity, hipStream_t stream)
{
  hipLaunchKernelGGL(k_inject_batch, dim3(count), dim3(256), 0, stream, dev, phase, parity);
  return hipGetLastError();
}

hipError_t launch_record_batch(const BatchInst *dev, int count, int max_rec, int parity, hipStream_t stream)
{
  if (max_rec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_record_batch, dim3(max_rec, count), dim3(64), 0, stream, dev, parity);
  return hipGetLastError();
}

hipError_t launch_step_done_batch(const BatchInst *dev, int count, hipStream_t stream)
{
  hipLaunchKernelGGL(k_step_done_batch, dim3((count + 63) / 64), dim3(64), 0, stream, dev, count);
  return hipGetLastError();
}


}  // namespace cw
