// Internal declarations shared by the host API and the kernels of libcwell.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cw {

enum Field { VR = 0, VT, VZ, SRR, STT, SZZ, SRT, SRZ, STZ, NF };

// Storage of the 9 fields (arithmetic is float32 in every case).
enum Storage { ST_F32 = 0, ST_F16, ST_BF16 };
constexpr int kMaxSlots = 64;       // max-abs slots per field (float16 scale tracking)
// after the NF * kMaxSlots maxima slots: one word whose bit q says that
// float16 field q overflowed (grew past its scale's headroom in one step)
constexpr int kOverflowWord = NF * kMaxSlots;

// Layer memory variables living in the radial slab i >= nr - npml_r.
enum PsiR {
  R_VR_DR = 0, R_VR_B, R_VT_DR, R_VT_B, R_VZ_DR, R_VZ_B,
  R_N_DR, R_N_B, R_RT_DR, R_RT_B, R_RZ_DR, R_TZ_B, NPSI_R
};
// ... and in the z slabs k < npml_z, k >= nz - 1 - npml_z.
enum PsiZ { Z_VR_DZ = 0, Z_VT_DZ, Z_VZ_DZ, Z_N_DZ, Z_RZ_DZ, Z_TZ_DZ, NPSI_Z };

// Rows of the packed radial layer table (each row nr floats): damping
// coefficients a, b of the radial profile at centres r_i and faces R_i, and
// of the integrated profile (stretching 1/r) at centres and faces.
enum TabR { AR_C = 0, BR_C, AR_F, BR_F, AT_C, BT_C, AT_F, BT_F, NTAB_R };
// Rows of the packed z table (each row nz floats): at z_k and z_{k+1/2}.
enum TabZ { AZ_C = 0, BZ_C, AZ_H, BZ_H, NTAB_Z };

// One point (or ring) injection: field[(i, j or all j, k)] += scale * amp[n].
struct Inject {
  int field, i, j, k;       // j = -1: the whole ring
  int phase;                // 0: after the velocity update, 1: after the stress update
  int nsamp;                // amp has nsamp entries
  float scale;              // 1, or the node buoyancy for force sources
  const float *amp;         // dt * w[n] / V, float32
};

// Everything one time step reads and writes, by value as a kernel argument.
struct StepArgs {
  int nr, nt, nz;
  // Zones of an azimuthally refined grid: ring0 is the global index of ring 0
  // (radii are (ring0 + i + 1/2) dr); m_last is the last ring the medium
  // arrays hold (nr - 1, or nr when they include the next zone's first
  // ring); ghost_in / ghost_out: the field arrays hold a ring at i = -1 / i =
  // nr with the neighbouring zone's values on this zone's azimuthal grid,
  // read instead of the zero closure.
  int ring0, m_last, ghost_in, ghost_out;
  int npr, npz, nzs;        // layer cells in r, in z (each end), z-slab rows (2 npz + 1)
  float dt, inv_dr, inv_dz, inv_dth;
  const float *inv_rc;      // 1 / r_i  [nr]
  const float *inv_rf;      // 1 / R_i  [nr]
  // medium at cell (i, j, k): index i m_ring + j m_row + k (m_row = 0 for a
  // medium stored once per (ring, depth) because it does not vary along theta)
  const float *rho, *lam, *mu;
  size_t m_ring;
  int m_row;
  const float *in[NF];      // state at level n (v^{n-1/2}, sigma^n)
  float *out[NF];           // state at level n+1
  float *psi_r[NPSI_R];     // [npr][nt][nz]
  float *psi_z[NPSI_Z];     // [nr][nt][nzs]
  const float *tab_r;       // [NTAB_R][nr]
  const float *tab_z;       // [NTAB_Z][nz]
  // 16-bit storage: a stored value times its field's scale is the physical
  // value.  scl_in scales the level-n buffer, scl_out the level-n+1 buffer;
  // maxabs collects the largest |value| written (float bits, kMaxSlots
  // slots per field, for the next step's scale), then the overflow word
  // (kOverflowWord).  Unused (scales 1) for float32 storage.
  const float *scl_in, *scl_out;
  unsigned *maxabs;
  // Source injections of a solo two-pass step: the list, its length, the
  // rings it touches and the device step counter that indexes the
  // amplitudes.  The one-cell stress update adds the stress sources itself.
  // inj == nullptr: none.
  const Inject *inj;
  int ninj, inj_i0, inj_i1;   // inj_i0..inj_i1: the rings the sources touch
  const int64_t *step;
  // bfloat16 storage: the step kernels round their field stores
  // stochastically (random bits from the cell, the field and *step) instead
  // of to nearest even
  int sr;
  // values from one ring of a field array to the next (a ring holds nt x nz;
  // the rest is padding): cell (i, j, k) of a field is at i rs + j nz + k.
  // The layer-memory slabs and the medium keep their own unpadded layouts.
  size_t rs;
};


// One receiver: trace[id][n] = ring mean or point value.
struct Receiver {
  int kind, field, i, j, k;
};

// Workgroups are dispatched to the 8 XCDs (each with its own L2) in
// round-robin order.  This remaps the dispatch index b of a grid of G
// workgroups so that each XCD receives one contiguous range of logical
// tiles: neighbouring tiles, which share halo cache lines, then run on the
// same XCD and share its L2.
__device__ __forceinline__ int xcd_tile_remap(int b, int G)
{
  const int q8 = G >> 3, r8 = G & 7, xcd = b & 7, idx = b >> 3;
  return xcd < r8 ? xcd * (q8 + 1) + idx : r8 * (q8 + 1) + (xcd - r8) * q8 + idx;
}
// Measured on MI355X: for these streaming kernels the plain dispatch order
// (all XCDs sweeping one compact address range together) is faster than the
// per-XCD contiguous ranges, although the latter fetches slightly fewer
// bytes; the remap is therefore off unless CW_XCD_REMAP is set.
#ifndef CW_XCD_REMAP
#define CW_XCD_REMAP 0
#endif
__device__ __forceinline__ int xcd_tile(int b, int G) { return CW_XCD_REMAP ? xcd_tile_remap(b, G) : b; }

// Column order of the column-form two-pass kernels.  A column is the depth
// line of one (ring i, azimuth j) pair; the kernels read the columns next to
// their own in radius and azimuth as well.  With kStripW > 0 columns are
// visited in strips of kStripW azimuth rows, ring by ring within a strip,
// which shortens the distance between the two reads of a radial neighbour
// column.  Measured on MI355X at 256 x 128 x 8192: strips of 8 to 32 rows
// fetch up to 11 % fewer bytes but run 20-40 % slower than whole rings
// (kStripW = 0), which keep the working set of the chip in a few megabytes
// of each array; whole rings are the default.
#ifndef CW_STRIP_W
#define CW_STRIP_W 0
#endif
constexpr int kStripW = CW_STRIP_W;
__device__ __forceinline__ void strip_column(int c, int nr, int nt, int &i, int &j)
{
  if (kStripW <= 0 || kStripW >= nt) {
    i = c / nt;
    j = c - i * nt;
    return;
  }
  const int per = nr * kStripW;
  const int s = c / per, rem = c - s * per;
  const int w = nt - s * kStripW < kStripW ? nt - s * kStripW : kStripW;
  i = rem / w;
  j = s * kStripW + (rem - i * w);
}

// One injection of the current step, as the fused kernel applies it.
struct InjectStep {
  int field, i, j, k, phase;
  float amp;                // scale * dt * w[n] / V for this step
};
constexpr int kMaxFusedInject = 12;

// Arguments of the fused step.  Arrays of one kind are contiguous in the
// workspace, so each kind is one base pointer and a stride: the 9 fields
// (Field order, stride n), the medium (rho, lambda, mu, stride n), the 12
// radial and 6 z layer memory arrays (stride slab_r / slab_z), each state
// and layer memory at level n (in) and n+1 (out).  Few pointers keep the
// kernel's arguments in scalar registers.
struct FusedArgs {
  int nr, nt, nz, npr, npz, nzs;
  float dt, inv_dr, inv_dz, inv_dth;
  size_t n, slab_r, slab_z;  // n: values from one field array to the next
  size_t rs;                  // ring stride of the field arrays (StepArgs::rs)
  const float *in;
  float *out;
  const float *med;
  size_t m_n, m_ring;       // medium: stride between rho, lambda, mu; values per ring
  int m_row;                //   values per theta row (0 when the medium does not vary along theta)
  const float *psi_r_in;
  float *psi_r_out;
  const float *psi_z_in;
  float *psi_z_out;
  const float *inv_rc, *inv_rf, *tab_r, *tab_z;
  int own_rows, ntile_z;
  int ninj;
  InjectStep inj[kMaxFusedInject];
};

// Launchers (step kernels), enqueued on `stream`.
int fused_tiles(int nt, int nz, int *own_rows, int *ntile_z);
size_t fused_lds_bytes(int nr);                 // dynamic LDS of the fused step
constexpr int kMaxFusedRings = 2048;            // nr limit of the fused step (LDS tables)
hipError_t launch_fused(const FusedArgs &f, hipStream_t stream);
// The previous step's receivers and step counter, folded into the next
// velocity launch (float32 storage): blocks = ceil(max(nrec, 1) / 4) extra
// workgroups take them; done is a zeroed finish counter, left at zero.
struct TailArgs {
  const Receiver *rec;
  int nrec, blocks;
  int64_t *step;
  int64_t cap;
  double *traces;
  unsigned *done;
};
// tail: nullptr, or the previous step's tail to fold in (float32 only)
hipError_t launch_velocity_basic(const StepArgs &a, int storage, hipStream_t stream, const TailArgs *tail = nullptr);
hipError_t launch_stress_basic(const StepArgs &a, int storage, hipStream_t stream);
// The sources of one phase of a.inj in a solo step (0: forces, after the
// velocity update; 1: stresses, after a stress update that does not add
// them itself), in list order.
hipError_t launch_sources(const StepArgs &a, int phase, int storage, hipStream_t stream);
// The last launch of a solo step: the receivers, then (in whichever
// workgroup finishes last) the float16 rescale and the step counter.
// done: a zeroed counter of finished workgroups, left at zero.
hipError_t launch_step_tail(const Receiver *dev_rec, int nrec, int64_t *step, int64_t cap, const StepArgs &a,
                            int storage, double *traces, unsigned *done, float *scl_written, float *scl_next,
                            unsigned *maxabs, hipStream_t stream);
// One ghost-ring fill of an azimuthally refined grid: dst[r][k] =
// sum_j M[r][j] src[j][k], rings of nz depth cells.
struct Transfer {
  const float *src;         // source ring [ns][nz]
  float *dst;               // ghost ring [nd][nz]
  const float *M;           // [nd][ns]
  int ns, nd;
};
size_t interp_lds_bytes(int max_ns);
hipError_t launch_interp(const Transfer *dev, int count, int nz, int max_ns, hipStream_t stream);

hipError_t launch_energy(const StepArgs &a, int storage, double *partials, int nblocks, double scale,
                         double *result, hipStream_t stream);
constexpr int kF16TargetExp = 11;   // scaled float16 maxima land in [2^10, 2^11)
// depth-vectorized two-pass kernels (4 cells per thread), when nz % 4 == 0
// the depth-vectorized kernels apply: nz a multiple of 4, and one ring of a
// float32 array below 4 GiB (it is addressed with 32-bit byte offsets)
bool vec_applies(int nt, int nz);
// One instance of a batched two-pass step (float32 storage): its step
// arguments for both buffer parities (parity p reads fields[p] and writes
// fields[1 - p]), its tile shape and share of the batched grid, and its
// sources, receivers and step counter.  Tile shape: a workgroup's four
// wavefronts cover tz_waves x 256 depth cells of 4 / tz_waves theta rows.
struct BatchInst {
  StepArgs a[2];
  long tile0;               // first workgroup of this instance
  long tiles;               // workgroups of this instance
  int tz_waves;             // 1, 2 or 4
  int nseg;                 // depth segments per column, ceil(nz / (256 tz_waves))
  const Inject *inject;
  int ninj;
  const Receiver *rec;
  int nrec;
  int64_t cap;
  double *traces;
  int64_t *step;
};
// wpe: minimum wavefronts per SIMD of the batched kernels' registers, one of
// 0 (no constraint), 7, 8 (batch_occupancy_supported)
bool batch_occupancy_supported(int wpe);
hipError_t launch_velocity_batch(const BatchInst *dev, const long *tile0, int count, long tiles, int parity, int wpe,
                                 hipStream_t stream);
hipError_t launch_stress_batch(const BatchInst *dev, const long *tile0, int count, long tiles, int parity, int wpe,
                               hipStream_t stream);
hipError_t launch_inject_batch(const BatchInst *dev, int count, int phase, int parity, hipStream_t stream);
hipError_t launch_record_batch(const BatchInst *dev, int count, int max_rec, int parity, hipStream_t stream);
hipError_t launch_step_done_batch(const BatchInst *dev, int count, hipStream_t stream);

// Adjoint of the two-pass step (adjoint.hip).  fb: adjoints of the 9
// fields (updated in place, one step back per launch_adjoint_step); pr, pz:
// adjoints of the layer memory (same layout as psi_r, psi_z); T: nine
// scratch arrays of n values for the adjoints of the update terms.
struct AdjArgs {
  int nr, nt, nz, npr, npz, nzs;
  size_t rs;                // ring stride of the fields, their adjoints and the term arrays (StepArgs::rs)
  float dt, inv_dr, inv_dz, inv_dth;
  const float *inv_rc, *inv_rf;
  const float *rho, *lam, *mu;
  size_t m_ring;
  int m_row;
  float *fb[NF];
  float *pr[NPSI_R];
  float *pz[NPSI_Z];
  float *T[9];
  const float *tab_r, *tab_z;
  // dt times the effective moduli and buoyancies of the medium's cells (the
  // medium's layout): dt mu_rt, dt mu_rz, dt mu_tz, dt b_r, dt b_t, dt b_z
  float *C[6];
};
enum { C_RT, C_RZ, C_TZ, C_BR, C_BT, C_BZ };
// Parameter region: cells [i0, i1) x all theta x [k0, k1); the gradient
// reads the strain rates of the nodes [ea, eb) x all theta x [za, zb)
// (one ring and one depth more on the inner / upper side).
struct AdjRegion {
  int i0, i1, k0, k1;
  int ea, eb, za, zb;
};
hipError_t launch_adjoint_step(const AdjArgs &a, const Receiver *rec, int nrec, const float *w, const AdjRegion &g,
                               const float *Z, double *glam, double *gmu, hipStream_t stream);
hipError_t launch_adjoint_coefs(const AdjArgs &a, hipStream_t stream);
hipError_t launch_adjoint_capture(const AdjArgs &a, const AdjRegion &g, const float *vr, const float *vt,
                                  const float *vz, float *Z, hipStream_t stream);
hipError_t launch_set_step(int64_t *step, int64_t value, hipStream_t stream);
bool stream_mix_supported(int r, int w);
hipError_t launch_stream(const void *base, size_t bytes_per_array, int lane_bytes, bool nt, int r, int w,
                         hipStream_t stream);
hipError_t launch_velocity_vec(const StepArgs &a, int storage, hipStream_t stream);
hipError_t launch_stress_vec(const StepArgs &a, int storage, hipStream_t stream);

}  // namespace cw
