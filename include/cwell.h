/*
 * cwell.h -- C ABI of the MI355X cased-well wave solver.
 *
 * The library advances the first-order velocity-stress system of dynamic
 * elasticity in cylindrical coordinates (r, theta, z) -- Eq. (1) of
 * Cheverda et al., "Parallel Modeling of the Acoustic Signal Propagation in
 * a Cased Well" (arXiv 2302.13907), Sec. 2 -- with the explicit staggered-grid
 * finite-difference scheme of Sec. 3 (material attached to the cell centre),
 * a perfectly matched absorbing layer in r and z that does not split the
 * azimuthal terms (Sec. 1, Sec. 6), the four point-source kinds of Sec. 2
 * and receivers that record seismograms (Sec. 5).  The fluid is the same
 * medium with zero shear modulus (Sec. 2).
 *
 * Grid.  Every field lives on the same nr x ntheta x nz index space, stored
 * C order [i][j][k] with k (depth z) fastest, float32.  Staggering:
 *     s_rr, s_tt, s_zz at (r_i, th_j, z_k);      v_r  at (R_i, th_j, z_k)
 *     v_t  at (r_i, th_j+1/2, z_k);               v_z  at (r_i, th_j, z_k+1/2)
 *     s_rt at (R_i, th_j+1/2, z_k);               s_rz at (R_i, th_j, z_k+1/2)
 *     s_tz at (r_i, th_j+1/2, z_k+1/2)
 * with r_i = (i+1/2) dr, R_i = (i+1) dr, th_j = j * 2 pi / ntheta, z_k = k dz.
 * theta is periodic.  Values with i or k outside the grid read as zero: no
 * unknown sits on the axis r = 0, and this closure is exact when the
 * innermost ring is fluid.
 *
 * Time.  Leapfrog: velocities at t_{n+1/2}, stresses at t_n, zero initial
 * data (Eq. (2)).  Step n: velocity update from sigma^n, force sources with
 * w[n]; stress update from v^{n+1/2}, stress sources with w[n]; receivers
 * record sigma^{n+1} (and v^{n+1/2}) into column n of the trace buffer.
 *
 * Calling sequence.
 *   cw_create -> cw_set_material (or cw_set_material_rz) -> [cw_set_pml]
 *   -> cw_set_dt -> [cw_add_source]* -> [cw_add_receiver]*
 *   -> [cw_set_trace_capacity] -> cw_workspace_bytes -> cw_bind
 *   -> { cw_step | cw_get_* | cw_set_field | cw_energy | cw_reset }*
 *   -> cw_destroy.
 * Configuration calls after cw_bind return CW_ERR_STATE.
 *
 * Ownership.  Host inputs are copied; the caller keeps them.  Outputs go to
 * caller-owned host buffers.  Device memory is one caller-owned workspace
 * (for example a torch uint8 tensor) handed over by cw_bind; the library
 * never allocates or frees device memory and never frees the workspace.
 * All device work is enqueued on the HIP stream given to cw_bind.
 *
 * Errors.  Every call returns a cw_status; no exception crosses the ABI.
 * cw_last_error() returns a message for the last failing call of the
 * calling thread.  One cw_sim must not be used by two threads at once.
 */
#ifndef CWELL_H
#define CWELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cw_status;
#define CW_OK 0
#define CW_ERR_ARG (-1)        /* null pointer, bad enum, bad size */
#define CW_ERR_RANGE (-2)      /* index or step count out of range */
#define CW_ERR_MATERIAL (-3)   /* rho <= 0, mu < 0, lambda + 2 mu <= 0, or not finite */
#define CW_ERR_UNSTABLE (-4)   /* dt above the Courant limit */
#define CW_ERR_STATE (-5)      /* call out of order */
#define CW_ERR_NONFINITE (-6)  /* a NaN or Inf was found */
#define CW_ERR_HIP (-7)        /* a HIP runtime call failed */
#define CW_ERR_NOMEM (-8)      /* host allocation failed or workspace too small */

typedef struct cw_sim cw_sim;

typedef struct {
  int32_t nr, ntheta, nz; /* cells in r, theta, z; each >= 1 */
  double dr, dz;          /* cell sizes in metres, > 0; dtheta = 2 pi / ntheta */
} cw_grid;

/* field identifiers (cw_get_field, cw_set_field, CW_REC_FIELD) */
enum { CW_VR = 0, CW_VT, CW_VZ, CW_SRR, CW_STT, CW_SZZ, CW_SRT, CW_SRZ, CW_STZ, CW_NFIELD };

/* source kinds of Sec. 2: volumetric point source (s_rr, s_tt, s_zz),
   transverse (radial) point force (v_r), longitudinal point force (v_z),
   torsion source (s_rt, s_tz) */
enum { CW_SRC_VOLUME = 0, CW_SRC_FORCE_R, CW_SRC_FORCE_Z, CW_SRC_TORSION };

/* receiver kinds: pressure -(s_rr + s_tt + s_zz)/3, or one field */
enum { CW_REC_PRESSURE = 0, CW_REC_FIELD };

/* Create a simulation for grid *g.  *out receives the handle. */
cw_status cw_create(const cw_grid *g, cw_sim **out);

/* Medium at the cell centres (Sec. 3), host float64 arrays in C order
   [nr][ntheta][nz], SI units (kg/m^3, Pa).  mu = 0 marks fluid (Sec. 2).
   Staggered nodes use the arithmetic mean of the two adjacent densities
   and the harmonic mean of the four adjacent shear moduli (zero if any of
   them is zero); neighbour indices beyond the last cell in r or z are
   clamped, theta wraps.  Copied.  Errors: CW_ERR_MATERIAL. */
cw_status cw_set_material(cw_sim *s, const double *rho, const double *lam, const double *mu);

/* Same for an axisymmetric medium: arrays [nr][nz], repeated over theta. */
cw_status cw_set_material_rz(cw_sim *s, const double *rho, const double *lam, const double *mu);

/* Absorbing layer (Sec. 1, Sec. 6): npml_r cells at the outer radius,
   npml_z cells at each z end (0 and 0 switch it off: then the zero-value
   closure is lossless).  Convolutional form with a quadratic damping
   profile d(x) = d0 x^2, d0 = -3 Vp_max ln(rc) / (2 L), a constant
   frequency shift alpha (1/s), and the 1/r metric stretched by the
   integrated radial profile; theta is never stretched.  Requires
   npml_r < nr, 2 npml_z + 2 <= nz, 0 < rc < 1, alpha >= 0.  Call before
   cw_set_dt. */
cw_status cw_set_pml(cw_sim *s, int32_t npml_r, int32_t npml_z, double rc, double alpha);

/* Courant limit: min over cells of 1 / (Vp sqrt(1/dr^2 + 1/(r_i dth)^2 + 1/dz^2)). */
cw_status cw_cfl_dt(const cw_sim *s, double *dt_cfl);

/* Time step in seconds; CW_ERR_UNSTABLE if above the Courant limit. */
cw_status cw_set_dt(cw_sim *s, double dt);

/* Add a source of `kind` at cell (i, j, k); j = -1 spreads it over the whole
   ring i.  w[0..n) are wavelet samples (copied): w[n] enters at step n,
   with unit strength per unit volume -- the amount added to each target
   node is dt * w[n] / V (force sources: dt * b * w[n] / V, b the node's
   buoyancy), V the node volume r dr dth dz (ring: 2 pi r dr dz), r the
   node's own radius.  Stress sources are best sampled at t_{n+1/2}, force
   sources at t_n. */
cw_status cw_add_source(cw_sim *s, int32_t kind, int32_t i, int32_t j, int32_t k,
                        const double *w, int64_t n);

/* Add a receiver at (i, j, k), j = -1 averaging over ring i.  `field` is
   used by CW_REC_FIELD only.  *id receives its row in the trace buffer. */
cw_status cw_add_receiver(cw_sim *s, int32_t kind, int32_t field, int32_t i, int32_t j,
                          int32_t k, int32_t *id);

/* Steps the trace buffer can hold (float64 [nreceivers][capacity]).
   Default 0; cw_step fails with CW_ERR_RANGE if receivers exist and the
   total step count would exceed it. */
cw_status cw_set_trace_capacity(cw_sim *s, int64_t nsteps);

/* Device bytes the workspace must provide for the current configuration. */
cw_status cw_workspace_bytes(const cw_sim *s, uint64_t *bytes);

/* Bind a device workspace of at least cw_workspace_bytes bytes (256-byte
   aligned) and the HIP stream (hipStream_t, 0 = null stream) all work is
   enqueued on; upload the medium, tables and wavelets; zero the state.
   Asynchronous with respect to the host. */
cw_status cw_bind(cw_sim *s, void *workspace, uint64_t bytes, void *stream);

/* Enqueue nsteps time steps.  Asynchronous. */
cw_status cw_step(cw_sim *s, int64_t nsteps);

/* Wait for all work enqueued by this simulation.  With float16 storage,
   CW_ERR_NONFINITE once a field has overflowed (see cw_set_storage). */
cw_status cw_sync(cw_sim *s);

/* Copy the traces recorded so far into out (float64, [nreceivers][cap]
   row-major, cap >= steps done).  *nsteps_done receives the step count.
   Synchronous.  CW_ERR_NONFINITE (traces copied) as cw_sync. */
cw_status cw_get_traces(cw_sim *s, double *out, int64_t cap, int64_t *nsteps_done);

/* Copy one field of the current state to host float32 [nr][ntheta][nz]
   (16-bit storage is converted, scale applied).  Synchronous.
   CW_ERR_NONFINITE (field copied) as cw_sync. */
cw_status cw_get_field(cw_sim *s, int32_t field, float *host_out);

/* Overwrite one field of the current state (initial conditions, restart);
   with float16 storage the field's scale is set from the input's largest
   magnitude.  CW_ERR_NONFINITE for NaN or Inf input. */
cw_status cw_set_field(cw_sim *s, int32_t field, const float *host_in);

/* Energy E^{n+1/2} in float64 after the last step: kinetic energy of
   v^{n+1/2} plus the strain energy as the product of sigma^{n+1} and
   sigma^n (zero-shear terms dropped), each node weighted by its radius
   times dr dth dz.  Constant to rounding when the layer is off and no
   source fires.  Requires at least one step.  Synchronous. */
cw_status cw_energy(cw_sim *s, double *E);

/* cw_energy for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid allocation):
   the same kernels and the same result, with the nblocks partial sums and
   the result kept in a static scratch array of the library instead of the
   workspace.  The array holds 4096 partial sums plus the result (32 KiB,
   one copy per GPU, held until the process ends); nblocks outside
   [1, 4096] returns CW_ERR_RANGE.  nblocks = 1024 gives bitwise the result
   of cw_energy.  Allocates nothing.  Calls that overlap on one GPU (from
   two threads or two streams) share the array and race; calls on one
   stream are ordered.  Synchronous; same errors as cw_energy. */
cw_status cw_energy_noalloc(cw_sim *s, int32_t nblocks, double *E);

/* Zero the state, the layer's memory and the traces; step count to 0. */
cw_status cw_reset(cw_sim *s);

/* Number of time steps done. */
cw_status cw_steps_done(const cw_sim *s, int64_t *n);

/* Storage of the 9 fields: float32 (default), float16 or bfloat16.  All
   arithmetic is float32 whatever the storage; the medium, the layer memory
   and the traces keep their own precision (float32, float32, float64).
   float16 values carry a power-of-two scale per field: after every step
   the device sets the next scale from the largest magnitude just written,
   so that the stored maxima sit in [2^10, 2^11) (no host round trip).
   A field may therefore grow by up to 2^5 from one step to the next; a
   larger jump (a state far from equilibrium, such as unrelated random
   stresses and velocities set with cw_set_field) stores infinities, and
   cw_sync, cw_get_field and cw_get_traces then return CW_ERR_NONFINITE
   until cw_reset.  A source does not cause it by itself: the first write
   of a field a source injects into takes the scale of its largest
   injected value.
   bfloat16 has float32's exponent range and needs no scale.  Rounding is
   to nearest even.  Call before cw_bind. */
enum { CW_STORE_F32 = 0, CW_STORE_F16, CW_STORE_BF16 };
cw_status cw_set_storage(cw_sim *s, int32_t storage);

/* Rounding of the bfloat16 field stores of the step kernels:
   CW_ROUND_NEAREST (default, nearest even) or CW_ROUND_STOCHASTIC (the
   MI355X's stochastic-rounding conversion: a value is rounded up with the
   probability of the fraction of a unit that rounding down would drop, so
   the rounding error has mean zero and per-step increments smaller than
   half a unit of the stored value are kept on average).  The random bits
   are an integer hash of the cell, the field and the step number, so runs
   are bitwise reproducible, graph replay included.  Source injections
   still round to nearest.  Other storages ignore the mode.  Callable at any
   time; CW_ERR_ARG for an unknown mode. */
enum { CW_ROUND_NEAREST = 0, CW_ROUND_STOCHASTIC };
cw_status cw_set_rounding(cw_sim *s, int32_t mode);

/* Kernel path of cw_step.  All paths compute the same scheme; results
   agree to float32 rounding.
   CW_PATH_TWO_PASS: a velocity launch and a stress launch per step, small
   launches that add the force and the stress sources (in the order they
   were added) after them when there are any, then one launch that samples
   the receivers, sets the float16 scales and advances the step counter
   (with float32 storage and the one-cell velocity update, the next step's
   velocity launch does that work for the step before it, and only the last
   step of a cw_step call or of a captured graph has this launch);
   any number of sources and any storage; one workgroup
   per (ring, theta row) depth segment, 4 depth cells per thread when nz is
   a multiple of 4 and a ring of one float32 array is under 4 GiB, one cell
   per thread otherwise.
   CW_PATH_FUSED: one launch per step (and the receiver launch) that
   marches each theta x depth tile outward through the rings and reads the
   state, the medium and the layer memory once (float32 storage only, at most 12 source injections -- 3 per
   volume source, 2 per torsion source, 1 per force -- and nr <= 2048).
   CW_PATH_AUTO (default): the path measured fastest on MI355X: the
   two-pass step, with the velocity and the stress update one cell per
   thread for float32 storage (1 % and 3 % faster per launch at the
   production size than four cells per thread; the one-cell stress update
   adds the stress sources itself, and a step's receivers and step counter
   are taken by the next step's velocity launch, so that a step with only
   stress sources is two launches, plus one receiver launch after the last
   step of a cw_step call or of a captured graph); otherwise exactly
   CW_PATH_TWO_PASS.  Results of the two kernel forms agree to float32
   rounding. */
enum { CW_PATH_AUTO = 0, CW_PATH_TWO_PASS, CW_PATH_FUSED };
cw_status cw_set_path(cw_sim *s, int32_t path);

/* Graph replay of the two-pass step.  With steps > 0 (even, at most 4096),
   cw_step records the kernel launches of `steps` consecutive steps into a
   HIP graph the first time it needs them and then advances the simulation
   by replaying that graph, one launch per `steps` steps; step counts that
   are not a whole number of graphs, and a start on an odd step, are done
   with ordinary launches.  Results are bitwise those of ordinary launches
   (the source and receiver kernels read the step number from device
   memory).  0 (default) switches it off.  Kernel timing (cw_profile) and
   CW_PATH_FUSED always use ordinary launches.  The graph belongs to the
   simulation and stays valid across cw_reset; changing the path drops it.
   Callable at any time; CW_ERR_RANGE for an odd or too large count. */
cw_status cw_set_graph(cw_sim *s, int32_t steps);

/* Kernel timing.  With enable = 1, cw_step brackets every launch of the
   step kernels with HIP events on the simulation's stream (a few
   microseconds of overhead per launch); enable = 0 stops recording and
   clears the records.  cw_profile_read waits for the recorded work and
   returns, for kernel `kernel` (CW_K_*), the summed device time in
   milliseconds and the number of launches recorded.  CW_K_RECORD is the
   receiver launch (receivers, scales, step counter; with the default
   float32 path once per call, the velocity launches time the rest); CW_K_INJECT the
   source launches. */
enum { CW_K_VELOCITY = 0, CW_K_STRESS, CW_K_FUSED, CW_K_INJECT, CW_K_RECORD, CW_K_COUNT };
cw_status cw_profile(cw_sim *s, int32_t enable);
cw_status cw_profile_read(cw_sim *s, int32_t kernel, double *total_ms, int64_t *launches);

/* Host helper: Ricker pulse of Sec. 2 with the printed delay 2/f0,
   out[m] = f(t[m]). */
cw_status cw_ricker(double f0, const double *t, int64_t n, double *out);

/* Adjoint gradient.  The loss is the sum, over steps n in [n0, n1) and
   pressure receivers m, of p_m(t_{n+1})^2.  Its parameters are the moduli
   of a region: rings [i0, i1), every theta, depth rows [k0, k0 + nbins *
   bin_rows) in bins of bin_rows rows; bin b's parameters shift the shear
   modulus mu and the bulk modulus K = lambda + 2 mu / 3 of all its cells.
   cw_gradient runs nsteps forward steps from rest (sources included),
   keeping a checkpoint of the whole state every checkpoint_every steps,
   then the discrete adjoint of the step backwards: segment by segment it
   recomputes the forward steps from the segment's checkpoint (storing the
   region's strain rates; those of the last segment are stored by the
   forward run itself, so checkpoint_every >= nsteps recomputes nothing, at
   the price of a strain-rate buffer for all nsteps steps) and then takes
   their adjoint steps, adding each
   step's contribution to the gradient (Eq. (1): the stress update is linear
   in lambda, mu and, through the harmonic means of the shear nodes, in the
   cells' mu).  Outputs: *loss, grad_mu[nbins] = dL/dmu_b (K fixed),
   grad_K[nbins] = dL/dK_b (mu fixed), all float64; the state afterwards is
   unspecified (call cw_reset before stepping again).  Float32 storage and
   the two-pass kernels only.

   cw_set_adjoint: before cw_bind, after cw_set_pml (its buffers -- the
   adjoint state, one checkpoint per segment but the last, one segment of
   strain rates -- become part of the workspace; the trace capacity is
   raised to nsteps).  The region must lie clear of the absorbing layer and
   the grid's edges: 1 <= i0 < i1 <= nr - max(npml_r, 2), max(npml_z + 1, 1)
   <= k0, k0 + nbins * bin_rows <= nz - 1 - max(npml_z, 1); CW_ERR_RANGE
   otherwise.  nsteps = 0 switches the adjoint off. */
cw_status cw_set_adjoint(cw_sim *s, int64_t nsteps, int32_t checkpoint_every, int32_t i0, int32_t i1, int32_t k0,
                         int32_t nbins, int32_t bin_rows);
/* Sets the region's moduli to those given by cw_set_material plus the
   per-bin shifts dmu[nbins], dK[nbins] (Pa), on the host copy and, once
   bound, on the device.  CW_ERR_MATERIAL if a shifted cell would have
   mu < 0 or lambda + 2 mu <= 0, CW_ERR_UNSTABLE if dt would exceed the
   Courant limit of a shifted cell; nothing changes then.  The absorbing
   layer's profile keeps the largest P speed of the original medium. */
cw_status cw_set_region_moduli(cw_sim *s, const double *dmu, const double *dK);
cw_status cw_gradient(cw_sim *s, int64_t n0, int64_t n1, double *loss, double *grad_mu, double *grad_K);

/* Batches: many simulations (of any sizes) advanced together, each step
   one velocity launch and one stress launch over the tiles of all of them
   (plus batched source, receiver and step-counter launches), so small and
   uneven instances share the device.  Every simulation must be bound on
   one device and one stream, use float32 storage, have nz a multiple of 4
   and rings of one array under 4 GiB (CW_ERR_RANGE otherwise), and have
   done steps of one parity; each keeps its own state, sources,
   receivers and traces (cw_get_traces, cw_get_field etc. work as usual) and
   gives bitwise the results of stepping it alone with CW_PATH_TWO_PASS.
   The batch descriptor lives in a small caller-owned device workspace
   (cw_batch_workspace_bytes, 256-byte aligned).  Tile shape per instance
   (cw_batch_set_tile, before cw_batch_bind): a workgroup covers tz_waves x
   256 depth cells of 4 / tz_waves theta rows, tz_waves in {1, 2, 4}
   (default 4); shallow or ragged columns waste fewer lanes with shorter
   tiles.  cw_batch_set_occupancy: the minimum wavefronts per SIMD the
   batched kernels' registers are sized for, 0 (the compiler's choice,
   default: 79 registers, 6 waves), 7 or 8 (fewer registers, some values
   spilled; CW_ERR_RANGE otherwise); one compiled variant each, same
   results; callable at any time.  The tile shapes and the occupancy
   are what the package's autotuner searches.  cw_batch_set_graph: as
   cw_set_graph, for the batch.  The batch must be destroyed before its
   simulations. */
typedef struct cw_batch cw_batch;
cw_status cw_batch_create(cw_sim *const *sims, int32_t count, cw_batch **out);
cw_status cw_batch_set_tile(cw_batch *b, int32_t index, int32_t tz_waves);
cw_status cw_batch_set_occupancy(cw_batch *b, int32_t waves_per_simd);
cw_status cw_batch_workspace_bytes(const cw_batch *b, uint64_t *bytes);
cw_status cw_batch_bind(cw_batch *b, void *workspace, uint64_t bytes);
cw_status cw_batch_set_graph(cw_batch *b, int32_t steps);
cw_status cw_batch_step(cw_batch *b, int64_t nsteps);
void cw_batch_destroy(cw_batch *b);

/* Azimuthally refined grid (Sec. 3).  The rings are split into zones;
   zone q holds rings [first_ring[q], first_ring[q + 1]) (the last zone up
   to nr) with ntheta[q] azimuthal cells, ntheta doubling from one zone to
   the next (the paper halves the azimuthal step each time the radius
   doubles, which keeps r dtheta bounded and lifts the axis-limited Courant
   step).  Within a zone the scheme is the uniform one.  Across the circle
   between two zones each side's stencils read the other side's edge ring
   on their own azimuthal grid: coarse -> fine by trigonometric
   interpolation (the Fourier transform of the coarse ring, padded with
   zeros, transformed back; the coarse Nyquist mode split evenly between
   +n/2 and -n/2; half-integer nodes shifted in phase), fine -> coarse by
   the transpose of that map times dtheta_fine / dtheta_coarse (which keeps
   the scheme's energy conserved).
   cw_refined_create: grid->ntheta must equal the outermost zone's ntheta
   (at most 229: the interpolation keeps a matrix and a tile in LDS), nz a
   multiple of 4 with ntheta * nz * 4 bytes under 4 GiB, first_ring[0] = 0,
   first rings
   increasing and below nr; CW_ERR_RANGE otherwise.  The medium must not
   vary along theta (cw_refined_set_material_rz, [nr][nz] float64).  The
   radial absorbing layer must lie inside the outermost zone.  Sources and
   receivers take a global ring i and an azimuthal index j of that ring's
   own grid (-1: the whole ring).  Fields are exchanged as the rings
   concatenated, ring 0 first, ring i holding ntheta_i x nz float32 values
   (cw_refined_cells of them).  Traces are [receiver][cap] as cw_get_traces.
   Float32 storage; the zones are stepped as one batch (one velocity and one
   stress launch per step) with one interpolation launch before each of
   them.  One workspace, one stream, as cw_bind. */
typedef struct cw_refined cw_refined;
cw_status cw_refined_create(const cw_grid *g, int32_t nzones, const int32_t *first_ring, const int32_t *ntheta,
                            cw_refined **out);
cw_status cw_refined_cells(const cw_refined *r, uint64_t *cells);
cw_status cw_refined_set_material_rz(cw_refined *r, const double *rho, const double *lam, const double *mu);
cw_status cw_refined_set_pml(cw_refined *r, int32_t npml_r, int32_t npml_z, double rc, double alpha);
cw_status cw_refined_cfl_dt(const cw_refined *r, double *dt_cfl);
cw_status cw_refined_set_dt(cw_refined *r, double dt);
cw_status cw_refined_add_source(cw_refined *r, int32_t kind, int32_t i, int32_t j, int32_t k, const double *w,
                                int64_t n);
cw_status cw_refined_add_receiver(cw_refined *r, int32_t kind, int32_t field, int32_t i, int32_t j, int32_t k,
                                  int32_t *id);
cw_status cw_refined_set_trace_capacity(cw_refined *r, int64_t nsteps);
cw_status cw_refined_workspace_bytes(const cw_refined *r, uint64_t *bytes);
cw_status cw_refined_bind(cw_refined *r, void *workspace, uint64_t bytes, void *stream);
cw_status cw_refined_step(cw_refined *r, int64_t nsteps);
cw_status cw_refined_get_field(cw_refined *r, int32_t field, float *host_out);
cw_status cw_refined_set_field(cw_refined *r, int32_t field, const float *host_in);
cw_status cw_refined_get_traces(cw_refined *r, double *out, int64_t cap, int64_t *nsteps_done);
cw_status cw_refined_energy(cw_refined *r, double *E);
cw_status cw_refined_reset(cw_refined *r);
void cw_refined_destroy(cw_refined *r);

/* Bandwidth reference (measurement only, not part of the scheme): stream
   nread + nwrite arrays of bytes_per_array bytes each, laid out back to
   back in the caller's device buffer `dev` (16-byte aligned, at least
   (nread + nwrite) * bytes_per_array bytes; its contents are overwritten):
   every group of the write arrays receives the sum of the same group of
   the read arrays, one group per thread, a group being lane_bytes = 16
   (four floats) or 4 (one float) bytes; CW_ERR_ARG for other widths.
   lane_bytes | CW_PROBE_NONTEMPORAL makes every load and store
   non-temporal (the lines are not kept): the rate of a stream none of
   whose data is read again.
   Runs 2 untimed passes and `reps` timed ones
   on `stream` (a hipStream_t, NULL for the default stream), waits, and
   returns the average milliseconds per pass.  Supported (nread, nwrite):
   (1, 1), (9, 3), (10, 3), (9, 6), (11, 6), (9, 9), (12, 9) -- the stream
   mixes of the step kernels; others give CW_ERR_RANGE. */
#define CW_PROBE_NONTEMPORAL 0x100
cw_status cw_stream_probe(void *dev, uint64_t bytes_per_array, int32_t nread, int32_t nwrite, int32_t lane_bytes,
                          int32_t reps, void *stream, double *ms_per_pass);

void cw_destroy(cw_sim *s);
const char *cw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CWELL_H */
