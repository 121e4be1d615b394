// Host side of libcwell: configuration, coefficient tables (float64 on the
// host, stored float32), workspace layout, and the time loop.
#include "cwell_internal.hpp"
#include "../../include/cwell.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace cw;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kEnergyBlocks = 1024;
constexpr int kMaxGraphSteps = 4096;
#ifndef CW_AUTO_FUSED
#define CW_AUTO_FUSED 0
#endif
constexpr bool kAutoFused = CW_AUTO_FUSED;    // what CW_PATH_AUTO picks when the fused step applies
#ifndef CW_USE_VEC
#define CW_USE_VEC 1
#endif
constexpr bool kUseVec = CW_USE_VEC;          // two-pass kernels: 4 depth cells per thread when nz % 4 == 0

thread_local std::string g_err;

cw_status fail(cw_status st, const char *fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return fail(CW_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

struct SourceSpec {
  int kind, i, j, k;
  std::vector<double> w;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// padding after each ring of a field array (see cw_sim::rs)
constexpr size_t kRingPadBytes = 4096, kRingPadSmallBytes = 1024;

struct cw_sim {
  // grid
  int nr = 0, nt = 0, nz = 0;
  double dr = 0, dz = 0, dth = 0;
  size_t n = 0;
  // a zone of an azimuthally refined grid (cw_refined_*): global index of
  // ring 0, ghost rings around the field arrays, medium rings stored beyond
  // the last one (the next zone's first), and the speed that sets the
  // absorbing profile (that of the whole grid; 0: this medium's own)
  int ring0 = 0;
  bool ghost_in = false, ghost_out = false;
  int med_extra = 0;
  double vp_ref = 0;
  // rs: values from one ring of a field array to the next.  A ring may be
  // followed by padding, which moves the radial neighbours a cell reads off
  // a power-of-two distance; how much is what measured fastest (same box,
  // alternated, ms per step unless stated; padding 0 / 1 / 2 / 4 / 6 KB):
  //   float32, 256 x 128 x 8192 (4 MB rings): 5.783 / 5.676 / 5.576 / 5.509 / 5.627
  //   float32, adjoint gradient at 128 x 64 x 2048 (512 KB rings), s:
  //     2.072 / 2.028 / 2.028 / 2.134 / 2.037
  //   bfloat16, 256 x 128 x 8192: 3.868 / 3.804 / 3.778 / 3.772 / 3.771
  //   float16, 256 x 128 x 8192: 3.940 / 4.071 / 3.969 / 3.974 / 3.960
  // With 1 KB on float32 rings from 128 KB to 4 MB the 48-instance batch
  // of 128 x 64 x Nz was 0.5 % slower and the 48 x 32 x 192 step unchanged.
  // So: 4 KB for float32 rings of 4 MB or more and for bfloat16, 1 KB for
  // float32 rings from 128 KB, none for float16 or smaller rings.
  size_t rs() const
  {
    const size_t ring = (size_t)nt * nz, eb = storage == ST_F32 ? 4 : 2, bytes = ring * eb;
    if (storage == ST_F16) return ring;
    if (storage == ST_BF16 || bytes >= ((size_t)4 << 20)) return ring + kRingPadBytes / eb;
    return ring + (bytes >= ((size_t)128 << 10) ? kRingPadSmallBytes / eb : 0);
  }
  size_t n_alloc() const { return (size_t)(nr + ghost_in + ghost_out) * rs(); }
  // medium (float32 copies, uploaded at bind) and what the setup derives from it
  std::vector<float> rho, lam, mu;
  bool have_material = false;
  double vp_max = 0, dt_cfl = 0;
  // layer
  int npr = 0, npz = 0;
  double rc = 1e-3, alpha = 0;
  // time step and derived tables
  double dt = 0;
  std::vector<float> tab_r, tab_z, inv_rc, inv_rf;
  // sources / receivers
  std::vector<SourceSpec> sources;
  std::vector<Receiver> receivers;
  int64_t trace_cap = 0;
  // device state
  bool bound = false;
  int device = 0;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  uint64_t ws_bytes = 0;
  float *fields[2][NF] = {};
  float *d_rho = nullptr, *d_lam = nullptr, *d_mu = nullptr;
  bool med_rz = false;          // medium identical along theta: stored [nr][nz]
  size_t nm = 0;                // values per medium array (n, or nr nz)
  float *d_inv_rc = nullptr, *d_inv_rf = nullptr, *d_tab_r = nullptr, *d_tab_z = nullptr;
  float *psi_r[2][NPSI_R] = {};  // two copies: the fused step reads one, writes the other
  float *psi_z[2][NPSI_Z] = {};
  int psi_cur = 0;
  int path = CW_PATH_AUTO;
  int storage = ST_F32;
  int rounding = CW_ROUND_NEAREST;   // rounding of the 16-bit field stores (cw_set_rounding)
  float *d_scl = nullptr;       // [3][NF]: scale of buffer 0, buffer 1, next write
  float scl_init[3 * NF] = {};  // host copy of the scales zero_state starts from
  unsigned *d_maxabs = nullptr; // [NF][kMaxSlots], then the float16 overflow word (kOverflowWord)
  Inject *d_inject = nullptr;
  int ninject = 0;
  std::vector<Inject> inject_host;
  std::vector<std::vector<float>> inject_amp;   // host copy of each injection's amplitudes
  Receiver *d_rec = nullptr;
  double *d_traces = nullptr;
  double *d_energy = nullptr;   // kEnergyBlocks partials + 1 result
  int64_t *d_step = nullptr;    // steps done, as the injection and receiver kernels read it
  bool force_src = false;       // a source injects into a velocity (phase 0)
  bool stress_src = false;      // a source injects into a stress (phase 1)
  int inj_i0 = 0, inj_i1 = -1;  // rings the sources touch
  unsigned *d_done = nullptr;   // workgroups of the step's last launch that have finished (zero between steps)
  // adjoint gradient (cw_set_adjoint): configuration and buffers in the workspace
  bool adj = false;
  int64_t adj_steps = 0;
  int adj_every = 0;
  int adj_i0 = 0, adj_i1 = 0, adj_k0 = 0, adj_nb = 0, adj_br = 0;
  float *adj_fb[NF] = {};
  float *adj_pr[NPSI_R] = {};
  float *adj_pz[NPSI_Z] = {};
  float *adj_T[9] = {};
  float *adj_C[6] = {};         // dt-scaled effective moduli and buoyancies (the medium's layout)
  float *adj_ckpt = nullptr;    // checkpoints [ncp - 1][9 n + 12 slab_r + 6 slab_z] (none of the last segment)
  float *adj_Z = nullptr;       // strain rates of one segment [every][6][region nodes]
  double *adj_glam = nullptr, *adj_gmu = nullptr;   // per region cell
  float *adj_w = nullptr;       // receiver adjoint weights [steps][receivers]
  std::vector<double> adj_mu0, adj_K0;   // the region's moduli as set by cw_set_material
  // graph replay of the two-pass step (cw_set_graph)
  int graph_steps = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;   // captures run here: the caller's stream may be the null stream
  void drop_graph()
  {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  int cur = 0;                  // fields[cur] holds the current state
  int64_t nstep = 0;
  // kernel timing: (kernel id, start, stop) per recorded launch
  bool profiling = false;
  struct Rec { int kernel; hipEvent_t start, stop; };
  std::vector<Rec> prof;
  std::vector<hipEvent_t> event_pool;
  ~cw_sim()
  {
    drop_graph();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (auto &r : prof) { event_pool.push_back(r.start); event_pool.push_back(r.stop); }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
  }
};

namespace {

int nzs_of(const cw_sim *s) { return s->npz > 0 ? 2 * s->npz + 1 : 0; }

size_t field_bytes(const cw_sim *s) { return s->storage == ST_F32 ? 4 : 2; }

// Number of float32 amplitude samples over all injections.
size_t amp_floats(const cw_sim *s)
{
  size_t t = 0;
  for (const auto &src : s->sources) {
    int targets = (src.kind == CW_SRC_VOLUME) ? 3 : (src.kind == CW_SRC_TORSION ? 2 : 1);
    t += (size_t)targets * src.w.size();
  }
  return t;
}

int inject_count(const cw_sim *s)
{
  int t = 0;
  for (const auto &src : s->sources)
    t += (src.kind == CW_SRC_VOLUME) ? 3 : (src.kind == CW_SRC_TORSION ? 2 : 1);
  return t;
}

struct Layout {
  size_t fields, material, metric, tabr, tabz, psir, psiz, inject, amp, rec, traces, energy, scales, step, adj,
      total;
};

// the adjoint's region and its sizes
AdjRegion adj_region(const cw_sim *s)
{
  AdjRegion g{};
  g.i0 = s->adj_i0; g.i1 = s->adj_i1; g.k0 = s->adj_k0; g.k1 = s->adj_k0 + s->adj_nb * s->adj_br;
  g.ea = g.i0 - 1; g.eb = g.i1; g.za = g.k0 - 1; g.zb = g.k1;
  return g;
}
size_t adj_region_nodes(const cw_sim *s)
{
  const AdjRegion g = adj_region(s);
  return (size_t)(g.eb - g.ea) * s->nt * (g.zb - g.za);
}
size_t adj_region_cells(const cw_sim *s)
{
  const AdjRegion g = adj_region(s);
  return (size_t)(g.i1 - g.i0) * s->nt * (g.k1 - g.k0);
}
size_t adj_state_floats(const cw_sim *s)
{
  return NF * s->n_alloc() + (size_t)NPSI_R * s->npr * s->nt * s->nz + (size_t)NPSI_Z * s->nr * s->nt * nzs_of(s);
}
size_t adj_bytes(const cw_sim *s)
{
  if (!s->adj) return 0;
  const size_t ncp = (size_t)((s->adj_steps + s->adj_every - 1) / s->adj_every);
  size_t f = adj_state_floats(s)               // adjoint fields and layer memory
             + 9 * s->n_alloc()                // term adjoints
             + 6 * s->nm                       // effective coefficients
             + 2 * 64                          // alignment of the two blocks above
             + (ncp - 1) * adj_state_floats(s) // checkpoints (the last segment needs none)
             + (size_t)s->adj_every * 6 * adj_region_nodes(s)
             + (size_t)s->adj_steps * s->receivers.size();
  return f * sizeof(float) + 2 * adj_region_cells(s) * sizeof(double) + 1024;
}

Layout layout(const cw_sim *s)
{
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.fields = take(2 * NF * s->n_alloc() * field_bytes(s));
  L.material = take(3 * s->nm * sizeof(float));
  L.metric = take(2 * (size_t)s->nr * sizeof(float));
  L.tabr = take(NTAB_R * (size_t)s->nr * sizeof(float));
  L.tabz = take(NTAB_Z * (size_t)s->nz * sizeof(float));
  L.psir = take(2 * (size_t)NPSI_R * s->npr * s->nt * s->nz * sizeof(float));
  L.psiz = take(2 * (size_t)NPSI_Z * s->nr * s->nt * nzs_of(s) * sizeof(float));
  L.inject = take((size_t)inject_count(s) * sizeof(Inject));
  L.amp = take(amp_floats(s) * sizeof(float));
  L.rec = take(s->receivers.size() * sizeof(Receiver));
  L.traces = take(s->receivers.size() * (size_t)s->trace_cap * sizeof(double));
  L.energy = take((kEnergyBlocks + 1) * sizeof(double));
  L.scales = take(3 * NF * sizeof(float) + (kOverflowWord + 1) * sizeof(unsigned));
  L.step = take(2 * sizeof(int64_t));   // the step counter, then the finish counter of the step's last launch
  L.adj = take(adj_bytes(s));
  L.total = off;
  return L;
}

// Courant limit over the cell centres with the azimuthal width r_i dth.
double courant(const cw_sim *s, const double *rho, const double *lam, const double *mu,
               bool rz_only)
{
  double best = INFINITY;
  const size_t per_ring = rz_only ? (size_t)s->nz : (size_t)s->nt * s->nz;
  for (int i = 0; i < s->nr; i++) {
    const double ra = (s->ring0 + i + 0.5) * s->dr * s->dth;
    const double g = std::sqrt(1.0 / (s->dr * s->dr) + 1.0 / (ra * ra) + 1.0 / (s->dz * s->dz));
    double vmax = 0;
    for (size_t c = 0; c < per_ring; c++) {
      const size_t p = (size_t)i * per_ring + c;
      vmax = std::max(vmax, std::sqrt((lam[p] + 2.0 * mu[p]) / rho[p]));
    }
    best = std::min(best, 1.0 / (vmax * g));
  }
  return best;
}

cw_status check_medium(size_t n, const double *rho, const double *lam, const double *mu)
{
  for (size_t p = 0; p < n; p++) {
    const double r = rho[p], l = lam[p], m = mu[p];
    if (!std::isfinite(r) || !std::isfinite(l) || !std::isfinite(m) || !(r > 0) || !(m >= 0) ||
        !(l + 2 * m > 0))
      return fail(CW_ERR_MATERIAL, "invalid medium at flat index %zu: rho=%g lambda=%g mu=%g", p, r, l, m);
  }
  return CW_OK;
}

// Damping coefficients of the recursive convolution for profile value d.
void conv_coef(double d, double alpha, double dt, float *a, float *b)
{
  const double bb = std::exp(-(d + alpha) * dt);
  *b = (float)bb;
  *a = d > 0 ? (float)(d * (bb - 1.0) / (d + alpha)) : 0.0f;
}

void build_tables(cw_sim *s)
{
  s->inv_rc.resize(s->nr);
  s->inv_rf.resize(s->nr);
  for (int i = 0; i < s->nr; i++) {
    s->inv_rc[i] = (float)(1.0 / ((s->ring0 + i + 0.5) * s->dr));
    s->inv_rf[i] = (float)(1.0 / ((s->ring0 + i + 1.0) * s->dr));
  }
  s->tab_r.assign(NTAB_R * (size_t)s->nr, 0.0f);
  s->tab_z.assign(NTAB_Z * (size_t)s->nz, 0.0f);
  const double Lr = s->npr * s->dr, Lz = s->npz * s->dz;
  const double vp = s->vp_ref > 0 ? s->vp_ref : s->vp_max;
  const double d0r = s->npr > 0 ? -3.0 * vp * std::log(s->rc) / (2.0 * Lr) : 0.0;
  const double d0z = s->npz > 0 ? -3.0 * vp * std::log(s->rc) / (2.0 * Lz) : 0.0;
  const double r0 = (s->ring0 + s->nr - s->npr) * s->dr;   // inner edge of the radial layer
  for (int i = 0; i < s->nr; i++) {
    for (int face = 0; face < 2; face++) {
      const double r = (s->ring0 + i + (face ? 1.0 : 0.5)) * s->dr;
      const double x = (s->npr > 0 && r > r0) ? (r - r0) / Lr : 0.0;
      const double d = d0r * x * x;                       // radial profile
      const double dint = s->npr > 0 ? d0r * Lr * x * x * x / (3.0 * r) : 0.0;  // (1/r) * integral of d
      float *T = s->tab_r.data();
      conv_coef(d, s->alpha, s->dt, &T[(face ? AR_F : AR_C) * s->nr + i], &T[(face ? BR_F : BR_C) * s->nr + i]);
      conv_coef(dint, s->alpha, s->dt, &T[(face ? AT_F : AT_C) * s->nr + i], &T[(face ? BT_F : BT_C) * s->nr + i]);
    }
  }
  for (int k = 0; k < s->nz; k++) {
    for (int half = 0; half < 2; half++) {
      const double z = (k + (half ? 0.5 : 0.0)) * s->dz;
      double x = 0.0;
      if (s->npz > 0) {
        x = std::max((s->npz * s->dz - z) / Lz, (z - (s->nz - 1 - s->npz) * s->dz) / Lz);
        x = std::max(x, 0.0);
      }
      float *T = s->tab_z.data();
      conv_coef(d0z * x * x, s->alpha, s->dt, &T[(half ? AZ_H : AZ_C) * s->nz + k], &T[(half ? BZ_H : BZ_C) * s->nz + k]);
    }
  }
}

bool configurable(cw_sim *s, cw_status *st)
{
  if (!s) { *st = fail(CW_ERR_ARG, "null simulation"); return false; }
  if (s->bound) { *st = fail(CW_ERR_STATE, "configuration after cw_bind"); return false; }
  return true;
}

StepArgs step_args(const cw_sim *s, int in, int out)
{
  StepArgs a{};
  a.nr = s->nr; a.nt = s->nt; a.nz = s->nz;
  a.ring0 = s->ring0;
  a.m_last = s->nr - 1 + s->med_extra;
  a.ghost_in = s->ghost_in;
  a.ghost_out = s->ghost_out;
  a.npr = s->npr; a.npz = s->npz; a.nzs = nzs_of(s);
  a.dt = (float)s->dt;
  a.inv_dr = (float)(1.0 / s->dr);
  a.inv_dz = (float)(1.0 / s->dz);
  a.inv_dth = (float)(1.0 / s->dth);
  a.inv_rc = s->d_inv_rc; a.inv_rf = s->d_inv_rf;
  a.rho = s->d_rho; a.lam = s->d_lam; a.mu = s->d_mu;
  a.m_ring = s->med_rz ? (size_t)s->nz : (size_t)s->nt * s->nz;
  a.m_row = s->med_rz ? 0 : s->nz;
  for (int q = 0; q < NF; q++) { a.in[q] = s->fields[in][q]; a.out[q] = s->fields[out][q]; }
  for (int q = 0; q < NPSI_R; q++) a.psi_r[q] = s->psi_r[s->psi_cur][q];
  for (int q = 0; q < NPSI_Z; q++) a.psi_z[q] = s->psi_z[s->psi_cur][q];
  a.tab_r = s->d_tab_r; a.tab_z = s->d_tab_z;
  a.scl_in = s->d_scl + in * NF;
  a.scl_out = s->d_scl + 2 * NF;
  a.maxabs = s->d_maxabs;
  a.step = s->d_step;
  a.sr = s->rounding == CW_ROUND_STOCHASTIC && s->storage == ST_BF16;
  a.rs = s->rs();
  return a;
}

hipError_t take_event(cw_sim *s, hipEvent_t *e)
{
  if (!s->event_pool.empty()) {
    *e = s->event_pool.back();
    s->event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Launch `fn` on the stream, bracketed by events when profiling.
template <class F>
cw_status timed(cw_sim *s, int kernel, F &&fn)
{
  if (!s->profiling) {
    HIPCHK(fn());
    return CW_OK;
  }
  cw_sim::Rec r{kernel, nullptr, nullptr};
  HIPCHK(take_event(s, &r.start));
  HIPCHK(take_event(s, &r.stop));
  HIPCHK(hipEventRecord(r.start, s->stream));
  HIPCHK(fn());
  HIPCHK(hipEventRecord(r.stop, s->stream));
  s->prof.push_back(r);
  return CW_OK;
}

cw_status zero_state(cw_sim *s)
{
  const Layout L = layout(s);
  HIPCHK(hipMemsetAsync(s->ws + L.fields, 0, 2 * NF * s->n_alloc() * field_bytes(s), s->stream));
  // Every buffer scale 1, no maxima yet.  The first write of a field a source
  // injects into takes the scale its largest injected value needs (the rule
  // of the per-step rescale), so a large or abrupt pulse cannot overflow
  // float16 before the scale has adapted; other fields start at 1 and adapt
  // from the values they first receive.  (Kept in the simulation: the copy
  // source must outlive the asynchronous copy.)
  float peak[NF] = {};
  for (size_t e = 0; e < s->inject_host.size(); e++)
    for (float a : s->inject_amp[e])
      peak[s->inject_host[e].field] = std::max(peak[s->inject_host[e].field], std::fabs(s->inject_host[e].scale * a));
  for (int q = 0; q < 3 * NF; q++) s->scl_init[q] = 1.0f;
  for (int q = 0; q < NF; q++)
    if (peak[q] > 0.0f) {
      int ex;
      std::frexp(peak[q], &ex);
      s->scl_init[2 * NF + q] = std::ldexp(1.0f, ex - kF16TargetExp);
    }
  HIPCHK(hipMemcpyAsync(s->d_scl, s->scl_init, sizeof s->scl_init, hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemsetAsync(s->d_maxabs, 0, (kOverflowWord + 1) * sizeof(unsigned), s->stream));
  const size_t psir = 2 * (size_t)NPSI_R * s->npr * s->nt * s->nz * sizeof(float);
  const size_t psiz = 2 * (size_t)NPSI_Z * s->nr * s->nt * nzs_of(s) * sizeof(float);
  if (psir) HIPCHK(hipMemsetAsync(s->ws + L.psir, 0, psir, s->stream));
  if (psiz) HIPCHK(hipMemsetAsync(s->ws + L.psiz, 0, psiz, s->stream));
  const size_t tb = s->receivers.size() * (size_t)s->trace_cap * sizeof(double);
  if (tb) HIPCHK(hipMemsetAsync(s->ws + L.traces, 0, tb, s->stream));
  HIPCHK(hipMemsetAsync(s->d_step, 0, 2 * sizeof(int64_t), s->stream));
  s->cur = 0;
  s->psi_cur = 0;
  s->nstep = 0;
  return CW_OK;
}

}  // namespace

extern "C" {

const char *cw_last_error(void) { return g_err.c_str(); }

cw_status cw_create(const cw_grid *g, cw_sim **out)
{
  if (!g || !out) return fail(CW_ERR_ARG, "null argument");
  if (g->nr < 1 || g->ntheta < 1 || g->nz < 1)
    return fail(CW_ERR_ARG, "grid sizes must be >= 1 (got %d %d %d)", g->nr, g->ntheta, g->nz);
  if (!(g->dr > 0) || !(g->dz > 0) || !std::isfinite(g->dr) || !std::isfinite(g->dz))
    return fail(CW_ERR_ARG, "cell sizes must be finite and > 0");
  cw_sim *s = new (std::nothrow) cw_sim();
  if (!s) return fail(CW_ERR_NOMEM, "out of host memory");
  s->nr = g->nr; s->nt = g->ntheta; s->nz = g->nz;
  s->dr = g->dr; s->dz = g->dz; s->dth = 2.0 * kPi / g->ntheta;
  s->n = (size_t)s->nr * s->nt * s->nz;
  *out = s;
  return CW_OK;
}

void cw_destroy(cw_sim *s) { delete s; }

// index of cell (i, j, k) in the stored medium arrays
static size_t mat_index(const cw_sim *s, int i, int j, int k)
{
  return s->med_rz ? (size_t)i * s->nz + k : ((size_t)i * s->nt + j) * s->nz + k;
}

static cw_status set_medium(cw_sim *s, const double *rho, const double *lam, const double *mu, bool rz)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (!rho || !lam || !mu) return fail(CW_ERR_ARG, "null medium array");
  if (s->med_extra && !rz) return fail(CW_ERR_ARG, "a zone takes an axisymmetric medium");
  const int mrings = s->nr + s->med_extra;
  const size_t nin = rz ? (size_t)mrings * s->nz : s->n;
  if ((st = check_medium(nin, rho, lam, mu)) != CW_OK) return st;
  // a 3-D medium identical along theta (bitwise) is stored like an axisymmetric one:
  // the kernels then read [nr][nz] tables, which stay in cache, instead of full arrays
  bool axisym = rz;
  if (!rz) {
    axisym = true;
    for (int i = 0; i < s->nr && axisym; i++)
      for (int j = 1; j < s->nt && axisym; j++) {
        const size_t a = (size_t)i * s->nt * s->nz, b = ((size_t)i * s->nt + j) * s->nz;
        for (int k = 0; k < s->nz; k++)
          if (rho[a + k] != rho[b + k] || lam[a + k] != lam[b + k] || mu[a + k] != mu[b + k]) {
            axisym = false;
            break;
          }
      }
  }
  const size_t nm = axisym ? (size_t)mrings * s->nz : s->n;
  try {
    s->rho.assign(nm, 0.0f); s->lam.assign(nm, 0.0f); s->mu.assign(nm, 0.0f);
  } catch (...) {
    return fail(CW_ERR_NOMEM, "out of host memory for the medium");
  }
  double vmax = 0;
  for (size_t p = 0; p < nin; p++) vmax = std::max(vmax, std::sqrt((lam[p] + 2 * mu[p]) / rho[p]));
  // source row: the input's (i, 0, k) for an axisymmetric store (rz input: (i, k))
  const int nrow = axisym ? 1 : s->nt;
  const size_t in_ring = rz ? (size_t)s->nz : (size_t)s->nt * s->nz;
  for (int i = 0; i < mrings; i++)
    for (int j = 0; j < nrow; j++) {
      const size_t dst = ((size_t)i * nrow + j) * s->nz;
      const size_t src = (size_t)i * in_ring + (size_t)j * s->nz;
      for (int k = 0; k < s->nz; k++) {
        s->rho[dst + k] = (float)rho[src + k];
        s->lam[dst + k] = (float)lam[src + k];
        s->mu[dst + k] = (float)mu[src + k];
      }
    }
  s->med_rz = axisym;
  s->nm = nm;
  s->vp_max = vmax;
  s->dt_cfl = courant(s, rho, lam, mu, rz);
  s->have_material = true;
  s->dt = 0;   // the tables depend on the medium: set_dt again
  return CW_OK;
}

cw_status cw_set_material(cw_sim *s, const double *rho, const double *lam, const double *mu)
{
  return set_medium(s, rho, lam, mu, false);
}

cw_status cw_set_material_rz(cw_sim *s, const double *rho, const double *lam, const double *mu)
{
  return set_medium(s, rho, lam, mu, true);
}

cw_status cw_set_pml(cw_sim *s, int32_t npml_r, int32_t npml_z, double rc, double alpha)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (npml_r < 0 || npml_z < 0) return fail(CW_ERR_RANGE, "negative layer width");
  if (npml_r >= s->nr) return fail(CW_ERR_RANGE, "npml_r=%d must be < nr=%d", npml_r, s->nr);
  if (npml_z > 0 && 2 * npml_z + 2 > s->nz)
    return fail(CW_ERR_RANGE, "2*npml_z+2=%d must be <= nz=%d", 2 * npml_z + 2, s->nz);
  if ((npml_r > 0 || npml_z > 0) && !(rc > 0 && rc < 1 && alpha >= 0 && std::isfinite(alpha)))
    return fail(CW_ERR_ARG, "need 0 < rc < 1 and alpha >= 0");
  s->npr = npml_r; s->npz = npml_z; s->rc = rc; s->alpha = alpha;
  s->dt = 0;
  return CW_OK;
}

cw_status cw_cfl_dt(const cw_sim *s, double *dt_cfl)
{
  if (!s || !dt_cfl) return fail(CW_ERR_ARG, "null argument");
  if (!s->have_material) return fail(CW_ERR_STATE, "medium not set");
  *dt_cfl = s->dt_cfl;
  return CW_OK;
}

cw_status cw_set_dt(cw_sim *s, double dt)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (!s->have_material) return fail(CW_ERR_STATE, "medium not set");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(CW_ERR_ARG, "dt must be finite and > 0");
  if (dt > s->dt_cfl * (1.0 + 1e-12))
    return fail(CW_ERR_UNSTABLE, "dt=%.6g above the Courant limit %.6g", dt, s->dt_cfl);
  s->dt = dt;
  build_tables(s);
  return CW_OK;
}

cw_status cw_add_source(cw_sim *s, int32_t kind, int32_t i, int32_t j, int32_t k,
                        const double *w, int64_t n)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (kind < CW_SRC_VOLUME || kind > CW_SRC_TORSION) return fail(CW_ERR_ARG, "bad source kind %d", kind);
  if (i < 0 || i >= s->nr || j < -1 || j >= s->nt || k < 0 || k >= s->nz)
    return fail(CW_ERR_RANGE, "source cell (%d,%d,%d) outside the grid", i, j, k);
  if (n < 0 || (n > 0 && !w)) return fail(CW_ERR_ARG, "bad wavelet");
  if (n > INT32_MAX) return fail(CW_ERR_RANGE, "wavelet too long");
  for (int64_t m = 0; m < n; m++)
    if (!std::isfinite(w[m])) return fail(CW_ERR_NONFINITE, "wavelet sample %lld not finite", (long long)m);
  if (!s->have_material) return fail(CW_ERR_STATE, "medium not set");
  if (!(s->dt > 0)) return fail(CW_ERR_STATE, "dt not set");
  SourceSpec src;
  src.kind = kind; src.i = i; src.j = j; src.k = k;
  src.w.assign(w, w + n);
  s->sources.push_back(std::move(src));
  return CW_OK;
}

cw_status cw_add_receiver(cw_sim *s, int32_t kind, int32_t field, int32_t i, int32_t j, int32_t k,
                          int32_t *id)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (kind != CW_REC_PRESSURE && kind != CW_REC_FIELD) return fail(CW_ERR_ARG, "bad receiver kind %d", kind);
  if (kind == CW_REC_FIELD && (field < 0 || field >= CW_NFIELD)) return fail(CW_ERR_ARG, "bad field %d", field);
  if (i < 0 || i >= s->nr || j < -1 || j >= s->nt || k < 0 || k >= s->nz)
    return fail(CW_ERR_RANGE, "receiver cell (%d,%d,%d) outside the grid", i, j, k);
  Receiver r{kind, kind == CW_REC_FIELD ? field : 0, i, j, k};
  s->receivers.push_back(r);
  if (id) *id = (int32_t)s->receivers.size() - 1;
  return CW_OK;
}

cw_status cw_set_trace_capacity(cw_sim *s, int64_t nsteps)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (nsteps < 0) return fail(CW_ERR_RANGE, "negative capacity");
  s->trace_cap = nsteps;
  return CW_OK;
}

cw_status cw_workspace_bytes(const cw_sim *s, uint64_t *bytes)
{
  if (!s || !bytes) return fail(CW_ERR_ARG, "null argument");
  *bytes = layout(s).total;
  return CW_OK;
}

cw_status cw_bind(cw_sim *s, void *workspace, uint64_t bytes, void *stream)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (!s->have_material) return fail(CW_ERR_STATE, "medium not set");
  if (!(s->dt > 0)) return fail(CW_ERR_STATE, "dt not set");
  if (!workspace) return fail(CW_ERR_ARG, "null workspace");
  s->drop_graph();
  if (((uintptr_t)workspace & 255) != 0) return fail(CW_ERR_ARG, "workspace not 256-byte aligned");
  const Layout L = layout(s);
  if (bytes < L.total)
    return fail(CW_ERR_NOMEM, "workspace of %llu bytes, need %llu", (unsigned long long)bytes,
                (unsigned long long)L.total);
  HIPCHK(hipGetDevice(&s->device));
  s->stream = (hipStream_t)stream;
  s->ws = (char *)workspace;
  s->ws_bytes = bytes;
  char *w = s->ws;
  for (int b = 0; b < 2; b++)
    for (int q = 0; q < NF; q++)
      s->fields[b][q] = (float *)(w + L.fields + (((size_t)b * NF + q) * s->n_alloc() +
                                                  (s->ghost_in ? s->rs() : 0)) * field_bytes(s));
  s->d_scl = (float *)(w + L.scales);
  s->d_maxabs = (unsigned *)(s->d_scl + 3 * NF);
  s->d_rho = (float *)(w + L.material);
  s->d_lam = s->d_rho + s->nm;
  s->d_mu = s->d_lam + s->nm;
  s->d_inv_rc = (float *)(w + L.metric);
  s->d_inv_rf = s->d_inv_rc + s->nr;
  s->d_tab_r = (float *)(w + L.tabr);
  s->d_tab_z = (float *)(w + L.tabz);
  const size_t slab_r = (size_t)s->npr * s->nt * s->nz, slab_z = (size_t)s->nr * s->nt * nzs_of(s);
  for (int c = 0; c < 2; c++) {
    for (int q = 0; q < NPSI_R; q++)
      s->psi_r[c][q] = slab_r ? (float *)(w + L.psir) + (c * NPSI_R + q) * slab_r : nullptr;
    for (int q = 0; q < NPSI_Z; q++)
      s->psi_z[c][q] = slab_z ? (float *)(w + L.psiz) + (c * NPSI_Z + q) * slab_z : nullptr;
  }
  s->d_inject = (Inject *)(w + L.inject);
  s->d_rec = (Receiver *)(w + L.rec);
  s->d_traces = (double *)(w + L.traces);
  s->d_energy = (double *)(w + L.energy);
  s->d_step = (int64_t *)(w + L.step);
  s->d_done = (unsigned *)(s->d_step + 1);
  if (s->adj) {
    float *p = (float *)(w + L.adj);
    for (int q = 0; q < NF; q++) { s->adj_fb[q] = p; p += s->n_alloc(); }
    for (int q = 0; q < NPSI_R; q++) { s->adj_pr[q] = slab_r ? p : nullptr; p += slab_r; }
    for (int q = 0; q < NPSI_Z; q++) { s->adj_pz[q] = slab_z ? p : nullptr; p += slab_z; }
    auto align64 = [](float *q) { return (float *)(((uintptr_t)q + 255) & ~(uintptr_t)255); };
    p = align64(p);                               // the term and coefficient arrays take 16-byte accesses
    for (int q = 0; q < 9; q++) { s->adj_T[q] = p; p += s->n_alloc(); }
    p = align64(p);
    for (int q = 0; q < 6; q++) { s->adj_C[q] = p; p += s->nm; }
    const size_t ncp = (size_t)((s->adj_steps + s->adj_every - 1) / s->adj_every);
    s->adj_ckpt = p; p += (ncp - 1) * adj_state_floats(s);
    s->adj_Z = p; p += (size_t)s->adj_every * 6 * adj_region_nodes(s);
    s->adj_w = p; p += (size_t)s->adj_steps * s->receivers.size();
    char *c = (char *)p;
    c += (256 - ((uintptr_t)c & 255)) & 255;
    s->adj_glam = (double *)c;
    s->adj_gmu = s->adj_glam + adj_region_cells(s);
  }

  // injections: dt * w[n] / V per target node, V the node (or ring) volume
  std::vector<float> amps(amp_floats(s));
  s->inject_host.clear();
  s->inject_amp.clear();
  size_t ao = 0;
  float *d_amp = (float *)(w + L.amp);
  for (const auto &src : s->sources) {
    struct T { int field; bool face; };   // face: the node sits at R_i, else at r_i
    std::vector<T> targets;
    int phase = 1;
    switch (src.kind) {
    case CW_SRC_VOLUME: targets = {{SRR, false}, {STT, false}, {SZZ, false}}; break;
    case CW_SRC_TORSION: targets = {{SRT, true}, {STZ, false}}; break;
    case CW_SRC_FORCE_R: targets = {{VR, true}}; phase = 0; break;
    case CW_SRC_FORCE_Z: targets = {{VZ, false}}; phase = 0; break;
    }
    for (const T &t : targets) {
      const double rad = (s->ring0 + src.i + (t.face ? 1.0 : 0.5)) * s->dr;
      const double vol = src.j < 0 ? 2.0 * kPi * rad * s->dr * s->dz : rad * s->dr * s->dth * s->dz;
      double scale = 1.0;
      if (t.field == VR || t.field == VZ) {
        // buoyancy at the node: 2 / (rho + rho of the next cell in r or z, clamped);
        // a ring source takes the ring's first cell, the medium being that of the caller
        const int jj = src.j < 0 ? 0 : src.j;
        const size_t p = mat_index(s, src.i, jj, src.k);
        const int i1 = std::min(src.i + 1, s->nr - 1 + s->med_extra), k1 = std::min(src.k + 1, s->nz - 1);
        const size_t p1 = t.field == VR ? mat_index(s, i1, jj, src.k) : mat_index(s, src.i, jj, k1);
        scale = 2.0 / ((double)s->rho[p] + (double)s->rho[p1]);
      }
      Inject e{};
      e.field = t.field; e.i = src.i; e.j = src.j; e.k = src.k; e.phase = phase;
      e.nsamp = (int)src.w.size();
      e.scale = (float)scale;
      e.amp = d_amp + ao;
      for (size_t m = 0; m < src.w.size(); m++) amps[ao + m] = (float)(s->dt * src.w[m] / vol);
      s->inject_amp.emplace_back(amps.begin() + ao, amps.begin() + ao + src.w.size());
      ao += src.w.size();
      s->inject_host.push_back(e);
    }
  }
  s->ninject = (int)s->inject_host.size();
  s->force_src = s->stress_src = false;
  s->inj_i0 = s->nr;
  s->inj_i1 = -1;
  for (const Inject &e : s->inject_host) {
    s->force_src = s->force_src || e.phase == 0;
    s->stress_src = s->stress_src || e.phase == 1;
    s->inj_i0 = std::min(s->inj_i0, e.i);
    s->inj_i1 = std::max(s->inj_i1, e.i);
  }

  HIPCHK(hipMemcpyAsync(s->d_rho, s->rho.data(), s->nm * sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_lam, s->lam.data(), s->nm * sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_mu, s->mu.data(), s->nm * sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_inv_rc, s->inv_rc.data(), s->nr * sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_inv_rf, s->inv_rf.data(), s->nr * sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_tab_r, s->tab_r.data(), s->tab_r.size() * sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_tab_z, s->tab_z.data(), s->tab_z.size() * sizeof(float), hipMemcpyHostToDevice, s->stream));
  if (s->ninject) {
    HIPCHK(hipMemcpyAsync(s->d_inject, s->inject_host.data(), s->ninject * sizeof(Inject), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(d_amp, amps.data(), amps.size() * sizeof(float), hipMemcpyHostToDevice, s->stream));
  }
  if (!s->receivers.empty())
    HIPCHK(hipMemcpyAsync(s->d_rec, s->receivers.data(), s->receivers.size() * sizeof(Receiver), hipMemcpyHostToDevice, s->stream));
  s->bound = true;
  if ((st = zero_state(s)) != CW_OK) { s->bound = false; return st; }
  // the host arrays above are pageable: finish the copies before they can go away
  HIPCHK(hipStreamSynchronize(s->stream));
  return CW_OK;
}

// Stress kernel form of the default (CW_PATH_AUTO) two-pass step per storage
// (bit 0 float32, bit 1 float16, bit 2 bfloat16 set: one cell per thread
// instead of four).
// Measured on MI355X at 256 x 128 x 8192 with non-temporal own-update
// accesses in both forms: float32 one cell per thread 3.32 ms against 3.41
// (four times as many threads keep more loads in flight); 16-bit storage
// four cells per thread, 2.17 / 2.31 ms against 4.92 / 6.05 (2-byte accesses).
#ifndef CW_STRESS_ONE_CELL
#define CW_STRESS_ONE_CELL 1
#endif
static bool stress_one_cell(int storage)
{
  const int bit = storage == ST_F32 ? 1 : storage == ST_F16 ? 2 : 4;
  return (CW_STRESS_ONE_CELL & bit) != 0;
}
// The same choice for the velocity update: float32 one cell per thread
// 2.68 ms against 2.715 for four (same box, same call); the 16-bit storages
// keep four cells per thread.
#ifndef CW_VELOCITY_ONE_CELL
#define CW_VELOCITY_ONE_CELL 1
#endif
static bool velocity_one_cell(int storage)
{
  const int bit = storage == ST_F32 ? 1 : storage == ST_F16 ? 2 : 4;
  return (CW_VELOCITY_ONE_CELL & bit) != 0;
}

cw_status cw_step(cw_sim *s, int64_t nsteps)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation");
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  if (nsteps < 0) return fail(CW_ERR_RANGE, "negative step count");
  if (!s->receivers.empty() && s->nstep + nsteps > s->trace_cap)
    return fail(CW_ERR_RANGE, "trace capacity %lld exceeded (%lld + %lld steps)", (long long)s->trace_cap,
                (long long)s->nstep, (long long)nsteps);
  HIPCHK(hipSetDevice(s->device));
  cw_status st;
  const int nrec = (int)s->receivers.size();
  // the fused step addresses a ring with 32-bit byte offsets
  const bool fits = s->ninject <= kMaxFusedInject && s->nr <= kMaxFusedRings &&
                    (uint64_t)s->nt * s->nz * 4 < (1ull << 32) && s->storage == ST_F32;
  const bool fused = s->path == CW_PATH_FUSED || (s->path == CW_PATH_AUTO && fits && kAutoFused);

  if (s->path == CW_PATH_FUSED && !fits)
    return fail(CW_ERR_RANGE, "the fused step takes float32 storage, at most %d injections and %d rings "
                "(have storage %d, %d injections, %d rings)", kMaxFusedInject, kMaxFusedRings, s->storage,
                s->ninject, s->nr);
  FusedArgs f{};
  if (fused) fused_tiles(s->nt, s->nz, &f.own_rows, &f.ntile_z);
  // two-pass kernel form: one workgroup per column segment with 4 depth cells
  // per thread; one thread per cell when nz is not a multiple of 4
  const bool vec = kUseVec && vec_applies(s->nt, s->nz);
  // the default path takes the faster form of each update; CW_PATH_TWO_PASS
  // keeps the four-cell column kernels (the form the batched kernels
  // reproduce bitwise)
  const bool vec_velocity = vec && !(s->path == CW_PATH_AUTO && velocity_one_cell(s->storage));
  const bool vec_stress = vec && !(s->path == CW_PATH_AUTO && stress_one_cell(s->storage));
  auto velocity = [&](const StepArgs &a, const TailArgs *tail) {
    return vec_velocity ? launch_velocity_vec(a, s->storage, s->stream)
                        : launch_velocity_basic(a, s->storage, s->stream, tail);
  };
  // With the one-cell float32 velocity update, a step's receivers and step
  // counter are taken by extra workgroups at the front of the next step's velocity
  // launch (it reads only the buffer they sample and does not read the
  // counter), so that only the last step of a run of steps -- a call, or a
  // captured graph -- has a launch of its own for them.  The 16-bit storages
  // keep the tail launch, which also sets the float16 scales.
  const bool fold_tail = !vec_velocity && s->storage == ST_F32;
  TailArgs tail{s->d_rec, nrec, std::max(1, (nrec + 3) / 4), s->d_step, s->trace_cap, s->d_traces, s->d_done};
  auto stress = [&](const StepArgs &a) {
    return vec_stress ? launch_stress_vec(a, s->storage, s->stream)
                      : launch_stress_basic(a, s->storage, s->stream);
  };
  // One step's launches.  Nothing in them depends on the host's step count
  // (the injection and receiver kernels read the device counter, which the
  // last launch advances), so the launches of an even number of two-pass
  // steps can be captured once and replayed.
  // the step's last launch: receivers, float16 rescale, step counter
  auto finish_step = [&](const StepArgs &a) -> cw_status {
    if ((st = timed(s, CW_K_RECORD, [&] {
          return launch_step_tail(s->d_rec, nrec, s->d_step, s->trace_cap, a, s->storage, s->d_traces, s->d_done,
                                  s->d_scl + (1 - s->cur) * NF, s->d_scl + 2 * NF, s->d_maxabs, s->stream);
        })) != CW_OK)
      return st;
    s->cur = 1 - s->cur;
    return CW_OK;
  };
  // velocity update, force sources (if any), stress update (the one-cell form
  // adds the stress sources itself, the four-cell one takes a source launch),
  // the tail: three launches for the default float32 path
  // prev_tail: fold the previous step's tail into this step's velocity
  // launch; own_tail: end the step with the tail launch (otherwise the next
  // step's velocity launch takes it)
  auto two_pass_step = [&](bool prev_tail, bool own_tail) -> cw_status {
    StepArgs a = step_args(s, s->cur, 1 - s->cur);
    if (s->ninject) {
      a.inj = s->d_inject;
      a.ninj = s->ninject;
      a.inj_i0 = s->inj_i0;
      a.inj_i1 = s->inj_i1;
      a.step = s->d_step;
    }
    if ((st = timed(s, CW_K_VELOCITY, [&] { return velocity(a, prev_tail ? &tail : nullptr); })) != CW_OK) return st;
    if (s->force_src &&
        (st = timed(s, CW_K_INJECT, [&] { return launch_sources(a, 0, s->storage, s->stream); })) != CW_OK)
      return st;
    if ((st = timed(s, CW_K_STRESS, [&] { return stress(a); })) != CW_OK) return st;
    if (s->stress_src && vec_stress &&
        (st = timed(s, CW_K_INJECT, [&] { return launch_sources(a, 1, s->storage, s->stream); })) != CW_OK)
      return st;
    if (own_tail) return finish_step(a);
    s->cur = 1 - s->cur;
    return CW_OK;
  };
  auto fused_step = [&](int64_t n) -> cw_status {   // source amplitudes of step n go in as arguments
    const StepArgs a = step_args(s, s->cur, 1 - s->cur);
    f.nr = s->nr; f.nt = s->nt; f.nz = s->nz; f.npr = s->npr; f.npz = s->npz; f.nzs = nzs_of(s);
    f.dt = a.dt; f.inv_dr = a.inv_dr; f.inv_dz = a.inv_dz; f.inv_dth = a.inv_dth;
    f.n = s->n_alloc();
    f.rs = s->rs();
    f.slab_r = (size_t)s->npr * s->nt * s->nz;
    f.slab_z = (size_t)s->nr * s->nt * nzs_of(s);
    f.in = s->fields[s->cur][0];
    f.out = s->fields[1 - s->cur][0];
    f.med = s->d_rho;
    f.m_n = s->nm;
    f.m_ring = a.m_ring;
    f.m_row = a.m_row;
    f.psi_r_in = s->psi_r[s->psi_cur][0]; f.psi_r_out = s->psi_r[1 - s->psi_cur][0];
    f.psi_z_in = s->psi_z[s->psi_cur][0]; f.psi_z_out = s->psi_z[1 - s->psi_cur][0];
    f.inv_rc = s->d_inv_rc; f.inv_rf = s->d_inv_rf; f.tab_r = s->d_tab_r; f.tab_z = s->d_tab_z;
    f.ninj = 0;
    for (int e = 0; e < s->ninject; e++) {
      const Inject &in = s->inject_host[e];
      if (n >= in.nsamp) continue;
      InjectStep &o = f.inj[f.ninj++];
      o.field = in.field; o.i = in.i; o.j = in.j; o.k = in.k; o.phase = in.phase;
      o.amp = in.scale * s->inject_amp[e][n];
    }
    if ((st = timed(s, CW_K_FUSED, [&] { return launch_fused(f, s->stream); })) != CW_OK) return st;
    s->psi_cur = 1 - s->psi_cur;
    return finish_step(a);
  };

  if (fused) {
    for (int64_t t = 0; t < nsteps; t++) {
      if ((st = fused_step(s->nstep)) != CW_OK) return st;
      s->nstep++;
    }
    return CW_OK;
  }
  const bool use_graph = s->graph_steps > 0 && !s->profiling;
  int64_t done = 0;
  bool pending = false;                        // the previous ordinary step left its tail to this one
  while (done < nsteps) {
    if (use_graph && s->cur == 0 && nsteps - done >= s->graph_steps) {
      if (!s->graph_exec) {
        // capture (nothing runs) on a stream of our own, since the caller's may be
        // the null stream, which cannot be captured; an even step count leaves the
        // buffers as they were
        if (!s->capture_stream) HIPCHK(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
        hipStream_t user = s->stream;
        s->stream = s->capture_stream;
        const hipError_t eb = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
        cw_status cst = eb == hipSuccess ? CW_OK : fail(CW_ERR_HIP, "graph capture: %s", hipGetErrorString(eb));
        for (int g = 0; g < s->graph_steps && cst == CW_OK; g++)
          cst = two_pass_step(fold_tail && g > 0, !fold_tail || g == s->graph_steps - 1);
        hipGraph_t gr = nullptr;
        const hipError_t ee = eb == hipSuccess ? hipStreamEndCapture(s->stream, &gr) : hipSuccess;
        s->stream = user;
        s->cur = 0;
        if (cst != CW_OK || ee != hipSuccess) {
          if (gr) (void)hipGraphDestroy(gr);
          return cst != CW_OK ? cst : fail(CW_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ee));
        }
        s->graph = gr;
        const hipError_t ei = hipGraphInstantiate(&s->graph_exec, gr, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
          s->drop_graph();
          return fail(CW_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
        }
      }
      HIPCHK(hipGraphLaunch(s->graph_exec, s->stream));
      done += s->graph_steps;
      s->nstep += s->graph_steps;
      continue;
    }
    // the last step of the call, or one a graph replay follows, runs its own tail
    const bool graph_next = use_graph && s->cur == 1 && nsteps - done - 1 >= s->graph_steps;
    const bool own = !fold_tail || done + 1 == nsteps || graph_next;
    if ((st = two_pass_step(pending, own)) != CW_OK) return st;
    pending = !own;
    done++;
    s->nstep++;
  }
  return CW_OK;
}

// After the stream has drained: CW_ERR_NONFINITE once a float16 field has
// overflowed (the device sets the field's bit; it stays set until the state
// is reset), else CW_OK.
static cw_status check_overflow(cw_sim *s)
{
  if (s->storage != ST_F16) return CW_OK;
  unsigned mask = 0u;
  HIPCHK(hipMemcpyAsync(&mask, s->d_maxabs + kOverflowWord, sizeof mask, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (!mask) return CW_OK;
  static const char *const name[NF] = {"vr", "vt", "vz", "srr", "stt", "szz", "srt", "srz", "stz"};
  int q = 0;
  while (!(mask >> q & 1u)) q++;
  return fail(CW_ERR_NONFINITE,
              "float16 field %s overflowed (fields mask 0x%x): it grew more than its scale's headroom of 2^%d "
              "in one step; the state is not valid until cw_reset or cw_bind",
              name[q], mask, 16 - kF16TargetExp);
}

cw_status cw_sync(cw_sim *s)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation");
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  HIPCHK(hipSetDevice(s->device));
  HIPCHK(hipStreamSynchronize(s->stream));
  return check_overflow(s);
}

cw_status cw_get_traces(cw_sim *s, double *out, int64_t cap, int64_t *nsteps_done)
{
  if (!s || (!out && !s->receivers.empty())) return fail(CW_ERR_ARG, "null argument");
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  if (cap < s->nstep) return fail(CW_ERR_RANGE, "cap %lld < steps done %lld", (long long)cap, (long long)s->nstep);
  if (nsteps_done) *nsteps_done = s->nstep;
  if (s->receivers.empty() || s->nstep == 0) return CW_OK;
  HIPCHK(hipSetDevice(s->device));
  HIPCHK(hipMemcpy2DAsync(out, cap * sizeof(double), s->d_traces, s->trace_cap * sizeof(double),
                          s->nstep * sizeof(double), s->receivers.size(), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return check_overflow(s);
}

// float16 scale for values up to maxabs: 2^(e - target), max = f 2^e
static float f16_scale(double maxabs)
{
  if (!(maxabs > 0) || !std::isfinite(maxabs)) return 1.0f;
  int e;
  std::frexp(maxabs, &e);
  return std::ldexp(1.0f, e - kF16TargetExp);
}

static float bf16_to_float(uint16_t h)
{
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static uint16_t float_to_bf16(float f)
{
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Copy between a packed host array [nr][nt][nz] of eb-byte values and a
// field array, whose rings lie rs() values apart.
static hipError_t field_copy(cw_sim *s, void *dst, const void *src, size_t eb, bool to_host)
{
  const size_t ring = (size_t)s->nt * s->nz * eb, pitch = s->rs() * eb;
  return to_host ? hipMemcpy2DAsync(dst, ring, src, pitch, ring, s->nr, hipMemcpyDeviceToHost, s->stream)
                 : hipMemcpy2DAsync(dst, pitch, src, ring, ring, s->nr, hipMemcpyHostToDevice, s->stream);
}

cw_status cw_get_field(cw_sim *s, int32_t field, float *host_out)
{
  if (!s || !host_out) return fail(CW_ERR_ARG, "null argument");
  if (field < 0 || field >= CW_NFIELD) return fail(CW_ERR_ARG, "bad field %d", field);
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  HIPCHK(hipSetDevice(s->device));
  if (s->storage == ST_F32) {
    HIPCHK(field_copy(s, host_out, s->fields[s->cur][field], sizeof(float), true));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CW_OK;
  }
  std::vector<uint16_t> raw;
  try { raw.resize(s->n); } catch (...) { return fail(CW_ERR_NOMEM, "out of host memory"); }
  float scl = 1.0f;
  HIPCHK(field_copy(s, raw.data(), s->fields[s->cur][field], 2, true));
  HIPCHK(hipMemcpyAsync(&scl, s->d_scl + s->cur * NF + field, sizeof(float), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (s->storage == ST_F16) {
    const _Float16 *h = reinterpret_cast<const _Float16 *>(raw.data());
    for (size_t p = 0; p < s->n; p++) host_out[p] = (float)h[p] * scl;
  } else {
    for (size_t p = 0; p < s->n; p++) host_out[p] = bf16_to_float(raw[p]);
  }
  return check_overflow(s);
}

cw_status cw_set_field(cw_sim *s, int32_t field, const float *host_in)
{
  if (!s || !host_in) return fail(CW_ERR_ARG, "null argument");
  if (field < 0 || field >= CW_NFIELD) return fail(CW_ERR_ARG, "bad field %d", field);
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  HIPCHK(hipSetDevice(s->device));
  for (size_t p = 0; p < s->n; p++)
    if (!std::isfinite(host_in[p])) return fail(CW_ERR_NONFINITE, "value %zu is not finite", p);
  if (s->storage == ST_F32) {
    HIPCHK(field_copy(s, s->fields[s->cur][field], host_in, sizeof(float), false));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CW_OK;
  }
  std::vector<uint16_t> raw;
  try { raw.resize(s->n); } catch (...) { return fail(CW_ERR_NOMEM, "out of host memory"); }
  float scl = 1.0f;
  if (s->storage == ST_F16) {
    double m = 0;
    for (size_t p = 0; p < s->n; p++) m = std::max(m, (double)std::fabs(host_in[p]));
    scl = f16_scale(m);
    _Float16 *h = reinterpret_cast<_Float16 *>(raw.data());
    for (size_t p = 0; p < s->n; p++) h[p] = (_Float16)(host_in[p] / scl);
  } else {
    for (size_t p = 0; p < s->n; p++) raw[p] = float_to_bf16(host_in[p]);
  }
  HIPCHK(field_copy(s, s->fields[s->cur][field], raw.data(), 2, false));
  // the buffer's scale, and the scale of the next write of this field
  HIPCHK(hipMemcpyAsync(s->d_scl + s->cur * NF + field, &scl, sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_scl + 2 * NF + field, &scl, sizeof(float), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return CW_OK;
}

cw_status cw_energy(cw_sim *s, double *E)
{
  if (!s || !E) return fail(CW_ERR_ARG, "null argument");
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  if (s->nstep < 1) return fail(CW_ERR_STATE, "energy needs at least one step");
  HIPCHK(hipSetDevice(s->device));
  const StepArgs a = step_args(s, 1 - s->cur, s->cur);   // in: level n, out: level n+1
  const double scale = s->dr * s->dr * s->dth * s->dz;  // radii are in units of dr
  StepArgs ae = a;
  ae.scl_out = s->d_scl + s->cur * NF;                  // the current buffer's own scales
  HIPCHK(launch_energy(ae, s->storage, s->d_energy, kEnergyBlocks, scale, s->d_energy + kEnergyBlocks, s->stream));
  HIPCHK(hipMemcpyAsync(E, s->d_energy + kEnergyBlocks, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (!std::isfinite(*E)) return fail(CW_ERR_NONFINITE, "energy is not finite");
  return CW_OK;
}

// ---- allocation-free energy ------------------------------------------------
// Scratch of cw_energy_noalloc: the per-workgroup partial sums and the result.
// One copy per GPU, held until the process ends.  In host code the array's
// name is only a stand-in; its device address comes from hipGetSymbolAddress,
// taken once per device and kept in g_scratch.
constexpr int kNoAllocMaxBlocks = 4096;
static __device__ __align__(256) double scratch[kNoAllocMaxBlocks + 1];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// device address of this device's scratch (the device must be current)
cw_status scratch_ptr(int device, double **out)
{
  if (device < 0 || device >= kMaxDevices) return fail(CW_ERR_ARG, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CW_ERR_HIP, "no device address for the energy scratch");
    g_scratch[device] = static_cast<double *>(p);
  }
  *out = g_scratch[device];
  return CW_OK;
}
}  // namespace

cw_status cw_energy_noalloc(cw_sim *s, int32_t nblocks, double *E)
{
  if (!s || !E) return fail(CW_ERR_ARG, "null argument");
  if (nblocks < 1 || nblocks > kNoAllocMaxBlocks)
    return fail(CW_ERR_RANGE, "nblocks %d outside [1, %d] (the static scratch holds %d partial sums)", nblocks,
                kNoAllocMaxBlocks, kNoAllocMaxBlocks);
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  if (s->nstep < 1) return fail(CW_ERR_STATE, "energy needs at least one step");
  HIPCHK(hipSetDevice(s->device));
  double *scr = nullptr;
  const cw_status st = scratch_ptr(s->device, &scr);
  if (st != CW_OK) return st;
  const StepArgs a = step_args(s, 1 - s->cur, s->cur);
  const double scale = s->dr * s->dr * s->dth * s->dz;
  StepArgs ae = a;
  ae.scl_out = s->d_scl + s->cur * NF;
  // every partial and the result are written by the kernels, so nothing is cleared
  HIPCHK(launch_energy(ae, s->storage, scr, nblocks, scale, scr + nblocks, s->stream));
  HIPCHK(hipMemcpyAsync(E, scr + nblocks, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (!std::isfinite(*E)) return fail(CW_ERR_NONFINITE, "energy is not finite");
  return CW_OK;
}

cw_status cw_reset(cw_sim *s)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation");
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  HIPCHK(hipSetDevice(s->device));
  return zero_state(s);
}

cw_status cw_set_storage(cw_sim *s, int32_t storage)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (storage < CW_STORE_F32 || storage > CW_STORE_BF16) return fail(CW_ERR_ARG, "bad storage %d", storage);
  s->storage = storage;
  return CW_OK;
}

cw_status cw_set_rounding(cw_sim *s, int32_t mode)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation");
  if (mode != CW_ROUND_NEAREST && mode != CW_ROUND_STOCHASTIC) return fail(CW_ERR_ARG, "bad rounding mode %d", mode);
  s->drop_graph();
  s->rounding = mode;
  return CW_OK;
}

cw_status cw_set_path(cw_sim *s, int32_t path)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation");
  if (path < CW_PATH_AUTO || path > CW_PATH_FUSED) return fail(CW_ERR_ARG, "bad path %d", path);
  if (path != s->path) s->drop_graph();
  s->path = path;
  return CW_OK;
}

cw_status cw_set_graph(cw_sim *s, int32_t steps)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation");
  if (steps < 0 || steps % 2 || steps > kMaxGraphSteps)
    return fail(CW_ERR_RANGE, "graph steps must be even and in [0, %d] (have %d)", kMaxGraphSteps, steps);
  s->drop_graph();
  s->graph_steps = steps;
  return CW_OK;
}

cw_status cw_profile(cw_sim *s, int32_t enable)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation");
  if (!enable) {
    if (!s->prof.empty() && s->bound) HIPCHK(hipStreamSynchronize(s->stream));
    for (auto &r : s->prof) { s->event_pool.push_back(r.start); s->event_pool.push_back(r.stop); }
    s->prof.clear();
  }
  s->profiling = enable != 0;
  return CW_OK;
}

cw_status cw_profile_read(cw_sim *s, int32_t kernel, double *total_ms, int64_t *launches)
{
  if (!s || !total_ms || !launches) return fail(CW_ERR_ARG, "null argument");
  if (kernel < 0 || kernel >= CW_K_COUNT) return fail(CW_ERR_ARG, "bad kernel id %d", kernel);
  double tot = 0;
  int64_t cnt = 0;
  for (auto &r : s->prof) {
    if (r.kernel != kernel) continue;
    HIPCHK(hipEventSynchronize(r.stop));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.start, r.stop));
    tot += ms;
    cnt++;
  }
  *total_ms = tot;
  *launches = cnt;
  return CW_OK;
}

cw_status cw_steps_done(const cw_sim *s, int64_t *n)
{
  if (!s || !n) return fail(CW_ERR_ARG, "null argument");
  *n = s->nstep;
  return CW_OK;
}

cw_status cw_ricker(double f0, const double *t, int64_t n, double *out)
{
  if (!(f0 > 0) || (n > 0 && (!t || !out)) || n < 0) return fail(CW_ERR_ARG, "bad Ricker arguments");
  for (int64_t m = 0; m < n; m++) {
    const double x = kPi * f0 * (t[m] - 2.0 / f0);
    const double x2 = x * x;
    out[m] = (1.0 - 2.0 * x2) * std::exp(-x2);
  }
  return CW_OK;
}

cw_status cw_stream_probe(void *dev, uint64_t bytes_per_array, int32_t nread, int32_t nwrite, int32_t lane_bytes,
                          int32_t reps, void *stream, double *ms_per_pass)
{
  if (!dev || !ms_per_pass || reps < 1) return fail(CW_ERR_ARG, "null buffer or result, or reps < 1");
  const bool nt = (lane_bytes & CW_PROBE_NONTEMPORAL) != 0;
  lane_bytes &= ~CW_PROBE_NONTEMPORAL;
  if (lane_bytes != 4 && lane_bytes != 16)
    return fail(CW_ERR_ARG, "lane_bytes must be 4 or 16 (with CW_PROBE_NONTEMPORAL or not)");
  if (((uintptr_t)dev & 15) || bytes_per_array < 16 || (bytes_per_array & 15))
    return fail(CW_ERR_ARG, "the buffer must be 16-byte aligned and each array a positive multiple of 16 bytes");
  if (!stream_mix_supported(nread, nwrite))
    return fail(CW_ERR_RANGE, "unsupported stream mix %d reads / %d writes", nread, nwrite);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CW_ERR_HIP, "hipEventCreate failed");
  }
  cw_status res = CW_OK;
  float ms = 0.0f;
  auto run = [&](int n) {
    for (int q = 0; q < n; q++)
      if (launch_stream(dev, bytes_per_array, lane_bytes, nt, nread, nwrite, st) != hipSuccess) return false;
    return true;
  };
  if (!run(2) || hipEventRecord(e0, st) != hipSuccess || !run(reps) || hipEventRecord(e1, st) != hipSuccess ||
      hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    res = fail(CW_ERR_HIP, "stream probe failed: %s", hipGetErrorString(hipGetLastError()));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res == CW_OK) *ms_per_pass = (double)ms / reps;
  return res;
}

static cw_status check_adjoint_region(const cw_sim *s)
{
  const int k1 = s->adj_k0 + s->adj_nb * s->adj_br;
  const int rmax = s->nr - std::max(s->npr, 2), zmax = s->nz - 1 - std::max(s->npz, 1);
  if (s->adj_i0 < 1 || s->adj_i1 <= s->adj_i0 || s->adj_i1 > rmax || s->adj_k0 < std::max(s->npz + 1, 1) ||
      k1 > zmax)
    return fail(CW_ERR_RANGE, "the parameter region (rings [%d, %d), depths [%d, %d)) must lie inside rings "
                "[1, %d) and depths [%d, %d), clear of the absorbing layer and the grid's edges",
                s->adj_i0, s->adj_i1, s->adj_k0, k1, rmax, std::max(s->npz + 1, 1), zmax);
  return CW_OK;
}

cw_status cw_set_adjoint(cw_sim *s, int64_t nsteps, int32_t checkpoint_every, int32_t i0, int32_t i1, int32_t k0,
                         int32_t nbins, int32_t bin_rows)
{
  cw_status st;
  if (!configurable(s, &st)) return st;
  if (nsteps < 0 || checkpoint_every < 1 || nbins < 1 || bin_rows < 1)
    return fail(CW_ERR_RANGE, "need nsteps >= 0, checkpoint_every >= 1, nbins >= 1, bin_rows >= 1");
  if (nsteps == 0) {
    s->adj = false;
    return CW_OK;
  }
  cw_sim t = {};
  t.nr = s->nr; t.nz = s->nz; t.npr = s->npr; t.npz = s->npz;
  t.adj_i0 = i0; t.adj_i1 = i1; t.adj_k0 = k0; t.adj_nb = nbins; t.adj_br = bin_rows;
  if ((st = check_adjoint_region(&t)) != CW_OK) return st;
  s->adj = true;
  s->adj_steps = nsteps;
  s->adj_every = (int)std::min<int64_t>(checkpoint_every, std::max<int64_t>(nsteps, 1));   // a segment holds at most the run
  s->adj_i0 = i0; s->adj_i1 = i1; s->adj_k0 = k0; s->adj_nb = nbins; s->adj_br = bin_rows;
  if (s->trace_cap < nsteps) s->trace_cap = nsteps;
  s->adj_mu0.clear();
  s->adj_K0.clear();
  return CW_OK;
}

// cells of the region as stored in the medium arrays (every theta row of a
// 3-D medium, one of an axisymmetric one), in the order the shifts walk them
extern "C++" template <class F>
static void for_region_medium(const cw_sim *s, F &&f)
{
  const int rows = s->med_rz ? 1 : s->nt;
  const int k1 = s->adj_k0 + s->adj_nb * s->adj_br;
  for (int i = s->adj_i0; i < s->adj_i1; i++)
    for (int j = 0; j < rows; j++)
      for (int k = s->adj_k0; k < k1; k++) f(i, j, k, (k - s->adj_k0) / s->adj_br, mat_index(s, i, j, k));
}

cw_status cw_set_region_moduli(cw_sim *s, const double *dmu, const double *dK)
{
  if (!s || !dmu || !dK) return fail(CW_ERR_ARG, "null argument");
  if (!s->adj) return fail(CW_ERR_STATE, "no parameter region: cw_set_adjoint first");
  if (!s->have_material) return fail(CW_ERR_STATE, "medium not set");
  if (s->adj_mu0.empty())
    for_region_medium(s, [&](int, int, int, int, size_t p) {
      s->adj_mu0.push_back(s->mu[p]);
      s->adj_K0.push_back((double)s->lam[p] + 2.0 * s->mu[p] / 3.0);
    });
  std::vector<float> mu_new, lam_new;
  size_t c = 0;
  bool ok = true;
  double worst = INFINITY;
  for_region_medium(s, [&](int i, int, int, int b, size_t p) {
    const double mu = s->adj_mu0[c] + dmu[b], K = s->adj_K0[c] + dK[b];
    const double lam = K - 2.0 * mu / 3.0;
    c++;
    if (!(mu >= 0) || !(lam + 2 * mu > 0) || !std::isfinite(mu) || !std::isfinite(K)) ok = false;
    const double vp = std::sqrt(std::max(lam + 2 * mu, 0.0) / s->rho[p]);
    const double ra = (i + 0.5) * s->dr * s->dth;
    const double g = std::sqrt(1.0 / (s->dr * s->dr) + 1.0 / (ra * ra) + 1.0 / (s->dz * s->dz));
    worst = std::min(worst, 1.0 / (vp * g));
    mu_new.push_back((float)mu);
    lam_new.push_back((float)lam);
  });
  if (!ok) return fail(CW_ERR_MATERIAL, "shifted moduli out of range (need mu >= 0, lambda + 2 mu > 0)");
  if (s->dt > worst) return fail(CW_ERR_UNSTABLE, "dt %.6g exceeds the Courant limit %.6g of the shifted region",
                                 s->dt, worst);
  c = 0;
  for_region_medium(s, [&](int, int, int, int, size_t p) {
    s->mu[p] = mu_new[c];
    s->lam[p] = lam_new[c];
    c++;
  });
  if (s->bound) {
    HIPCHK(hipSetDevice(s->device));
    // the rings of the region, whole (contiguous in both medium layouts)
    const size_t ring = s->med_rz ? (size_t)s->nz : (size_t)s->nt * s->nz;
    const size_t off = (size_t)s->adj_i0 * ring, cnt = (size_t)(s->adj_i1 - s->adj_i0) * ring;
    HIPCHK(hipMemcpyAsync(s->d_mu + off, s->mu.data() + off, cnt * sizeof(float), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->d_lam + off, s->lam.data() + off, cnt * sizeof(float), hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  return CW_OK;
}

cw_status cw_gradient(cw_sim *s, int64_t n0, int64_t n1, double *loss, double *grad_mu, double *grad_K)
{
  if (!s || !loss || !grad_mu || !grad_K) return fail(CW_ERR_ARG, "null argument");
  if (!s->bound) return fail(CW_ERR_STATE, "cw_bind first");
  if (!s->adj) return fail(CW_ERR_STATE, "cw_set_adjoint before cw_bind");
  if (s->storage != ST_F32) return fail(CW_ERR_STATE, "the gradient runs with float32 storage");
  if (s->path == CW_PATH_FUSED) return fail(CW_ERR_STATE, "the gradient runs on the two-pass path");
  cw_status st;
  if ((st = check_adjoint_region(s)) != CW_OK) return st;
  HIPCHK(hipSetDevice(s->device));
  const int64_t N = s->adj_steps, C = s->adj_every, ncp = (N + C - 1) / C;
  const size_t nst = adj_state_floats(s), n = s->n_alloc();
  const size_t slab_r = (size_t)s->npr * s->nt * s->nz, slab_z = (size_t)s->nr * s->nt * nzs_of(s);
  const int nrec = (int)s->receivers.size();
  const AdjRegion g = adj_region(s);
  const size_t nreg = adj_region_nodes(s), ncell = adj_region_cells(s);
  std::vector<int> ck_cur(ncp);
  auto state_copy = [&](float *ck, int buf, bool save) -> cw_status {
    float *parts[3] = {s->fields[buf][0], slab_r ? s->psi_r[s->psi_cur][0] : nullptr,
                       slab_z ? s->psi_z[s->psi_cur][0] : nullptr};
    const size_t cnt[3] = {NF * n, NPSI_R * slab_r, NPSI_Z * slab_z};
    size_t o = 0;
    for (int q = 0; q < 3; q++) {
      if (cnt[q])
        HIPCHK(hipMemcpyAsync(save ? ck + o : parts[q], save ? parts[q] : ck + o, cnt[q] * sizeof(float),
                              hipMemcpyDeviceToDevice, s->stream));
      o += cnt[q];
    }
    return CW_OK;
  };
  // the adjoint step's arguments and coefficients (the capture of the strain
  // rates needs the grid's metric from them)
  const StepArgs sa = step_args(s, 0, 1);
  AdjArgs a{};
  a.nr = s->nr; a.nt = s->nt; a.nz = s->nz; a.npr = s->npr; a.npz = s->npz; a.nzs = nzs_of(s);
  a.rs = sa.rs;
  a.dt = sa.dt; a.inv_dr = sa.inv_dr; a.inv_dz = sa.inv_dz; a.inv_dth = sa.inv_dth;
  a.inv_rc = sa.inv_rc; a.inv_rf = sa.inv_rf;
  a.rho = sa.rho; a.lam = sa.lam; a.mu = sa.mu; a.m_ring = sa.m_ring; a.m_row = sa.m_row;
  for (int q = 0; q < NF; q++) a.fb[q] = s->adj_fb[q];
  for (int q = 0; q < NPSI_R; q++) a.pr[q] = s->adj_pr[q];
  for (int q = 0; q < NPSI_Z; q++) a.pz[q] = s->adj_pz[q];
  for (int q = 0; q < 9; q++) a.T[q] = s->adj_T[q];
  for (int q = 0; q < 6; q++) a.C[q] = s->adj_C[q];
  a.tab_r = sa.tab_r; a.tab_z = sa.tab_z;
  HIPCHK(launch_adjoint_coefs(a, s->stream));
  // forward from rest, a checkpoint at the start of every segment but the
  // last, whose strain rates are stored as it is run, so that the backward
  // sweep starts without recomputing it (with one segment nothing is
  // recomputed)
  if ((st = zero_state(s)) != CW_OK) return st;
  for (int64_t t = 0; t < N; t += C) {
    if (t / C < ncp - 1) {
      ck_cur[t / C] = s->cur;
      if ((st = state_copy(s->adj_ckpt + (size_t)(t / C) * nst, s->cur, true)) != CW_OK) return st;
      if ((st = cw_step(s, C)) != CW_OK) return st;
      continue;
    }
    for (int64_t u = t; u < N; u++) {
      if ((st = cw_step(s, 1)) != CW_OK) return st;
      HIPCHK(launch_adjoint_capture(a, g, s->fields[s->cur][VR], s->fields[s->cur][VT],
                                    s->fields[s->cur][VZ], s->adj_Z + (size_t)(u - t) * 6 * nreg, s->stream));
    }
  }
  // loss and the receivers' adjoint weights
  std::vector<double> tr((size_t)nrec * s->trace_cap);
  HIPCHK(hipStreamSynchronize(s->stream));
  if (nrec) HIPCHK(hipMemcpy(tr.data(), s->d_traces, tr.size() * sizeof(double), hipMemcpyDeviceToHost));
  double L = 0.0;
  std::vector<float> w((size_t)N * nrec, 0.0f);
  for (int m = 0; m < nrec; m++) {
    const Receiver &r = s->receivers[m];
    if (r.kind != CW_REC_PRESSURE) continue;
    const int cells = r.j < 0 ? s->nt : 1;
    for (int64_t t = std::max<int64_t>(n0, 0); t < std::min(n1, N); t++) {
      const double p = tr[(size_t)m * s->trace_cap + t];
      L += p * p;
      w[(size_t)t * nrec + m] = (float)(2.0 * p * (-1.0 / (3.0 * cells)));
    }
  }
  *loss = L;
  if (nrec) HIPCHK(hipMemcpy(s->adj_w, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
  // adjoint state and accumulators from zero
  HIPCHK(hipMemsetAsync(s->adj_fb[0], 0, nst * sizeof(float), s->stream));
  HIPCHK(hipMemsetAsync(s->adj_glam, 0, 2 * ncell * sizeof(double), s->stream));
  // segments backwards: recompute the segment's strain rates (but for the
  // last segment's, stored by the forward run), then its adjoint steps
  for (int64_t seg = ncp - 1; seg >= 0; seg--) {
    const int64_t t0 = seg * C, t1 = std::min(t0 + C, N);
    if (seg < ncp - 1) {
      if ((st = state_copy(s->adj_ckpt + (size_t)seg * nst, ck_cur[seg], false)) != CW_OK) return st;
      s->cur = ck_cur[seg];
      s->nstep = t0;
      HIPCHK(launch_set_step(s->d_step, t0, s->stream));
    }
    for (int64_t t = t0; t < t1 && seg < ncp - 1; t++) {
      if ((st = cw_step(s, 1)) != CW_OK) return st;
      HIPCHK(launch_adjoint_capture(a, g, s->fields[s->cur][VR], s->fields[s->cur][VT], s->fields[s->cur][VZ],
                                    s->adj_Z + (size_t)(t - t0) * 6 * nreg, s->stream));
    }
    for (int64_t t = t1 - 1; t >= t0; t--)
      HIPCHK(launch_adjoint_step(a, s->d_rec, nrec, s->adj_w + (size_t)t * nrec, g,
                                 s->adj_Z + (size_t)(t - t0) * 6 * nreg, s->adj_glam, s->adj_gmu, s->stream));
  }
  std::vector<double> glam(ncell), gmu(ncell);
  HIPCHK(hipStreamSynchronize(s->stream));
  HIPCHK(hipMemcpy(glam.data(), s->adj_glam, ncell * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(gmu.data(), s->adj_gmu, ncell * sizeof(double), hipMemcpyDeviceToHost));
  for (int b = 0; b < s->adj_nb; b++) { grad_mu[b] = 0.0; grad_K[b] = 0.0; }
  const int nk = g.k1 - g.k0;
  for (size_t c = 0; c < ncell; c++) {
    const int b = (int)(c % nk) / s->adj_br;
    grad_mu[b] += gmu[c] - (2.0 / 3.0) * glam[c];
    grad_K[b] += glam[c];
  }
  return CW_OK;
}

/* ------------------------------ batches ------------------------------ */
struct cw_batch {
  std::vector<cw_sim *> sims;
  std::vector<int> tz;                 // tile shape per instance (wavefronts along depth)
  int wpe = 0;                         // minimum wavefronts per SIMD of the batched kernels (0: none)
  bool bound = false;
  int device = 0;
  hipStream_t stream = nullptr;
  BatchInst *d_inst = nullptr;
  long *d_tile0 = nullptr;
  long tiles = 0;
  int max_rec = 0;
  bool any_inject = false;
  int graph_steps = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;
  void drop_graph()
  {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  ~cw_batch()
  {
    drop_graph();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
};

static cw_status check_batch_member(const cw_batch *b, const cw_sim *s)
{
  if (!s) return fail(CW_ERR_ARG, "null simulation in the batch");
  if (!s->bound) return fail(CW_ERR_STATE, "every simulation of a batch must be bound");
  if (s->storage != ST_F32) return fail(CW_ERR_STATE, "batches take float32 storage");
  if (!vec_applies(s->nt, s->nz))
    return fail(CW_ERR_RANGE, "batches need nz a multiple of 4 and rings below 4 GiB (have %d x %d)", s->nt, s->nz);
  if (!b->sims.empty()) {
    const cw_sim *f = b->sims[0];
    if (s->device != f->device || s->stream != f->stream)
      return fail(CW_ERR_ARG, "the simulations of a batch must share one device and one stream");
    if (s->cur != f->cur) return fail(CW_ERR_STATE, "the simulations of a batch must have done steps of one parity");
  }
  return CW_OK;
}

cw_status cw_batch_create(cw_sim *const *sims, int32_t count, cw_batch **out)
{
  if (!sims || !out || count < 1 || count > 65535) return fail(CW_ERR_ARG, "need 1..65535 simulations");
  cw_batch *b = new (std::nothrow) cw_batch;
  if (!b) return fail(CW_ERR_NOMEM, "out of host memory");
  for (int q = 0; q < count; q++) {
    const cw_status st = check_batch_member(b, sims[q]);
    if (st != CW_OK) {
      delete b;
      return st;
    }
    b->sims.push_back(sims[q]);
    b->tz.push_back(4);
  }
  b->device = sims[0]->device;
  b->stream = sims[0]->stream;
  *out = b;
  return CW_OK;
}

void cw_batch_destroy(cw_batch *b) { delete b; }

cw_status cw_batch_set_tile(cw_batch *b, int32_t index, int32_t tz_waves)
{
  if (!b) return fail(CW_ERR_ARG, "null batch");
  if (b->bound) return fail(CW_ERR_STATE, "tile shapes are set before cw_batch_bind");
  if (index < 0 || index >= (int)b->sims.size()) return fail(CW_ERR_RANGE, "no instance %d", index);
  if (tz_waves != 1 && tz_waves != 2 && tz_waves != 4) return fail(CW_ERR_RANGE, "tile depth must be 1, 2 or 4 wavefronts");
  b->tz[index] = tz_waves;
  return CW_OK;
}

cw_status cw_batch_set_occupancy(cw_batch *b, int32_t waves_per_simd)
{
  if (!b) return fail(CW_ERR_ARG, "null batch");
  if (!batch_occupancy_supported(waves_per_simd))
    return fail(CW_ERR_RANGE, "waves per SIMD must be 0 (no constraint), 7 or 8 (have %d)", waves_per_simd);
  if (waves_per_simd != b->wpe) b->drop_graph();
  b->wpe = waves_per_simd;
  return CW_OK;
}

static size_t batch_bytes(const cw_batch *b)
{
  return align256(b->sims.size() * sizeof(BatchInst)) + align256(b->sims.size() * sizeof(long));
}

cw_status cw_batch_workspace_bytes(const cw_batch *b, uint64_t *bytes)
{
  if (!b || !bytes) return fail(CW_ERR_ARG, "null argument");
  *bytes = batch_bytes(b);
  return CW_OK;
}

cw_status cw_batch_bind(cw_batch *b, void *workspace, uint64_t bytes)
{
  if (!b || !workspace) return fail(CW_ERR_ARG, "null argument");
  if (b->bound) return fail(CW_ERR_STATE, "already bound");
  if ((uintptr_t)workspace & 255) return fail(CW_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < batch_bytes(b)) return fail(CW_ERR_RANGE, "workspace of %llu bytes, need %llu", (unsigned long long)bytes,
                                          (unsigned long long)batch_bytes(b));
  const int n = (int)b->sims.size();
  std::vector<BatchInst> h(n);
  std::vector<long> t0(n);
  long tiles = 0;
  for (int q = 0; q < n; q++) {
    const cw_sim *s = b->sims[q];
    BatchInst &I = h[q];
    I.a[0] = step_args(s, 0, 1);
    I.a[1] = step_args(s, 1, 0);
    const int w = b->tz[q], rows = 4 / w;
    I.tz_waves = w;
    I.nseg = (s->nz + 256 * w - 1) / (256 * w);
    I.tiles = (long)s->nr * ((s->nt + rows - 1) / rows) * I.nseg;
    I.tile0 = tiles;
    t0[q] = tiles;
    tiles += I.tiles;
    I.inject = s->d_inject; I.ninj = s->ninject;
    I.rec = s->d_rec; I.nrec = (int)s->receivers.size();
    I.cap = s->trace_cap; I.traces = s->d_traces; I.step = s->d_step;
    b->max_rec = std::max(b->max_rec, I.nrec);
    b->any_inject = b->any_inject || s->ninject > 0;
  }
  if (tiles > 0x7fffffff) return fail(CW_ERR_RANGE, "%ld workgroups exceed one launch", tiles);
  b->tiles = tiles;
  char *w = (char *)workspace;
  b->d_inst = (BatchInst *)w;
  b->d_tile0 = (long *)(w + align256(n * sizeof(BatchInst)));
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipMemcpy(b->d_inst, h.data(), n * sizeof(BatchInst), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b->d_tile0, t0.data(), n * sizeof(long), hipMemcpyHostToDevice));
  b->bound = true;
  return CW_OK;
}

cw_status cw_batch_set_graph(cw_batch *b, int32_t steps)
{
  if (!b) return fail(CW_ERR_ARG, "null batch");
  if (steps < 0 || steps % 2 || steps > kMaxGraphSteps)
    return fail(CW_ERR_RANGE, "graph steps must be even and in [0, %d] (have %d)", kMaxGraphSteps, steps);
  b->drop_graph();
  b->graph_steps = steps;
  return CW_OK;
}

// one batched step's launches on `stream` (parity = the instances' common buffer parity)
static cw_status batch_launches(cw_batch *b, int parity, hipStream_t stream)
{
  const int n = (int)b->sims.size();
  HIPCHK(launch_velocity_batch(b->d_inst, b->d_tile0, n, b->tiles, parity, b->wpe, stream));
  if (b->any_inject) HIPCHK(launch_inject_batch(b->d_inst, n, 0, parity, stream));
  HIPCHK(launch_stress_batch(b->d_inst, b->d_tile0, n, b->tiles, parity, b->wpe, stream));
  if (b->any_inject) HIPCHK(launch_inject_batch(b->d_inst, n, 1, parity, stream));
  HIPCHK(launch_record_batch(b->d_inst, n, b->max_rec, parity, stream));
  HIPCHK(launch_step_done_batch(b->d_inst, n, stream));
  return CW_OK;
}

cw_status cw_batch_step(cw_batch *b, int64_t nsteps)
{
  if (!b) return fail(CW_ERR_ARG, "null batch");
  if (!b->bound) return fail(CW_ERR_STATE, "cw_batch_bind first");
  if (nsteps < 0) return fail(CW_ERR_RANGE, "negative step count");
  cw_batch probe;
  for (cw_sim *s : b->sims) {
    cw_status st = check_batch_member(&probe, s);
    if (st != CW_OK) return st;
    if (s->cur != b->sims[0]->cur) return fail(CW_ERR_STATE, "the instances' buffer parities differ");
    if (!s->receivers.empty() && s->nstep + nsteps > s->trace_cap)
      return fail(CW_ERR_RANGE, "trace capacity %lld exceeded", (long long)s->trace_cap);
    probe.sims.push_back(s);
  }
  HIPCHK(hipSetDevice(b->device));
  cw_status st;
  auto advance = [&](int64_t k) {
    for (cw_sim *s : b->sims) {
      s->nstep += k;
      if (k & 1) s->cur = 1 - s->cur;
    }
  };
  int64_t done = 0;
  while (done < nsteps) {
    const int parity = b->sims[0]->cur;
    if (b->graph_steps > 0 && parity == 0 && nsteps - done >= b->graph_steps) {
      if (!b->graph_exec) {
        if (!b->capture_stream) HIPCHK(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        const hipError_t eb = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        cw_status cst = eb == hipSuccess ? CW_OK : fail(CW_ERR_HIP, "graph capture: %s", hipGetErrorString(eb));
        for (int g = 0; g < b->graph_steps && cst == CW_OK; g++) cst = batch_launches(b, g & 1, b->capture_stream);
        hipGraph_t gr = nullptr;
        const hipError_t ee = eb == hipSuccess ? hipStreamEndCapture(b->capture_stream, &gr) : hipSuccess;
        if (cst != CW_OK || ee != hipSuccess) {
          if (gr) (void)hipGraphDestroy(gr);
          return cst != CW_OK ? cst : fail(CW_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ee));
        }
        b->graph = gr;
        const hipError_t ei = hipGraphInstantiate(&b->graph_exec, gr, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
          b->drop_graph();
          return fail(CW_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
        }
      }
      HIPCHK(hipGraphLaunch(b->graph_exec, b->stream));
      done += b->graph_steps;
      advance(b->graph_steps);
      continue;
    }
    if ((st = batch_launches(b, parity, b->stream)) != CW_OK) return st;
    done++;
    advance(1);
  }
  return CW_OK;
}


// ---------------------------------------------------------------------------
// Azimuthally refined grid (Sec. 3): zones of rings whose azimuthal cell
// count doubles from one zone to the next.  Each zone is a simulation of its
// own (ring offset, ghost rings, the next zone's first medium ring); one
// batch steps them together, and before each half step a transfer launch
// fills every ghost ring with the neighbouring zone's edge ring on the
// zone's own azimuthal grid.

struct cw_refined {
  int nr = 0, nz = 0;
  double dr = 0, dz = 0;
  std::vector<int> first, nth;               // zone q: rings [first[q], first[q + 1]), nth[q] cells
  std::vector<cw_sim *> zones;
  cw_batch *batch = nullptr;
  std::vector<std::pair<int, int>> rec;      // receiver id -> (zone, id in the zone)
  bool bound = false;
  hipStream_t stream = nullptr;
  int device = 0;
  Transfer *d_tr[2][2] = {};                 // [parity][0: before the velocity, 1: before the stress update]
  int ntr[2][2] = {};
  float *d_mat = nullptr;
  int max_ns = 1;
  ~cw_refined()
  {
    delete batch;
    for (cw_sim *z : zones) delete z;
  }
  int zone_of(int i) const
  {
    int q = 0;
    while (q + 1 < (int)first.size() && first[q + 1] <= i) q++;
    return q;
  }
  int rings(int q) const { return (q + 1 < (int)first.size() ? first[q + 1] : nr) - first[q]; }
};

}  // extern "C"

namespace {

// Trigonometric interpolation kernel of n equispaced samples (the even-n
// Nyquist mode split evenly between +n/2 and -n/2): the interpolant through
// samples x_j at t_j is sum_j x_j D_n(t - t_j).
double dirichlet(int n, double t)
{
  double v = 1.0;
  for (int m = 1; 2 * m < n; m++) v += 2.0 * std::cos(m * t);
  if (n % 2 == 0) v += std::cos(0.5 * n * t);
  return v / n;
}

// Coarse (nc) -> fine (2 nc) interpolation matrix P [2 nc][nc] on integer
// (half = 0) or half-integer (half = 1) azimuthal nodes, float64.
std::vector<double> prolong_matrix(int nc, int half)
{
  const int nf = 2 * nc;
  const double s = half ? 0.5 : 0.0;
  std::vector<double> P((size_t)nf * nc);
  for (int jf = 0; jf < nf; jf++)
    for (int jc = 0; jc < nc; jc++)
      P[(size_t)jf * nc + jc] = dirichlet(nc, (jf + s) * 2.0 * kPi / nf - (jc + s) * 2.0 * kPi / nc);
  return P;
}

size_t refined_aux_floats(const cw_refined *r)
{
  size_t f = 0;
  for (size_t q = 1; q < r->nth.size(); q++) f += 4 * (size_t)r->nth[q - 1] * r->nth[q];
  return f;
}

size_t refined_bytes(const cw_refined *r, size_t *zone_bytes, size_t *batch_off, size_t *tr_off, size_t *mat_off)
{
  size_t off = 0;
  for (size_t q = 0; q < r->zones.size(); q++) {
    zone_bytes[q] = align256(layout(r->zones[q]).total);
    off += zone_bytes[q];
  }
  *batch_off = off;
  off += align256(r->zones.size() * sizeof(BatchInst)) + align256(r->zones.size() * sizeof(long));
  *tr_off = off;
  off += align256(4 * 4 * r->zones.size() * sizeof(Transfer));
  *mat_off = off;
  off += align256(refined_aux_floats(r) * sizeof(float));
  return off;
}

}  // namespace

extern "C" {

cw_status cw_refined_create(const cw_grid *g, int32_t nzones, const int32_t *first_ring, const int32_t *ntheta,
                            cw_refined **out)
{
  if (!g || !first_ring || !ntheta || !out) return fail(CW_ERR_ARG, "null argument");
  if (nzones < 1 || nzones > 32) return fail(CW_ERR_RANGE, "1..32 zones (have %d)", nzones);
  if (g->nr < 1 || g->nz < 4 || g->nz % 4) return fail(CW_ERR_RANGE, "need nr >= 1 and nz a positive multiple of 4");
  if (!(g->dr > 0) || !(g->dz > 0) || !std::isfinite(g->dr) || !std::isfinite(g->dz))
    return fail(CW_ERR_ARG, "cell sizes must be finite and > 0");
  if (first_ring[0] != 0) return fail(CW_ERR_RANGE, "the first zone starts at ring 0");
  for (int q = 0; q < nzones; q++) {
    if (ntheta[q] < 1) return fail(CW_ERR_RANGE, "zone %d: ntheta must be >= 1", q);
    if (q > 0 && (first_ring[q] <= first_ring[q - 1] || ntheta[q] != 2 * ntheta[q - 1]))
      return fail(CW_ERR_RANGE, "zone %d: zones start at increasing rings and double ntheta", q);
  }
  if (first_ring[nzones - 1] >= g->nr) return fail(CW_ERR_RANGE, "a zone starts beyond the last ring");
  if (ntheta[nzones - 1] != g->ntheta)
    return fail(CW_ERR_RANGE, "the outermost zone's ntheta (%d) must be the grid's (%d)", ntheta[nzones - 1], g->ntheta);
  if (interp_lds_bytes(g->ntheta) > 160 * 1024)
    return fail(CW_ERR_RANGE, "ntheta %d: the interpolation needs %zu bytes of LDS, above 160 KiB (ntheta <= 229)",
                g->ntheta, interp_lds_bytes(g->ntheta));
  if (!vec_applies(g->ntheta, g->nz))
    return fail(CW_ERR_RANGE, "a ring of %d x %d cells reaches 4 GiB (the zones' kernels address a ring with 32-bit offsets)",
                g->ntheta, g->nz);
  cw_refined *r = new (std::nothrow) cw_refined();
  if (!r) return fail(CW_ERR_NOMEM, "out of host memory");
  r->nr = g->nr; r->nz = g->nz; r->dr = g->dr; r->dz = g->dz;
  r->first.assign(first_ring, first_ring + nzones);
  r->nth.assign(ntheta, ntheta + nzones);
  for (int q = 0; q < nzones; q++) {
    cw_grid zg{r->rings(q), ntheta[q], g->nz, g->dr, g->dz};
    cw_sim *z = nullptr;
    const cw_status st = cw_create(&zg, &z);
    if (st != CW_OK) { delete r; return st; }
    z->ring0 = first_ring[q];
    z->ghost_in = q > 0;
    z->ghost_out = q + 1 < nzones;
    z->med_extra = q + 1 < nzones ? 1 : 0;
    r->zones.push_back(z);
  }
  *out = r;
  return CW_OK;
}

void cw_refined_destroy(cw_refined *r) { delete r; }

cw_status cw_refined_cells(const cw_refined *r, uint64_t *cells)
{
  if (!r || !cells) return fail(CW_ERR_ARG, "null argument");
  uint64_t c = 0;
  for (const cw_sim *z : r->zones) c += z->n;
  *cells = c;
  return CW_OK;
}

cw_status cw_refined_set_material_rz(cw_refined *r, const double *rho, const double *lam, const double *mu)
{
  if (!r || !rho || !lam || !mu) return fail(CW_ERR_ARG, "null argument");
  if (r->bound) return fail(CW_ERR_STATE, "configuration after cw_refined_bind");
  cw_status st;
  if ((st = check_medium((size_t)r->nr * r->nz, rho, lam, mu)) != CW_OK) return st;
  double vmax = 0;
  for (size_t p = 0; p < (size_t)r->nr * r->nz; p++) vmax = std::max(vmax, std::sqrt((lam[p] + 2 * mu[p]) / rho[p]));
  for (size_t q = 0; q < r->zones.size(); q++) {
    const size_t o = (size_t)r->first[q] * r->nz;
    if ((st = set_medium(r->zones[q], rho + o, lam + o, mu + o, true)) != CW_OK) return st;
    r->zones[q]->vp_ref = vmax;
  }
  return CW_OK;
}

cw_status cw_refined_set_pml(cw_refined *r, int32_t npml_r, int32_t npml_z, double rc, double alpha)
{
  if (!r) return fail(CW_ERR_ARG, "null argument");
  if (r->bound) return fail(CW_ERR_STATE, "configuration after cw_refined_bind");
  const int last = (int)r->zones.size() - 1;
  if (npml_r < 0 || npml_r >= r->rings(last))
    return fail(CW_ERR_RANGE, "the radial layer (%d rings) must lie inside the outermost zone (%d rings)", npml_r,
                r->rings(last));
  for (int q = 0; q <= last; q++) {
    const cw_status st = cw_set_pml(r->zones[q], q == last ? npml_r : 0, npml_z, rc, alpha);
    if (st != CW_OK) return st;
  }
  return CW_OK;
}

cw_status cw_refined_cfl_dt(const cw_refined *r, double *dt_cfl)
{
  if (!r || !dt_cfl) return fail(CW_ERR_ARG, "null argument");
  double best = INFINITY;
  for (const cw_sim *z : r->zones) {
    if (!z->have_material) return fail(CW_ERR_STATE, "medium not set");
    best = std::min(best, z->dt_cfl);
  }
  *dt_cfl = best;
  return CW_OK;
}

cw_status cw_refined_set_dt(cw_refined *r, double dt)
{
  if (!r) return fail(CW_ERR_ARG, "null argument");
  if (r->bound) return fail(CW_ERR_STATE, "configuration after cw_refined_bind");
  for (cw_sim *z : r->zones) {
    const cw_status st = cw_set_dt(z, dt);
    if (st != CW_OK) return st;
  }
  return CW_OK;
}

cw_status cw_refined_add_source(cw_refined *r, int32_t kind, int32_t i, int32_t j, int32_t k, const double *w,
                                int64_t n)
{
  if (!r) return fail(CW_ERR_ARG, "null argument");
  if (r->bound) return fail(CW_ERR_STATE, "configuration after cw_refined_bind");
  if (i < 0 || i >= r->nr) return fail(CW_ERR_RANGE, "source ring %d outside the grid", i);
  const int q = r->zone_of(i);
  return cw_add_source(r->zones[q], kind, i - r->first[q], j, k, w, n);
}

cw_status cw_refined_add_receiver(cw_refined *r, int32_t kind, int32_t field, int32_t i, int32_t j, int32_t k,
                                  int32_t *id)
{
  if (!r) return fail(CW_ERR_ARG, "null argument");
  if (r->bound) return fail(CW_ERR_STATE, "configuration after cw_refined_bind");
  if (i < 0 || i >= r->nr) return fail(CW_ERR_RANGE, "receiver ring %d outside the grid", i);
  const int q = r->zone_of(i);
  int32_t lid = 0;
  const cw_status st = cw_add_receiver(r->zones[q], kind, field, i - r->first[q], j, k, &lid);
  if (st != CW_OK) return st;
  r->rec.emplace_back(q, lid);
  if (id) *id = (int32_t)r->rec.size() - 1;
  return CW_OK;
}

cw_status cw_refined_set_trace_capacity(cw_refined *r, int64_t nsteps)
{
  if (!r) return fail(CW_ERR_ARG, "null argument");
  for (cw_sim *z : r->zones) {
    const cw_status st = cw_set_trace_capacity(z, nsteps);
    if (st != CW_OK) return st;
  }
  return CW_OK;
}

cw_status cw_refined_workspace_bytes(const cw_refined *r, uint64_t *bytes)
{
  if (!r || !bytes) return fail(CW_ERR_ARG, "null argument");
  std::vector<size_t> zb(r->zones.size());
  size_t b, t, m;
  *bytes = refined_bytes(r, zb.data(), &b, &t, &m);
  return CW_OK;
}

cw_status cw_refined_bind(cw_refined *r, void *workspace, uint64_t bytes, void *stream)
{
  if (!r || !workspace) return fail(CW_ERR_ARG, "null argument");
  if (r->bound) return fail(CW_ERR_STATE, "already bound");
  if ((uintptr_t)workspace & 255) return fail(CW_ERR_ARG, "workspace not 256-byte aligned");
  const int nzn = (int)r->zones.size();
  std::vector<size_t> zb(nzn);
  size_t boff, troff, moff;
  const size_t need = refined_bytes(r, zb.data(), &boff, &troff, &moff);
  if (bytes < need)
    return fail(CW_ERR_NOMEM, "workspace of %llu bytes, need %llu", (unsigned long long)bytes, (unsigned long long)need);
  char *w = (char *)workspace;
  size_t off = 0;
  cw_status st;
  for (int q = 0; q < nzn; q++) {
    if ((st = cw_bind(r->zones[q], w + off, zb[q], stream)) != CW_OK) return st;
    off += zb[q];
  }
  r->stream = (hipStream_t)stream;
  r->device = r->zones[0]->device;
  if ((st = cw_batch_create(r->zones.data(), nzn, &r->batch)) != CW_OK) return st;
  if ((st = cw_batch_bind(r->batch, w + boff, troff - boff)) != CW_OK) return st;

  // interpolation matrices per interface: P_int, P_half [nf][nc], R_int, R_half [nc][nf] (R = P^T / 2)
  std::vector<float> mats(refined_aux_floats(r));
  std::vector<size_t> mo(nzn, 0);
  size_t mp = 0;
  for (int q = 1; q < nzn; q++) {
    const int nc = r->nth[q - 1], nf = r->nth[q];
    mo[q] = mp;
    for (int half = 0; half < 2; half++) {
      const std::vector<double> P = prolong_matrix(nc, half);
      float *Pm = mats.data() + mp + (size_t)half * nf * nc;
      float *Rm = mats.data() + mp + (size_t)(2 + half) * nf * nc;
      for (int jf = 0; jf < nf; jf++)
        for (int jc = 0; jc < nc; jc++) {
          Pm[(size_t)jf * nc + jc] = (float)P[(size_t)jf * nc + jc];
          Rm[(size_t)jc * nf + jf] = (float)(0.5 * P[(size_t)jf * nc + jc]);
        }
    }
    mp += 4 * (size_t)nf * nc;
  }
  r->d_mat = (float *)(w + moff);
  // transfers: for parity p, the state is in fields[p] (stresses at level n)
  // and the velocities of level n+1/2 go to fields[1 - p]
  Transfer *dtr = (Transfer *)(w + troff);
  std::vector<Transfer> h[2][2];
  r->max_ns = 1;
  for (int p = 0; p < 2; p++)
    for (int q = 1; q < nzn; q++) {
      const cw_sim *C = r->zones[q - 1], *F = r->zones[q];
      const int nc = r->nth[q - 1], nf = r->nth[q];
      const size_t cring = C->rs(), fring = F->rs();   // ring strides of the two zones' field arrays
      const float *Pint = r->d_mat + mo[q], *Phalf = Pint + (size_t)nf * nc;
      const float *Rint = Pint + 2 * (size_t)nf * nc, *Rhalf = Pint + 3 * (size_t)nf * nc;
      auto c_last = [&](int b, int f) { return C->fields[b][f] + (size_t)(C->nr - 1) * cring; };
      auto c_ghost = [&](int b, int f) { return C->fields[b][f] + (size_t)C->nr * cring; };
      auto f_first = [&](int b, int f) { return F->fields[b][f]; };
      auto f_ghost = [&](int b, int f) { return F->fields[b][f] - fring; };
      // before the velocity update: sigma_rr, sigma_tt of the fine ring for the coarse
      // zone's v_r; sigma_rt, sigma_rz of the coarse ring for the fine zone's v_t, v_z
      h[p][0].push_back({f_first(p, SRR), c_ghost(p, SRR), Rint, nf, nc});
      h[p][0].push_back({f_first(p, STT), c_ghost(p, STT), Rint, nf, nc});
      h[p][0].push_back({c_last(p, SRT), f_ghost(p, SRT), Phalf, nc, nf});
      h[p][0].push_back({c_last(p, SRZ), f_ghost(p, SRZ), Pint, nc, nf});
      // before the stress update: v_r of the coarse ring for the fine zone's normal
      // stresses; v_t, v_z of the fine ring for the coarse zone's sigma_rt, sigma_rz
      h[p][1].push_back({c_last(1 - p, VR), f_ghost(1 - p, VR), Pint, nc, nf});
      h[p][1].push_back({f_first(1 - p, VT), c_ghost(1 - p, VT), Rhalf, nf, nc});
      h[p][1].push_back({f_first(1 - p, VZ), c_ghost(1 - p, VZ), Rint, nf, nc});
      r->max_ns = std::max(r->max_ns, nf);
    }
  HIPCHK(hipSetDevice(r->device));
  size_t to = 0;
  for (int p = 0; p < 2; p++)
    for (int ph = 0; ph < 2; ph++) {
      r->d_tr[p][ph] = dtr + to;
      r->ntr[p][ph] = (int)h[p][ph].size();
      if (!h[p][ph].empty())
        HIPCHK(hipMemcpy(dtr + to, h[p][ph].data(), h[p][ph].size() * sizeof(Transfer), hipMemcpyHostToDevice));
      to += h[p][ph].size();
    }
  if (!mats.empty()) HIPCHK(hipMemcpy(r->d_mat, mats.data(), mats.size() * sizeof(float), hipMemcpyHostToDevice));
  r->bound = true;
  return CW_OK;
}

cw_status cw_refined_step(cw_refined *r, int64_t nsteps)
{
  if (!r) return fail(CW_ERR_ARG, "null argument");
  if (!r->bound) return fail(CW_ERR_STATE, "cw_refined_bind first");
  if (nsteps < 0) return fail(CW_ERR_RANGE, "negative step count");
  for (cw_sim *z : r->zones)
    if (!z->receivers.empty() && z->nstep + nsteps > z->trace_cap)
      return fail(CW_ERR_RANGE, "trace capacity %lld exceeded", (long long)z->trace_cap);
  HIPCHK(hipSetDevice(r->device));
  cw_batch *b = r->batch;
  const int n = (int)r->zones.size();
  for (int64_t t = 0; t < nsteps; t++) {
    const int p = r->zones[0]->cur;
    HIPCHK(launch_interp(r->d_tr[p][0], r->ntr[p][0], r->nz, r->max_ns, r->stream));
    HIPCHK(launch_velocity_batch(b->d_inst, b->d_tile0, n, b->tiles, p, b->wpe, r->stream));
    if (b->any_inject) HIPCHK(launch_inject_batch(b->d_inst, n, 0, p, r->stream));
    HIPCHK(launch_interp(r->d_tr[p][1], r->ntr[p][1], r->nz, r->max_ns, r->stream));
    HIPCHK(launch_stress_batch(b->d_inst, b->d_tile0, n, b->tiles, p, b->wpe, r->stream));
    if (b->any_inject) HIPCHK(launch_inject_batch(b->d_inst, n, 1, p, r->stream));
    HIPCHK(launch_record_batch(b->d_inst, n, b->max_rec, p, r->stream));
    HIPCHK(launch_step_done_batch(b->d_inst, n, r->stream));
    for (cw_sim *z : r->zones) {
      z->nstep++;
      z->cur = 1 - z->cur;
    }
  }
  return CW_OK;
}

cw_status cw_refined_get_field(cw_refined *r, int32_t field, float *host_out)
{
  if (!r || !host_out) return fail(CW_ERR_ARG, "null argument");
  size_t off = 0;
  for (cw_sim *z : r->zones) {
    const cw_status st = cw_get_field(z, field, host_out + off);
    if (st != CW_OK) return st;
    off += z->n;
  }
  return CW_OK;
}

cw_status cw_refined_set_field(cw_refined *r, int32_t field, const float *host_in)
{
  if (!r || !host_in) return fail(CW_ERR_ARG, "null argument");
  size_t off = 0;
  for (cw_sim *z : r->zones) {
    const cw_status st = cw_set_field(z, field, host_in + off);
    if (st != CW_OK) return st;
    off += z->n;
  }
  return CW_OK;
}

cw_status cw_refined_get_traces(cw_refined *r, double *out, int64_t cap, int64_t *nsteps_done)
{
  if (!r || (!out && !r->rec.empty())) return fail(CW_ERR_ARG, "null argument");
  if (!r->bound) return fail(CW_ERR_STATE, "cw_refined_bind first");
  const int64_t done = r->zones[0]->nstep;
  if (cap < done) return fail(CW_ERR_RANGE, "cap %lld < steps done %lld", (long long)cap, (long long)done);
  if (nsteps_done) *nsteps_done = done;
  std::vector<double> buf;
  for (size_t q = 0; q < r->zones.size(); q++) {
    cw_sim *z = r->zones[q];
    if (z->receivers.empty()) continue;
    buf.assign(z->receivers.size() * (size_t)cap, 0.0);
    const cw_status st = cw_get_traces(z, buf.data(), cap, nullptr);
    if (st != CW_OK) return st;
    for (size_t m = 0; m < r->rec.size(); m++)
      if (r->rec[m].first == (int)q)
        std::memcpy(out + m * (size_t)cap, buf.data() + (size_t)r->rec[m].second * cap, (size_t)done * sizeof(double));
  }
  return CW_OK;
}

cw_status cw_refined_energy(cw_refined *r, double *E)
{
  if (!r || !E) return fail(CW_ERR_ARG, "null argument");
  double sum = 0;
  for (cw_sim *z : r->zones) {
    double e = 0;
    const cw_status st = cw_energy(z, &e);
    if (st != CW_OK) return st;
    sum += e;
  }
  *E = sum;
  return CW_OK;
}

cw_status cw_refined_reset(cw_refined *r)
{
  if (!r) return fail(CW_ERR_ARG, "null argument");
  for (cw_sim *z : r->zones) {
    const cw_status st = cw_reset(z);
    if (st != CW_OK) return st;
  }
  return CW_OK;
}

}  // extern "C"
