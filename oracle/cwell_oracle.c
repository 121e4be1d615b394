/*
 * cwell_oracle.c -- plain, slow FP64 CPU reference of the cased-well time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link
 * or call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or table with the HIP path.
 *
 * What it computes (Cheverda et al., "Parallel Modeling of the Acoustic Signal
 * Propagation in a Cased Well", arXiv 2302.13907):
 *
 *   Eq. (1), the first-order velocity-stress system of dynamic elasticity in
 *   cylindrical coordinates (r, theta, z), written out component by component
 *   from the matrices A, B, C, D (Sec. 2) with the stress vector ordered
 *   (s_rr, s_tt, s_zz, s_rt, s_tz, s_rz) as those matrices imply, in the
 *   stiffness form (the compliance M of Sec. 2 is singular in the fluid, where
 *   the shear modulus is set to zero, Sec. 2 last paragraph before the sources).
 *
 *   Space: the staggered grid of Virieux adapted to cylindrical coordinates,
 *   material attached to the cell centre (Sec. 3).  Placement:
 *       s_rr, s_tt, s_zz : (r_i,     th_j,     z_k)
 *       v_r              : (R_i,     th_j,     z_k)
 *       v_t              : (r_i,     th_j+1/2, z_k)
 *       v_z              : (r_i,     th_j,     z_k+1/2)
 *       s_rt             : (R_i,     th_j+1/2, z_k)
 *       s_rz             : (R_i,     th_j,     z_k+1/2)
 *       s_tz             : (r_i,     th_j+1/2, z_k+1/2)
 *   with r_i = (i+1/2) dr, R_i = (i+1) dr, th_j = j dth, dth = 2 pi / Nt,
 *   z_k = k dz.  Every field lives on the same Nr x Nt x Nz index space,
 *   C order [i][j][k].  theta is periodic; any value with i or k outside the
 *   grid reads as zero (this closes the axis r = 0 and the outer faces).
 *
 *   Time: explicit leapfrog (Sec. 4 calls the scheme explicit): v at half
 *   steps, stress at whole steps, zero initial data (Eq. (2)).
 *
 *   Absorbing layer: an unsplit convolutional PML in r and z only, theta is
 *   never stretched (Sec. 1 and Sec. 6: the layer does not split variables
 *   in azimuth).  d/dr -> (1/s_r) d/dr and every 1/r -> 1/(r s~_r) with
 *   s~_r built from the integrated profile; d/dz -> (1/s_z) d/dz.  Each
 *   stretched term X is replaced by X + psi with psi <- b psi + a X.
 *
 *   Sources: the four kinds of Sec. 2 (volumetric, transverse force,
 *   longitudinal force, torsion), injected with unit strength per unit
 *   volume; the wavelet samples are an input array (the Ricker pulse of
 *   Sec. 2 is provided separately by orc_ricker).
 *
 *   Adjoint: the transpose of the step, obtained by reversing each of its
 *   statements (every read becomes a scattered add), and from it the
 *   gradient of a receiver loss with respect to the moduli of a region
 *   (orc_gradient): forward run storing the region's strains, then the
 *   adjoint steps back from the last one, each adding the derivative of the
 *   stress update with respect to lambda and mu (through the harmonic means
 *   at the shear nodes) times the stress adjoints.
 *
 * Memory variables are stored on the full grid here (zero outside the layer),
 * which is wasteful but plainly correct.
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared -fopenmp -ffp-contract=off
 *        (no fast-math: IEEE FP64 throughout).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* field identifiers */
enum { VR, VT, VZ, SRR, STT, SZZ, SRT, SRZ, STZ, NFIELD };
/* source kinds (Sec. 2) */
enum { SRC_VOLUME, SRC_FORCE_R, SRC_FORCE_Z, SRC_TORSION };
/* receiver kinds */
enum { REC_PRESSURE, REC_FIELD };
/* memory variables: which node, which stretched term */
enum {
  P_VR_DR, P_VR_B, P_VR_DZ,
  P_VT_DR, P_VT_B, P_VT_DZ,
  P_VZ_DR, P_VZ_B, P_VZ_DZ,
  P_N_DR, P_N_B, P_N_DZ,
  P_RT_DR, P_RT_B,
  P_RZ_DR, P_RZ_DZ,
  P_TZ_B, P_TZ_DZ,
  NPSI
};

typedef struct { int kind, i, j, k; double *w; long ns; } orc_src;
typedef struct { int kind, field, i, j, k; } orc_rec;

typedef struct orc {
  int nr, nt, nz;
  double dr, dz, dth, dt;
  size_t n;
  double *f[NFIELD];
  double *rho, *lam, *mu;
  /* staggered coefficients: buoyancies and effective shear moduli */
  double *b_r, *b_t, *b_z, *mu_rt, *mu_rz, *mu_tz;
  int have_material;
  /* absorbing layer */
  int npr, npz;
  double rc, alpha;
  double *psi[NPSI];
  /* 1-D coefficient tables: radial profile at centres (c) and faces (f),
     integrated radial profile at centres and faces, z profile at whole (c)
     and half (h) positions */
  double *ar_c, *br_c, *ar_f, *br_f, *at_c, *bt_c, *at_f, *bt_f;
  double *az_c, *bz_c, *az_h, *bz_h;
  /* sources and receivers */
  orc_src *src; int nsrc;
  orc_rec *rec; int nrec;
  long nstep;
} orc;

static size_t IDX(const orc *s, int i, int j, int k)
{
  return ((size_t)i * s->nt + j) * s->nz + k;
}

/* zero outside [0,nr) x [0,nz); periodic in theta */
static double at(const orc *s, const double *a, int i, int j, int k)
{
  if (i < 0 || i >= s->nr || k < 0 || k >= s->nz) return 0.0;
  j = ((j % s->nt) + s->nt) % s->nt;
  return a[IDX(s, i, j, k)];
}

static double rc_(const orc *s, int i) { return (i + 0.5) * s->dr; } /* r_i */
static double rf_(const orc *s, int i) { return (i + 1.0) * s->dr; } /* R_i */

/* ------------------------------------------------------------------ */
orc *orc_create(int nr, int nt, int nz, double dr, double dz)
{
  if (nr < 1 || nt < 1 || nz < 1 || !(dr > 0) || !(dz > 0)) return NULL;
  orc *s = (orc *)calloc(1, sizeof(orc));
  s->nr = nr; s->nt = nt; s->nz = nz; s->dr = dr; s->dz = dz;
  s->dth = 2.0 * M_PI / nt;
  s->n = (size_t)nr * nt * nz;
  for (int q = 0; q < NFIELD; q++) s->f[q] = (double *)calloc(s->n, sizeof(double));
  s->rho = (double *)calloc(s->n, sizeof(double));
  s->lam = (double *)calloc(s->n, sizeof(double));
  s->mu = (double *)calloc(s->n, sizeof(double));
  s->b_r = (double *)calloc(s->n, sizeof(double));
  s->b_t = (double *)calloc(s->n, sizeof(double));
  s->b_z = (double *)calloc(s->n, sizeof(double));
  s->mu_rt = (double *)calloc(s->n, sizeof(double));
  s->mu_rz = (double *)calloc(s->n, sizeof(double));
  s->mu_tz = (double *)calloc(s->n, sizeof(double));
  return s;
}

static void free_pml(orc *s)
{
  for (int q = 0; q < NPSI; q++) { free(s->psi[q]); s->psi[q] = NULL; }
  double **t[] = {&s->ar_c, &s->br_c, &s->ar_f, &s->br_f, &s->at_c, &s->bt_c,
                  &s->at_f, &s->bt_f, &s->az_c, &s->bz_c, &s->az_h, &s->bz_h};
  for (size_t q = 0; q < sizeof(t) / sizeof(t[0]); q++) { free(*t[q]); *t[q] = NULL; }
}

void orc_free(orc *s)
{
  if (!s) return;
  for (int q = 0; q < NFIELD; q++) free(s->f[q]);
  free(s->rho); free(s->lam); free(s->mu);
  free(s->b_r); free(s->b_t); free(s->b_z);
  free(s->mu_rt); free(s->mu_rz); free(s->mu_tz);
  free_pml(s);
  for (int q = 0; q < s->nsrc; q++) free(s->src[q].w);
  free(s->src); free(s->rec);
  free(s);
}

/* Harmonic mean of four moduli; zero as soon as one of them is zero, so a
   shear node touching the fluid carries no shear stress. */
static double hm4(double a, double b, double c, double d)
{
  if (a == 0.0 || b == 0.0 || c == 0.0 || d == 0.0) return 0.0;
  return 4.0 / (1.0 / a + 1.0 / b + 1.0 / c + 1.0 / d);
}

/* Material at the cell centre (Sec. 3).  Staggered nodes take the arithmetic
   mean of the two adjacent densities and the harmonic mean of the four
   adjacent shear moduli; beyond the last cell in r or z the neighbour index
   is clamped, theta wraps. */
int orc_set_material(orc *s, const double *rho, const double *lam, const double *mu)
{
  for (size_t p = 0; p < s->n; p++) {
    if (!(rho[p] > 0) || !(mu[p] >= 0) || !(lam[p] + 2.0 * mu[p] > 0) ||
        !isfinite(rho[p]) || !isfinite(lam[p]) || !isfinite(mu[p]))
      return -3;
  }
  memcpy(s->rho, rho, s->n * sizeof(double));
  memcpy(s->lam, lam, s->n * sizeof(double));
  memcpy(s->mu, mu, s->n * sizeof(double));
  for (int i = 0; i < s->nr; i++) {
    int i1 = i + 1 < s->nr ? i + 1 : s->nr - 1;
    for (int j = 0; j < s->nt; j++) {
      int j1 = (j + 1) % s->nt;
      for (int k = 0; k < s->nz; k++) {
        int k1 = k + 1 < s->nz ? k + 1 : s->nz - 1;
        size_t p = IDX(s, i, j, k);
        s->b_r[p] = 2.0 / (rho[p] + rho[IDX(s, i1, j, k)]);
        s->b_t[p] = 2.0 / (rho[p] + rho[IDX(s, i, j1, k)]);
        s->b_z[p] = 2.0 / (rho[p] + rho[IDX(s, i, j, k1)]);
        s->mu_rt[p] = hm4(mu[p], mu[IDX(s, i1, j, k)], mu[IDX(s, i, j1, k)], mu[IDX(s, i1, j1, k)]);
        s->mu_rz[p] = hm4(mu[p], mu[IDX(s, i1, j, k)], mu[IDX(s, i, j, k1)], mu[IDX(s, i1, j, k1)]);
        s->mu_tz[p] = hm4(mu[p], mu[IDX(s, i, j1, k)], mu[IDX(s, i, j, k1)], mu[IDX(s, i, j1, k1)]);
      }
    }
  }
  s->have_material = 1;
  return 0;
}

double orc_vpmax(const orc *s)
{
  double vmax = 0.0;
  for (size_t p = 0; p < s->n; p++) {
    double vp = sqrt((s->lam[p] + 2.0 * s->mu[p]) / s->rho[p]);
    if (vp > vmax) vmax = vp;
  }
  return vmax;
}

/* Courant limit over the cell centres, with the azimuthal cell width r_i dth
   (smallest next to the axis). */
double orc_cfl_dt(const orc *s)
{
  double best = INFINITY;
  for (int i = 0; i < s->nr; i++) {
    double ra = rc_(s, i) * s->dth;
    double g = sqrt(1.0 / (s->dr * s->dr) + 1.0 / (ra * ra) + 1.0 / (s->dz * s->dz));
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        double vp = sqrt((s->lam[p] + 2.0 * s->mu[p]) / s->rho[p]);
        double t = 1.0 / (vp * g);
        if (t < best) best = t;
      }
  }
  return best;
}

/* Ricker pulse of Sec. 2 with the printed delay 2/f0. */
double orc_ricker(double f0, double t)
{
  double tau = t - 2.0 / f0;
  double a = M_PI * M_PI * f0 * f0 * tau * tau;
  return (1.0 - 2.0 * a) * exp(-a);
}

/* ---------------------------- absorbing layer ---------------------- */
static void pml_coef(double d, double alpha, double dt, double *a, double *b)
{
  *b = exp(-(d + alpha) * dt);
  *a = d > 0.0 ? d * (*b - 1.0) / (d + alpha) : 0.0;
}

static void build_pml_tables(orc *s)
{
  double vpm = orc_vpmax(s);
  double Lr = s->npr * s->dr, Lz = s->npz * s->dz;
  double d0r = s->npr > 0 ? -3.0 * vpm * log(s->rc) / (2.0 * Lr) : 0.0;
  double d0z = s->npz > 0 ? -3.0 * vpm * log(s->rc) / (2.0 * Lz) : 0.0;
  double rp = (s->nr - s->npr) * s->dr;
  for (int i = 0; i < s->nr; i++) {
    double rr[2] = {rc_(s, i), rf_(s, i)};
    for (int w = 0; w < 2; w++) {
      double r = rr[w];
      double x = 0.0;
      if (s->npr > 0 && r > rp) x = (r - rp) / Lr;
      double d = d0r * x * x;
      double dtl = s->npr > 0 ? d0r * Lr * x * x * x / (3.0 * r) : 0.0;
      if (w == 0) {
        pml_coef(d, s->alpha, s->dt, &s->ar_c[i], &s->br_c[i]);
        pml_coef(dtl, s->alpha, s->dt, &s->at_c[i], &s->bt_c[i]);
      } else {
        pml_coef(d, s->alpha, s->dt, &s->ar_f[i], &s->br_f[i]);
        pml_coef(dtl, s->alpha, s->dt, &s->at_f[i], &s->bt_f[i]);
      }
    }
  }
  for (int k = 0; k < s->nz; k++) {
    double zz[2] = {k * s->dz, (k + 0.5) * s->dz};
    for (int w = 0; w < 2; w++) {
      double z = zz[w], x = 0.0;
      if (s->npz > 0) {
        double x1 = (s->npz * s->dz - z) / Lz;
        double x2 = (z - (s->nz - 1 - s->npz) * s->dz) / Lz;
        x = x1 > x2 ? x1 : x2;
        if (x < 0) x = 0;
      }
      double d = d0z * x * x;
      if (w == 0) pml_coef(d, s->alpha, s->dt, &s->az_c[k], &s->bz_c[k]);
      else pml_coef(d, s->alpha, s->dt, &s->az_h[k], &s->bz_h[k]);
    }
  }
}

/* npr / npz cells of layer in r (outer side) and z (both ends); rc is the
   target reflection coefficient, alpha the constant frequency shift.
   npr = npz = 0 switches the layer off.  Must precede orc_set_dt. */
int orc_set_pml(orc *s, int npr, int npz, double rc, double alpha)
{
  if (npr < 0 || npz < 0 || npr >= s->nr || (npz > 0 && 2 * npz + 2 > s->nz)) return -2;
  if ((npr > 0 || npz > 0) && !(rc > 0 && rc < 1 && alpha >= 0)) return -1;
  free_pml(s);
  s->npr = npr; s->npz = npz; s->rc = rc; s->alpha = alpha;
  if (npr == 0 && npz == 0) return 0;
  for (int q = 0; q < NPSI; q++) s->psi[q] = (double *)calloc(s->n, sizeof(double));
  double **t[] = {&s->ar_c, &s->br_c, &s->ar_f, &s->br_f, &s->at_c, &s->bt_c, &s->at_f, &s->bt_f};
  for (int q = 0; q < 8; q++) *t[q] = (double *)calloc(s->nr, sizeof(double));
  s->az_c = (double *)calloc(s->nz, sizeof(double));
  s->bz_c = (double *)calloc(s->nz, sizeof(double));
  s->az_h = (double *)calloc(s->nz, sizeof(double));
  s->bz_h = (double *)calloc(s->nz, sizeof(double));
  return 0;
}

int orc_set_dt(orc *s, double dt)
{
  if (!s->have_material || !(dt > 0)) return -5;
  s->dt = dt;
  if (s->psi[0]) build_pml_tables(s);
  return 0;
}

/* ------------------------- spatial operators ----------------------- */
/* Each velocity right-hand side is split into a radial-derivative part Dr,
   the 1/r bracket B (azimuthal derivative and curvature terms) and a
   z-derivative part Dz: the layer stretches each part separately. */

/* rho dv_r/dt = ds_rr/dr + (1/r)(ds_rt/dth + s_rr - s_tt) + ds_rz/dz, at (R_i, th_j, z_k) */
static void vr_parts(const orc *s, int i, int j, int k, double *Dr, double *B, double *Dz)
{
  const double *srr = s->f[SRR], *stt = s->f[STT], *srt = s->f[SRT], *srz = s->f[SRZ];
  *Dr = (at(s, srr, i + 1, j, k) - at(s, srr, i, j, k)) / s->dr;
  *B = (1.0 / rf_(s, i)) *
       ((at(s, srt, i, j, k) - at(s, srt, i, j - 1, k)) / s->dth
        + 0.5 * (at(s, srr, i + 1, j, k) + at(s, srr, i, j, k))
        - 0.5 * (at(s, stt, i + 1, j, k) + at(s, stt, i, j, k)));
  *Dz = (at(s, srz, i, j, k) - at(s, srz, i, j, k - 1)) / s->dz;
}

/* rho dv_t/dt = ds_rt/dr + (1/r)(ds_tt/dth + 2 s_rt) + ds_tz/dz, at (r_i, th_j+1/2, z_k) */
static void vt_parts(const orc *s, int i, int j, int k, double *Dr, double *B, double *Dz)
{
  const double *stt = s->f[STT], *srt = s->f[SRT], *stz = s->f[STZ];
  *Dr = (at(s, srt, i, j, k) - at(s, srt, i - 1, j, k)) / s->dr;
  *B = (1.0 / rc_(s, i)) *
       ((at(s, stt, i, j + 1, k) - at(s, stt, i, j, k)) / s->dth
        + (at(s, srt, i, j, k) + at(s, srt, i - 1, j, k)));
  *Dz = (at(s, stz, i, j, k) - at(s, stz, i, j, k - 1)) / s->dz;
}

/* rho dv_z/dt = ds_rz/dr + (1/r)(ds_tz/dth + s_rz) + ds_zz/dz, at (r_i, th_j, z_k+1/2) */
static void vz_parts(const orc *s, int i, int j, int k, double *Dr, double *B, double *Dz)
{
  const double *szz = s->f[SZZ], *srz = s->f[SRZ], *stz = s->f[STZ];
  *Dr = (at(s, srz, i, j, k) - at(s, srz, i - 1, j, k)) / s->dr;
  *B = (1.0 / rc_(s, i)) *
       ((at(s, stz, i, j, k) - at(s, stz, i, j - 1, k)) / s->dth
        + 0.5 * (at(s, srz, i, j, k) + at(s, srz, i - 1, j, k)));
  *Dz = (at(s, szz, i, j, k + 1) - at(s, szz, i, j, k)) / s->dz;
}

/* strain rates at the centre: e_rr = dv_r/dr, e_tt = (1/r)(dv_t/dth + v_r),
   e_zz = dv_z/dz */
static void n_parts(const orc *s, int i, int j, int k, double *err, double *ett, double *ezz)
{
  const double *vr = s->f[VR], *vt = s->f[VT], *vz = s->f[VZ];
  *err = (at(s, vr, i, j, k) - at(s, vr, i - 1, j, k)) / s->dr;
  *ett = (1.0 / rc_(s, i)) *
         ((at(s, vt, i, j, k) - at(s, vt, i, j - 1, k)) / s->dth
          + 0.5 * (at(s, vr, i, j, k) + at(s, vr, i - 1, j, k)));
  *ezz = (at(s, vz, i, j, k) - at(s, vz, i, j, k - 1)) / s->dz;
}

/* g_rt = dv_t/dr + (1/r)(dv_r/dth - v_t), at (R_i, th_j+1/2, z_k) */
static void rt_parts(const orc *s, int i, int j, int k, double *Dr, double *B)
{
  const double *vr = s->f[VR], *vt = s->f[VT];
  *Dr = (at(s, vt, i + 1, j, k) - at(s, vt, i, j, k)) / s->dr;
  *B = (1.0 / rf_(s, i)) *
       ((at(s, vr, i, j + 1, k) - at(s, vr, i, j, k)) / s->dth
        - 0.5 * (at(s, vt, i + 1, j, k) + at(s, vt, i, j, k)));
}

/* g_rz = dv_z/dr + dv_r/dz, at (R_i, th_j, z_k+1/2) */
static void rz_parts(const orc *s, int i, int j, int k, double *Dr, double *Dz)
{
  const double *vr = s->f[VR], *vz = s->f[VZ];
  *Dr = (at(s, vz, i + 1, j, k) - at(s, vz, i, j, k)) / s->dr;
  *Dz = (at(s, vr, i, j, k + 1) - at(s, vr, i, j, k)) / s->dz;
}

/* g_tz = (1/r) dv_z/dth + dv_t/dz, at (r_i, th_j+1/2, z_k+1/2) */
static void tz_parts(const orc *s, int i, int j, int k, double *B, double *Dz)
{
  const double *vt = s->f[VT], *vz = s->f[VZ];
  *B = (1.0 / rc_(s, i)) * (at(s, vz, i, j + 1, k) - at(s, vz, i, j, k)) / s->dth;
  *Dz = (at(s, vt, i, j, k + 1) - at(s, vt, i, j, k)) / s->dz;
}

/* psi <- b psi + a X ; returns X + psi.  With the layer off, returns X. */
static double stretch(orc *s, int q, size_t p, double a, double b, double X)
{
  if (!s->psi[0]) return X;
  s->psi[q][p] = b * s->psi[q][p] + a * X;
  return X + s->psi[q][p];
}

/* Operators exposed for the checks: the divergence part of the velocity
   equations (right-hand sides without density, source or layer) applied to
   the stress fields given in sig[6] (order s_rr, s_tt, s_zz, s_rt, s_rz,
   s_tz), and the strain rates (e_rr, e_tt, e_zz, g_rt, g_rz, g_tz) of the
   velocity fields in vel[3].  The current state is saved and restored. */
void orc_apply_div(orc *s, double *const sig[6], double *out[3])
{
  double *save[6];
  for (int q = 0; q < 6; q++) { save[q] = s->f[SRR + q]; s->f[SRR + q] = sig[q]; }
  for (int i = 0; i < s->nr; i++)
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        double a, b, c;
        vr_parts(s, i, j, k, &a, &b, &c); out[0][p] = a + b + c;
        vt_parts(s, i, j, k, &a, &b, &c); out[1][p] = a + b + c;
        vz_parts(s, i, j, k, &a, &b, &c); out[2][p] = a + b + c;
      }
  for (int q = 0; q < 6; q++) s->f[SRR + q] = save[q];
}

void orc_apply_strain(orc *s, double *const vel[3], double *out[6])
{
  double *save[3];
  for (int q = 0; q < 3; q++) { save[q] = s->f[VR + q]; s->f[VR + q] = vel[q]; }
  for (int i = 0; i < s->nr; i++)
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        double a, b, c;
        n_parts(s, i, j, k, &a, &b, &c);
        out[0][p] = a; out[1][p] = b; out[2][p] = c;
        rt_parts(s, i, j, k, &a, &b); out[3][p] = a + b;
        rz_parts(s, i, j, k, &a, &c); out[4][p] = a + c;
        tz_parts(s, i, j, k, &b, &c); out[5][p] = b + c;
      }
  for (int q = 0; q < 3; q++) s->f[VR + q] = save[q];
}

/* ------------------------- sources / receivers --------------------- */
int orc_add_source(orc *s, int kind, int i, int j, int k, const double *w, long ns)
{
  if (kind < SRC_VOLUME || kind > SRC_TORSION) return -1;
  if (i < 0 || i >= s->nr || j < -1 || j >= s->nt || k < 0 || k >= s->nz || ns < 0) return -2;
  s->src = (orc_src *)realloc(s->src, (s->nsrc + 1) * sizeof(orc_src));
  orc_src *q = &s->src[s->nsrc++];
  q->kind = kind; q->i = i; q->j = j; q->k = k; q->ns = ns;
  q->w = (double *)malloc((ns > 0 ? ns : 1) * sizeof(double));
  if (ns > 0) memcpy(q->w, w, ns * sizeof(double));
  return 0;
}

int orc_add_receiver(orc *s, int kind, int field, int i, int j, int k)
{
  if (kind != REC_PRESSURE && kind != REC_FIELD) return -1;
  if (kind == REC_FIELD && (field < 0 || field >= NFIELD)) return -1;
  if (i < 0 || i >= s->nr || j < -1 || j >= s->nt || k < 0 || k >= s->nz) return -2;
  s->rec = (orc_rec *)realloc(s->rec, (s->nrec + 1) * sizeof(orc_rec));
  orc_rec *q = &s->rec[s->nrec++];
  q->kind = kind; q->field = field; q->i = i; q->j = j; q->k = k;
  return s->nrec - 1;
}

/* Add dt*amp to field q at (i, j, k), or on the whole ring when j == -1.
   The strength is per unit volume: the point cell volume is
   rad*dr*dth*dz, the ring volume 2 pi rad dr dz, rad being the node's own
   radius. */
static void inject(orc *s, int q, double rad, const double *coef, int i, int j, int k, double amp)
{
  double vol = (j < 0) ? 2.0 * M_PI * rad * s->dr * s->dz : rad * s->dr * s->dth * s->dz;
  int j0 = j < 0 ? 0 : j, j1 = j < 0 ? s->nt : j + 1;
  for (int jj = j0; jj < j1; jj++) {
    size_t p = IDX(s, i, jj, k);
    double c = coef ? coef[p] : 1.0;
    s->f[q][p] += s->dt * c * amp / vol;
  }
}

static void apply_sources(orc *s, long n, int stress_phase)
{
  for (int m = 0; m < s->nsrc; m++) {
    orc_src *q = &s->src[m];
    double w = n < q->ns ? q->w[n] : 0.0;
    if (w == 0.0) continue;
    switch (q->kind) {
    case SRC_VOLUME:
      if (stress_phase) {
        inject(s, SRR, rc_(s, q->i), NULL, q->i, q->j, q->k, w);
        inject(s, STT, rc_(s, q->i), NULL, q->i, q->j, q->k, w);
        inject(s, SZZ, rc_(s, q->i), NULL, q->i, q->j, q->k, w);
      }
      break;
    case SRC_TORSION:
      if (stress_phase) {
        inject(s, SRT, rf_(s, q->i), NULL, q->i, q->j, q->k, w);
        inject(s, STZ, rc_(s, q->i), NULL, q->i, q->j, q->k, w);
      }
      break;
    case SRC_FORCE_R:
      if (!stress_phase) inject(s, VR, rf_(s, q->i), s->b_r, q->i, q->j, q->k, w);
      break;
    case SRC_FORCE_Z:
      if (!stress_phase) inject(s, VZ, rc_(s, q->i), s->b_z, q->i, q->j, q->k, w);
      break;
    }
  }
}

static double sample(const orc *s, const orc_rec *q)
{
  int j0 = q->j < 0 ? 0 : q->j, j1 = q->j < 0 ? s->nt : q->j + 1;
  double acc = 0.0;
  for (int j = j0; j < j1; j++) {
    size_t p = IDX(s, q->i, j, q->k);
    if (q->kind == REC_PRESSURE)
      acc += s->f[SRR][p] + s->f[STT][p] + s->f[SZZ][p];
    else
      acc += s->f[q->field][p];
  }
  if (q->kind == REC_PRESSURE) return -acc / (3.0 * (j1 - j0));
  return acc / (j1 - j0);
}

/* ------------------------------ energy ----------------------------- */
/* E^{n+1/2}: kinetic energy of v^{n+1/2} plus the strain energy written as
   the product of sigma^{n+1} and sigma^n, each term weighted by its node's
   radius times dr dth dz.  Conserved exactly by the leapfrog when the layer
   is off and nothing is injected. */
static double energy(const orc *s, double *const sold[6])
{
  const double *vr = s->f[VR], *vt = s->f[VT], *vz = s->f[VZ];
  const double *n0 = s->f[SRR], *n1 = s->f[STT], *n2 = s->f[SZZ];
  double E = 0.0;
  for (int i = 0; i < s->nr; i++) {
    double ri = rc_(s, i), Ri = rf_(s, i);
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        E += 0.5 * Ri * vr[p] * vr[p] / s->b_r[p];
        E += 0.5 * ri * vt[p] * vt[p] / s->b_t[p];
        E += 0.5 * ri * vz[p] * vz[p] / s->b_z[p];
        double K = s->lam[p] + 2.0 * s->mu[p] / 3.0;
        double t1 = n0[p] + n1[p] + n2[p];
        double t0 = sold[0][p] + sold[1][p] + sold[2][p];
        E += 0.5 * ri * t1 * t0 / (9.0 * K);
        if (s->mu[p] > 0) {
          double d1[3] = {n0[p] - t1 / 3.0, n1[p] - t1 / 3.0, n2[p] - t1 / 3.0};
          double d0[3] = {sold[0][p] - t0 / 3.0, sold[1][p] - t0 / 3.0, sold[2][p] - t0 / 3.0};
          E += 0.5 * ri * (d1[0] * d0[0] + d1[1] * d0[1] + d1[2] * d0[2]) / (2.0 * s->mu[p]);
        }
        if (s->mu_rt[p] > 0) E += 0.5 * Ri * s->f[SRT][p] * sold[3][p] / s->mu_rt[p];
        if (s->mu_rz[p] > 0) E += 0.5 * Ri * s->f[SRZ][p] * sold[4][p] / s->mu_rz[p];
        if (s->mu_tz[p] > 0) E += 0.5 * ri * s->f[STZ][p] * sold[5][p] / s->mu_tz[p];
      }
  }
  return E * s->dr * s->dth * s->dz;
}

/* ------------------------------ time step -------------------------- */
static void step_velocity(orc *s)
{
  const double dt = s->dt;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < s->nr; i++)
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        double Dr, B, Dz;
        int L = s->psi[0] != NULL;
        vr_parts(s, i, j, k, &Dr, &B, &Dz);
        if (L) {
          Dr = stretch(s, P_VR_DR, p, s->ar_f[i], s->br_f[i], Dr);
          B = stretch(s, P_VR_B, p, s->at_f[i], s->bt_f[i], B);
          Dz = stretch(s, P_VR_DZ, p, s->az_c[k], s->bz_c[k], Dz);
        }
        double dvr = dt * s->b_r[p] * (Dr + B + Dz);
        vt_parts(s, i, j, k, &Dr, &B, &Dz);
        if (L) {
          Dr = stretch(s, P_VT_DR, p, s->ar_c[i], s->br_c[i], Dr);
          B = stretch(s, P_VT_B, p, s->at_c[i], s->bt_c[i], B);
          Dz = stretch(s, P_VT_DZ, p, s->az_c[k], s->bz_c[k], Dz);
        }
        double dvt = dt * s->b_t[p] * (Dr + B + Dz);
        vz_parts(s, i, j, k, &Dr, &B, &Dz);
        if (L) {
          Dr = stretch(s, P_VZ_DR, p, s->ar_c[i], s->br_c[i], Dr);
          B = stretch(s, P_VZ_B, p, s->at_c[i], s->bt_c[i], B);
          Dz = stretch(s, P_VZ_DZ, p, s->az_h[k], s->bz_h[k], Dz);
        }
        double dvz = dt * s->b_z[p] * (Dr + B + Dz);
        /* the velocity right-hand sides read only stresses: in place is safe */
        s->f[VR][p] += dvr;
        s->f[VT][p] += dvt;
        s->f[VZ][p] += dvz;
      }
}

static void step_stress(orc *s)
{
  const double dt = s->dt;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < s->nr; i++)
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        int L = s->psi[0] != NULL;
        double err, ett, ezz;
        n_parts(s, i, j, k, &err, &ett, &ezz);
        if (L) {
          err = stretch(s, P_N_DR, p, s->ar_c[i], s->br_c[i], err);
          ett = stretch(s, P_N_B, p, s->at_c[i], s->bt_c[i], ett);
          ezz = stretch(s, P_N_DZ, p, s->az_c[k], s->bz_c[k], ezz);
        }
        double lam = s->lam[p], mu = s->mu[p];
        double tr = err + ett + ezz;
        double d_rr = dt * (lam * tr + 2.0 * mu * err);
        double d_tt = dt * (lam * tr + 2.0 * mu * ett);
        double d_zz = dt * (lam * tr + 2.0 * mu * ezz);
        double Dr, B, Dz;
        rt_parts(s, i, j, k, &Dr, &B);
        if (L) {
          Dr = stretch(s, P_RT_DR, p, s->ar_f[i], s->br_f[i], Dr);
          B = stretch(s, P_RT_B, p, s->at_f[i], s->bt_f[i], B);
        }
        double d_rt = dt * s->mu_rt[p] * (Dr + B);
        rz_parts(s, i, j, k, &Dr, &Dz);
        if (L) {
          Dr = stretch(s, P_RZ_DR, p, s->ar_f[i], s->br_f[i], Dr);
          Dz = stretch(s, P_RZ_DZ, p, s->az_h[k], s->bz_h[k], Dz);
        }
        double d_rz = dt * s->mu_rz[p] * (Dr + Dz);
        tz_parts(s, i, j, k, &B, &Dz);
        if (L) {
          B = stretch(s, P_TZ_B, p, s->at_c[i], s->bt_c[i], B);
          Dz = stretch(s, P_TZ_DZ, p, s->az_h[k], s->bz_h[k], Dz);
        }
        double d_tz = dt * s->mu_tz[p] * (B + Dz);
        s->f[SRR][p] += d_rr;
        s->f[STT][p] += d_tt;
        s->f[SZZ][p] += d_zz;
        s->f[SRT][p] += d_rt;
        s->f[SRZ][p] += d_rz;
        s->f[STZ][p] += d_tz;
      }
}

/* Advance nsteps.  Step n: v^{n-1/2} -> v^{n+1/2} from sigma^n, then force
   sources with w[n]; sigma^n -> sigma^{n+1} from v^{n+1/2}, then stress
   sources with w[n]; then every receiver records into
   traces[m*nsteps + (n - n_first)].  If energy is non-NULL, energy[n-n_first]
   receives E^{n+1/2}. */
int orc_run(orc *s, long nsteps, double *traces, double *energy_out)
{
  if (!(s->dt > 0)) return -5;
  double *sold[6] = {0};
  if (energy_out)
    for (int q = 0; q < 6; q++) sold[q] = (double *)malloc(s->n * sizeof(double));
  for (long t = 0; t < nsteps; t++) {
    long n = s->nstep;
    step_velocity(s);
    apply_sources(s, n, 0);
    if (energy_out)
      for (int q = 0; q < 6; q++) memcpy(sold[q], s->f[SRR + q], s->n * sizeof(double));
    step_stress(s);
    apply_sources(s, n, 1);
    if (traces)
      for (int m = 0; m < s->nrec; m++) traces[(size_t)m * nsteps + t] = sample(s, &s->rec[m]);
    if (energy_out) energy_out[t] = energy(s, sold);
    s->nstep++;
  }
  if (energy_out)
    for (int q = 0; q < 6; q++) free(sold[q]);
  return 0;
}

/* ---------------------------- state access ------------------------- */
int orc_get_field(const orc *s, int q, double *out)
{
  if (q < 0 || q >= NFIELD) return -1;
  memcpy(out, s->f[q], s->n * sizeof(double));
  return 0;
}

int orc_set_field(orc *s, int q, const double *in)
{
  if (q < 0 || q >= NFIELD) return -1;
  memcpy(s->f[q], in, s->n * sizeof(double));
  return 0;
}

/* staggered coefficients, for the checks: 0..5 = b_r b_t b_z mu_rt mu_rz mu_tz */
int orc_get_coef(const orc *s, int q, double *out)
{
  const double *src[6] = {s->b_r, s->b_t, s->b_z, s->mu_rt, s->mu_rz, s->mu_tz};
  if (q < 0 || q > 5) return -1;
  memcpy(out, src[q], s->n * sizeof(double));
  return 0;
}

long orc_steps_done(const orc *s) { return s->nstep; }

#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif
double orc_get_dt(const orc *s) { return s->dt; }

/* ============================== adjoint ============================= */
/* Discrete adjoint of the time step (the exact transpose of the linear map
   (v^{n-1/2}, sigma^n, psi^n) -> (v^{n+1/2}, sigma^{n+1}, psi^{n+1}); the
   sources do not depend on the state and drop out), written as the
   reverse of each statement of step_velocity and step_stress: every read
   X = c * f[q](i, j, k) of the forward code becomes fb[q](i, j, k) += c * Xb,
   every read outside the grid (a zero ghost) contributes nothing. */

/* transpose of at(): scatter into a(i, j, k), nothing outside the grid */
static void addv(const orc *s, double *a, int i, int j, int k, double v)
{
  if (i < 0 || i >= s->nr || k < 0 || k >= s->nz) return;
  j = ((j % s->nt) + s->nt) % s->nt;
  a[IDX(s, i, j, k)] += v;
}

/* transpose of stretch(): forward psi' = b psi + a X, out = X + psi';
   given out_b and pb[q][p] = adjoint of psi', returns X_b and leaves the
   adjoint of psi in pb[q][p]. */
static double stretch_adj(orc *s, double **pb, int q, size_t p, double a, double b, double outb)
{
  if (!s->psi[0]) return outb;
  double t = pb[q][p] + outb;
  pb[q][p] = b * t;
  return outb + a * t;
}

/* transposes of the strain parts: scatter the adjoints of the parts into the velocity adjoints */
static void n_parts_adj(const orc *s, double **fb, int i, int j, int k, double err, double ett, double ezz)
{
  double *vr = fb[VR], *vt = fb[VT], *vz = fb[VZ];
  addv(s, vr, i, j, k, err / s->dr);
  addv(s, vr, i - 1, j, k, -err / s->dr);
  double c = 1.0 / rc_(s, i);
  addv(s, vt, i, j, k, c * ett / s->dth);
  addv(s, vt, i, j - 1, k, -c * ett / s->dth);
  addv(s, vr, i, j, k, 0.5 * c * ett);
  addv(s, vr, i - 1, j, k, 0.5 * c * ett);
  addv(s, vz, i, j, k, ezz / s->dz);
  addv(s, vz, i, j, k - 1, -ezz / s->dz);
}

static void rt_parts_adj(const orc *s, double **fb, int i, int j, int k, double Dr, double B)
{
  double *vr = fb[VR], *vt = fb[VT];
  addv(s, vt, i + 1, j, k, Dr / s->dr);
  addv(s, vt, i, j, k, -Dr / s->dr);
  double c = 1.0 / rf_(s, i);
  addv(s, vr, i, j + 1, k, c * B / s->dth);
  addv(s, vr, i, j, k, -c * B / s->dth);
  addv(s, vt, i + 1, j, k, -0.5 * c * B);
  addv(s, vt, i, j, k, -0.5 * c * B);
}

static void rz_parts_adj(const orc *s, double **fb, int i, int j, int k, double Dr, double Dz)
{
  addv(s, fb[VZ], i + 1, j, k, Dr / s->dr);
  addv(s, fb[VZ], i, j, k, -Dr / s->dr);
  addv(s, fb[VR], i, j, k + 1, Dz / s->dz);
  addv(s, fb[VR], i, j, k, -Dz / s->dz);
}

static void tz_parts_adj(const orc *s, double **fb, int i, int j, int k, double B, double Dz)
{
  double c = 1.0 / rc_(s, i);
  addv(s, fb[VZ], i, j + 1, k, c * B / s->dth);
  addv(s, fb[VZ], i, j, k, -c * B / s->dth);
  addv(s, fb[VT], i, j, k + 1, Dz / s->dz);
  addv(s, fb[VT], i, j, k, -Dz / s->dz);
}

/* transposes of the velocity parts: scatter into the stress adjoints */
static void vr_parts_adj(const orc *s, double **fb, int i, int j, int k, double Dr, double B, double Dz)
{
  double *srr = fb[SRR], *stt = fb[STT], *srt = fb[SRT], *srz = fb[SRZ];
  addv(s, srr, i + 1, j, k, Dr / s->dr);
  addv(s, srr, i, j, k, -Dr / s->dr);
  double c = 1.0 / rf_(s, i);
  addv(s, srt, i, j, k, c * B / s->dth);
  addv(s, srt, i, j - 1, k, -c * B / s->dth);
  addv(s, srr, i + 1, j, k, 0.5 * c * B);
  addv(s, srr, i, j, k, 0.5 * c * B);
  addv(s, stt, i + 1, j, k, -0.5 * c * B);
  addv(s, stt, i, j, k, -0.5 * c * B);
  addv(s, srz, i, j, k, Dz / s->dz);
  addv(s, srz, i, j, k - 1, -Dz / s->dz);
}

static void vt_parts_adj(const orc *s, double **fb, int i, int j, int k, double Dr, double B, double Dz)
{
  double *stt = fb[STT], *srt = fb[SRT], *stz = fb[STZ];
  addv(s, srt, i, j, k, Dr / s->dr);
  addv(s, srt, i - 1, j, k, -Dr / s->dr);
  double c = 1.0 / rc_(s, i);
  addv(s, stt, i, j + 1, k, c * B / s->dth);
  addv(s, stt, i, j, k, -c * B / s->dth);
  addv(s, srt, i, j, k, c * B);
  addv(s, srt, i - 1, j, k, c * B);
  addv(s, stz, i, j, k, Dz / s->dz);
  addv(s, stz, i, j, k - 1, -Dz / s->dz);
}

static void vz_parts_adj(const orc *s, double **fb, int i, int j, int k, double Dr, double B, double Dz)
{
  double *szz = fb[SZZ], *srz = fb[SRZ], *stz = fb[STZ];
  addv(s, srz, i, j, k, Dr / s->dr);
  addv(s, srz, i - 1, j, k, -Dr / s->dr);
  double c = 1.0 / rc_(s, i);
  addv(s, stz, i, j, k, c * B / s->dth);
  addv(s, stz, i, j - 1, k, -c * B / s->dth);
  addv(s, srz, i, j, k, 0.5 * c * B);
  addv(s, srz, i - 1, j, k, 0.5 * c * B);
  addv(s, szz, i, j, k + 1, Dz / s->dz);
  addv(s, szz, i, j, k, -Dz / s->dz);
}

/* Reverse of step_stress.  On entry fb[S*] hold the adjoints of sigma^{n+1},
   fb[V*] of v^{n+1/2}, pb of psi^{n+1} (stress terms); on return fb[V*]
   hold the adjoints of v^{n+1/2} as an input of the stress update added
   in, pb the adjoints of psi^n.  The stress adjoints are unchanged: sigma^n
   enters sigma^{n+1} with coefficient 1. */
static void adj_stress(orc *s, double **fb, double **pb)
{
  const double dt = s->dt;
  for (int i = 0; i < s->nr; i++)
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        double g_rr = fb[SRR][p], g_tt = fb[STT][p], g_zz = fb[SZZ][p];
        double lam = s->lam[p], mu = s->mu[p];
        double gs = g_rr + g_tt + g_zz;
        double err = dt * (lam * gs + 2.0 * mu * g_rr);
        double ett = dt * (lam * gs + 2.0 * mu * g_tt);
        double ezz = dt * (lam * gs + 2.0 * mu * g_zz);
        err = stretch_adj(s, pb, P_N_DR, p, s->ar_c[i], s->br_c[i], err);
        ett = stretch_adj(s, pb, P_N_B, p, s->at_c[i], s->bt_c[i], ett);
        ezz = stretch_adj(s, pb, P_N_DZ, p, s->az_c[k], s->bz_c[k], ezz);
        n_parts_adj(s, fb, i, j, k, err, ett, ezz);
        double g = dt * s->mu_rt[p] * fb[SRT][p];
        double Dr = stretch_adj(s, pb, P_RT_DR, p, s->ar_f[i], s->br_f[i], g);
        double B = stretch_adj(s, pb, P_RT_B, p, s->at_f[i], s->bt_f[i], g);
        rt_parts_adj(s, fb, i, j, k, Dr, B);
        g = dt * s->mu_rz[p] * fb[SRZ][p];
        Dr = stretch_adj(s, pb, P_RZ_DR, p, s->ar_f[i], s->br_f[i], g);
        double Dz = stretch_adj(s, pb, P_RZ_DZ, p, s->az_h[k], s->bz_h[k], g);
        rz_parts_adj(s, fb, i, j, k, Dr, Dz);
        g = dt * s->mu_tz[p] * fb[STZ][p];
        B = stretch_adj(s, pb, P_TZ_B, p, s->at_c[i], s->bt_c[i], g);
        Dz = stretch_adj(s, pb, P_TZ_DZ, p, s->az_h[k], s->bz_h[k], g);
        tz_parts_adj(s, fb, i, j, k, B, Dz);
      }
}

/* Reverse of step_velocity: fb[V*] hold the adjoints of v^{n+1/2}; the
   stress adjoints receive the transposed divergence, pb the adjoints of
   the velocity terms' psi^n; fb[V*] are unchanged (v^{n-1/2} enters with
   coefficient 1). */
static void adj_velocity(orc *s, double **fb, double **pb)
{
  const double dt = s->dt;
  for (int i = 0; i < s->nr; i++)
    for (int j = 0; j < s->nt; j++)
      for (int k = 0; k < s->nz; k++) {
        size_t p = IDX(s, i, j, k);
        double g = dt * s->b_r[p] * fb[VR][p];
        double Dr = stretch_adj(s, pb, P_VR_DR, p, s->ar_f[i], s->br_f[i], g);
        double B = stretch_adj(s, pb, P_VR_B, p, s->at_f[i], s->bt_f[i], g);
        double Dz = stretch_adj(s, pb, P_VR_DZ, p, s->az_c[k], s->bz_c[k], g);
        vr_parts_adj(s, fb, i, j, k, Dr, B, Dz);
        g = dt * s->b_t[p] * fb[VT][p];
        Dr = stretch_adj(s, pb, P_VT_DR, p, s->ar_c[i], s->br_c[i], g);
        B = stretch_adj(s, pb, P_VT_B, p, s->at_c[i], s->bt_c[i], g);
        Dz = stretch_adj(s, pb, P_VT_DZ, p, s->az_c[k], s->bz_c[k], g);
        vt_parts_adj(s, fb, i, j, k, Dr, B, Dz);
        g = dt * s->b_z[p] * fb[VZ][p];
        Dr = stretch_adj(s, pb, P_VZ_DR, p, s->ar_c[i], s->br_c[i], g);
        B = stretch_adj(s, pb, P_VZ_B, p, s->at_c[i], s->bt_c[i], g);
        Dz = stretch_adj(s, pb, P_VZ_DZ, p, s->az_h[k], s->bz_h[k], g);
        vz_parts_adj(s, fb, i, j, k, Dr, B, Dz);
      }
}

/* One source-free step of the current state (for the adjoint checks). */
void orc_step_linear(orc *s)
{
  step_velocity(s);
  step_stress(s);
}

/* One adjoint step in place: fb[NFIELD] (n arrays each) and pb[NPSI] (n
   arrays each, ignored with the layer off) hold the adjoint of the state
   after a step and receive the adjoint of the state before it. */
void orc_adjoint_step(orc *s, double *const fb_in[NFIELD], double *const pb_in[NPSI])
{
  double *fb[NFIELD], *pb[NPSI];
  for (int q = 0; q < NFIELD; q++) fb[q] = fb_in[q];
  for (int q = 0; q < NPSI; q++) pb[q] = s->psi[0] ? pb_in[q] : NULL;
  adj_stress(s, fb, pb);
  adj_velocity(s, fb, pb);
}

int orc_get_psi(const orc *s, int q, double *out)
{
  if (q < 0 || q >= NPSI || !s->psi[0]) return -1;
  memcpy(out, s->psi[q], s->n * sizeof(double));
  return 0;
}

int orc_set_psi(orc *s, int q, const double *in)
{
  if (q < 0 || q >= NPSI || !s->psi[0]) return -1;
  memcpy(s->psi[q], in, s->n * sizeof(double));
  return 0;
}

/* d HM4 / d a at (a, b, c, d); the one-sided limit 4 when a alone is zero */
static double dhm4(double a, double b, double c, double d)
{
  if (b == 0.0 || c == 0.0 || d == 0.0) return 0.0;
  if (a == 0.0) return 4.0;
  double h = hm4(a, b, c, d);
  return h * h / (4.0 * a * a);
}

/* Gradient of L = sum over steps n in [n0, n1) and pressure receivers m of
   p_m(t_{n+1})^2 with respect to the moduli of the parameter region:
   rings [i0, i1), every theta, depth rows [k0, k0 + nbins*bin_rows) in bins
   of bin_rows rows.  Bin b's parameters shift mu and the bulk modulus
   K = lambda + 2 mu / 3 of all its cells together, so
     dL/dmu_b = sum over its cells of (dL/dmu|lambda - (2/3) dL/dlambda),
     dL/dK_b  = sum over its cells of dL/dlambda.
   Runs the forward steps 0..nsteps-1 from the zero state (with the
   sources), storing the strains of the region's nodes, then the adjoint
   steps back from the last one.  The region must lie outside the absorbing
   layer (its strains are then the plain ones).  Returns 0, or <0 for a bad
   argument / state. */
int orc_gradient(orc *s, long nsteps, long n0, long n1, int i0, int i1, int k0, int nbins, int bin_rows,
                 double *loss, double *g_mu, double *g_K)
{
  if (!(s->dt > 0) || s->nstep != 0) return -5;
  int k1 = k0 + nbins * bin_rows;
  if (i0 < 0 || i1 > s->nr || i0 >= i1 || k0 < 0 || k1 > s->nz || nbins < 1 || bin_rows < 1) return -2;
  if (s->psi[0] && (i1 > s->nr - s->npr || k0 < s->npz + 1 || k1 > s->nz - 1 - s->npz - 1)) return -2;
  /* nodes whose strains the gradient needs: rings i0-1..i1-1, depths k0-1..k1-1 */
  int ea = i0 > 0 ? i0 - 1 : 0, eb = i1, za = k0 > 0 ? k0 - 1 : 0, zb = k1;
  size_t nreg = (size_t)(eb - ea) * s->nt * (zb - za);
  double *Z = (double *)malloc((size_t)nsteps * nreg * 6 * sizeof(double));
  double *tr = (double *)malloc((size_t)(s->nrec > 0 ? s->nrec : 1) * nsteps * sizeof(double));
  if (!Z || !tr) { free(Z); free(tr); return -8; }
#define ZI(t, i, j, k) ((((size_t)(t) * (eb - ea) + ((i) - ea)) * s->nt + (j)) * (zb - za) + ((k) - za))
  /* forward */
  for (long t = 0; t < nsteps; t++) {
    step_velocity(s);
    apply_sources(s, t, 0);
    for (int i = ea; i < eb; i++)
      for (int j = 0; j < s->nt; j++)
        for (int k = za; k < zb; k++) {
          double *z = Z + ZI(t, i, j, k) * 6;
          double a, b;
          n_parts(s, i, j, k, &z[0], &z[1], &z[2]);
          rt_parts(s, i, j, k, &a, &b); z[3] = a + b;
          rz_parts(s, i, j, k, &a, &b); z[4] = a + b;
          tz_parts(s, i, j, k, &a, &b); z[5] = a + b;
        }
    step_stress(s);
    apply_sources(s, t, 1);
    for (int m = 0; m < s->nrec; m++) tr[(size_t)m * nsteps + t] = sample(s, &s->rec[m]);
    s->nstep++;
  }
  double L = 0.0;
  for (int m = 0; m < s->nrec; m++)
    if (s->rec[m].kind == REC_PRESSURE)
      for (long t = n0; t < n1 && t < nsteps; t++) L += tr[(size_t)m * nsteps + t] * tr[(size_t)m * nsteps + t];
  *loss = L;
  /* adjoint */
  double *fb[NFIELD], *pb[NPSI] = {0};
  for (int q = 0; q < NFIELD; q++) fb[q] = (double *)calloc(s->n, sizeof(double));
  if (s->psi[0])
    for (int q = 0; q < NPSI; q++) pb[q] = (double *)calloc(s->n, sizeof(double));
  double *glam = (double *)calloc(s->n, sizeof(double)), *gmu = (double *)calloc(s->n, sizeof(double));
  const double dt = s->dt;
  for (long t = nsteps - 1; t >= 0; t--) {
    /* receivers: dL/dsigma^{t+1} */
    if (t >= n0 && t < n1)
      for (int m = 0; m < s->nrec; m++) {
        const orc_rec *q = &s->rec[m];
        if (q->kind != REC_PRESSURE) continue;
        int j0 = q->j < 0 ? 0 : q->j, j1 = q->j < 0 ? s->nt : q->j + 1;
        double g = 2.0 * tr[(size_t)m * nsteps + t] * (-1.0 / (3.0 * (j1 - j0)));
        for (int j = j0; j < j1; j++) {
          size_t p = IDX(s, q->i, j, q->k);
          fb[SRR][p] += g; fb[STT][p] += g; fb[SZZ][p] += g;
        }
      }
    /* moduli: sigma^{t+1} = sigma^t + dt C(lambda, mu) Z^{t+1/2} */
    for (int i = ea; i < eb; i++)
      for (int j = 0; j < s->nt; j++)
        for (int k = za; k < zb; k++) {
          size_t p = IDX(s, i, j, k);
          const double *z = Z + ZI(t, i, j, k) * 6;
          if (i >= i0 && k >= k0) {
            double gs = fb[SRR][p] + fb[STT][p] + fb[SZZ][p];
            glam[p] += dt * (z[0] + z[1] + z[2]) * gs;
            gmu[p] += 2.0 * dt * (z[0] * fb[SRR][p] + z[1] * fb[STT][p] + z[2] * fb[SZZ][p]);
          }
          /* shear nodes of this index: their effective modulus is HM4 of four cells */
          int i1c = i + 1 < s->nr ? i + 1 : s->nr - 1, j1c = (j + 1) % s->nt;
          int k1c = k + 1 < s->nz ? k + 1 : s->nz - 1;
          const double *mu = s->mu;
          double grt = dt * z[3] * fb[SRT][p], grz = dt * z[4] * fb[SRZ][p], gtz = dt * z[5] * fb[STZ][p];
          size_t c00 = p, ci = IDX(s, i1c, j, k), cj = IDX(s, i, j1c, k), cij = IDX(s, i1c, j1c, k);
          size_t ck = IDX(s, i, j, k1c), cik = IDX(s, i1c, j, k1c), cjk = IDX(s, i, j1c, k1c);
          /* rt: (i, j), (i+1, j), (i, j+1), (i+1, j+1) */
          size_t rt[4] = {c00, ci, cj, cij};
          size_t rz[4] = {c00, ci, ck, cik};
          size_t tz[4] = {c00, cj, ck, cjk};
          for (int w = 0; w < 4; w++) {
            int o1 = (w + 1) % 4, o2 = (w + 2) % 4, o3 = (w + 3) % 4;
            gmu[rt[w]] += grt * dhm4(mu[rt[w]], mu[rt[o1]], mu[rt[o2]], mu[rt[o3]]);
            gmu[rz[w]] += grz * dhm4(mu[rz[w]], mu[rz[o1]], mu[rz[o2]], mu[rz[o3]]);
            gmu[tz[w]] += gtz * dhm4(mu[tz[w]], mu[tz[o1]], mu[tz[o2]], mu[tz[o3]]);
          }
        }
    adj_stress(s, fb, pb);
    adj_velocity(s, fb, pb);
  }
  for (int b = 0; b < nbins; b++) { g_mu[b] = 0.0; g_K[b] = 0.0; }
  for (int i = i0; i < i1; i++)
    for (int j = 0; j < s->nt; j++)
      for (int k = k0; k < k1; k++) {
        size_t p = IDX(s, i, j, k);
        int b = (k - k0) / bin_rows;
        g_mu[b] += gmu[p] - (2.0 / 3.0) * glam[p];
        g_K[b] += glam[p];
      }
#undef ZI
  for (int q = 0; q < NFIELD; q++) free(fb[q]);
  for (int q = 0; q < NPSI; q++) free(pb[q]);
  free(glam); free(gmu); free(Z); free(tr);
  return 0;
}
