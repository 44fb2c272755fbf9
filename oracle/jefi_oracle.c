/*
 * jefi_oracle.c -- plain, slow FP64 CPU oracle of the discretised Jefimenko
 * sums.  TEST INFRASTRUCTURE ONLY: it exists to check the HIP library and is
 * used by the tests, the smoke check and the CPU-baseline leg of the bench.
 * It shares no code, header or constant with the library.
 *
 * What it computes (paper, section "GPU implementation of Jefimenko's
 * equations", the discretised equations for E, B and the retarded time):
 *
 *   E(r,t) =  1/(4 pi) sum_cells [ d rho(t_r)/R^3 + d rho_dot(t_r)/R^2 - J_dot(t_r)/R ] dOmega
 *   B(r,t) = -1/(4 pi) sum_cells [ d x J(t_r)/R^3 + d x J_dot(t_r)/R^2 ] dOmega
 *   t_r    = t - R/c,     d = r - r',  R = |d|,  dOmega = dx' dy' dz'
 *
 * with rationalised Lorentz-Heaviside units (section "Jefimenko's
 * equations"), time derivatives taken as the backward difference
 * [q(t_r) - q(t_r - dt)]/dt, and the sources read from a stored history of
 * slices (section "Parameter dependence": rho and J kept for all relevant
 * times).  Readings of points the paper leaves open:
 *   - step s of the history sits at t0 + s*dt; the window holds the nt steps
 *     newest-nt+1 .. newest (logical slice 0 = oldest);
 *   - values between slices are linear interpolations in time; the backward
 *     difference is applied to that interpolant, so the derivative is the
 *     same linear interpolation of the slice-wise differences
 *     D_k = (h_k - h_(k-1))/dt;
 *   - slices before the oldest stored one are zero (the paper's sources
 *     vanish before t = 0), including h_(-1) inside D_0;
 * Two alternative readings of those last two points are selectable through
 * the `stencil` bits of orc_eval (the default, 0, is the reading above):
 *   - bit 0: the time derivative is the slope of the linear interpolant on
 *     the interval holding t_r, (h_(k+1) - h_k)/dt, instead of the
 *     interpolated backward difference;
 *   - bit 1: slices before the oldest stored one hold the oldest slice's
 *     values (sources constant before the retained window), so h_(-1) = h_0
 *     inside D_0 and no pair is ever wholly in an empty past;
 *   - bit 2: cubic time interpolation: value and time derivative from the
 *     cubic through slices k-2, k-1, k, k+1 (the Lagrange polynomial on
 *     those four nodes, evaluated at position f past slice k, and its
 *     derivative divided by dt).  Its nodes end at k+1, so it reads no slice
 *     the linear stencil does not reach at the top, and a pair whose k+1
 *     lies before the oldest slice still contributes nothing.  It cannot be
 *     combined with bit 0;
 *   - bit 3: the history starts at the oldest slice: a pair whose retarded
 *     time precedes it (k < 0) contributes nothing, and stencils that reach
 *     before it read the oldest slice's values (as bit 1), so no time
 *     derivative is taken across the start.  For sources switched on at the
 *     oldest slice this leaves out the switch-on shell that the zero past
 *     gives (the step's derivative).  It cannot be combined with bit 1.
 * None of them changes the slice index k or the screening decision.
 *   - the slice index is k = a_i + floor(u), u = a_f - R*inv_cdt with the
 *     host split a = (t - t0)/dt - s_old = a_i + a_f, all in FP64 with no
 *     contraction; the interpolation weight is f = u - floor(u) and slice
 *     k+1 is not read when f == 0;
 *   - coarse screening (fields in a cell come only from other cells): a pair
 *     is left out when |dx| <= delta_x, |dy| <= delta_y and |dz| <= delta_z,
 *     and always when R == 0;
 *   - cell centres are origin + index*spacing (mul, then add).
 * Sums over source cells run in linear cell order with Neumaier-compensated
 * FP64 accumulators; observation points are independent (OpenMP), so the
 * result does not depend on the thread count.
 *
 * Build: cc -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t n[3];
  double origin[3];
  double spacing[3];
} orc_grid;

typedef struct {
  int64_t s_old;   /* absolute step of logical slice 0 */
  int64_t a_i;     /* floor of the evaluation time in logical slice units */
  double a_f;      /* its fractional part */
  double inv_cdt;  /* 1/(c*dt) */
} orc_time;

#define ORC_SCREENED INT32_MIN

/* ---- small helpers -------------------------------------------------- */

typedef struct { double s, c; } orc_nsum;

static void orc_nadd(orc_nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static int64_t orc_cells(const orc_grid* g) {
  return (int64_t)g->n[0] * g->n[1] * g->n[2];
}

static void orc_centre(const orc_grid* g, int64_t lin, double r[3]) {
  int64_t i = lin % g->n[0];
  int64_t j = (lin / g->n[0]) % g->n[1];
  int64_t k = lin / ((int64_t)g->n[0] * g->n[1]);
  r[0] = g->origin[0] + (double)i * g->spacing[0];
  r[1] = g->origin[1] + (double)j * g->spacing[1];
  r[2] = g->origin[2] + (double)k * g->spacing[2];
}

static int orc_grid_ok(const orc_grid* g) {
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 0) return 0;
    if (!isfinite(g->origin[a]) || !isfinite(g->spacing[a])) return 0;
  }
  return 1;
}

/* ---- time prelude --------------------------------------------------- */

/* Place t on the logical slice axis.  Returns 0, or -1 for bad arguments,
 * -2 when t lies after the newest slice (beyond a hair of rounding). */
int orc_time_prelude(double t, double t0, double dt, int64_t newest, int32_t nt,
                     double c, orc_time* out) {
  if (!(dt > 0.0) || !(c > 0.0) || nt < 1 || !isfinite(t) || !isfinite(t0)) return -1;
  int64_t s_old = newest - (int64_t)nt + 1;
  double a = (t - t0) / dt - (double)s_old;
  double top = (double)(nt - 1);
  if (!(a <= top)) {
    double slack = 1e-9 * (1.0 + fabs(a) + fabs((double)s_old));
    if (a - top <= slack)
      a = top;
    else
      return -2;
  }
  double fl = floor(a);
  out->s_old = s_old;
  out->a_i = (int64_t)fl;
  out->a_f = a - fl;
  out->inv_cdt = 1.0 / (c * dt);
  return 0;
}

/* ---- per-pair decision ---------------------------------------------- */

/* The canonical FP64 decision for one pair.  Returns 1 when the pair is
 * screened (or R == 0), else 0 and fills R, the unclamped slice index k and
 * the weight f. */
static int orc_pair(const double ro[3], const double rs[3], const double delta[3],
                    const orc_time* tm, double d[3], double* R, int64_t* k, double* f) {
  d[0] = ro[0] - rs[0];
  d[1] = ro[1] - rs[1];
  d[2] = ro[2] - rs[2];
  if (fabs(d[0]) <= delta[0] && fabs(d[1]) <= delta[1] && fabs(d[2]) <= delta[2]) return 1;
  double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
  double r = sqrt(r2);
  if (r == 0.0) return 1;
  double u = tm->a_f - r * tm->inv_cdt;
  double m = floor(u);
  *R = r;
  *k = tm->a_i + (int64_t)m;
  *f = u - m;
  return 0;
}

/* History value of channel ch at logical slice j.  Before slice 0 it is
 * zero, or slice 0's value when `hold` is set. */
static double orc_h(const double* hist, int64_t ns, int64_t j, int ch, int64_t s, int hold) {
  if (j < 0) {
    if (!hold) return 0.0;
    j = 0;
  }
  return hist[(j * 4 + ch) * ns + s];
}

/* Cubic time interpolation (stencil bit 2): the Lagrange polynomial through
 * slices k-2 .. k+1, placed at nodes x = -2 .. 1, evaluated at x = f; val =
 * sum_i w_i h_(k+i) and der = sum_i w_i' h_(k+i) / dt with
 *   w_i(f)  = prod_(j != i) (f - x_j) / (x_i - x_j),
 *   w_i'(f) = sum_(m != i) [1 / (x_i - x_m)] prod_(j != i, m) (f - x_j) / (x_i - x_j). */
static void orc_cubic(const double* hist, int64_t ns, int64_t k, double f, double inv_dt, int64_t s,
                      int hold, double val[4], double der[4]) {
  static const double x[4] = {-2.0, -1.0, 0.0, 1.0};
  double w[4], dw[4];
  for (int i = 0; i < 4; ++i) {
    double p = 1.0, dp = 0.0;
    for (int j = 0; j < 4; ++j) {
      if (j == i) continue;
      p *= (f - x[j]) / (x[i] - x[j]);
    }
    for (int m = 0; m < 4; ++m) {
      if (m == i) continue;
      double q = 1.0 / (x[i] - x[m]);
      for (int j = 0; j < 4; ++j) {
        if (j == i || j == m) continue;
        q *= (f - x[j]) / (x[i] - x[j]);
      }
      dp += q;
    }
    w[i] = p;
    dw[i] = dp;
  }
  for (int ch = 0; ch < 4; ++ch) {
    double v = 0.0, d = 0.0;
    for (int i = 0; i < 4; ++i) {
      double h = orc_h(hist, ns, k - 2 + i, ch, s, hold);
      v += w[i] * h;
      d += dw[i] * h;
    }
    val[ch] = v;
    der[ch] = d * inv_dt;
  }
}

/* ---- field evaluation ----------------------------------------------- */

/* Evaluate E and B at the selected observation points.
 *   hist  : FP64 [nt][4][n_src], logical slice 0 = oldest (absolute step
 *           newest-nt+1), channel 0 = rho, 1..3 = Jx, Jy, Jz
 *   sel   : linear observation indices to evaluate (NULL = all, n_sel ignored)
 *   E, B  : FP64 [3][n_out] with n_out = n_sel or n_obs, component-major
 *   delta : screening half-widths
 *   threads: OpenMP threads (0 = runtime default)
 *   stencil: reading of the time stencil (bits in the header comment; 0 = default)
 * Returns 0, -1 (bad arguments) or -2 (t after the newest slice). */
int orc_eval(const orc_grid* src, const orc_grid* obs, const double* hist, int32_t nt,
             double dt, double c, double t, double t0, int64_t newest, const double delta[3],
             const int64_t* sel, int64_t n_sel, double* E, double* B, int32_t threads,
             int32_t stencil) {
  if (!src || !obs || !hist || !E || !B || !delta) return -1;
  if (stencil < 0 || stencil > 15 || (stencil & 5) == 5 || (stencil & 10) == 10) return -1;
  const int slope = (stencil & 1) != 0, cubic = (stencil & 4) != 0, cut = (stencil & 8) != 0;
  const int hold = (stencil & 2) != 0 || cut; /* slices before the oldest read as the oldest */
  if (!orc_grid_ok(src) || !orc_grid_ok(obs)) return -1;
  orc_time tm;
  int rc = orc_time_prelude(t, t0, dt, newest, nt, c, &tm);
  if (rc) return rc;
  const int64_t ns = orc_cells(src);
  const int64_t no = orc_cells(obs);
  const int64_t nout = sel ? n_sel : no;
  const double pref = (src->spacing[0] * src->spacing[1] * src->spacing[2]) / (4.0 * M_PI);
  const double inv_dt = 1.0 / dt;
  int bad = 0;
#ifdef _OPENMP
  int nth = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth) reduction(| : bad)
#endif
  for (int64_t q = 0; q < nout; ++q) {
    int64_t o = sel ? sel[q] : q;
    if (o < 0 || o >= no) { bad |= 1; continue; }
    double ro[3];
    orc_centre(obs, o, ro);
    orc_nsum acc[6];
    memset(acc, 0, sizeof acc);
    for (int64_t s = 0; s < ns; ++s) {
      double rs[3], d[3], R, f;
      int64_t k;
      orc_centre(src, s, rs);
      if (orc_pair(ro, rs, delta, &tm, d, &R, &k, &f)) continue;
      if (cut && k < 0) continue;    /* retarded time before the start of the history */
      if (k < -1 && !hold) continue; /* the whole stencil lies before the oldest slice */
      if ((f != 0.0 || slope || cubic) && k + 1 > (int64_t)nt - 1) { bad |= 2; continue; }
      double val[4], der[4];
      if (cubic) {
        orc_cubic(hist, ns, k, f, inv_dt, s, hold, val, der);
      } else {
      for (int ch = 0; ch < 4; ++ch) {
        double h0 = orc_h(hist, ns, k, ch, s, hold);
        double hm = orc_h(hist, ns, k - 1, ch, s, hold);
        double d0 = (h0 - hm) * inv_dt;
        double v = (1.0 - f) * h0;
        double w = (1.0 - f) * d0;
        if (f != 0.0) {
          double h1 = orc_h(hist, ns, k + 1, ch, s, hold);
          double d1 = (h1 - h0) * inv_dt;
          v += f * h1;
          w += f * d1;
        }
        /* slope reading: the interpolant's derivative on [k, k+1], also at f == 0 */
        if (slope) w = (orc_h(hist, ns, k + 1, ch, s, hold) - h0) * inv_dt;
        val[ch] = v;
        der[ch] = w;
      }
      }
      double rho = val[0], rhod = der[0];
      const double* J = &val[1];
      const double* Jd = &der[1];
      double iR = 1.0 / R;
      double iR2 = iR * iR;
      double iR3 = iR2 * iR;
      for (int a = 0; a < 3; ++a) orc_nadd(&acc[a], d[a] * rho * iR3 + d[a] * rhod * iR2 - Jd[a] * iR);
      /* B: -(d x J / R^3 + d x Jdot / R^2) */
      double cJ[3] = {d[1] * J[2] - d[2] * J[1], d[2] * J[0] - d[0] * J[2], d[0] * J[1] - d[1] * J[0]};
      double cD[3] = {d[1] * Jd[2] - d[2] * Jd[1], d[2] * Jd[0] - d[0] * Jd[2], d[0] * Jd[1] - d[1] * Jd[0]};
      for (int a = 0; a < 3; ++a) orc_nadd(&acc[3 + a], -(cJ[a] * iR3 + cD[a] * iR2));
    }
    for (int a = 0; a < 3; ++a) {
      E[a * nout + q] = (acc[a].s + acc[a].c) * pref;
      B[a * nout + q] = (acc[3 + a].s + acc[3 + a].c) * pref;
    }
  }
  if (bad & 1) return -1;
  if (bad & 2) return -2;
  return 0;
}

/* Per-pair slice-index dump for small problems: out[o * n_src + s] is
 * ORC_SCREENED for a screened pair (or R == 0), -2 for a pair whose whole
 * stencil lies before the oldest slice (k < -1), else k in [-1, nt-1]. */
int orc_slice_index_dump(const orc_grid* src, const orc_grid* obs, int32_t nt, double dt, double c,
                         double t, double t0, int64_t newest, const double delta[3], int32_t* out) {
  if (!src || !obs || !out || !delta) return -1;
  if (!orc_grid_ok(src) || !orc_grid_ok(obs)) return -1;
  orc_time tm;
  int rc = orc_time_prelude(t, t0, dt, newest, nt, c, &tm);
  if (rc) return rc;
  const int64_t ns = orc_cells(src);
  const int64_t no = orc_cells(obs);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t o = 0; o < no; ++o) {
    double ro[3];
    orc_centre(obs, o, ro);
    for (int64_t s = 0; s < ns; ++s) {
      double rs[3], d[3], R, f;
      int64_t k;
      orc_centre(src, s, rs);
      int32_t code;
      if (orc_pair(ro, rs, delta, &tm, d, &R, &k, &f))
        code = ORC_SCREENED;
      else
        code = k < -1 ? -2 : (int32_t)k;
      out[o * ns + s] = code;
    }
  }
  return 0;
}

/* Per-observation-point fingerprint of the slice decisions over the pairs
 * that are neither screened nor entirely before the oldest slice:
 *   fp[4*o+0] = number of such pairs
 *   fp[4*o+1] = sum of k
 *   fp[4*o+2] = sum of k*(s+1) (wrapping 64-bit)
 *   fp[4*o+3] = number of screened pairs (including R == 0)          */
int orc_slice_fingerprint(const orc_grid* src, const orc_grid* obs, int32_t nt, double dt,
                          double c, double t, double t0, int64_t newest, const double delta[3],
                          const int64_t* sel, int64_t n_sel, int64_t* fp) {
  if (!src || !obs || !fp || !delta) return -1;
  if (!orc_grid_ok(src) || !orc_grid_ok(obs)) return -1;
  orc_time tm;
  int rc = orc_time_prelude(t, t0, dt, newest, nt, c, &tm);
  if (rc) return rc;
  const int64_t ns = orc_cells(src);
  const int64_t no = orc_cells(obs);
  const int64_t nout = sel ? n_sel : no;
  int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
#endif
  for (int64_t q = 0; q < nout; ++q) {
    int64_t o = sel ? sel[q] : q;
    if (o < 0 || o >= no) { bad = 1; continue; }
    double ro[3];
    orc_centre(obs, o, ro);
    int64_t nlive = 0, sk = 0, nscr = 0;
    uint64_t skw = 0;
    for (int64_t s = 0; s < ns; ++s) {
      double rs[3], d[3], R, f;
      int64_t k;
      orc_centre(src, s, rs);
      if (orc_pair(ro, rs, delta, &tm, d, &R, &k, &f)) { ++nscr; continue; }
      if (k < -1) continue;
      ++nlive;
      sk += k;
      skw += (uint64_t)k * (uint64_t)(s + 1);
    }
    fp[4 * q + 0] = nlive;
    fp[4 * q + 1] = sk;
    fp[4 * q + 2] = (int64_t)skw;
    fp[4 * q + 3] = nscr;
  }
  return bad ? -1 : 0;
}

/* Number of OpenMP threads a parallel region would use. */
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
