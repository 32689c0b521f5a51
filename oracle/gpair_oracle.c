/*
 * gpair_oracle.c -- plain float64 CPU oracle of the GPAIR direct operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code with the HIP
 * path and must never be used as a fallback for it.
 *
 * What it computes (arXiv 2602.03893, Methods):
 *  - the pressure a single isotropic Gaussian kernel (amplitude A, width
 *    sigma, centre at distance r from the detector) produces at time t,
 *    keeping only the outgoing term: Eq. (single_forward),
 *        p = A/(2r) * d * exp(-d^2/(2 sigma^2)),  d = r - v t;
 *  - kept only inside the window |d| <= n_sigma*sigma (the "3 sigma
 *    principle" that follows that equation; inclusive edges);
 *  - summed over all kernels (linearity of the wave equation, stated at the
 *    start of the Methods section) and evaluated at every sample t = t0 + n dt
 *    of every sensor: the direct enumeration over source-detector pairs the
 *    paper describes at the start of the "Adaptive supersampling alignment"
 *    subsection;
 *  - the transpose of that linear map (the "Adjoint Operator" subsection's
 *    principle: the adjoint is the transpose of the forward), and the
 *    derivative of Eq. (single_forward) with respect to sigma.
 *
 * Everything is float64 with plain loops; inputs are the float32 arrays the
 * GPU receives, promoted exactly.  Window membership of each candidate sample
 * is decided by evaluating |d| <= n_sigma*sigma directly.  Build with
 * -ffp-contract=off so every operation is separately rounded.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* r = |s - c| in float64 from float32 coordinates. */
static double pair_distance(const float *s, float cx, float cy, float cz) {
  double dx = (double)s[0] - (double)cx;
  double dy = (double)s[1] - (double)cy;
  double dz = (double)s[2] - (double)cz;
  return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Candidate sample range [lo, hi] (clipped to the trace) that surely contains
 * every n with |r - v (t0 + n dt)| <= half; membership is then tested per n. */
static void candidate_range(double r, double half, double v, double dt,
                            double t0, int64_t nt, int64_t *lo, int64_t *hi) {
  double a = (r - half) / v - t0;
  double b = (r + half) / v - t0;
  int64_t l = (int64_t)floor(a / dt) - 1;
  int64_t h = (int64_t)ceil(b / dt) + 1;
  if (l < 0) l = 0;
  if (h > nt - 1) h = nt - 1;
  *lo = l;
  *hi = h;
}

/*
 * Forward: y[j*nt + n] = sum_k [|d| <= nsig*sigma_k] A_k/(2r) d exp(-d^2/(2 sigma_k^2)).
 * y is float64 [nd][nt], overwritten.
 */
void oracle_forward(int64_t m, const float *cx, const float *cy,
                    const float *cz, const double *amp, const double *sigma,
                    int64_t nd, const float *sensors, int64_t nt, double dt,
                    double t0, double v, double nsig, double *y) {
  int64_t j;
#pragma omp parallel for schedule(dynamic, 1)
  for (j = 0; j < nd; ++j) {
    double *row = y + j * nt;
    for (int64_t n = 0; n < nt; ++n) row[n] = 0.0;
    const float *s = sensors + 3 * j;
    for (int64_t k = 0; k < m; ++k) {
      double r = pair_distance(s, cx[k], cy[k], cz[k]);
      double sg = (double)sigma[k];
      double half = nsig * sg;
      double a = (double)amp[k];
      int64_t lo, hi;
      candidate_range(r, half, v, dt, t0, nt, &lo, &hi);
      for (int64_t n = lo; n <= hi; ++n) {
        double t = t0 + (double)n * dt;
        double d = r - v * t;
        if (fabs(d) <= half) {
          row[n] += a / (2.0 * r) * d * exp(-(d * d) / (2.0 * sg * sg));
        }
      }
    }
  }
}

/*
 * Adjoint: gA[k] = sum_j sum_{n in W} delta[j][n] d e / (2r);
 *          gsig[k] = sum_j sum_{n in W} delta[j][n] A_k d^3 e / (2 r sigma_k^3).
 * delta is float64 [nd][nt]; gA, gsig float64 [m], overwritten (gsig may be
 * NULL).
 */
void oracle_adjoint(int64_t m, const float *cx, const float *cy,
                    const float *cz, const double *amp, const double *sigma,
                    int64_t nd, const float *sensors, int64_t nt, double dt,
                    double t0, double v, double nsig, const double *delta,
                    double *ga, double *gsig) {
  int64_t k;
#pragma omp parallel for schedule(static)
  for (k = 0; k < m; ++k) {
    double sg = (double)sigma[k];
    double half = nsig * sg;
    double acc_a = 0.0, acc_s = 0.0;
    for (int64_t j = 0; j < nd; ++j) {
      const float *s = sensors + 3 * j;
      double r = pair_distance(s, cx[k], cy[k], cz[k]);
      int64_t lo, hi;
      candidate_range(r, half, v, dt, t0, nt, &lo, &hi);
      for (int64_t n = lo; n <= hi; ++n) {
        double t = t0 + (double)n * dt;
        double d = r - v * t;
        if (fabs(d) <= half) {
          double e = exp(-(d * d) / (2.0 * sg * sg));
          double dl = delta[j * nt + n];
          acc_a += dl * d * e / (2.0 * r);
          acc_s += dl * d * d * d * e / (2.0 * r);
        }
      }
    }
    ga[k] = acc_a;
    if (gsig) gsig[k] = acc_s * (double)amp[k] / (sg * sg * sg);
  }
}

/*
 * Gradient with respect to the kernel centres (learnable centres, named as
 * future work in the paper's Discussion): the derivative of
 * Eq. (single_forward) through r = |s - c_k| at fixed window membership (the
 * indicator is locally constant in c_k, as it is in sigma_k):
 *   dp/dr  = A e / (2r) * (1 - d^2 / sigma^2 - d / r),
 *   dr/dc_k = (c_k - s) / r,
 *   gc[k]  = sum_j sum_{n in W} delta_j[n] dp/dr (c_k - s_j) / r.
 * delta float64 [nd][nt]; gc float64 [m][3], overwritten.
 */
void oracle_adjoint_centres(int64_t m, const float *cx, const float *cy,
                            const float *cz, const double *amp,
                            const double *sigma, int64_t nd,
                            const float *sensors, int64_t nt, double dt,
                            double t0, double v, double nsig,
                            const double *delta, double *gc) {
  int64_t k;
#pragma omp parallel for schedule(static)
  for (k = 0; k < m; ++k) {
    double sg = (double)sigma[k];
    double half = nsig * sg;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < nd; ++j) {
      const float *s = sensors + 3 * j;
      double r = pair_distance(s, cx[k], cy[k], cz[k]);
      int64_t lo, hi;
      candidate_range(r, half, v, dt, t0, nt, &lo, &hi);
      double sum = 0.0;
      for (int64_t n = lo; n <= hi; ++n) {
        double t = t0 + (double)n * dt;
        double d = r - v * t;
        if (fabs(d) <= half) {
          double e = exp(-(d * d) / (2.0 * sg * sg));
          double dpdr = amp[k] * e / (2.0 * r) * (1.0 - d * d / (sg * sg) - d / r);
          sum += delta[j * nt + n] * dpdr;
        }
      }
      acc[0] += sum * ((double)cx[k] - (double)s[0]) / r;
      acc[1] += sum * ((double)cy[k] - (double)s[1]) / r;
      acc[2] += sum * ((double)cz[k] - (double)s[2]) / r;
    }
    gc[3 * k] = acc[0];
    gc[3 * k + 1] = acc[1];
    gc[3 * k + 2] = acc[2];
  }
}

/*
 * Number of in-window taps of every pair, summed (the work count the
 * benchmark reports), and the number of pairs with at least one tap.
 */
void oracle_count_taps(int64_t m, const float *cx, const float *cy,
                       const float *cz, const double *sigma, int64_t nd,
                       const float *sensors, int64_t nt, double dt, double t0,
                       double v, double nsig, int64_t *taps, int64_t *pairs) {
  int64_t total = 0, live = 0, j;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total, live)
  for (j = 0; j < nd; ++j) {
    const float *s = sensors + 3 * j;
    for (int64_t k = 0; k < m; ++k) {
      double r = pair_distance(s, cx[k], cy[k], cz[k]);
      double half = nsig * (double)sigma[k];
      int64_t lo, hi, c = 0;
      candidate_range(r, half, v, dt, t0, nt, &lo, &hi);
      for (int64_t n = lo; n <= hi; ++n) {
        double d = r - v * (t0 + (double)n * dt);
        if (fabs(d) <= half) ++c;
      }
      total += c;
      if (c) ++live;
    }
  }
  *taps = total;
  *pairs = live;
}

/* Threads the OpenMP loops above use (reported with CPU timings). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * ASSA operators (Methods, "Adaptive supersampling alignment"), written per
 * kernel-sensor pair: the composition of the projection onto the upsampled
 * grid, the transposed convolution with h and the decimation contributes,
 * for a pair with snapped index k = floor((r/v - t0) f_up + 0.5) on the
 * alpha-times finer grid, amp/r * h[alpha n - k] to every sample n with
 * |alpha n - k| <= K.  The adjoint is the transpose of the same sum.
 *   h[k] = 0.5 * d * exp(-d^2 / (2 sigma^2)),  d = -v k dt / alpha.
 * Pairs whose snapped index lies outside [0, alpha nt) contribute nothing
 * (the impulse grid has alpha nt points).
 */
static int64_t floor_div(int64_t a, int64_t b) {  /* b > 0 */
  int64_t q = a / b;
  if ((a % b) != 0 && a < 0) --q;
  return q;
}

static double *assa_kernel(double dt, double v, double sigma, int64_t alpha, int64_t K) {
  double *h = (double *)malloc(sizeof(double) * (size_t)(2 * K + 1));
  for (int64_t k = -K; k <= K; ++k) {
    double d = -v * (double)k * (dt / (double)alpha);
    h[k + K] = 0.5 * d * exp(-(d * d) / (2.0 * sigma * sigma));
  }
  return h;
}

static int64_t assa_index(double r, double v, double t0, double f_up) {
  return (int64_t)floor((r / v - t0) * f_up + 0.5);
}

void oracle_assa_forward(int64_t m, const float *cx, const float *cy, const float *cz,
                         const double *amp, int64_t nd, const float *sens, int64_t nt,
                         double dt, double t0, double v, double sigma, int64_t alpha,
                         int64_t K, double *y) {
  double *h = assa_kernel(dt, v, sigma, alpha, K);
  const double f_up = (double)alpha / dt;
  const int64_t ntu = alpha * nt;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t j = 0; j < nd; ++j) {
    double *yj = y + j * nt;
    for (int64_t n = 0; n < nt; ++n) yj[n] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      const double r = pair_distance(sens + 3 * j, cx[i], cy[i], cz[i]);
      const int64_t k = assa_index(r, v, t0, f_up);
      if (k < 0 || k >= ntu) continue;
      const double w = amp[i] / r;
      int64_t lo = -floor_div(-(k - K), alpha);  /* ceil((k - K) / alpha) */
      int64_t hi = floor_div(k + K, alpha);
      if (lo < 0) lo = 0;
      if (hi > nt - 1) hi = nt - 1;
      for (int64_t n = lo; n <= hi; ++n) yj[n] += w * h[alpha * n - k + K];
    }
  }
  free(h);
}

void oracle_assa_adjoint(int64_t m, const float *cx, const float *cy, const float *cz,
                         int64_t nd, const float *sens, int64_t nt, double dt, double t0,
                         double v, double sigma, int64_t alpha, int64_t K,
                         const double *delta, double *g) {
  double *h = assa_kernel(dt, v, sigma, alpha, K);
  const double f_up = (double)alpha / dt;
  const int64_t ntu = alpha * nt;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    double acc = 0.0;
    for (int64_t j = 0; j < nd; ++j) {
      const double r = pair_distance(sens + 3 * j, cx[i], cy[i], cz[i]);
      const int64_t k = assa_index(r, v, t0, f_up);
      if (k < 0 || k >= ntu) continue;
      int64_t lo = -floor_div(-(k - K), alpha);
      int64_t hi = floor_div(k + K, alpha);
      if (lo < 0) lo = 0;
      if (hi > nt - 1) hi = nt - 1;
      double s = 0.0;
      for (int64_t n = lo; n <= hi; ++n) s += h[alpha * n - k + K] * delta[j * nt + n];
      acc += s / r;
    }
    g[i] = acc;
  }
  free(h);
}

/* ------------------------------------------------------------------------
 * Anisotropic kernels (learnable anisotropic Gaussians, named as future work
 * in the paper's Discussion).  Kernel k has p0 = A_k exp(-(x - c_k)^T
 * Sigma_k^-1 (x - c_k) / 2) with Sigma_k symmetric positive definite, given
 * as six numbers (xx, yy, zz, xy, xz, yz).  Reading of the far field: the
 * detector's sphere is taken as flat across the kernel (the same far-field
 * step that keeps only the outgoing term in Eq. (single_forward)), so the
 * surface integral of p0 is the kernel's marginal along n = (s - c)/r:
 * 2 pi sqrt(det Sigma)/sigma_n exp(-d^2/(2 sigma_n^2)), sigma_n^2 = n^T Sigma
 * n, and Eq. (pa_wave) gives
 *     p = A sqrt(det Sigma)/sigma_n^3 * d/(2r) * exp(-d^2/(2 sigma_n^2)),
 * inside |d| <= n_sigma sigma_n.  With Sigma = sigma^2 I this is
 * Eq. (single_forward) exactly.
 * ------------------------------------------------------------------------ */

/* det and sigma_n^2 of one pair: q = u^T Sigma u / |u|^2 with u = s - c. */
static double aniso_det(const double *S) {
  double xx = S[0], yy = S[1], zz = S[2], xy = S[3], xz = S[4], yz = S[5];
  return xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
}

static double aniso_sn2(const double *S, double ux, double uy, double uz, double r2) {
  double q = S[0] * ux * ux + S[1] * uy * uy + S[2] * uz * uz +
             2.0 * (S[3] * ux * uy + S[4] * ux * uz + S[5] * uy * uz);
  return q / r2;
}

/* Forward: y[j*nt + n] = sum_k [|d| <= nsig sigma_n] p_k(s_j, t_n), p as
 * above.  sigma6 float64 [m][6]; y float64 [nd][nt], overwritten. */
void oracle_forward_aniso(int64_t m, const float *cx, const float *cy, const float *cz,
                          const double *amp, const double *sigma6, int64_t nd,
                          const float *sensors, int64_t nt, double dt, double t0, double v,
                          double nsig, double *y) {
  int64_t j;
#pragma omp parallel for schedule(dynamic, 1)
  for (j = 0; j < nd; ++j) {
    double *row = y + j * nt;
    for (int64_t n = 0; n < nt; ++n) row[n] = 0.0;
    const float *s = sensors + 3 * j;
    for (int64_t k = 0; k < m; ++k) {
      const double *S = sigma6 + 6 * k;
      double ux = (double)s[0] - (double)cx[k];
      double uy = (double)s[1] - (double)cy[k];
      double uz = (double)s[2] - (double)cz[k];
      double r2 = ux * ux + uy * uy + uz * uz;
      double r = sqrt(r2);
      double sn2 = aniso_sn2(S, ux, uy, uz, r2);
      double sn = sqrt(sn2);
      double half = nsig * sn;
      double a = amp[k] * sqrt(aniso_det(S)) / (sn2 * sn);
      int64_t lo, hi;
      candidate_range(r, half, v, dt, t0, nt, &lo, &hi);
      for (int64_t n = lo; n <= hi; ++n) {
        double t = t0 + (double)n * dt;
        double d = r - v * t;
        if (fabs(d) <= half) row[n] += a / (2.0 * r) * d * exp(-(d * d) / (2.0 * sn2));
      }
    }
  }
}

/* Adjoint and the gradient with respect to Sigma.  With w = sqrt(det)/
 * sigma_n^3 /(2r) and the window held fixed:
 *   gA[k] = sum_j sum_{n in W} delta w d e,
 *   dp/dSigma = p [Sigma^-1 / 2 + (d^2/(2 sigma_n^4) - 3/(2 sigma_n^2)) n n^T]
 * (d sqrt(det)/dSigma = sqrt(det) Sigma^-1 / 2, d sigma_n^2/dSigma = n n^T),
 * reported for the six parameters (xx, yy, zz, xy, xz, yz) of the symmetric
 * matrix: an off-diagonal parameter stands for two entries, so its gradient
 * is twice the matrix entry's.  delta float64 [nd][nt]; gA float64 [m];
 * gsig6 float64 [m][6] or NULL. */
void oracle_adjoint_aniso(int64_t m, const float *cx, const float *cy, const float *cz,
                          const double *amp, const double *sigma6, int64_t nd,
                          const float *sensors, int64_t nt, double dt, double t0, double v,
                          double nsig, const double *delta, double *ga, double *gsig6) {
  int64_t k;
#pragma omp parallel for schedule(static)
  for (k = 0; k < m; ++k) {
    const double *S = sigma6 + 6 * k;
    double det = aniso_det(S);
    double sq = sqrt(det);
    double acc_a = 0.0;
    double acc_n[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t j = 0; j < nd; ++j) {
      const float *s = sensors + 3 * j;
      double ux = (double)s[0] - (double)cx[k];
      double uy = (double)s[1] - (double)cy[k];
      double uz = (double)s[2] - (double)cz[k];
      double r2 = ux * ux + uy * uy + uz * uz;
      double r = sqrt(r2);
      double sn2 = aniso_sn2(S, ux, uy, uz, r2);
      double sn = sqrt(sn2);
      double half = nsig * sn;
      double w = sq / (sn2 * sn) / (2.0 * r);
      int64_t lo, hi;
      candidate_range(r, half, v, dt, t0, nt, &lo, &hi);
      double s1 = 0.0, s3 = 0.0;
      for (int64_t n = lo; n <= hi; ++n) {
        double t = t0 + (double)n * dt;
        double d = r - v * t;
        if (fabs(d) <= half) {
          double e = exp(-(d * d) / (2.0 * sn2));
          double dl = delta[j * nt + n];
          s1 += dl * d * e;
          s3 += dl * d * d * d * e;
        }
      }
      acc_a += w * s1;
      /* the n n^T part: A w [s3/(2 sn^4) - 3 s1/(2 sn^2)] n n^T */
      double g = w * (s3 / (2.0 * sn2 * sn2) - 3.0 * s1 / (2.0 * sn2)) / r2;
      acc_n[0] += g * ux * ux;
      acc_n[1] += g * uy * uy;
      acc_n[2] += g * uz * uz;
      acc_n[3] += g * ux * uy;
      acc_n[4] += g * ux * uz;
      acc_n[5] += g * uy * uz;
    }
    ga[k] = acc_a;
    if (gsig6) {
      double a = amp[k];
      double xx = S[0], yy = S[1], zz = S[2], xy = S[3], xz = S[4], yz = S[5];
      /* Sigma^-1 by cofactors */
      double i_xx = (yy * zz - yz * yz) / det, i_yy = (xx * zz - xz * xz) / det;
      double i_zz = (xx * yy - xy * xy) / det, i_xy = (xz * yz - xy * zz) / det;
      double i_xz = (xy * yz - xz * yy) / det, i_yz = (xy * xz - xx * yz) / det;
      double h = 0.5 * a * acc_a;  /* sum delta p times 1/2 */
      double *o = gsig6 + 6 * k;
      o[0] = h * i_xx + a * acc_n[0];
      o[1] = h * i_yy + a * acc_n[1];
      o[2] = h * i_zz + a * acc_n[2];
      o[3] = 2.0 * (h * i_xy + a * acc_n[3]);
      o[4] = 2.0 * (h * i_xz + a * acc_n[4]);
      o[5] = 2.0 * (h * i_yz + a * acc_n[5]);
    }
  }
}

/* Gradient of <forward_aniso, delta> with respect to the kernel centres at
 * fixed windows.  With u = s - c, r = |u|, n = u/r, sigma_n^2 = n^T Sigma n,
 * d = r - v t and p = A sqrt(det)/sigma_n^3 d/(2r) exp(-d^2/(2 sigma_n^2)):
 *   dp/dr (sigma_n held)  = A sqrt(det)/sigma_n^3 e/(2r) (1 - d^2/sigma_n^2 - d/r),
 *   dp/d(sigma_n^2)       = p (d^2/(2 sigma_n^4) - 3/(2 sigma_n^2)),
 *   dr/du = n,  d(sigma_n^2)/du = (2/r)(Sigma n - sigma_n^2 n),  du/dc = -I,
 * so gc[k] = -sum_j sum_{n in W} delta (dp/dr n + dp/d(sigma_n^2) (2/r)(Sigma n -
 * sigma_n^2 n)).  delta float64 [nd][nt]; gc float64 [m][3], overwritten. */
void oracle_adjoint_aniso_centres(int64_t m, const float *cx, const float *cy, const float *cz,
                                  const double *amp, const double *sigma6, int64_t nd,
                                  const float *sensors, int64_t nt, double dt, double t0,
                                  double v, double nsig, const double *delta, double *gc) {
  int64_t k;
#pragma omp parallel for schedule(static)
  for (k = 0; k < m; ++k) {
    const double *S = sigma6 + 6 * k;
    double sq = sqrt(aniso_det(S));
    double a = amp[k];
    double g[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < nd; ++j) {
      const float *s = sensors + 3 * j;
      double ux = (double)s[0] - (double)cx[k];
      double uy = (double)s[1] - (double)cy[k];
      double uz = (double)s[2] - (double)cz[k];
      double r2 = ux * ux + uy * uy + uz * uz;
      double r = sqrt(r2);
      double sn2 = aniso_sn2(S, ux, uy, uz, r2);
      double sn = sqrt(sn2);
      double half = nsig * sn;
      int64_t lo, hi;
      candidate_range(r, half, v, dt, t0, nt, &lo, &hi);
      double T0 = 0.0, T1 = 0.0, T2 = 0.0, T3 = 0.0;
      for (int64_t n = lo; n <= hi; ++n) {
        double t = t0 + (double)n * dt;
        double d = r - v * t;
        if (fabs(d) <= half) {
          double e = exp(-(d * d) / (2.0 * sn2));
          double dl = delta[j * nt + n] * e;
          T0 += dl;
          T1 += dl * d;
          T2 += dl * d * d;
          T3 += dl * d * d * d;
        }
      }
      double W0 = a * sq / (sn2 * sn) / (2.0 * r);
      double dpr = W0 * (T0 - T2 / sn2 - T1 / r);
      double dps = W0 * (T3 / (2.0 * sn2 * sn2) - 3.0 * T1 / (2.0 * sn2));
      double nx = ux / r, ny = uy / r, nz = uz / r;
      double Snx = S[0] * nx + S[3] * ny + S[4] * nz;
      double Sny = S[3] * nx + S[1] * ny + S[5] * nz;
      double Snz = S[4] * nx + S[5] * ny + S[2] * nz;
      double f = dps * 2.0 / r;
      g[0] -= dpr * nx + f * (Snx - sn2 * nx);
      g[1] -= dpr * ny + f * (Sny - sn2 * ny);
      g[2] -= dpr * nz + f * (Snz - sn2 * nz);
    }
    gc[3 * k + 0] = g[0];
    gc[3 * k + 1] = g[1];
    gc[3 * k + 2] = g[2];
  }
}
