/*
 * Plain FP64 CPU oracle for one smooth particle-mesh Ewald (SPME)
 * reciprocal-space step.  TEST INFRASTRUCTURE ONLY: the GPU product path never
 * links, loads or calls this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg do.
 *
 * The paper (§III.A, "Long-Range Pipeline") describes the step as: spread
 * each charge onto the 4x4x4 surrounding grid points with cardinal B-splines
 * (§III.A.1), forward 3D FFT, multiply by Green's function data, inverse 3D
 * FFT (§III.A.2), then interpolate forces from the potential grid with
 * B-spline derivatives (§III.A.3).  The paper does not print the equations;
 * they are those of the SPME method it cites (Essmann et al. 1995), and each
 * function below names the step it implements:
 *
 *   O1  fractional coordinates s = a*.r, wrapped into [0,1); u = K s,
 *       g = floor(u) mod K, w = u - floor(u)
 *   O2  cardinal B-splines M_n and their derivatives
 *   O3  charge grid Q(k) = sum_i q_i prod_a M_p(...)
 *   O4  B-spline moduli |b(m)|^2
 *   O5  F(m) = sum_k Q(k) exp(+2 pi i m.k/K)             (unnormalised)
 *   O6  G(m) = c B(m) exp(-pi^2 |m|^2/beta^2) / (pi V |m|^2),  G(0) = 0
 *       (m = sum_a mt_a a*_a with mt_a = m_a or m_a - K_a, |mt_a| <= K_a/2;
 *       a Nyquist index K_a/2 counts half as +K_a/2 and half as -K_a/2)
 *   O7  E = 1/2 sum_m G(m) |F(m)|^2
 *   O8  virial P_ab = 1/2 sum_m G|F|^2 (delta_ab - 2 (1 + pi^2|m|^2/beta^2)
 *                                        m_a m_b / |m|^2)
 *   O9  phi(k) = sum_m G(m) F(m) exp(-2 pi i m.k/K)       (unnormalised)
 *   O10 F_i = -q_i sum_k phi(k) grad_i [prod_a M_p(...)]
 *
 * Everything is single-threaded FP64 loops with no blocking or fusion, built
 * with -ffp-contract=off.  The brute-force Ewald sums at the end are the
 * textbook definitions used to pin the SPME result.
 */
#include "spme_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_PI 3.14159265358979323846264338327950288
#define ORC_MAXP 16

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------ */
/* Box geometry: reciprocal vectors a*_a with a*_a . a_b = delta_ab    */
/* (no factor 2 pi), and the cell volume V = a1 . (a2 x a3).          */
/* ------------------------------------------------------------------ */
static void cross3(const double *u, const double *v, double *w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}
static double dot3(const double *u, const double *v) {
  return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}

/* rec[3*a + c] = component c of a*_a. */
static int box_recip(const double box[9], double rec[9], double *vol) {
  double c[3];
  cross3(box + 3, box + 6, c);
  double V = dot3(box, c);
  if (!(fabs(V) > 0.0)) return -1;
  cross3(box + 3, box + 6, rec + 0);
  cross3(box + 6, box + 0, rec + 3);
  cross3(box + 0, box + 3, rec + 6);
  for (int i = 0; i < 9; ++i) rec[i] /= V;
  *vol = fabs(V);
  return 0;
}

static int imod(long a, int K) {
  long r = a % K;
  return (int)(r < 0 ? r + K : r);
}

/* ------------------------------------------------------------------ */
/* O2: cardinal B-splines.                                             */
/*   M_2(x) = 1 - |x - 1| on [0,2], zero elsewhere                     */
/*   M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1)        */
/*   M_n'(x) = M_{n-1}(x) - M_{n-1}(x - 1)                             */
/* ------------------------------------------------------------------ */
double orc_bspline_M(int n, double x) {
  if (n < 2) return 0.0;
  if (n == 2) return (x >= 0.0 && x <= 2.0) ? 1.0 - fabs(x - 1.0) : 0.0;
  return (x * orc_bspline_M(n - 1, x) + (n - x) * orc_bspline_M(n - 1, x - 1.0)) /
         (double)(n - 1);
}

int orc_bspline(int p, double w, double *theta, double *dtheta) {
  if (p < 3 || p > ORC_MAXP) return -1;
  for (int j = 0; j < p; ++j) {
    double x = w + (double)(p - 1 - j);
    if (theta) theta[j] = orc_bspline_M(p, x);
    if (dtheta) dtheta[j] = orc_bspline_M(p - 1, x) - orc_bspline_M(p - 1, x - 1.0);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* O4: |b(m)|^2 = 1 / | sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K) |^2 */
/* For odd p the denominator vanishes at m = K/2; that entry takes the */
/* mean of its two neighbours.                                         */
/* ------------------------------------------------------------------ */
int orc_moduli(int p, int K, double *bsq) {
  if (p < 3 || p > ORC_MAXP || K < 2) return -1;
  double *den = (double *)malloc(sizeof(double) * (size_t)K);
  for (int m = 0; m < K; ++m) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k <= p - 2; ++k) {
      double mk = orc_bspline_M(p, (double)(k + 1));
      double ang = 2.0 * ORC_PI * (double)m * (double)k / (double)K;
      sr += mk * cos(ang);
      si += mk * sin(ang);
    }
    den[m] = sr * sr + si * si;
  }
  for (int m = 0; m < K; ++m) {
    if (den[m] > 1e-10) {
      bsq[m] = 1.0 / den[m];
    } else {
      double a = 1.0 / den[(m + K - 1) % K], b = 1.0 / den[(m + 1) % K];
      bsq[m] = 0.5 * (a + b);
    }
  }
  free(den);
  return 0;
}

/* ------------------------------------------------------------------ */
/* O5/O9: unnormalised DFT  X_k = sum_j x_j exp(sign 2 pi i j k / n).  */
/* Recursive decimation in time by the smallest prime factor r of n:   */
/* the n-point sum splits into r interleaved n/r-point sums, which are */
/* recombined with the explicit phase factors of the definition.      */
/* ------------------------------------------------------------------ */
static int smallest_factor(int n) {
  for (int r = 2; r * r <= n; ++r)
    if (n % r == 0) return r;
  return n;
}

static void dft_rec(int n, const double complex *x, int xs, double complex *y, int sign) {
  if (n == 1) {
    y[0] = x[0];
    return;
  }
  int r = smallest_factor(n);
  int m = n / r;
  if (r == n) { /* prime length: the definition, directly */
    for (int k = 0; k < n; ++k) {
      double complex acc = 0.0;
      for (int j = 0; j < n; ++j) {
        double ang = 2.0 * ORC_PI * (double)(((long)j * k) % n) / (double)n;
        acc += x[(long)j * xs] * (cos(ang) + sign * sin(ang) * I);
      }
      y[k] = acc;
    }
    return;
  }
  /* sub-transform a holds sum_t x[a + r t] exp(sign 2 pi i t k / m) */
  double complex *sub = (double complex *)malloc(sizeof(double complex) * (size_t)n);
  for (int a = 0; a < r; ++a) dft_rec(m, x + (long)a * xs, xs * r, sub + (long)a * m, sign);
  for (int s = 0; s < r; ++s) {
    for (int k = 0; k < m; ++k) {
      int kk = k + m * s; /* output index */
      double complex acc = 0.0;
      for (int a = 0; a < r; ++a) {
        double ang = 2.0 * ORC_PI * (double)(((long)a * kk) % n) / (double)n;
        acc += sub[(long)a * m + k] * (cos(ang) + sign * sin(ang) * I);
      }
      y[kk] = acc;
    }
  }
  free(sub);
}

int orc_fft1d(int n, double *re, double *im, int sign) {
  if (n < 1 || (sign != 1 && sign != -1)) return -1;
  double complex *x = (double complex *)malloc(sizeof(double complex) * (size_t)n);
  double complex *y = (double complex *)malloc(sizeof(double complex) * (size_t)n);
  for (int j = 0; j < n; ++j) x[j] = re[j] + im[j] * I;
  dft_rec(n, x, 1, y, sign);
  for (int j = 0; j < n; ++j) {
    re[j] = creal(y[j]);
    im[j] = cimag(y[j]);
  }
  free(x);
  free(y);
  return 0;
}

/* Transform every line of the grid along one axis. */
static void fft_axis(int K1, int K2, int K3, double *re, double *im, int axis, int sign) {
  int K[3] = {K1, K2, K3};
  long stride[3] = {1, K1, (long)K1 * K2};
  int n = K[axis];
  int o1 = (axis == 0) ? 1 : 0, o2 = (axis == 2) ? 1 : 2; /* the other two axes */
  double *lr = (double *)malloc(sizeof(double) * (size_t)n);
  double *li = (double *)malloc(sizeof(double) * (size_t)n);
  for (int b = 0; b < K[o2]; ++b) {
    for (int a = 0; a < K[o1]; ++a) {
      long base = a * stride[o1] + b * stride[o2];
      for (int j = 0; j < n; ++j) {
        lr[j] = re[base + j * stride[axis]];
        li[j] = im[base + j * stride[axis]];
      }
      orc_fft1d(n, lr, li, sign);
      for (int j = 0; j < n; ++j) {
        re[base + j * stride[axis]] = lr[j];
        im[base + j * stride[axis]] = li[j];
      }
    }
  }
  free(lr);
  free(li);
}

int orc_fft3d(int K1, int K2, int K3, double *re, double *im, int sign) {
  if (K1 < 1 || K2 < 1 || K3 < 1 || (sign != 1 && sign != -1)) return -1;
  fft_axis(K1, K2, K3, re, im, 0, sign);
  fft_axis(K1, K2, K3, re, im, 1, sign);
  fft_axis(K1, K2, K3, re, im, 2, sign);
  return 0;
}

/* ------------------------------------------------------------------ */
/* O1: fractional coordinate of one atom along reciprocal vector a*.   */
/* ------------------------------------------------------------------ */
static void frac_coord(const double *r, const double *astar, int K, int *g, double *w) {
  double s = dot3(astar, r);
  s = s - floor(s);
  double u = (double)K * s;
  double fl = floor(u);
  int gi = (int)fl;
  *w = u - fl;
  if (gi >= K) gi -= K; /* s rounded up to 1.0: u == K, w == 0 */
  *g = gi;
}

/* ------------------------------------------------------------------ */
/* The full FP64 step, O1..O10.                                        */
/* ------------------------------------------------------------------ */
int orc_spme(const double *pos, const double *q, int N, const double box[9],
             int K1, int K2, int K3, int p, double beta, double coulomb,
             double *forces, double *ev, double *Q, double *phi, double *times) {
  if (N < 0 || K1 < 2 || K2 < 2 || K3 < 2 || p < 3 || p > ORC_MAXP || !(beta > 0.0))
    return -1;
  double rec[9], V;
  if (box_recip(box, rec, &V)) return -1;
  int K[3] = {K1, K2, K3};
  long ng = (long)K1 * K2 * K3;
  double t0 = now_s();

  /* O1 + O2: per atom and axis the base index g and the p weights. */
  int *gidx = (int *)malloc(sizeof(int) * 3 * (size_t)(N > 0 ? N : 1));
  double *th = (double *)malloc(sizeof(double) * 3 * (size_t)p * (size_t)(N > 0 ? N : 1));
  double *dth = (double *)malloc(sizeof(double) * 3 * (size_t)p * (size_t)(N > 0 ? N : 1));
  for (int i = 0; i < N; ++i) {
    for (int a = 0; a < 3; ++a) {
      double w;
      frac_coord(pos + 3 * i, rec + 3 * a, K[a], &gidx[3 * i + a], &w);
      orc_bspline(p, w, th + ((long)3 * i + a) * p, dth + ((long)3 * i + a) * p);
    }
  }

  /* O3: Q(k) = sum_i q_i theta_1 theta_2 theta_3 over the p^3 points
   * g_a - p + 1 + j_a (mod K_a). */
  double *re = (double *)calloc((size_t)ng, sizeof(double));
  double *im = (double *)calloc((size_t)ng, sizeof(double));
  for (int i = 0; i < N; ++i) {
    const double *t1 = th + ((long)3 * i + 0) * p;
    const double *t2 = th + ((long)3 * i + 1) * p;
    const double *t3 = th + ((long)3 * i + 2) * p;
    for (int j3 = 0; j3 < p; ++j3) {
      int k3 = imod((long)gidx[3 * i + 2] - p + 1 + j3, K3);
      for (int j2 = 0; j2 < p; ++j2) {
        int k2 = imod((long)gidx[3 * i + 1] - p + 1 + j2, K2);
        for (int j1 = 0; j1 < p; ++j1) {
          int k1 = imod((long)gidx[3 * i + 0] - p + 1 + j1, K1);
          re[((long)k3 * K2 + k2) * K1 + k1] += q[i] * t1[j1] * t2[j2] * t3[j3];
        }
      }
    }
  }
  if (Q) memcpy(Q, re, sizeof(double) * (size_t)ng);
  double t1s = now_s();

  /* O5: F = forward transform with exp(+2 pi i m.k/K). */
  orc_fft3d(K1, K2, K3, re, im, +1);
  double t2s = now_s();

  /* O4 + O6..O8: influence function, energy and virial; F <- G F.
   * A Nyquist index m_a = K_a/2 (K_a even) aliases +K_a/2 and -K_a/2 equally;
   * its mode is split half and half between the two wave vectors, so G,
   * the energy and the virial of that mode are averages over the sign
   * choices (this keeps the off-diagonal virial symmetric under reflection;
   * in an orthorhombic cell only off-diagonal virial terms are affected). */
  double *bsq[3];
  for (int a = 0; a < 3; ++a) {
    bsq[a] = (double *)malloc(sizeof(double) * (size_t)K[a]);
    orc_moduli(p, K[a], bsq[a]);
  }
  double E = 0.0, P[6] = {0, 0, 0, 0, 0, 0};
  for (int m3 = 0; m3 < K3; ++m3) {
    for (int m2 = 0; m2 < K2; ++m2) {
      for (int m1 = 0; m1 < K1; ++m1) {
        long idx = ((long)m3 * K2 + m2) * K1 + m1;
        int m[3] = {m1, m2, m3};
        int mt[3], nyq[3], nq = 0;
        for (int a = 0; a < 3; ++a) {
          mt[a] = (m[a] <= K[a] / 2) ? m[a] : m[a] - K[a];
          nyq[a] = (K[a] % 2 == 0 && 2 * m[a] == K[a]);
          nq += nyq[a];
        }
        double G = 0.0;
        if (m1 != 0 || m2 != 0 || m3 != 0) {
          double B = bsq[0][m1] * bsq[1][m2] * bsq[2][m3];
          double f2 = re[idx] * re[idx] + im[idx] * im[idx];
          int nvar = 1 << nq;
          for (int v = 0; v < nvar; ++v) {
            double ms[3];
            for (int a = 0, bit = 0; a < 3; ++a) {
              ms[a] = mt[a];
              if (nyq[a]) {
                if ((v >> bit) & 1) ms[a] = -ms[a];
                ++bit;
              }
            }
            double mv[3];
            for (int c = 0; c < 3; ++c)
              mv[c] = ms[0] * rec[0 + c] + ms[1] * rec[3 + c] + ms[2] * rec[6 + c];
            double msq = dot3(mv, mv);
            double Gv = coulomb * B * exp(-ORC_PI * ORC_PI * msq / (beta * beta)) /
                        (ORC_PI * V * msq) / nvar;
            double e = 0.5 * Gv * f2;
            double fac = 2.0 * (1.0 + ORC_PI * ORC_PI * msq / (beta * beta)) / msq;
            G += Gv;
            E += e;
            P[0] += e * (1.0 - fac * mv[0] * mv[0]);
            P[1] += e * (1.0 - fac * mv[1] * mv[1]);
            P[2] += e * (1.0 - fac * mv[2] * mv[2]);
            P[3] += e * (0.0 - fac * mv[0] * mv[1]);
            P[4] += e * (0.0 - fac * mv[0] * mv[2]);
            P[5] += e * (0.0 - fac * mv[1] * mv[2]);
          }
        }
        re[idx] *= G;
        im[idx] *= G;
      }
    }
  }
  double t3s = now_s();

  /* O9: phi = inverse transform with exp(-2 pi i m.k/K); real by symmetry. */
  orc_fft3d(K1, K2, K3, re, im, -1);
  if (phi) memcpy(phi, re, sizeof(double) * (size_t)ng);
  double t4s = now_s();

  /* O10: F_i = -q_i sum phi(k) [dth1 th2 th3 K1 a*_1 + th1 dth2 th3 K2 a*_2
   *                             + th1 th2 dth3 K3 a*_3]. */
  if (forces) {
    for (int i = 0; i < N; ++i) {
      const double *a1 = th + ((long)3 * i + 0) * p, *d1 = dth + ((long)3 * i + 0) * p;
      const double *a2 = th + ((long)3 * i + 1) * p, *d2 = dth + ((long)3 * i + 1) * p;
      const double *a3 = th + ((long)3 * i + 2) * p, *d3 = dth + ((long)3 * i + 2) * p;
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int j3 = 0; j3 < p; ++j3) {
        int k3 = imod((long)gidx[3 * i + 2] - p + 1 + j3, K3);
        for (int j2 = 0; j2 < p; ++j2) {
          int k2 = imod((long)gidx[3 * i + 1] - p + 1 + j2, K2);
          for (int j1 = 0; j1 < p; ++j1) {
            int k1 = imod((long)gidx[3 * i + 0] - p + 1 + j1, K1);
            double ph = re[((long)k3 * K2 + k2) * K1 + k1];
            s1 += d1[j1] * a2[j2] * a3[j3] * ph;
            s2 += a1[j1] * d2[j2] * a3[j3] * ph;
            s3 += a1[j1] * a2[j2] * d3[j3] * ph;
          }
        }
      }
      for (int c = 0; c < 3; ++c)
        forces[3 * i + c] = -q[i] * (s1 * K1 * rec[0 + c] + s2 * K2 * rec[3 + c] +
                                     s3 * K3 * rec[6 + c]);
    }
  }
  double t5s = now_s();

  if (ev) {
    ev[0] = E;
    for (int c = 0; c < 6; ++c) ev[1 + c] = P[c];
  }
  if (times) {
    times[0] = t1s - t0;
    times[1] = (t2s - t1s) + (t4s - t3s);
    times[2] = t3s - t2s;
    times[3] = t5s - t4s;
  }
  for (int a = 0; a < 3; ++a) free(bsq[a]);
  free(re);
  free(im);
  free(gidx);
  free(th);
  free(dth);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Quantised mirror of the fixed-point charge grid.                    */
/*                                                                     */
/* The GPU path accumulates charge in 64-bit fixed point so that the   */
/* grid does not depend on summation order.  Its result is reproducible*/
/* bit for bit only under one fixed arithmetic recipe, restated here:  */
/*  Q1 per axis s = x * (1.0/L) in FP64 (diagonal box) or, for a      */
/*     general cell, s = a*_a . r = (a*_a0 r0 + a*_a1 r1) + a*_a2 r2    */
/*     with a*_a from box_recip; s -= floor(s), u = K s,               */
/*     g = floor(u) mod K, w = u - floor(u) (exact), w32 = (float)w    */
/*  Q2 q32 = (float)q                                                  */
/*  Q3 single-precision B-spline recursion (orc_mirror_spline)         */
/*  Q4 c = ((q32 * th_z) * th_y) * th_x in float, that order           */
/*  Q5 c_int = round-half-even((double)c * 2^F) as int64               */
/*  Q6 Q_int(k) = sum of c_int, two's complement                       */
/*  Q7 Q32(k) = (float)((double)Q_int(k) * 2^-F)                       */
/* ------------------------------------------------------------------ */

/* Q3.  d_n[j] = M_n(w + n - 1 - j).  d_2 = {1 - w, w}; for n = 3..p:
 *   d_n[j] = ((w + (n-1-j)) d_{n-1}[j-1] + ((j+1) - w) d_{n-1}[j]) * c_n
 * with c_n = (float)(1/(n-1)) and out-of-range d_{n-1} entries taken as 0;
 * the derivative uses the order-(p-1) array: dth[j] = d_{p-1}[j-1] - d_{p-1}[j]. */
int orc_mirror_spline(int p, float w, float *theta, float *dtheta) {
  if (p < 3 || p > ORC_MAXP) return -1;
  float d[ORC_MAXP + 1], e[ORC_MAXP + 1];
  d[0] = 1.0f - w;
  d[1] = w;
  for (int n = 3; n <= p; ++n) {
    if (n == p && dtheta) {
      for (int j = 0; j < p; ++j) {
        float lo = (j >= 1) ? d[j - 1] : 0.0f;
        float hi = (j <= p - 2) ? d[j] : 0.0f;
        dtheta[j] = lo - hi;
      }
    }
    float c = 1.0f / (float)(n - 1);
    for (int j = 0; j < n; ++j) {
      float t1 = (j >= 1) ? (w + (float)(n - 1 - j)) * d[j - 1] : 0.0f;
      float t2 = (j <= n - 2) ? ((float)(j + 1) - w) * d[j] : 0.0f;
      e[j] = (t1 + t2) * c;
    }
    for (int j = 0; j < n; ++j) d[j] = e[j];
  }
  if (theta)
    for (int j = 0; j < p; ++j) theta[j] = d[j];
  return 0;
}

int orc_mirror_grid(const double *pos, const double *q, int N, const double box[9],
                    int K1, int K2, int K3, int p, int frac_bits, int64_t *Qint,
                    float *Q32) {
  if (N < 0 || K1 < 2 || K2 < 2 || K3 < 2 || p < 3 || p > ORC_MAXP) return -1;
  if (frac_bits < 1 || frac_bits > 52) return -1;
  int diag = box[1] == 0.0 && box[2] == 0.0 && box[3] == 0.0 && box[5] == 0.0 &&
             box[6] == 0.0 && box[7] == 0.0;
  double invL[3] = {0.0, 0.0, 0.0}, rec[9], V;
  if (diag) {
    double L[3] = {box[0], box[4], box[8]};
    if (!(L[0] > 0.0 && L[1] > 0.0 && L[2] > 0.0)) return -1;
    for (int a = 0; a < 3; ++a) invL[a] = 1.0 / L[a];
  } else if (box_recip(box, rec, &V)) {
    return -1;
  }
  int K[3] = {K1, K2, K3};
  long ng = (long)K1 * K2 * K3;
  double scale = ldexp(1.0, frac_bits);
  uint64_t *acc = (uint64_t *)calloc((size_t)ng, sizeof(uint64_t));
  int status = 0;
  for (int i = 0; i < N; ++i) {
    int g[3];
    float w32[3];
    int ok = isfinite(q[i]);
    for (int a = 0; a < 3; ++a) ok = ok && isfinite(pos[3 * i + a]);
    if (!ok) { status = -2; continue; }
    for (int a = 0; a < 3; ++a) {
      double s = diag ? pos[3 * i + a] * invL[a] : dot3(rec + 3 * a, pos + 3 * i);
      s = s - floor(s);
      double u = s * (double)K[a];
      double fl = floor(u);
      int gi = (int)fl;
      double w = u - fl;
      if (gi >= K[a]) gi -= K[a];
      g[a] = gi;
      w32[a] = (float)w;
    }
    float q32 = (float)q[i];
    float tx[ORC_MAXP], ty[ORC_MAXP], tz[ORC_MAXP];
    orc_mirror_spline(p, w32[0], tx, NULL);
    orc_mirror_spline(p, w32[1], ty, NULL);
    orc_mirror_spline(p, w32[2], tz, NULL);
    for (int j3 = 0; j3 < p; ++j3) {
      int k3 = imod((long)g[2] - p + 1 + j3, K3);
      float cz = q32 * tz[j3];
      for (int j2 = 0; j2 < p; ++j2) {
        int k2 = imod((long)g[1] - p + 1 + j2, K2);
        float cy = cz * ty[j2];
        for (int j1 = 0; j1 < p; ++j1) {
          int k1 = imod((long)g[0] - p + 1 + j1, K1);
          float c = cy * tx[j1];
          int64_t ci = (int64_t)llrint((double)c * scale);
          acc[((long)k3 * K2 + k2) * K1 + k1] += (uint64_t)ci;
        }
      }
    }
  }
  double inv_scale = ldexp(1.0, -frac_bits);
  for (long k = 0; k < ng; ++k) {
    int64_t v = (int64_t)acc[k];
    if (Qint) Qint[k] = v;
    if (Q32) Q32[k] = (float)((double)v * inv_scale);
  }
  free(acc);
  return status;
}

/* ------------------------------------------------------------------ */
/* Brute-force Ewald reciprocal sum (the quantity SPME approximates):  */
/*   S(m) = sum_j q_j exp(2 pi i m.r_j),  m = sum_a m_a a*_a           */
/*   E = c/(2 pi V) sum_{m != 0} exp(-pi^2 m^2/beta^2)/m^2 |S(m)|^2    */
/*   F_i = (2 c q_i / V) sum_m exp(-pi^2 m^2/beta^2)/m^2 m             */
/*                             Im[exp(2 pi i m.r_i) conj(S(m))]        */
/*   virial as O8 with G = c exp(-pi^2 m^2/beta^2)/(pi V m^2), B = 1.  */
/* ------------------------------------------------------------------ */
int orc_ewald_recip(const double *pos, const double *q, int N, const double box[9],
                    double beta, double coulomb, int mmax, double *forces, double *ev) {
  if (N < 0 || mmax < 0 || !(beta > 0.0)) return -1;
  double rec[9], V;
  if (box_recip(box, rec, &V)) return -1;
  double *sfrac = (double *)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
  for (int i = 0; i < N; ++i)
    for (int a = 0; a < 3; ++a) sfrac[3 * i + a] = dot3(rec + 3 * a, pos + 3 * i);
  if (forces)
    for (int i = 0; i < 3 * N; ++i) forces[i] = 0.0;
  double E = 0.0, P[6] = {0, 0, 0, 0, 0, 0};
  double *cs = (double *)malloc(sizeof(double) * 2 * (size_t)(N > 0 ? N : 1));
  for (int m1 = -mmax; m1 <= mmax; ++m1)
    for (int m2 = -mmax; m2 <= mmax; ++m2)
      for (int m3 = -mmax; m3 <= mmax; ++m3) {
        if (m1 == 0 && m2 == 0 && m3 == 0) continue;
        double mv[3];
        for (int c = 0; c < 3; ++c) mv[c] = m1 * rec[0 + c] + m2 * rec[3 + c] + m3 * rec[6 + c];
        double msq = dot3(mv, mv);
        double f = exp(-ORC_PI * ORC_PI * msq / (beta * beta)) / msq;
        double Sr = 0.0, Si = 0.0;
        for (int j = 0; j < N; ++j) {
          double ph = 2.0 * ORC_PI *
                      (m1 * sfrac[3 * j] + m2 * sfrac[3 * j + 1] + m3 * sfrac[3 * j + 2]);
          cs[2 * j] = cos(ph);
          cs[2 * j + 1] = sin(ph);
          Sr += q[j] * cs[2 * j];
          Si += q[j] * cs[2 * j + 1];
        }
        double s2 = Sr * Sr + Si * Si;
        double e = coulomb / (2.0 * ORC_PI * V) * f * s2;
        double fac = 2.0 * (1.0 + ORC_PI * ORC_PI * msq / (beta * beta)) / msq;
        E += e;
        P[0] += e * (1.0 - fac * mv[0] * mv[0]);
        P[1] += e * (1.0 - fac * mv[1] * mv[1]);
        P[2] += e * (1.0 - fac * mv[2] * mv[2]);
        P[3] += e * (0.0 - fac * mv[0] * mv[1]);
        P[4] += e * (0.0 - fac * mv[0] * mv[2]);
        P[5] += e * (0.0 - fac * mv[1] * mv[2]);
        if (forces) {
          for (int i = 0; i < N; ++i) {
            /* Im[(c + i s)(Sr - i Si)] = s Sr - c Si */
            double imv = cs[2 * i + 1] * Sr - cs[2 * i] * Si;
            double a = 2.0 * coulomb * q[i] / V * f * imv;
            for (int c = 0; c < 3; ++c) forces[3 * i + c] += a * mv[c];
          }
        }
      }
  if (ev) {
    ev[0] = E;
    for (int c = 0; c < 6; ++c) ev[1 + c] = P[c];
  }
  free(cs);
  free(sfrac);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Ewald real-space sum and self term (harness for absolute checks).   */
/*   E_real = (c/2) sum_{i,j,n}' q_i q_j erfc(beta r)/r,               */
/*            r = |r_i - r_j + n|, n = n1 a1 + n2 a2 + n3 a3,          */
/*            the prime dropping i == j at n == 0                      */
/*   E_self = -c beta/sqrt(pi) sum_i q_i^2                             */
/* ------------------------------------------------------------------ */
/* The real-space terms of atom i: its pair energies added to *E (each pair
 * term halved, in the order j, n1, n2, n3) and its force added to f[3]
 * (when f is not NULL). */
static void real_terms_of(int i, const double *pos, const double *q, int N, const double box[9],
                          double beta, double coulomb, int nimg, double rcut, double *E,
                          double *f) {
  for (int j = 0; j < N; ++j) {
    for (int n1 = -nimg; n1 <= nimg; ++n1)
      for (int n2 = -nimg; n2 <= nimg; ++n2)
        for (int n3 = -nimg; n3 <= nimg; ++n3) {
          if (i == j && n1 == 0 && n2 == 0 && n3 == 0) continue;
          double d[3];
          for (int c = 0; c < 3; ++c)
            d[c] = pos[3 * i + c] - pos[3 * j + c] + n1 * box[0 + c] + n2 * box[3 + c] +
                   n3 * box[6 + c];
          double r = sqrt(dot3(d, d));
          if (rcut > 0.0 && r > rcut) continue;
          *E += 0.5 * coulomb * q[i] * q[j] * erfc(beta * r) / r;
          if (f) {
            double a = coulomb * q[i] * q[j] *
                       (erfc(beta * r) / (r * r) +
                        2.0 * beta / sqrt(ORC_PI) * exp(-beta * beta * r * r) / r) /
                       r;
            for (int c = 0; c < 3; ++c) f[c] += a * d[c];
          }
        }
  }
}

int orc_ewald_real(const double *pos, const double *q, int N, const double box[9],
                   double beta, double coulomb, int nimg, double rcut, double *forces,
                   double *e_real, double *e_self) {
  if (N < 0 || nimg < 0 || !(beta > 0.0)) return -1;
  double E = 0.0, S = 0.0;
  if (forces)
    for (int i = 0; i < 3 * N; ++i) forces[i] = 0.0;
  for (int i = 0; i < N; ++i) {
    S += q[i] * q[i];
    real_terms_of(i, pos, q, N, box, beta, coulomb, nimg, rcut, &E,
                  forces ? forces + 3 * i : NULL);
  }
  if (e_real) *e_real = E;
  if (e_self) *e_self = -coulomb * beta / sqrt(ORC_PI) * S;
  return 0;
}

/* Real-space forces on the listed atoms only (the rows of orc_ewald_real's
 * forces for those atoms, same arithmetic): checks of large systems on a
 * sample of atoms. */
int orc_ewald_real_atoms(const double *pos, const double *q, int N, const double box[9],
                         double beta, double coulomb, int nimg, double rcut, const int *atoms,
                         int n_atoms, double *forces) {
  if (N < 0 || nimg < 0 || !(beta > 0.0) || n_atoms < 0) return -1;
  for (int k = 0; k < n_atoms; ++k) {
    if (atoms[k] < 0 || atoms[k] >= N) return -1;
    double E = 0.0;
    for (int c = 0; c < 3; ++c) forces[3 * k + c] = 0.0;
    real_terms_of(atoms[k], pos, q, N, box, beta, coulomb, nimg, rcut, &E, forces + 3 * k);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Exclusion correction of the Ewald sum.  For a pair whose direct     */
/* interaction is excluded (e.g. atoms of one molecule), the Ewald     */
/* terms still carry it: erfc(beta r)/r in the real-space sum when     */
/* r <= rcut, erf(beta r)/r in the reciprocal sum.  The correction     */
/* removes both for the minimum-image distance r of the pair:          */
/*   E_excl = -(c/2) sum_i sum_{j in excl(i)} q_i q_j                  */
/*            [erf(beta r)/r + (r <= rcut ? erfc(beta r)/r : 0)]       */
/* over symmetric lists (each pair appears in both atoms' lists).      */
/* Orthorhombic (diagonal) boxes; rcut <= 0 means no cutoff.           */
/* ------------------------------------------------------------------ */
int orc_ewald_excl(const double *pos, const double *q, int N, const double box[9],
                   double beta, double coulomb, double rcut, const int *excl_off,
                   const int *excl_idx, double *forces, double *e_excl) {
  if (N < 0 || !(beta > 0.0)) return -1;
  if (box[1] != 0.0 || box[2] != 0.0 || box[3] != 0.0 || box[5] != 0.0 || box[6] != 0.0 ||
      box[7] != 0.0)
    return -1;
  double L[3] = {box[0], box[4], box[8]};
  double E = 0.0;
  if (forces)
    for (int i = 0; i < 3 * N; ++i) forces[i] = 0.0;
  for (int i = 0; i < N; ++i) {
    for (int k = excl_off[i]; k < excl_off[i + 1]; ++k) {
      int j = excl_idx[k];
      if (j < 0 || j >= N || j == i) return -1;
      double d[3];
      for (int c = 0; c < 3; ++c) {
        d[c] = pos[3 * i + c] - pos[3 * j + c];
        d[c] -= L[c] * nearbyint(d[c] / L[c]);
      }
      double r = sqrt(dot3(d, d));
      int inside = !(rcut > 0.0) || r <= rcut;
      /* energy of the removed interaction, and -dE/dr of it */
      double u = inside ? 1.0 / r : erf(beta * r) / r;
      double du = inside ? -1.0 / (r * r)
                         : (2.0 * beta / sqrt(ORC_PI) * exp(-beta * beta * r * r) - erf(beta * r) / r) / r;
      E -= 0.5 * coulomb * q[i] * q[j] * u;
      if (forces) {
        /* F_i = -dE/dr_i with E_pair = -c q_i q_j u(r) (counted from i's list and j's) */
        double a = coulomb * q[i] * q[j] * du / r;
        for (int c = 0; c < 3; ++c) forces[3 * i + c] += a * d[c];
      }
    }
  }
  if (e_excl) *e_excl = E;
  return 0;
}
