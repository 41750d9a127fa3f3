/*
 * Plain FP64 CPU oracle for one smooth particle-mesh Ewald (SPME)
 * reciprocal-space step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * shares no code with it (no headers, no tables, no helpers).
 *
 * What it computes follows the paper's long-range pipeline (§III.A: charge
 * spreading with 4x4x4 cardinal B-splines, forward 3D FFT, multiplication by
 * the Green's function, inverse 3D FFT, force interpolation with B-spline
 * derivatives) with the equations of the SPME method the paper cites in §I
 * and §II (Essmann et al., J. Chem. Phys. 103:8577, 1995).
 *
 * Conventions (all functions):
 *   - box[9] holds the three cell vectors as rows a1, a2, a3 (Angstrom).
 *   - grids are [K3][K2][K1] with index k1 fastest.
 *   - pos is [N][3] (Angstrom), q is [N] (e), forces [N][3].
 *   - ev[7] = { E, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz }, energies in coulomb*e^2/A.
 *   - return value 0 on success, negative on invalid arguments.
 */
#ifndef SPME_ORACLE_H
#define SPME_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Cardinal B-spline M_n(x) from its recursive definition. */
double orc_bspline_M(int n, double x);

/* theta[j] = M_p(w + p-1-j), dtheta[j] = M_p'(w + p-1-j), j = 0..p-1:
 * the weights of grid points g-p+1+j for an atom at g + w. */
int orc_bspline(int p, double w, double *theta, double *dtheta);

/* Squared B-spline moduli |b(m)|^2, m = 0..K-1. */
int orc_moduli(int p, int K, double *bsq);

/* Unnormalised complex DFT, in place, sign = +1 or -1 (e^{sign 2 pi i jk/n}). */
int orc_fft1d(int n, double *re, double *im, int sign);

/* Unnormalised 3D complex DFT of a [K3][K2][K1] grid, in place. */
int orc_fft3d(int K1, int K2, int K3, double *re, double *im, int sign);

/* Full FP64 SPME reciprocal step.  Any of forces/ev/Q/phi/times may be NULL.
 * times[4] receives seconds spent in spreading, forward+inverse FFT,
 * influence function (energy/virial), and interpolation. */
int orc_spme(const double *pos, const double *q, int N, const double box[9],
             int K1, int K2, int K3, int p, double beta, double coulomb,
             double *forces, double *ev, double *Q, double *phi,
             double *times);

/* Quantised mirror of the fixed-point charge grid: orthorhombic box only
 * (box must be diagonal).  Produces the int64 grid Q_int and, if Q32 is not
 * NULL, its single-precision image.  Returns -2 if a coordinate or charge is
 * not finite. */
int orc_mirror_grid(const double *pos, const double *q, int N,
                    const double box[9], int K1, int K2, int K3, int p,
                    int frac_bits, int64_t *Qint, float *Q32);

/* The single-precision B-spline recursion the mirror uses. */
int orc_mirror_spline(int p, float w, float *theta, float *dtheta);

/* Brute-force Ewald reciprocal sum over all integer m with |m_a| <= mmax,
 * m != 0.  forces / ev may be NULL. */
int orc_ewald_recip(const double *pos, const double *q, int N,
                    const double box[9], double beta, double coulomb,
                    int mmax, double *forces, double *ev);

/* Ewald real-space sum over periodic images |n_a| <= nimg (pairs with
 * distance > rcut are skipped; rcut <= 0 means no cutoff), plus the
 * self term returned separately.  forces may be NULL. */
int orc_ewald_real(const double *pos, const double *q, int N,
                   const double box[9], double beta, double coulomb,
                   int nimg, double rcut, double *forces, double *e_real,
                   double *e_self);

/* The real-space forces of orc_ewald_real on the n_atoms listed atoms only
 * (forces [n_atoms][3], same arithmetic as the full sum's rows). */
int orc_ewald_real_atoms(const double *pos, const double *q, int N, const double box[9],
                         double beta, double coulomb, int nimg, double rcut, const int *atoms,
                         int n_atoms, double *forces);

/* Exclusion correction: removes, for every excluded pair listed in the
 * symmetric CSR lists (excl_off[N+1], excl_idx), the erfc/r real-space part
 * (r <= rcut) and the erf/r reciprocal part of its Ewald interaction at the
 * minimum-image distance.  Diagonal boxes.  forces may be NULL. */
int orc_ewald_excl(const double *pos, const double *q, int N, const double box[9],
                   double beta, double coulomb, double rcut, const int *excl_off,
                   const int *excl_idx, double *forces, double *e_excl);

#ifdef __cplusplus
}
#endif

#endif
