/*
 * qmcjastrow — one- and two-body Jastrow factors with 1D cubic B-spline
 * functors, and distance-table rows, on MI355X (gfx950).  Part of the same
 * library as qmcspline.h (libqmcspline.so); same conventions: plain
 * pointers, "device" = HIP device memory, `stream` = hipStream_t as void*,
 * status SPL_OK or a negative SPL_E* code with spline_last_error().
 *
 * What is computed (Mathuriya et al., SC'17):
 *  - Section 3, the Jastrow equation: J = sum_I sum_i U_{s(I)}(|r_I - r_i|)
 *    + sum_{i<j} U_2(|r_i - r_j|); the functors are one-dimensional cubic
 *    B-splines.  The ratio equations: moving electron k changes J by
 *    Delta J_1 + Delta J_2, the change of the terms that involve k.
 *  - Section 7 (DistTable, Jastrow; compute on the fly): the distance-table
 *    row of electron k (distances and displacements to all electrons and
 *    ions, structure-of-arrays) is computed when needed, and the Jastrow
 *    terms of a move are summed from it on the fly instead of being kept in
 *    N x N matrices.
 *
 * Readings (the paper gives no formulas for these):
 *  - Functor: M uniform intervals of width h = rcut/M on [0, rcut),
 *    coefficients c_0..c_{M+2}, coefficient j centred at r = (j-1) h,
 *    U(r) = sum_j c_j B(r/h - (j-1)) for r < rcut and 0 beyond (the cutoff
 *    branch); B is the centred cubic B-spline.
 *  - Two-body functors are spin-resolved: electrons 0..n_up-1 are up; equal
 *    spins use functor n_species, opposite spins functor n_species+1.
 *    One-body functor s serves ions of species s.
 *  - Pairs count once in J (which is what Delta J_2 implies).
 *  - Distances: minimum image in an orthorhombic cell; every cutoff must be
 *    <= half the shortest cell length, so no other image is ever inside one.
 *  - A pair at distance 0 adds U(0) to J and nothing to the derivatives.
 *  - Arithmetic in FP32 (the paper's mixed-precision DistTable and Jastrow);
 *    positions are FP32 structure-of-arrays.
 *
 * Electron positions: R_dev float; coordinate a (0 = x, 1 = y, 2 = z) of
 * electron i of walker w is R_dev[w*wstride + a*ld + i], ld >= n_elec,
 * wstride >= 3*ld.  A walker list (walkers[s]) must address walkers inside
 * the caller's buffer (the library does not know its extent); a negative
 * index gives NaN outputs for its slot, or is skipped by jastrow_accept.
 */
#ifndef QMCJASTROW_H
#define QMCJASTROW_H

#include <stddef.h>
#include <stdint.h>

#include "qmcspline.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_elec;    /* electrons per walker (>= 1) */
    int32_t n_up;      /* spin-up electrons, 0..n_elec */
    int32_t n_ion;     /* ions (>= 0) */
    int32_t n_species; /* ion species = one-body functors (1..16) */
    double cell[3];    /* orthorhombic cell lengths (> 0, finite) */
} jastrow_desc;

typedef struct jastrow_s jastrow_t;

/* Device bytes a Jastrow factor needs, or 0 on invalid arguments.
 * intervals[f] (1..256) for the n_species + 2 functors f. */
size_t jastrow_bytes(const jastrow_desc* d, const int32_t* intervals);

/* Creates a Jastrow factor.  Host inputs (read during the call only):
 *   ions      [n_ion][3] Cartesian positions (double)
 *   species   [n_ion] species index in [0, n_species)
 *   intervals [n_species+2], rcut [n_species+2] (0 < rcut <= min(cell)/2),
 *   coefs     the functors' coefficients, concatenated: intervals[f]+3 values
 *             per functor, in functor order (double; stored as float)
 * dev: caller-owned device buffer of >= jastrow_bytes() bytes, 256-byte
 * aligned, outliving the handle.  Synchronises `stream`.  SPL_EINVAL on any
 * invalid value (non-finite, out-of-range species, cutoff too long). */
int jastrow_create(const jastrow_desc* d, const double* ions, const int32_t* species, const int32_t* intervals,
                   const double* rcut, const double* coefs, void* dev, size_t bytes, void* stream,
                   jastrow_t** out);
int jastrow_destroy(jastrow_t* j);

/* A batch of proposed single-electron moves (Algorithm 1: ratio and
 * derivatives steps).  Slot s: walker w = walkers ? walkers[s] : s, electron
 * k = k_dev[s] in [0, n_elec), new position rnew[s] (device, [count][3]
 * double).  Out (device, [count][5] float): Delta J (J after minus J before
 * the move; the Jastrow ratio is exp(Delta J)), then grad_k J (x, y, z) and
 * lap_k J at the new position.  No distance row is stored: each pair term is
 * formed from the electron positions on the fly.  A slot with k out of range
 * gets NaN.  count == 0 is a no-op. */
int jastrow_move(const jastrow_t* j, const float* R_dev, int64_t ld, int64_t wstride, const int32_t* walkers,
                 const int32_t* k_dev, const double* rnew, int64_t count, float* out, void* stream);

/* Full evaluation for W walkers (the local energy's kinetic term needs every
 * electron's gradient and Laplacian).  Out (device): J [W] float,
 * G [W][3][n_elec] float (structure of arrays), L [W][n_elec] float. */
int jastrow_evaluate(const jastrow_t* j, const float* R_dev, int64_t ld, int64_t wstride, int64_t W, float* J,
                     float* G, float* L, void* stream);

/* Distance-table rows (Section 7: row k computed when needed) for positions
 * r[count][3] (device, double) against the electrons of walker
 * walkers[s] (or s) and against the ions: de [count][n_elec], dre
 * [count][3][n_elec], di [count][n_ion], dri [count][3][n_ion] (device,
 * float), with dr = r_other - r (minimum image) and d = |dr|.  di/dri may be
 * NULL when n_ion == 0. */
int jastrow_dist_rows(const jastrow_t* j, const float* R_dev, int64_t ld, int64_t wstride, const int32_t* walkers,
                      const double* r, int64_t count, float* de, float* dre, float* di, float* dri, void* stream);

/* Accepted moves: R[w][:, k] = rnew[s] for slot s (walkers/k as in
 * jastrow_move; slots with k out of range are skipped). */
int jastrow_accept(const jastrow_t* j, float* R_dev, int64_t ld, int64_t wstride, const int32_t* walkers,
                   const int32_t* k_dev, const double* rnew, int64_t count, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* QMCJASTROW_H */
