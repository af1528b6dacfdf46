/*
 * qmcspline — periodic tricubic B-spline orbital evaluation on MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  "host" pointers are ordinary CPU
 * memory; "device" pointers are HIP device memory (for example the data
 * pointer of a torch tensor on a ROCm device); `stream` is a hipStream_t
 * passed as void* (NULL = the null stream).  The caller owns every buffer;
 * handles own host-side metadata only.  No exception crosses this boundary.
 *
 * Status codes: SPL_OK (0) or a negative SPL_E* value; after a non-zero
 * status, spline_last_error() returns a thread-local message.  Kernel
 * launches are asynchronous: a fault inside a kernel surfaces at the
 * caller's next synchronisation of that stream.
 *
 * Threads: evaluation calls only read a handle and may run concurrently on
 * one handle from several host threads; calls that change a handle (tile
 * setters, autotuners, spline_set_lattice, spline_destroy) must not overlap
 * any other call on that handle.  Autotuners that share a cache file should
 * not run at the same time (each appends one line per search).
 *
 * The method (Mathuriya et al., "Embracing a new era of highly efficient and
 * productive quantum Monte Carlo simulations", SC'17):
 *  - Section 3: each Slater matrix row A(i,j) = phi_i(r_j) needs all N
 *    orbitals at the proposed position r'_k, and the "derivatives" step of
 *    Algorithm 1 and the local-energy equation need their gradient and
 *    Laplacian; the non-local pseudopotential needs values at quadrature
 *    points.  One "orbital-VGL" is (V, Gx, Gy, Gz, L) of one orbital at one
 *    position.
 *  - Sections 2, 3 and 8.2: orbitals are stored as a read-only 3D cubic
 *    B-spline table indexed by three grid axes and the orbital ("4-dimensional"),
 *    periodic over the supercell (Table 1: FFT grids of whole unit cells).
 *  - Section 7.2: the table and its evaluation run in reduced precision while
 *    the precision-critical step (here the reduction of a position to a cell
 *    index and fractional offset) stays in double.
 *
 * Basis (the paper does not write it down): uniform cubic B-spline, tensor
 * product over three axes, coefficient j centred on grid point j*cell/n,
 * periodic wrap, lower cell at knots.  For an orthorhombic cell the
 * Laplacian is the sum of the three diagonal second derivatives.
 */
#ifndef QMCSPLINE_H
#define QMCSPLINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage type of the coefficient table.  FP64 and FP32 store c as is (FP32
 * rounded to nearest even).  BF16 and FP16 store q(c / s_m) with a
 * power-of-two per-orbital scale s_m = 2^ceil(log2 max_j |c_jm|) (1 for an
 * all-zero orbital), rounded to nearest even directly from FP64; FP16 keeps
 * subnormals.  Evaluation accumulates in FP32 (FP64 for SPL_F64) and
 * multiplies the five sums by s_m at the end.  The last two names only widen
 * the type to every int32 value, so that any value a caller passes is well
 * defined (and rejected with SPL_EINVAL unless it is one of the four). */
typedef enum {
    SPL_F64 = 0,
    SPL_F32 = 1,
    SPL_BF16 = 2,
    SPL_F16 = 3,
    SPL_DTYPE_LOW_ = -0x7fffffff - 1,
    SPL_DTYPE_HIGH_ = 0x7fffffff
} spline_dtype;

enum {
    SPL_OK = 0,
    SPL_EINVAL = -1,       /* null pointer, bad size or bad enum */
    SPL_ENOMEM = -2,       /* size overflow, or a caller buffer too small */
    SPL_EHIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
    SPL_EUNSUPPORTED = -4  /* valid request the library cannot serve (e.g. tile shape) */
};

/* Grid: n[d] >= 1 points per axis; cell[d] > 0, finite: orthorhombic cell
 * lengths (all 1.0 for a unit cube). */
typedef struct {
    int32_t n[3];
    double cell[3];
} spline_grid;

typedef struct spline_s spline_t;

/* Memory layout of a table in the device buffer, as chosen by this library.
 * The table holds (n0+3)(n1+3)(n2+3) rows: the grid plus a wrap-around halo
 * of one plane below and two above on each axis, so that the 4x4x4 stencil of
 * any cell is contiguous in z and needs no modulo.  A row holds the orbitals
 * of one grid point, orbital fastest, zero-padded to row_bytes. */
typedef struct {
    int64_t row_bytes;      /* bytes per grid point: a multiple of 256 when the
                               orbitals take more than 256 B, else of 64 (of 128
                               for FP64) */
    int64_t n_pad;          /* orbitals per row including zero padding */
    int64_t table_bytes;    /* rows * row_bytes, at offset 0 of the buffer */
    int64_t scales_offset;  /* byte offset of float scales[n_pad] (256-byte aligned) */
    int64_t total_bytes;    /* what spline_table_bytes returns */
    int32_t elem_bytes;     /* 8, 4, 2, 2 */
    int32_t padded[3];      /* n[d] + 3 */
} spline_layout;

/* Kernel tile shape.  A group of `lpp` lanes (16, 32 or 64) evaluates one
 * position; each lane loads `nch` chunks of `cw` 32-bit words per stencil
 * point, so a tile covers lpp*nch*cw*4 bytes of a row.  `pb` positions are
 * reduced to the lattice per workgroup and their weights staged in LDS. */
typedef struct {
    int32_t cw, nch, lpp, pb;
} spline_tile;

/* Bytes of device memory a table needs (table + scales), or 0 on invalid
 * arguments or size overflow. */
size_t spline_table_bytes(const spline_grid* grid, int32_t n_orb, spline_dtype store);

/* Fills *out with the layout for (grid, n_orb, store).  Host only. */
int spline_get_layout(const spline_grid* grid, int32_t n_orb, spline_dtype store, spline_layout* out);

/* Host-only packing: quantizes coefs_host ([n0][n1][n2][n_orb], FP64, orbital
 * fastest) to `store`, builds the halo layout and writes the scales, into a
 * host buffer of at least spline_table_bytes() bytes.  Used by
 * spline_create; exposed so the layout can be checked without a GPU.
 * A non-finite coefficient is rejected with SPL_EINVAL. */
int spline_pack_host(const spline_grid* grid, int32_t n_orb, const double* coefs_host,
                     spline_dtype store, void* host_buf, size_t buf_bytes);

/* Creates a table: packs coefs_host (caller-owned, only read during the
 * call) and copies it into table_dev (caller-owned device buffer of at least
 * spline_table_bytes() bytes, which must outlive the handle; 256-byte
 * alignment required).  Synchronises `stream` before returning.  The handle
 * starts with a default tile shape for (n_orb, store). */
int spline_create(const spline_grid* grid, int32_t n_orb, const double* coefs_host,
                  spline_dtype store, void* table_dev, size_t table_bytes, void* stream,
                  spline_t** out);

/* Value, gradient and Laplacian of all orbitals at B positions.
 *   pos_dev  device, [B][3] FP64 Cartesian positions (any finite value; wrapped
 *            periodically; a non-finite coordinate gives NaN outputs for that
 *            position, with no out-of-range access)
 *   V        device, [B][n_orb]
 *   G        device, [B][3][n_orb]   (x, y, z components, each orbital-contiguous)
 *   L        device, [B][n_orb]
 * Outputs are float (double when the table is SPL_F64).  Asynchronous on
 * `stream`; B == 0 is a no-op.  Output buffers must not overlap the table or
 * each other. */
int spline_eval_vgl(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                    void* stream);

/* Value only (the quadrature-point ratios of the non-local pseudopotential,
 * Section 3): V device [B][n_orb], same conventions as spline_eval_vgl. */
int spline_eval_v(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* stream);

/* Locality-ordered evaluation of a large batch (the GPU counterpart of the
 * table tiling of Section 8.4: positions, not the table, are reordered).
 * The positions are bucketed on the device by the block of grid cells they
 * fall in (blocks of 2^s cells per dimension, s chosen so there are at most
 * 32 blocks per dimension; blocks in Morton order), then evaluated in that
 * order, so positions that share table rows run together and re-read the
 * rows from cache instead of HBM.  Inputs, outputs and conventions are those
 * of spline_eval_vgl / spline_eval_v, and so are the results, bit for bit
 * (each output row is written by the same per-position arithmetic; only the
 * order of evaluation differs).  Pays when B is large against the grid (many
 * positions per table row); costs four small extra launches.
 *   workspace_dev  caller-owned device scratch, 256-byte aligned, at least
 *                  spline_sorted_workspace_bytes(s, B) bytes (0 for a NULL
 *                  handle or B outside [0, 2^31)); its contents on entry
 *                  do not matter and are overwritten.
 * For a general cell (after spline_set_lattice) spline_eval_vgl_sorted
 * sorts by the fractional coordinates and runs the general-cell kernel; the
 * value-only form is for orthorhombic cells (SPL_EUNSUPPORTED otherwise).
 * SPL_ENOMEM for a short workspace; B == 0 is a no-op.  Asynchronous on
 * `stream`; calls that share a workspace must not overlap. */
size_t spline_sorted_workspace_bytes(const spline_t* s, int64_t B);
int spline_eval_vgl_sorted(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                           void* workspace_dev, size_t workspace_bytes, void* stream);
int spline_eval_v_sorted(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* workspace_dev,
                         size_t workspace_bytes, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * spline_eval_vgl_sorted without a workspace argument.  Its scratch is a
 * static device array of 6.4 MB (the sort of up to 524288 positions), one
 * copy per GPU, created with the library's code object and held until the
 * process ends; its address is looked up on the first call on each device
 * (hipGetSymbolAddress, outside any capture the first time).  No hipMalloc,
 * hipFree or other allocating call.  B > 524288 gives SPL_ENOMEM; B == 0 is
 * a no-op.  Results equal spline_eval_vgl_sorted's bit for bit.  Every call
 * on one GPU shares that GPU's array: the bucket counts are cleared by a
 * kernel at the start of each call and the rest is overwritten before it is
 * read, but calls that overlap on one GPU (other streams, other host
 * threads) race on it. */
int spline_eval_vgl_sorted_noalloc(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                                   void* stream);
/* spline_eval_vgh in locality order (same arguments and results, bit for
 * bit), with the workspace above.  Its shape: 16-lane groups with the widest
 * chunk compiled for the storage type where it fits the row (else the
 * VGH-family tile's), at most 8 positions per workgroup; a general cell's
 * spline_eval_vgl_sorted uses the same.  spline_get_sorted_vgh_tile reads
 * it. */
int spline_eval_vgh_sorted(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* H,
                           void* workspace_dev, size_t workspace_bytes, void* stream);
int spline_get_sorted_vgh_tile(const spline_t* s, spline_tile* tile);
/* The fused determinant ratio in locality order: arguments and errors of
 * spline_eval_ratio_vgl / spline_eval_ratio_v, plus the workspace of
 * spline_eval_vgl_sorted.  Uses the sorted tile shape (the sorted value
 * tile for the ratio alone).  The order of the ratio's partial sums depends on the
 * tile shape, so the results equal those of the plain entry point run with
 * the same shape, bit for bit (and differ from other shapes by rounding). */
int spline_eval_ratio_vgl_sorted(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev,
                                 int64_t ld, const int32_t* rows_dev, void* D, void* workspace_dev,
                                 size_t workspace_bytes, void* stream);
int spline_eval_ratio_v_sorted(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev,
                               int64_t ld, const int32_t* rows_dev, void* R, void* workspace_dev,
                               size_t workspace_bytes, void* stream);
/* The locality-ordered paths have their own tile shapes: one for VGL and
 * one for value only and the value ratio (initially the plain VGL and value
 * shapes).  spline_set_sorted_tile sets both (the value shape when that
 * shape has a value-only kernel); spline_get_sorted_value_tile reads the
 * value shape.  spline_autotune_sorted works as spline_autotune over these
 * paths: it tunes both shapes (bitwise cross-check of every candidate; the
 * candidates also include 8 positions per workgroup), with cache keys
 * "<key> sorted" and "<key> sorted V", and returns the VGL shape. */
int spline_set_sorted_tile(spline_t* s, const spline_tile* tile);
int spline_get_sorted_tile(const spline_t* s, spline_tile* tile);
int spline_get_sorted_value_tile(const spline_t* s, spline_tile* tile);
int spline_autotune_sorted(spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                           void* workspace_dev, size_t workspace_bytes, int32_t reps, const char* cache_path,
                           void* stream, spline_tile* chosen);

/* Determinant ratio fused into the evaluation (Section 3: the ratio
 * equation and the matrix determinant lemma).  With A(i,j) = phi_i(r_j),
 * moving electron k to r'_k multiplies det A by sum_i Ainv(k,i) phi_i(r'_k),
 * the dot product of row k of A^-1 with the orbital values at the new
 * position; the same dot product with the orbital gradients and Laplacians
 * gives grad det(A') / det(A) and lap det(A') / det(A) (the "derivatives"
 * step of Algorithm 1).  The orbital values are consumed inside the kernel
 * and never written.
 *   pos_dev   device, [B][3] FP64 positions r' (conventions of spline_eval_vgl)
 *   ainv_dev  device; the row for position b is the n_orb elements starting
 *             at ainv_dev + (rows_dev ? rows_dev[b] : b) * ld, float (double
 *             for an SPL_F64 table), aligned to the element size.  For a
 *             sweep over all electrons of walkers stored as [walkers][n][n]
 *             inverses, rows_dev = NULL and ld = n_orb; for one electron k of
 *             every walker, ainv_dev = first inverse + k*n_orb, ld = n_orb^2;
 *             for quadrature points sharing an electron, rows_dev maps each
 *             point to its electron's row.  The rows must lie inside the
 *             caller's buffer (not checked).
 *   ld        elements between row indices 0 and 1 (>= 0)
 *   D         device, [B][5] (ratio_vgl): sum_i a_i V_i, sum_i a_i Gx_i,
 *             sum_i a_i Gy_i, sum_i a_i Gz_i, sum_i a_i L_i for the row a of
 *             position b; D[b][0] is det A'/det A, D[b][1..3]/D[b][0] the
 *             gradient of log det A' with respect to r', D[b][4]/D[b][0] its
 *             lap det(A')/det(A').  R device, [B] (ratio_v): the ratio only,
 *             for the quadrature points of the non-local pseudopotential.
 * Outputs float (double for SPL_F64); per-position sums are added in a fixed
 * order, so results are reproducible bit for bit for a given tile shape.
 * The handle's VGL (value) tile shape is used.  For a table with a general
 * cell (spline_set_lattice) the ratio with derivatives is formed by the
 * VGH-family kernel (the handle's VGH tile shape; Cartesian G and L from the
 * full Hessian) and the locality-ordered form uses the locality-ordered VGH
 * shape; the value ratio needs no derivatives and is the same kernel in any
 * cell.  Asynchronous on `stream`; B == 0 is a no-op.  SPL_EINVAL on NULL
 * pointers, ld < 0 or misaligned rows; SPL_EUNSUPPORTED when no ratio kernel
 * exists for the tile shape. */
int spline_eval_ratio_vgl(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev,
                          int64_t ld, const int32_t* rows_dev, void* D, void* stream);
int spline_eval_ratio_v(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev,
                        int64_t ld, const int32_t* rows_dev, void* R, void* stream);

/* Sherman-Morrison update of inverse Slater matrices after accepted moves
 * (Section 3: once the proposed r'_k is accepted, A^-1 is updated with the
 * Sherman-Morrison formula).  For each slot j in [0, count): walker
 * w = walkers_dev ? walkers_dev[j] : j, electron k = k_dev[j], and
 * phi = phi_dev + j*ld_phi, the n orbital values at the accepted position
 * (spline_eval_v gives them).  The n x n row-major inverse of walker w, at
 * ainv_dev + w*walker_stride elements, becomes the inverse of A with column k
 * replaced by phi:  t = A^-1 phi,  rho = t_k (the determinant ratio),
 * A^-1 <- A^-1 - (t - e_k)(row k of A^-1)/rho.  In place; every row is read
 * and written once (two launches: rows i != k, then row k).
 *   dtype       SPL_F32 or SPL_F64: element type of ainv and phi (the
 *               paper's mixed-precision code keeps A^-1 in single precision)
 *   n           orbitals = electrons of the determinant, with (2n+4) elements
 *               fitting in 64 KB of LDS (n <= 8190 FP32, 4094 FP64)
 *   walker_stride >= n*n; ld_phi >= n; pointers element-aligned
 * A slot with k outside [0, n) or a negative walker index leaves its walker
 * untouched; other walker indices must address inverses inside the caller's
 * buffer (the library does not know its extent).  Listing one walker twice in
 * a call races; rho == 0 (a move that
 * must not be accepted) gives non-finite entries.  Asynchronous on `stream`;
 * count == 0 is a no-op.  SPL_EINVAL on bad sizes or pointers. */
int spline_det_update(void* ainv_dev, int32_t n, int64_t walker_stride, const int32_t* walkers_dev,
                      const int32_t* k_dev, const void* phi_dev, int64_t ld_phi, int64_t count,
                      spline_dtype dtype, void* stream);

/* Delayed update of inverse Slater matrices (the Woodbury-identity scheme of
 * the paper's outlook: several accepted moves are evaluated before A^-1 is
 * updated, so the update becomes one rank-j product).  FP32; the inverses
 * are n x n row-major at ainv + w*walker_stride, as for spline_det_update.
 * Per walker the workspace keeps the pending moves: their orbital vectors
 * phi_l, electrons k_l, and S^-1 with S[i][l] = a_{k_i} . phi_l (a_i: rows of
 * the stale inverse).
 *   spline_dlu_workspace_bytes / spline_dlu_create: device workspace for
 *     `walkers` walkers, n orbitals (1..2048) and at most `delay` (1..64,
 *     <= n) pending moves; caller-owned, 256-byte aligned; create clears it
 *     (asynchronously on `stream`).  The handle holds host metadata only.
 *   spline_dlu_ratio: slot s (walker walkers[s] or s, electron k[s], orbital
 *     quantities of the proposed position V[s][n] and, optionally, G[s][3][n]
 *     and L[s][n] as written by spline_eval_vgl; with walkers == NULL,
 *     count <= walkers of the workspace, else SPL_EINVAL) gets
 *       a_k . q - t^T S^-1 y,  t_i = a_k . phi_i,  y_i = a_{k_i} . q,
 *     for q = V (out[count]) or q = V, Gx, Gy, Gz, L (out[count][5]): the
 *     determinant ratio and derivative sums against the current matrix.  k
 *     may be a pending electron of its walker: row k of the current inverse
 *     then carries the correction of its replaced column, t_i - [k_i == k].
 *     A slot with k or its walker out of range, or whose walker is marked
 *     (below), gets NaN.
 *   spline_dlu_accept: slots with k in [0, n) append their move (phi = V[s])
 *     and border S^-1 (the Schur complement is the ratio); k = -1 marks a
 *     rejected move, and a slot whose walker is out of range is skipped.  At
 *     most `delay` accept calls between flushes (SPL_EINVAL otherwise); a
 *     walker may appear once per call.  The pending electrons of a walker
 *     must be distinct: an accept of an electron that is already pending is
 *     not applied and marks the walker, whose ratios are NaN from then on (a
 *     flush keeps the mark; spline_dlu_create clears it) -- flush before
 *     moving an electron a second time.
 *   spline_dlu_accept_ratio: one call for the accept of the previous move
 *     (k_acc[s], V_acc[s], as spline_dlu_accept) followed by the ratio of the
 *     next proposal (k[s], V/G/L[s], as spline_dlu_ratio) in slot s, for a
 *     step loop that evaluates the next proposal's orbitals before the
 *     previous move's accept; results equal the two calls bit for bit, in
 *     one launch (two when S^-1 does not fit in LDS).  k_acc[s] < 0: nothing
 *     to accept.  If that accept is refused as a second move of a pending
 *     electron, the slot's ratio is NaN.
 *   spline_dlu_flush: A^-1 -= (A^-1 Phi - Q) S^-1 R for every walker (R: rows
 *     k_l of A^-1, Q: columns e_{k_l}), then no move is pending.  ainv must
 *     hold the inverses of all `walkers` walkers of the workspace.
 * All asynchronous on `stream`. */
typedef struct spline_dlu_s spline_dlu_t;
size_t spline_dlu_workspace_bytes(int32_t n, int32_t delay, int64_t walkers);
int spline_dlu_create(int32_t n, int32_t delay, int64_t walkers, void* ws_dev, size_t ws_bytes, void* stream,
                      spline_dlu_t** out);
int spline_dlu_destroy(spline_dlu_t* h);
int spline_dlu_ratio(const spline_dlu_t* h, const float* ainv_dev, int64_t walker_stride, const int32_t* walkers_dev,
                     const int32_t* k_dev, const float* V, const float* G, const float* L, int64_t count, float* out,
                     void* stream);
int spline_dlu_accept(spline_dlu_t* h, const float* ainv_dev, int64_t walker_stride, const int32_t* walkers_dev,
                      const int32_t* k_dev, const float* V, int64_t count, void* stream);
int spline_dlu_accept_ratio(spline_dlu_t* h, const float* ainv_dev, int64_t walker_stride,
                            const int32_t* walkers_dev, const int32_t* k_acc_dev, const float* V_acc,
                            const int32_t* k_dev, const float* V, const float* G, const float* L, int64_t count,
                            float* out, void* stream);
int spline_dlu_flush(spline_dlu_t* h, float* ainv_dev, int64_t walker_stride, void* stream);

/* General (triclinic) cells.
 *
 * spline_set_lattice gives the table a general cell.  lattice: host, 9
 * doubles, row-major; row d is the Cartesian lattice vector a_d along which
 * the n[d] grid points of axis d run (grid.cell is then ignored).  A position
 * r = sum_d u_d a_d is reduced through its fractional coordinates
 * u = r Lat^-1 in FP64, periodic with period 1 in each u_d.  Table 1's
 * graphite cell is hexagonal, for example.  SPL_EINVAL if the matrix is not
 * finite or is singular.  Host only; the table is not touched.  Afterwards
 * spline_eval_vgh, spline_eval_vgl (a general-cell kernel that forms the
 * Laplacian from the full Hessian), spline_eval_v, spline_eval_ratio_v,
 * spline_eval_ratio_vgl, their locality-ordered forms, plans and
 * spline_autotune (which then tunes the general-cell kernels) serve the
 * cell; the surrogate's spline fallback returns SPL_EUNSUPPORTED for such a
 * table (the surrogate's features are periodic in an orthorhombic cell).
 * spline_get_lattice returns it (diag(cell) for an orthorhombic table). */
int spline_set_lattice(spline_t* s, const double* lattice);
int spline_get_lattice(const spline_t* s, double* lattice);

/* Value, gradient and full Hessian of all orbitals (the paper's Bspline-vgh
 * kernel, Section 8; the Hessian is what a non-orthogonal cell needs for its
 * Laplacian).  For any table, orthorhombic or general.
 *   V device [B][n_orb], G device [B][3][n_orb] (Cartesian x, y, z),
 *   H device [B][6][n_orb]: Cartesian xx, xy, xz, yy, yz, zz.
 * Outputs float (double for SPL_F64); the ten grid-frame sums accumulate in
 * FP32 (FP64) and are mapped to Cartesian axes with the inverse lattice.
 * Conventions of spline_eval_vgl otherwise.  The VGH kernels have their own
 * tile shapes: spline_vgh_tile_candidates / spline_set_vgh_tile /
 * spline_get_vgh_tile, and spline_autotune_vgh times them all on a batch
 * (outputs of every candidate must agree bit for bit, else SPL_EUNSUPPORTED). */
int spline_eval_vgh(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* H,
                    void* stream);
int spline_vgh_tile_candidates(const spline_t* s, spline_tile* out, int32_t cap, int32_t* n);
int spline_set_vgh_tile(spline_t* s, const spline_tile* tile);
int spline_get_vgh_tile(const spline_t* s, spline_tile* tile);
int spline_autotune_vgh(spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* H,
                        int32_t reps, void* stream, spline_tile* chosen);

/* Tile shape control.  spline_tile_candidates lists the shapes valid for this
 * table (up to `cap`, count in *n); spline_set_tile validates and selects one. */
int spline_tile_candidates(const spline_t* s, spline_tile* out, int32_t cap, int32_t* n);
int spline_set_tile(spline_t* s, const spline_tile* tile);
int spline_get_tile(const spline_t* s, spline_tile* tile);

/* Autotuner: times every candidate tile shape on the given batch with HIP
 * events (`reps` timed launches each, after one warm-up), checks that every
 * candidate's outputs on the first positions are bit-identical to the first
 * candidate's, and selects the fastest, separately for VGL (written to
 * *chosen) and for value-only evaluation (read back with
 * spline_get_value_tile; the value-only and value-ratio kernels use it).
 * With a non-NULL cache_path, matching entries (key: device arch, grid,
 * n_orb, store, B bucket; " V" appended for value only) are used without
 * searching, and new results are appended; an unreadable or corrupt cache is
 * ignored.  cache_path == NULL takes the file named by the environment
 * variable QMCSPLINE_TUNE_CACHE when it is set and not empty (no cache
 * otherwise); the same holds for spline_autotune_sorted.  Outputs V/G/L are overwritten.  For a table with a general
 * lattice it tunes the general-cell VGL kernels instead (no cache). */
int spline_autotune(spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                    int32_t reps, const char* cache_path, void* stream, spline_tile* chosen);
int spline_get_value_tile(const spline_t* s, spline_tile* tile);

/* ---- Ragged multi-table plans --------------------------------------------
 * The walker population fluctuates from generation to generation and each
 * walker carries its own electrons (Section 6 and Algorithm 1: per-walker
 * loops over a variable N_w), and a workload may hold several tables; the
 * paper proposes tiling the large table and evaluating the tiles in parallel
 * (Section 8.4).  A plan evaluates B[t] positions of each of n_tabs tables
 * (same storage type, same device) in ONE persistent work-queue launch:
 * workgroups pop (table, position block) tasks from a device counter, widest
 * tables first.  The launch (a counter-reset kernel and the persistent
 * kernel) is captured once into a HIP graph at creation; every
 * spline_plan_launch is one graph launch.  The plan is bound to the given
 * position and output buffers (same shapes and element types as
 * spline_eval_vgl) and to the workspace; their contents may change between
 * launches, their addresses may not.  Concurrent launches of one plan race on
 * its workspace.  When a table has a general cell (spline_set_lattice) every
 * task of the plan runs the VGH-family kernel (the Laplacian from the full
 * Hessian; orthorhombic tables through their diagonal lattice, equal to
 * spline_eval_vgl within rounding) and the shapes are the VGH family's; a
 * general table's outputs equal its spline_eval_vgl under the plan's shape
 * bit for bit.  Otherwise every table's outputs equal its spline_eval_vgl
 * bit for bit. */
typedef struct spline_plan_s spline_plan_t;

/* Device workspace bytes a plan over these batch sizes needs (counter, table
 * descriptors, task list); 0 on invalid input. */
size_t spline_plan_workspace_bytes(int32_t n_tabs, const int64_t* B_per_tab);

/* Creates a plan.  tabs[n_tabs]: handles (not owned); B_per_tab[t] >= 0;
 * pos_dev[t], V[t], G[t], L[t]: device buffers of table t (may be NULL when
 * B_per_tab[t] == 0); workspace_dev: caller-owned device buffer of at least
 * spline_plan_workspace_bytes() bytes, 256-byte aligned, alive as long as
 * the plan.  tune_reps > 0 times every shape that divides all tables' rows
 * (tune_reps launches each) and keeps the fastest, after checking that all
 * give bit-identical outputs; 0 takes a default.  The tuning launches write
 * the outputs.  Synchronises `stream`. */
int spline_plan_create(const spline_t* const* tabs, int32_t n_tabs, const int64_t* B_per_tab,
                       const double* const* pos_dev, void* const* V, void* const* G, void* const* L,
                       void* workspace_dev, size_t workspace_bytes, int32_t tune_reps, void* stream,
                       spline_plan_t** out);

/* A plan whose every launch first sorts each table's positions on the
 * device into locality order (as spline_eval_vgl_sorted) and then deals
 * the task list to the XCDs in eight contiguous segments (workgroups steal
 * from the other segments once theirs is exhausted), so tasks that share
 * table rows share an L2.  Same arguments and outputs as spline_plan_create
 * (bit for bit); the workspace also holds each table's sort scratch:
 * spline_plan_workspace_bytes_sorted() bytes (0 on invalid input or a
 * table with 2^31 or more positions). */
size_t spline_plan_workspace_bytes_sorted(int32_t n_tabs, const int64_t* B_per_tab);
int spline_plan_create_sorted(const spline_t* const* tabs, int32_t n_tabs, const int64_t* B_per_tab,
                              const double* const* pos_dev, void* const* V, void* const* G, void* const* L,
                              void* workspace_dev, size_t workspace_bytes, int32_t tune_reps, void* stream,
                              spline_plan_t** out);

/* One replay of the captured graph on `stream` (asynchronous). */
int spline_plan_launch(const spline_plan_t* plan, void* stream);

/* The same two kernels launched directly, without the graph (for checking
 * the graph against eager execution). */
int spline_plan_launch_eager(const spline_plan_t* plan, void* stream);

/* Chosen tile shape, number of tasks and of persistent workgroups. */
int spline_plan_get_info(const spline_plan_t* plan, spline_tile* tile, int32_t* n_tasks, int32_t* n_blocks);

/* Releases the graph and the handle (not the workspace). NULL is accepted. */
int spline_plan_destroy(spline_plan_t* plan);

/* ---- Learned surrogate of a table ----------------------------------------
 * A small periodic network replaces the table where it is accurate enough:
 * features [sin 2pi k_j.u, cos 2pi k_j.u] (u = r / cell, 48 integer k_j),
 * two hidden layers of 256 SiLU units, N outputs mapped to orbitals by a
 * per-orbital affine map V = sd*y + mu.  V, G and L come from forward-mode
 * derivatives (five streams: value, d/dx, d/dy, d/dz, Laplacian) through
 * BF16 matrix-core products with FP32 accumulation.  It is trained on the
 * GPU against the spline's own VGL (Sobolev loss, Adam), an empirical error
 * map over spatial bins is built against the spline, and evaluation routes
 * positions in bins whose error exceeds a tolerance back to the spline.  The
 * paper has no network; the surrogate answers the memory-footprint question
 * it raises (Sections 7.2, 8.2: the table is the largest read-only object). */
typedef struct spline_mlp_s spline_mlp_t;

/* Shape: n_freq = 48, width = {96, 256, 256, N} with N a multiple of 16 in
 * [16, 256] (the compiled shape; other shapes give SPL_EUNSUPPORTED). */
typedef struct {
    int32_t n_freq;
    int32_t width[4];
} spline_mlp_desc;

/* Feature frequencies for a table (setup, host only): the `count` integer
 * vectors k, one of each pair +-k with 0 < |k|_2 <= kmax, whose pair carries
 * the most energy sum_m |c_hat_m(k)|^2 + |c_hat_m(-k)|^2 in the discrete
 * Fourier transform c_hat_m(k) = sum_j c_m[j] exp(-2 pi i sum_d k_d j_d /
 * n_d) of the coefficients coefs_host [n0][n1][n2][n_orb] (host, FP64,
 * orbital fastest).  The representative of a pair is the lexicographically
 * larger of k and -k; pairs are ordered by energy, equal energies by
 * increasing k.  freqs_out: host [count][3] int32.  energy_out (host, may be
 * NULL): count + 2 doubles -- the chosen pairs' energies, then the energy at
 * k = 0, then the whole spectrum's (n0 n1 n2 sum c^2, by Parseval), so the
 * share of the table's energy that the chosen features leave out can be
 * read.  kmax in [1, 16]; count at most the number of pairs (128 for
 * kmax = 4).  Uses up to 16 host threads. */
int spline_mlp_select_frequencies(const spline_grid* grid, int32_t n_orb, const double* coefs_host, int32_t count,
                                  int32_t kmax, int32_t* freqs_out, double* energy_out);

/* Byte offsets inside the parameter buffer (all 256-byte aligned), and the
 * element offsets of each tensor inside the flat FP32 parameter vector
 * [W1 (256x96) | b1 | W2 (256x256) | b2 | W3 (Nx256) | b3], weights stored
 * [out][in].  weights_bf16 holds the BF16 copies of W1, W2, W3 that the
 * evaluation reads, each in matrix-core fragment order: fragment (b, t),
 * rows 16b..16b+15 and columns 32t..32t+31, is 512 consecutive values (b
 * major), row 16b+c, columns 32t+8g..32t+8g+7 at 8(16g+c).  The buffer is
 * the whole network state: copying it is a checkpoint, and spline_mlp_attach
 * resumes from one.  Its last bytes, from meta + 256 to total, are scratch
 * that spline_mlp_init_output uses (no state), so that call allocates
 * nothing. */
typedef struct {
    int64_t n_params;
    int64_t W1, b1, W2, b2, W3, b3;
    int64_t params, adam_m, adam_v, weights_bf16, mu, sd, loss_w, freqs, bin_err, meta, total;
    int32_t max_bins;
} spline_mlp_layout;

size_t spline_mlp_param_bytes(const spline_mlp_desc* desc);
int spline_mlp_get_layout(const spline_mlp_desc* desc, spline_mlp_layout* out);

/* New network in the caller's device buffer params_dev (>= param_bytes,
 * 256-byte aligned): freqs_host [48][3] integer frequencies, cell[3] the
 * orthorhombic cell, params_host the flat initial parameters (n_params
 * FP32).  Adam moments start at zero, mu = 0, sd = 1, and every bin of the
 * error map starts as untrusted.  Synchronises `stream`. */
int spline_mlp_create(const spline_mlp_desc* desc, const int32_t* freqs_host, const double* cell,
                      const float* params_host, void* params_dev, size_t bytes, void* stream, spline_mlp_t** out);

/* Handle over an existing network state (a restored checkpoint). */
int spline_mlp_attach(const spline_mlp_desc* desc, const double* cell, void* params_dev, size_t bytes, void* stream,
                      spline_mlp_t** out);

/* Sets the output map and the loss weights from a target batch V [B][N],
 * G [B][3][N], L [B][N] (device, B >= 2): mu_n and sd_n are the mean and the
 * population standard deviation of orbital n's V over the batch (sd floored
 * at 1e-12); the weight of V, G (components pooled) and L is 1 / the mean
 * over orbitals of the variance of Q_n / sd_n about its own mean (1 for V).
 * Statistics are summed in FP64.  Synchronises `stream`. */
int spline_mlp_init_output(spline_mlp_t* mlp, const float* V, const float* G, const float* L, int64_t B,
                           void* stream);

/* Training.  Targets as above (the spline's VGL at pos [B][3]); ws: device
 * workspace of spline_mlp_train_workspace_bytes(mlp, B) bytes.
 * spline_mlp_grad writes the loss (device float) and the gradient of the
 * Sobolev loss (device, n_params floats, flat layout) without updating;
 * spline_mlp_train_step does one Adam step (beta 0.9/0.999, eps 1e-8) with
 * learning rate lr and refreshes the BF16 weights. */
size_t spline_mlp_train_workspace_bytes(const spline_mlp_t* mlp, int64_t B);
int spline_mlp_grad(spline_mlp_t* mlp, const double* pos, const float* tV, const float* tG, const float* tL, int64_t B,
                    void* ws, size_t ws_bytes, float* grad_out, float* loss_out, void* stream);
int spline_mlp_train_step(spline_mlp_t* mlp, const double* pos, const float* tV, const float* tG, const float* tL,
                          int64_t B, float lr, void* ws, size_t ws_bytes, float* loss_out, void* stream);

/* Network-only VGL (no fallback) at pos [B][3]: V [B][N], G [B][3][N],
 * L [B][N], FP32, device, each 16-byte aligned (SPL_EINVAL otherwise).
 * Asynchronous. */
int spline_mlp_forward(const spline_mlp_t* mlp, const double* pos, int64_t B, float* V, float* G, float* L,
                       void* stream);

/* Error map: evaluates the network and the spline table it stands in for (same N, same cell, FP32
 * outputs) at n_val validation positions and stores, per spatial bin
 * (bins_per_dim^3 bins, <= 16 per axis), the largest error over its points,
 * orbitals and quantities (V, each component of G, L), each relative to
 * that orbital's largest |V|, |G_d| or |L| of the spline over all
 * validation points (1 where that is 0).  Bin of a position: along axis d,
 * floor(nb * f) for its fractional coordinate f = u - floor(u), u = r_d /
 * cell_d in FP64 (f rounded up to 1 is the last bin; a non-finite
 * coordinate is bin 0); index (i0 * nb + i1) * nb + i2.  A NaN error term
 * counts as +inf; bins without points get +inf (untrusted).  The map is FP32
 * at layout.bin_err.  The estimate is empirical, not a bound. */
size_t spline_mlp_errmap_workspace_bytes(const spline_mlp_t* mlp, int64_t n_val);
int spline_mlp_build_error_map(spline_mlp_t* mlp, const spline_t* table, const double* val_pos, int64_t n_val,
                               int32_t bins_per_dim, void* ws, size_t ws_bytes, void* stream);

/* Evaluation with fallback: the network at every position, then the
 * fallback table (may be NULL: network only) re-evaluates, in place, every
 * position whose bin error is not <= tol (compared in FP32: tol < 0 or NaN
 * routes everything, +inf bins always route unless tol is +inf).  Routed
 * rows equal spline_eval_vgl's bit for bit, the others
 * spline_mlp_forward's.  n_fallback (device int32, may be NULL) receives the
 * number routed.  ws: device workspace of spline_mlp_eval_workspace_bytes(B)
 * bytes.  V, G, L as for spline_mlp_forward.  The fallback must have the
 * network's N orbitals, a non-FP64 storage type (FP32 outputs) and the
 * network's orthorhombic cell (SPL_EINVAL / SPL_EUNSUPPORTED otherwise). */
size_t spline_mlp_eval_workspace_bytes(int64_t B);
int spline_mlp_eval_vgl(const spline_mlp_t* mlp, const spline_t* fallback, float tol, const double* pos, int64_t B,
                        float* V, float* G, float* L, void* ws, size_t ws_bytes, int32_t* n_fallback, void* stream);

/* Adam steps taken and bins per axis of the current error map. */
int spline_mlp_get_info(const spline_mlp_t* mlp, int64_t* step, int32_t* bins_per_dim);
int spline_mlp_destroy(spline_mlp_t* mlp);

/* Measurement aid: one launch of a plain streaming-read kernel over `bytes`
 * bytes of buf (device, 16-byte aligned; floor(bytes/16) float4 loads, 16
 * bytes per lane, grid-stride), writing one float per thread to out (device,
 * grid*256 floats).  Timing it gives the HBM rate a simple read attains, to
 * set beside the published peak.  Asynchronous. */
int spline_probe_stream_read(const void* buf, size_t bytes, float* out, int32_t grid, void* stream);

/* Handle metadata queries. */
int spline_get_info(const spline_t* s, spline_grid* grid, int32_t* n_orb, spline_dtype* store,
                    spline_layout* layout);

/* Releases the handle (not table_dev). NULL is accepted. */
int spline_destroy(spline_t* s);

/* Thread-local text of the last error in this thread ("" if none). */
const char* spline_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QMCSPLINE_H */
