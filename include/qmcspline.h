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
 * multiplies the five sums by s_m at the end. */
typedef enum { SPL_F64 = 0, SPL_F32 = 1, SPL_BF16 = 2, SPL_F16 = 3 } spline_dtype;

enum {
    SPL_OK = 0,
    SPL_EINVAL = -1,       /* null pointer, bad size or bad enum */
    SPL_ENOMEM = -2,       /* size overflow, or a caller buffer too small */
    SPL_EHIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
    SPL_EUNSUPPORTED = -4  /* valid request this build cannot serve (e.g. tile shape) */
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
    int64_t row_bytes;      /* bytes per grid point (multiple of 256) */
    int64_t n_pad;          /* orbitals per row including zero padding */
    int64_t table_bytes;    /* rows * row_bytes, at offset 0 of the buffer */
    int64_t scales_offset;  /* byte offset of float scales[n_pad] */
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

/* Tile shape control.  spline_tile_candidates lists the shapes valid for this
 * table (up to `cap`, count in *n); spline_set_tile validates and selects one. */
int spline_tile_candidates(const spline_t* s, spline_tile* out, int32_t cap, int32_t* n);
int spline_set_tile(spline_t* s, const spline_tile* tile);
int spline_get_tile(const spline_t* s, spline_tile* tile);

/* Autotuner: times every candidate tile shape on the given batch with HIP
 * events (`reps` timed launches each, after one warm-up), checks that every
 * candidate's outputs on the first positions are bit-identical to the first
 * candidate's, selects the fastest and writes it to *chosen.  With a
 * non-NULL cache_path, a matching entry (key: device arch, grid, n_orb,
 * store, B bucket) is used without searching, and a new result is appended;
 * an unreadable or corrupt cache is ignored.  Outputs V/G/L are overwritten. */
int spline_autotune(spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                    int32_t reps, const char* cache_path, void* stream, spline_tile* chosen);

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
 * its workspace. */
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

/* One replay of the captured graph on `stream` (asynchronous). */
int spline_plan_launch(const spline_plan_t* plan, void* stream);

/* The same two kernels launched directly, without the graph (for checking
 * the graph against eager execution). */
int spline_plan_launch_eager(const spline_plan_t* plan, void* stream);

/* Chosen tile shape, number of tasks and of persistent workgroups. */
int spline_plan_get_info(const spline_plan_t* plan, spline_tile* tile, int32_t* n_tasks, int32_t* n_blocks);

/* Releases the graph and the handle (not the workspace). NULL is accepted. */
int spline_plan_destroy(spline_plan_t* plan);

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
