/*
 * mt.h -- C ABI of the MI355X (gfx950) histogram-sampling muon transport.
 *
 * The library implements the particle transport loop of Algorithm 1
 * ("Particle Transport Simulation Loop", Section "Simulation") for many
 * muons at once: per step a break test, a material lookup in a set of
 * axis-aligned boxes, a momentum-bin lookup, a draw of fractional momentum
 * loss and transverse kick from the material's 2D histogram for that bin
 * (exact inverse CDF over integer counts plus uniform jitter inside the
 * cell and an isotropic azimuth), the rotation of that kick into the muon's
 * frame with the Rodrigues formula of Eq. (2), and a fourth-order
 * Runge-Kutta push through the magnetic field (Eq. (3) with E = 0), the
 * field being fetched once at the start of the step.
 *
 * Conventions shared by every entry point:
 *   - units: metres, GeV/c, tesla; kappa = 0.299792458 GeV/(c T m);
 *   - every function returns an int32 status: MT_OK (0) or a negative
 *     MT_ERR_* code; mt_last_error() then gives a message (thread-local);
 *   - argument and shape validation is synchronous and happens before any
 *     launch; no C++ exception crosses the ABI;
 *   - loaders take HOST arrays, deep-copy them into library-owned device
 *     tables and return after the copy; the caller may free its arrays at
 *     once.  Reloading replaces the tables; do not reload while a launch that
 *     reads them may still run;
 *   - mt_propagate* take DEVICE pointers owned by the caller and enqueue
 *     work on the caller's HIP stream (NULL = the null stream) without
 *     waiting for it; the buffers must stay alive until that work is done;
 *   - asynchronous device faults surface as MT_ERR_HIP at a later call.
 *
 * The library runs on the device that is current when a loader is first
 * called; every later call must be made with that device current.
 */
#ifndef MT_H_
#define MT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MT_OK               0
#define MT_ERR_INVALID_ARG (-1)  /* null pointer, bad size, unsorted edges ... */
#define MT_ERR_SHAPE       (-2)  /* sizes inconsistent with the loaded tables */
#define MT_ERR_EMPTY_HIST  (-3)  /* a histogram with zero total or total >= 2^32 */
#define MT_ERR_NOT_LOADED  (-4)  /* propagate before the tables were loaded */
#define MT_ERR_OOM         (-5)  /* device allocation failed */
#define MT_ERR_HIP         (-6)  /* a HIP runtime call failed */
#define MT_ERR_LIMIT       (-7)  /* beyond a documented table limit */

/* ---- per-muon status (data, not errors) ------------------------------ */
#define MT_ST_RUNNING   0
#define MT_ST_PMIN      1        /* |p| < p_min */
#define MT_ST_ZMAX      2        /* z >= z_max */
#define MT_ST_XMAX      3        /* |x| >= x_max */
#define MT_ST_YMAX      4        /* |y| >= y_max */
#define MT_ST_MAXSTEPS  5        /* step cap reached */
#define MT_ST_INVALID   6        /* non-finite input, |p| = 0 or |q| != 1 */

/* ---- launch forms ------------------------------------------------------ */
#define MT_MODE_PLAIN       0    /* one lane per muon until it stops */
#define MT_MODE_PERSISTENT  1    /* compacting form: step-synchronised passes of
                                    compact_every steps over the whole batch; the
                                    muons still running after a pass are compacted
                                    into the list the next pass runs on */
#define MT_MODE_VARIANT_WAVES 2  /* G lanes of a wavefront hold G variants of one muon and
                                    share its random stream, G = the largest power of two
                                    dividing n_variants, at most 64: one Philox block per
                                    lane per G steps instead of one per step; no trace */

/* ---- samplers of the histogram cell ------------------------------------ */
#define MT_SAMPLER_CDF      0    /* exact inverse CDF over integer counts */
#define MT_SAMPLER_ALIAS    1    /* Walker alias method (Section "The Alias Method") */

/* ---- field map lookup and field evaluation ------------------------------ */
#define MT_INTERP_TRILINEAR 0    /* trilinear interpolation of the map */
#define MT_INTERP_NEAREST   1    /* value of the nearest node (Section "Simulation", item 3) */

/* Documented table limits. */
#define MT_MAX_BOXES      64     /* boxes in the geometry */
#define MT_MAX_PBINS      1024   /* momentum bins */
#define MT_MAX_HISTS      4096   /* n_mat * n_pbin histograms */
#define MT_MAX_CELLS      65536  /* n_loss * n_scat per histogram */
#define MT_MAX_MAGNETS    16     /* scaled magnets */

/*
 * Histograms H[M][i] (Section "Building histograms"): for material m and
 * momentum bin i, counts over n_loss linear bins of the fractional loss f in
 * [loss_lo, loss_hi) and n_scat linear bins of the transverse kick tau =
 * dPt/|P| in [scat_lo, scat_hi).
 *
 *   p_edges  host double [n_pbin+1], strictly ascending, > 0.  Bin i holds
 *            e_i <= |p| < e_{i+1}; momenta below e_0 use bin 0, at or above
 *            e_P use bin P-1 (no interpolation between bins).
 *   counts   host uint32 [n_mat][n_pbin][n_loss][n_scat] (loss index major);
 *            each histogram's total must lie in [1, 2^32).
 * Both samplers' tables are built: inclusive cumulative counts (with a guide
 * table) for MT_SAMPLER_CDF and Walker Prob/Alias tables for
 * MT_SAMPLER_ALIAS (Section "The Alias Method"), exact in integers.
 * Limits: n_pbin <= MT_MAX_PBINS, n_mat * n_pbin <= MT_MAX_HISTS,
 * n_loss * n_scat <= MT_MAX_CELLS.
 * Errors: MT_ERR_INVALID_ARG, MT_ERR_EMPTY_HIST, MT_ERR_LIMIT, MT_ERR_OOM,
 *         MT_ERR_HIP.
 */
int mt_load_histograms(int32_t n_mat, int32_t n_pbin, const double *p_edges,
                       int32_t n_loss, double loss_lo, double loss_hi,
                       int32_t n_scat, double scat_lo, double scat_hi,
                       const uint32_t *counts);

/* Axis flags of mt_load_histograms_ex. */
#define MT_AXIS_LOG_LOSS    1    /* loss bins uniform in log10 f over [loss_lo, loss_hi] */
#define MT_AXIS_LOG_SCAT    2    /* kick bins uniform in log10 tau over [scat_lo, scat_hi] */

/*
 * mt_load_histograms with logarithmic axes (Section "Building histograms":
 * log(-dPz/|P|) and log(dPt/|P|)).  On a log axis the bounds must be > 0,
 * bin a covers [lo (hi/lo)^(a/n), lo (hi/lo)^((a+1)/n)), and the jitter of a
 * drawn cell is uniform in log10 of the value.  axes = 0 is mt_load_histograms.
 */
int mt_load_histograms_ex(int32_t n_mat, int32_t n_pbin, const double *p_edges,
                          int32_t n_loss, double loss_lo, double loss_hi,
                          int32_t n_scat, double scat_lo, double scat_hi,
                          const uint32_t *counts, int32_t axes);

/*
 * Optimal momentum binning by bounded variation (appendix "Optimal Momentum
 * Binning"), a host computation: given an estimator phi (e.g. the pilot mean
 * of log10 of the fractional loss) at n_probe ascending probe momenta, the
 * edges start at p_probe[0]; after edge p_a the next edge is the first probe
 * whose phi differs from phi(p_a) by more than eps (the supremum of the bins
 * [p_a, p) whose probes all stay within eps), or the last probe.
 *
 *   edges     host double [max_edges] receives p_0 < ... < p_N
 *   n_edges   receives N + 1
 * Errors: MT_ERR_INVALID_ARG (n_probe < 2, unsorted probes, non-finite values,
 *         eps < 0), MT_ERR_LIMIT (more than max_edges edges).
 */
int mt_optimal_edges(const double *p_probe, const double *phi, int32_t n_probe, double eps,
                     double *edges, int32_t max_edges, int32_t *n_edges);

/*
 * Geometry (Section "Simulation", item 1, specialised to axis-aligned boxes).
 *
 *   box       host double [n_box][6] = xlo, xhi, ylo, yhi, zlo, zhi with
 *             lo < hi; containment is half-open [lo, hi) on every axis and
 *             overlapping boxes resolve to the lowest index.
 *   material  host int32 [n_box]: material index, or -1 for vacuum (no
 *             sampling; the box may still carry a field).
 *   b_box     host float [n_box][3]: uniform field of the box in tesla, or
 *             NULL for none.
 *   magnet    host int32 [n_box] in [-1, n_mag): the field scale that
 *             multiplies b_box (-1 = unscaled), or NULL.
 *   world     host double [3] = x_max, y_max, z_max of the break test
 *             |x| >= x_max, |y| >= y_max, z >= z_max.
 * Limits: 0 <= n_box <= MT_MAX_BOXES, n_mag <= MT_MAX_MAGNETS.  Material
 * indices must be < n_mat of the loaded histograms at propagate time.
 */
int mt_load_geometry(int32_t n_box, const double *box, const int32_t *material,
                     const float *b_box, const int32_t *magnet, int32_t n_mag,
                     const double *world);

/*
 * Geometry of convex blocks (Section "Simulation", item 1, Eq. (1)); replaces
 * any loaded geometry.  Block b spans z_lo <= z < z_hi; its cross-section at
 * height z is the quadrilateral whose vertices interpolate linearly between
 * the quad at z_lo and the quad at z_hi (t = (z - z_lo) / (z_hi - z_lo)).  A
 * point is inside when the edge cross products S_i = e_ix (y - v_iy) -
 * e_iy (x - v_ix) of that slice are all >= 0 or all <= 0; overlapping blocks
 * resolve to the lowest index.  Candidates are pruned with a uniform grid
 * (at most 1024 cells) over the blocks' bounding box.
 *
 *   block     host double [n][18] = z_lo, z_hi, (x, y) of the 4 vertices at
 *             z_lo, (x, y) of the same 4 vertices at z_hi.  Both quads must
 *             be strictly convex and listed in the same rotational order (the
 *             mid-height slice is checked too).
 *   material, b_box, magnet, n_mag, world: as for mt_load_geometry, per block.
 * Limits: 1 <= n <= MT_MAX_BOXES.  The differentiable form and the per-stage
 * field (stage_field = 1) need box geometry.
 * Errors: MT_ERR_INVALID_ARG, MT_ERR_LIMIT, MT_ERR_OOM, MT_ERR_HIP.
 */
int mt_load_blocks(int32_t n, const double *block, const int32_t *material, const float *b_box,
                   const int32_t *magnet, int32_t n_mag, const double *world);

/*
 * Field map on a regular 3D grid (Section "Simulation", item 3), added to
 * the per-box field and interpolated trilinearly.  Node (i, j, k) sits at
 * lo + (i, j, k) * (hi - lo) / (n - 1); outside [lo, hi] the map gives zero.
 *
 *   b   host float [nz][ny][nx][3] tesla, every value finite; NULL unloads
 *       the map.
 * Requires nx, ny, nz >= 2 and lo < hi on every axis.  The device holds a
 * cell-major copy, each cell's trilinear interpolant as 8 polynomial
 * coefficients (formed in double precision from the cell's 8 corner values
 * and rounded to float) in one 128-byte record (128 (nx-1)(ny-1)(nz-1)
 * bytes), so that a trilinear lookup reads one cache line, and a node-major
 * copy (16 nx ny nz bytes) for the nearest node.
 * Limits: nx ny nz < 2^31, nx < 2^24 and ny nz < 2^24 (MT_ERR_LIMIT).
 * Errors: MT_ERR_INVALID_ARG (also when a coefficient overflows float, which
 * needs values near FLT_MAX), MT_ERR_OOM, MT_ERR_HIP.
 */
int mt_load_field(int32_t nx, int32_t ny, int32_t nz, const double *lo, const double *hi,
                  const float *b);

/* Device structure-of-arrays muon states (metres, GeV/c, charge +-1). */
typedef struct mt_muons {
    double *x, *y, *z, *px, *py, *pz;
    int8_t *q;
} mt_muons;

/* Device per-lane outcomes. */
typedef struct mt_result {
    int32_t *status;    /* MT_ST_* */
    int32_t *n_steps;   /* completed RK4 pushes */
    int32_t *volume;    /* box containing the final position, -1 = none */
} mt_result;

/*
 * Run parameters.  A launch processes lanes = n_variants * n muon copies: lane
 * g = v * n + j transports input muon j under field-scale variant v and writes
 * slot g of the outputs.  All variants of muon j draw the same random numbers
 * (common random numbers): the Philox4x32-10 key is the 64-bit seed and the
 * counter is (j mod 2^32, j / 2^32, step, 0).  Vacuum steps draw nothing.
 * A material step turns the four output words w0..w3 into a cell and a
 * point in it: the cell from w0 (MT_SAMPLER_CDF: t = floor(w0 T / 2^32),
 * first cell whose cumulative count exceeds t; MT_SAMPLER_ALIAS: column
 * floor(w0 K / 2^32), kept when floor(x T / 2^24) is below its threshold,
 * else its alias, with x = the low bytes of w1, w2, w3 as a 24-bit number),
 * the jitters inside the cell and the azimuth from the top 24 bits of w1,
 * w2 and w3.
 */
typedef struct mt_params {
    double   step_m;          /* fixed step length d (> 0) */
    int32_t  max_steps;       /* step cap (>= 0) */
    double   p_min;           /* momentum threshold of the break test */
    uint64_t seed;
    int32_t  n_variants;      /* >= 1 */
    const float *scales;      /* device [n_variants][n_mag] or NULL (all 1) */
    int32_t  mode;            /* MT_MODE_PLAIN / MT_MODE_PERSISTENT / MT_MODE_VARIANT_WAVES */
    int32_t  block;           /* threads per block, multiple of 64 in [64, 1024]; 0 = default */
    int32_t  compact_every;   /* persistent: steps per pass, >= 1 (0 = 128); raised to
                                 ceil((max_steps + 1) / 64) so there are at most 64
                                 passes; >= max_steps + 1: one pass */
    int32_t  use_graph;       /* persistent and variant-wave forms: capture the launch once
                                 as a hipGraph and replay */
    /* differentiable form */
    int32_t  ckpt_every;      /* 0 = off, or 16: checkpoint (r, p) every 16 steps */
    double  *ckpt;            /* device [ceil(max_steps/16)][6][lanes] */
    float   *tape;            /* device [max_steps][lanes][3]: local kick of every step */
    /* per-step trace for the first n_trace lanes */
    int32_t *trace;           /* device [n_trace][trace_steps][3] = volume, bin, cell; or NULL */
    int64_t  n_trace;
    int32_t  trace_steps;
    /* per-variant tallies at a detector plane (design scan) */
    double  *tally;           /* device [n_variants][3] or NULL: see mt_propagate */
    double   z_det, r_ap, r_scale;
    int32_t  sampler;         /* MT_SAMPLER_CDF (0) or MT_SAMPLER_ALIAS */
    int32_t  interp;          /* MT_INTERP_TRILINEAR (0) or MT_INTERP_NEAREST */
    int32_t  stage_field;     /* 0: field fetched once at the step start and held over the
                                 RK4 stages (Algorithm 1); 1: evaluated at every stage
                                 position (box lookup + map there) */
} mt_params;

/*
 * Transport n input muons (lanes = n_variants * n).
 *
 *   in    device SoA of n muons; out and res: device SoA of `lanes` entries.
 *         out may alias in when n_variants == 1 and ckpt_every == 0.
 *   hip_stream  hipStream_t (NULL = null stream).
 * Per-muon outcomes are in res; status MT_ST_INVALID marks bad inputs.
 * If params->tally is set, after transport it receives for each variant
 * (count of lanes with status MT_ST_ZMAX, count of those whose straight-line
 * extension reaches the plane z = z_det within radius r_ap, and the sum of
 * sigmoid((r_ap - r)/r_scale) over them), summed in a fixed order.
 * With use_graph, the first call for a given argument set captures
 * queue reset + transport (+ tallies) into a hipGraph that later identical
 * calls replay; changing any pointer or parameter captures a new graph.
 * Library-owned workspaces (the compacting form's counters and survivor
 * lists, the tally and scale-gradient partial sums, the adjoint's segment
 * history) are shared
 * by every call: calls whose device work may overlap (on different streams)
 * race on them, so issue such calls on one stream or wait between them.
 * Errors: MT_ERR_NOT_LOADED, MT_ERR_INVALID_ARG, MT_ERR_SHAPE, MT_ERR_HIP.
 */
int mt_propagate(const mt_params *params, int64_t n, const mt_muons *in, mt_muons *out,
                 mt_result *res, void *hip_stream);

/*
 * mt_propagate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, kernels and results (bit for bit) as mt_propagate, but the
 * library workspace this call needs -- the persistent form's work counter
 * and the tally partial sums -- lives in a fixed device array of
 * MT_NOALLOC_SCRATCH_BYTES per device instead of library allocations.  The
 * call makes no hipMalloc or hipFree; it neither captures nor replays a graph
 * (use_graph must be 0), does not checkpoint (ckpt_every must be 0), uses
 * the block given (0 = 256), not the autotuner's choice, and runs the
 * compacting form (MT_MODE_PERSISTENT) as one pass over the whole step range
 * (the survivor lists of several passes would need 112 bytes per lane).  The tables must have been loaded (loaders do
 * allocate).
 * Limit: with a tally, 256 + 24 * n_variants * min(256, max(1, ceil(n /
 * 4096))) bytes must fit in MT_NOALLOC_SCRATCH_BYTES, else MT_ERR_LIMIT.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the counter is cleared by a kernel at the start of each
 * persistent launch; the partial sums are written before they are read):
 * calls whose device work overlaps on one GPU (different streams) race on
 * it, so issue them on one stream or wait between them.
 * Errors: as mt_propagate, plus MT_ERR_LIMIT.
 */
#define MT_NOALLOC_SCRATCH_BYTES 1048576   /* 1 MiB */
int mt_propagate_noalloc(const mt_params *params, int64_t n, const mt_muons *in, mt_muons *out,
                         mt_result *res, void *hip_stream);

/*
 * Pathwise adjoint of a checkpointed mt_propagate (the differentiable
 * extension suggested in Section "Discussion and Conclusion"): sampled
 * losses, kicks, azimuths, materials, bins and step counts are held fixed.
 * Requires the same params, in, res, ckpt and tape as the forward call,
 * which must have used ckpt_every = 16 and MT_MODE_PLAIN.  The differentiable
 * form supports the held trilinear field only: checkpointing with
 * MT_INTERP_NEAREST or stage_field = 1 is rejected (MT_ERR_INVALID_ARG).
 *
 *   g_out     device double [6][lanes]: dL/d(final x, y, z, px, py, pz)
 *   g_in      device double [6][lanes]: receives dL/d(initial state)
 *   g_scales  device double [n_variants][n_mag] or NULL: receives dL/d(scale)
 *             summed over each variant's lanes in a fixed order.
 * Errors: as mt_propagate.
 */
int mt_propagate_backward(const mt_params *params, int64_t n, const mt_muons *in,
                          const mt_result *res, const double *g_out, double *g_in,
                          double *g_scales, void *hip_stream);

/*
 * Pick block size and pass length of the compacting form by timing
 * candidate launches of this exact call (blocks {64,128,256,512} x steps
 * per pass {32,64,128,256,512, the whole step range}) on the caller's stream; for
 * MT_MODE_VARIANT_WAVES only the block size is tuned (best_compact gets 0).
 * Outputs are overwritten (every candidate writes identical bits).  The
 * choice is returned and remembered for later calls with compact_every = 0
 * and block = 0 on the same workload shape.
 */
int mt_autotune(const mt_params *params, int64_t n, const mt_muons *in, mt_muons *out,
                mt_result *res, void *hip_stream, int32_t *best_block,
                int32_t *best_compact, float *best_ms);

/*
 * Tuning switches of the library; none of them changes a result bit (each is
 * compared bit for bit with the default by a GPU test).  Settings are global,
 * kept until mt_release() and default as listed.
 *
 *   MT_OPT_GUIDE_BITS           resolution (bits of the cell word) of the
 *                               inverse-CDF guide table: 0 = automatic (one
 *                               entry per two cells, at most 2^16; default) or
 *                               1..16.  Applies from the next histogram load.
 *   MT_OPT_ADJOINT_BLOCK        threads per block of the adjoint kernel: 64
 *                               (default), 128, 192 or 256.
 *   MT_OPT_ADJOINT_LDS_HISTORY  1: the adjoint keeps a segment's pre-kick
 *                               momenta in LDS instead of device memory
 *                               (geometries without a field map; ignored with
 *                               one); 0 (default).
 * Errors: MT_ERR_INVALID_ARG (unknown option or value out of range).
 */
#define MT_OPT_GUIDE_BITS           1
#define MT_OPT_ADJOINT_BLOCK        2
#define MT_OPT_ADJOINT_LDS_HISTORY  3
int mt_set_option(int32_t option, int64_t value);

/* Thread-local message of the last failing call ("" if none). */
const char *mt_last_error(void);

/* Free every library-owned table, workspace and cached graph. */
void mt_release(void);

/* Device and build facts: fills info[0..3] = compute units, XCD count guess,
 * LDS bytes per block, wave size.  For reports only. */
int mt_device_info(int32_t *info);

#ifdef __cplusplus
}
#endif

#endif /* MT_H_ */
