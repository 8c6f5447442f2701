// Private structures shared by the host API (mt_api.hip) and the kernels
// (mt_kernels.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mt.h"

namespace mt {

constexpr int kWave = 64;
constexpr int kCkptEvery = 16;             // RK4 state checkpoint interval
constexpr double kKappa = 0.299792458;     // GeV / (c T m)
constexpr int kBlockRec = 20;              // doubles per convex block record
constexpr int kGridCells = 1024;           // cells of the block grid (LDS-resident)

// Histogram tables on the device.  cdf[h][c] is the inclusive cumulative
// count of cell c of histogram h = material * n_pbin + bin; guide[h][g]
// brackets the answer of the inverse-CDF search for every word whose top
// gbits bits equal g: x = first candidate cell lo (low 16 bits) and last
// candidate hi (high 16 bits), y = cdf[h][lo], so that any bucket spanning
// at most two cells resolves without a probe of cdf.
struct DevHist {
    const uint32_t *cdf;
    const uint2 *guide;          // [h][2^gbits]
    const uint32_t *totals;      // [n_hist]
    const double *edges2;        // [n_pbin + 1] squared momentum edges
    const uint2 *alias;          // [h][c] alias method: (24-bit threshold split, alias cell)
    int32_t n_mat, n_pbin, n_loss, n_scat, n_cells, gbits;
    uint32_t nscat_magic;        // floor((2^32 - 1) / n_scat): c / n_scat = umulhi(c + 1, it),
                                 // exact for n_scat >= 1 and c < 2^16
    float loss_lo, loss_w, scat_lo, scat_w;   // log10 units on a logarithmic axis
    int32_t log_loss, log_scat;  // axis binned uniformly in log10 of the value
};

// Geometry: boxes split into z-slabs.  Slab s covers [slab_z[s], slab_z[s+1])
// with slab_z[0] = -inf and slab_z[n_slab] = +inf; slab_mask[s] has bit b set
// when box b spans the whole slab in z, so inside the slab only the x and y
// ranges of those boxes need testing, lowest index first.
struct DevGeom {
    int32_t n_box, n_slab, n_mag;    // n_box: volumes (boxes or blocks)
    int32_t n_poly;              // > 0: the volumes are convex blocks
    const double *poly;          // [n_poly][kBlockRec]
    const uint64_t *grid;        // [gz][gy][gx] candidate masks of the block grid
    int32_t gx, gy, gz;
    double g0[3], ginv[3];       // grid origin and cells per metre
    int32_t disjoint;            // no two boxes overlap: a box that holds a point is its box
    const double *box4;          // [n_box][4] xlo, xhi, ylo, yhi
    const int32_t *material;     // [n_box]
    const float4 *bfield;        // [n_box] (bx, by, bz, 0)
    const int32_t *magnet;       // [n_box]
    const double *slab_z;        // [n_slab + 1]
    const uint64_t *slab_mask;   // [n_slab]
    double x_max, y_max, z_max;
};

struct DevField {
    const float4 *map;           // cell-major [nz-1][ny-1][nx-1][8] (bx, by, bz, 0): the cell's
                                 // trilinear interpolant as coefficients of 1, fx, fy, fz, fx fy,
                                 // fx fz, fy fz, fx fy fz; nullptr = no map
    const float4 *nodes;         // node-major [nz][ny][nx] (bx, by, bz, 0), for the nearest node
    int32_t nx, ny, nz;
    double lo[3];
    double inv_d[3];             // (n - 1) / (hi - lo)
    double umax[3];              // n - 1: the largest grid coordinate inside the map
    double off[3];               // -lo (n - 1) / (hi - lo): u = x inv_d + off
};

// Byte offsets of the tables staged in LDS by every block.
struct LdsLayout {
    int32_t off_e2, off_tot, off_box4, off_mat, off_bf, off_mag, off_slabz, off_slabm;
    int32_t off_blk, off_grid;
    int32_t bytes;
};

struct DevRun {
    double h;                    // step length
    int32_t sampler;             // MT_SAMPLER_*
    int32_t interp;              // MT_INTERP_*
    int32_t stage_field;         // 0: field held from the step start, 1: at every RK4 stage
    int32_t share_shift;         // variant-wave form: log2 of the lanes sharing a random stream
    double pmin2;
    int32_t max_steps;
    uint32_t key0, key1;
    int64_t n;                   // input muons
    int64_t lanes;               // n_variants * n
    const float *scales;         // [n_variants][n_mag] or nullptr
    double *ckpt;                // [n_ckpt][6][lanes] or nullptr
    float *tape;                 // [max_steps][lanes][3] or nullptr
    int32_t *trace;
    int64_t n_trace;
    int32_t trace_steps;
};

struct DevIO {
    const double *x, *y, *z, *px, *py, *pz;
    const int8_t *q;
    double *ox, *oy, *oz, *opx, *opy, *opz;
    int32_t *status, *n_steps, *volume;
};

struct Tables {
    DevHist hist;
    DevGeom geom;
    DevField field;
    LdsLayout lds;
};

// One pass of the compacting form: the items (the launch's lanes, or the
// output slots listed by the previous pass) step from k_begin up to the
// DevRun::max_steps of the launch;
// every muon is stored in its output slot, and the slots of those still
// running there are appended to `out` for the next pass.
struct PassArgs {
    int32_t k_begin;             // first step of the pass (its last is DevRun::max_steps)
    int32_t max_steps;           // the real step cap
    const unsigned long long *n_in;   // slots listed by the previous pass, or nullptr: all lanes
    const int64_t *in;           // [*n_in] output slots to resume
    unsigned long long *n_out;   // slots appended by this pass (zeroed beforehand)
    int64_t *out;                // [lanes] at most
};

// Launchers implemented in mt_kernels.hip.
hipError_t launch_plain(const Tables &T, const DevRun &R, const DevIO &io, int block,
                        hipStream_t s);
// One pass of the compacting form (see PassArgs).
hipError_t launch_pass(const Tables &T, const DevRun &R, const DevIO &io, int block,
                       const PassArgs &P, hipStream_t s);
// Variant-wave form: groups of 2^R.share_shift lanes hold variants of one muon.
hipError_t launch_variant_waves(const Tables &T, const DevRun &R, const DevIO &io, int block,
                               hipStream_t s);
hipError_t launch_queue_reset(unsigned long long *queue, double *zero, int64_t n_zero,
                              hipStream_t s);
hipError_t launch_adjoint(const Tables &T, const DevRun &R, const DevIO &io,
                          const double *g_out, double *g_in, double *gs_lane, void *scratch,
                          int block, bool lds_history, hipStream_t s);
// Deterministic per-variant sums.  tally: (zmax count, hit count, sigmoid sum);
// column sums: out[v][c] = sum over lanes of variant v of vals[c][lane].
hipError_t launch_tally(const DevIO &io, int64_t n, int32_t n_variants, double z_det,
                        double r_ap, double r_scale, double *partial, int32_t n_part_blocks,
                        double *out, hipStream_t s);
hipError_t launch_column_sums(const double *vals, int32_t n_cols, int64_t n, int32_t n_variants,
                              double *partial, int32_t n_part_blocks, double *out, hipStream_t s);
int64_t adjoint_scratch_bytes(const Tables &T, int64_t lanes);

}  // namespace mt
