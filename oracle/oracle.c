/*
 * FP64 CPU oracle for histogram-sampling muon transport.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may build, load or call it; the
 * product path never does.  It shares no source with the HIP library.
 *
 * What it computes: the particle transport loop of the paper (Algorithm 1,
 * "Particle Transport Simulation Loop", Section "Simulation"), one muon at a
 * time, in double precision, with these readings of points the paper leaves
 * open:
 *   - sampler: exact inverse CDF over integer cumulative counts of the
 *     flattened 2D histogram (loss index major); one Philox4x32-10 block per
 *     material step gives the cell word and three jitter/azimuth words.
 *     Alternatively the alias method of Section "The Alias Method" (Walker's
 *     Prob/Alias tables, built exactly in integers), which takes its column
 *     from the cell word and its threshold from the low bytes of the other
 *     three words;
 *   - jitter: uniform within the drawn cell on both axes (Section
 *     "Simulation", item 2); on an axis binned in log10 (the parameterisation
 *     of Section "Building histograms") the jitter is uniform in log10 and the
 *     value is 10 to that power;
 *   - kick: dp_local = |p| (tau cos phi, tau sin phi, -f), rotated into the
 *     global frame with the Rodrigues formula of Eq. (2), axis k = z x p_hat
 *     normalised and theta the angle between z and p_hat;
 *   - field: per-box uniform field times the magnet's scale plus a trilinear
 *     interpolation of a node-centred map (zero outside it), evaluated once at
 *     the start of the step and held fixed through the RK4 stages (Algorithm
 *     1 fetches B once before RK4Step).  Options: the map read by
 *     nearest-neighbour lookup (the retrieval Section "Simulation", item 3
 *     names), and the field evaluated afresh at every RK4 stage position
 *     (the textbook RK4 of a position-dependent force);
 *   - equation of motion: the Lorentz force of Eq. (3) with E = 0 written in
 *     arc length s: dr/ds = p/|p|, dp/ds = kappa q (p/|p|) x B with
 *     kappa = 0.299792458 GeV/(c T m), integrated with classical RK4 over the
 *     fixed step d;
 *   - break test: |p| < p_min, z >= z_max, |x| >= x_max, |y| >= y_max, in
 *     that order, at the top of each iteration; the step cap ends the loop;
 *   - containment: half-open boxes, lowest index wins; momentum bin i with
 *     e_i <= |p| < e_{i+1}, clamped to [0, P-1].  Alternatively the geometry
 *     is a list of convex blocks (Section "Simulation", item 1): each has a
 *     z range [z_lo, z_hi) and a quadrilateral at either end; the slice at
 *     height z interpolates the two linearly and a point is inside when the
 *     edge cross products S_i of Eq. (1) (the sign test) are all >= 0 or all
 *     <= 0; lowest index wins.  The oracle tests every block (the spatial
 *     hashing grid of the paper only prunes candidates).
 *
 * Parity pins for every function here live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KAPPA 0.299792458
#define ORC_PI 3.14159265358979323846

typedef struct {
    /* histograms */
    int32_t n_mat, n_pbin, n_loss, n_scat;
    const double *p_edges;          /* [n_pbin+1] ascending */
    double loss_lo, loss_hi, scat_lo, scat_hi;
    const uint32_t *counts;         /* [n_mat][n_pbin][n_loss][n_scat] */
    /* geometry */
    int32_t n_box;
    const double *box;              /* [n_box][6] xlo xhi ylo yhi zlo zhi */
    int32_t n_poly;                 /* > 0: the volumes are these blocks, not boxes */
    const double *poly;             /* [n_poly][18] z_lo, z_hi, quad at z_lo (x0 y0 .. x3 y3),
                                       quad at z_hi (same vertex order) */
    const int32_t *material;        /* [n_box], -1 vacuum */
    const float *b_box;             /* [n_box][3] tesla, or NULL */
    const int32_t *magnet;          /* [n_box], -1 unscaled, or NULL */
    int32_t n_mag;
    double world[3];                /* x_max, y_max, z_max */
    /* field map (nx = 0: none) */
    int32_t nx, ny, nz;
    double map_lo[3], map_hi[3];
    const float *map;               /* [nz][ny][nx][3] */
    /* run */
    double step;
    int32_t max_steps;
    double p_min;
    uint64_t seed;
    const double *scales;           /* [n_variants][n_mag] or NULL (all 1) */
    int32_t sampler;                /* 0 inverse CDF, 1 alias method */
    int32_t log_loss, log_scat;     /* axis binned uniformly in log10 of the value */
    int32_t interp;                 /* map lookup: 0 trilinear, 1 nearest node */
    int32_t stage_field;            /* 0 B held from the step start, 1 B at every stage */
} orc_problem;

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random      */
/* numbers: as easy as 1, 2, 3").  Round: two 32x32->64 products of the   */
/* even counter words with the multipliers, outputs permuted and xored    */
/* with the odd words and the round key; the key is bumped by the Weyl    */
/* constants between rounds.                                              */
/* ---------------------------------------------------------------------- */
void oracle_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t MULT_A = 0xD2511F53u, MULT_B = 0xCD9E8D57u;
    const uint32_t WEYL_A = 0x9E3779B9u, WEYL_B = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)MULT_A * (uint64_t)c[0];
        uint64_t prod_b = (uint64_t)MULT_B * (uint64_t)c[2];
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t n0 = hi_b ^ c[1] ^ k[0];
        uint32_t n1 = lo_b;
        uint32_t n2 = hi_a ^ c[3] ^ k[1];
        uint32_t n3 = lo_a;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k[0] += WEYL_A;
        k[1] += WEYL_B;
    }
    memcpy(out, c, sizeof(c));
}

/* Uniform in [0,1) from the top 24 bits of a word: exact in FP32 and FP64. */
static double orc_unit(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/* ---------------------------------------------------------------------- */
/* Inverse CDF over integer counts.                                       */
/* ---------------------------------------------------------------------- */
/* Inclusive cumulative counts C[c] = sum_{c' <= c} counts[c'].  Returns 0 on
 * success, -1 if the total is zero or does not fit in 32 bits. */
int oracle_cdf_build(const uint32_t *counts, int64_t K, uint32_t *cdf)
{
    uint64_t acc = 0;
    for (int64_t c = 0; c < K; ++c) {
        acc += counts[c];
        if (acc > 0xFFFFFFFFull) return -1;
        cdf[c] = (uint32_t)acc;
    }
    return acc == 0 ? -1 : 0;
}

/* t = floor(w * T / 2^32), an integer uniform over [0, T) up to 2^-32. */
uint32_t oracle_cdf_t(uint32_t w, uint32_t total)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)total) >> 32);
}

/* Smallest c with C[c] > t (upper bound), for 0 <= t < C[K-1]. */
int64_t oracle_cdf_cell(const uint32_t *cdf, int64_t K, uint32_t t)
{
    int64_t lo = 0, hi = K - 1;     /* answer in [lo, hi] */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* ---------------------------------------------------------------------- */
/* Alias method (Section "The Alias Method"; Walker 1977).  The K cells are */
/* recast as K equally likely columns; column c keeps its own cell with    */
/* probability prob[c] / T and otherwise yields cell alias[c].             */
/*                                                                        */
/* Built exactly in integers: every column has capacity T (the histogram  */
/* total) and starts with weight w_c = K * count_c, so the weights sum to  */
/* K * T.  Two LIFO worklists hold the columns below capacity ("small")   */
/* and at or above it ("large"), each filled in ascending cell order.     */
/* Until "small" is empty: take the top small column s and the top large   */
/* column l; s keeps prob[s] = w_s and aliases l; l gives up T - w_s of    */
/* its weight and, once below capacity, moves from "large" to "small".     */
/* Columns left in "large" then hold exactly T: prob = T, alias = self.    */
/* ---------------------------------------------------------------------- */
/* Returns 0, -1 for a zero or oversized total, -2 when out of memory. */
int oracle_alias_build(const uint32_t *counts, int64_t K, uint32_t *prob, int32_t *alias)
{
    uint64_t T = 0;
    for (int64_t c = 0; c < K; ++c) T += counts[c];
    if (T == 0 || T > 0xFFFFFFFFull) return -1;
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)K);
    int64_t *small = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    int64_t *large = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    if (!w || !small || !large) { free(w); free(small); free(large); return -2; }
    int64_t ns = 0, nl = 0;
    for (int64_t c = 0; c < K; ++c) {
        w[c] = (uint64_t)K * counts[c];
        if (w[c] < T) small[ns++] = c; else large[nl++] = c;
    }
    while (ns > 0 && nl > 0) {
        int64_t sc = small[--ns];
        int64_t lc = large[nl - 1];
        prob[sc] = (uint32_t)w[sc];
        alias[sc] = (int32_t)lc;
        w[lc] -= T - w[sc];
        if (w[lc] < T) {
            --nl;
            small[ns++] = lc;
        }
    }
    /* exact arithmetic leaves "small" empty and every remaining large column
     * at exactly T */
    while (nl > 0) {
        int64_t lc = large[--nl];
        prob[lc] = (uint32_t)T;
        alias[lc] = (int32_t)lc;
    }
    int bad = ns != 0;
    free(w); free(small); free(large);
    return bad ? -1 : 0;
}

/* Column j = floor(w0 * K / 2^32).  Threshold t = floor(x * T / 2^24) with
 * x the 24-bit word made of the low bytes of w1, w2, w3 (bits the jitter and
 * azimuth do not use).  The cell is j when t < prob[j], else alias[j]. */
int64_t oracle_alias_cell(const uint32_t *prob, const int32_t *alias, int64_t K, uint32_t total,
                          const uint32_t w[4])
{
    int64_t j = (int64_t)(((uint64_t)w[0] * (uint64_t)K) >> 32);
    uint64_t x = (uint64_t)(w[1] & 0xFFu) | ((uint64_t)(w[2] & 0xFFu) << 8) |
                 ((uint64_t)(w[3] & 0xFFu) << 16);
    uint64_t t = (x * (uint64_t)total) >> 24;
    return t < prob[j] ? j : (int64_t)alias[j];
}

/* ---------------------------------------------------------------------- */
/* Rotation of the local kick into the global frame, Eq. (2):             */
/*   p <- p + dp cos(theta) + (k x dp) sin(theta) + (1 - cos theta)(k.dp)k */
/* with k the unit vector along z x p_hat and theta = angle(z, p_hat), so  */
/* that the rotation maps the local z axis onto the direction of travel.  */
/* ---------------------------------------------------------------------- */
void oracle_rotate(const double p[3], const double dp[3], double out[3])
{
    double pm = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    double nx = p[0] / pm, ny = p[1] / pm, nz = p[2] / pm;
    /* z x n = (-ny, nx, 0); |z x n| = sin(theta); n.z = cos(theta) */
    double sin_t = sqrt(nx * nx + ny * ny);
    double cos_t = nz;
    double r[3];
    if (sin_t == 0.0) {
        if (cos_t > 0.0) {          /* theta = 0: identity */
            r[0] = dp[0]; r[1] = dp[1]; r[2] = dp[2];
        } else {                    /* theta = pi about x: (x, y, z) -> (x, -y, -z) */
            r[0] = dp[0]; r[1] = -dp[1]; r[2] = -dp[2];
        }
    } else {
        double kx = -ny / sin_t, ky = nx / sin_t, kz = 0.0;
        double cx = ky * dp[2] - kz * dp[1];
        double cy = kz * dp[0] - kx * dp[2];
        double cz = kx * dp[1] - ky * dp[0];
        double kd = kx * dp[0] + ky * dp[1] + kz * dp[2];
        r[0] = dp[0] * cos_t + cx * sin_t + (1.0 - cos_t) * kd * kx;
        r[1] = dp[1] * cos_t + cy * sin_t + (1.0 - cos_t) * kd * ky;
        r[2] = dp[2] * cos_t + cz * sin_t + (1.0 - cos_t) * kd * kz;
    }
    out[0] = p[0] + r[0];
    out[1] = p[1] + r[1];
    out[2] = p[2] + r[2];
}

/* ---------------------------------------------------------------------- */
/* Classical RK4 on y = (r, p) with B frozen over the step.               */
/* ---------------------------------------------------------------------- */
static void orc_deriv(const double y[6], double q, const double B[3], double dy[6])
{
    double pm = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
    double ux = y[3] / pm, uy = y[4] / pm, uz = y[5] / pm;
    dy[0] = ux;
    dy[1] = uy;
    dy[2] = uz;
    dy[3] = ORC_KAPPA * q * (uy * B[2] - uz * B[1]);
    dy[4] = ORC_KAPPA * q * (uz * B[0] - ux * B[2]);
    dy[5] = ORC_KAPPA * q * (ux * B[1] - uy * B[0]);
}

void oracle_rk4(const double y_in[6], double q, const double B[3], double h, double y_out[6])
{
    double k1[6], k2[6], k3[6], k4[6], t[6];
    orc_deriv(y_in, q, B, k1);
    for (int a = 0; a < 6; ++a) t[a] = y_in[a] + 0.5 * h * k1[a];
    orc_deriv(t, q, B, k2);
    for (int a = 0; a < 6; ++a) t[a] = y_in[a] + 0.5 * h * k2[a];
    orc_deriv(t, q, B, k3);
    for (int a = 0; a < 6; ++a) t[a] = y_in[a] + h * k3[a];
    orc_deriv(t, q, B, k4);
    for (int a = 0; a < 6; ++a)
        y_out[a] = y_in[a] + h / 6.0 * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]);
}

/* ---------------------------------------------------------------------- */
/* Geometry: lowest-index half-open box containing r, or -1.              */
/* ---------------------------------------------------------------------- */
/* Slice of block b at height z: vertex i = (1 - t) bottom_i + t top_i with
 * t = (z - z_lo) / (z_hi - z_lo). */
static void orc_poly_slice(const double *pb, double z, double v[4][2])
{
    double t = (z - pb[0]) / (pb[1] - pb[0]);
    for (int i = 0; i < 4; ++i) {
        v[i][0] = (1.0 - t) * pb[2 + 2 * i] + t * pb[10 + 2 * i];
        v[i][1] = (1.0 - t) * pb[3 + 2 * i] + t * pb[11 + 2 * i];
    }
}

/* Eq. (1): S_i = e_ix (p_y - v_iy) - e_iy (p_x - v_ix), e_i = v_{i+1} - v_i. */
static void orc_poly_signs(const double v[4][2], const double r[3], double S[4])
{
    for (int i = 0; i < 4; ++i) {
        const double *a = v[i], *b = v[(i + 1) % 4];
        double ex = b[0] - a[0], ey = b[1] - a[1];
        S[i] = ex * (r[1] - a[1]) - ey * (r[0] - a[0]);
    }
}

int32_t oracle_poly_inside(const double *pb, const double r[3])
{
    if (!(pb[0] <= r[2] && r[2] < pb[1])) return 0;
    double v[4][2], S[4];
    orc_poly_slice(pb, r[2], v);
    orc_poly_signs(v, r, S);
    int pos = 1, neg = 1;
    for (int i = 0; i < 4; ++i) {
        if (S[i] < 0.0) pos = 0;
        if (S[i] > 0.0) neg = 0;
    }
    return pos || neg;
}

int32_t oracle_lookup(const orc_problem *P, const double r[3])
{
    if (P->n_poly > 0) {
        for (int32_t b = 0; b < P->n_poly; ++b)
            if (oracle_poly_inside(P->poly + 18 * b, r)) return b;
        return -1;
    }
    for (int32_t b = 0; b < P->n_box; ++b) {
        const double *bx = P->box + 6 * b;
        if (bx[0] <= r[0] && r[0] < bx[1] &&
            bx[2] <= r[1] && r[1] < bx[3] &&
            bx[4] <= r[2] && r[2] < bx[5])
            return b;
    }
    return -1;
}

/* ---------------------------------------------------------------------- */
/* Decision margins.  For the tests' boundary-tie rule only: how far the   */
/* state may move before a discrete decision of the transport loop        */
/* changes.  A GPU result that parts ways with this oracle at a decision   */
/* whose margin is below the GPU's own rounding deviation is a tie.        */
/* Positions are measured in the max-norm over the axes (the largest       */
/* coordinate change); for convex blocks the in-slice part is Euclidean    */
/* (see oracle_geom_margin).                                              */
/* ---------------------------------------------------------------------- */

/* Max-norm distance from r to the nearest point at which box b's
 * containment of r changes: inside, the nearest face; outside, the largest
 * per-axis violation (every violated axis must be crossed). */
static double orc_box_change(const double *bx, const double r[3])
{
    double inside = INFINITY, violation = 0.0;
    for (int a = 0; a < 3; ++a) {
        double dlo = r[a] - bx[2 * a], dhi = bx[2 * a + 1] - r[a];
        if (dlo >= 0.0 && dhi > 0.0) {
            double d = dlo < dhi ? dlo : dhi;
            if (d < inside) inside = d;
        } else {
            double v = dlo < 0.0 ? -dlo : -dhi;
            if (v > violation) violation = v;
        }
    }
    return violation > 0.0 ? violation : inside;
}

/* Euclidean distance from (x, y) to the segment a-b. */
static double orc_seg_dist(const double a[2], const double b[2], double x, double y)
{
    double ex = b[0] - a[0], ey = b[1] - a[1];
    double L2 = ex * ex + ey * ey;
    double t = L2 > 0.0 ? ((x - a[0]) * ex + (y - a[1]) * ey) / L2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double dx = x - (a[0] + t * ex), dy = y - (a[1] + t * ey);
    return sqrt(dx * dx + dy * dy);
}

/* Distance from r to the nearest point at which block pb's containment of
 * r changes, in the metric max(|dz|, |d(x, y)|): inside, the nearer z face
 * or the nearest edge line of the slice at r's height (|S_i| / |e_i|, the
 * in-slice distance to the boundary of a convex polygon); outside, both the
 * z gap and the in-slice distance to the slice polygon (the nearest edge
 * segment) must be closed, the latter taken in the slice at the nearer end
 * when r is outside the z range.  Exact for blocks with vertical faces; for
 * a face of horizontal slope s per metre of z the true distance is smaller
 * by at most the factor 1 / (1 + s). */
static double orc_block_change(const double *pb, const double r[3])
{
    double v[4][2], S[4];
    const int in_z = pb[0] <= r[2] && r[2] < pb[1];
    double zgap = 0.0, zs = r[2];
    if (!in_z) {
        zgap = r[2] < pb[0] ? pb[0] - r[2] : r[2] - pb[1];
        zs = r[2] < pb[0] ? pb[0] : pb[1];
    }
    orc_poly_slice(pb, zs, v);
    orc_poly_signs(v, r, S);
    int pos = 1, neg = 1;
    for (int i = 0; i < 4; ++i) {
        if (S[i] < 0.0) pos = 0;
        if (S[i] > 0.0) neg = 0;
    }
    if (in_z && (pos || neg)) {
        double d = r[2] - pb[0];
        if (pb[1] - r[2] < d) d = pb[1] - r[2];
        for (int i = 0; i < 4; ++i) {
            double ex = v[(i + 1) % 4][0] - v[i][0], ey = v[(i + 1) % 4][1] - v[i][1];
            double e = sqrt(ex * ex + ey * ey);
            if (e > 0.0 && fabs(S[i]) / e < d) d = fabs(S[i]) / e;
        }
        return d;
    }
    double dxy = 0.0;
    if (!(pos || neg)) {
        dxy = INFINITY;
        for (int i = 0; i < 4; ++i) {
            double d = orc_seg_dist(v[i], v[(i + 1) % 4], r[0], r[1]);
            if (d < dxy) dxy = d;
        }
    }
    return zgap > dxy ? zgap : dxy;
}

/* Decision margin of the volume lookup at r: the distance r may move before
 * the lowest-index volume holding it changes.  That happens when r leaves
 * the volume v it is in, or enters a volume of lower index than v (any
 * volume when v = -1); volumes of higher index than v cannot change the
 * answer while r stays in v.  Boxes: exact in the max-norm.  Blocks: as
 * orc_block_change. */
double oracle_geom_margin(const orc_problem *P, const double r[3])
{
    double m = INFINITY;
    int32_t v = oracle_lookup(P, r);
    int32_t n = P->n_poly > 0 ? P->n_poly : P->n_box;
    int32_t last = v >= 0 ? v : n - 1;
    for (int32_t b = 0; b <= last; ++b) {
        double d = P->n_poly > 0 ? orc_block_change(P->poly + 18 * b, r)
                                 : orc_box_change(P->box + 6 * b, r);
        if (d < m) m = d;
    }
    return m;
}

/* Margins of the break test at position r with momentum magnitude pm: the
 * conditions are tested in the order p_min, z_max, x_max, y_max, and the
 * outcome (continue, or the status of the first condition that holds)
 * changes only when that condition, or one tested before it, flips; when
 * none holds, any of the four.  Position distances in metres (max-norm),
 * the momentum distance relative to pm.  Returns the position margin and
 * stores the momentum margin in *margin_p.  The step cap is an integer
 * count and has no margin. */
double oracle_break_margin(const orc_problem *P, const double r[3], double pm, double *margin_p)
{
    double mp = fabs(pm - P->p_min) / pm, mpos = INFINITY, d;
    if (pm < P->p_min) { *margin_p = mp; return mpos; }
    d = fabs(r[2] - P->world[2]);
    if (d < mpos) mpos = d;
    if (r[2] >= P->world[2]) { *margin_p = mp; return mpos; }
    d = fabs(fabs(r[0]) - P->world[0]);
    if (d < mpos) mpos = d;
    if (fabs(r[0]) >= P->world[0]) { *margin_p = mp; return mpos; }
    d = fabs(fabs(r[1]) - P->world[1]);
    if (d < mpos) mpos = d;
    *margin_p = mp;
    return mpos;
}

/* Margin of the momentum-bin decision for bin ibin at magnitude pm,
 * relative to pm: the distance to the edges at which the bin changes.  The
 * bin's lower edge counts only above bin 0 and its upper edge only below
 * bin P-1 (momenta beyond the outer edges are clamped into those bins). */
double oracle_bin_margin(const orc_problem *P, int32_t ibin, double pm)
{
    double d = INFINITY;
    if (ibin > 0) d = fabs(pm - P->p_edges[ibin]) / pm;
    if (ibin < P->n_pbin - 1 && fabs(P->p_edges[ibin + 1] - pm) / pm < d)
        d = fabs(P->p_edges[ibin + 1] - pm) / pm;
    return d;
}

/* Momentum bin: e_i <= pm < e_{i+1}; below e_0 -> 0, at or above e_P -> P-1. */
int32_t oracle_pbin(const orc_problem *P, double pm)
{
    int32_t n = P->n_pbin;
    if (pm < P->p_edges[0]) return 0;
    if (pm >= P->p_edges[n]) return n - 1;
    int32_t lo = 0, hi = n - 1;      /* answer in [lo, hi] */
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (P->p_edges[mid] <= pm) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* ---------------------------------------------------------------------- */
/* Field: per-box uniform field (scaled) + trilinear map.                 */
/* ---------------------------------------------------------------------- */
void oracle_trilinear(const orc_problem *P, const double r[3], double B[3])
{
    B[0] = B[1] = B[2] = 0.0;
    if (P->nx <= 0 || P->map == NULL) return;
    const int32_t n[3] = {P->nx, P->ny, P->nz};
    int32_t i0[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        if (r[a] < P->map_lo[a] || r[a] > P->map_hi[a]) return;
        double u = (r[a] - P->map_lo[a]) / (P->map_hi[a] - P->map_lo[a]) * (double)(n[a] - 1);
        int32_t i = (int32_t)floor(u);
        if (i > n[a] - 2) i = n[a] - 2;
        if (i < 0) i = 0;
        i0[a] = i;
        w[a] = u - (double)i;
    }
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) *
                            (dz ? w[2] : 1.0 - w[2]);
                int64_t node = ((int64_t)(i0[2] + dz) * n[1] + (i0[1] + dy)) * n[0] + (i0[0] + dx);
                const float *b = P->map + 3 * node;
                B[0] += wt * (double)b[0];
                B[1] += wt * (double)b[1];
                B[2] += wt * (double)b[2];
            }
}

/* Nearest-neighbour lookup: the value of the node closest to r on every axis
 * (a point half-way between two nodes takes the higher one), zero outside
 * [lo, hi] as for the trilinear form. */
void oracle_nearest(const orc_problem *P, const double r[3], double B[3])
{
    B[0] = B[1] = B[2] = 0.0;
    if (P->nx <= 0 || P->map == NULL) return;
    const int32_t n[3] = {P->nx, P->ny, P->nz};
    int32_t i[3];
    for (int a = 0; a < 3; ++a) {
        if (r[a] < P->map_lo[a] || r[a] > P->map_hi[a]) return;
        double u = (r[a] - P->map_lo[a]) / (P->map_hi[a] - P->map_lo[a]) * (double)(n[a] - 1);
        int32_t k = (int32_t)floor(u + 0.5);
        if (k > n[a] - 1) k = n[a] - 1;
        i[a] = k;
    }
    int64_t node = ((int64_t)i[2] * n[1] + i[1]) * n[0] + i[0];
    const float *b = P->map + 3 * node;
    B[0] = (double)b[0];
    B[1] = (double)b[1];
    B[2] = (double)b[2];
}

/* Decision margin of the map lookup at r (max-norm, metres).  The map
 * gives zero outside [lo, hi] on every axis, so whether r is inside is a
 * decision: inside, the distance to the nearest face of the domain;
 * outside, the largest per-axis violation.  The trilinear interpolant is
 * continuous across cell faces (no decision there); the nearest-node
 * lookup also changes its node at the mid-planes between nodes, whose
 * distance counts for points inside. */
double oracle_map_margin(const orc_problem *P, const double r[3])
{
    if (P->nx <= 0 || P->map == NULL) return INFINITY;
    const int32_t n[3] = {P->nx, P->ny, P->nz};
    double inside = INFINITY, violation = 0.0;
    for (int a = 0; a < 3; ++a) {
        double dlo = r[a] - P->map_lo[a], dhi = P->map_hi[a] - r[a];
        if (dlo >= 0.0 && dhi >= 0.0) {
            double d = dlo < dhi ? dlo : dhi;
            if (d < inside) inside = d;
        } else {
            double v = dlo < 0.0 ? -dlo : -dhi;
            if (v > violation) violation = v;
        }
    }
    if (violation > 0.0) return violation;
    double m = inside;
    if (P->interp == 1) {
        for (int a = 0; a < 3; ++a) {
            double sp = (P->map_hi[a] - P->map_lo[a]) / (double)(n[a] - 1);
            double u = (r[a] - P->map_lo[a]) / sp;
            double f = u - floor(u);              /* mid-planes at f = 0.5 */
            double d = fabs(f - 0.5) * sp;
            if (d < m) m = d;
        }
    }
    return m;
}

static void orc_map(const orc_problem *P, const double r[3], double B[3])
{
    if (P->interp == 1) oracle_nearest(P, r, B);
    else oracle_trilinear(P, r, B);
}

static void orc_field(const orc_problem *P, int32_t vol, int32_t variant, const double r[3],
                      double B[3])
{
    orc_map(P, r, B);
    if (vol >= 0 && P->b_box != NULL) {
        double s = 1.0;
        if (P->magnet != NULL && P->magnet[vol] >= 0 && P->scales != NULL)
            s = P->scales[(int64_t)variant * P->n_mag + P->magnet[vol]];
        B[0] += s * (double)P->b_box[3 * vol + 0];
        B[1] += s * (double)P->b_box[3 * vol + 1];
        B[2] += s * (double)P->b_box[3 * vol + 2];
    }
}

/* RK4 step with the field evaluated at every stage position: the field
 * there is the scaled field of the box containing that point plus the map.
 * *margin (if not NULL) receives the smallest decision margin (volume
 * lookup, map) over the three stage points after the first. */
static void orc_rk4_stages(const orc_problem *P, int32_t variant, const double y_in[6], double q,
                           double h, double y_out[6], double *margin)
{
    double k1[6], k2[6], k3[6], k4[6], t[6], B[3], d;
    orc_field(P, oracle_lookup(P, y_in), variant, y_in, B);
    orc_deriv(y_in, q, B, k1);
    double *ks[3] = {k2, k3, k4};
    const double *prev[3] = {k1, k2, k3};
    const double c[3] = {0.5 * h, 0.5 * h, h};
    for (int s = 0; s < 3; ++s) {
        for (int a = 0; a < 6; ++a) t[a] = y_in[a] + c[s] * prev[s][a];
        if (margin) {
            d = oracle_geom_margin(P, t);
            if (d < *margin) *margin = d;
            d = oracle_map_margin(P, t);
            if (d < *margin) *margin = d;
        }
        orc_field(P, oracle_lookup(P, t), variant, t, B);
        orc_deriv(t, q, B, ks[s]);
    }
    for (int a = 0; a < 6; ++a)
        y_out[a] = y_in[a] + h / 6.0 * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]);
}

/* ---------------------------------------------------------------------- */
/* The transport loop.                                                    */
/* ---------------------------------------------------------------------- */
enum { ST_PMIN = 1, ST_ZMAX = 2, ST_XMAX = 3, ST_YMAX = 4, ST_STEPS = 5, ST_INVALID = 6 };

typedef struct {
    const double *x, *y, *z, *px, *py, *pz;
    const int8_t *q;
    const int64_t *ids;             /* Philox muon index of each muon */
    const int32_t *variant;         /* or NULL: variant 0 */
} orc_in;

typedef struct {
    double *x, *y, *z, *px, *py, *pz;
    int32_t *status, *n_steps, *volume;
    double *margin_pos, *margin_p;  /* minimum decision margins, or NULL */
    int32_t *trace;                 /* [n][trace_steps][3] (vol, bin, cell) or NULL */
    int32_t trace_steps;
    float *kicks;                   /* [n][kick_steps][3] (f, tau, phi/2pi) or NULL */
    int32_t kick_steps;
    double *step_margin;            /* [n][trace_steps + 1][2] (pos, p) per step, or NULL */
    uint64_t *digest;               /* [n] 64-bit FNV-1a hash of every step's (vol, bin,
                                       cell), or NULL: equal traces, equal digests */
} orc_out;

/* FNV-1a over the 12 bytes of one step's (vol, bin, cell), little-endian. */
static uint64_t orc_digest_step(uint64_t h, int32_t vol, int32_t ibin, int32_t cell)
{
    const int32_t v[3] = {vol, ibin, cell};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 4; ++b) {
            h ^= (uint64_t)(((uint32_t)v[a] >> (8 * b)) & 0xFFu);
            h *= 0x100000001B3ull;
        }
    return h;
}

/* Sampling tables of every histogram h = material * n_pbin + bin. */
typedef struct {
    uint32_t *cdf;                  /* [n_hist][K] inclusive cumulative counts */
    uint32_t *prob;                 /* [n_hist][K] alias thresholds (alias method only) */
    int32_t *alias;                 /* [n_hist][K] alias cells (alias method only) */
} orc_tables;

static void orc_one(const orc_problem *P, const orc_tables *tab, const orc_in *in,
                    const orc_out *out, int64_t j)
{
    double r[3] = {in->x[j], in->y[j], in->z[j]};
    double p[3] = {in->px[j], in->py[j], in->pz[j]};
    double q = (double)in->q[j];
    int64_t mu = in->ids[j];
    int32_t var = in->variant ? in->variant[j] : 0;
    int32_t status = 0, k = 0;
    double mpos = INFINITY, mp = INFINITY;
    const int64_t K = (int64_t)P->n_loss * P->n_scat;
    const uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
    /* axis origin and bin width, in log10 units on a logarithmic axis */
    const double l0 = P->log_loss ? log10(P->loss_lo) : P->loss_lo;
    const double l1 = P->log_loss ? log10(P->loss_hi) : P->loss_hi;
    const double s0 = P->log_scat ? log10(P->scat_lo) : P->scat_lo;
    const double s1 = P->log_scat ? log10(P->scat_hi) : P->scat_hi;
    const double wl = (l1 - l0) / P->n_loss;
    const double ws = (s1 - s0) / P->n_scat;

    double pm0 = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]) && isfinite(pm0)) || pm0 == 0.0 ||
        (in->q[j] != 1 && in->q[j] != -1))
        status = ST_INVALID;

    /* decision margins are formed only when asked for */
    const int margins = out->margin_pos || out->margin_p || out->step_margin;
    double *sm = NULL;              /* this step's (pos, p) margins */
    uint64_t digest = 0xCBF29CE484222325ull;
    while (status == 0) {
        double pm = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        double kpos = INFINITY, kp = INFINITY;
        sm = (out->step_margin && k <= out->trace_steps)
                 ? out->step_margin + ((int64_t)j * (out->trace_steps + 1) + k) * 2 : NULL;
        /* margins of the break test */
        double d = INFINITY;
        if (margins) kpos = oracle_break_margin(P, r, pm, &kp);
        if (kpos < mpos) mpos = kpos;
        if (kp < mp) mp = kp;
        if (sm) { sm[0] = kpos; sm[1] = kp; }
        if (pm < P->p_min) { status = ST_PMIN; break; }
        if (r[2] >= P->world[2]) { status = ST_ZMAX; break; }
        if (fabs(r[0]) >= P->world[0]) { status = ST_XMAX; break; }
        if (fabs(r[1]) >= P->world[1]) { status = ST_YMAX; break; }
        if (k >= P->max_steps) { status = ST_STEPS; break; }

        int32_t vol = oracle_lookup(P, r);
        if (margins) d = oracle_geom_margin(P, r);
        if (d < mpos) mpos = d;
        if (sm && d < sm[0]) sm[0] = d;
        int32_t mat = vol >= 0 ? P->material[vol] : -1;
        int32_t ibin = -1;
        int64_t cell = -1;
        if (mat >= 0) {
            ibin = oracle_pbin(P, pm);
            if (margins) d = oracle_bin_margin(P, ibin, pm);
            if (d < mp) mp = d;
            if (sm && d < sm[1]) sm[1] = d;
            uint32_t ctr[4] = {(uint32_t)mu, (uint32_t)((uint64_t)mu >> 32), (uint32_t)k, 0u};
            uint32_t w[4];
            oracle_philox(ctr, key, w);
            const int64_t h = (int64_t)mat * P->n_pbin + ibin;
            const uint32_t *C = tab->cdf + h * K;
            if (P->sampler == 1) {
                cell = oracle_alias_cell(tab->prob + h * K, tab->alias + h * K, K, C[K - 1], w);
            } else {
                uint32_t t = oracle_cdf_t(w[0], C[K - 1]);
                cell = oracle_cdf_cell(C, K, t);
            }
            int64_t il = cell / P->n_scat, is = cell % P->n_scat;
            double f = l0 + ((double)il + orc_unit(w[1])) * wl;
            double tau = s0 + ((double)is + orc_unit(w[2])) * ws;
            if (P->log_loss) f = pow(10.0, f);
            if (P->log_scat) tau = pow(10.0, tau);
            double phi = 2.0 * ORC_PI * orc_unit(w[3]);
            double dp[3] = {pm * tau * cos(phi), pm * tau * sin(phi), -pm * f};
            double pn[3];
            oracle_rotate(p, dp, pn);
            p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
            if (out->kicks && k < out->kick_steps) {
                float *kk = out->kicks + ((int64_t)j * out->kick_steps + k) * 3;
                kk[0] = (float)f; kk[1] = (float)tau; kk[2] = (float)orc_unit(w[3]);
            }
        }
        if (out->trace && k < out->trace_steps) {
            int32_t *tr = out->trace + ((int64_t)j * out->trace_steps + k) * 3;
            tr[0] = vol; tr[1] = ibin; tr[2] = (int32_t)cell;
        }
        if (out->digest) digest = orc_digest_step(digest, vol, ibin, (int32_t)cell);
        if (margins) d = oracle_map_margin(P, r);
        if (d < mpos) mpos = d;
        if (sm && d < sm[0]) sm[0] = d;
        double y[6] = {r[0], r[1], r[2], p[0], p[1], p[2]}, yn[6];
        if (P->stage_field) {
            double ms = INFINITY;
            orc_rk4_stages(P, var, y, q, P->step, yn, margins ? &ms : NULL);
            if (ms < mpos) mpos = ms;
            if (sm && ms < sm[0]) sm[0] = ms;
        } else {
            double B[3];
            orc_field(P, vol, var, r, B);
            oracle_rk4(y, q, B, P->step, yn);
        }
        r[0] = yn[0]; r[1] = yn[1]; r[2] = yn[2];
        p[0] = yn[3]; p[1] = yn[4]; p[2] = yn[5];
        ++k;
    }
    out->x[j] = r[0]; out->y[j] = r[1]; out->z[j] = r[2];
    out->px[j] = p[0]; out->py[j] = p[1]; out->pz[j] = p[2];
    out->status[j] = status;
    out->n_steps[j] = k;
    out->volume[j] = status == ST_INVALID ? -1 : oracle_lookup(P, r);
    if (status != ST_INVALID && margins) {
        double d = oracle_geom_margin(P, r);  /* the final-volume lookup */
        if (d < mpos) mpos = d;
        if (sm && d < sm[0]) sm[0] = d;
    }
    if (out->margin_pos) out->margin_pos[j] = mpos;
    if (out->margin_p) out->margin_p[j] = mp;
    if (out->digest) out->digest[j] = digest;
}

/* Propagate n muons.  Returns 0, or -1 for an empty/oversized histogram, or
 * -2 when memory for the sampling tables cannot be allocated.  Uses
 * n_threads OpenMP threads (<= 0: the OpenMP default). */
int oracle_propagate(const orc_problem *P, int64_t n, const orc_in *in, const orc_out *out,
                     int32_t n_threads)
{
    const int64_t K = (int64_t)P->n_loss * P->n_scat;
    const int64_t n_hist = (int64_t)P->n_mat * P->n_pbin;
    const size_t cells = (size_t)(K * n_hist > 0 ? K * n_hist : 1);
    orc_tables tab = {NULL, NULL, NULL};
    int rc = 0;
    tab.cdf = (uint32_t *)malloc(sizeof(uint32_t) * cells);
    if (P->sampler == 1) {
        tab.prob = (uint32_t *)malloc(sizeof(uint32_t) * cells);
        tab.alias = (int32_t *)malloc(sizeof(int32_t) * cells);
    }
    if (!tab.cdf || (P->sampler == 1 && (!tab.prob || !tab.alias))) rc = -2;
    for (int64_t h = 0; h < n_hist && rc == 0; ++h) {
        if (oracle_cdf_build(P->counts + h * K, K, tab.cdf + h * K) != 0) rc = -1;
        else if (P->sampler == 1)
            rc = oracle_alias_build(P->counts + h * K, K, tab.prob + h * K, tab.alias + h * K);
    }
    if (rc == 0) {
#ifdef _OPENMP
        if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
        for (int64_t j = 0; j < n; ++j) orc_one(P, &tab, in, out, j);
    }
    free(tab.cdf); free(tab.prob); free(tab.alias);
    return rc;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
