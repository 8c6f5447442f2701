// HIP kernels of the histogram-sampling muon transport for gfx950 (MI355X).
//
// One lane carries one muon through the transport loop of Algorithm 1
// (Section "Simulation").  Muon state (r, p) lives in FP64 registers for the
// whole trajectory; the per-step arithmetic (kick, rotation, RK4 stages) is
// FP32 and its increments are accumulated into the FP64 state.  Every
// discrete decision (break test, box, momentum bin) is an FP64 compare, and
// the histogram cell is drawn by an exact integer inverse CDF, so decisions
// agree with a double-precision reference except at stated boundary ties.
//
// Build with -ffp-contract=off: every fused multiply-add is written out as
// fmaf(), so the same source yields the same bits in every kernel that
// inlines it (plain, persistent and the adjoint's re-forward).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <array>
#include <utility>

#include "mt_internal.h"

namespace mt {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each forming
// the 64-bit products of counter words 0 and 2 with the two multipliers,
// the high halves xored with words 1 and 3 and the round key, the key then
// advanced by the two Weyl increments.  The key is the same for every lane.
//
// The counter is (j mod 2^32, j / 2^32, step, 0) for muon j.  Everything in
// rounds 1 and 2 that does not depend on the step is the same for all steps
// of a muon, so it is formed once per muon (philox_prefix) and each step
// starts from it (philox_step): one product in each of the first two rounds
// instead of two.
// ---------------------------------------------------------------------------
constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;

struct PhiloxPrefix {
    uint32_t c1;   // round 1: j_hi ^ key0
    uint32_t c4;   // round 2: hi(kMulB * n2_1) ^ (key0 + kWeylA)
    uint32_t c5;   // round 2: lo(kMulB * n2_1)
    uint32_t c6;   // round 2: n3_1 ^ (key1 + kWeylB)
};

__device__ __forceinline__ PhiloxPrefix philox_prefix(uint32_t jlo, uint32_t jhi, uint32_t k0,
                                                      uint32_t k1) {
    const uint64_t pa1 = (uint64_t)kMulA * jlo;
    const uint32_t n2_1 = (uint32_t)(pa1 >> 32) ^ k1;   // round 1, word 2 (counter word 3 is 0)
    const uint32_t n3_1 = (uint32_t)pa1;
    const uint64_t pb2 = (uint64_t)kMulB * n2_1;
    PhiloxPrefix P;
    P.c1 = jhi ^ k0;
    P.c4 = (uint32_t)(pb2 >> 32) ^ (k0 + kWeylA);
    P.c5 = (uint32_t)pb2;
    P.c6 = n3_1 ^ (k1 + kWeylB);
    return P;
}

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96), a gfx950 instruction
// the compiler does not form from two xors by itself.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox_step(const PhiloxPrefix &P, uint32_t step, uint32_t k0,
                                             uint32_t k1) {
    // The round keys k + r (Weyl increment) are formed here, by scalar adds,
    // at every call: hoisted out of a step loop they would be 16 more
    // long-lived scalar registers, which the step loops do not have (they
    // were spilled to vector-register lanes and read back with v_readlane,
    // a vector instruction, plus a wait, for every round of every step).
    __asm__ volatile("" : "+s"(k0), "+s"(k1));
    // round 1: only the product with the step word varies
    const uint64_t pb1 = (uint64_t)kMulB * step;
    const uint32_t n0_1 = (uint32_t)(pb1 >> 32) ^ P.c1;
    const uint32_t n1_1 = (uint32_t)pb1;
    // round 2
    const uint64_t pa2 = (uint64_t)kMulA * n0_1;
    uint32_t c0 = n1_1 ^ P.c4;
    uint32_t c1 = P.c5;
    uint32_t c2 = (uint32_t)(pa2 >> 32) ^ P.c6;
    uint32_t c3 = (uint32_t)pa2;
    k0 += 2u * kWeylA;
    k1 += 2u * kWeylB;
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Tables staged in LDS by every block.
// ---------------------------------------------------------------------------
struct Lds {
    const double *e2;
    const uint32_t *tot;
    const double *box4;
    const int32_t *mat;
    const float4 *bf;
    const int32_t *mag;
    const double *slabz;
    const uint64_t *slabm;
    const double *blk;          // convex blocks [n_poly][kBlockRec]
    const uint64_t *grid;       // block grid candidate masks
};

template <bool POLY>
__device__ __forceinline__ Lds stage_tables(char *smem, const Tables &T) {
    const LdsLayout &L = T.lds;
    double *e2 = reinterpret_cast<double *>(smem + L.off_e2);
    uint32_t *tot = reinterpret_cast<uint32_t *>(smem + L.off_tot);
    double *box4 = reinterpret_cast<double *>(smem + L.off_box4);
    int32_t *mat = reinterpret_cast<int32_t *>(smem + L.off_mat);
    float4 *bf = reinterpret_cast<float4 *>(smem + L.off_bf);
    int32_t *mag = reinterpret_cast<int32_t *>(smem + L.off_mag);
    double *slabz = reinterpret_cast<double *>(smem + L.off_slabz);
    uint64_t *slabm = reinterpret_cast<uint64_t *>(smem + L.off_slabm);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i <= T.hist.n_pbin; i += nt) e2[i] = T.hist.edges2[i];
    const int nh = T.hist.n_mat * T.hist.n_pbin;
    for (int i = tid; i < nh; i += nt) tot[i] = T.hist.totals[i];
    for (int i = tid; i < T.geom.n_box; i += nt) {
        mat[i] = T.geom.material[i];
        bf[i] = T.geom.bfield[i];
        mag[i] = T.geom.magnet[i];
    }
    double *blk = reinterpret_cast<double *>(smem + L.off_blk);
    uint64_t *grid = reinterpret_cast<uint64_t *>(smem + L.off_grid);
    if constexpr (POLY) {
        for (int i = tid; i < kBlockRec * T.geom.n_poly; i += nt) blk[i] = T.geom.poly[i];
        const int G = T.geom.gx * T.geom.gy * T.geom.gz;
        for (int i = tid; i < G; i += nt) grid[i] = T.geom.grid[i];
    } else {
        for (int i = tid; i < 4 * T.geom.n_box; i += nt) box4[i] = T.geom.box4[i];
        for (int i = tid; i <= T.geom.n_slab; i += nt) slabz[i] = T.geom.slab_z[i];
        for (int i = tid; i < T.geom.n_slab; i += nt) slabm[i] = T.geom.slab_mask[i];
    }
    __syncthreads();
    return Lds{e2, tot, box4, mat, bf, mag, slabz, slabm, blk, grid};
}

// ---------------------------------------------------------------------------
// Lane state.  Besides the muon, a lane caches what rarely changes from one
// step to the next: the z-slab, the box, the momentum bin and the scaled
// field of the box.  Cached values are the
// same numbers a fresh lookup gives, so caching never changes a result.
// ---------------------------------------------------------------------------
struct Lane {
    double x, y, z, px, py, pz;
    double zlo, zhi;
    double e2lo, e2hi;
    float q;
    float bx, by, bz;     // scaled field of box bvol
    int32_t k, status, ibin, slab, vol, bvol, var;
    PhiloxPrefix ph;
    int64_t g;
    int32_t mcell;        // field-map cell whose corner values are in mc (-1: none)
    float mc[24];         // its 8 corners (bx, by, bz), corner order of the cell record
};

// Lane state of output slot g = var * n + j (input muon j, variant var).
__device__ __forceinline__ void load_lane_at(Lane &L, int64_t j, int64_t var, int64_t g,
                                             const DevIO &io, const DevRun &R) {
    L.x = io.x[j];
    L.y = io.y[j];
    L.z = io.z[j];
    L.px = io.px[j];
    L.py = io.py[j];
    L.pz = io.pz[j];
    const int qi = io.q[j];
    L.q = (float)qi;
    L.var = (int32_t)var;
    L.ph = philox_prefix((uint32_t)j, (uint32_t)((uint64_t)j >> 32), R.key0, R.key1);
    L.g = g;
    L.k = 0;
    L.ibin = -1;
    L.slab = -1;
    L.vol = -1;
    L.bvol = -2;
    L.mcell = -1;
    L.bx = L.by = L.bz = 0.0f;
    L.zlo = INFINITY;
    L.zhi = -INFINITY;
    L.e2lo = INFINITY;
    L.e2hi = -INFINITY;
    L.status = MT_ST_RUNNING;
    const double p2 = L.px * L.px + L.py * L.py + L.pz * L.pz;
    const bool ok = isfinite(L.x) && isfinite(L.y) && isfinite(L.z) && isfinite(p2) &&
                    p2 > 0.0 && (qi == 1 || qi == -1);
    if (!ok) L.status = MT_ST_INVALID;
}

__device__ __forceinline__ void load_lane(Lane &L, int64_t g, const DevIO &io, const DevRun &R) {
    int64_t var = 0, j = g;
    if (R.lanes != R.n) {
        if (R.lanes <= 0xFFFFFFFFll) {
            var = (uint32_t)g / (uint32_t)R.n;
        } else {
            var = g / R.n;
        }
        j = g - var * R.n;
    }
    load_lane_at(L, j, var, g, io, R);
}

// ---------------------------------------------------------------------------
// Geometry: z-slab, then the slab's candidate boxes in index order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_slab(const Lds &S, int n_slab, double z, int s) {
    if (s < 0) {                       // largest s with slabz[s] <= z (slabz[0] = -inf)
        int lo = 0, hi = n_slab - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.slabz[mid] <= z) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    while (s > 0 && z < S.slabz[s]) --s;
    while (s < n_slab - 1 && z >= S.slabz[s + 1]) ++s;
    return s;
}

// Branch-free: the four bounds come in two 16-byte LDS reads and the four
// compares are combined with bitwise ands (short-circuit && would turn every
// compare into a branch with its own dependent LDS read).
__device__ __forceinline__ bool in_box_xy(const Lds &S, int b, double x, double y) {
    const double2 *bx = reinterpret_cast<const double2 *>(S.box4 + 4 * b);
    const double2 xr = bx[0], yr = bx[1];
    return (xr.x <= x) & (x < xr.y) & (yr.x <= y) & (y < yr.y);
}

__device__ __forceinline__ int find_box(const Lds &S, int s, double x, double y) {
    uint64_t m = S.slabm[s];
    while (m) {
        const int b = __builtin_ctzll(m);
        if (in_box_xy(S, b, x, y)) return b;
        m &= m - 1;
    }
    return -1;
}

// Box containing the lane's position (lowest index), using the cached slab
// and, for geometries without overlapping boxes, the cached box.
__device__ __forceinline__ int locate(Lane &L, const Tables &T, const Lds &S) {
    const bool same_slab = L.z >= L.zlo && L.z < L.zhi;
    if (!same_slab) {
        L.slab = find_slab(S, T.geom.n_slab, L.z, L.slab);
        L.zlo = S.slabz[L.slab];
        L.zhi = S.slabz[L.slab + 1];
    } else if (L.vol >= 0 && T.geom.disjoint && in_box_xy(S, L.vol, L.x, L.y)) {
        return L.vol;
    }
    L.vol = find_box(S, L.slab, L.x, L.y);
    return L.vol;
}

// Convex block b holds (x, y, z): z_lo <= z < z_hi and the edge cross
// products of the slice at z (Eq. (1)) all >= 0 or all <= 0.
__device__ __forceinline__ bool in_block(const Lds &S, int b, double x, double y, double z) {
    const double *r = S.blk + kBlockRec * b;
    if (!(r[0] <= z && z < r[1])) return false;
    const double t = (z - r[0]) * r[2];
    double vx[4], vy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        vx[i] = fma(t, r[12 + 2 * i], r[4 + 2 * i]);
        vy[i] = fma(t, r[13 + 2 * i], r[5 + 2 * i]);
    }
    bool pos = true, neg = true;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        const double si = (vx[j] - vx[i]) * (y - vy[i]) - (vy[j] - vy[i]) * (x - vx[i]);
        pos = pos && si >= 0.0;
        neg = neg && si <= 0.0;
    }
    return pos || neg;
}

// Is (x, y, z) inside block b with every edge product beyond the block's
// margin (sigma S_i > tau, record word 3 = sigma tau, 0 = never)?  Then no
// block of lower index holds the point (the loader checked that each of
// them lies on the outer side of one of b's edge lines up to tau / 2).
__device__ __forceinline__ bool in_block_clear(const Lds &S, int b, double x, double y, double z) {
    const double *r = S.blk + kBlockRec * b;
    const double m = r[3];
    if (m == 0.0 || !(r[0] <= z && z < r[1])) return false;
    const double t = (z - r[0]) * r[2];
    double vx[4], vy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        vx[i] = fma(t, r[12 + 2 * i], r[4 + 2 * i]);
        vy[i] = fma(t, r[13 + 2 * i], r[5 + 2 * i]);
    }
    const double m2 = m * m;
    bool clear = true;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        const double si = (vx[j] - vx[i]) * (y - vy[i]) - (vy[j] - vy[i]) * (x - vx[i]);
        clear = clear & (si * m > m2);
    }
    return clear;
}

// Lowest-index block holding the lane's position: the block of the previous
// step if the point is clear inside it, else the grid cell's candidate mask,
// then the sign test, lowest index first.
__device__ __forceinline__ int locate_block(Lane &L, const Tables &T, const Lds &S) {
    if (L.vol >= 0 && in_block_clear(S, L.vol, L.x, L.y, L.z)) return L.vol;
    const DevGeom &G = T.geom;
    const double u = (L.x - G.g0[0]) * G.ginv[0];
    const double v = (L.y - G.g0[1]) * G.ginv[1];
    const double w = (L.z - G.g0[2]) * G.ginv[2];
    int vol = -1;
    if (u >= 0.0 && v >= 0.0 && w >= 0.0 && u < (double)G.gx && v < (double)G.gy &&
        w < (double)G.gz) {
        uint64_t m = S.grid[((int)w * G.gy + (int)v) * G.gx + (int)u];
        while (m) {
            const int b = __builtin_ctzll(m);
            if (in_block(S, b, L.x, L.y, L.z)) {
                vol = b;
                break;
            }
            m &= m - 1;
        }
    }
    L.vol = vol;
    return vol;
}

// Momentum bin i with e_i^2 <= |p|^2 < e_{i+1}^2, clamped to [0, P-1]; the
// previous step's bin is the starting guess.
__device__ __forceinline__ int find_bin(const Lds &S, int P, double p2, int i) {
    if (i < 0) {
        int lo = 0, hi = P - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.e2[mid] <= p2) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    while (i > 0 && p2 < S.e2[i]) --i;
    while (i < P - 1 && p2 >= S.e2[i + 1]) ++i;
    return i;
}

__device__ __forceinline__ int bin_of(Lane &L, const Tables &T, const Lds &S, double p2) {
    if (!(p2 >= L.e2lo && p2 < L.e2hi)) {
        const int P = T.hist.n_pbin;
        const int i = find_bin(S, P, p2, L.ibin);
        L.ibin = i;
        L.e2lo = i > 0 ? S.e2[i] : -INFINITY;
        L.e2hi = i < P - 1 ? S.e2[i + 1] : INFINITY;
    }
    return L.ibin;
}

// Exact inverse CDF: t = floor(w * T / 2^32), cell = smallest c with C[c] > t.
// The guide entry of the word's top bits brackets c in [lo, hi] and carries
// C[lo]: t < C[lo] gives lo at once, a bracket of two cells gives hi, and only
// wider brackets probe C.
__device__ __forceinline__ int sample_cell(const DevHist &H, const Lds &S, int h, uint32_t w0) {
    const uint32_t T = S.tot[h];
    const uint32_t t = __umulhi(w0, T);
    // h < 2^12 and gbits <= 16: the entry index fits in 32 bits
    const uint2 e = H.guide[((uint32_t)h << H.gbits) | (w0 >> (32 - H.gbits))];
    int lo = (int)(e.x & 0xFFFFu);
    int hi = (int)(e.x >> 16);
    if (t < e.y) return lo;
    ++lo;
    const uint32_t *C = H.cdf + (size_t)h * H.n_cells;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (C[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Alias method: column j = floor(w0 K / 2^32); the 24-bit threshold word x
// (low bytes of w1, w2, w3, which the jitters and the azimuth leave unused)
// keeps cell j when x is below the column's split, else gives its alias.
// One 8-byte load per draw.
__device__ __forceinline__ int alias_cell(const DevHist &H, int h, uint4 w) {
    const uint32_t j = __umulhi(w.x, (uint32_t)H.n_cells);
    const uint2 e = H.alias[(size_t)h * H.n_cells + j];
    const uint32_t x = (w.y & 0xFFu) | ((w.z & 0xFFu) << 8) | ((w.w & 0xFFu) << 16);
    return (int)(x < e.x ? j : e.y);
}

// ---------------------------------------------------------------------------
// Kick: p <- p + R(p_hat) (|p| u), u = (tau cos phi, tau sin phi, -f).  The
// rotation maps the local z axis onto p_hat, so the loss part is exactly
// -f p and is applied in FP64 (it is what accumulates over a trajectory);
// the transverse part uses the division-free Rodrigues form
// R v = c v + a x v + (a.v) a / (1 + c), a = z x p_hat = (-ny, nx, 0),
// c = nz (equal to Eq. (2) with k = a/|a|), in FP32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void kick(Lane &L, double p2, float ux, float uy, float uz) {
    const float p2f = (float)p2;
    const float rinv = __builtin_amdgcn_rsqf(p2f);
    const float pm = p2f * rinv;
    const float nx = (float)L.px * rinv, ny = (float)L.py * rinv, nz = (float)L.pz * rinv;
    const float dx = pm * ux, dy = pm * uy;
    const float opc = 1.0f + nz;
    float tx, ty, tz;
    if (opc > 0.0f) {
        const float coef = fmaf(nx, dy, -ny * dx) * __builtin_amdgcn_rcpf(opc);
        tx = fmaf(nz, dx, -coef * ny);
        ty = fmaf(nz, dy, coef * nx);
        tz = -fmaf(nx, dx, ny * dy);
    } else {                           // exactly backwards: rotation by pi about x
        tx = dx;
        ty = -dy;
        tz = 0.0f;
    }
    const double keep = 1.0 + (double)uz;       // 1 - f, exact
    L.px = fma(L.px, keep, (double)tx);
    L.py = fma(L.py, keep, (double)ty);
    L.pz = fma(L.pz, keep, (double)tz);
}

// ---------------------------------------------------------------------------
// Field at the start of the step: scaled per-box field + trilinear map.
// ---------------------------------------------------------------------------
// The trilinear interpolant of a map cell as a polynomial in the point's
// fractional coordinates (fx, fy, fz) in the cell:
//   B = k0 + k1 fx + k2 fy + k3 fz + k4 fx fy + k5 fx fz + k6 fy fz + k7 fx fy fz,
// the coefficients formed by the loader in FP64 from the cell's 8 corner
// values (k0 = B000, k1 = B100 - B000, ..., k7 the alternating sum of all
// eight) and stored as the cell's 128-byte record.  It equals the nested
// linear interpolation of the corners (the oracle's form) up to rounding,
// and takes 7 FMAs per component instead of 14 operations.
struct CellPoly {
    float4 k[8];
    float fx, fy, fz;
};

// Grid coordinates of a point: u = (x - lo) / d as one FMA, x (n - 1)/(hi -
// lo) - lo (n - 1)/(hi - lo), with both factors formed on the host.  Every
// map lookup (forward, replay, stage points) uses this, so the forward and
// the adjoint's replay see the same cells and weights.
__device__ __forceinline__ void map_coords(const DevField &F, double x, double y, double z,
                                           double &u, double &v, double &w) {
    u = fma(x, F.inv_d[0], F.off[0]);
    v = fma(y, F.inv_d[1], F.off[1]);
    w = fma(z, F.inv_d[2], F.off[2]);
}

// Inside the map's node range on all three axes (closed): six compares
// combined without branches, against the node counts as doubles.
__device__ __forceinline__ bool in_map(const DevField &F, double u, double v, double w) {
    return (u >= 0.0) & (u <= F.umax[0]) & (v >= 0.0) & (v <= F.umax[1]) & (w >= 0.0) &
           (w <= F.umax[2]);
}

__device__ __forceinline__ bool map_cell(const DevField &F, double x, double y, double z,
                                         CellPoly &c) {
    double u, v, w;
    map_coords(F, x, y, z, u, v, w);
    if (!in_map(F, u, v, w))
        return false;
    const int i = min((int)u, F.nx - 2), j = min((int)v, F.ny - 2), k = min((int)w, F.nz - 2);
    c.fx = (float)(u - (double)i);
    c.fy = (float)(v - (double)j);
    c.fz = (float)(w - (double)k);
    const float4 *b = F.map + (((size_t)k * (F.ny - 1) + j) * (F.nx - 1) + i) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) c.k[q] = b[q];
    return true;
}

// One component of the cell polynomial, grouped as
// k0 + fz k3 + fy (k2 + fz k6) + fx (k1 + fy (k4 + fz k7) + fz k5).
__device__ __forceinline__ float cell_poly1(float k0, float k1, float k2, float k3, float k4,
                                            float k5, float k6, float k7, float fx, float fy,
                                            float fz) {
    const float a = fmaf(fz, k5, fmaf(fy, fmaf(fz, k7, k4), k1));
    const float b = fmaf(fy, fmaf(fz, k6, k2), fmaf(fz, k3, k0));
    return fmaf(fx, a, b);
}

__device__ __forceinline__ float3 cell_field(const CellPoly &c) {
    float3 r;
    r.x = cell_poly1(c.k[0].x, c.k[1].x, c.k[2].x, c.k[3].x, c.k[4].x, c.k[5].x, c.k[6].x,
                     c.k[7].x, c.fx, c.fy, c.fz);
    r.y = cell_poly1(c.k[0].y, c.k[1].y, c.k[2].y, c.k[3].y, c.k[4].y, c.k[5].y, c.k[6].y,
                     c.k[7].y, c.fx, c.fy, c.fz);
    r.z = cell_poly1(c.k[0].z, c.k[1].z, c.k[2].z, c.k[3].z, c.k[4].z, c.k[5].z, c.k[6].z,
                     c.k[7].z, c.fx, c.fy, c.fz);
    return r;
}

__device__ __forceinline__ float3 box_field(const Tables &T, const Lds &S, const DevRun &R,
                                            int vol, int var) {
    float3 B = make_float3(0.f, 0.f, 0.f);
    if (vol >= 0) {
        const float4 b = S.bf[vol];
        const int m = S.mag[vol];
        const float s = (m >= 0 && R.scales != nullptr) ? R.scales[var * T.geom.n_mag + m] : 1.0f;
        B = make_float3(b.x * s, b.y * s, b.z * s);
    }
    return B;
}

template <bool MAP>
__device__ __forceinline__ float3 add_map(const Tables &T, float3 B, double x, double y, double z) {
    if (MAP) {
        CellPoly c;
        if (map_cell(T.field, x, y, z, c)) {
            const float3 m = cell_field(c);
            B.x += m.x;
            B.y += m.y;
            B.z += m.z;
        }
    }
    return B;
}

// Trilinear map at a point (the lane's position, or an RK4 stage point near
// it) with the lane's current cell's corners kept in registers: consecutive
// 2 cm steps and their stage points mostly stay in one cell, so the 128-byte
// record is loaded only when the point lies in another cell (which then
// becomes the lane's cell).  Same values and arithmetic as map_cell +
// cell_field.
__device__ __forceinline__ float3 add_map_cached(Lane &L, const DevField &F, float3 B, double x,
                                                  double y, double z) {
    double u, v, w;
    map_coords(F, x, y, z, u, v, w);
    if (!in_map(F, u, v, w))
        return B;
    const int i = min((int)u, F.nx - 2), j = min((int)v, F.ny - 2), k = min((int)w, F.nz - 2);
    // 24-bit products: the loader keeps nx and ny nz below 2^24
    const int cell = (int)__umul24(__umul24((uint32_t)k, (uint32_t)(F.ny - 1)) + (uint32_t)j,
                                   (uint32_t)(F.nx - 1)) + i;
    if (cell != L.mcell) {
        const float4 *b = F.map + (size_t)cell * 8;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float4 q = b[c];
            L.mc[3 * c] = q.x;
            L.mc[3 * c + 1] = q.y;
            L.mc[3 * c + 2] = q.z;
        }
        L.mcell = cell;
    }
    CellPoly c;
    c.fx = (float)(u - (double)i);
    c.fy = (float)(v - (double)j);
    c.fz = (float)(w - (double)k);
#pragma unroll
    for (int q = 0; q < 8; ++q) c.k[q] = make_float4(L.mc[3 * q], L.mc[3 * q + 1], L.mc[3 * q + 2], 0.f);
    const float3 m = cell_field(c);
    return make_float3(B.x + m.x, B.y + m.y, B.z + m.z);
}

// Nearest node with the last node's value kept in registers (mcell holds the
// node index, mc[0..2] its value).
__device__ __forceinline__ float3 add_nearest_cached(Lane &L, const DevField &F, float3 B,
                                                      double x, double y, double z) {
    double u, v, w;
    map_coords(F, x, y, z, u, v, w);
    if (!in_map(F, u, v, w))
        return B;
    const int i = min((int)(u + 0.5), F.nx - 1), j = min((int)(v + 0.5), F.ny - 1),
              k = min((int)(w + 0.5), F.nz - 1);
    const int node = (int)__umul24(__umul24((uint32_t)k, (uint32_t)F.ny) + (uint32_t)j,
                                   (uint32_t)F.nx) + i;
    if (node != L.mcell) {
        const float4 q = F.nodes[node];
        L.mc[0] = q.x;
        L.mc[1] = q.y;
        L.mc[2] = q.z;
        L.mcell = node;
    }
    return make_float3(B.x + L.mc[0], B.y + L.mc[1], B.z + L.mc[2]);
}

// Nearest-node lookup of the map: the node closest to (x, y, z) on every axis
// (half-way points take the higher node), zero outside the grid.  One
// 16-byte load from the node-major copy of the map.
__device__ __forceinline__ float3 map_nearest(const DevField &F, double x, double y, double z) {
    double u, v, w;
    map_coords(F, x, y, z, u, v, w);
    if (!in_map(F, u, v, w))
        return make_float3(0.f, 0.f, 0.f);
    const int i = min((int)(u + 0.5), F.nx - 1), j = min((int)(v + 0.5), F.ny - 1),
              k = min((int)(w + 0.5), F.nz - 1);
    const float4 b = F.nodes[((size_t)k * F.ny + j) * F.nx + i];
    return make_float3(b.x, b.y, b.z);
}

// ---------------------------------------------------------------------------
// RK4 over arc length with B frozen: dr/ds = p/|p|, dp/ds = kappa q (p/|p|) x B.
// FP32 stages, increments added to the FP64 state.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z),
                       fmaf(a.x, b.y, -a.y * b.x));
}

__device__ __forceinline__ float norm2(float3 a) { return fmaf(a.x, a.x, fmaf(a.y, a.y, a.z * a.z)); }

__device__ __forceinline__ float3 axpy(float a, float3 x, float3 y) {
    return make_float3(fmaf(a, x.x, y.x), fmaf(a, x.y, y.y), fmaf(a, x.z, y.z));
}

__device__ __forceinline__ float3 scale3(float a, float3 x) {
    return make_float3(a * x.x, a * x.y, a * x.z);
}

__device__ __forceinline__ float3 add3(float3 a, float3 b) {
    return make_float3(a.x + b.x, a.y + b.y, a.z + b.z);
}

struct StepConst {
    float h, h2, h6, h3;   // d, d/2, d/6, d/3
};

__device__ __forceinline__ float3 stage0(const Lane &L) {
    return make_float3((float)L.px, (float)L.py, (float)L.pz);
}

// a0 must be stage0(L) (the FP32 momentum the stages start from).
__device__ __forceinline__ void rk4_from(Lane &L, float3 a0, float3 B, const StepConst &c) {
    const float r0 = __builtin_amdgcn_rsqf(norm2(a0));
    const float3 n0 = scale3(r0, a0);
    float drx, dry, drz;
    if (B.x == 0.0f && B.y == 0.0f && B.z == 0.0f) {
        drx = c.h * n0.x;
        dry = c.h * n0.y;
        drz = c.h * n0.z;
    } else {
        const float kq = (float)kKappa * L.q;
        const float3 cb = scale3(kq, B);
        const float3 k1 = cross3(n0, cb);
        const float3 a1 = axpy(c.h2, k1, a0);
        const float3 n1 = scale3(__builtin_amdgcn_rsqf(norm2(a1)), a1);
        const float3 k2 = cross3(n1, cb);
        const float3 a2 = axpy(c.h2, k2, a0);
        const float3 n2 = scale3(__builtin_amdgcn_rsqf(norm2(a2)), a2);
        const float3 k3 = cross3(n2, cb);
        const float3 a3 = axpy(c.h, k3, a0);
        const float3 n3 = scale3(__builtin_amdgcn_rsqf(norm2(a3)), a3);
        const float3 k4 = cross3(n3, cb);
        // h/6 (v1 + 2 v2 + 2 v3 + v4)
        drx = c.h6 * (fmaf(2.0f, n1.x + n2.x, n0.x) + n3.x);
        dry = c.h6 * (fmaf(2.0f, n1.y + n2.y, n0.y) + n3.y);
        drz = c.h6 * (fmaf(2.0f, n1.z + n2.z, n0.z) + n3.z);
        const float dpx = c.h6 * (fmaf(2.0f, k2.x + k3.x, k1.x) + k4.x);
        const float dpy = c.h6 * (fmaf(2.0f, k2.y + k3.y, k1.y) + k4.y);
        const float dpz = c.h6 * (fmaf(2.0f, k2.z + k3.z, k1.z) + k4.z);
        L.px += (double)dpx;
        L.py += (double)dpy;
        L.pz += (double)dpz;
    }
    // the position update is shared by both branches (keeps every Lane field
    // in registers: no store through a selected address)
    L.x += (double)drx;
    L.y += (double)dry;
    L.z += (double)drz;
}

__device__ __forceinline__ void rk4(Lane &L, float3 B, const StepConst &c) {
    rk4_from(L, stage0(L), B, c);
}

// Compile-time features of a transport kernel (bit mask).
enum : unsigned {
    kMap = 1u,       // a field map is loaded
    kTape = 2u,      // write checkpoints and the kick tape (differentiable form)
    kTrace = 4u,     // per-step (volume, bin, cell) trace of the first lanes
    kAlias = 8u,     // alias-method sampler instead of the inverse CDF
    kNearest = 16u,  // nearest-node map lookup instead of trilinear (with kMap)
    kStages = 32u,   // field evaluated at every RK4 stage position
    kPoly = 64u,     // convex-block geometry instead of boxes
    kLog = 128u,     // a histogram axis is binned in log10
    kFeatures = 256u,// number of masks
    kShared = 256u   // the step's Philox words come from the caller (not a mask bit)
};

// Masks that have a kernel: the tape belongs to the differentiable form,
// whose adjoint holds the trilinear field over each step, and the
// nearest-node lookup needs a map.
constexpr bool valid_mask(unsigned F) {
    return !((F & kTape) && (F & (kNearest | kStages))) && !((F & kNearest) && !(F & kMap)) &&
           !((F & kPoly) && (F & (kTape | kStages)));
}

// Map part of the field at a point.
template <unsigned F>
__device__ __forceinline__ float3 map_field(const Tables &T, float3 B, double x, double y,
                                            double z) {
    if constexpr ((F & kNearest) != 0) {
        const float3 m = map_nearest(T.field, x, y, z);
        return make_float3(B.x + m.x, B.y + m.y, B.z + m.z);
    } else {
        return add_map<(F & kMap) != 0>(T, B, x, y, z);
    }
}

// Field at a stage point: scaled field of the box holding it plus the map,
// read through the lane's cached map cell or node.
template <unsigned F>
__device__ __forceinline__ float3 field_at_point(const Tables &T, const Lds &S, const DevRun &R,
                                                 Lane &L, double x, double y, double z) {
    const int s = find_slab(S, T.geom.n_slab, z, L.slab);
    const int vol = find_box(S, s, x, y);
    float3 B;
    if (vol == L.bvol) B = make_float3(L.bx, L.by, L.bz);
    else B = box_field(T, S, R, vol, L.var);
    if constexpr ((F & kMap) != 0 && (F & kNearest) == 0) return add_map_cached(L, T.field, B, x, y, z);
    else if constexpr ((F & kNearest) != 0) return add_nearest_cached(L, T.field, B, x, y, z);
    else return B;
}

// RK4 with the field evaluated afresh at each stage position (stage s sits
// at r + c_s h v_{s-1}, c = 1/2, 1/2, 1); B1 is the step-start field.
template <unsigned F>
__device__ __forceinline__ void rk4_stages(Lane &L, float3 B1, const Tables &T, const Lds &S,
                                           const DevRun &R, const StepConst &c) {
    const float kq = (float)kKappa * L.q;
    const float3 a0 = stage0(L);
    const float3 n0 = scale3(__builtin_amdgcn_rsqf(norm2(a0)), a0);
    const float3 k1 = cross3(n0, scale3(kq, B1));
    const float3 a1 = axpy(c.h2, k1, a0);
    const float3 n1 = scale3(__builtin_amdgcn_rsqf(norm2(a1)), a1);
    const float3 B2 = field_at_point<F>(T, S, R, L, L.x + (double)(c.h2 * n0.x),
                                        L.y + (double)(c.h2 * n0.y), L.z + (double)(c.h2 * n0.z));
    const float3 k2 = cross3(n1, scale3(kq, B2));
    const float3 a2 = axpy(c.h2, k2, a0);
    const float3 n2 = scale3(__builtin_amdgcn_rsqf(norm2(a2)), a2);
    const float3 B3 = field_at_point<F>(T, S, R, L, L.x + (double)(c.h2 * n1.x),
                                        L.y + (double)(c.h2 * n1.y), L.z + (double)(c.h2 * n1.z));
    const float3 k3 = cross3(n2, scale3(kq, B3));
    const float3 a3 = axpy(c.h, k3, a0);
    const float3 n3 = scale3(__builtin_amdgcn_rsqf(norm2(a3)), a3);
    const float3 B4 = field_at_point<F>(T, S, R, L, L.x + (double)(c.h * n2.x),
                                        L.y + (double)(c.h * n2.y), L.z + (double)(c.h * n2.z));
    const float3 k4 = cross3(n3, scale3(kq, B4));
    L.px += (double)(c.h6 * (fmaf(2.0f, k2.x + k3.x, k1.x) + k4.x));
    L.py += (double)(c.h6 * (fmaf(2.0f, k2.y + k3.y, k1.y) + k4.y));
    L.pz += (double)(c.h6 * (fmaf(2.0f, k2.z + k3.z, k1.z) + k4.z));
    L.x += (double)(c.h6 * (fmaf(2.0f, n1.x + n2.x, n0.x) + n3.x));
    L.y += (double)(c.h6 * (fmaf(2.0f, n1.y + n2.y, n0.y) + n3.y));
    L.z += (double)(c.h6 * (fmaf(2.0f, n1.z + n2.z, n0.z) + n3.z));
}

// ---------------------------------------------------------------------------
// One iteration of the transport loop.  Returns false (with L.status set)
// when a break condition holds at the top of the iteration.
// ---------------------------------------------------------------------------
template <unsigned F>
__device__ __forceinline__ bool advance(Lane &L, const Tables &T, const Lds &S, const DevRun &R,
                                        const StepConst &sc, uint4 w_shared = uint4{}) {
    constexpr bool MAP = (F & kMap) != 0, TAPE = (F & kTape) != 0, TRACE = (F & kTrace) != 0;
    const double p2 = L.px * L.px + L.py * L.py + L.pz * L.pz;
    // Break test in the order p_min, z_max, x_max, y_max, step cap (the first
    // that holds decides the status).  The five compares are or-ed as masks;
    // the status is picked only on the rare step that stops.
    const bool c_pmin = p2 < R.pmin2, c_z = L.z >= T.geom.z_max;
    const bool c_x = fabs(L.x) >= T.geom.x_max, c_y = fabs(L.y) >= T.geom.y_max;
    const bool c_k = L.k >= R.max_steps;
    int vol;
    if constexpr ((F & kPoly) != 0) vol = locate_block(L, T, S);
    else vol = locate(L, T, S);
    if (c_pmin | c_z | c_x | c_y | c_k) {   // the muon stops here; vol is its final volume
        L.status = c_pmin ? MT_ST_PMIN
                 : c_z    ? MT_ST_ZMAX
                 : c_x    ? MT_ST_XMAX
                 : c_y    ? MT_ST_YMAX
                          : MT_ST_MAXSTEPS;
        return false;
    }
    const int mat = vol >= 0 ? S.mat[vol] : -1;
    float ux = 0.0f, uy = 0.0f, uz = 0.0f;
    int cell = -1;
    if (mat >= 0) {
        const int ibin = bin_of(L, T, S, p2);
        uint4 w;
        if constexpr ((F & kShared) != 0) w = w_shared;
        else w = philox_step(L.ph, (uint32_t)L.k, R.key0, R.key1);
        // mat < 2^12 and n_pbin <= 1024: a full-rate 24-bit multiply
        const int h = (int)__umul24((uint32_t)mat, (uint32_t)T.hist.n_pbin) + ibin;
        if constexpr ((F & kAlias) != 0) cell = alias_cell(T.hist, h, w);
        else cell = sample_cell(T.hist, S, h, w.x);
        // cell / n_scat as umulhi(cell + 1, floor((2^32 - 1) / n_scat)): exact
        // for every n_scat >= 1 and cell < 2^16
        const int il = (int)__umulhi((uint32_t)cell + 1u, T.hist.nscat_magic);
        const int is = cell - il * T.hist.n_scat;
        const float v1 = (float)(w.y >> 8) * 0x1p-24f;
        const float v2 = (float)(w.z >> 8) * 0x1p-24f;
        const float v3 = (float)(w.w >> 8) * 0x1p-24f;
        float f = fmaf((float)il + v1, T.hist.loss_w, T.hist.loss_lo);
        float tau = fmaf((float)is + v2, T.hist.scat_w, T.hist.scat_lo);
        if constexpr ((F & kLog) != 0) {      // jitter uniform in log10 of the value
            // 10^u = 2^(u log2 10) on the hardware exp2 (relative error ~1e-6
            // for |u| <= 7, far inside the FP32 kick arithmetic around it)
            constexpr float kLog2Of10 = 3.32192809488736f;
            if (T.hist.log_loss) f = __builtin_amdgcn_exp2f(f * kLog2Of10);
            if (T.hist.log_scat) tau = __builtin_amdgcn_exp2f(tau * kLog2Of10);
        }
        // v_sin_f32 / v_cos_f32 take their argument in revolutions: sin(2 pi v3).
        const float sn = __builtin_amdgcn_sinf(v3);
        const float cs = __builtin_amdgcn_cosf(v3);
        ux = tau * cs;
        uy = tau * sn;
        uz = -f;
        kick(L, p2, ux, uy, uz);
    }
    if (TAPE) {   // the local kick; the replay finds the volume again from the state
        float *t = R.tape + ((size_t)L.k * R.lanes + L.g) * 3;
        t[0] = ux;
        t[1] = uy;
        t[2] = uz;
    }
    if (TRACE && L.g < R.n_trace && L.k < R.trace_steps) {
        int32_t *tr = R.trace + ((size_t)L.g * R.trace_steps + L.k) * 3;
        tr[0] = vol;
        tr[1] = mat >= 0 ? L.ibin : -1;
        tr[2] = cell;
    }
    if (vol != L.bvol) {
        const float3 b = box_field(T, S, R, vol, L.var);
        L.bx = b.x;
        L.by = b.y;
        L.bz = b.z;
        L.bvol = vol;
    }
    float3 B;
    if constexpr ((F & kMap) != 0 && (F & kNearest) == 0)
        B = add_map_cached(L, T.field, make_float3(L.bx, L.by, L.bz), L.x, L.y, L.z);
    else if constexpr ((F & kNearest) != 0)
        B = add_nearest_cached(L, T.field, make_float3(L.bx, L.by, L.bz), L.x, L.y, L.z);
    else
        B = map_field<F>(T, make_float3(L.bx, L.by, L.bz), L.x, L.y, L.z);
    if constexpr ((F & kStages) != 0) rk4_stages<F>(L, B, T, S, R, sc);
    else rk4(L, B, sc);
    ++L.k;
    return true;
}

__device__ __forceinline__ StepConst step_const(const DevRun &R) {
    StepConst c;
    c.h = (float)R.h;
    c.h2 = (float)(0.5 * R.h);
    c.h6 = (float)(R.h / 6.0);
    c.h3 = (float)(R.h / 3.0);
    return c;
}

__device__ __forceinline__ void store_lane(const Lane &L, const Tables &T, const Lds &S,
                                           const DevIO &io) {
    const int64_t g = L.g;
    io.ox[g] = L.x;
    io.oy[g] = L.y;
    io.oz[g] = L.z;
    io.opx[g] = L.px;
    io.opy[g] = L.py;
    io.opz[g] = L.pz;
    io.status[g] = L.status;
    io.n_steps[g] = L.k;
    io.volume[g] = L.status == MT_ST_INVALID ? -1 : L.vol;
}

__device__ __forceinline__ void write_ckpt(const Lane &L, const DevRun &R) {
    double *c = R.ckpt + (size_t)(L.k / kCkptEvery) * 6 * R.lanes + L.g;
    c[0] = L.x;
    c[R.lanes] = L.y;
    c[2 * R.lanes] = L.z;
    c[3 * R.lanes] = L.px;
    c[4 * R.lanes] = L.py;
    c[5 * R.lanes] = L.pz;
}

// ---------------------------------------------------------------------------
// Plain form: one lane per (variant, muon) until it stops.
//
// With a trilinear map held over the step, the lane's 24 cached interpolation
// values leave the kernel a few registers above the 96 that 5 waves/SIMD
// allow; asking for 5 waves moves two rarely used values to scratch and runs
// the shield 11 % faster than 4 waves.
// ---------------------------------------------------------------------------
constexpr int plain_min_waves(unsigned F) {
    return ((F & kMap) && !(F & (kStages | kNearest | kTape))) ? 5 : 1;
}

template <unsigned F>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(plain_min_waves(F))))
k_plain(Tables T, DevRun R, DevIO io) {
    constexpr bool CKPT = (F & kTape) != 0;
    extern __shared__ __align__(16) char smem[];
    const Lds S = stage_tables<(F & kPoly) != 0>(smem, T);
    const StepConst sc = step_const(R);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R.lanes) return;
    Lane L;
    load_lane(L, g, io, R);
    if (L.status == MT_ST_RUNNING) {
        for (;;) {
            if (CKPT && (L.k % kCkptEvery) == 0 && L.k < R.max_steps) write_ckpt(L, R);
            if (!advance<F>(L, T, S, R, sc)) break;
        }
    }
    store_lane(L, T, S, io);
}

// ---------------------------------------------------------------------------
// Compacting form: step-synchronised passes.
//
// The whole batch advances in passes of S steps: pass p takes every muon
// still in flight from step p S to step (p + 1) S (the last pass runs to the
// step cap), and the muons still running there are compacted into the list
// the next pass runs on, so every wave of a pass starts full.
// Muons in flight at any time are within S steps of each other, i.e. at
// about the same depth in z, so the part of a field map they read is a slab
// of the map, not the whole map: its lines stay in the caches instead of
// streaming from HBM.  A wave of a pass runs at most S steps, so lanes
// whose muon stops early idle for at most S steps.
//
// One lane per item as in the plain form (item i of the pass: lane i of the
// launch in the first pass, entry i of the previous pass's list after it).
// Every lane stores its muon in its output slot as the plain form does; a
// muon still running at the pass's end is stored there too (status running, its step
// count, its state) and its slot is appended to the list, with one atomic
// add per wavefront (ballot, then each lane at the wave's base + the
// survivors of lower lanes) and no block barrier, so a wave that is done
// leaves at once.  The next pass resumes the muon from its output slot.
// Results are bit-identical to the plain form: the random stream is keyed by
// (muon, step), the state moves exactly, and the lookup caches are rebuilt
// when a muon is resumed.
// ---------------------------------------------------------------------------

// Lane state of the muon of output slot g resumed at step k from that slot.
__device__ __forceinline__ void resume_lane(Lane &L, int64_t g, int32_t k, const DevIO &io,
                                            const DevRun &R) {
    int64_t var = 0, j = g;
    if (R.lanes != R.n) {
        var = R.lanes <= 0xFFFFFFFFll ? (int64_t)((uint32_t)g / (uint32_t)R.n) : g / R.n;
        j = g - var * R.n;
    }
    load_lane_at(L, j, var, g, io, R);      // charge, Philox prefix, caches reset
    L.x = io.ox[g];
    L.y = io.oy[g];
    L.z = io.oz[g];
    L.px = io.opx[g];
    L.py = io.opy[g];
    L.pz = io.opz[g];
    L.k = k;
    L.status = MT_ST_RUNNING;
}

template <unsigned F>     // F never holds kTape
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(plain_min_waves(F))))
k_pass(Tables T, DevRun R, DevIO io, PassArgs P) {
    extern __shared__ __align__(16) char smem[];
    // items of this pass: the launch's lanes (first pass) or the survivors
    // of the previous pass, whose count that pass left in memory
    const int64_t items = P.n_in ? (int64_t)*P.n_in : R.lanes;
    if ((int64_t)blockIdx.x * blockDim.x >= items) return;     // the whole block
    const Lds S = stage_tables<(F & kPoly) != 0>(smem, T);
    const StepConst sc = step_const(R);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool parked = false;        // still running at the pass's end: goes on in the next pass
    int64_t slot = 0;           // its output slot
    if (i < items) {
        Lane L;
        if (P.n_in) resume_lane(L, P.in[i], P.k_begin, io, R);
        else load_lane(L, i, io, R);
        // The pass ends where R.max_steps says (the host sets it to the
        // pass's last step, or to the step cap in the last pass), so the
        // step loop is the plain form's: a muon that meets no other break
        // condition at the pass's end stops with the step-cap status, and
        // is parked here if the real cap lies beyond.  The break test it
        // passed there is the one the next pass repeats at the same step.
        if (L.status == MT_ST_RUNNING) {
            for (;;) {
                if (!advance<F>(L, T, S, R, sc)) break;
            }
        }
        if (L.status == MT_ST_MAXSTEPS && L.k < P.max_steps) {
            parked = true;
            slot = L.g;
            L.status = MT_ST_RUNNING;
        }
        store_lane(L, T, S, io);            // status running if parked
    }
    // wave-aggregated append of the survivors' slots (no block barrier: a
    // wave that is done leaves at once and frees its registers for the next)
    const uint64_t m = __ballot(parked);
    if (m) {
        unsigned long long base = 0;
        if ((threadIdx.x & (kWave - 1)) == 0)
            base = atomicAdd(P.n_out, (unsigned long long)__popcll(m));
        base = __builtin_amdgcn_readfirstlane((uint32_t)base) |
               ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32);
        if (parked) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            P.out[base + rank] = slot;
        }
    }
}

// ---------------------------------------------------------------------------
// Variant-wave form (field variants of the same muons).  All variants of
// muon j draw the same random words at step k, so G lanes that hold G
// variants of one muon need one Philox block per step, not G.  G is the
// largest power of two that divides the variant count, at most 64 (the
// design scan's 64 variants give G = 64: a whole wavefront per muon).  Every
// G steps lane l forms the block of step k + (l mod G) for its group's muon
// into the wavefront's 1 KB of LDS, and at step k every lane reads its
// group's entry k mod G (one address per group, which the LDS broadcasts;
// the wavefront's own LDS writes and reads are executed in order, so only
// the compiler's ordering needs a wave barrier).  The lanes of a wavefront step in lockstep (all start at step 0,
// and each pass of the loop is one step for every lane still running), which
// is what makes the shared block the right one; a lane whose muon has
// stopped still forms its block for the others.  Wavefront w takes the
// 64 / G consecutive (muon, group of G variants) units from w 64 / G on.
// Results are bit-identical to the other forms (same words, same arithmetic,
// same output slots).
// ---------------------------------------------------------------------------
template <unsigned F>     // F holds neither kTape nor kTrace
__global__ void __launch_bounds__(1024) k_variant_waves(Tables T, DevRun R, DevIO io) {
    extern __shared__ __align__(16) char smem[];
    const Lds S = stage_tables<(F & kPoly) != 0>(smem, T);
    const StepConst sc = step_const(R);
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int gs = R.share_shift, gm = (1 << gs) - 1;   // G = 2^gs lanes per muon
    const int64_t n = R.n;
    const int64_t vgroups = (R.lanes / n) >> gs;       // groups of G variants per muon
    const int64_t units = n * vgroups;
    // the first unit of the wavefront is the same for all its lanes
    const int64_t first = ((int64_t)blockIdx.x * (blockDim.x / kWave) +
                           __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave))) *
                          (kWave >> gs);
    if (first >= units) return;
    const int64_t unit = first + (lane >> gs);
    const bool valid = unit < units;                   // the last wavefront may be ragged
    const int64_t j = valid ? unit / vgroups : 0;
    const int64_t var = valid ? (unit - j * vgroups) * (gm + 1) + (lane & gm) : 0;
    Lane L;
    bool running = false;
    if (valid) {
        load_lane_at(L, j, var, 0, io, R);         // output slot formed after the loop
        running = L.status == MT_ST_RUNNING;
    }
    const PhiloxPrefix P =
        philox_prefix((uint32_t)j, (uint32_t)((uint64_t)j >> 32), R.key0, R.key1);
    // the wavefront's Philox blocks: lane l holds its group's block of step
    // k0 + (l mod G), 1 KB of LDS per wavefront
    uint4 *wblk = reinterpret_cast<uint4 *>(smem + ((T.lds.bytes + 15) & ~15)) +
                  (threadIdx.x & ~(unsigned)(kWave - 1));
    const int base = lane & ~gm;
    for (int k = 0; __ballot(running) != 0; ++k) {
        const int sl = k & gm;
        if (sl == 0) {
            // the wavefront's LDS accesses are executed in order; the wave
            // barriers keep the compiler from moving the reads of the last
            // group of steps below this write or the reads of the next group
            // above it
            __builtin_amdgcn_wave_barrier();
            wblk[lane] = philox_step(P, (uint32_t)(k + (lane & gm)), R.key0, R.key1);
            __builtin_amdgcn_wave_barrier();
        }
        if (running) {
            const uint4 w = wblk[base + sl];      // one address per group: a broadcast
            running = advance<F | kShared>(L, T, S, R, sc, w);
        }
    }
    if (valid) {
        L.g = (int64_t)L.var * n + j;
        store_lane(L, T, S, io);
    }
}

__global__ void k_queue_reset(unsigned long long *queue, double *zero, int64_t n_zero) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *queue = 0ull;
    if (i < n_zero) zero[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Adjoint (pathwise; sampled kicks, decisions and step count held fixed).
//
// Forward step, in the order of the plain kernel:
//   a0 = p + |p| R(p_hat) u                          (kick, if in material)
//   k_i = c n_i x B, n_i = a_i/|a_i|, c = kappa q     (RK4 stages)
//   a1 = a0 + h/2 k1, a2 = a0 + h/2 k2, a3 = a0 + h k3
//   r' = r + h/6 (n0 + 2 n1 + 2 n2 + n3),  p' = a0 + h/6 (k1 + 2 k2 + 2 k3 + k4)
// The reverse sweep maps (lr', lp') to (lr, lp) and accumulates lB . dB/ds
// into the magnet's scale gradient.  The identity part of every Jacobian is
// applied in FP64; the O(h) and O(f, tau) corrections are formed in FP32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 unit_jt(float3 n, float rinv, float3 l) {
    // (I - n n^T) l / |a|
    const float d = fmaf(n.x, l.x, fmaf(n.y, l.y, n.z * l.z));
    return make_float3(rinv * fmaf(-d, n.x, l.x), rinv * fmaf(-d, n.y, l.y),
                       rinv * fmaf(-d, n.z, l.z));
}

__device__ __forceinline__ float dot3(float3 a, float3 b) {
    return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z));
}

// Gradient of l . g_u(p) with g_u(p) = p_z u + A x u + (A.u) A / (|p| + p_z),
// A = (-p_y, p_x, 0): the kick is p -> p + g_u(p).
__device__ __forceinline__ float3 kick_adjoint_corr(float3 p, float3 u, float3 l) {
    // hardware reciprocal square root and reciprocal: these are FP32
    // corrections to an FP64 adjoint, where 1-ulp accuracy is ample
    const float p2 = norm2(p);
    const float invP = __builtin_amdgcn_rsqf(p2);
    const float P = p2 * invP;
    const float D = P + p.z;
    const float alpha = fmaf(-p.y, u.x, p.x * u.y);
    const float beta = fmaf(-p.y, l.x, p.x * l.y);
    const float3 v = cross3(u, l);
    const float invD = __builtin_amdgcn_rcpf(D);
    const float Q = alpha * beta * invD;
    float3 g;
    g.x = v.y + (beta * u.y + alpha * l.y) * invD - Q * invD * (p.x * invP);
    g.y = -v.x + (-beta * u.x - alpha * l.x) * invD - Q * invD * (p.y * invP);
    g.z = dot3(l, u) - Q * invD * (p.z * invP + 1.0f);
    return g;
}

// d(trilinear)/dr contracted with lB.
__device__ __forceinline__ float3 map_grad_t(const DevField &F, const CellPoly &c, float3 lB) {
    // lB . k_q for the seven non-constant coefficients, then the partial
    // derivatives of the cell polynomial in fx, fy, fz
    auto dot4 = [&](float4 a) { return fmaf(lB.x, a.x, fmaf(lB.y, a.y, lB.z * a.z)); };
    const float v1 = dot4(c.k[1]), v2 = dot4(c.k[2]), v3 = dot4(c.k[3]), v4 = dot4(c.k[4]);
    const float v5 = dot4(c.k[5]), v6 = dot4(c.k[6]), v7 = dot4(c.k[7]);
    const float dx = fmaf(c.fy, fmaf(c.fz, v7, v4), fmaf(c.fz, v5, v1));
    const float dy = fmaf(c.fx, fmaf(c.fz, v7, v4), fmaf(c.fz, v6, v2));
    const float dz = fmaf(c.fx, fmaf(c.fy, v7, v5), fmaf(c.fy, v6, v3));
    return make_float3(dx * (float)F.inv_d[0], dy * (float)F.inv_d[1], dz * (float)F.inv_d[2]);
}

// One reverse step: (lr, lp) of the state after step k -> before step k, and
// the step's contribution to the scale gradient of its magnet.  p0 is the
// momentum at the start of the step (FP32 is enough for Jacobians), (rx, ry,
// rz) its position (used only with a field map).
template <bool MAP>
__device__ __forceinline__ void reverse_step(const Tables &T, const Lds &S, const DevRun &R,
                                             const StepConst &sc, float kq, float3 p0, float3 a0,
                                             double rx, double ry, double rz, int vol, float3 u,
                                             float3 Bbox, double lr[3], double lp[3], int &mag_out,
                                             double &dsg) {
    const int mat = vol >= 0 ? S.mat[vol] : -1;
    const float3 B = add_map<MAP>(T, Bbox, rx, ry, rz);
    const float3 Lr = make_float3((float)lr[0], (float)lr[1], (float)lr[2]);
    const float3 Lp = make_float3((float)lp[0], (float)lp[1], (float)lp[2]);
    // RK4 stages of the step (the straight-line shortcut of the forward pass
    // equals them at B = 0, so one form serves both).
    const float3 cb = scale3(kq, B);
    const float r0 = __builtin_amdgcn_rsqf(norm2(a0));
    const float3 n0 = scale3(r0, a0);
    const float3 k1v = cross3(n0, cb);
    const float3 a1 = axpy(sc.h2, k1v, a0);
    const float r1 = __builtin_amdgcn_rsqf(norm2(a1));
    const float3 n1 = scale3(r1, a1);
    const float3 k2v = cross3(n1, cb);
    const float3 a2 = axpy(sc.h2, k2v, a0);
    const float r2 = __builtin_amdgcn_rsqf(norm2(a2));
    const float3 n2 = scale3(r2, a2);
    const float3 k3v = cross3(n2, cb);
    const float3 a3 = axpy(sc.h, k3v, a0);
    const float r3 = __builtin_amdgcn_rsqf(norm2(a3));
    const float3 n3 = scale3(r3, a3);
    // Reverse through k4 = c n3 x B, a3 = a0 + h k3, ..., k1 = c n0 x B.
    float3 lk3 = scale3(sc.h3, Lp);
    float3 lk2 = scale3(sc.h3, Lp);
    float3 lk1 = scale3(sc.h6, Lp);
    const float3 lk4 = scale3(sc.h6, Lp);
    float3 lBc = cross3(lk4, n3);
    float3 la = unit_jt(n3, r3, axpy(sc.h6, Lr, cross3(cb, lk4)));
    float3 corr = la;
    lk3 = axpy(sc.h, la, lk3);
    lBc = add3(lBc, cross3(lk3, n2));
    la = unit_jt(n2, r2, axpy(sc.h3, Lr, cross3(cb, lk3)));
    corr = add3(corr, la);
    lk2 = axpy(sc.h2, la, lk2);
    lBc = add3(lBc, cross3(lk2, n1));
    la = unit_jt(n1, r1, axpy(sc.h3, Lr, cross3(cb, lk2)));
    corr = add3(corr, la);
    lk1 = axpy(sc.h2, la, lk1);
    lBc = add3(lBc, cross3(lk1, n0));
    la = unit_jt(n0, r0, axpy(sc.h6, Lr, cross3(cb, lk1)));
    corr = add3(corr, la);
    const float3 lB = scale3(kq, lBc);
    // lambda of a0 (post-kick momentum), then through the kick
    double la0[3] = {lp[0] + (double)corr.x, lp[1] + (double)corr.y, lp[2] + (double)corr.z};
    if (mat >= 0) {
        const float3 l = make_float3((float)la0[0], (float)la0[1], (float)la0[2]);
        const float3 kc = kick_adjoint_corr(p0, u, l);
        la0[0] += (double)kc.x;
        la0[1] += (double)kc.y;
        la0[2] += (double)kc.z;
    }
    lp[0] = la0[0];
    lp[1] = la0[1];
    lp[2] = la0[2];
    mag_out = -1;
    dsg = 0.0;
    if (vol >= 0) {
        const int m = S.mag[vol];
        if (m >= 0) {
            const float4 b = S.bf[vol];
            mag_out = m;
            dsg = (double)fmaf(lB.x, b.x, fmaf(lB.y, b.y, lB.z * b.z));
        }
    }
    if (MAP) {
        CellPoly cc;
        if (map_cell(T.field, rx, ry, rz, cc)) {
            const float3 gr = map_grad_t(T.field, cc, lB);
            lr[0] += (double)gr.x;
            lr[1] += (double)gr.y;
            lr[2] += (double)gr.z;
        }
    }
}

// One FP32 momentum of the adjoint's segment history (12 bytes, so a
// wavefront's records of a step are one contiguous 768-byte run).
struct Float3r {
    float x, y, z;
};

// The stage-0 momentum of a step formed again from its FP32 pre-kick
// momentum: the forward's kick arithmetic on (double)p0 instead of the FP64
// state it was rounded from.  It agrees with the forward's a0 to the last bit
// or, rarely, one unit in the last place (the FP64 state and its FP32
// rounding differ by ~1e-8 relative), which is what the FP32 Jacobians
// built from it need.
__device__ __forceinline__ float3 kick_again(float3 p0, float3 u) {
    Lane K;
    K.px = (double)p0.x;
    K.py = (double)p0.y;
    K.pz = (double)p0.z;
    const double p2 = K.px * K.px + K.py * K.py + K.pz * K.pz;
    kick(K, p2, u.x, u.y, u.z);
    return stage0(K);
}

// Re-run one step of a segment with its recorded kick (the arithmetic of
// advance(), so the same bits).  The volume is looked up again from the
// state, which is the forward's to the bit, so it is the forward's volume.
// B caches the field of volume bvol.  Returns the volume.
template <bool MAP>
__device__ __forceinline__ int replay_step(Lane &L, const Tables &T, const Lds &S,
                                           const DevRun &R, const StepConst &sc, int var,
                                           float3 u) {
    const int vol = locate(L, T, S);
    const int mat = vol >= 0 ? S.mat[vol] : -1;
    if (mat >= 0) {
        const double p2 = L.px * L.px + L.py * L.py + L.pz * L.pz;
        kick(L, p2, u.x, u.y, u.z);
    }
    if (vol != L.bvol) {
        const float3 b = box_field(T, S, R, vol, var);
        L.bx = b.x;
        L.by = b.y;
        L.bz = b.z;
        L.bvol = vol;
    }
    const float3 B = add_map<MAP>(T, make_float3(L.bx, L.by, L.bz), L.x, L.y, L.z);
    const float3 a0 = stage0(L);
    rk4_from(L, a0, B, sc);
    return vol;
}

// The segment's start momenta are kept either in LDS (LDSH) or in a per-lane
// scratch area in device memory; with a field map the start positions are
// needed too and always go to the scratch area.
// Without a map the kernel needs 103 VGPRs (4 waves/SIMD); asking for 5 waves
// spills a few values kept across the segment loops and runs 3 % faster.
template <bool MAP, bool LDSH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MAP ? 1 : 5)))
k_adjoint(Tables T, DevRun R, DevIO io, const double *g_out,
                                                 double *g_in, double *gs_lane, char *scratch) {
    extern __shared__ __align__(16) char smem[];
    const Lds S = stage_tables<false>(smem, T);
    const StepConst sc = step_const(R);
    const int bd = blockDim.x;
    const int n_mag = T.geom.n_mag;
    double *sgs = reinterpret_cast<double *>(smem + ((T.lds.bytes + 15) & ~15)) + threadIdx.x;
    float *hist = reinterpret_cast<float *>(smem + ((T.lds.bytes + 15) & ~15) +
                                            (size_t)n_mag * bd * sizeof(double)) + threadIdx.x;
    // volume of every step of the segment, found again by the replay and
    // read back by the reverse sweep: [step][thread], one byte each
    int8_t *vh = reinterpret_cast<int8_t *>(smem + ((T.lds.bytes + 15) & ~15) +
                                           (size_t)n_mag * bd * sizeof(double) +
                                           (LDSH ? (size_t)kCkptEvery * 3 * bd * sizeof(float) : 0)) +
                 threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g0 < R.lanes;
    const int64_t g = live ? g0 : R.lanes - 1;   // lanes past the end idle below
    const int64_t lanes = R.lanes;
    for (int m = 0; m < n_mag; ++m) sgs[m * bd] = 0.0;
    double lr[3], lp[3];
    for (int a = 0; a < 3; ++a) {
        lr[a] = g_out[a * lanes + g];
        lp[a] = g_out[(3 + a) * lanes + g];
    }
    const int ns = io.n_steps[g];
    const int status = io.status[g];
    int var = 0;
    if (R.lanes != R.n) var = (int)(g / R.n);
    const float q = (float)io.q[g - (int64_t)var * R.n];
    const float kq = (float)kKappa * q;

    // The lanes of a wavefront walk the checkpoint segments together, from
    // the wavefront's last one down: a lane whose own last segment is lower
    // waits until the walk reaches it.  Lanes then read the same tape and
    // checkpoint rows at the same time (one cache line per 8 lanes), where
    // each lane starting at its own last segment would split a wavefront's
    // reads over several rows.  Every lane's arithmetic and its order are
    // unchanged.
    const int top = (live && status != MT_ST_INVALID && ns > 0) ? (ns - 1) / kCkptEvery : -1;
    int wtop = top;
    for (int o = kWave / 2; o > 0; o >>= 1) wtop = max(wtop, __shfl_xor(wtop, o));
    wtop = __builtin_amdgcn_readfirstlane(wtop);

    {
        for (int seg = wtop; seg >= 0; --seg) {
            if (seg > top) continue;
            const int k0 = seg * kCkptEvery;
            const int k1 = min(k0 + kCkptEvery, ns);
            Lane L;
            const double *c = R.ckpt + (size_t)seg * 6 * lanes + g;
            L.x = c[0];
            L.y = c[lanes];
            L.z = c[2 * lanes];
            L.px = c[3 * lanes];
            L.py = c[4 * lanes];
            L.pz = c[5 * lanes];
            L.q = q;
            // kick records of the segment: three floats per (step, lane)
            const float *rec = R.tape + ((size_t)k0 * lanes + g) * 3;
            L.bvol = -2;
            L.vol = -1;                  // lookup caches start empty
            L.slab = -1;
            L.zlo = INFINITY;
            L.zhi = -INFINITY;
            // history of the segment: the pre-kick momentum p0 of every step
            // (FP32), [step][3][thread] in LDS (LDSH) or one 12-byte record per
            // (step, lane) in device memory.  The stage-0 momentum a0 is formed
            // again from p0 in the reverse sweep (kick_again), which halves the
            // history traffic the adjoint is bound by.
            float *hp;
            int64_t hs;
            if (LDSH) {
                hp = hist;
                hs = bd;
            } else {
                hp = nullptr;
                hs = 0;
            }
            Float3r *h3 = reinterpret_cast<Float3r *>(scratch) + g;
            double *hr = reinterpret_cast<double *>(
                scratch + (size_t)kCkptEvery * sizeof(Float3r) * lanes) + g;
            // running pointers (one 64-bit add per array and step) rather
            // than (k - k0) * lanes products
            const size_t rs = (size_t)lanes * 3;     // record stride between steps
            const float *rp = rec;
            Float3r *h3p = h3;
            double *hrp = hr;
            float3 next = make_float3(rp[0], rp[1], rp[2]);
            for (int k = k0; k < k1; ++k) {
                const float3 cur = next;
                rp += rs;
                if (k + 1 < k1) next = make_float3(rp[0], rp[1], rp[2]);
                const float p0x = (float)L.px, p0y = (float)L.py, p0z = (float)L.pz;
                if (MAP) {
                    hrp[0] = L.x;
                    hrp[lanes] = L.y;
                    hrp[2 * lanes] = L.z;
                    hrp += 3 * lanes;
                }
                vh[(k - k0) * bd] = (int8_t)replay_step<MAP>(L, T, S, R, sc, var, cur);
                if (LDSH) {
                    float *h = hp + (size_t)(k - k0) * 3 * hs;
                    h[0] = p0x;
                    h[hs] = p0y;
                    h[2 * hs] = p0z;
                } else {
                    *h3p = Float3r{p0x, p0y, p0z};
                    h3p += lanes;
                }
            }
            int bvol = -2;
            float3 bb = make_float3(0.f, 0.f, 0.f);
            int acc_m = -1;
            double acc = 0.0;
            // the reverse sweep loads step k-1's kick record and history
            // while it works on step k
            rp -= rs;                    // step k1 - 1
            h3p -= lanes;
            hrp -= 3 * lanes;
            next = make_float3(rp[0], rp[1], rp[2]);
            Float3r nP{0.f, 0.f, 0.f};
            double nx = 0.0, ny = 0.0, nz = 0.0;
            if (!LDSH) nP = *h3p;
            if (MAP) {
                nx = hrp[0];
                ny = hrp[lanes];
                nz = hrp[2 * lanes];
            }
            for (int k = k1 - 1; k >= k0; --k) {
                const float3 cur = next;
                const Float3r P = nP;
                const double rx = nx, ry = ny, rz = nz;
                if (k > k0) {
                    rp -= rs;
                    next = make_float3(rp[0], rp[1], rp[2]);
                    if (!LDSH) {
                        h3p -= lanes;
                        nP = *h3p;
                    }
                    if (MAP) {
                        hrp -= 3 * lanes;
                        nx = hrp[0];
                        ny = hrp[lanes];
                        nz = hrp[2 * lanes];
                    }
                }
                float3 p0;
                if (LDSH) {
                    const float *h = hp + (size_t)(k - k0) * 3 * hs;
                    p0 = make_float3(h[0], h[hs], h[2 * hs]);
                } else {
                    p0 = make_float3(P.x, P.y, P.z);
                }
                const int vol = vh[(k - k0) * bd];
                const float3 a0 = (vol >= 0 && S.mat[vol] >= 0) ? kick_again(p0, cur) : p0;
                if (vol != bvol) {
                    bb = box_field(T, S, R, vol, var);
                    bvol = vol;
                }
                int m;
                double d;
                reverse_step<MAP>(T, S, R, sc, kq, p0, a0, rx, ry, rz, vol,
                                  make_float3(cur.x, cur.y, cur.z), bb, lr, lp, m, d);
                // scale gradient: accumulate in a register while the magnet is unchanged
                if (m != acc_m) {
                    if (acc_m >= 0) sgs[acc_m * bd] += acc;
                    acc_m = m;
                    acc = 0.0;
                }
                acc += d;
            }
            if (acc_m >= 0) sgs[acc_m * bd] += acc;
        }
    }
    if (!live) return;
    for (int a = 0; a < 3; ++a) {
        g_in[a * lanes + g] = lr[a];
        g_in[(3 + a) * lanes + g] = lp[a];
    }
    for (int m = 0; m < n_mag; ++m) gs_lane[(size_t)m * lanes + g] = sgs[m * bd];
}

// ---------------------------------------------------------------------------
// Deterministic per-variant sums (fixed chunking and fixed tree order).
// ---------------------------------------------------------------------------
constexpr int kRedBlock = 256;

template <int NC, typename F>
__device__ __forceinline__ void block_partial(F &&term, int64_t begin, int64_t end,
                                              double *partial_out) {
    __shared__ double red[NC][kRedBlock];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    // eight elements per thread in flight; each accumulator still adds its
    // elements in index order
    int64_t i = begin + threadIdx.x;
    for (; i + 7 * kRedBlock < end; i += 8 * kRedBlock) {
#pragma unroll
        for (int u = 0; u < 8; ++u) term(i + u * kRedBlock, acc);
    }
    for (; i < end; i += kRedBlock) term(i, acc);
#pragma unroll
    for (int c = 0; c < NC; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < NC; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) partial_out[c] = red[c][0];
    }
}

__global__ void __launch_bounds__(kRedBlock) k_tally_pass1(DevIO io, int64_t n, double z_det,
                                                           double r_ap, double r_scale,
                                                           double *partial) {
    const int v = blockIdx.y, b = blockIdx.x, nb = gridDim.x;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t base = (int64_t)v * n;
    const int64_t begin = base + min((int64_t)b * chunk, n);
    const int64_t end = base + min((int64_t)(b + 1) * chunk, n);
    auto term = [&](int64_t i, double *acc) {
        if (io.status[i] == MT_ST_ZMAX) {
            const double dz = z_det - io.oz[i];
            const double xd = io.ox[i] + dz * io.opx[i] / io.opz[i];
            const double yd = io.oy[i] + dz * io.opy[i] / io.opz[i];
            const double r = sqrt(xd * xd + yd * yd);
            acc[0] += 1.0;
            acc[1] += (r < r_ap) ? 1.0 : 0.0;
            acc[2] += 1.0 / (1.0 + exp(-(r_ap - r) / r_scale));
        }
    };
    block_partial<3>(term, begin, end, partial + ((size_t)v * nb + b) * 3);
}

// One block per (chunk b, variant v, column c): each column is summed on
// its own, in the same order and tree as every other column.
__global__ void __launch_bounds__(kRedBlock) k_colsum_pass1(const double *vals, int n_cols,
                                                            int64_t n, int64_t lanes,
                                                            double *partial) {
    const int v = blockIdx.y, b = blockIdx.x, nb = gridDim.x, c = blockIdx.z;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t base = (int64_t)v * n;
    const int64_t begin = base + min((int64_t)b * chunk, n);
    const int64_t end = base + min((int64_t)(b + 1) * chunk, n);
    const double *col = vals + (size_t)c * lanes;
    auto term = [&](int64_t i, double *acc) { acc[0] += col[i]; };
    block_partial<1>(term, begin, end, partial + ((size_t)v * nb + b) * n_cols + c);
}

// out[v][c] = sum over b of partial[v][b][c], in order of b.
__global__ void k_pass2(const double *partial, int nb, int n_cols, int n_variants, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_variants * n_cols) return;
    const int v = i / n_cols, c = i - v * n_cols;
    const double *p = partial + (size_t)v * nb * n_cols + c;
    double s = 0.0;
    int b = 0;
    for (; b + 8 <= nb; b += 8) {        // loads of eight partials in flight, sums in order of b
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = p[(size_t)(b + u) * n_cols];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u];
    }
    for (; b < nb; ++b) s += p[(size_t)b * n_cols];
    out[i] = s;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <unsigned F>
static const void *plain_kernel() {
    if constexpr (valid_mask(F)) return reinterpret_cast<const void *>(&k_plain<F>);
    else return nullptr;
}

template <unsigned F>
static const void *persistent_kernel() {
    if constexpr (valid_mask(F) && !(F & kTape))
        return reinterpret_cast<const void *>(&k_pass<F>);
    else return nullptr;
}

template <unsigned F>
static const void *variant_waves_kernel() {
    if constexpr (valid_mask(F) && !(F & (kTape | kTrace)))
        return reinterpret_cast<const void *>(&k_variant_waves<F>);
    else return nullptr;
}

template <size_t... I>
static std::array<const void *, sizeof...(I)> variant_waves_kernels(std::index_sequence<I...>) {
    return {variant_waves_kernel<(unsigned)I>()...};
}

template <size_t... I>
static std::array<const void *, sizeof...(I)> plain_kernels(std::index_sequence<I...>) {
    return {plain_kernel<(unsigned)I>()...};
}

template <size_t... I>
static std::array<const void *, sizeof...(I)> persistent_kernels(std::index_sequence<I...>) {
    return {persistent_kernel<(unsigned)I>()...};
}

static unsigned feature_mask(const Tables &T, const DevRun &R) {
    const bool map = T.field.map != nullptr;
    return (map ? kMap : 0u) | (R.ckpt != nullptr ? kTape : 0u) |
           (R.n_trace > 0 ? kTrace : 0u) | (R.sampler == MT_SAMPLER_ALIAS ? kAlias : 0u) |
           (map && R.interp == MT_INTERP_NEAREST ? kNearest : 0u) |
           (R.stage_field ? kStages : 0u) | (T.geom.n_poly > 0 ? kPoly : 0u) |
           (T.hist.log_loss || T.hist.log_scat ? kLog : 0u);
}

hipError_t launch_plain(const Tables &T, const DevRun &R, const DevIO &io, int block,
                        hipStream_t s) {
    static const auto fns = plain_kernels(std::make_index_sequence<kFeatures>());
    if (R.lanes == 0) return hipSuccess;
    const unsigned grid = (unsigned)((R.lanes + block - 1) / block);
    Tables t = T;
    DevRun r = R;
    DevIO o = io;
    void *args[] = {&t, &r, &o};
    const void *fn = fns[feature_mask(T, R)];
    if (fn == nullptr) return hipErrorInvalidValue;     // excluded by argument validation
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, (size_t)T.lds.bytes, s);
}

static size_t persistent_lds(const Tables &T) { return (size_t)T.lds.bytes; }

static const void *persistent_fn(unsigned mask) {
    static const auto fns = persistent_kernels(std::make_index_sequence<kFeatures>());
    return fns[mask];
}

hipError_t launch_pass(const Tables &T, const DevRun &R, const DevIO &io, int block,
                       const PassArgs &P, hipStream_t s) {
    if (R.lanes == 0) return hipSuccess;
    // sized for every lane (the survivors of a pass are at most that many);
    // blocks past the pass's items exit before staging their tables
    const unsigned grid = (unsigned)((R.lanes + block - 1) / block);
    Tables t = T;
    DevRun r = R;
    DevIO o = io;
    PassArgs pa = P;
    void *args[] = {&t, &r, &o, &pa};
    const void *fn = persistent_fn(feature_mask(T, R) & ~kTape);
    if (fn == nullptr) return hipErrorInvalidValue;     // excluded by argument validation
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, persistent_lds(T), s);
}

hipError_t launch_variant_waves(const Tables &T, const DevRun &R, const DevIO &io, int block,
                               hipStream_t s) {
    static const auto fns = variant_waves_kernels(std::make_index_sequence<kFeatures>());
    if (R.lanes == 0) return hipSuccess;
    // (muon, group of G variants) units, 64 / G per wavefront
    const int64_t units = R.lanes >> R.share_shift;
    const int64_t per_wave = kWave >> R.share_shift;
    const int64_t waves = (units + per_wave - 1) / per_wave;
    const int64_t per_block = block / kWave;
    const unsigned grid = (unsigned)((waves + per_block - 1) / per_block);
    Tables t = T;
    DevRun r = R;
    DevIO o = io;
    void *args[] = {&t, &r, &o};
    const void *fn = fns[feature_mask(T, R)];
    if (fn == nullptr) return hipErrorInvalidValue;     // excluded by argument validation
    const size_t lds = (size_t)((T.lds.bytes + 15) & ~15) + (size_t)block * sizeof(uint4);
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, s);
}

hipError_t launch_queue_reset(unsigned long long *queue, double *zero, int64_t n_zero,
                              hipStream_t s) {
    const int64_t n = n_zero > 1 ? n_zero : 1;
    hipLaunchKernelGGL(k_queue_reset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, queue,
                       zero, n_zero);
    return hipGetLastError();
}

int64_t adjoint_scratch_bytes(const Tables &T, int64_t lanes) {
    return (int64_t)kCkptEvery * (sizeof(Float3r) + 3 * sizeof(double)) * lanes;
}

// Where the adjoint keeps a segment's start states: device memory (default;
// at 16 steps x 12 B per lane it stays L2/Infinity-Cache resident and leaves
// LDS free for occupancy) or, on request and without a field map, LDS.
hipError_t launch_adjoint(const Tables &T, const DevRun &R, const DevIO &io,
                          const double *g_out, double *g_in, double *gs_lane, void *scratch,
                          int block, bool lds_history, hipStream_t s) {
    if (R.lanes == 0) return hipSuccess;
    const int64_t grid = (R.lanes + block - 1) / block;
    const bool map = T.field.map != nullptr;
    const bool ldsh = lds_history && !map;
    size_t shm = (size_t)((T.lds.bytes + 15) & ~15) + (size_t)T.geom.n_mag * block * sizeof(double);
    if (ldsh) shm += (size_t)kCkptEvery * 3 * block * sizeof(float);   // p0 per step
    shm += (size_t)kCkptEvery * block;                                   // volume per step
    char *sc = reinterpret_cast<char *>(scratch);
    if (map)
        hipLaunchKernelGGL((k_adjoint<true, false>), dim3((unsigned)grid), dim3(block), shm, s, T, R, io, g_out, g_in, gs_lane, sc);
    else if (ldsh)
        hipLaunchKernelGGL((k_adjoint<false, true>), dim3((unsigned)grid), dim3(block), shm, s, T, R, io, g_out, g_in, gs_lane, sc);
    else
        hipLaunchKernelGGL((k_adjoint<false, false>), dim3((unsigned)grid), dim3(block), shm, s, T, R, io, g_out, g_in, gs_lane, sc);
    return hipGetLastError();
}

hipError_t launch_tally(const DevIO &io, int64_t n, int32_t n_variants, double z_det,
                        double r_ap, double r_scale, double *partial, int32_t n_part_blocks,
                        double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_tally_pass1, dim3(n_part_blocks, n_variants), dim3(kRedBlock), 0, s, io,
                       n, z_det, r_ap, r_scale, partial);
    const int nout = n_variants * 3;
    hipLaunchKernelGGL(k_pass2, dim3((nout + 127) / 128), dim3(128), 0, s, partial, n_part_blocks,
                       3, n_variants, out);
    return hipGetLastError();
}

hipError_t launch_column_sums(const double *vals, int32_t n_cols, int64_t n, int32_t n_variants,
                              double *partial, int32_t n_part_blocks, double *out, hipStream_t s) {
    if (n_cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colsum_pass1, dim3(n_part_blocks, n_variants, n_cols), dim3(kRedBlock),
                       0, s, vals, n_cols, n, n * n_variants, partial);
    const int nout = n_variants * n_cols;
    hipLaunchKernelGGL(k_pass2, dim3((nout + 127) / 128), dim3(128), 0, s, partial, n_part_blocks,
                       n_cols, n_variants, out);
    return hipGetLastError();
}

}  // namespace mt
