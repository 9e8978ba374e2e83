// Batched rank-Greville update with the stream state on chip and blocks of
// rows applied through FP64 matrix-core products (v_mfma_f64_16x16x4f64).
//
// The dual basis Ct = (C C^T)^-1 C of Section 2.1 is kept in factored form:
// C (the accepted raw rows, exact in FP32 for FP32 inputs) and
// H^-1 = (C C^T)^-1 in FP64, so that every projection gamma = Ct Gamma is
// formed as H^-1 (C Gamma) with FP64 arithmetic on exact FP32 rows.  An
// FP32-stored Ct would perturb the projections by about 2^-24 kappa(C), and
// that error does not cancel in x; in factored form it is about
// 2^-52 kappa(C)^2.  The independent update of Theorem 6 (Ct <- [Ct - gamma
// K^T; K^T]) is, on the factors, the bordering of H^-1 with the rejection's
// squared norm as Schur complement:
//   H^-1 <- [[H^-1 + gamma gamma^T / s, -gamma / s], [-gamma^T / s, 1 / s]],
//   s = ||Gamma_r||^2,
// O(r^2) instead of the O(r m) update of an explicit Ct.
//
// One workgroup of NW waves (4 or 8) owns one stream for a whole push.  Lane
// l of wave w has i = l & 15 and g = l >> 4.  Residency:
//   C     LDS, in the element type of the stream (FP32; FP64 in the FP64
//         variant), row-major, leading dimension MMAX.  Logical chunk of four
//         elements c of row k sits at physical chunk c ^ (k & 15), so that the
//         16 rows a matrix-core operand touches fall into different banks;
//   P^-1, H^-1  registers, FP64, 16 x 16 output tiles (u', u) for the column
//         tiles u = w + NW ups of this wave:
//         p[u'][ups][v] = P^-1[16u' + 4v + g][16u + i], h likewise;
//   w     registers, FP64: wr[ups][v] = w[16 (w + NW ups) + 4v + g].
// The matrix-core operands of v_mfma_f64_16x16x4f64 are A[i][g] and B[g][i]
// on lane (i, g), and the result D[4v + g][i] sits in register v of lane
// (i, g); the layouts above are chosen so that results feed later products
// without shuffles.  P^-1 and H^-1 are symmetric, so the same registers are
// the A operand of products with them.
//
// Rows are taken in two modes.
//  Row mode (Algorithm 1, one row): v = C Gamma over LDS with 16-lane DPP
//   sums; gamma = H^-1 v, C^T gamma, zeta = P^-1 gamma and gamma^T w per
//   column tile with one reduce-scatter over the 4 lane groups each; rank
//   test on workgroup sums; then the dependent update of P^-1 and w
//   (Theorems 5 and 6), or the independent one (bordering of H^-1 and P^-1,
//   appends to C and w; Theorems 4 and 6).
//  Block mode (up to 16 rows): V = Gamma_blk C^T, G = V H^-1 and the
//   rejections R = Gamma_blk - G C on the matrix cores; the rank test of
//   Section 3 on every row.
//   A prefix of dependent rows (nd rows) is applied at once: applying the
//   rows j = 0..nd-1 one after another is the same as the Woodbury form with
//   Z = P^-1 G^T, S = I + G Z:
//     P^-1 <- P^-1 - Z S^-1 Z^T,   w <- w + Z S^-1 (y - G w),
//   and the pivots of the Cholesky factor S = L L^T are exactly the
//   sequential Greville denominators 1 + gamma_j^T P_j^-1 gamma_j, so their
//   test is the same.  With T = Z L^-T the updates are P^-1 -= T T^T and
//   w += T (L^-1 (y - G w)).
//   A prefix of independent rows (ni rows) is appended at once: with
//   R R^T = L L^T (its pivots are the sequential squared rejection norms, so
//   the rank test of every row is the row-by-row test) and W = L^-1,
//     H^-1 <- [[H^-1, 0], [0, 0]] + U U^T,  U = [G^T W^T; -W^T],
//   C <- [C; Gamma_blk], P^-1 <- diag(P^-1, I), w <- [w; y_blk].
//   The first row of the other kind ends the block.
// Every branch is on workgroup-uniform values.
#include <algorithm>

#include "rg_classes.h"
#include "rg_lanes.h"

namespace rg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Independent runs: a Gram pivot below this fraction of its diagonal ends the run.
constexpr double PIV_AMBIG = 1e-4;

// 1/sqrt(x) in FP64: the hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2, each of which doubles the number of correct bits.
__device__ inline double rsqrt_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

template <int RMAX_, int MMAX_, int NW_, typename E_ = float>
struct MF {
    static constexpr int RMAX = RMAX_, MMAX = MMAX_, NW = NW_;
    using E = E_;                                 // element type of C and of the rows (FP32 or FP64)
    static constexpr int EW = sizeof(E) / 4;      // 32-bit words per element
    static_assert((RMAX == 64 || RMAX == 128) && (RMAX / 16) % NW == 0, "whole row tiles per wave");
    static_assert(MMAX % 64 == 0 && MMAX <= 256 && (NW == 4 || NW == 8), "4 or 8 waves");
    static constexpr int NT = 64 * NW;
    static constexpr int NU = RMAX / 16, UPW = NU / NW;               // 16-row tiles, per wave
    static constexpr int NTT = MMAX / 16, TPW = (NTT + NW - 1) / NW;  // 16-column tiles, per wave
    static_assert(TPW <= 4 && UPW <= 2, "one reduce-scatter holds the column and zeta totals");
    static constexpr int RS = 4 * NW;                                 // row stride of a thread in row mode
    static constexpr int NB = RMAX / RS;                              // C rows per thread in row mode
    static constexpr int KB = 16;                                     // rows per block
    static constexpr int CH = MMAX / 4;                               // chunks of 4 elements per row
    // X1 (doubles): block-mode scalars and partial sums, or the row-mode vectors
    static constexpr int X1_RR = 0, X1_GW = 16 * NW, X1_GG = 32 * NW, X1_YV = 32 * NW + 16;
    // S partials: 4 records of 16 x 16 with row stride 17, so that reading one row per lane is free of bank conflicts
    static constexpr int SPR = 17, SPS = 16 * SPR;
    static constexpr int X1_SP = 32 * NW + 64, X1_L = X1_SP + 4 * SPS, X1_C = X1_L + 256, X1_COL = X1_C + 32;
    // Waves per SIMD the register allocation is held to: two for the 4-wave
    // variants whose LDS footprint lets two workgroups share a CU (m <= 192)
    static constexpr int OCC = (NW == 4 && MMAX <= 192 && EW == 1) ? 2 : 1;
    // HG: H^-1 stays in the stream's state in global memory (L2-resident) instead of
    // registers, where P^-1 and H^-1 together would not fit (RMAX = 128).  It is
    // only read by dependent rows, and each lane reads and writes its own tile
    // elements, in the register layout, when rows are appended.
    static constexpr bool HG = RMAX == 128;
    static constexpr int X1_DW = X1_COL + 96;
    // block mode, between the projections and the rejections: per-wave partial
    // sums of gamma^T v, ||gamma||^2, ||v||^2 and ||Gamma||^2 (4 x 16 NW doubles in
    // the S records' space)
    static constexpr int X1_CT = X1_SP;
    static_assert(4 * 16 * NW <= 4 * SPS, "room for the projection records");
    static constexpr int X1_W = X1_SP;  // independent block: W = L^-1 (row-major 16 x 16), after the records are read
    // row mode: gamma, zeta, v = C Gamma, the reduction records, Gamma_r (three separate
    // vectors, so that no row writes one that a wave may still read for the row before)
    static constexpr int X1_GAM = 0, X1_ZETA = RMAX, X1_V = 2 * RMAX, X1_RED = 3 * RMAX, X1_GR = 3 * RMAX + 4 * NW;
    static constexpr int X1_D = cmax(cmax(KB * MMAX * EW / 2, X1_DW + RMAX), X1_GR + MMAX);
    // X2 (doubles): V and G (16 x RMAX), then Z, T or U (RMAX x 16); or the row ring
    static constexpr int X2_D = cmax(KB * RMAX, 3 * MMAX * EW / 2);
    // X3 (doubles, FP64 variant only): the rejections R (16 x MMAX, swizzled like
    // the block rows) and V2 = R C^T, then G2 = V2 H^-1 (16 x RMAX), for the
    // second projection of a block's rejections
    static constexpr int X3_D = EW == 2 ? 16 * MMAX + 16 * RMAX : 0;
};

// Chunks of four elements: float4 for FP32 streams, double4 for FP64 streams.
template <typename T>
struct V4T;
template <>
struct V4T<float> {
    typedef float4 type;
};
template <>
struct V4T<double> {
    typedef double4 type;
};
template <typename T>
__device__ inline typename V4T<T>::type mk4(T a, T b, T c, T d);
template <>
__device__ inline float4 mk4<float>(float a, float b, float c, float d) {
    return make_float4(a, b, c, d);
}
template <>
__device__ inline double4 mk4<double>(double a, double b, double c, double d) {
    return make_double4(a, b, c, d);
}

// Swizzled positions of G[j][kk] (16 x RMAX) and of Z, T, U [kk][j] (RMAX x 16).
template <int RMAX>
__device__ inline int gpos(int j, int kk) { return j * RMAX + (kk ^ (4 * (j & 7))); }
__device__ inline int zpos(int kk, int j) { return kk * 16 + (j ^ (4 * ((kk >> 1) & 3))); }

// Sums of four per-lane partials over the workgroup (every thread gets them).
template <int NW>
__device__ inline void block_sum4(double &a, double &b, double &c, double &d, double *sred) {
    a = sum64(a);
    b = sum64(b);
    c = sum64(c);
    d = sum64(d);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sred[4 * wid] = a;
        sred[4 * wid + 1] = b;
        sred[4 * wid + 2] = c;
        sred[4 * wid + 3] = d;
    }
    __syncthreads();
    a = b = c = d = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        a += sred[4 * q];
        b += sred[4 * q + 1];
        c += sred[4 * q + 2];
        d += sred[4 * q + 3];
    }
}

// One stream's push by the whole workgroup (every thread calls it with the same
// b_id and returns at the same point).
template <class K>
__device__ __forceinline__ void push_stream(const PushArgs<typename K::E> &a, int ra, int b_id, double *smem) {
    using E = typename K::E;
    using V4 = typename V4T<E>::type;
    constexpr int RMAX = K::RMAX, MMAX = K::MMAX, NU = K::NU, UPW = K::UPW, TPW = K::TPW;
    constexpr int NB = K::NB, KB = K::KB, CH = K::CH, NW = K::NW, NTT = K::NTT, RS = K::RS;
    E *sct = reinterpret_cast<E *>(smem);  // C: ra x MMAX (ra: multiple of 16)
    double *x1 = smem + (size_t)ra * MMAX * K::EW / 2;
    double *x2 = x1 + K::X1_D;
    E *x1f = reinterpret_cast<E *>(x1);   // block rows, 16 x MMAX, swizzled like C
    E *ring = reinterpret_cast<E *>(x2);  // row mode: 3 rows of MMAX

    // the wave index is uniform over the wave: held in a scalar register, so that
    // branches and addresses that depend only on it are scalar
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    StreamMeta *M = a.meta + b_id;
    const int m = M->m, rmax = M->r_max, ldm = M->ldm;
    int r = M->r;
    uint32_t flags = M->flags;
    E *Cg = a.state + M->state_off;
    double *Pg = a.preg + M->p_off;
    double *Hg = a.hreg + M->h_off;
    double *wg = a.wreg + M->w_off;
    int64_t i0, i1, goff;
    if (a.row_ptr) {
        i0 = a.row_ptr[b_id];
        i1 = a.row_ptr[b_id + 1];
        goff = a.gamma_off[b_id];
    } else {
        i0 = 0;
        i1 = a.k_single;
        goff = 0;
    }
    if (flags != 0u || i0 >= i1) return;  // whole workgroup: nothing to do
    const E *G0 = a.gamma + goff;     // row i starts at G0 + (i - i0) * m
    const int cba4 = (m + 63) / 64;       // 64-column groups (row mode)
    const int nq = (m + 15) / 16;         // 16-column chunks (block mode)

    // ---- load the state ------------------------------------------------------
    double trh = 0.0;  // trace(C C^T) = sum of the squared norms of the rows of C
    for (int idx = t; idx < ra * CH; idx += K::NT) {
        const int k = idx / CH, c = idx - k * CH;
        E v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * c + e;
            v[e] = (k < r && j < m) ? Cg[(size_t)k * ldm + j] : 0.0f;
            trh += (double)v[e] * (double)v[e];
        }
        *reinterpret_cast<V4 *>(sct + (size_t)k * MMAX + 4 * (c ^ (k & 15))) = mk4<E>(v[0], v[1], v[2], v[3]);
    }
    {
        double z0 = 0.0, z1 = 0.0, z2 = 0.0;
        block_sum4<NW>(trh, z0, z1, z2, x1 + K::X1_RED);
    }
    const int li = lane & 15, lg = lane >> 4;
    constexpr int NUH = K::HG ? 1 : NU, UPWH = K::HG ? 1 : UPW;
    d4 p[NU][UPW], h[NUH][UPWH];
    double wr[UPW][4];
    // Tile (u2, u = wv + NW ups) of H^-1 for the current rank rr (entries past
    // rr read as zero), and its store (entries past rr are not written)
    // Raw tile loads (HG): unconditional, element 0 for entries past rr, so that
    // the loads of several tiles are in flight together; hmask zeroes those
    // entries where the tile is used.
    // (the _t forms name the column tile ut and take the rows rlo .. rlim-1 only, rlim <= rr)
    auto hraw_t = [&](int u2, int ut, int rr, int rlo, int rlim) -> d4 {
        const int col = 16 * ut + (lane & 15);
        d4 o;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * u2 + 4 * v + (lane >> 4);
            const bool in = row >= rlo && row < rlim && col < rr;
            int64_t idx = in ? (int64_t)row * rmax + col : 0;
            asm("" : "+v"(idx));
            o[v] = Hg[idx];
        }
        return o;
    };
    auto hmask_t = [&](int u2, int ut, int rr, int rlo, int rlim, const d4 &raw) -> d4 {
        const int col = 16 * ut + (lane & 15);
        d4 o;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * u2 + 4 * v + (lane >> 4);
            o[v] = row >= rlo && row < rlim && col < rr ? raw[v] : 0.0;
        }
        return o;
    };
    auto hraw = [&](int u2, int ups, int rr) -> d4 { return hraw_t(u2, wv + NW * ups, rr, 0, rr); };
    auto hmask = [&](int u2, int ups, int rr, const d4 &raw) -> d4 { return hmask_t(u2, wv + NW * ups, rr, 0, rr, raw); };
    auto hload = [&](int u2, int ups, int rr) -> d4 {
        if constexpr (K::HG) {
            return hmask(u2, ups, rr, hraw(u2, ups, rr));
        } else {
            return h[u2][ups];
        }
    };
    auto hstore = [&](int u2, int ups, const d4 &val, int rr) {
        if constexpr (K::HG) {
            const int col = 16 * (wv + NW * ups) + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * u2 + 4 * v + (lane >> 4);
                if (row < rr && col < rr) Hg[(size_t)row * rmax + col] = val[v];
            }
        } else {
            h[u2][ups] = val;
        }
    };
#pragma unroll
    for (int ups = 0; ups < UPW; ++ups) {
        const int col = 16 * (wv + NW * ups) + li;
#pragma unroll
        for (int u2 = 0; u2 < NU; ++u2)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * u2 + 4 * v + lg;
                const bool in = row < r && col < r;
                p[u2][ups][v] = in ? Pg[(size_t)row * rmax + col] : 0.0;
                if constexpr (!K::HG) h[u2][ups][v] = in ? Hg[(size_t)row * rmax + col] : 0.0;
            }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = 16 * (wv + NW * ups) + 4 * v + lg;
            wr[ups][v] = kk < r ? wg[kk] : 0.0;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // Block rows come through registers: pfv holds rows pf_i .. pf_i + 15 as
    // chunks of four elements (thread tl has chunks tl + NT e), pfy the target of row
    // pf_i + (lane & 15).
    constexpr int PFB = (KB * CH + K::NT - 1) / K::NT;
    V4 pfv[PFB];
    E pfy = 0;
    int64_t pf_i = -1;
    auto fetch_block = [&](const E *src0, const E *ysrc, int nrows, int mm, int tid, V4 (&dst)[PFB], E &ydst) {
#pragma unroll
        for (int e = 0; e < PFB; ++e) {
            const int idx = tid + K::NT * e, j = idx / CH, cc = idx - j * CH;
            const E *src = src0 + (int64_t)j * mm;
            E v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = 4 * cc + q;
                v[q] = (idx < KB * CH && j < nrows && col < mm) ? src[col] : 0.0f;
            }
            dst[e] = mk4<E>(v[0], v[1], v[2], v[3]);
        }
        ydst = (tid & 15) < nrows ? ysrc[tid & 15] : 0.0f;
    };
    const bool use_blocks = !(a.opts & OPT_ROW_BY_ROW);
    const bool ind_blocks = use_blocks && !(a.opts & OPT_DEPENDENT_BLOCKS_ONLY);
    int64_t i = i0, applied = 0;
    bool block_mode = ind_blocks;
    bool ring_ok = false;  // row mode: row i is in ring slot cur, pre holds row i + 1
    int cur = 0;
    constexpr int PF = (MMAX + K::NT - 1) / K::NT;
    E pre[PF];
    E y_next = 0;

    while (i < i1) {
        // Lane indices are re-derived from an opaque copy of the lane id in every
        // iteration, so the per-lane (swizzled) LDS addresses are computed where
        // they are used instead of being held in registers across the loop.
        int lane_l = lane;
        asm volatile("" : "+v"(lane_l));
        const int li = lane_l & 15, lg = lane_l >> 4, tl = 64 * wv + lane_l;
        const int pk = tl >> 4, pj = tl & 15, pk15 = pk & 15;
        // C[4s + g][16 ct + i] in FP64 from LDS (rows past the rank and columns
        // past m are zero there; column tiles past MMAX read as zero)
        auto cval = [&](int s, int ct) -> double {
            if (ct >= NTT) return 0.0;
            const int k = 4 * s + lg, col = 16 * ct + li;
            return (double)sct[(size_t)k * MMAX + 4 * ((col >> 2) ^ (k & 15)) + (col & 3)];
        };
        if (block_mode) {
            // ================= block of up to KB rows =================
            __syncthreads();  // earlier readers of X1 / X2 are done
            const int nblk = (int)min((int64_t)KB, i1 - i);
            if (pf_i != i) fetch_block(G0 + (i - i0) * (int64_t)m, a.y + i, nblk, m, tl, pfv, pfy);
#pragma unroll
            for (int e = 0; e < PFB; ++e) {
                const int idx = tl + K::NT * e, j = idx / CH, cc = idx - j * CH;
                if (idx < KB * CH) *reinterpret_cast<V4 *>(x1f + j * MMAX + 4 * (cc ^ j)) = pfv[e];
            }
            const double yrow = (double)pfy;
            __syncthreads();
            // the next block's rows are requested now (used if all of this block applies)
            pf_i = i + nblk;
            if (pf_i < i1) fetch_block(G0 + (pf_i - i0) * (int64_t)m, a.y + pf_i, (int)min((int64_t)KB, i1 - pf_i), m, tl, pfv, pfy);

            // ---- V = Gamma_blk C^T: tiles u = wv + NW ups of V^T ----
            const int nur = (r + 15) / 16;
            // SIMD balance of the RMAX = 128 variants (one tile per wave, wave w on
            // SIMD w % 4).  With nur = 5 or 6 tiles, the waves w >= nur would idle
            // while SIMDs 0 and 1 carry two tiles each: they take pieces instead.
            // Tile 4 (nur = 5) is cut into 4 pieces of its inner dimension, tiles 4
            // and 5 (nur = 6) into 2, piece 0 staying with the tile's own wave and
            // piece p >= 1 going to wave nur + (p - 1) kx + (tile - 4); the pieces
            // meet in LDS in the free tile slots past nur and are summed in piece
            // order by the tile's own wave (a fixed order).  Every SIMD then carries
            // 1.25 or 1.5 tiles of V and of G = V H^-1.
            const int kx = nur - 4;
            const bool split = K::HG && (kx == 1 || kx == 2);
            int vt = wv, vp = 0, vpt = 1;  // this wave's tile, its piece, the tile's pieces
            if (split) {
                if (wv >= nur) {
                    vt = 4 + (wv - nur) % kx;
                    vp = 1 + (wv - nur) / kx;
                }
                if (vt >= 4) vpt = 4 / kx;
            }
            const int vslot = vp == 0 ? vt : nur + (vp - 1) * kx + (vt - 4);  // LDS tile slot of the result
            d4 gacc[UPW];
            double gsq = 0.0;
            if constexpr (UPW == 1) {
                // chunk 4q + g of a row with (row & 15) == i sits at physical chunk (4q + g) ^ i
                d4 ga0 = (d4){0.0, 0.0, 0.0, 0.0}, ga1 = ga0;
                const int qs = vp * nq / vpt, qe = (vp + 1) * nq / vpt;
                const E *gbase = x1f + li * MMAX;
                if (vt < nur && qs < qe) {
                    const E *cb = sct + (size_t)(16 * vt + li) * MMAX;
                    auto ldg = [&](int q) { return *reinterpret_cast<const V4 *>(gbase + 4 * ((4 * q + lg) ^ li)); };
                    auto ldc = [&](int q) { return *reinterpret_cast<const V4 *>(cb + 4 * ((4 * q + lg) ^ li)); };
                    // two accumulators, so that consecutive products do not wait on each other
                    auto prod = [&](const V4 &gq, const V4 &cq) {
                        ga0 = mma((double)cq.x, (double)gq.x, ga0);
                        ga1 = mma((double)cq.y, (double)gq.y, ga1);
                        ga0 = mma((double)cq.z, (double)gq.z, ga0);
                        ga1 = mma((double)cq.w, (double)gq.w, ga1);
                    };
                    // two operand buffers: the loads of chunk q + 1 are in flight while
                    // chunk q is multiplied (past the range they load chunk qe - 1 again);
                    // the scheduling barriers keep the compiler from moving the loads
                    // down to their first use, and the loop has a single exit so that
                    // the accumulators stay where the products write them
                    V4 g0 = ldg(qs), c0 = ldc(qs);
                    int q = qs;
#pragma unroll 1
                    for (; q + 1 < qe; q += 2) {
                        const V4 g1 = ldg(q + 1), c1 = ldc(q + 1);
                        __builtin_amdgcn_sched_barrier(0);
                        prod(g0, c0);
                        const int q2 = min(q + 2, qe - 1);
                        g0 = ldg(q2);
                        c0 = ldc(q2);
                        __builtin_amdgcn_sched_barrier(0);
                        prod(g1, c1);
                    }
                    if (q < qe) prod(g0, c0);  // an odd last chunk (already loaded)
                }
                gacc[0] = ga0 + ga1;
#pragma unroll 1
                for (int q = wv; q < nq; q += NW) {  // this wave's share of ||Gamma_i||^2
                    const V4 gq = *reinterpret_cast<const V4 *>(gbase + 4 * ((4 * q + lg) ^ li));
                    const double b0 = gq.x, b1 = gq.y, b2 = gq.z, b3 = gq.w;
                    gsq += b0 * b0 + b1 * b1 + b2 * b2 + b3 * b3;
                }
            } else {
                d4 gacc2[UPW];
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) gacc[ups] = gacc2[ups] = (d4){0.0, 0.0, 0.0, 0.0};
                // chunk 4q + g of a row with (row & 15) == i sits at physical chunk (4q + g) ^ i;
                // the operands of chunk q + 1 are loaded while chunk q is multiplied
                const E *gbase = x1f + li * MMAX;
                const E *cbase[UPW];
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) cbase[ups] = sct + (size_t)(16 * (wv + NW * ups) + li) * MMAX;
                V4 gb = *reinterpret_cast<const V4 *>(gbase + 4 * (lg ^ li));
                V4 ca[UPW];
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups)
                    ca[ups] = wv + NW * ups < nur ? *reinterpret_cast<const V4 *>(cbase[ups] + 4 * (lg ^ li))
                                                  : mk4<E>(0, 0, 0, 0);
#pragma unroll 1
                for (int q = 0; q < nq; ++q) {
                    const V4 gq = gb;
                    V4 cq[UPW];
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) cq[ups] = ca[ups];
                    if (q + 1 < nq) {
                        const int phn = (4 * q + 4 + lg) ^ li;
                        gb = *reinterpret_cast<const V4 *>(gbase + 4 * phn);
#pragma unroll
                        for (int ups = 0; ups < UPW; ++ups)
                            if (wv + NW * ups < nur) ca[ups] = *reinterpret_cast<const V4 *>(cbase[ups] + 4 * phn);
                    }
                    const double b0 = gq.x, b1 = gq.y, b2 = gq.z, b3 = gq.w;
                    if ((q & (NW - 1)) == wv) gsq += b0 * b0 + b1 * b1 + b2 * b2 + b3 * b3;  // this wave's share
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) {
                        if (wv + NW * ups < nur) {
                            // two accumulators, so that consecutive products do not wait on each other
                            gacc[ups] = mma((double)cq[ups].x, b0, gacc[ups]);
                            gacc2[ups] = mma((double)cq[ups].y, b1, gacc2[ups]);
                            gacc[ups] = mma((double)cq[ups].z, b2, gacc[ups]);
                            gacc2[ups] = mma((double)cq[ups].w, b3, gacc2[ups]);
                        }
                    }
                }
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) gacc[ups] += gacc2[ups];
            }
            // this wave's share of ||Gamma_i||^2 (chunks wv, wv + NW, ...); the
            // shares are summed after the projections, in a fixed order
            gsq = sum_rows(gsq);
            if constexpr (UPW == 1) {
                if (vt < nur) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) x2[gpos<RMAX>(li, 16 * vslot + 4 * v + lg)] = gacc[0][v];
                }
            } else {
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                const int u = wv + NW * ups;
                if (u < nur) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) x2[gpos<RMAX>(li, 16 * u + 4 * v + lg)] = gacc[ups][v];
                }
            }
            }
            double gi[TPW][4];  // Gamma_blk[i][16 tl + 4 v + g] for this wave's column tiles
#pragma unroll
            for (int tau = 0; tau < TPW; ++tau)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    gi[tau][v] = wv + NW * tau < NTT ? (double)x1f[li * MMAX + 4 * ((4 * (wv + NW * tau) + v) ^ li) + lg] : 0.0;
            __syncthreads();
            if (split) {
                // V tiles 4 .. nur-1: the tile's own wave adds the other pieces
                if (wv >= 4 && wv < nur) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        double sv = x2[gpos<RMAX>(li, 16 * wv + 4 * v + lg)];
#pragma unroll
                        for (int pp = 1; pp < 4; ++pp)
                            if (pp < vpt) sv += x2[gpos<RMAX>(li, 16 * (nur + (pp - 1) * kx + (wv - 4)) + 4 * v + lg)];
                        x2[gpos<RMAX>(li, 16 * wv + 4 * v + lg)] = sv;
                    }
                }
                __syncthreads();
            }

            // ---- G^T = H^-1 V^T on this wave's row tiles (H^-1 symmetric) ----
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                const int u = wv + NW * ups;
                gacc[ups] = (d4){0.0, 0.0, 0.0, 0.0};
                if ((K::HG ? vt : u) < nur) {
                    d4 g2acc = (d4){0.0, 0.0, 0.0, 0.0};
                    if constexpr (K::HG) {
                        // tiles of H^-1 from L2, HB tiles' loads in flight at a time;
                        // this wave's piece takes the V tiles gs .. ge-1 of tile vt (the
                        // batches stay aligned to HB; tiles outside the piece read as zero)
                        constexpr int HB = 4;
                        const int gs = vp * nur / vpt, ge = (vp + 1) * nur / vpt;
                        const int rlo = 16 * gs, rlim = min(r, 16 * ge);
#pragma unroll 1
                        for (int ub = 0; ub < ge; ub += HB) {
                            d4 ht[HB];
#pragma unroll
                            for (int q = 0; q < HB; ++q)
                                ht[q] = hmask_t(ub + q, vt, r, rlo, rlim, hraw_t(ub + q, vt, r, rlo, rlim));
#pragma unroll
                            for (int q = 0; q < HB; ++q)
                                if (ub + q >= gs && ub + q < ge)
#pragma unroll
                                    for (int v = 0; v < 4; v += 2) {
                                        gacc[ups] = mma(ht[q][v], x2[gpos<RMAX>(li, 16 * (ub + q) + 4 * v + lg)], gacc[ups]);
                                        g2acc = mma(ht[q][v + 1], x2[gpos<RMAX>(li, 16 * (ub + q) + 4 * v + 4 + lg)], g2acc);
                                    }
                        }
                    } else {
#pragma unroll
                        for (int u2 = 0; u2 < NU; ++u2) {
                            if (u2 < nur) {
                                const d4 ht = hload(u2, ups, r);
#pragma unroll
                                for (int v = 0; v < 4; v += 2) {
                                    gacc[ups] = mma(ht[v], x2[gpos<RMAX>(li, 16 * u2 + 4 * v + lg)], gacc[ups]);
                                    g2acc = mma(ht[v + 1], x2[gpos<RMAX>(li, 16 * u2 + 4 * v + 4 + lg)], g2acc);
                                }
                            }
                        }
                    }
                    gacc[ups] += g2acc;
                }
            }
            if (split) {
                // G tiles 4 .. nur-1: the pieces go to the free slots past nur (V
                // stays in the slots below nur), the tile's own wave adds them
                if (vp > 0) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) x2[gpos<RMAX>(li, 16 * vslot + 4 * v + lg)] = gacc[0][v];
                }
                __syncthreads();
                if (wv >= 4 && wv < nur) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
#pragma unroll
                        for (int pp = 1; pp < 4; ++pp)
                            if (pp < vpt) gacc[0][v] += x2[gpos<RMAX>(li, 16 * (nur + (pp - 1) * kx + (wv - 4)) + 4 * v + lg)];
                }
            }
            // this wave's parts of gamma_i^T v_i, ||gamma_i||^2 and ||v_i||^2 (V is still in X2)
            double pgv = 0.0, pgg = 0.0, pvv = 0.0;
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                const int u = wv + NW * ups;
                if (u < nur) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double vv = x2[gpos<RMAX>(li, 16 * u + 4 * v + lg)];
                        pgv += gacc[ups][v] * vv;
                        pgg += gacc[ups][v] * gacc[ups][v];
                        pvv += vv * vv;
                    }
                }
            }
            __syncthreads();  // every read of V is done
            double gwp = 0.0;  // this wave's part of (G w)_i
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                const int u = wv + NW * ups;
                if (u < nur) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        gwp += gacc[ups][v] * wr[ups][v];
                        x2[gpos<RMAX>(li, 16 * u + 4 * v + lg)] = gacc[ups][v];
                    }
                }
            }
            gwp = sum_rows(gwp);
            pgv = sum_rows(pgv);
            pgg = sum_rows(pgg);
            pvv = sum_rows(pvv);
            if (lg == 0) {
                x1[K::X1_CT + 16 * wv + li] = pgv;
                x1[K::X1_CT + 16 * NW + 16 * wv + li] = pgg;
                x1[K::X1_CT + 32 * NW + 16 * wv + li] = pvv;
                x1[K::X1_CT + 48 * NW + 16 * wv + li] = gsq;
            }
            __syncthreads();

            // ---- rows that are dependent beyond doubt ----
            // ||R_i||^2 = ||Gamma_i||^2 - gamma_i^T v_i in exact arithmetic.  Its
            // rounding is bounded by 2^-52 (8 ||Gamma_i||^2 + 4 r ||gamma_i|| ||v_i||
            // + 64 r trace(C C^T) ||gamma_i||^2): the last term covers H^-1 as the
            // inverse of C C^T perturbed by a few r units of roundoff relative to
            // its norm.  When this bound keeps every row of the block below the
            // rank threshold of Section 3, all rows are dependent and the
            // rejections are not formed; otherwise they are, as below.
            bool skip_r;
            {
                double cgv = 0.0, cgg = 0.0, cvv = 0.0;
                gsq = 0.0;  // ||Gamma_i||^2
                // all records are requested before they are summed (the scheduling
                // barrier keeps the compiler from moving each read down to its sum,
                // which would serialise the reads)
                double rec[4][NW];
#pragma unroll
                for (int q = 0; q < NW; ++q)
#pragma unroll
                    for (int f = 0; f < 4; ++f) rec[f][q] = x1[K::X1_CT + 16 * NW * f + 16 * q + li];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    cgv += rec[0][q];
                    cgg += rec[1][q];
                    cvv += rec[2][q];
                    gsq += rec[3][q];
                }
                const double eps0 = a.eps >= 0.0 ? a.eps : ((double)m * m * r + (double)m * r + (double)m) * 0x1p-52;
                const double est = gsq - cgv;
                const double bnd = 0x1p-52 * (8.0 * gsq + 4.0 * r * sqrt(cgg * cvv) + 64.0 * r * trh * cgg);
                const bool sure = li >= nblk ||
                                  (isfinite(gsq) && isfinite(yrow) && est + bnd < eps0 * eps0 * fmax(1.0, gsq));
                skip_r = (__ballot(!sure) & 0xFFFFull) == 0 && !(a.opts & OPT_EXPLICIT_REJECTIONS);
            }

            // ---- R^T = Gamma_blk^T - C^T G^T, ||R_i||^2 and this wave's part of R R^T ----
            double rsq = 0.0;
            d4 sacc_r = (d4){0.0, 0.0, 0.0, 0.0};
            if constexpr (K::EW == 1) {
#pragma unroll
                for (int tau = 0; tau < TPW; ++tau) {
                    const int ct = wv + NW * tau;
                    if (ct < nq && !skip_r) {
                        d4 d = (d4){gi[tau][0], gi[tau][1], gi[tau][2], gi[tau][3]};
                        if constexpr (K::HG) {
#pragma unroll 1
                            for (int u2 = 0; u2 < nur; ++u2) {
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int s = 4 * u2 + v;
                                    d = mma(cval(s, ct), -x2[gpos<RMAX>(li, 4 * s + lg)], d);
                                }
                            }
                        } else {
#pragma unroll
                        for (int u2 = 0; u2 < NU; ++u2) {
                            if (u2 < nur) {
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int s = 4 * u2 + v;
                                    d = mma(cval(s, ct), -x2[gpos<RMAX>(li, 4 * s + lg)], d);
                                }
                            }
                        }
                        }
                        rsq += d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + d[3] * d[3];
#pragma unroll
                        for (int v = 0; v < 4; ++v) sacc_r = mma(d[v], d[v], sacc_r);
                    }
                }
            } else {
                // FP64 streams: the projections carry kappa(C)^2 2^-52 relative error
                // through H^-1, more than a small eps tolerates, so the rejections are
                // projected a second time (as in classical Gram-Schmidt with
                // reorthogonalisation): G2 = (R C^T) H^-1, R <- R - G2 C and G <- G + G2,
                // the refined coordinates of the block rows.
                static_assert(!K::HG, "H^-1 in registers");
                d4 dt[TPW];
#pragma unroll
                for (int tau = 0; tau < TPW; ++tau) {
                    const int ct = wv + NW * tau;
                    dt[tau] = (d4){0.0, 0.0, 0.0, 0.0};
                    if (ct < nq && !skip_r) {
                        d4 d = (d4){gi[tau][0], gi[tau][1], gi[tau][2], gi[tau][3]};
#pragma unroll
                        for (int u2 = 0; u2 < NU; ++u2) {
                            if (u2 < nur) {
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    const int s = 4 * u2 + v;
                                    d = mma(cval(s, ct), -x2[gpos<RMAX>(li, 4 * s + lg)], d);
                                }
                            }
                        }
                        dt[tau] = d;
                    }
                }
                if (!skip_r) {
                    double *xr = x2 + K::X2_D, *xv = xr + 16 * MMAX;
                    // R to X3, row i with chunk c at c ^ i (like the block rows)
#pragma unroll
                    for (int tau = 0; tau < TPW; ++tau) {
                        const int ct = wv + NW * tau;
                        if (ct < nq) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) xr[li * MMAX + 4 * ((4 * ct + v) ^ li) + lg] = dt[tau][v];
                        }
                    }
                    __syncthreads();
                    // V2 = R C^T on this wave's row tiles
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) {
                        const int u = wv + NW * ups;
                        if (u < nur) {
                            d4 va = (d4){0.0, 0.0, 0.0, 0.0}, vb = va;
#pragma unroll 1
                            for (int q = 0; q < nq; ++q) {
                                const int ph = (4 * q + lg) ^ li;
                                const V4 rv = *reinterpret_cast<const V4 *>(xr + li * MMAX + 4 * ph);
                                const V4 cv = *reinterpret_cast<const V4 *>(sct + (size_t)(16 * u + li) * MMAX + 4 * ph);
                                va = mma(cv.x, rv.x, va);
                                vb = mma(cv.y, rv.y, vb);
                                va = mma(cv.z, rv.z, va);
                                vb = mma(cv.w, rv.w, vb);
                            }
                            va += vb;
#pragma unroll
                            for (int v = 0; v < 4; ++v) xv[gpos<RMAX>(li, 16 * u + 4 * v + lg)] = va[v];
                        }
                    }
                    __syncthreads();
                    // G2 = V2 H^-1 on this wave's row tiles, and its part of G2 w
                    d4 g2[UPW];
                    double g2w = 0.0;
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) {
                        const int u = wv + NW * ups;
                        g2[ups] = (d4){0.0, 0.0, 0.0, 0.0};
                        if (u < nur) {
                            d4 gb2 = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                            for (int u2 = 0; u2 < NU; ++u2) {
                                if (u2 < nur) {
                                    const d4 ht = hload(u2, ups, r);
#pragma unroll
                                    for (int v = 0; v < 4; v += 2) {
                                        g2[ups] = mma(ht[v], xv[gpos<RMAX>(li, 16 * u2 + 4 * v + lg)], g2[ups]);
                                        gb2 = mma(ht[v + 1], xv[gpos<RMAX>(li, 16 * u2 + 4 * v + 4 + lg)], gb2);
                                    }
                                }
                            }
                            g2[ups] += gb2;
#pragma unroll
                            for (int v = 0; v < 4; ++v) g2w += g2[ups][v] * wr[ups][v];
                        }
                    }
                    gwp += sum_rows(g2w);
                    __syncthreads();  // every read of V2 is done
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) {
                        const int u = wv + NW * ups;
                        if (u < nur) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                xv[gpos<RMAX>(li, 16 * u + 4 * v + lg)] = g2[ups][v];
                                x2[gpos<RMAX>(li, 16 * u + 4 * v + lg)] += g2[ups][v];
                            }
                        }
                    }
                    __syncthreads();
                    // R <- R - (G2 C)^T
#pragma unroll
                    for (int tau = 0; tau < TPW; ++tau) {
                        const int ct = wv + NW * tau;
                        if (ct < nq) {
                            d4 d = dt[tau];
#pragma unroll
                            for (int u2 = 0; u2 < NU; ++u2) {
                                if (u2 < nur) {
#pragma unroll
                                    for (int v = 0; v < 4; ++v) {
                                        const int s = 4 * u2 + v;
                                        d = mma(cval(s, ct), -xv[gpos<RMAX>(li, 4 * s + lg)], d);
                                    }
                                }
                            }
                            dt[tau] = d;
                        }
                    }
                }
#pragma unroll
                for (int tau = 0; tau < TPW; ++tau) {
                    const int ct = wv + NW * tau;
                    if (ct < nq && !skip_r) {
                        const d4 d = dt[tau];
                        rsq += d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + d[3] * d[3];
#pragma unroll
                        for (int v = 0; v < 4; ++v) sacc_r = mma(d[v], d[v], sacc_r);
                    }
                }
            }
            rsq = sum_rows(rsq);
            if (lg == 0) {
                x1[K::X1_RR + 16 * wv + li] = rsq;
                x1[K::X1_GW + 16 * wv + li] = gwp;
                if (wv == 0) {
                    x1[K::X1_GG + li] = gsq;
                    x1[K::X1_YV + li] = yrow;
                }
            }
            __syncthreads();

            // ---- rank test of every row; nd = longest dependent prefix ----
            // every lane tests row i; the first failing row over lanes 0..15 ends the block
            const double eps = a.eps >= 0.0 ? a.eps : ((double)m * m * r + (double)m * r + (double)m) * 0x1p-52;
            int nd;
            uint32_t stop = 0u;
            double g2row;  // ||Gamma_i||^2 of block row i
            double r2row;  // ||R_i||^2: its rejection against the span of C
            bool badrow;   // block row i or its target is not finite
            // the records of ||R_i||^2 and (G w)_i are requested together before they
            // are summed (as for the certificate above)
            double rrec[NW], wrec[NW];
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                rrec[q] = x1[K::X1_RR + 16 * q + li];
                wrec[q] = x1[K::X1_GW + 16 * q + li];
            }
            const double g2 = x1[K::X1_GG + li], yj = x1[K::X1_YV + li];
            __builtin_amdgcn_sched_barrier(0);
            {
                double r2 = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) r2 += rrec[q];
                const bool bad = li < nblk && (!isfinite(g2) || !isfinite(yj));
                g2row = g2;
                r2row = r2;
                badrow = bad;
                const double nr = sqrt(r2);
                const bool indep = li < nblk && !((r2 == 0.0) || (nr < eps) || (nr < eps * sqrt(g2)));
                const uint64_t fail = __ballot(bad || indep) & 0xFFFFull;
                const uint64_t nonf = __ballot(bad) & 0xFFFFull;
                nd = fail ? (int)__builtin_ctzll(fail) : nblk;
                if (fail && ((nonf >> nd) & 1ull)) stop = FLAG_NONFINITE;
            }
            double gwi = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) gwi += wrec[q];
            const double dyi = yrow - gwi;
            if (nd == 0 && (stop || !ind_blocks)) {
                if (stop) {
                    flags |= stop;
                    break;
                }
                block_mode = false;
                ring_ok = false;
                continue;
            }
            // nd == 0: row i is independent and starts a block of independent rows
            const bool indblk = nd == 0;
            const int r0 = r, nst = min(nblk, rmax - r0);  // rows that fit below the rank capacity
            if (indblk && r0 == rmax) {
                flags |= FLAG_RANK_CAPACITY;
                break;
            }
            const bool rowok = li < nd;
            d4 z[UPW];
            d4 sacc = (d4){0.0, 0.0, 0.0, 0.0};
            if (indblk) {
                // independent rows: the Gram matrix R R^T of the rejections
                sacc = sacc_r;
            } else {
            // ---- Z = P^-1 G^T and this wave's part of S = I + G Z ----
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                const int u = wv + NW * ups;
                z[ups] = (d4){0.0, 0.0, 0.0, 0.0};
                if (u < nur) {
                    d4 z2 = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int u2 = 0; u2 < NU; ++u2) {
                        if (u2 < nur) {
#pragma unroll
                            for (int v = 0; v < 4; v += 2) {
                                const double gb0 = x2[gpos<RMAX>(li, 16 * u2 + 4 * v + lg)];
                                const double gb1 = x2[gpos<RMAX>(li, 16 * u2 + 4 * v + 4 + lg)];
                                z[ups] = mma(p[u2][ups][v], rowok ? gb0 : 0.0, z[ups]);
                                z2 = mma(p[u2][ups][v + 1], rowok ? gb1 : 0.0, z2);
                            }
                        }
                    }
                    z[ups] += z2;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double ga = rowok ? x2[gpos<RMAX>(li, 16 * u + 4 * v + lg)] : 0.0;
                        sacc = mma(ga, z[ups][v], sacc);
                    }
                }
            }
            }
            // four records of partial sums of S (or R R^T); with 8 waves the upper half folds in first
            if (NW == 8) {
                if (wv >= 4) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) x1[K::X1_SP + K::SPS * (wv - 4) + K::SPR * (4 * v + lg) + li] = sacc[v];
                }
                __syncthreads();
                if (wv < 4) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) sacc[v] += x1[K::X1_SP + K::SPS * wv + K::SPR * (4 * v + lg) + li];
                }
            }
            if (wv < 4) {
#pragma unroll
                for (int v = 0; v < 4; ++v) x1[K::X1_SP + K::SPS * wv + K::SPR * (4 * v + lg) + li] = sacc[v];
            }
            __syncthreads();

            // ---- Cholesky S = L L^T (lane i holds row i), c = L^-1 (y - G w) ----
            // Wave 0 factors S column by column, lane i holding row i (the four
            // DPP rows of the wave hold copies).  Row k of the trailing matrix is
            // broadcast from lane k of each row of 16 lanes (one 64-bit DPP move
            // per entry) and stands for column k, S being symmetric: each step is
            // an elimination step, row i -= (S[i][k] / S[k][k]) row k, which in
            // exact arithmetic is the outer-product update of the lower triangle;
            // every lane scales and updates its own row.  A pivot that is not
            // positive and finite ends the prefix of applied rows (ndd); what
            // follows it is computed but never used.
            // Z to LDS for the substitution (every read of G ended at the barrier
            // above), before the factorization, so that Z need not stay in registers
            if (!indblk) {
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) {
                    const int u = wv + NW * ups;
                    if (u < nur) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) x2[zpos(16 * u + 4 * v + lg, li)] = z[ups][v];
                    }
                }
            }
            if (wv == 0) {
                // row li of S: lane group lg reads row li of record lg (all loads in
                // flight together), and the four lane groups are summed
                double srow[16];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) srow[cc] = x1[K::X1_SP + K::SPS * lg + K::SPR * li + cc];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) srow[cc] = sum_rows(srow[cc]) + ((cc == li && !indblk) ? 1.0 : 0.0);
                double cy = rowok ? dyi : 0.0;
                double mypiv = 1.0, myc = 0.0, myinv = 0.0;
                static_for<16>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    double cv[16];  // row k: S[k][j] from lane k of the row of 16, j >= k
#pragma unroll
                    for (int j = k; j < 16; ++j) cv[j] = bcast16<k>(srow[j]);
                    const double cyk = bcast16<k>(cy);
                    const double piv = cv[k];
                    const double inv = rsqrt_f64(piv), lkk = piv * inv;
                    const double ck = cyk * inv;
                    const double lik = srow[k] * inv;  // L[i][k] for i > k
                    const double fik = lik * inv;      // S[i][k] / S[k][k]: one product per trailing entry
                    if (li == k) {
                        mypiv = piv;
                        myc = ck;
                        myinv = inv;
                    }
                    // Entries of the rows above k (lanes i < k) and their c are never
                    // read again: they are updated like the others instead of being
                    // masked, and only the lower triangle of L is used.
                    srow[k] = li == k ? lkk : lik;
                    cy -= lik * ck;
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) srow[j] -= fik * cv[j];
                });
                if (!indblk) {
                const uint64_t badp = __ballot(!(mypiv > 0.0 && isfinite(mypiv))) & 0xFFFFull;
                const int nbad = badp ? (int)__builtin_ctzll(badp) : 16;
                const int nk = nbad < nd ? nbad : nd;
                if (lg == 0) {
#pragma unroll
                    for (int k = 0; k < 16; ++k) x1[K::X1_L + 16 * li + k] = srow[k];
                    x1[K::X1_C + li] = li < nk ? myc : 0.0;
                    x1[K::X1_C + 16 + li] = li < nk ? myinv : 0.0;
                }
                if (li == 0 && lg == 0) x1[K::X1_COL] = (double)nk;
                } else {
                    // Pivot j of R R^T is the squared norm of row j's rejection against
                    // the span of C and of the block rows before it: the sequential rank
                    // test of Section 3 for every row at once.  ni = the longest prefix of
                    // finite rows that pass it and fit below the rank capacity.
                    const double epsl = a.eps >= 0.0 ? a.eps
                                                     : ((double)m * m * (r0 + li) + (double)m * (r0 + li) + (double)m) * 0x1p-52;
                    // A pivot below PIV_AMBIG of the row's squared rejection against C
                    // carries the rounding of that subtraction at a relative size that
                    // a small eps (FP64 streams) cannot resolve: the run ends before
                    // the row, which the next block tests with its explicit rejection
                    // against the grown C (its own pivot there is its diagonal).
                    const double nrm = sqrt(mypiv);
                    const bool ok = li < nst && !badrow && mypiv > 0.0 && isfinite(mypiv) && !(nrm < epsl) &&
                                    !(nrm < epsl * sqrt(g2row)) && mypiv >= PIV_AMBIG * r2row;
                    const uint64_t failm = __ballot(!ok) & 0xFFFFull;
                    const uint64_t badm = __ballot(li < nblk && badrow) & 0xFFFFull;
                    const int ni = failm ? (int)__builtin_ctzll(failm) : 16;
                    if (lg == 0) {
#pragma unroll
                        for (int k = 0; k < 16; ++k) x1[K::X1_L + 16 * li + k] = srow[k];
                        x1[K::X1_C + 16 + li] = myinv;
                    }
                    __builtin_amdgcn_wave_barrier();
                    // column i of W = L^-1 on the first ni rows (zero elsewhere)
                    double wc[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        double a0 = li == j ? 1.0 : 0.0, a1 = 0.0;
                        const double2 *lrow = reinterpret_cast<const double2 *>(x1 + K::X1_L + 16 * j);
#pragma unroll
                        for (int j2 = 0; j2 < j; j2 += 2) {
                            const double2 l2 = lrow[j2 / 2];
                            a0 -= wc[j2] * l2.x;
                            if (j2 + 1 < j) a1 -= wc[j2 + 1] * l2.y;
                        }
                        wc[j] = j < ni ? (a0 + a1) * x1[K::X1_C + 16 + j] : 0.0;
                    }
                    // W row-major: W[j][i] at X1_W + 16 j + i (the records are read by now)
                    if (lg == 0) {
#pragma unroll
                        for (int j = 0; j < 16; ++j) x1[K::X1_W + 16 * j + li] = wc[j];
                    }
                    if (li == 0 && lg == 0) {
                        x1[K::X1_COL] = (double)ni;
                        x1[K::X1_COL + 1] = ((badm >> ni) & 1ull) ? 1.0 : 0.0;
                    }
                }
            }
            __syncthreads();
            if (indblk) {
                // ---- independent rows 0 .. ni-1 of the block: H^-1 += U U^T with
                //      U = [G^T W^T; -W^T], appends to C, P^-1 and w ----
                const int ni = __builtin_amdgcn_readfirstlane((int)x1[K::X1_COL]);
                const bool nonf = x1[K::X1_COL + 1] != 0.0;
                if (ni == 0) {
                    // the first row failed the pivot test although its rejection passed
                    // the row test (the two sums round differently): take it alone
                    block_mode = false;
                    ring_ok = false;
                    continue;
                }
                const int nurn = (r0 + ni + 15) / 16;
                // Q = G^T W^T on this wave's row tiles: A = G^T[16u + i][4ks + g],
                // B = W^T[4ks + g][i] = W[i][4ks + g]
                d4 q[UPW];
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) {
                    const int u = wv + NW * ups;
                    q[ups] = (d4){0.0, 0.0, 0.0, 0.0};
                    if (u < nurn) {
#pragma unroll
                        for (int ks = 0; ks < 4; ++ks) {
                            const int j = 4 * ks + lg;
                            const double ga = j < ni ? x2[gpos<RMAX>(j, 16 * u + li)] : 0.0;
                            q[ups] = mma(ga, x1[K::X1_W + 16 * li + j], q[ups]);
                        }
                    }
                }
                __syncthreads();  // every read of G is done
                // U to X2: rows kk < r0 are Q, rows r0 .. r0 + ni - 1 are -W^T
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) {
                    const int u = wv + NW * ups;
                    if (u < nurn) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int kk = 16 * u + 4 * v + lg;
                            const double val = kk < r0 ? q[ups][v]
                                                       : (kk < r0 + ni ? -x1[K::X1_W + 16 * li + (kk - r0)] : 0.0);
                            x2[zpos(kk, li)] = val;
                        }
                    }
                }
                // rows r0 .. r0 + ni - 1 of C: the raw block rows
                for (int idx = t; idx < ni * CH; idx += K::NT) {
                    const int j = idx / CH, cc = idx - j * CH, k = r0 + j;
                    const E *src = G0 + (i - i0 + j) * (int64_t)m;
                    E v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        // unconditional loads (column 0 past m), all in flight together
                        int col = 4 * cc + e < m ? 4 * cc + e : 0;
                        asm("" : "+v"(col));
                        const E x = src[col];
                        v[e] = 4 * cc + e < m ? x : 0.0f;
                    }
                    *reinterpret_cast<V4 *>(sct + (size_t)k * MMAX + 4 * (cc ^ (k & 15))) =
                        mk4<E>(v[0], v[1], v[2], v[3]);
                }
                __syncthreads();
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) {
                    const int u = wv + NW * ups;
                    if (u < nurn) {
                        double bt[4];
#pragma unroll
                        for (int ks = 0; ks < 4; ++ks) bt[ks] = x2[zpos(16 * u + li, 4 * ks + lg)];
                        if constexpr (K::HG) {
                            // four tiles' loads in flight at a time
#pragma unroll 1
                            for (int ub = 0; ub < nurn; ub += 4) {
                                d4 acc[4];
#pragma unroll
                                for (int q = 0; q < 4; ++q) acc[q] = hload(ub + q, ups, r0);
#pragma unroll
                                for (int q = 0; q < 4; ++q)
                                    if (ub + q < nurn) {
#pragma unroll
                                        for (int ks = 0; ks < 4; ++ks)
                                            acc[q] = mma(x2[zpos(16 * (ub + q) + li, 4 * ks + lg)], bt[ks], acc[q]);
                                        hstore(ub + q, ups, acc[q], r0 + ni);
                                    }
                            }
                        } else {
#pragma unroll
                            for (int u2 = 0; u2 < NU; ++u2) {
                                if (u2 < nurn) {
                                    d4 acc = hload(u2, ups, r0);
#pragma unroll
                                    for (int ks = 0; ks < 4; ++ks) acc = mma(x2[zpos(16 * u2 + li, 4 * ks + lg)], bt[ks], acc);
                                    hstore(u2, ups, acc, r0 + ni);
                                }
                            }
                        }
                    }
                }
                // appends: P^-1 = 1 on the new diagonal, w = y (Theorem 4 in coordinates)
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) {
                    const int u = wv + NW * ups;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int kk = 16 * u + 4 * v + lg;
                        if (kk >= r0 && kk < r0 + ni) wr[ups][v] = x1[K::X1_YV + (kk - r0)];  // y of block row kk - r0
#pragma unroll
                        for (int u2 = 0; u2 < NU; ++u2) {
                            const int row = 16 * u2 + 4 * v + lg, colp = 16 * u + li;
                            if (row == colp && row >= r0 && row < r0 + ni) p[u2][ups][v] = 1.0;
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) trh += j < ni ? x1[K::X1_GG + j] : 0.0;
                r = r0 + ni;
                i += ni;
                applied += ni;
                if (nonf && ni < nblk) {
                    flags |= FLAG_NONFINITE;
                    break;
                }
                continue;
            }
            const int ndd = __builtin_amdgcn_readfirstlane((int)x1[K::X1_COL]);

            // ---- T = Z L^-T (row kk per thread, in place) and dw = T c ----
            if (tl < 16 * nur) {
                // T[kk][j] = (Z[kk][j] - sum_{j2 < j} T[kk][j2] L[j][j2]) / L[j][j]; columns
                // from ndd on are zero (a failed pivot leaves non-finite values there)
                double tr[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) tr[j] = x2[zpos(tl, j)];
                double dw = 0.0;
                // the entries of row j + 1 of L (with its 1/L[j+1][j+1] and c) are
                // requested before row j is used, so that each step's LDS reads are
                // in flight during the step before it
                double2 ln[8];
                double invn = x1[K::X1_C + 16], cn = x1[K::X1_C];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    double2 lc[8];
#pragma unroll
                    for (int e = 0; e < (j + 1) / 2; ++e) lc[e] = ln[e];
                    const double invj = invn, cj = cn;
                    if (j + 1 < 16) {
                        const double2 *lrow = reinterpret_cast<const double2 *>(x1 + K::X1_L + 16 * (j + 1));
#pragma unroll
                        for (int e = 0; e < (j + 2) / 2; ++e) ln[e] = lrow[e];
                        invn = x1[K::X1_C + 16 + j + 1];
                        cn = x1[K::X1_C + j + 1];
                    }
                    double a0 = tr[j], a1 = 0.0;
#pragma unroll
                    for (int j2 = 0; j2 < j; j2 += 2) {
                        const double2 l2 = lc[j2 / 2];
                        a0 -= tr[j2] * l2.x;
                        if (j2 + 1 < j) a1 -= tr[j2 + 1] * l2.y;
                    }
                    tr[j] = j < ndd ? (a0 + a1) * invj : 0.0;
                    dw += tr[j] * cj;
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) x2[zpos(tl, j)] = tr[j];
                x1[K::X1_DW + tl] = dw;
            }
            __syncthreads();

            // ---- w += T c, P^-1 -= T T^T ----
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                const int u = wv + NW * ups;
                if (u < nur) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) wr[ups][v] += x1[K::X1_DW + 16 * u + 4 * v + lg];
                    double bt[4];
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) bt[ks] = x2[zpos(16 * u + li, 4 * ks + lg)];
#pragma unroll
                    for (int u2 = 0; u2 < NU; ++u2) {
                        if (u2 < nur) {
                            d4 acc = p[u2][ups];
#pragma unroll
                            for (int ks = 0; ks < 4; ++ks) acc = mma(-x2[zpos(16 * u2 + li, 4 * ks + lg)], bt[ks], acc);
                            p[u2][ups] = acc;
                        }
                    }
                }
            }
            i += ndd;
            applied += ndd;
            if (ndd < nd) {
                flags |= FLAG_DENOMINATOR;
                break;
            }
            if (nd < nblk) {
                if (stop) {
                    flags |= stop;
                    break;
                }
                block_mode = false;
                ring_ok = false;
            }
            continue;
        }

        // ================= one row (Algorithm 1) =================
        E *sg_ring = ring;
        if (!ring_ok) {
            __syncthreads();  // X2 may still be read by a block step
            const E *Gi = G0 + (i - i0) * (int64_t)m;
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int j = tl + K::NT * e;
                if (j < MMAX) sg_ring[cur * MMAX + j] = j < m ? Gi[j] : 0.0f;
            }
            const E *Gn = Gi + m;
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int j = tl + K::NT * e;
                pre[e] = (i + 1 < i1 && j < m) ? Gn[j] : 0.0f;
            }
            y_next = a.y[i];
            ring_ok = true;
            __syncthreads();
        }
        // Row i is in slot cur; row i+1 (in pre) goes to slot nxt, which row
        // i-2 read two barriers ago; row i+2 is requested now.
        const int nxt = cur == 2 ? 0 : cur + 1;
        if (i + 1 < i1) {
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int j = tl + K::NT * e;
                if (j < MMAX) sg_ring[nxt * MMAX + j] = pre[e];
            }
        }
        if (i + 2 < i1) {
            const E *Gn = G0 + (i + 2 - i0) * (int64_t)m;
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int j = tl + K::NT * e;
                pre[e] = j < m ? Gn[j] : 0.0f;
            }
        }
        const double yv = (double)y_next;
        if (i + 1 < i1) y_next = a.y[i + 1];
        const E *gcur = sg_ring + cur * MMAX;
        double *sgam = x1 + K::X1_GAM, *szeta = x1 + K::X1_ZETA, *sv = x1 + K::X1_V;
        double *sred = x1 + K::X1_RED, *sgr = x1 + K::X1_GR;

        // ---- A: v = C Gamma (rows k = pk + RS b, 16-lane sums) ----
        double gam[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) gam[b] = 0.0;
#pragma unroll 1
        for (int c4 = 0; c4 < cba4; ++c4) {
            const int ph = 16 * c4 + pj, lc = ph ^ pk15;  // physical chunk of C rows k (k & 15 == pk & 15), logical chunk
            const V4 gv = *reinterpret_cast<const V4 *>(gcur + 4 * lc);
            const double g0 = gv.x, g1 = gv.y, g2v = gv.z, g3 = gv.w;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int k = pk + RS * b;
                V4 v = *reinterpret_cast<const V4 *>(sct + (size_t)min(k, ra - 1) * MMAX + 4 * ph);
                if (k >= ra) v = mk4<E>(0, 0, 0, 0);
                gam[b] += (double)v.x * g0;
                gam[b] += (double)v.y * g1;
                gam[b] += (double)v.z * g2v;
                gam[b] += (double)v.w * g3;
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            gam[b] = sum16(gam[b]);
            if (pj == 0) sv[pk + RS * b] = gam[b];
        }
        __syncthreads();

        // ---- A2: gamma = H^-1 v per column tile, one reduce-scatter ----
        const int nur = (r + 15) / 16;
        {
            double hacc[2] = {0.0, 0.0};
            if constexpr (K::HG) {
#pragma unroll 1
                for (int u2 = 0; u2 < nur; ++u2) {
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) {
                        const d4 ht = hload(u2, ups, r);
#pragma unroll
                        for (int v = 0; v < 4; ++v) hacc[ups] += ht[v] * sv[16 * u2 + 4 * v + lg];
                    }
                }
            } else {
#pragma unroll
            for (int u2 = 0; u2 < NU; ++u2) {
                if (u2 < nur) {
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) {
                        const d4 ht = hload(u2, ups, r);
#pragma unroll
                        for (int v = 0; v < 4; ++v) hacc[ups] += ht[v] * sv[16 * u2 + 4 * v + lg];
                    }
                }
            }
            }
            const double tg = scatter4(hacc[0], hacc[1], 0.0, 0.0);  // gamma[16 (w + NW g) + i] on lane group g < UPW
            if (lg < UPW) sgam[16 * (wv + NW * lg) + li] = tg;
        }
        __syncthreads();

        // ---- B: C^T gamma, zeta = P^-1 gamma, gamma^T w per column tile ----
        double acc[4] = {0.0, 0.0, 0.0, 0.0}, zacc[2] = {0.0, 0.0};
#pragma unroll
        for (int u2 = 0; u2 < NU; ++u2) {
            if (u2 < nur) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int s = 4 * u2 + v;
                    const double gs = sgam[4 * s + lg];
#pragma unroll
                    for (int tau = 0; tau < TPW; ++tau) acc[tau] += cval(s, wv + NW * tau) * gs;
#pragma unroll
                    for (int ups = 0; ups < UPW; ++ups) zacc[ups] += p[u2][ups][v] * gs;
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // one row tile at a time: bounds the live conversions
        }
        double dyp = 0.0;
#pragma unroll
        for (int ups = 0; ups < UPW; ++ups)
#pragma unroll
            for (int v = 0; v < 4; ++v) dyp += wr[ups][v] * sgam[16 * (wv + NW * ups) + 4 * v + lg];
        const double tcol = scatter4(acc[0], acc[1], acc[2], acc[3]);  // (C^T gamma) of column 16 (w + 4 g) + i
        const double tz = scatter4(zacc[0], zacc[1], dyp, 0.0);        // zeta (g < UPW) or gamma^T w (g == 2)
        double sp = 0.0, dp = 0.0, gw = 0.0, g2 = 0.0;
        if (lg < TPW && wv + NW * lg < NTT) {
            const int col = 16 * (wv + NW * lg) + li;
            const double gc = (double)gcur[col];
            const double v = gc - tcol;
            sgr[col] = v;
            sp = v * v;
            g2 = gc * gc;
        }
        if (lg < UPW) {
            const int kk = 16 * (wv + NW * lg) + li;
            szeta[kk] = tz;
            dp = tz * sgam[kk];
        }
        if (lg == 2 && li == 0) gw = tz;
        block_sum4<NW>(sp, dp, gw, g2, sred);
        if (!isfinite(g2) || !isfinite(yv)) {
            flags |= FLAG_NONFINITE;
            break;
        }
        const double eps = a.eps >= 0.0 ? a.eps : ((double)m * m * r + (double)m * r + (double)m) * 0x1p-52;
        const double nr = sqrt(sp), ng = sqrt(g2);
        const bool dependent = (sp == 0.0) || (nr < eps) || (nr < eps * ng);

        if (dependent) {
            if (r > 0) {
                const double d = 1.0 + dp;
                if (!(d > 0.0) || !isfinite(d)) {
                    flags |= FLAG_DENOMINATOR;
                    break;
                }
                const double inv_d = 1.0 / d;
                const double f = (yv - gw) * inv_d;
#pragma unroll
                for (int ups = 0; ups < UPW; ++ups) {
                    const double zc = szeta[16 * (wv + NW * ups) + li] * inv_d;
#pragma unroll
                    for (int u2 = 0; u2 < NU; ++u2) {
                        if (u2 < nur) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) p[u2][ups][v] -= szeta[16 * u2 + 4 * v + lg] * zc;
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) wr[ups][v] += szeta[16 * (wv + NW * ups) + 4 * v + lg] * f;
                }
            }
            block_mode = use_blocks;
        } else {
            if (r == rmax) {
                flags |= FLAG_RANK_CAPACITY;
                break;
            }
            // H^-1 <- [[H^-1 + gamma gamma^T / s, -gamma / s], [-gamma^T / s, 1 / s]]
            const double inv_s = 1.0 / sp;
            // tile (u2, u) of the bordered H^-1
            auto border = [&](int u2, int ups) {
                const int colh = 16 * (wv + NW * ups) + li;
                const double gcol = colh < r ? sgam[colh] : 0.0;
                d4 ht = hload(u2, ups, r);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * u2 + 4 * v + lg;
                    const double grow = row < r ? sgam[row] : 0.0;
                    if (row < r && colh < r) ht[v] += (grow * gcol) * inv_s;
                    else if (row < r && colh == r) ht[v] = -grow * inv_s;
                    else if (row == r && colh < r) ht[v] = -gcol * inv_s;
                    else if (row == r && colh == r) ht[v] = inv_s;
                }
                hstore(u2, ups, ht, r + 1);
            };
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                if constexpr (K::HG) {
#pragma unroll 1
                    for (int u2 = 0; 16 * u2 <= r; ++u2) border(u2, ups);
                } else {
#pragma unroll
                    for (int u2 = 0; u2 < NU; ++u2)
                        if (16 * u2 <= r) border(u2, ups);
                }
            }
            // append: row r of C (the raw row), P^-1[r][r] = 1, w[r] = y
            if (tl < CH) {
                const V4 gv = *reinterpret_cast<const V4 *>(gcur + 4 * tl);
                *reinterpret_cast<V4 *>(sct + (size_t)r * MMAX + 4 * (tl ^ (r & 15))) = gv;
            }
#pragma unroll
            for (int ups = 0; ups < UPW; ++ups) {
                const int u = wv + NW * ups;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (16 * u + 4 * v + lg == r) {
                        wr[ups][v] = yv;
#pragma unroll
                        for (int u2 = 0; u2 < NU; ++u2)
                            if (u2 == u && li == (r & 15)) p[u2][ups][v] = 1.0;
                    }
                }
            }
            r += 1;
            trh += g2;
            block_mode = ind_blocks;
            __syncthreads();
        }
        ++i;
        ++applied;
        cur = nxt;
    }

    // ---- write the state back ------------------------------------------------
    // The stores use freshly derived addresses (opaque copies of the strides and
    // the lane id), so the compiler does not keep the load-time addresses of all
    // register-resident state live across the row loop.
    __syncthreads();
    int ldm_w = ldm, rmax_w = rmax, lane_w = lane;
    asm volatile("" : "+s"(ldm_w), "+s"(rmax_w), "+v"(lane_w));
    const int li_w = lane_w & 15, lg_w = lane_w >> 4;
    for (int idx = t; idx < ra * CH; idx += K::NT) {
        const int k = idx / CH, cc = idx - k * CH;
        if (k < r) {
            const V4 v = *reinterpret_cast<const V4 *>(sct + (size_t)k * MMAX + 4 * (cc ^ (k & 15)));
            const E vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * cc + e < m) Cg[(size_t)k * ldm_w + 4 * cc + e] = vv[e];
        }
    }
#pragma unroll
    for (int ups = 0; ups < UPW; ++ups) {
        const int col = 16 * (wv + NW * ups) + li_w;
#pragma unroll
        for (int u2 = 0; u2 < NU; ++u2)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * u2 + 4 * v + lg_w;
                if (row < r && col < r) {
                    Pg[(size_t)row * rmax_w + col] = p[u2][ups][v];
                    if constexpr (!K::HG) Hg[(size_t)row * rmax_w + col] = h[u2][ups][v];
                }
            }
        if (li_w == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kk = 16 * (wv + NW * ups) + 4 * v + lg_w;
                if (kk < r) wg[kk] = wr[ups][v];
            }
        }
    }
    if (t == 0) {
        M->r = r;
        M->flags = flags;
        M->rows_seen += applied;
    }
    __syncthreads();
}

// Grid of one workgroup per stream (a.persistent == 0), or a persistent grid
// whose workgroups take streams from the family's queue head, in the order of
// a.order (longest expected cost first), until the queue is empty.  The queue
// head is read by thread 0 and handed to the workgroup through LDS; the
// barrier after the last stream's stores keeps that read and the previous
// stream's thread-0 stores in separate barrier intervals.
template <class K>
__global__ void __launch_bounds__(K::NT, K::OCC) k_push_mf(PushArgs<typename K::E> a, int ra) {
    extern __shared__ double smem[];
    if (!a.persistent) {
        push_stream<K>(a, ra, a.order[blockIdx.x], smem);
        return;
    }
    int *slot = reinterpret_cast<int *>(smem + (size_t)ra * K::MMAX * K::EW / 2);  // first word of X1
    for (;;) {
        if (threadIdx.x == 0) *slot = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int q = *slot;
        __syncthreads();
        if (q >= a.n_order) break;
        push_stream<K>(a, ra, a.order[q], smem);
    }
}

template <class K>
size_t lds_bytes(int ra) {
    return sizeof(typename K::E) * (size_t)ra * K::MMAX + sizeof(double) * (size_t)(K::X1_D + K::X2_D + K::X3_D);
}

// Rows of Ct reserved in LDS: r_max rounded up to whole 16-row tiles.
inline int rows16(int r_max) { return (r_max + 15) / 16 * 16; }

using F0 = MF<64, 128, 4>;
using F1 = MF<128, 128, 8>;
using F2 = MF<64, 192, 4>;
using F3 = MF<128, 192, 8>;
using F4 = MF<64, 256, 4>;
using F5 = MF<128, 256, 8>;
// FP64 streams: C and the rows in FP64 (the variant of FP64 single streams such
// as m = 64, r = 16 and of small FP64 batches)
using D0 = MF<64, 128, 4, double>;

template <class K>
bool fits_k(int m, int r_max) {
    return m <= K::MMAX && r_max <= K::RMAX && lds_bytes<K>(rows16(r_max)) <= 160 * 1024;
}
// Set once per variant, to the LDS the variant needs at its full rank
// capacity (the limit is process-wide: a later handle must not lower it under
// the launches of a live one).
// Workgroups of variant K resident on the chip at once for a given LDS need
// (the persistent grid), looked up when a handle is set up, never during a
// push, so that a push can be captured into a graph.
template <class K>
struct Resident {
    static int per_ra[K::RMAX / 16 + 1];  // by rows16(r_max) / 16; 0 = not looked up
    static int cus;
};
template <class K>
int Resident<K>::per_ra[K::RMAX / 16 + 1] = {};
template <class K>
int Resident<K>::cus = 0;

template <class K>
hipError_t prepare_k(int r_max) {
    const int ra = rows16(r_max);
    if (lds_bytes<K>(ra) > 160 * 1024) return hipErrorInvalidValue;
    static_assert(sizeof(typename K::E) * K::RMAX * K::MMAX + sizeof(double) * (K::X1_D + K::X2_D + K::X3_D) <= 160 * 1024,
                  "every variant fits the LDS at its full capacity");
    static const hipError_t once = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_push_mf<K>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)lds_bytes<K>(K::RMAX));
    if (once != hipSuccess) return once;
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_push_mf<K>, K::NT, lds_bytes<K>(ra));
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    Resident<K>::per_ra[ra / 16] = per_cu > 0 ? per_cu : 1;
    Resident<K>::cus = cus;
    return hipSuccess;
}
template <class K>
hipError_t launch_k(const PushArgs<typename K::E> &a, int r_max, hipStream_t s) {
    const int ra = rows16(r_max);
    const size_t lds = lds_bytes<K>(ra);
    if (lds > 160 * 1024 || ra > K::RMAX) return hipErrorInvalidValue;
    int grid = a.n_order;
    if (a.persistent) {
        // as many workgroups as fit on the chip at once, each taking streams from the queue
        const int per_cu = Resident<K>::per_ra[ra / 16];
        if (per_cu <= 0 || Resident<K>::cus <= 0) return hipErrorNotInitialized;
        grid = std::max(1, std::min(a.n_order, per_cu * Resident<K>::cus));
    }
    hipLaunchKernelGGL(k_push_mf<K>, dim3(grid), dim3(K::NT), lds, s, a, ra);
    return hipGetLastError();
}

}  // namespace

int mf_choose(int m, int r_max) {
    if (fits_k<F0>(m, r_max)) return 0;
    if (fits_k<F1>(m, r_max)) return 1;
    if (fits_k<F2>(m, r_max)) return 2;
    if (fits_k<F3>(m, r_max)) return 3;
    if (fits_k<F4>(m, r_max)) return 4;
    if (fits_k<F5>(m, r_max)) return 5;
    return -1;
}

bool mf_fits(int v, int m, int r_max) {
    switch (v) {
        case 0: return fits_k<F0>(m, r_max);
        case 1: return fits_k<F1>(m, r_max);
        case 2: return fits_k<F2>(m, r_max);
        case 3: return fits_k<F3>(m, r_max);
        case 4: return fits_k<F4>(m, r_max);
        case 5: return fits_k<F5>(m, r_max);
    }
    return false;
}

int mf_mmax(int v) {
    switch (v) {
        case 0: return F0::MMAX;
        case 1: return F1::MMAX;
        case 2: return F2::MMAX;
        case 3: return F3::MMAX;
        case 4: return F4::MMAX;
        case 5: return F5::MMAX;
    }
    return 0;
}

int mf_threads(int v) {
    switch (v) {
        case 0: return F0::NT;
        case 1: return F1::NT;
        case 2: return F2::NT;
        case 3: return F3::NT;
        case 4: return F4::NT;
        case 5: return F5::NT;
    }
    return 0;
}

int mf_rmax(int v) {
    switch (v) {
        case 0: return F0::RMAX;
        case 1: return F1::RMAX;
        case 2: return F2::RMAX;
        case 3: return F3::RMAX;
        case 4: return F4::RMAX;
        case 5: return F5::RMAX;
    }
    return 0;
}

hipError_t mf_prepare(int v, int r_max) {
    switch (v) {
        case 0: return prepare_k<F0>(r_max);
        case 1: return prepare_k<F1>(r_max);
        case 2: return prepare_k<F2>(r_max);
        case 3: return prepare_k<F3>(r_max);
        case 4: return prepare_k<F4>(r_max);
        case 5: return prepare_k<F5>(r_max);
    }
    return hipErrorInvalidValue;
}

bool mf64_fits(int m, int r_max) { return fits_k<D0>(m, r_max); }
int mf64_rmax() { return D0::RMAX; }
int mf64_mmax() { return D0::MMAX; }
int mf64_threads() { return D0::NT; }
hipError_t mf64_prepare(int r_max) { return prepare_k<D0>(r_max); }
hipError_t mf64_launch(const PushArgs<double> &a, int r_max, hipStream_t s) { return launch_k<D0>(a, r_max, s); }

hipError_t mf_launch(int v, const PushArgs<float> &a, int r_max, hipStream_t s) {
    switch (v) {
        case 0: return launch_k<F0>(a, r_max, s);
        case 1: return launch_k<F1>(a, r_max, s);
        case 2: return launch_k<F2>(a, r_max, s);
        case 3: return launch_k<F3>(a, r_max, s);
        case 4: return launch_k<F4>(a, r_max, s);
        case 5: return launch_k<F5>(a, r_max, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace rg
