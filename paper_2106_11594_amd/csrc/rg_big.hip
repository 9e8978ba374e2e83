// The stream of a single-stream handle that no on-chip class holds (FP64
// streams, and FP32 streams beyond the classes' m and r_max), spread over
// the whole GPU in blocks of up to 16 rows.
//
// The state is the factored form of the blocked on-chip kernels: C (the
// accepted raw rows, r x m), H^-1 = (C C^T)^-1 and P^-1 (FP64, r_max x r_max
// row-major) and the coordinates w (FP64), with x = C^T H^-1 w and the dual
// basis Ct = H^-1 C of Section 2.1 never formed.
//
// A block of k rows Gamma_blk (rows of any mix of kinds) is taken in one pass
// of five grid-wide kernels on the handle's stream, with every intermediate
// in a device scratch area, so the host never waits on the device:
//   v       V = Gamma_blk C^T                        16 rows of C per tile;
//           one workgroup also takes ||Gamma_j||^2, finiteness and y_j
//   g       G = V H^-1 (the projections gamma_j of every row at once) and
//           the partial sums of G w                   16 columns per tile
//   rz      R = Gamma_blk - G C, the rejections, with the partial Gram
//           matrices R R^T over 64-column slices; Z = P^-1 G^T and the
//           partial sums of G Z                        per 16 rows of Z
//   decide  one workgroup: the rows in order, as Algorithm 1 takes them
//   apply   the rank-k updates of P^-1, H^-1 and w, and the appended rows
//
// The rows of a block are decided in order, each against the state that the
// rows before it leave (Section 3's rank test, Theorems 4-6).  Let I be the
// block rows appended to the basis so far and L_I the Cholesky factor of
// R_I R_I^T.  Row l's rejection against C and the rows of I is the pivot
// R R^T[l][l] - ||L_I^-1 R_I R_l^T||^2, so the rank test of every row follows
// from the Gram matrix of the block's rejections against C.  A dependent row
// l has, in the basis [C; Gamma_I], the coordinates
//   gamma^_l = [gamma_l - c_l^T G_I; c_l],  c_l = L_I^-T L_I^-1 R_I R_l^T,
// and the block's dependent rows D update P and w as a Woodbury block:
// with Gamma^ the |D| coordinate rows, Pd^-1 = diag(P^-1, I_|I|) and
// S = I + Gamma^ Pd^-1 Gamma^^T = L_S L_S^T (whose pivots are the sequential
// Greville denominators 1 + gamma^^T P^-1 gamma^, in row order),
//   P^-1 <- Pd^-1 - T T^T,   w <- [w; y_I] + T L_S^-1 (y_D - Gamma^ [w; y_I]),
//   T = Pd^-1 Gamma^^T L_S^-T.
// The appended rows border H^-1 with their Schur complement R_I R_I^T:
//   H^-1 <- [[H^-1, 0], [0, 0]] + U U^T,  U = [G_I^T W^T; -W^T],  W = L_I^-1.
// Applying the rows one after another gives the same P^-1, H^-1 and w up to
// rounding.  A Gram pivot loses about half its digits when row l is nearly in
// the span of earlier rows of the same block; when a pivot falls below 1e-4
// of the row's own squared rejection against C, and the row would be
// independent but for the block rows, the block is redone with explicit
// rejections (classical Gram-Schmidt, twice) over the stored R, so that the
// rank test sees the rejection norm the row-by-row algorithm computes.
//
// The rank at the start of a block and whether the stream is still active are
// double-buffered by block parity: the kernels of block b read slot b & 1 and
// the decision writes slot (b + 1) & 1, so no kernel reads a value that
// another kernel of the same block may still change.  Partial sums are
// reduced in a fixed order: results do not depend on scheduling.
#include "rg_internal.h"
#include "rg_lanes.h"

#include <algorithm>

namespace rg {
namespace {

constexpr int BT = 256;        // threads per workgroup
constexpr int NWV = BT / 64;   // waves per workgroup
constexpr int KB = 16;         // rows per block
constexpr int SL = 64;         // columns per rejection slice
constexpr int PT = 32;         // apply tile (PT x PT elements of P^-1 and H^-1)
constexpr double TAU = 1e-4;   // Gram pivots below TAU of the row's squared rejection are recomputed

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// p[i] as a double if ok, else 0.  The load itself is unconditional, from
// p[0] when !ok (every caller's p[0] is valid): a load under a condition
// becomes a branch that waits for it, and a run of them waits one by one.
// The empty asm hides the clamped index from the optimiser, which would
// otherwise fold the clamp and the select back into a conditional load.
template <typename P>
__device__ inline double ld_or0(const P *p, int64_t i, bool ok) {
    int64_t k = ok ? i : 0;
    __asm__("" : "+v"(k));
    const double v = (double)p[k];
    return ok ? v : 0.0;
}

// p[0..3] as doubles with 16-byte loads (p 16-byte aligned).
__device__ inline void ld4(const float *p, double *v) {
    const float4 f = *reinterpret_cast<const float4 *>(p);
    v[0] = f.x;
    v[1] = f.y;
    v[2] = f.z;
    v[3] = f.w;
}
__device__ inline void ld4(const double *p, double *v) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 c = *reinterpret_cast<const double2 *>(p + 2);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = c.x;
    v[3] = c.y;
}

// Device control record at the start of the scratch area.
struct BigCtl {
    int32_t rank[2];    // rank at the start of a block, by block parity
    int32_t active[2];  // stream not flagged at the start of a block, by parity
    int64_t applied;    // rows applied in this push
    int32_t ni, nd;     // rows of the block appended / taken as dependent
    int32_t napp;       // rows of the block applied (the rest follow a flagged row)
    int32_t pad;
    int32_t piv[KB];    // block rows appended, in order
    int32_t bad[KB];    // block row j or its target is not finite
    double g2[KB];      // ||Gamma_j||^2
    double y[KB];       // y_j
};
constexpr size_t CTL_DOUBLES = 128;
static_assert(sizeof(BigCtl) <= CTL_DOUBLES * sizeof(double), "control record");

// The k x k results of the decision (row-major KB x KB, zero outside their
// ranges): P^-1 top-left update Z AP Z^T, cross block -Z BP, bottom block BRP;
// H^-1 top-left update G^T AH G, cross block -G^T BH, bottom block BRH; the
// top of w moves by Z qc, its appended entries are wbot.
constexpr int SM_AP = 0, SM_BP = 256, SM_BRP = 512, SM_AH = 768, SM_BH = 1024, SM_BRH = 1280, SM_QC = 1536,
              SM_WB = 1552, SM_SIZE = 1568;

template <typename T>
struct BigArgs {
    StreamMeta *meta;
    BigCtl *ctl;
    T *C;               // r_max x ldm
    double *P, *H, *w;  // r_max x r_max (stride r_max), r_max
    const T *gam;       // first row of this push (row-major n x m)
    const T *y;         // first target of this push
    int64_t n;          // rows in this push
    int m, rmax, ldm, kb, ns;
    int gvec;           // rows of gam are 16-byte aligned (vector loads)
    double eps;         // < 0: default of Section 3 at the current rank
    double *V, *G, *Z, *gwp, *gzp, *R, *rrp, *Q, *sm;
};

// ---------------------------------------------------------------------------
// The three product kernels run 8-wave workgroups (BW threads) that split
// the inner dimension of a 16 x 16 output tile over their waves and sum the
// wave results in LDS in a fixed order.  Each wave issues UB iterations'
// loads before their matrix-core products: these kernels are bound by load
// latency, not by bandwidth or arithmetic.
constexpr int BW = 512;
constexpr int NWB = BW / 64;
constexpr int UB = 8;
// V = Gamma_blk C^T of FP64 streams: each 16-column tile of V is split over
// vsplit workgroups along the columns of C (a stream of a few hundred rows
// then occupies four times as many CUs); k_bb_g adds the partial tiles in
// split order.  FP32 streams keep one workgroup per tile (splitting them
// gained nothing for m = 2048 and lost 2 % for m = 1024).  The scratch holds
// VS_MAX partial tiles either way.
constexpr int VS_MAX = 4;
template <typename T>
constexpr int vsplit() { return sizeof(T) == 8 ? 4 : 1; }
static_assert(NWB % 4 == 0, "four column tiles per slice");

// Sum of the waves' 16 x 16 tiles (d4 per lane) into wave 0 (fixed order).
__device__ inline d4 waves_sum(d4 d, d4 (*red)[64], int nw) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    red[wid][lane] = d;
    __syncthreads();
    d4 acc = red[0][lane];
    if (wid == 0)
        for (int q = 1; q < nw; ++q) acc += red[q][lane];
    return acc;
}

// The V tiles of k_bb_v.  Each lane reads 4 consecutive columns of its row
// with 16-byte loads in groups of 16 columns.  Rows of C are padded to ldm (a
// multiple of 16 bytes), so a load at a column below ldm stays in the state;
// the block rows take 16-byte loads when they are 16-byte aligned with m a
// multiple of 4 elements (GV), else element loads.  Columns past the end load
// from column 0 and are masked: no load sits under a branch.
template <typename T, bool GV>
__device__ void v_tiles(const BigArgs<T> &b, int r0, int nb, const T *gb, int ntw, d4 (*red)[64]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    constexpr int UV = sizeof(T) == 4 ? 8 : 4;  // groups per wave and batch
    const int ngrp = (b.m + 15) / 16;
    const bool grow = li < nb;
    const T *grw = gb + (int64_t)(grow ? li : 0) * b.m;
    constexpr int VS = vsplit<T>();
    const int ntiles = (r0 + 15) / 16;
    for (int item = blockIdx.x; item < ntiles * VS; item += ntw) {
        const int t = item / VS, sp = item - t * VS;  // tile, split of the columns
        const int g0 = sp * ngrp / VS, g1 = (sp + 1) * ngrp / VS;
        const int nit = (g1 - g0 - wid + NWB - 1) / NWB;
        const int a0 = 16 * t;
        const bool crok = a0 + li < r0;
        const T *crow = b.C + (size_t)(crok ? a0 + li : 0) * b.ldm;
        d4 d = {0.0, 0.0, 0.0, 0.0};
        for (int it0 = 0; it0 < nit; it0 += UV) {
            double gv[UV][4], cv[UV][4];
#pragma unroll
            for (int u = 0; u < UV; ++u) {
                const bool itok = it0 + u < nit;
                const int c = 16 * (g0 + wid + NWB * (it0 + u)) + 4 * lg;
                ld4(crow + ((itok && c < b.ldm) ? c : 0), cv[u]);
                if constexpr (GV) {
                    ld4(grw + ((itok && c < b.m) ? c : 0), gv[u]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) gv[u][e] = ld_or0(grw, c + e, itok && c + e < b.m);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const bool ok = itok && c + e < b.m;
                    gv[u][e] = (grow && ok) ? gv[u][e] : 0.0;
                    cv[u][e] = (crok && ok) ? cv[u][e] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < UV; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) d = mma(gv[u][e], cv[u][e], d);
        }
        const d4 acc = waves_sum(d, red, NWB);
        // D[4v + lg][li] = V[j = 4v + lg][a0 + li]
        if (wid == 0 && crok)
#pragma unroll
            for (int v = 0; v < 4; ++v) b.V[((size_t)sp * KB + 4 * v + lg) * b.rmax + a0 + li] = acc[v];
        __syncthreads();
    }
}

// v: V = Gamma_blk C^T, 16 rows of C per tile, the columns split over the
// waves; the last KB workgroups take the norm, finiteness and target of one
// block row each.
template <typename T>
__global__ void __launch_bounds__(BW) k_bb_v(BigArgs<T> b, int64_t blk) {
    BigCtl *ctl = b.ctl;
    const int s = (int)(blk & 1);
    if (!ctl->active[s]) return;
    const int r0 = ctl->rank[s];
    const int64_t i0 = blk * b.kb;
    const int nb = (int)min((int64_t)b.kb, b.n - i0);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const T *gb = b.gam + i0 * b.m;
    const int ntw = gridDim.x - KB;  // the last KB workgroups take one block row each
    if ((int)blockIdx.x >= ntw) {
        __shared__ double nred[2][NWB];
        const int j = blockIdx.x - ntw;
        double g2 = 0.0, bad = 0.0;
        if (j < nb) {
            const T *row = gb + (int64_t)j * b.m;
            for (int c0 = threadIdx.x; c0 < b.m; c0 += BW * UB) {
                double v[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) v[u] = ld_or0(row, c0 + u * BW, c0 + u * BW < b.m);
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    g2 += v[u] * v[u];
                    bad += isfinite(v[u]) ? 0.0 : 1.0;
                }
            }
        }
        g2 = sum64(g2);
        bad = sum64(bad);
        if (lane == 0) {
            nred[0][wid] = g2;
            nred[1][wid] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            g2 = 0.0;
            bad = 0.0;
            for (int q = 0; q < NWB; ++q) {
                g2 += nred[0][q];
                bad += nred[1][q];
            }
            const double yv = j < nb ? (double)b.y[i0 + j] : 0.0;
            ctl->g2[j] = g2;
            ctl->y[j] = yv;
            ctl->bad[j] = (j < nb && (bad != 0.0 || !isfinite(g2) || !isfinite(yv))) ? 1 : 0;
        }
        return;
    }
    __shared__ d4 red[NWB][64];
    if (b.gvec)
        v_tiles<T, true>(b, r0, nb, gb, ntw, red);
    else
        v_tiles<T, false>(b, r0, nb, gb, ntw, red);
}

// g: G = V H^-1, 16 columns per tile, the inner dimension split over the
// waves; and the partial sums of G w per tile.
template <typename T>
__global__ void __launch_bounds__(BW) k_bb_g(BigArgs<T> b, int64_t blk) {
    BigCtl *ctl = b.ctl;
    const int s = (int)(blk & 1);
    if (!ctl->active[s]) return;
    const int r0 = ctl->rank[s];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
    __shared__ d4 red[NWB][64];
    const int nq = (r0 + 3) / 4;
    const int nit = (nq - wid + NWB - 1) / NWB;
    for (int t = blockIdx.x; 16 * t < r0; t += gridDim.x) {
        const int b0 = 16 * t;
        const bool colok = b0 + li < r0;
        d4 d = {0.0, 0.0, 0.0, 0.0};
        for (int it0 = 0; it0 < nit; it0 += UB) {
            double av[UB], bv[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int a = 4 * (wid + NWB * (it0 + u)) + lg;
                const bool ok = it0 + u < nit && a < r0;
                double sv = 0.0;
#pragma unroll
                for (int sp = 0; sp < vsplit<T>(); ++sp) sv += ld_or0(b.V, ((int64_t)sp * KB + li) * b.rmax + a, ok);
                av[u] = sv;
                bv[u] = ld_or0(b.H, (int64_t)a * b.rmax + b0 + li, ok && colok);
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) d = mma(av[u], bv[u], d);
        }
        const d4 acc = waves_sum(d, red, NWB);
        if (wid == 0) {
            const double wv = ld_or0(b.w, b0 + li, colok);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 4 * v + lg;
                if (colok) b.G[(size_t)j * b.rmax + b0 + li] = acc[v];
                const double gw = sum16(colok ? acc[v] * wv : 0.0);
                if (li == 0) b.gwp[(size_t)t * KB + j] = gw;
            }
        }
        __syncthreads();
    }
}

// rz: the first ns_grid workgroups form the rejections R = Gamma_blk - G C
// over 64-column slices (4 column tiles x 4 splits of the inner dimension)
// and the partial Gram matrices R R^T; the others form Z = P^-1 G^T per 16
// rows (inner dimension split over the waves) and the partial sums G Z.
template <typename T>
__global__ void __launch_bounds__(BW) k_bb_rz(BigArgs<T> b, int64_t blk, int ns_grid) {
    BigCtl *ctl = b.ctl;
    const int s = (int)(blk & 1);
    if (!ctl->active[s]) return;
    const int r0 = ctl->rank[s];
    const int64_t i0 = blk * b.kb;
    const int nb = (int)min((int64_t)b.kb, b.n - i0);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, li = lane & 15, lg = lane >> 4;
    const int nq = (r0 + 3) / 4;
    __shared__ d4 red[NWB][64];
    if ((int)blockIdx.x < ns_grid) {
        __shared__ double sR[KB][SL + 1];
        const T *gb = b.gam + i0 * b.m;
        constexpr int NKS = NWB / 4;            // splits of the inner dimension
        const int ct = wid & 3, ks = wid >> 2;  // column tile, split
        const int nit = (nq - ks + NKS - 1) / NKS;
        for (int sl = blockIdx.x; sl < b.ns; sl += ns_grid) {
            const int col = SL * sl + 16 * ct + li;
            const bool colok = col < b.m;
            d4 d = {0.0, 0.0, 0.0, 0.0};
            for (int it0 = 0; it0 < nit; it0 += UB) {
                double av[UB], bv[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int a = 4 * (ks + NKS * (it0 + u)) + lg;
                    const bool ok = it0 + u < nit && a < r0;
                    av[u] = ld_or0(b.G, (int64_t)li * b.rmax + a, ok);
                    bv[u] = ld_or0(b.C, (int64_t)a * b.ldm + col, ok && colok);
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) d = mma(av[u], bv[u], d);
            }
            red[wid][lane] = d;
            __syncthreads();
            if (ks == 0) {
                d4 acc = red[ct][lane];
#pragma unroll
                for (int q = 1; q < NKS; ++q) acc += red[ct + 4 * q][lane];
                // D[4v + lg][li] = (G C)[j = 4v + lg][col]
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = 4 * v + lg;
                    const double gv = ld_or0(gb, (int64_t)j * b.m + col, j < nb && colok);
                    const double rv = gv - acc[v];
                    sR[j][16 * ct + li] = rv;
                    if (colok) b.R[(size_t)j * b.m + col] = rv;
                }
            }
            __syncthreads();
            if (tid < KB * KB) {
                const int j = tid >> 4, l = tid & 15;
                double acc = 0.0;
#pragma unroll 8
                for (int c = 0; c < SL; ++c) acc += sR[j][c] * sR[l][c];
                b.rrp[(size_t)sl * (KB * KB) + tid] = acc;
            }
            __syncthreads();
        }
        return;
    }
    __shared__ double sZ[16][KB + 1];
    const int zg = gridDim.x - ns_grid;
    const int nit = (nq - wid + NWB - 1) / NWB;
    for (int t = blockIdx.x - ns_grid; 16 * t < r0; t += zg) {
        const int a0 = 16 * t;
        const bool rowok = a0 + li < r0;
        d4 d = {0.0, 0.0, 0.0, 0.0};
        for (int it0 = 0; it0 < nit; it0 += UB) {
            double av[UB], bv[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int c = 4 * (wid + NWB * (it0 + u)) + lg;
                const bool ok = it0 + u < nit && c < r0;
                av[u] = ld_or0(b.P, (int64_t)(a0 + li) * b.rmax + c, ok && rowok);
                bv[u] = ld_or0(b.G, (int64_t)li * b.rmax + c, ok);
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) d = mma(av[u], bv[u], d);
        }
        const d4 acc = waves_sum(d, red, NWB);
        if (wid == 0) {
            // D[4v + lg][li] = Z[a0 + 4v + lg][j = li]
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = a0 + 4 * v + lg;
                const double zv = a < r0 ? acc[v] : 0.0;
                sZ[4 * v + lg][li] = zv;
                if (a < r0) b.Z[(size_t)a * KB + li] = zv;
            }
        }
        __syncthreads();
        if (tid < KB * KB) {
            const int j = tid >> 4, l = tid & 15;
            double gv[16];
#pragma unroll
            for (int aa = 0; aa < 16; ++aa) gv[aa] = ld_or0(b.G, (int64_t)j * b.rmax + a0 + aa, a0 + aa < r0);
            double acc2 = 0.0;
#pragma unroll
            for (int aa = 0; aa < 16; ++aa) acc2 += gv[aa] * sZ[aa][l];
            b.gzp[(size_t)t * (KB * KB) + tid] = acc2;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// decide: one workgroup.
//  A  kinds (wave 0): the rank test of every row in order.  Rows before the
//     first one that is independent by its own rejection norm are dependent
//     with no block row in the basis (tested in parallel); from there on the
//     rows go one by one: L[l][.] = W_I R_I R_l^T, pivot, test; a new basis
//     row extends W_I = L_I^-1, a dependent row keeps c_l = W_I^T L[l][.].
//  B  the dependent rows at once: M (row d: e_l - sum_p c_p e_{piv_p}),
//     S = I + M G P^-1 G^T M^T + C C^T and dy = y_D - M G w - C y_I; then
//     Gauss-Jordan on [S | I | dy] (wave 0, one row of S per lane).  Without
//     pivot exchanges its pivots are the Cholesky pivots of S, i.e. the
//     sequential Greville denominators, so the denominator test stops the
//     block where the row-by-row algorithm would, and the leading block of
//     the inverse is what remains valid.
//  C  the k x k results from S^-1, S^-1 dy and W_I^T W_I.
struct DecideShared {
    double RR[KB][KB + 1], GZ[KB][KB + 1];
    double WI[KB][KB + 1];  // W_I = L_I^-1 (pivot order, lower triangular)
    double Cc[KB][KB + 1];  // row d: c of dependent row dep[d] (pivot-slot order)
    double M[KB][KB + 1];   // row d: e_{dep[d]} - sum_p c_p e_{piv_p}
    double U[KB][KB + 1];   // M G P^-1 G^T
    double Si[KB][KB + 1];  // S, then S^-1 (leading nd x nd)
    double X[KB][KB + 1], Xc[KB][KB + 1];  // S^-1 M, S^-1 C
    double WW[KB][KB + 1];  // W_I^T W_I
    double Lx[KB][KB + 1];  // explicit mode: L[l][p] per row l
    double gw[KB], g2[KB], y[KB], px[KB], dy[KB], sd[KB], ell[KB];
    double red[NWV][KB];
    int bad[KB], piv[KB], slot[KB], dep[KB];
    int ni, nd, napp, flag, amb;
};

__device__ inline void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline double eps_at(double eps_opt, int m, int r) {
    return eps_opt >= 0.0 ? eps_opt : ((double)m * m * r + (double)m * r + (double)m) * 0x1p-52;
}

// Phase A (wave 0; lanes 0..15 hold vector entries).  Gram mode stops with
// amb = 1 at the first row whose Gram pivot is not reliable; explicit mode
// reads L[l][.] and the pivots computed from the stored rejections.
__device__ void decide_kinds(DecideShared &S, int nb, int r0, int m, int rmax, double eps_opt, bool expl) {
    const int lane = threadIdx.x & 63;
    const bool lo = lane < KB;
    int ni = 0, nd = 0, napp = nb, flag = 0, amb = 0;
    int l0 = 0;
    if (!expl) {
        // rows before the first candidate basis row or non-finite row
        const double e0 = eps_at(eps_opt, m, r0);
        bool stop = false;
        if (lane < nb) {
            const double nr = sqrt(S.RR[lane][lane]), ng = sqrt(S.g2[lane]);
            const double p = S.RR[lane][lane];
            stop = S.bad[lane] || !(p <= 0.0 || nr < e0 || nr < e0 * ng);
        }
        const uint64_t mask = __ballot(stop) & 0xFFFFull;
        l0 = mask ? (int)__builtin_ctzll(mask) : nb;
        if (lane < l0) S.dep[lane] = lane;
        nd = l0;
        wsync();
    }
    for (int l = l0; l < nb; ++l) {
        const double diag = S.RR[l][l];
        double ell = 0.0, piv;
        if (!expl) {
            if (lane < ni)
                for (int q = 0; q <= lane; ++q) ell += S.WI[lane][q] * S.RR[S.piv[q]][l];
            piv = diag - read_lane(sum16(lane < ni ? ell * ell : 0.0), 0);
        } else {
            ell = lane < ni ? S.Lx[l][lane] : 0.0;
            piv = S.px[l];
        }
        const int rc = r0 + ni;
        const double eps = eps_at(eps_opt, m, rc);
        const double ng = sqrt(S.g2[l]);
        if (S.bad[l]) {
            flag = FLAG_NONFINITE;
            napp = l;
            break;
        }
        if (!expl && ni > 0) {
            const double nd0 = sqrt(diag);
            if (!(nd0 < eps || nd0 < eps * ng) && !(piv >= TAU * diag)) {
                amb = 1;
                napp = l;
                break;
            }
        }
        const double nr = sqrt(fmax(piv, 0.0));
        const bool indep = !(piv <= 0.0 || nr < eps || nr < eps * ng);
        if (lo) S.ell[lane] = ell;
        wsync();
        // lane q: sum_{p >= q} ell_p W_I[p][q], i.e. (W_I^T ell)_q
        double wte = 0.0;
        if (lane < ni)
            for (int p = lane; p < ni; ++p) wte += S.ell[p] * S.WI[p][lane];
        if (indep) {
            if (rc == rmax) {
                flag = FLAG_RANK_CAPACITY;
                napp = l;
                break;
            }
            // new row of W_I: [-(ell^T W_I) / L_ll, 1 / L_ll]
            const double inv = 1.0 / sqrt(piv);
            if (lo) S.WI[ni][lane] = lane < ni ? -wte * inv : (lane == ni ? inv : 0.0);
            if (lane == 0) {
                S.piv[ni] = l;
                S.slot[l] = ni;
            }
            wsync();
            ++ni;
        } else {
            if (lo) S.Cc[nd][lane] = lane < ni ? wte : 0.0;
            if (lane == 0) S.dep[nd] = l;
            wsync();
            ++nd;
        }
    }
    if (lane == 0) {
        S.ni = ni;
        S.nd = nd;
        S.napp = napp;
        S.flag = flag;
        S.amb = amb;
    }
}

// Phase B's inversion (wave 0): Gauss-Jordan on [S | I | dy] over the
// leading nd rows, lane i holding row i.  Stops at the first pivot that is
// not positive and finite; returns the number of pivots taken, with S^-1 of
// that leading block in S.Si and S^-1 dy in S.sd.
__device__ int gauss_jordan(DecideShared &S, int nd) {
    const int lane = threadIdx.x & 63;
    const bool act = lane < nd;
    double a[KB], b[KB], c;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        a[j] = act ? S.Si[lane][j] : 0.0;
        b[j] = (act && j == lane) ? 1.0 : 0.0;
    }
    c = act ? S.dy[lane] : 0.0;
    int done = nd;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < done) {
            const double pk = read_lane(a[k], k);
            if (!(pk > 0.0) || !isfinite(pk)) {
                done = k;
            } else {
                const double inv = 1.0 / pk;
                const double f = lane == k ? 0.0 : a[k] * inv;
                const double pc = read_lane(c, k);
#pragma unroll
                for (int j = k + 1; j < KB; ++j) {
                    const double pa = read_lane(a[j], k);
                    a[j] = lane == k ? a[j] * inv : a[j] - f * pa;
                }
#pragma unroll
                for (int j = 0; j <= k; ++j) {
                    const double pb = read_lane(b[j], k);
                    b[j] = lane == k ? b[j] * inv : b[j] - f * pb;
                }
                c = lane == k ? c * inv : c - f * pc;
                a[k] = lane == k ? 1.0 : 0.0;
            }
        }
    }
    if (lane < done) {
#pragma unroll
        for (int j = 0; j < KB; ++j) S.Si[lane][j] = j < done ? b[j] : 0.0;
        S.sd[lane] = c;
    }
    return done;
}

// Sums of up to KB per-thread partials over the workgroup (fixed order).
__device__ inline void block_sums(double *acc, int n, DecideShared &S, double *out) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        if (p < n) {
            const double v = sum64(acc[p]);
            if (lane == 0) S.red[wid][p] = v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        if (p < n) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NWV; ++q) v += S.red[q][p];
            out[p] = v;
        }
    }
    __syncthreads();
}

// Explicit rejections of the block rows (whole workgroup): row l against the
// orthonormalised rejections q_p of the rows appended before it, classical
// Gram-Schmidt applied twice.  Gives L[l][p] = <R_l, q_p> and the pivot
// ||R_l - sum_p L[l][p] q_p||^2, with the rank test of decide_kinds to choose
// the rows that join the q_p (the other outcomes of the rows are left to it).
template <typename T>
__device__ void explicit_rows(const BigArgs<T> &b, DecideShared &S, int nb, int r0) {
    const int tid = threadIdx.x;
    const int m = b.m;
    int npv = 0;
    for (int l = 0; l < nb; ++l) {
        if (S.bad[l]) break;
        const double *Rl = b.R + (size_t)l * m;
        double d1[KB], d2[KB], acc[KB];
#pragma unroll
        for (int p = 0; p < KB; ++p) acc[p] = 0.0;
        for (int c = tid; c < m; c += BT) {
            const double rv = Rl[c];
            double qv[KB];
#pragma unroll
            for (int p = 0; p < KB; ++p) qv[p] = ld_or0(b.Q, (int64_t)p * m + c, p < npv);
#pragma unroll
            for (int p = 0; p < KB; ++p) acc[p] += rv * qv[p];
        }
        block_sums(acc, npv, S, d1);
#pragma unroll
        for (int p = 0; p < KB; ++p) acc[p] = 0.0;
        for (int c = tid; c < m; c += BT) {
            double e = Rl[c];
            double qv[KB];
#pragma unroll
            for (int p = 0; p < KB; ++p) qv[p] = ld_or0(b.Q, (int64_t)p * m + c, p < npv);
#pragma unroll
            for (int p = 0; p < KB; ++p)
                if (p < npv) e -= d1[p] * qv[p];
#pragma unroll
            for (int p = 0; p < KB; ++p) acc[p] += e * qv[p];
        }
        block_sums(acc, npv, S, d2);
        double nn = 0.0;
        double *qn = b.Q + (size_t)npv * m;
        for (int c = tid; c < m; c += BT) {
            double e = Rl[c];
            double qv[KB];
#pragma unroll
            for (int p = 0; p < KB; ++p) qv[p] = ld_or0(b.Q, (int64_t)p * m + c, p < npv);
#pragma unroll
            for (int p = 0; p < KB; ++p)
                if (p < npv) e -= (d1[p] + d2[p]) * qv[p];
            nn += e * e;
            qn[c] = e;
        }
        double nsum[1];
        block_sums(&nn, 1, S, nsum);
#pragma unroll
        for (int p = 0; p < KB; ++p)
            if (tid == p) S.Lx[l][p] = p < npv ? d1[p] + d2[p] : 0.0;
        if (tid == 0) S.px[l] = nsum[0];
        const int rc = r0 + npv;
        const double eps = eps_at(b.eps, m, rc);
        const double nr = sqrt(fmax(nsum[0], 0.0)), ng = sqrt(S.g2[l]);
        const bool indep = !(nsum[0] <= 0.0 || nr < eps || nr < eps * ng);
        if (indep) {
            if (rc == b.rmax) break;
            const double inv = 1.0 / nr;
            __syncthreads();
            for (int c = tid; c < m; c += BT) qn[c] *= inv;
            ++npv;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(BT) k_bb_decide(BigArgs<T> b, int64_t blk) {
    BigCtl *ctl = b.ctl;
    const int s = (int)(blk & 1);
    const int tid = threadIdx.x, wid = tid >> 6;
    if (!ctl->active[s]) {
        if (tid == 0) {
            ctl->active[s ^ 1] = 0;
            ctl->rank[s ^ 1] = ctl->rank[s];
            ctl->ni = 0;
            ctl->nd = 0;
            ctl->napp = 0;
        }
        return;
    }
    __shared__ DecideShared S;
    const int r0 = ctl->rank[s];
    const int64_t i0 = blk * b.kb;
    const int nb = (int)min((int64_t)b.kb, b.n - i0);
    const int nt = (r0 + 15) / 16;
    const int x = tid >> 4, yy = tid & 15;
    {
        // partial sums in slice / tile order, UB loads in flight at a time
        double rr = 0.0, gz = 0.0;
        for (int q0 = 0; q0 < b.ns; q0 += UB) {
            double v[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) v[u] = ld_or0(b.rrp, (int64_t)(q0 + u) * (KB * KB) + tid, q0 + u < b.ns);
#pragma unroll
            for (int u = 0; u < UB; ++u) rr += v[u];
        }
        for (int q0 = 0; q0 < nt; q0 += UB) {
            double v[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) v[u] = ld_or0(b.gzp, (int64_t)(q0 + u) * (KB * KB) + tid, q0 + u < nt);
#pragma unroll
            for (int u = 0; u < UB; ++u) gz += v[u];
        }
        S.RR[x][yy] = rr;
        S.GZ[x][yy] = gz;
        S.WI[x][yy] = 0.0;
        S.Cc[x][yy] = 0.0;
        if (tid < KB) {
            double gw = 0.0;
            for (int q0 = 0; q0 < nt; q0 += UB) {
                double v[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) v[u] = ld_or0(b.gwp, (int64_t)(q0 + u) * KB + tid, q0 + u < nt);
#pragma unroll
                for (int u = 0; u < UB; ++u) gw += v[u];
            }
            S.gw[tid] = gw;
            S.g2[tid] = ctl->g2[tid];
            S.y[tid] = ctl->y[tid];
            S.bad[tid] = ctl->bad[tid];
            S.slot[tid] = -1;
            S.piv[tid] = 0;
            S.dep[tid] = 0;
        }
    }
    __syncthreads();
    {
        // rows from the first non-finite one on are never applied: their
        // entries (possibly NaN) are cleared so that zero weights stay zero
        int nf = nb;
        for (int j = 0; j < nb; ++j)
            if (S.bad[j]) {
                nf = j;
                break;
            }
        if (x >= nf || yy >= nf) {
            S.RR[x][yy] = 0.0;
            S.GZ[x][yy] = 0.0;
        }
        if (tid < KB && tid >= nf) S.gw[tid] = 0.0;
    }
    __syncthreads();
    // A: kinds
    if (wid == 0) decide_kinds(S, nb, r0, b.m, b.rmax, b.eps, false);
    __syncthreads();
    if (S.amb) {
        explicit_rows(b, S, nb, r0);
        S.WI[x][yy] = 0.0;
        S.Cc[x][yy] = 0.0;
        if (tid < KB) S.slot[tid] = -1;
        __syncthreads();
        if (wid == 0) decide_kinds(S, nb, r0, b.m, b.rmax, b.eps, true);
        __syncthreads();
    }
    int ni = S.ni, nd = S.nd;
    // B: S and dy of the dependent rows, then their inversion
    {
        double mv = 0.0;
        if (x < nd) {
            mv = yy == S.dep[x] ? 1.0 : 0.0;
            const int sl = S.slot[yy];
            if (sl >= 0 && sl < ni) mv -= S.Cc[x][sl];
        }
        S.M[x][yy] = mv;
    }
    __syncthreads();
    {
        double u = 0.0;
#pragma unroll
        for (int j = 0; j < KB; ++j) u += S.M[x][j] * S.GZ[j][yy];
        S.U[x][yy] = u;
    }
    __syncthreads();
    {
        double sv = x == yy ? 1.0 : 0.0;
        if (x < nd && yy < nd) {
#pragma unroll
            for (int j = 0; j < KB; ++j) sv += S.U[x][j] * S.M[yy][j];
            for (int q = 0; q < ni; ++q) sv += S.Cc[x][q] * S.Cc[yy][q];
        }
        S.Si[x][yy] = sv;
        if (tid < nd) {
            double t1 = 0.0, t2 = 0.0;
#pragma unroll
            for (int j = 0; j < KB; ++j) t1 += S.M[tid][j] * S.gw[j];
            for (int q = 0; q < ni; ++q) t2 += S.Cc[tid][q] * S.y[S.piv[q]];
            S.dy[tid] = (S.y[S.dep[tid]] - t1) - t2;
        }
    }
    __syncthreads();
    if (wid == 0) {
        const int done = gauss_jordan(S, nd);
        if (done < nd && threadIdx.x == 0) {
            // the denominator of dependent row dep[done] fails: the block ends there
            const int lstop = S.dep[done];
            int nk = 0;
            while (nk < S.ni && S.piv[nk] < lstop) ++nk;
            S.ni = nk;
            S.nd = done;
            S.napp = lstop;
            S.flag = FLAG_DENOMINATOR;
        }
    }
    __syncthreads();
    ni = S.ni;
    nd = S.nd;
    // C: X = S^-1 M, Xc = S^-1 C, W_I^T W_I
    {
        double xv = 0.0, xc = 0.0, ww = 0.0;
        if (x < nd)
            for (int e = 0; e < nd; ++e) {
                xv += S.Si[x][e] * S.M[e][yy];
                xc += S.Si[x][e] * S.Cc[e][yy];
            }
        if (x < ni && yy < ni)
            for (int p = max(x, yy); p < ni; ++p) ww += S.WI[p][x] * S.WI[p][yy];
        S.X[x][yy] = xv;
        S.Xc[x][yy] = yy < ni ? xc : 0.0;
        S.WW[x][yy] = ww;
    }
    __syncthreads();
    {
        double ap = 0.0, bp = 0.0, brp = 0.0;
        for (int d = 0; d < nd; ++d) {
            ap += S.M[d][x] * S.X[d][yy];
            bp += S.M[d][x] * S.Xc[d][yy];
            brp += S.Cc[d][x] * S.Xc[d][yy];
        }
        double *sm = b.sm;
        sm[SM_AP + tid] = ap;
        sm[SM_BP + tid] = yy < ni ? bp : 0.0;
        sm[SM_BRP + tid] = (x < ni && yy < ni) ? (x == yy ? 1.0 : 0.0) - brp : 0.0;
        const int sx = S.slot[x], sy = S.slot[yy];
        const bool px = sx >= 0 && sx < ni, py = sy >= 0 && sy < ni;
        sm[SM_AH + tid] = (px && py) ? S.WW[sx][sy] : 0.0;
        sm[SM_BH + tid] = (px && yy < ni) ? S.WW[sx][yy] : 0.0;
        sm[SM_BRH + tid] = S.WW[x][yy];
        if (tid < KB) {
            double qc = 0.0, wb = 0.0;
            for (int d = 0; d < nd; ++d) {
                qc += S.M[d][tid] * S.sd[d];
                wb += S.Cc[d][tid] * S.sd[d];
            }
            sm[SM_QC + tid] = qc;
            sm[SM_WB + tid] = tid < ni ? S.y[S.piv[tid]] + wb : 0.0;
            ctl->piv[tid] = S.piv[tid];
        }
    }
    if (tid == 0) {
        ctl->ni = ni;
        ctl->nd = nd;
        ctl->napp = S.napp;
        ctl->rank[s ^ 1] = r0 + ni;
        ctl->active[s ^ 1] = S.flag == 0 ? 1 : 0;
        ctl->applied += S.napp;
        if (S.flag) b.meta->flags |= (uint32_t)S.flag;
    }
}

// apply: w, the appended rows of C, then PT x PT tiles of the new P^-1 and
// H^-1 (r1 = r0 + ni), grid-stride.  Every element is written by one thread.
template <typename T>
__global__ void __launch_bounds__(BT) k_bb_apply(BigArgs<T> b, int64_t blk) {
    BigCtl *ctl = b.ctl;
    const int s = (int)(blk & 1);
    if (!ctl->active[s]) return;
    const int r0 = ctl->rank[s], ni = ctl->ni, nd = ctl->nd, r1 = r0 + ni, napp = ctl->napp;
    if (ni == 0 && nd == 0) return;
    const int tid = threadIdx.x;
    const int64_t gt = (int64_t)blockIdx.x * BT + tid, gs = (int64_t)gridDim.x * BT;
    const int nt1 = (r1 + PT - 1) / PT;
    if ((int64_t)blockIdx.x * BT >= max((int64_t)r0, (int64_t)ni * b.m) && (int)blockIdx.x >= nt1 * nt1) return;
    __shared__ double sm[SM_SIZE];
    __shared__ int spiv[KB];
    {
        constexpr int NL = (SM_SIZE + BT - 1) / BT;
        double v[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) v[k] = ld_or0(b.sm, tid + k * BT, tid + k * BT < SM_SIZE);
#pragma unroll
        for (int k = 0; k < NL; ++k)
            if (tid + k * BT < SM_SIZE) sm[tid + k * BT] = v[k];
    }
    if (tid < KB) spiv[tid] = ctl->piv[tid];
    __syncthreads();
    if (nd > 0)
        for (int64_t a = gt; a < r0; a += gs) {
            double zv[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) zv[j] = ld_or0(b.Z, a * KB + j, j < napp);
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < KB; ++j) acc += zv[j] * sm[SM_QC + j];
            b.w[a] += acc;
        }
    if (gt < ni) b.w[r0 + gt] = sm[SM_WB + gt];
    const int64_t i0 = blk * b.kb;
    for (int64_t e = gt; e < (int64_t)ni * b.m; e += gs) {
        const int p = (int)(e / b.m), c = (int)(e - (int64_t)p * b.m);
        b.C[(size_t)(r0 + p) * b.ldm + c] = b.gam[(i0 + spiv[p]) * b.m + c];
    }
    __shared__ double sZa[PT][KB + 1], sZb[PT][KB + 1], sGa[PT][KB + 1], sGb[PT][KB + 1];
    __shared__ double sYp[PT][KB + 1], sYh[PT][KB + 1];
    constexpr int NE = PT * KB / BT;  // tile entries per thread
    static_assert(PT * KB % BT == 0 && PT * PT == 4 * BT, "apply tile shape");
    for (int tile = blockIdx.x; tile < nt1 * nt1; tile += gridDim.x) {
        const int a0 = PT * (tile / nt1), b0 = PT * (tile % nt1);
        {
            double za[NE], zb[NE], ga[NE], gb[NE];
#pragma unroll
            for (int k = 0; k < NE; ++k) {
                const int e = tid + k * BT, rr = e / KB, j = e % KB;
                const int a = a0 + rr, bb = b0 + rr;
                const bool jok = j < napp;
                za[k] = ld_or0(b.Z, (int64_t)a * KB + j, jok && a < r0);
                zb[k] = ld_or0(b.Z, (int64_t)bb * KB + j, jok && bb < r0);
                ga[k] = ld_or0(b.G, (int64_t)j * b.rmax + a, jok && a < r0);
                gb[k] = ld_or0(b.G, (int64_t)j * b.rmax + bb, jok && bb < r0);
            }
#pragma unroll
            for (int k = 0; k < NE; ++k) {
                const int e = tid + k * BT, rr = e / KB, j = e % KB;
                sZa[rr][j] = za[k];
                sZb[rr][j] = zb[k];
                sGa[rr][j] = ga[k];
                sGb[rr][j] = gb[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const int e = tid + k * BT, rr = e / KB, j = e % KB;
            double yp = 0.0, yh = 0.0;
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                yp += sm[SM_AP + j * KB + l] * sZb[rr][l];
                yh += sm[SM_AH + j * KB + l] * sGb[rr][l];
            }
            sYp[rr][j] = yp;
            sYh[rr][j] = yh;
        }
        __syncthreads();
        const int aa = tid >> 3, bq = (tid & 7) * 4;
        const int a = a0 + aa;
        double pold[4], hold[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = b0 + bq + e;
            const bool tl = a < r0 && c < r0;
            pold[e] = ld_or0(b.P, (int64_t)a * b.rmax + c, tl && nd > 0);
            hold[e] = ld_or0(b.H, (int64_t)a * b.rmax + c, tl && ni > 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int bb = bq + e, c = b0 + bb;
            if (a >= r1 || c >= r1) continue;
            double *pp = b.P + (size_t)a * b.rmax + c;
            double *hp = b.H + (size_t)a * b.rmax + c;
            if (a < r0 && c < r0) {
                if (nd > 0) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < KB; ++j) acc += sZa[aa][j] * sYp[bb][j];
                    *pp = pold[e] - acc;
                }
                if (ni > 0) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < KB; ++j) acc += sGa[aa][j] * sYh[bb][j];
                    *hp = hold[e] + acc;
                }
            } else if (a < r0) {
                double ap = 0.0, ah = 0.0;
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    ap += sZa[aa][j] * sm[SM_BP + j * KB + (c - r0)];
                    ah += sGa[aa][j] * sm[SM_BH + j * KB + (c - r0)];
                }
                *pp = -ap;
                *hp = -ah;
            } else if (c < r0) {
                double ap = 0.0, ah = 0.0;
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    ap += sZb[bb][j] * sm[SM_BP + j * KB + (a - r0)];
                    ah += sGb[bb][j] * sm[SM_BH + j * KB + (a - r0)];
                }
                *pp = -ap;
                *hp = -ah;
            } else {
                *pp = sm[SM_BRP + (a - r0) * KB + (c - r0)];
                *hp = sm[SM_BRH + (a - r0) * KB + (c - r0)];
            }
        }
        __syncthreads();
    }
}

__global__ void k_bb_begin(StreamMeta *meta, BigCtl *ctl) {
    if (threadIdx.x == 0) {
        ctl->rank[0] = meta->r;
        ctl->active[0] = meta->flags == 0u ? 1 : 0;
        ctl->applied = 0;
    }
}

__global__ void k_bb_end(StreamMeta *meta, const BigCtl *ctl, int parity) {
    if (threadIdx.x == 0) {
        meta->r = ctl->rank[parity];
        meta->rows_seen += ctl->applied;
    }
}

// Solution x = C^T (H^-1 w) of the large stream: u = H^-1 w one wave per row
// of H^-1, then x over 64-column tiles with the rank split over the 4 waves.
__global__ void __launch_bounds__(BT) k_bs_u(const StreamMeta *meta, const double *H, const double *w, double *u,
                                              int rmax) {
    const int r = meta->r;
    const int lane = threadIdx.x & 63, row = blockIdx.x * NWV + (threadIdx.x >> 6);
    if (row >= r) return;
    const double *hr = H + (size_t)row * rmax;
    double acc = 0.0;
    for (int k = lane; k < r; k += 64) acc += hr[k] * w[k];
    acc = sum64(acc);
    if (lane == 0) u[row] = acc;
}

template <typename T>
__global__ void __launch_bounds__(BT) k_bs_x(const StreamMeta *meta, const T *C, const double *u, T *x, int m,
                                              int ldm) {
    __shared__ double red[NWV][64];
    const int r = meta->r;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (col < m)
        for (int k0 = wid * UB; k0 < r; k0 += NWV * UB) {
            double cv[UB];
            double uv[UB];
#pragma unroll
            for (int e = 0; e < UB; ++e) {
                cv[e] = ld_or0(C, (int64_t)(k0 + e) * ldm + col, k0 + e < r);
                uv[e] = ld_or0(u, k0 + e, k0 + e < r);
            }
#pragma unroll
            for (int e = 0; e < UB; ++e) acc += cv[e] * uv[e];
        }
    red[wid][lane] = acc;
    __syncthreads();
    if (wid == 0 && col < m) {
        double t = red[0][lane];
#pragma unroll
        for (int q = 1; q < NWV; ++q) t += red[q][lane];
        x[col] = (T)t;
    }
}

struct BigLayout {
    size_t V, G, Z, gwp, gzp, R, rrp, Q, sm, total;
};

BigLayout big_layout(int m, int rmax) {
    BigLayout L;
    const size_t nt = (size_t)(rmax + 15) / 16, ns = (size_t)(m + SL - 1) / SL;
    size_t off = CTL_DOUBLES;
    L.sm = off;
    off += SM_SIZE;
    L.V = off;
    off += (size_t)VS_MAX * KB * rmax;
    L.G = off;
    off += (size_t)KB * rmax;
    L.Z = off;
    off += (size_t)rmax * KB;
    L.gwp = off;
    off += nt * KB;
    L.gzp = off;
    off += nt * KB * KB;
    L.R = off;
    off += (size_t)KB * m;
    L.rrp = off;
    off += ns * KB * KB;
    L.Q = off;
    off += (size_t)KB * m;
    L.total = off;
    return L;
}

}  // namespace

size_t big_scratch_doubles(int m, int rmax) { return big_layout(m, rmax).total; }

template <typename T>
hipError_t launch_push_big(const PushArgs<T> &a, const StreamMeta &M, double *scratch, const T *gam, const T *y,
                           int64_t n, int num_cus, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const BigLayout L = big_layout(M.m, M.r_max);
    BigArgs<T> b;
    b.meta = a.meta;
    b.ctl = reinterpret_cast<BigCtl *>(scratch);
    b.C = a.state + M.state_off;
    b.P = a.preg + M.p_off;
    b.H = a.hreg + M.h_off;
    b.w = a.wreg + M.w_off;
    b.gam = gam;
    b.y = y;
    b.n = n;
    b.m = M.m;
    b.rmax = M.r_max;
    b.ldm = M.ldm;
    b.kb = (a.opts & OPT_ROW_BY_ROW) ? 1 : KB;
    b.ns = (M.m + SL - 1) / SL;
    b.gvec = (M.m % (int)(16 / sizeof(T)) == 0 && ((uintptr_t)gam & 15u) == 0) ? 1 : 0;
    b.eps = a.eps;
    b.V = scratch + L.V;
    b.G = scratch + L.G;
    b.Z = scratch + L.Z;
    b.gwp = scratch + L.gwp;
    b.gzp = scratch + L.gzp;
    b.R = scratch + L.R;
    b.rrp = scratch + L.rrp;
    b.Q = scratch + L.Q;
    b.sm = scratch + L.sm;
    const int tiles16 = (M.r_max + 15) / 16;
    const int g_v = std::min(tiles16 * vsplit<T>(), 2 * num_cus) + KB;
    const int g_g = std::min(tiles16, 2 * num_cus);
    const int ns_grid = std::min(b.ns, 2 * num_cus);
    const int g_rz = ns_grid + std::min(tiles16, 2 * num_cus);
    const int t32 = (M.r_max + PT - 1) / PT;
    const int g_ap = (int)std::min<int64_t>((int64_t)t32 * t32, 2 * (int64_t)num_cus);
    const int64_t nblk = (n + b.kb - 1) / b.kb;
    hipLaunchKernelGGL(k_bb_begin, dim3(1), dim3(64), 0, st, a.meta, b.ctl);
    for (int64_t blk = 0; blk < nblk; ++blk) {
        hipLaunchKernelGGL(k_bb_v<T>, dim3(g_v), dim3(BW), 0, st, b, blk);
        hipLaunchKernelGGL(k_bb_g<T>, dim3(g_g), dim3(BW), 0, st, b, blk);
        hipLaunchKernelGGL(k_bb_rz<T>, dim3(g_rz), dim3(BW), 0, st, b, blk, ns_grid);
        hipLaunchKernelGGL(k_bb_decide<T>, dim3(1), dim3(BT), 0, st, b, blk);
        hipLaunchKernelGGL(k_bb_apply<T>, dim3(g_ap), dim3(BT), 0, st, b, blk);
    }
    hipLaunchKernelGGL(k_bb_end, dim3(1), dim3(64), 0, st, a.meta, b.ctl, (int)(nblk & 1));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_solution_big(const StreamMeta *meta, const StreamMeta &M, const T *state, const double *hreg,
                               const double *wreg, double *scratch, T *x, hipStream_t st) {
    const BigLayout L = big_layout(M.m, M.r_max);
    double *u = scratch + L.V;
    hipLaunchKernelGGL(k_bs_u, dim3((M.r_max + NWV - 1) / NWV), dim3(BT), 0, st, meta, hreg + M.h_off,
                       wreg + M.w_off, u, M.r_max);
    hipLaunchKernelGGL(k_bs_x<T>, dim3((M.m + 63) / 64), dim3(BT), 0, st, meta, state + M.state_off, u,
                       x + M.x_off, M.m, M.ldm);
    return hipGetLastError();
}

template hipError_t launch_solution_big<float>(const StreamMeta *, const StreamMeta &, const float *,
                                               const double *, const double *, double *, float *, hipStream_t);
template hipError_t launch_solution_big<double>(const StreamMeta *, const StreamMeta &, const double *,
                                                const double *, const double *, double *, double *, hipStream_t);
template hipError_t launch_push_big<float>(const PushArgs<float> &, const StreamMeta &, double *, const float *,
                                           const float *, int64_t, int, hipStream_t);
template hipError_t launch_push_big<double>(const PushArgs<double> &, const StreamMeta &, double *, const double *,
                                            const double *, int64_t, int, hipStream_t);

}  // namespace rg
