// Batched rank-Greville update with the stream state on chip (FP32 state).
//
// One workgroup owns one stream for a whole push and walks its rows in order.
// Threads form a 2-D grid: lane pj (0..15) of a DPP row x row-group pk
// (0..PK-1, four per wave).  Thread (pk, pj) owns
//   columns J(pj) = { 64 c4 + 4 pj + e : c4 < CB4, e < 4 }   (float4 groups)
//   rows    K(pk) = { pk + PK b : b < RB }
//   P^-1 rows I(pj) = { pj + 16 a : a < IA }
// Residency during the push:
//   Ct    LDS, FP32, row-major with leading dimension MMAX (float4 reads);
//   C     registers, FP32, block K(pk) x J(pj);
//   P^-1  registers, FP64, block I(pj) x K(pk);
//   w     registers, FP64, entries K(pk) (same on the 16 lanes of a row);
//   Gamma LDS, FP32, double-buffered; the next row is prefetched into
//         registers while the current row is processed.
// Per row (Algorithm 1, the dependent case in the coordinates w = C x):
//   A  gamma_k = sum_j Ct[k][j] Gamma_j        partial over J(pj), all-reduced
//                                              over the 16 lanes of a DPP row
//   B  partials over K(pk) of (C^T gamma)_j, zeta_i = (P^-1 gamma)_i and
//      gamma^T w, reduced over the 4 DPP rows of a wave, then written to LDS
//   C  totals over the waves: Gamma_r = Gamma - C^T gamma, ||Gamma_r||^2,
//      1 + gamma^T zeta, y - gamma^T w (all FP64), then the rank test
//   D  dependent: P^-1 -= zeta zeta^T / d, w += zeta (y - gamma^T w) / d
//      independent: second projection pass, Ct -= gamma K^T, append
//      K^T to Ct, Gamma^T to C, a unit diagonal to P^-1 and y to w.
// Every branch condition is a workgroup-wide value (reduced through LDS), so
// all waves take the same path and meet the same barriers.
#include <vector>

#include "rg_classes.h"
#include "rg_lanes.h"

namespace rg {
namespace {

template <int PK_, int RB_, int CB4_>
struct Cls {
    static constexpr int PK = PK_, RB = RB_, CB4 = CB4_;
    static constexpr int NT = 16 * PK;
    static constexpr int NW = NT / 64;
    static constexpr int RMAX = PK * RB;
    static constexpr int MMAX = 64 * CB4;
    static constexpr int CB = 4 * CB4;
    static constexpr int IA = (RMAX + 15) / 16;
    static constexpr int ZP = 16 * IA;                // zeta slots per record (i = pj + 16 a)
    static constexpr int SP = MMAX + ZP + 2;
    static constexpr int NR = NW;  // one LDS record of partials per wave
    static_assert(NW <= 4, "at most 4 waves per stream");
    static constexpr int PF = (MMAX + NT - 1) / NT;
    static_assert(PK % 4 == 0, "row-groups come in whole waves");
};

// Phase B of a row: this thread's partial sums over its rows K(pk) of
//   q_j   = sum_k C[k][j] gamma_k          (columns J(pj))
//   z_i   = sum_k P^-1[i][k] gamma_k       (rows I(pj), when WITH_Z)
//   dyp   = sum_k gamma_k w_k              (when WITH_Z)
// reduced over the 4 DPP rows of the wave four values at a time, each row
// writing one of every four totals into the wave's LDS record.  The caller's
// next barrier makes the records visible.
template <class K, bool WITH_Z>
__device__ inline void partials(const float (&cr)[K::RB][K::CB], const double (&pr)[K::IA][K::RB],
                                const double (&wr)[K::RB], const double (&gam)[K::RB], double *spart) {
    constexpr int SP = K::SP, MMAX = K::MMAX, ZP = K::ZP, IA = K::IA, RB = K::RB, CB4 = K::CB4;
    const int t = threadIdx.x, pj = t & 15, lane = t & 63, wv = t >> 6, q = lane >> 4;
    double *rec = spart + wv * SP;
#pragma unroll
    for (int c4 = 0; c4 < CB4; ++c4) {
        double v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                float c = cr[b][4 * c4 + e];
                // The second projection pass converts C again instead of
                // keeping the first pass's FP64 copies of C live all row.
                if constexpr (!WITH_Z) asm volatile("" : "+v"(c));
                acc += (double)c * gam[b];
            }
            v[e] = acc;
        }
        rec[64 * c4 + 4 * pj + q] = scatter4(v[0], v[1], v[2], v[3]);
    }
    if constexpr (WITH_Z) {
        constexpr int NZ = IA + 1;  // the P^-1 rows, then gamma^T w
#pragma unroll
        for (int g = 0; g < (NZ + 3) / 4; ++g) {
            double v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int idx = 4 * g + e;
                double acc = 0.0;
                if (idx < IA) {
#pragma unroll
                    for (int b = 0; b < RB; ++b) acc += pr[idx][b] * gam[b];
                } else if (idx == IA) {
#pragma unroll
                    for (int b = 0; b < RB; ++b) acc += gam[b] * wr[b];
                }
                v[e] = acc;
            }
            const double tot = scatter4(v[0], v[1], v[2], v[3]);
            const int idx = 4 * g + q;
            if (idx < IA)
                rec[MMAX + pj + 16 * idx] = tot;
            else if (idx == IA && pj == 0)
                rec[MMAX + ZP] = tot;
        }
    }
}

template <int NW>
__device__ inline void block_sum2(double &a, double &b, double *sred) {
    a = sum64(a);
    b = sum64(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sred[2 * wid] = a;
        sred[2 * wid + 1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        a += sred[2 * i];
        b += sred[2 * i + 1];
    }
}

template <class K>
__global__ void __launch_bounds__(K::NT) k_push_rk(PushArgs<float> a, int rows_alloc) {
    constexpr int PK = K::PK, RB = K::RB, CB4 = K::CB4, CB = K::CB, NT = K::NT, NW = K::NW;
    constexpr int RMAX = K::RMAX, MMAX = K::MMAX, IA = K::IA, ZP = K::ZP, SP = K::SP, PF = K::PF, NR = K::NR;
    extern __shared__ double smem[];
    float *sct = reinterpret_cast<float *>(smem);      // rows_alloc x MMAX
    float *sg = sct + (size_t)rows_alloc * MMAX;        // 3 x MMAX (ring of rows)
    double *sgr = reinterpret_cast<double *>(sg + 4 * MMAX);  // MMAX (after a 3-row ring, 16-B aligned)
    double *spart = sgr + MMAX;                          // NW x SP
    double *sgam = spart + NR * SP;                      // RMAX
    double *szeta = sgam + RMAX;                         // RMAX
    double *sred = szeta + RMAX;                         // 2 NW

    const int t = threadIdx.x, pj = t & 15, pk = t >> 4;
    const int b_id = a.order[blockIdx.x];
    StreamMeta *M = a.meta + b_id;
    const int m = M->m, rmax = M->r_max, ldm = M->ldm;
    int r = M->r;
    uint32_t flags = M->flags;
    float *Cg = a.state + M->state_off;
    float *Ctg = Cg + (size_t)rmax * ldm;
    double *Pg = a.preg + M->p_off;
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
    const int cba4 = (m + 63) / 64;

    // ---- load the state ------------------------------------------------------
    for (int idx = t; idx < rows_alloc * MMAX; idx += NT) {
        const int k = idx / MMAX, j = idx - k * MMAX;
        sct[idx] = (k < r && j < m) ? Ctg[(size_t)k * ldm + j] : 0.0f;
    }
    float cr[RB][CB];
    double pr[IA][RB];
    double wr[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const int k = pk + PK * b;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int j = 64 * (c >> 2) + 4 * pj + (c & 3);
            cr[b][c] = (k < r && j < m) ? Cg[(size_t)k * ldm + j] : 0.0f;
        }
#pragma unroll
        for (int aa = 0; aa < IA; ++aa) {
            const int i = pj + 16 * aa;
            pr[aa][b] = (i < r && k < r) ? Pg[(size_t)i * rmax + k] : 0.0;
        }
        wr[b] = (k < r) ? wg[k] : 0.0;
    }
    for (int idx = t; idx < 3 * MMAX; idx += NT) sg[idx] = 0.0f;
    __syncthreads();
    float pre[PF];
    {
        const float *G0 = a.gamma + goff;
#pragma unroll
        for (int e = 0; e < PF; ++e) {
            const int j = t + NT * e;
            if (j < m) sg[j] = G0[j];
        }
        const float *G1 = G0 + m;
#pragma unroll
        for (int e = 0; e < PF; ++e) {
            const int j = t + NT * e;
            pre[e] = (i0 + 1 < i1 && j < m) ? G1[j] : 0.0f;
        }
    }
    __syncthreads();

    const bool reproject = !(a.opts & OPT_NO_REPROJECT);
    int rba = (r + PK - 1) / PK;
    int cur = 0;  // ring slot of row i
    int64_t applied = 0;
    float y_next = a.y[i0];
    // Finish the state loads here, so no wait inside the row loop has to
    // drain them (vector-memory waits complete in issue order).
    __builtin_amdgcn_s_waitcnt(0);
    for (int64_t i = i0; i < i1; ++i) {
        // Rows arrive through a 3-slot LDS ring: row i+1, requested one row
        // earlier, is stored now into slot cur+1 (last read by row i-2, two
        // barriers ago; read by row i+1 after this row's barriers); row i+2 is
        // requested now.  Targets are prefetched one row ahead the same way.
        const int nxt = cur == 2 ? 0 : cur + 1;
        if (i + 1 < i1) {
            float *gn = sg + nxt * MMAX;
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int j = t + NT * e;
                if (j < m) gn[j] = pre[e];
            }
        }
        if (i + 2 < i1) {
            const float *Gn = a.gamma + goff + (i + 2 - i0) * (int64_t)m;
#pragma unroll
            for (int e = 0; e < PF; ++e) {
                const int j = t + NT * e;
                pre[e] = (j < m) ? Gn[j] : 0.0f;
            }
        }
        const double yv = (double)y_next;
        if (i + 1 < i1) y_next = a.y[i + 1];
        const float *gcur = sg + cur * MMAX;

        // ---- A: gamma = Ct Gamma --------------------------------------------
        // All RB row slots are processed (rows k >= r hold zeros), so no
        // per-slot branch splits the accumulation chains; the 64-column
        // groups are a runtime loop to keep few loads in flight.
        double g2 = 0.0;
        double gam[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) gam[b] = 0.0;
#pragma unroll 1
        for (int c4 = 0; c4 < cba4; ++c4) {
            const float4 gv = *reinterpret_cast<const float4 *>(gcur + 64 * c4 + 4 * pj);
            const double g0 = gv.x, g1 = gv.y, g2v = gv.z, g3 = gv.w;
            g2 += g0 * g0 + g1 * g1 + g2v * g2v + g3 * g3;
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const int k = pk + PK * b;
                float4 v = *reinterpret_cast<const float4 *>(sct + (size_t)min(k, rows_alloc - 1) * MMAX + 64 * c4 + 4 * pj);
                if (k >= rows_alloc) v = make_float4(0.f, 0.f, 0.f, 0.f);
                gam[b] += (double)v.x * g0;
                gam[b] += (double)v.y * g1;
                gam[b] += (double)v.z * g2v;
                gam[b] += (double)v.w * g3;
            }
        }
        g2 = sum16(g2);
        if (!isfinite(g2) || !isfinite(yv)) {
            flags |= FLAG_NONFINITE;
            break;
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) gam[b] = sum16(gam[b]);
        // ---- B: partials over K(pk) ----------------------------------------
        partials<K, true>(cr, pr, wr, gam, spart);
        if (pj == 0) {
#pragma unroll
            for (int b = 0; b < RB; ++b) sgam[pk + PK * b] = gam[b];
        }
        __syncthreads();

        // ---- C: totals over the waves ----------------------------------------
        double sp = 0.0, dp = 0.0;
        for (int j = t; j < m; j += NT) {
            double v = (double)gcur[j];
#pragma unroll
            for (int w = 0; w < NR; ++w) v -= spart[w * SP + j];
            sgr[j] = v;
            sp += v * v;
        }
        for (int ii = t; ii < r; ii += NT) {
            double zz = 0.0;
#pragma unroll
            for (int w = 0; w < NR; ++w) zz += spart[w * SP + MMAX + ii];
            szeta[ii] = zz;
            dp += sgam[ii] * zz;
        }
        double gw = 0.0;
#pragma unroll
        for (int w = 0; w < NR; ++w) gw += spart[w * SP + MMAX + ZP];
        block_sum2<NW>(sp, dp, sred);
        const double s = sp;
        const double eps = a.eps >= 0.0 ? a.eps
                                        : ((double)m * m * r + (double)m * r + (double)m) * 0x1p-52;
        const double nr = sqrt(s), ng = sqrt(g2);
        const bool dependent = (s == 0.0) || (nr < eps) || (nr < eps * ng);

        if (dependent) {
            if (r > 0) {
                const double d = 1.0 + dp;
                if (!(d > 0.0) || !isfinite(d)) {
                    flags |= FLAG_DENOMINATOR;
                    break;
                }
                const double inv_d = 1.0 / d;
                const double f = (yv - gw) * inv_d;
                double zk[RB], zi[IA];
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const int k = pk + PK * b;
                    zk[b] = (k < r) ? szeta[k] : 0.0;
                }
#pragma unroll
                for (int aa = 0; aa < IA; ++aa) {
                    const int i = pj + 16 * aa;
                    zi[aa] = (i < r) ? szeta[min(i, RMAX - 1)] : 0.0;
                }
#pragma unroll
                for (int aa = 0; aa < IA; ++aa) {
                    const double za = zi[aa] * inv_d;
#pragma unroll
                    for (int b = 0; b < RB; ++b) pr[aa][b] -= za * zk[b];
                }
#pragma unroll
                for (int b = 0; b < RB; ++b) wr[b] += zk[b] * f;
            }
        } else {
            if (r == rmax) {
                flags |= FLAG_RANK_CAPACITY;
                break;
            }
            double s_use = s;
            if (reproject && r > 0) {
                // second pass ("twice is enough"): gamma2 = Ct Gamma_r, Gamma_r -= C^T gamma2;
                // zero in exact arithmetic, it removes the rounding left in Gamma_r.
                double gam2[RB];
#pragma unroll
                for (int b = 0; b < RB; ++b) gam2[b] = 0.0;
#pragma unroll 1
                for (int c4 = 0; c4 < cba4; ++c4) {
                    const int j0 = 64 * c4 + 4 * pj;
                    const double r0 = j0 < m ? sgr[j0] : 0.0, r1 = j0 + 1 < m ? sgr[j0 + 1] : 0.0;
                    const double r2 = j0 + 2 < m ? sgr[j0 + 2] : 0.0, r3 = j0 + 3 < m ? sgr[j0 + 3] : 0.0;
#pragma unroll
                    for (int b = 0; b < RB; ++b) {
                        const int k = pk + PK * b;
                        float4 v = *reinterpret_cast<const float4 *>(sct + (size_t)min(k, rows_alloc - 1) * MMAX + j0);
                        if (k >= rows_alloc) v = make_float4(0.f, 0.f, 0.f, 0.f);
                        gam2[b] += (double)v.x * r0 + (double)v.y * r1 + (double)v.z * r2 + (double)v.w * r3;
                    }
                }
#pragma unroll
                for (int b = 0; b < RB; ++b) gam2[b] = sum16(gam2[b]);
                partials<K, false>(cr, pr, wr, gam2, spart);
                __syncthreads();
                double sp2 = 0.0, unused = 0.0;
                for (int j = t; j < m; j += NT) {
                    double v = sgr[j];
#pragma unroll
                    for (int w = 0; w < NR; ++w) v -= spart[w * SP + j];
                    sgr[j] = v;
                    sp2 += v * v;
                }
                block_sum2<NW>(sp2, unused, sred);
                s_use = sp2;
#pragma unroll
                for (int b = 0; b < RB; ++b) gam[b] += gam2[b];
            }
            const double inv_s = 1.0 / s_use;
            float Kf[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = 64 * (c >> 2) + 4 * pj + (c & 3);
                Kf[c] = (j < m) ? (float)(sgr[j] * inv_s) : 0.0f;
            }
            // Ct <- Ct - gamma K^T on rows k < r
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const int k = pk + PK * b;
                if (b < rba && k < r) {
                    const float gb = (float)gam[b];
#pragma unroll
                    for (int c4 = 0; c4 < CB4; ++c4)
                        if (c4 < cba4) {
                            float4 *p4 = reinterpret_cast<float4 *>(sct + (size_t)k * MMAX + 64 * c4 + 4 * pj);
                            float4 v = *p4;
                            v.x = fmaf(-gb, Kf[4 * c4 + 0], v.x);
                            v.y = fmaf(-gb, Kf[4 * c4 + 1], v.y);
                            v.z = fmaf(-gb, Kf[4 * c4 + 2], v.z);
                            v.w = fmaf(-gb, Kf[4 * c4 + 3], v.w);
                            *p4 = v;
                        }
                }
            }
            // append: row r of Ct and C, P^-1[r][r] = 1, w[r] = y
            if (pk == r % PK) {
                const int br = r / PK;
#pragma unroll
                for (int c4 = 0; c4 < CB4; ++c4)
                    if (c4 < cba4) {
                        float4 v;
                        v.x = Kf[4 * c4 + 0];
                        v.y = Kf[4 * c4 + 1];
                        v.z = Kf[4 * c4 + 2];
                        v.w = Kf[4 * c4 + 3];
                        *reinterpret_cast<float4 *>(sct + (size_t)r * MMAX + 64 * c4 + 4 * pj) = v;
                    }
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    if (b == br) {
#pragma unroll
                        for (int c = 0; c < CB; ++c) {
                            const int j = 64 * (c >> 2) + 4 * pj + (c & 3);
                            cr[b][c] = (j < m) ? gcur[j] : 0.0f;
                        }
                        wr[b] = yv;
                        if (pj == r % 16) {
#pragma unroll
                            for (int aa = 0; aa < IA; ++aa)
                                if (aa == r / 16) pr[aa][b] = 1.0;
                        }
                    }
                }
            }
            r += 1;
            rba = (r + PK - 1) / PK;
            __syncthreads();
        }
        ++applied;
        cur = nxt;
    }

    // ---- write the state back ------------------------------------------------
    __syncthreads();
    for (int idx = t; idx < rows_alloc * MMAX; idx += NT) {
        const int k = idx / MMAX, j = idx - k * MMAX;
        if (k < r && j < m) Ctg[(size_t)k * ldm + j] = sct[idx];
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const int k = pk + PK * b;
        if (k < r) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = 64 * (c >> 2) + 4 * pj + (c & 3);
                if (j < m) Cg[(size_t)k * ldm + j] = cr[b][c];
            }
#pragma unroll
            for (int aa = 0; aa < IA; ++aa) {
                const int i = pj + 16 * aa;
                if (i < r) Pg[(size_t)i * rmax + k] = pr[aa][b];
            }
            if (pj == 0) wg[k] = wr[b];
        }
    }
    if (t == 0) {
        M->r = r;
        M->flags = flags;
        M->rows_seen += applied;
    }
    __syncthreads();
}

// Row-by-row size classes (PK, RB, CB4): RMAX = PK*RB rows, MMAX = 64*CB4
// columns.  Larger streams go to the blocked kernel (rg_mf.hip).
using C0 = Cls<4, 3, 1>;
using C1 = Cls<4, 9, 1>;
using C2 = Cls<16, 2, 2>;

template <class K>
size_t lds_bytes(int rows_alloc) {
    return sizeof(float) * ((size_t)rows_alloc * K::MMAX + 4 * K::MMAX) +
           sizeof(double) * ((size_t)K::MMAX + K::NR * K::SP + 2 * K::RMAX + 2 * K::NW);
}

template <class K>
bool fits(int m, int r_max) {
    const int rows_alloc = r_max;
    return m <= K::MMAX && r_max <= K::RMAX && lds_bytes<K>(rows_alloc) <= 160 * 1024;
}

// The dynamic-LDS limit of a class kernel is process-wide state: it is set
// once, to what the class needs at its full rank capacity, so that a handle
// created later can never lower it under the launches of a live handle.
template <class K>
hipError_t prepare(int rows_alloc) {
    if (lds_bytes<K>(rows_alloc) > 160 * 1024) return hipErrorInvalidValue;
    static const hipError_t once = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_push_rk<K>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)lds_bytes<K>(K::RMAX));
    return once;
}

template <class K>
hipError_t launch(const PushArgs<float> &a, int rows_alloc, hipStream_t s) {
    const size_t lds = lds_bytes<K>(rows_alloc);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_push_rk<K>, dim3(a.n_order), dim3(K::NT), lds, s, a, rows_alloc);
    return hipGetLastError();
}

}  // namespace

// Classes 0..2 are this file's kernel, 3..8 the blocked kernel's variants 0..5,
// RG_CLASS_F64 the blocked kernel's FP64 variant.
int class_rmax(int cls) {
    switch (cls) {
        case 0: return C0::RMAX;
        case 1: return C1::RMAX;
        case 2: return C2::RMAX;
        case RG_CLASS_F64: return mf64_rmax();
    }
    return cls >= 3 ? mf_rmax(cls - 3) : 0;
}

bool class_factored(int cls) { return cls >= 3 && cls <= RG_CLASS_F64; }

bool class_fits(int cls, int m, int r_max) {
    switch (cls) {
        case 0: return fits<C0>(m, r_max);
        case 1: return fits<C1>(m, r_max);
        case 2: return fits<C2>(m, r_max);
        case RG_CLASS_F64: return mf64_fits(m, r_max);
    }
    return cls >= 3 && cls < RG_NUM_CLASSES && mf_fits(cls - 3, m, r_max);
}

int class_mmax(int cls) {
    switch (cls) {
        case 0: return C0::MMAX;
        case 1: return C1::MMAX;
        case 2: return C2::MMAX;
        case RG_CLASS_F64: return mf64_mmax();
    }
    return cls >= 3 ? mf_mmax(cls - 3) : 0;
}

int class_threads(int cls) {
    switch (cls) {
        case 0: return C0::NT;
        case 1: return C1::NT;
        case 2: return C2::NT;
        case RG_CLASS_F64: return mf64_threads();
    }
    return cls >= 3 ? mf_threads(cls - 3) : 0;
}

namespace {
struct ClassRule {
    int m_hi, r_max_hi, cls;
};
std::vector<ClassRule> g_rules;  // empty: the built-in order below
}  // namespace

void set_class_rules(const int *m_hi, const int *r_max_hi, const int *cls, int n) {
    g_rules.clear();
    for (int k = 0; k < n; ++k) g_rules.push_back({m_hi[k], r_max_hi[k], cls[k]});
}

int choose_class(int m, int r_max, int dtype) {
    if (dtype != 0) return mf64_fits(m, r_max) ? RG_CLASS_F64 : -1;  // FP64 state: one class
    for (const ClassRule &rule : g_rules) {
        if (m > rule.m_hi || r_max > rule.r_max_hi) continue;
        if (rule.cls < 0) return -1;
        if (class_fits(rule.cls, m, r_max)) return rule.cls;
    }
    // built-in: the smallest blocked variant that holds the stream (factored
    // dual basis); the row-by-row classes only where a rule asks for them
    const int v = mf_choose(m, r_max);
    if (v >= 0) return 3 + v;
    if (fits<C0>(m, r_max)) return 0;
    if (fits<C1>(m, r_max)) return 1;
    if (fits<C2>(m, r_max)) return 2;
    return -1;
}

hipError_t prepare_class(int cls, int rows_alloc) {
    switch (cls) {
        case 0: return prepare<C0>(rows_alloc);
        case 1: return prepare<C1>(rows_alloc);
        case 2: return prepare<C2>(rows_alloc);
        case RG_CLASS_F64: return mf64_prepare(rows_alloc);
    }
    return cls >= 3 ? mf_prepare(cls - 3, rows_alloc) : hipErrorInvalidValue;
}

template <>
hipError_t launch_push_class<float>(int cls, const PushArgs<float> &a, int rows_alloc, hipStream_t s) {
    switch (cls) {
        case 0: return launch<C0>(a, rows_alloc, s);
        case 1: return launch<C1>(a, rows_alloc, s);
        case 2: return launch<C2>(a, rows_alloc, s);
    }
    return cls >= 3 && cls < RG_NUM_CLASSES ? mf_launch(cls - 3, a, rows_alloc, s) : hipErrorInvalidValue;
}

template <>
hipError_t launch_push_class<double>(int cls, const PushArgs<double> &a, int rows_alloc, hipStream_t s) {
    return cls == RG_CLASS_F64 ? mf64_launch(a, rows_alloc, s) : hipErrorInvalidValue;
}

}  // namespace rg
