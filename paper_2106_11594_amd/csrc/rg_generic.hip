// Generic rank-Greville kernels for gfx950: state read and written in global
// memory (L2 / HBM), any m and r_max that fit the LDS work vectors.
//
// One workgroup (4 wave64) owns one stream at a time and walks its rows in
// order; workgroups take streams from a device-side queue (largest first).
// Per row, following Algorithm 1 (UpdateLeastSquares):
//   gamma   = Ct Gamma                 one wave per row k of Ct, lanes over j
//   Gamma_r = Gamma - C^T gamma        one thread per column j, FP64 sum
//   rank test of Section 3 on ||Gamma_r|| (FP64), uniform per workgroup
//   independent (Theorems 4, 6): optional second projection pass,
//       K = Gamma_r / ||Gamma_r||^2, Ct <- [Ct - gamma K^T; K^T],
//       C <- [C; Gamma^T], P^-1 <- diag(P^-1, 1), w <- [w; y]
//   dependent (Theorems 5, 6): zeta = P^-1 gamma, d = 1 + gamma^T zeta,
//       P^-1 <- P^-1 - zeta zeta^T / d, w <- w + zeta (y - gamma^T w) / d
// The solution is kept in coordinates w = C x (x = Ct^T w because
// Ct C^T = I), which removes the pass over Ct that forms the dependent-case
// gain K = Ct^T zeta / d; x is formed on demand by the solution kernel.
#include "rg_internal.h"
#include "rg_lanes.h"

namespace rg {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

// Accumulation type of gamma = Ct Gamma and zeta = P^-1 gamma.  FP64 for both
// state types: with FP32 accumulation the x error roughly doubles on poorly
// conditioned bases (measured against the FP64 oracle).
template <typename T> struct AccG { using type = double; };

// Sum over the 64 lanes of a wave with DPP and permlane steps (no LDS round
// trips); every lane gets the same bits.
__device__ inline double wave_sum(double v) { return sum64(v); }

// Sum a and b over the workgroup; every thread gets the totals.  Fixed
// order, so the result does not depend on scheduling.
__device__ inline void block_sum2(double &a, double &b, double *sRed) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        sRed[2 * wid] = a;
        sRed[2 * wid + 1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        a += sRed[2 * i];
        b += sRed[2 * i + 1];
    }
}

// dst[k] = sum_j Ct[k][j] v[j] for k < r.
template <typename T, typename Acc>
__device__ inline void project(const T *Ct, int ldm, const double *v, double *dst, int r, int m) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = wid; k < r; k += NW) {
        const T *row = Ct + (size_t)k * ldm;
        Acc acc = 0;
        for (int j = lane; j < m; j += 64) acc += (Acc)row[j] * (Acc)v[j];
        acc = wave_sum(acc);
        if (lane == 0) dst[k] = (double)acc;
    }
}

// out[j] = v[j] - sum_k C[k][j] g[k] in FP64; returns this thread's share of
// sum_j out[j]^2 (out may alias v).
template <typename T>
__device__ inline double reject(const T *C, int ldm, const double *v, const double *g, double *out, int r,
                                int m) {
    double s = 0.0;
    for (int j = threadIdx.x; j < m; j += NT) {
        double acc = v[j];
        for (int k = 0; k < r; ++k) acc -= (double)C[(size_t)k * ldm + j] * g[k];
        out[j] = acc;
        s += acc * acc;
    }
    return s;
}

// Bytes of one stream's state held in LDS (C and Ct, rmax x ldm each, then
// P^-1 and w in doubles).
template <typename T>
__host__ __device__ inline size_t lds_state_bytes(int rmax, int ldm) {
    const size_t ct = 2 * (size_t)rmax * ldm * sizeof(T);
    return (ct + 7) / 8 * 8 + sizeof(double) * ((size_t)rmax * rmax + rmax);
}

template <typename T>
__device__ void run_stream(const PushArgs<T> &a, int b, double *sG, double *sGr, double *sGam, double *sGam2,
                           double *sZ, double *sRed, double *sState) {
    StreamMeta *M = a.meta + b;
    const int m = M->m, rmax = M->r_max, ldm = M->ldm;
    int r = M->r;
    uint32_t flags = M->flags;
    T *const Cg = a.state + M->state_off;
    double *const Pg = a.preg + M->p_off;
    double *const wg = a.wreg + M->w_off;
    T *C = Cg;
    T *Ct = C + (size_t)rmax * ldm;
    double *P = Pg;
    double *w = wg;
    // With sState (the launch reserved room for the largest stream), the push
    // works on an LDS copy of the state: loaded here, written back at the end.
    if (sState) {
        C = reinterpret_cast<T *>(sState);
        Ct = C + (size_t)rmax * ldm;
        P = sState + (2 * (size_t)rmax * ldm * sizeof(T) + 7) / 8;
        w = P + (size_t)rmax * rmax;
        for (int idx = threadIdx.x; idx < r * ldm; idx += NT) {
            C[idx] = Cg[idx];
            Ct[idx] = Cg[(size_t)rmax * ldm + idx];
        }
        for (int idx = threadIdx.x; idx < r * r; idx += NT) {
            const int ii = idx / r, k = idx - ii * r;
            P[(size_t)ii * rmax + k] = Pg[(size_t)ii * rmax + k];
        }
        for (int k = threadIdx.x; k < r; k += NT) w[k] = wg[k];
        __syncthreads();
    }
    int64_t i0, i1, goff;
    if (a.row_ptr) {
        i0 = a.row_ptr[b];
        i1 = a.row_ptr[b + 1];
        goff = a.gamma_off[b];
    } else {
        i0 = 0;
        i1 = a.k_single;
        goff = 0;
    }
    const int tid = threadIdx.x;
    int64_t applied = 0;
    using Acc = typename AccG<T>::type;
    for (int64_t i = i0; i < i1 && flags == 0; ++i) {
        const T *G = a.gamma + goff + (i - i0) * (int64_t)m;
        double g2 = 0.0, bad = 0.0;
        for (int j = tid; j < m; j += NT) {
            const double g = (double)G[j];
            sG[j] = g;
            g2 += g * g;
            if (!isfinite(g)) bad = 1.0;
        }
        const double yv = (double)a.y[i];
        block_sum2(g2, bad, sRed);
        if (bad != 0.0 || !isfinite(yv)) {
            flags |= FLAG_NONFINITE;
            break;
        }
        project<T, Acc>(Ct, ldm, sG, sGam, r, m);
        __syncthreads();
        double s = reject(C, ldm, sG, sGam, sGr, r, m), unused = 0.0;
        block_sum2(s, unused, sRed);
        const double eps = a.eps >= 0.0 ? a.eps
                                        : ((double)m * m * r + (double)m * r + (double)m) * 0x1p-52;
        const double nr = sqrt(s), ng = sqrt(g2);
        const bool dependent = (s == 0.0) || (nr < eps) || (nr < eps * ng);
        if (!dependent) {
            if (r == rmax) {
                flags |= FLAG_RANK_CAPACITY;
                break;
            }
            if (!(a.opts & OPT_NO_REPROJECT) && r > 0) {
                // second pass ("twice is enough"): gamma2 = Ct Gamma_r, Gamma_r -= C^T gamma2;
                // zero in exact arithmetic, it removes the rounding left in Gamma_r.
                project<T, Acc>(Ct, ldm, sGr, sGam2, r, m);
                __syncthreads();
                s = reject(C, ldm, sGr, sGam2, sGr, r, m);
                unused = 0.0;
                block_sum2(s, unused, sRed);
                for (int k = tid; k < r; k += NT) sGam[k] += sGam2[k];
                __syncthreads();
            }
            if (a.opts & (OPT_ORTHOGONAL | OPT_ORTHONORMAL)) {
                // Orthogonal rank factorization (Section 2.2): C gets alpha Gamma_r, Ct gets
                // Gamma_r / (alpha ||Gamma_r||^2) and keeps its other rows, P^-1 is bordered
                // with -alpha zeta and alpha^2 (1 + gamma^T zeta), zeta = P^-1 gamma; in
                // coordinates the new entry of w is alpha (y - gamma^T w).
                for (int ii = tid; ii < r; ii += NT) {
                    double acc = 0.0;
                    for (int k = 0; k < r; ++k) acc += P[(size_t)k * rmax + ii] * sGam[k];
                    sZ[ii] = acc;
                }
                __syncthreads();
                double gz = 0.0, gw = 0.0;
                for (int k = tid; k < r; k += NT) {
                    gz += sGam[k] * sZ[k];
                    gw += sGam[k] * w[k];
                }
                block_sum2(gz, gw, sRed);
                const bool unit = (a.opts & OPT_ORTHONORMAL) != 0;
                const double alpha = unit ? 1.0 / sqrt(s) : 1.0;
                const double inv_as = 1.0 / (alpha * s);
                for (int j = tid; j < m; j += NT) {
                    const double cj = alpha * sGr[j];
                    C[(size_t)r * ldm + j] = (T)cj;
                    Ct[(size_t)r * ldm + j] = unit ? (T)cj : (T)(sGr[j] * inv_as);
                }
                for (int k = tid; k < r; k += NT) {
                    P[(size_t)r * rmax + k] = -alpha * sZ[k];
                    P[(size_t)k * rmax + r] = -alpha * sZ[k];
                }
                if (tid == 0) {
                    P[(size_t)r * rmax + r] = alpha * alpha * (1.0 + gz);
                    w[r] = alpha * (yv - gw);
                }
                r += 1;
                ++applied;
                __syncthreads();
                continue;
            }
            const double inv_s = 1.0 / s;
            for (int j = tid; j < m; j += NT) {
                const double K = sGr[j] * inv_s;
                if constexpr (sizeof(T) == 4) {
                    const float Kf = (float)K;
                    for (int k = 0; k < r; ++k) {
                        float &c = Ct[(size_t)k * ldm + j];
                        c = fmaf(-(float)sGam[k], Kf, c);
                    }
                } else {
                    for (int k = 0; k < r; ++k) {
                        double &c = Ct[(size_t)k * ldm + j];
                        c = fma(-sGam[k], K, c);
                    }
                }
                Ct[(size_t)r * ldm + j] = (T)K;
                C[(size_t)r * ldm + j] = (T)sG[j];
            }
            for (int k = tid; k < r; k += NT) {
                P[(size_t)r * rmax + k] = 0.0;
                P[(size_t)k * rmax + r] = 0.0;
            }
            if (tid == 0) {
                P[(size_t)r * rmax + r] = 1.0;
                w[r] = yv;
            }
            r += 1;
        } else if (r > 0) {
            // zeta_i = sum_k P[k][i] gamma_k  (P^-1 is symmetric; column reads coalesce)
            for (int ii = tid; ii < r; ii += NT) {
                double acc = 0.0;
                for (int k = 0; k < r; ++k) acc += P[(size_t)k * rmax + ii] * sGam[k];
                sZ[ii] = acc;
            }
            __syncthreads();
            double gz = 0.0, gw = 0.0;
            for (int k = tid; k < r; k += NT) {
                gz += sGam[k] * sZ[k];
                gw += sGam[k] * w[k];
            }
            block_sum2(gz, gw, sRed);
            const double d = 1.0 + gz;
            if (!(d > 0.0) || !isfinite(d)) {
                flags |= FLAG_DENOMINATOR;
                break;
            }
            const double inv_d = 1.0 / d;
            const double dy = yv - gw;
            // P^-1 <- P^-1 - zeta zeta^T / d (FP64; the product order keeps it exactly symmetric)
            const int rr = r * r;
            for (int idx = tid; idx < rr; idx += NT) {
                const int ii = idx / r, k = idx - ii * r;
                P[(size_t)ii * rmax + k] -= (sZ[ii] * sZ[k]) * inv_d;
            }
            for (int k = tid; k < r; k += NT) w[k] += sZ[k] * (dy * inv_d);
        }
        ++applied;
        __syncthreads();
    }
    __syncthreads();
    if (sState) {
        for (int idx = tid; idx < r * ldm; idx += NT) {
            Cg[idx] = C[idx];
            Cg[(size_t)rmax * ldm + idx] = Ct[idx];
        }
        for (int idx = tid; idx < r * r; idx += NT) {
            const int ii = idx / r, k = idx - ii * r;
            Pg[(size_t)ii * rmax + k] = P[(size_t)ii * rmax + k];
        }
        for (int k = tid; k < r; k += NT) wg[k] = w[k];
    }
    if (tid == 0) {
        M->r = r;
        M->flags = flags;
        M->rows_seen += applied;
    }
    // Keep a barrier between these thread-0 stores and the thread-0 queue pop
    // at the top of the caller's loop: without it the compiler may merge the
    // two thread-0 regions across the loop back-edge, which gives the loop a
    // second entry at the barrier and lets the other threads loop without the
    // pop (the queue head then never advances).
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(NT) k_push_generic(PushArgs<T> a, int m_max, int r_max_max, int lds_state) {
    extern __shared__ double smem[];
    double *sG = smem;
    double *sGr = sG + m_max;
    double *sGam = sGr + m_max;
    double *sGam2 = sGam + r_max_max;
    double *sZ = sGam2 + r_max_max;
    double *sRed = sZ + r_max_max;
    double *sState = lds_state ? sRed + 2 * NW : nullptr;
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= a.n_order) break;
        const int b = a.order[idx];
        if (a.meta[b].cls < 0) run_stream<T>(a, b, sG, sGr, sGam, sGam2, sZ, sRed, sState);
    }
}

__global__ void k_reset_counter(uint32_t *c) {
    if (threadIdx.x < 64) c[threadIdx.x] = 0u;  // the 256-byte counter block
}

__global__ void k_reset_streams(StreamMeta *meta, int B) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        meta[b].r = 0;
        meta[b].flags = 0u;
        meta[b].rows_seen = 0;
    }
}

// dst[k] = sum_l H[k][l] v[l] for k < r (H symmetric r_max x r_max, row-major;
// thread k reads column k, so the reads of a wave coalesce).
__device__ inline void hmul(const double *H, int rmax, const double *v, double *dst, int r) {
    for (int k = threadIdx.x; k < r; k += NT) {
        double acc = 0.0;
        for (int l = 0; l < r; ++l) acc += H[(size_t)l * rmax + k] * v[l];
        dst[k] = acc;
    }
}

// The same for k_solution, whose sums take SU terms per step with their
// loads all in flight together (clamped indices past r, masked) and add
// them in l order: each step of the plain loop waited for its load.
constexpr int SU = 8;
__device__ inline void hmul_batched(const double *H, int rmax, const double *v, double *dst, int r) {
    for (int k = threadIdx.x; k < r; k += NT) {
        double acc = 0.0;
        for (int l0 = 0; l0 < r; l0 += SU) {
            double hv[SU], vv[SU];
#pragma unroll
            for (int e = 0; e < SU; ++e) {
                const int l = l0 + e < r ? l0 + e : r - 1;
                hv[e] = H[(size_t)l * rmax + k];
                vv[e] = v[l];
            }
#pragma unroll
            for (int e = 0; e < SU; ++e)
                if (l0 + e < r) acc += hv[e] * vv[e];
        }
        dst[k] = acc;
    }
}

// x_b = Ct_b^T w_b, FP64 sums, one workgroup per stream.  Factored-form
// streams (Ct = H^-1 C) first form u = H^-1 w, then x = C^T u.
template <typename T>
__global__ void __launch_bounds__(NT) k_solution(const StreamMeta *meta, const T *state, const double *hreg,
                                                 const double *wreg, T *x) {
    extern __shared__ double su[];
    const StreamMeta M = meta[blockIdx.x];
    const double *w = wreg + M.w_off;
    const T *B;
    if (M.h_off >= 0) {
        hmul_batched(hreg + M.h_off, M.r_max, w, su, M.r);
        __syncthreads();
        w = su;
        B = state + M.state_off;
    } else {
        B = state + M.state_off + (size_t)M.r_max * M.ldm;
    }
    for (int j = threadIdx.x; j < M.m; j += NT) {
        double acc = 0.0;
        for (int k0 = 0; k0 < M.r; k0 += SU) {
            double bv[SU], wv[SU];
#pragma unroll
            for (int e = 0; e < SU; ++e) {
                const int k = k0 + e < M.r ? k0 + e : M.r - 1;
                bv[e] = (double)B[(size_t)k * M.ldm + j];
                wv[e] = w[k];
            }
#pragma unroll
            for (int e = 0; e < SU; ++e)
                if (k0 + e < M.r) acc += bv[e] * wv[e];
        }
        x[M.x_off + j] = (T)acc;
    }
}

// Ct = H^-1 C of one factored-form stream, FP64 sums, rounded to T: thread
// (k, j-range) forms row k of Ct.
template <typename T>
__global__ void __launch_bounds__(NT) k_ctilde(const StreamMeta *meta, int b, const T *state, const double *hreg,
                                               T *dst, int r) {
    const StreamMeta M = meta[b];
    const T *C = state + M.state_off;
    const double *H = hreg + M.h_off;
    for (int64_t idx = blockIdx.x * (int64_t)NT + threadIdx.x; idx < (int64_t)r * M.m; idx += (int64_t)gridDim.x * NT) {
        const int k = (int)(idx / M.m), j = (int)(idx - (int64_t)k * M.m);
        double acc = 0.0;
        for (int l = 0; l < r; ++l) acc += H[(size_t)k * M.r_max + l] * (double)C[(size_t)l * M.ldm + j];
        dst[idx] = (T)acc;
    }
}

// Adjoint at constant rank, one workgroup per stream.  Preamble (O(r m)):
//   x = Ct^T w, u = Ct g, v = Ct x, s = Ct^T P^-1 u, t = Ct^T P^-1 v, p = g - C^T u;
// then one pass over the rows of A: a_i = A_i s, b_i = A_i t, rho_i = Y_i - A_i x,
//   dY_i = a_i, dA_i = -a_i x + rho_i s + b_i p.
// Factored-form streams (Ct = H^-1 C) apply Ct and Ct^T as H^-1 C and
// C^T H^-1, with the same algebra.
template <typename T>
__global__ void __launch_bounds__(NT) k_adjoint(const StreamMeta *meta, const T *state, const double *preg,
                                                const double *hreg, const double *wreg, const T *A, const T *Y,
                                                const int64_t *row_ptr, const int64_t *a_off, const T *g, T *dA,
                                                T *dY, int m_max, int r_max_max) {
    extern __shared__ double smem[];
    const int b = blockIdx.x;
    const StreamMeta M = meta[b];
    const int m = M.m, r = M.r, ldm = M.ldm, rmax = M.r_max;
    const bool fd = M.h_off >= 0;
    const T *C = state + M.state_off;
    const T *Ct = fd ? C : C + (size_t)rmax * ldm;  // factored form: the rows multiplied by H^-1
    const double *H = fd ? hreg + M.h_off : nullptr;
    const double *P = preg + M.p_off;
    const double *w = wreg + M.w_off;
    double *sx = smem, *sg = sx + m_max, *ss = sg + m_max, *st = ss + m_max, *sp = st + m_max;
    double *su = sp + m_max, *sv = su + r_max_max, *su2 = sv + r_max_max, *sv2 = su2 + r_max_max;
    double *sh = sv2 + r_max_max, *sh2 = sh + r_max_max;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (fd) {
        hmul_batched(H, rmax, w, sh, r);  // x = C^T (H^-1 w)
        __syncthreads();
    }
    const double *wx = fd ? sh : w;
    // (the sums over k below take SU terms per step with their loads in flight
    // together, in k order, as in k_solution)
    for (int j = tid; j < m; j += NT) {
        double acc = 0.0;
        for (int k0 = 0; k0 < r; k0 += SU) {
            double cv[SU];
#pragma unroll
            for (int e = 0; e < SU; ++e) cv[e] = (double)Ct[(size_t)(k0 + e < r ? k0 + e : r - 1) * ldm + j];
#pragma unroll
            for (int e = 0; e < SU; ++e)
                if (k0 + e < r) acc += cv[e] * wx[k0 + e];
        }
        sx[j] = acc;
        sg[j] = (double)g[M.x_off + j];
    }
    __syncthreads();
    project<T, double>(Ct, ldm, sg, fd ? sh : su, r, m);
    project<T, double>(Ct, ldm, sx, fd ? sh2 : sv, r, m);
    __syncthreads();
    if (fd) {
        hmul_batched(H, rmax, sh, su, r);
        hmul_batched(H, rmax, sh2, sv, r);
        __syncthreads();
    }
    for (int i = tid; i < r; i += NT) {
        double a1 = 0.0, a2 = 0.0;
        for (int k0 = 0; k0 < r; k0 += SU) {
            double pv[SU];
#pragma unroll
            for (int e = 0; e < SU; ++e) pv[e] = P[(size_t)(k0 + e < r ? k0 + e : r - 1) * rmax + i];
#pragma unroll
            for (int e = 0; e < SU; ++e)
                if (k0 + e < r) {
                    a1 += pv[e] * su[k0 + e];
                    a2 += pv[e] * sv[k0 + e];
                }
        }
        su2[i] = a1;
        sv2[i] = a2;
    }
    __syncthreads();
    if (fd) {
        hmul_batched(H, rmax, su2, sh, r);
        hmul_batched(H, rmax, sv2, sh2, r);
        __syncthreads();
        su2 = sh;
        sv2 = sh2;
    }
    for (int j = tid; j < m; j += NT) {
        double a1 = 0.0, a2 = 0.0, a3 = sg[j];
        for (int k0 = 0; k0 < r; k0 += SU) {
            double ctv[SU], cv[SU];
#pragma unroll
            for (int e = 0; e < SU; ++e) {
                const size_t k = (size_t)(k0 + e < r ? k0 + e : r - 1);
                ctv[e] = (double)Ct[k * ldm + j];
                cv[e] = (double)C[k * ldm + j];
            }
#pragma unroll
            for (int e = 0; e < SU; ++e)
                if (k0 + e < r) {
                    a1 += ctv[e] * su2[k0 + e];
                    a2 += ctv[e] * sv2[k0 + e];
                    a3 -= cv[e] * su[k0 + e];
                }
        }
        ss[j] = a1;
        st[j] = a2;
        sp[j] = a3;
    }
    __syncthreads();
    const int64_t i0 = row_ptr[b], i1 = row_ptr[b + 1];
    const T *Ab = A + a_off[b];
    T *dAb = dA + a_off[b];
    // 16 lanes per row, four rows per wave at a time, so that many rows' loads
    // are in flight; the row sums are 16-lane DPP reductions
    const int q = lane & 15, grp = lane >> 4;
    for (int64_t ib = i0 + 4 * wid; ib < i1; ib += 4 * NW) {  // wave-uniform
        const int64_t i = ib + grp;
        const bool ok = i < i1;
        const T *row = Ab + (i - i0) * (int64_t)m;
        double ca = 0.0, cb = 0.0, cx = 0.0;
        if (ok) {
#pragma unroll 8
            for (int j = q; j < m; j += 16) {
                const double v = (double)row[j];
                ca += v * ss[j];
                cb += v * st[j];
                cx += v * sx[j];
            }
        }
        ca = sum16(ca);
        cb = sum16(cb);
        cx = sum16(cx);
        if (ok) {
            const double rho = (double)Y[i] - cx;
            T *drow = dAb + (i - i0) * (int64_t)m;
#pragma unroll 8
            for (int j = q; j < m; j += 16) drow[j] = (T)(-ca * sx[j] + rho * ss[j] + cb * sp[j]);
            if (q == 0) dY[i] = (T)ca;
        }
    }
}

// Pseudoinverse of stream b from its factorisation (Theorem 1:
// A^+ = Ct^T P^-1 B^T with B = A Ct^T), one row of A at a time: column i of
// A^+ is Ct^T P^-1 (Ct A_i^T).  FP64 sums; A^+ is m x n row-major.
template <typename T>
__global__ void __launch_bounds__(NT) k_pinv(const StreamMeta *meta, const T *state, const double *preg,
                                             const double *hreg, const T *A, const int64_t *row_ptr,
                                             const int64_t *a_off, T *Ap, int m_max, int r_max_max) {
    extern __shared__ double smem[];
    const int b = blockIdx.x;
    const StreamMeta M = meta[b];
    const int m = M.m, r = M.r, ldm = M.ldm, rmax = M.r_max;
    const bool fd = M.h_off >= 0;  // factored form: Ct = H^-1 C
    const T *Ct = state + M.state_off + (fd ? 0 : (size_t)rmax * ldm);
    const double *H = fd ? hreg + M.h_off : nullptr;
    const double *P = preg + M.p_off;
    double *sa = smem, *sb = sa + m_max, *sq = sb + r_max_max, *st = sq + r_max_max;
    const int64_t i0 = row_ptr[b], i1 = row_ptr[b + 1], n = i1 - i0;
    const T *Ab = A + a_off[b];
    T *Apb = Ap + a_off[b];
    const int tid = threadIdx.x;
    for (int64_t i = 0; i < n; ++i) {
        for (int j = tid; j < m; j += NT) sa[j] = (double)Ab[i * m + j];
        __syncthreads();
        project<T, double>(Ct, ldm, sa, fd ? st : sb, r, m);  // b = Ct A_i^T
        __syncthreads();
        if (fd) {
            hmul(H, rmax, st, sb, r);
            __syncthreads();
        }
        for (int a2 = tid; a2 < r; a2 += NT) {       // q = P^-1 b (symmetric: column reads coalesce)
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc += P[(size_t)k * rmax + a2] * sb[k];
            sq[a2] = acc;
        }
        __syncthreads();
        const double *q = sq;
        if (fd) {
            hmul(H, rmax, sq, st, r);
            __syncthreads();
            q = st;
        }
        for (int j = tid; j < m; j += NT) {
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc += (double)Ct[(size_t)k * ldm + j] * q[k];
            Apb[(int64_t)j * n + i] = (T)acc;
        }
        __syncthreads();
    }
}

}  // namespace

template <typename T>
hipError_t launch_pinv(const StreamMeta *meta, int B, const T *state, const double *preg, const double *hreg,
                       const T *A, const int64_t *row_ptr, const int64_t *a_off, T *Ap, int m_max, int r_max_max,
                       hipStream_t s) {
    const size_t lds = sizeof(double) * ((size_t)m_max + 3 * (size_t)r_max_max);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pinv<T>, dim3(B), dim3(NT), lds, s, meta, state, preg, hreg, A, row_ptr, a_off, Ap, m_max,
                       r_max_max);
    return hipGetLastError();
}
template hipError_t launch_pinv<float>(const StreamMeta *, int, const float *, const double *, const double *,
                                       const float *, const int64_t *, const int64_t *, float *, int, int,
                                       hipStream_t);
template hipError_t launch_pinv<double>(const StreamMeta *, int, const double *, const double *, const double *,
                                        const double *, const int64_t *, const int64_t *, double *, int, int,
                                        hipStream_t);

template <typename T>
hipError_t launch_ctilde(const StreamMeta *meta, int b, const T *state, const double *hreg, T *dst, int r,
                         hipStream_t s) {
    if (r <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ctilde<T>, dim3(64), dim3(NT), 0, s, meta, b, state, hreg, dst, r);
    return hipGetLastError();
}
template hipError_t launch_ctilde<float>(const StreamMeta *, int, const float *, const double *, float *, int,
                                         hipStream_t);
template hipError_t launch_ctilde<double>(const StreamMeta *, int, const double *, const double *, double *, int,
                                          hipStream_t);

template <typename T>
size_t generic_lds_bytes(int m_max, int r_max_max, bool lds_state) {
    const size_t base = sizeof(double) * (2 * (size_t)m_max + 3 * (size_t)r_max_max + 2 * NW);
    const int ldm_max = (int)((m_max + 16 / sizeof(T) - 1) / (16 / sizeof(T)) * (16 / sizeof(T)));
    return base + (lds_state ? lds_state_bytes<T>(r_max_max, ldm_max) : 0);
}

template <typename T>
bool generic_state_in_lds(int m_max, int r_max_max) {
    return generic_lds_bytes<T>(m_max, r_max_max, true) <= 64 * 1024;
}

template <typename T>
hipError_t launch_push_generic(const PushArgs<T> &a, int grid, int m_max, int r_max_max, hipStream_t s) {
    const bool in_lds = generic_state_in_lds<T>(m_max, r_max_max);
    const size_t lds = generic_lds_bytes<T>(m_max, r_max_max, in_lds);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_push_generic<T>, dim3(grid), dim3(NT), lds, s, a, m_max, r_max_max, in_lds ? 1 : 0);
    return hipGetLastError();
}
template size_t generic_lds_bytes<float>(int, int, bool);
template size_t generic_lds_bytes<double>(int, int, bool);
template bool generic_state_in_lds<float>(int, int);
template bool generic_state_in_lds<double>(int, int);

hipError_t launch_reset_counter(uint32_t *counter, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_reset_streams(StreamMeta *meta, int B, hipStream_t s) {
    const int grid = (B + 255) / 256;
    hipLaunchKernelGGL(k_reset_streams, dim3(grid), dim3(256), 0, s, meta, B);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_solution(const StreamMeta *meta, int B, const T *state, const double *hreg, const double *wreg,
                           T *x, int r_max_max, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)r_max_max;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_solution<T>, dim3(B), dim3(NT), lds, s, meta, state, hreg, wreg, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint(const StreamMeta *meta, int B, const T *state, const double *preg, const double *hreg,
                          const double *wreg, const T *A, const T *Y, const int64_t *row_ptr, const int64_t *a_off,
                          const T *g, T *dA, T *dY, int m_max, int r_max_max, hipStream_t s) {
    const size_t lds = sizeof(double) * (5 * (size_t)m_max + 6 * (size_t)r_max_max);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adjoint<T>, dim3(B), dim3(NT), lds, s, meta, state, preg, hreg, wreg, A, Y, row_ptr, a_off,
                       g, dA, dY, m_max, r_max_max);
    return hipGetLastError();
}

template hipError_t launch_push_generic<float>(const PushArgs<float> &, int, int, int, hipStream_t);
template hipError_t launch_push_generic<double>(const PushArgs<double> &, int, int, int, hipStream_t);
template hipError_t launch_solution<float>(const StreamMeta *, int, const float *, const double *, const double *,
                                           float *, int, hipStream_t);
template hipError_t launch_solution<double>(const StreamMeta *, int, const double *, const double *,
                                            const double *, double *, int, hipStream_t);
template hipError_t launch_adjoint<float>(const StreamMeta *, int, const float *, const double *, const double *,
                                          const double *, const float *, const float *, const int64_t *,
                                          const int64_t *, const float *, float *, float *, int, int, hipStream_t);
template hipError_t launch_adjoint<double>(const StreamMeta *, int, const double *, const double *,
                                           const double *, const double *, const double *, const double *,
                                           const int64_t *, const int64_t *, const double *, double *, double *, int,
                                           int, hipStream_t);

}  // namespace rg
