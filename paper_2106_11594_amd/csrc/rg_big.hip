// One large stream (m >= BIG_M_MIN, not held on chip) spread over the whole
// GPU.  Each row of Algorithm 1 is a short chain of grid-wide kernels on the
// handle's stream, with every intermediate in a small device scratch area, so
// the host never waits on the device:
//   proj   gamma = Ct Gamma            one wave per row of Ct (DPP sums)
//   rej    Gamma_r = Gamma - C^T gamma 64 columns per workgroup, the rank r
//                                      split over its 4 waves; partial norms;
//                                      in pass 1 also partial zeta = P^-1 gamma
//                                      over a slice of the rows of P^-1
//   proj   pass 2: workgroup 0 takes the decision (rank test of Section 3
//          on the summed partials; for a dependent row zeta = P^-1 gamma,
//          d = 1 + gamma^T zeta and the step (y - gamma^T w) / d, Theorems 5
//          and 6); for an independent row every workgroup projects Gamma_r
//   rej    pass 2 for an independent row ("twice is enough")
//   apply  dependent: P^-1 -= zeta zeta^T / d, w += zeta (y - gamma^T w) / d;
//          independent: Ct <- [Ct - gamma K^T; K^T], C <- [C; Gamma],
//          P^-1 <- diag(P^-1, 1), w <- [w; y] (Theorems 4, 6)
// The rank is double-buffered by row parity: the kernels of row i read slot
// i & 1, and apply writes slot (i + 1) & 1, so no kernel reads a value that a
// workgroup of the same launch may still change.  Decisions, norms and
// partial sums are reduced in a fixed order: results do not depend on
// scheduling.
#include "rg_internal.h"
#include "rg_lanes.h"

#include <algorithm>

namespace rg {
namespace {

constexpr int BT = 256;  // threads per workgroup
constexpr int MODE_NONE = 0, MODE_DEP = 1, MODE_IND = 2;

struct BigArgs {
    StreamMeta *meta;
    double *sc;      // scalars: [0] mode, [1] s (pass 1), [2] g2, [3] inv_d, [4] step, [5] y, [6] reprojected
    int32_t *rs;     // rs[0], rs[1]: rank by row parity; rs[2]: rows applied in this push
    double *gr;      // Gamma_r (m)
    double *gam;     // gamma (r_max)
    double *gam2;    // second-pass gamma (r_max)
    double *zeta;    // P^-1 gamma (r_max)
    double *part;    // partial sums: [NP][4] pass 1, then [NP][4] pass 2
    double *zpart;   // partial P^-1 gamma: [NP][r_max], workgroup q over its slice of the rows of P^-1
    int np;          // workgroups of rej (64 columns each)
};

template <typename T>
struct BigState {
    T *C, *Ct;
    double *P, *w;
    int m, rmax, ldm;
};

template <typename T>
__device__ inline BigState<T> big_state(const PushArgs<T> &a) {
    const StreamMeta &M = a.meta[0];
    BigState<T> s;
    s.C = a.state + M.state_off;
    s.Ct = s.C + (size_t)M.r_max * M.ldm;
    s.P = a.preg + M.p_off;
    s.w = a.wreg + M.w_off;
    s.m = M.m;
    s.rmax = M.r_max;
    s.ldm = M.ldm;
    return s;
}

__global__ void k_big_begin(StreamMeta *meta, int32_t *rs) {
    if (threadIdx.x == 0) {
        rs[0] = meta->r;
        rs[2] = 0;
    }
}

__global__ void k_big_end(StreamMeta *meta, const int32_t *rs, int parity) {
    if (threadIdx.x == 0) {
        meta->r = rs[parity];
        meta->rows_seen += rs[2];
    }
}

// Whether row i is independent and takes the second projection, from the
// pass-1 partial sums (every workgroup gets the same answer).
template <typename T>
__device__ inline bool second_pass(const PushArgs<T> &a, const BigArgs &b, int m, int rmax, int r, int64_t i) {
    double sr = 0.0, sg = 0.0, sb = 0.0;
    for (int q = 0; q < b.np; ++q) {  // fixed order
        sr += b.part[4 * q];
        sg += b.part[4 * q + 1];
        sb += b.part[4 * q + 2];
    }
    const double yv = (double)a.y[i];
    if (sb != 0.0 || !isfinite(sg) || !isfinite(yv)) return false;
    const double eps = a.eps >= 0.0 ? a.eps : ((double)m * m * r + (double)m * r + (double)m) * 0x1p-52;
    const double nr = sqrt(sr), ng = sqrt(sg);
    const bool dependent = (sr == 0.0) || (nr < eps) || (nr < eps * ng);
    return !dependent && r < rmax && r > 0 && !(a.opts & OPT_NO_REPROJECT);
}

// Rank test and the dependent-row scalars (one workgroup: workgroup 0 of the
// second-pass projection launch).  Writes the decision read by apply.
template <typename T>
__device__ void big_decide(const PushArgs<T> &a, const BigArgs &b, int64_t i, double *sred) {
    const BigState<T> s = big_state(a);
    StreamMeta *M = a.meta;
    const int r = b.rs[i & 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double sr = 0.0, sg = 0.0, sb = 0.0;
    for (int q = 0; q < b.np; ++q) {  // fixed order (the same sums as second_pass)
        sr += b.part[4 * q];
        sg += b.part[4 * q + 1];
        sb += b.part[4 * q + 2];
    }
    const double yv = (double)a.y[i];
    uint32_t flag = 0u;
    int mode = MODE_NONE;
    double inv_d = 0.0, step = 0.0;
    if (sb != 0.0 || !isfinite(sg) || !isfinite(yv)) {
        flag = FLAG_NONFINITE;
    } else {
        const double eps = a.eps >= 0.0 ? a.eps : ((double)s.m * s.m * r + (double)s.m * r + (double)s.m) * 0x1p-52;
        const double nr = sqrt(sr), ng = sqrt(sg);
        const bool dependent = (sr == 0.0) || (nr < eps) || (nr < eps * ng);
        if (!dependent) {
            if (r == s.rmax) flag = FLAG_RANK_CAPACITY;
            else mode = MODE_IND;
        } else if (r > 0) {
            // zeta = P^-1 gamma from the partials of rej, summed in a fixed order
            for (int ii = tid; ii < r; ii += BT) {
                double acc = 0.0;
                for (int q = 0; q < b.np; ++q) acc += b.zpart[(size_t)q * s.rmax + ii];
                b.zeta[ii] = acc;
            }
            __syncthreads();
            double gz = 0.0, gw = 0.0;
            for (int k = tid; k < r; k += BT) {
                gz += b.gam[k] * b.zeta[k];
                gw += b.gam[k] * s.w[k];
            }
            gz = sum64(gz);
            gw = sum64(gw);
            if (lane == 0) {
                sred[2 * wid] = gz;
                sred[2 * wid + 1] = gw;
            }
            __syncthreads();
            gz = gw = 0.0;
#pragma unroll
            for (int q = 0; q < BT / 64; ++q) {
                gz += sred[2 * q];
                gw += sred[2 * q + 1];
            }
            const double d = 1.0 + gz;
            if (!(d > 0.0) || !isfinite(d)) {
                flag = FLAG_DENOMINATOR;
            } else {
                mode = MODE_DEP;
                inv_d = 1.0 / d;
                step = (yv - gw) * inv_d;
            }
        }
    }
    if (tid == 0) {
        b.sc[0] = mode;
        b.sc[1] = sr;
        b.sc[2] = sg;
        b.sc[3] = inv_d;
        b.sc[4] = step;
        b.sc[5] = yv;
        b.sc[6] = (mode == MODE_IND && r > 0 && !(a.opts & OPT_NO_REPROJECT)) ? 1.0 : 0.0;
        if (flag) M->flags = flag;
        else b.rs[2] += 1;  // the row is applied (a dependent row at rank 0 is a no-op)
    }
}

// dst[k] = sum_j Ct[k][j] v[j] for k < r; v is row i of the input (pass 1)
// or Gamma_r (pass 2, only for an independent row with r > 0).  In pass 2
// workgroup 0 first takes the decision of the row.
template <typename T>
__global__ void __launch_bounds__(BT) k_big_proj(PushArgs<T> a, BigArgs b, int64_t i, int pass) {
    __shared__ double sred[2 * (BT / 64)];
    const BigState<T> s = big_state(a);
    const int r = b.rs[i & 1];
    if (a.meta->flags != 0u) {
        if (pass == 2 && blockIdx.x == 0 && threadIdx.x == 0) b.sc[0] = MODE_NONE;
        return;
    }
    if (pass == 2) {
        // the flags are re-read after this point by no workgroup of this launch
        const bool two = second_pass(a, b, s.m, s.rmax, r, i);
        if (blockIdx.x == 0) big_decide(a, b, i, sred);
        if (!two) return;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const T *g = a.gamma + i * (int64_t)s.m;
    double *dst = pass == 1 ? b.gam : b.gam2;
    for (int k = blockIdx.x * (BT / 64) + wid; k < r; k += gridDim.x * (BT / 64)) {
        const T *row = s.Ct + (size_t)k * s.ldm;
        double acc = 0.0;
        if (pass == 1) {
            for (int j = lane; j < s.m; j += 64) acc += (double)row[j] * (double)g[j];
        } else {
            for (int j = lane; j < s.m; j += 64) acc += (double)row[j] * b.gr[j];
        }
        acc = sum64(acc);
        if (lane == 0) dst[k] = acc;
    }
}

// Gamma_r[j] = v[j] - sum_{k<r} C[k][j] g[k] for the 64 columns of this
// workgroup (the k range split over the 4 waves); partial sums of Gamma_r^2
// (and, in pass 1, of Gamma^2 and of non-finite entries) per workgroup.
template <typename T>
__global__ void __launch_bounds__(BT) k_big_rej(PushArgs<T> a, BigArgs b, int64_t i, int pass) {
    __shared__ double red[BT / 64][64];
    const BigState<T> s = big_state(a);
    const int r = b.rs[i & 1];
    if (a.meta->flags != 0u) return;
    if (pass == 2 && !second_pass(a, b, s.m, s.rmax, r, i)) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane;
    const double *g = pass == 1 ? b.gam : b.gam2;
    double acc = 0.0;
    if (col < s.m) {
#pragma unroll 8
        for (int k = wid; k < r; k += BT / 64) acc += (double)s.C[(size_t)k * s.ldm + col] * g[k];
    }
    red[wid][lane] = acc;
    __syncthreads();
    double sr = 0.0, sg = 0.0, sb = 0.0;
    if (wid == 0) {
        if (col < s.m) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < BT / 64; ++q) t += red[q][lane];
            double v;
            if (pass == 1) {
                v = (double)a.gamma[i * (int64_t)s.m + col];
                sg = v * v;
                sb = isfinite(v) ? 0.0 : 1.0;
            } else {
                v = b.gr[col];
            }
            const double rv = v - t;
            b.gr[col] = rv;
            sr = rv * rv;
        }
        sr = sum64(sr);
        sg = sum64(sg);
        sb = sum64(sb);
        if (lane == 0) {
            double *pp = b.part + (size_t)(pass == 1 ? 0 : b.np) * 4 + (size_t)blockIdx.x * 4;
            pp[0] = sr;
            pp[1] = sg;
            pp[2] = sb;
        }
    }
    if (pass == 1) {
        // partial zeta[ii] = sum over this workgroup's rows k of P^-1[k][ii] gamma_k
        // (P^-1 is symmetric; row reads coalesce); used if the row is dependent
        const int per = (r + b.np - 1) / b.np, k0 = blockIdx.x * per, k1 = min(r, k0 + per);
        for (int ii = threadIdx.x; ii < r; ii += BT) {
            double z = 0.0;
            for (int k = k0; k < k1; ++k) z += s.P[(size_t)k * s.rmax + ii] * b.gam[k];
            b.zpart[(size_t)blockIdx.x * s.rmax + ii] = z;
        }
    }
}

// The update of the chosen branch, grid-stride over its elements; writes the
// rank of the next row.
template <typename T>
__global__ void __launch_bounds__(BT) k_big_apply(PushArgs<T> a, BigArgs b, int64_t i) {
    const BigState<T> s = big_state(a);
    const int r = b.rs[i & 1];
    const int mode = (int)b.sc[0];
    const int64_t gtid = (int64_t)blockIdx.x * BT + threadIdx.x, gsz = (int64_t)gridDim.x * BT;
    if (gtid == 0) b.rs[(i + 1) & 1] = r + (mode == MODE_IND ? 1 : 0);
    if (mode == MODE_DEP) {
        const double inv_d = b.sc[3], step = b.sc[4];
        const int64_t rr = (int64_t)r * r;
        for (int64_t e = gtid; e < rr; e += gsz) {
            const int ii = (int)(e / r), k = (int)(e - (int64_t)ii * r);
            s.P[(size_t)ii * s.rmax + k] -= (b.zeta[ii] * b.zeta[k]) * inv_d;
        }
        for (int64_t k = gtid; k < r; k += gsz) s.w[k] += b.zeta[k] * step;
    } else if (mode == MODE_IND) {
        double sr = b.sc[1];
        const bool two = b.sc[6] != 0.0;
        if (two) {
            sr = 0.0;
            for (int q = 0; q < b.np; ++q) sr += b.part[(size_t)(b.np + q) * 4];
        }
        const double inv_s = 1.0 / sr;
        const int64_t rm = (int64_t)r * s.m;
        for (int64_t e = gtid; e < rm; e += gsz) {
            const int k = (int)(e / s.m), j = (int)(e - (int64_t)k * s.m);
            const double gk = two ? b.gam[k] + b.gam2[k] : b.gam[k];
            const double K = b.gr[j] * inv_s;
            if constexpr (sizeof(T) == 4) {
                float &c = s.Ct[(size_t)k * s.ldm + j];
                c = fmaf(-(float)gk, (float)K, c);
            } else {
                double &c = s.Ct[(size_t)k * s.ldm + j];
                c = fma(-gk, K, c);
            }
        }
        for (int64_t j = gtid; j < s.m; j += gsz) {
            s.Ct[(size_t)r * s.ldm + j] = (T)(b.gr[j] * inv_s);
            s.C[(size_t)r * s.ldm + j] = a.gamma[i * (int64_t)s.m + j];
        }
        for (int64_t k = gtid; k < r; k += gsz) {
            s.P[(size_t)r * s.rmax + k] = 0.0;
            s.P[(size_t)k * s.rmax + r] = 0.0;
        }
        if (gtid == 0) {
            s.P[(size_t)r * s.rmax + r] = 1.0;
            s.w[r] = b.sc[5];
        }
    }
}

}  // namespace

size_t big_scratch_doubles(int m, int rmax) {
    const int np = (m + 63) / 64;
    return 16 + 2 + (size_t)m + 3 * (size_t)rmax + 8 * (size_t)np + (size_t)np * rmax;
}

template <typename T>
hipError_t launch_push_big(const PushArgs<T> &a, double *scratch, int m, int rmax, int num_cus, hipStream_t st) {
    BigArgs b;
    b.meta = a.meta;
    b.sc = scratch;
    b.rs = reinterpret_cast<int32_t *>(scratch + 16);
    b.gr = scratch + 18;
    b.gam = b.gr + m;
    b.gam2 = b.gam + rmax;
    b.zeta = b.gam2 + rmax;
    b.np = (m + 63) / 64;
    b.part = b.zeta + rmax;
    b.zpart = b.part + 8 * (size_t)b.np;
    const int gproj = std::min((rmax + BT / 64 - 1) / (BT / 64), num_cus);
    const int gapply = 4 * num_cus;
    hipLaunchKernelGGL(k_big_begin, dim3(1), dim3(64), 0, st, a.meta, b.rs);
    for (int64_t i = 0; i < a.k_single; ++i) {
        hipLaunchKernelGGL(k_big_proj<T>, dim3(gproj), dim3(BT), 0, st, a, b, i, 1);
        hipLaunchKernelGGL(k_big_rej<T>, dim3(b.np), dim3(BT), 0, st, a, b, i, 1);
        hipLaunchKernelGGL(k_big_proj<T>, dim3(gproj), dim3(BT), 0, st, a, b, i, 2);
        hipLaunchKernelGGL(k_big_rej<T>, dim3(b.np), dim3(BT), 0, st, a, b, i, 2);
        hipLaunchKernelGGL(k_big_apply<T>, dim3(gapply), dim3(BT), 0, st, a, b, i);
    }
    hipLaunchKernelGGL(k_big_end, dim3(1), dim3(64), 0, st, a.meta, b.rs, (int)(a.k_single & 1));
    return hipGetLastError();
}

template hipError_t launch_push_big<float>(const PushArgs<float> &, double *, int, int, int, hipStream_t);
template hipError_t launch_push_big<double>(const PushArgs<double> &, double *, int, int, int, hipStream_t);

}  // namespace rg
