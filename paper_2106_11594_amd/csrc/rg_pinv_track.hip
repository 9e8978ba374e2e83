// Pseudoinverse maintained row by row (Theorems 2 and 3), FP64, gfx950.
//
// One workgroup (4 wave64) owns one problem of a batch and walks its rows in
// order.  Per row Gamma (with target y), the update of Algorithm 1 plus the
// O(m n) pseudoinverse update:
//   gamma   = Ct Gamma, Gamma_r = Gamma - C^T gamma, rank test of Section 3
//   zeta    = P^-1 gamma and beta = B zeta, both with the state before the row
//   gain K  = Gamma_r / ||Gamma_r||^2            (independent, Theorem 2/4)
//           = Ct^T zeta / (1 + gamma^T zeta)     (dependent, Theorem 3/5)
//   A^+    <- [A^+ - K beta^T, K]                 (a new column per row)
//   x      <- x + K (y - Gamma^T x)
//   factors (Theorem 6): independent appends Gamma to C, K to Ct (after
//   Ct -= gamma K^T), borders P^-1 with 1 and B with the unit coordinate
//   e_{r+1}; dependent downdates P^-1 by zeta zeta^T / (1 + gamma^T zeta) and
//   appends gamma to B.
// B (n x r_max, stored transposed) is the coordinate factor of A = B C; it
// is needed only for beta, which is what makes the pseudoinverse update
// O(m n) per row.  beta lives in LDS when it fits.
//
// The A^+ update reads and writes m x (i+1) values per row i, so the kernel is
// bound by memory traffic to the L2 / HBM, not by arithmetic: per row it moves
// about 16 m (i+1) bytes of A^+ plus 8 (i + 3 m r) bytes of B, C and Ct.
#include "../../include/rg.h"
#include <hip/hip_runtime.h>

#include "rg_lanes.h"
#include <cfloat>
#include <cmath>
#include <mutex>

namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

// Sum over the 64 lanes of a wave (DPP and permlane steps, the same bits on
// every lane).
__device__ inline double wsum(double v) { return rg::sum64(v); }

// Sum a, b and c over the workgroup in a fixed order; every thread gets the
// same totals, so decisions taken on them are uniform.
__device__ inline void block_sum3(double &a, double &b, double &c, double *red) {
    a = wsum(a);
    b = wsum(b);
    c = wsum(c);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[3 * w] = a;
        red[3 * w + 1] = b;
        red[3 * w + 2] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        a += red[3 * i];
        b += red[3 * i + 1];
        c += red[3 * i + 2];
    }
}

inline size_t per_problem(int n, int m, int rmax) {
    return 2 * (size_t)rmax * m + (size_t)rmax * rmax + (size_t)n * rmax + (size_t)n;
}

__global__ void __launch_bounds__(NT) k_pinv_track(const double *A, const double *Y, int n, int m, int q, int rmax,
                                                   double eps_in, double *Ap, double *X, int32_t *rank,
                                                   uint32_t *flags, double *work, size_t per, bool beta_lds) {
    extern __shared__ double sm[];
    double *sG = sm, *sR = sG + m, *sK = sR + m, *sg = sK + m, *sz = sg + rmax, *sdy = sz + rmax, *red = sdy + q;
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double *C = work + (size_t)b * per;
    double *Ct = C + (size_t)rmax * m;
    double *P = Ct + (size_t)rmax * m;
    double *Bf = P + (size_t)rmax * rmax;  // B^T: column t of B (row t of A's coordinates) at stride n
    // beta in LDS after the other vectors when it fits there, else in the workspace
    double *beta = beta_lds ? red + 3 * NW : Bf + (size_t)n * rmax;
    const double *Ab = A + (size_t)b * n * m;
    const double *Yb = Y + (size_t)b * n * q;
    double *Apb = Ap + (size_t)b * m * n;
    double *Xb = X + (size_t)b * m * q;

    // Zero P^-1 and B: bordering then only writes the new diagonal / unit entry.
    for (size_t t = tid; t < (size_t)rmax * rmax; t += NT) P[t] = 0.0;
    for (size_t t = tid; t < (size_t)n * rmax; t += NT) Bf[t] = 0.0;
    for (int j = tid; j < m * q; j += NT) Xb[j] = 0.0;
    __syncthreads();

    int r = 0;
    uint32_t fl = 0;
    for (int i = 0; i < n; ++i) {
        const double *G = Ab + (size_t)i * m;
        const double *yi = Yb + (size_t)i * q;
        for (int j = tid; j < m; j += NT) sG[j] = G[j];
        __syncthreads();
        // gamma = Ct Gamma (tasks k < r) and the a priori residuals
        // dy_c = y_c - Gamma^T X[:, c] (tasks r + c): one wave per task, lanes over j.
        for (int task = wid; task < r + q; task += NW) {
            double acc = 0.0;
            if (task < r) {
                for (int j = lane; j < m; j += 64) acc += Ct[(size_t)task * m + j] * sG[j];
            } else {
                const int c = task - r;
                for (int j = lane; j < m; j += 64) acc += sG[j] * Xb[(size_t)j * q + c];
            }
            acc = wsum(acc);
            if (lane == 0) {
                if (task < r) sg[task] = acc;
                else sdy[task - r] = yi[task - r] - acc;
            }
        }
        __syncthreads();
        // Gamma_r = Gamma - C^T gamma, with ||Gamma_r||^2 and ||Gamma||^2.
        double s = 0.0, g2 = 0.0, unused = 0.0;
        for (int j = tid; j < m; j += NT) {
            const double gj = sG[j];
            double acc = gj;
            for (int k = 0; k < r; ++k) acc -= C[(size_t)k * m + j] * sg[k];
            sR[j] = acc;
            s += acc * acc;
            g2 += gj * gj;
        }
        block_sum3(s, g2, unused, red);
        bool finite_y = true;
        for (int c = 0; c < q; ++c) finite_y = finite_y && isfinite(sdy[c]);
        if (!isfinite(g2) || !finite_y) {
            fl |= RG_FLAG_NONFINITE;
            break;
        }
        // Rank test (Section 3): dependent iff ||Gamma_r|| < eps or < eps ||Gamma||;
        // an exactly zero rejection is dependent for every eps (eps = 0 is the
        // exact test Gamma_r == 0 of Algorithm 1).
        const double eps = eps_in < 0.0 ? ((double)m * m * r + (double)m * r + m) * DBL_EPSILON : eps_in;
        const double nr = sqrt(s), ng = sqrt(g2);
        const bool indep = !(s == 0.0 || nr < eps || nr < eps * ng);
        if (indep && r == rmax) {
            fl |= RG_FLAG_RANK_CAPACITY;
            break;
        }
        // zeta = P^-1 gamma (P^-1 symmetric: column reads coalesce).
        for (int a = tid; a < r; a += NT) {
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc += P[(size_t)k * rmax + a] * sg[k];
            sz[a] = acc;
        }
        __syncthreads();
        // beta = B zeta over the i rows so far (B stored transposed: the
        // threads of a wave read consecutive rows t).
        for (int t = tid; t < i; t += NT) {
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc += Bf[(size_t)k * n + t] * sz[k];
            beta[t] = acc;
        }
        double den = 1.0;
        if (!indep) {
            double gz = 0.0, u0 = 0.0, u1 = 0.0;
            for (int a = tid; a < r; a += NT) gz += sg[a] * sz[a];
            block_sum3(gz, u0, u1, red);
            den = 1.0 + gz;
            if (!(den > 0.0) || !isfinite(den)) {
                fl |= RG_FLAG_DENOMINATOR;
                break;
            }
        }
        for (int j = tid; j < m; j += NT) {
            double kj;
            if (indep) {
                kj = sR[j] / s;
            } else {
                double acc = 0.0;
                for (int k = 0; k < r; ++k) acc += Ct[(size_t)k * m + j] * sz[k];
                kj = acc / den;
            }
            sK[j] = kj;
        }
        __syncthreads();  // K and beta complete
        // A^+ <- [A^+ - K beta^T, K]: each wave takes four rows j at a time, lanes
        // over pairs of columns (16-byte accesses, the four rows' loads in flight
        // together).  Rows start 16-byte aligned when n is even and A^+ is; column
        // i of the pair that straddles it receives K_j from the same store.
        if ((n & 1) == 0 && (reinterpret_cast<uintptr_t>(Apb) & 15) == 0) {
            for (int j0 = wid; j0 < m; j0 += 4 * NW) {
                double kq[4];
                double *aq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int jq = j0 + u * NW;
                    kq[u] = jq < m ? sK[jq] : 0.0;
                    aq[u] = Apb + (size_t)(jq < m ? jq : j0) * n;
                }
                for (int c = 2 * lane; c < i; c += 128) {
                    // c + 1 <= i <= n - 1: the pair is inside the row (beta has n entries)
                    const double2 bt = make_double2(beta[c], beta[c + 1]);
                    double2 av[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) av[u] = *reinterpret_cast<const double2 *>(aq[u] + c);
                    const bool last = c + 1 == i;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        av[u].x -= kq[u] * bt.x;
                        av[u].y = last ? kq[u] : av[u].y - kq[u] * bt.y;
                        if (j0 + u * NW < m) *reinterpret_cast<double2 *>(aq[u] + c) = av[u];
                    }
                }
                if (lane == 0 && (i & 1) == 0) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (j0 + u * NW < m) aq[u][i] = kq[u];
                }
            }
        } else {
            for (int j = wid; j < m; j += NW) {
                const double kj = sK[j];
                double *arow = Apb + (size_t)j * n;
                for (int c = lane; c < i; c += 64) arow[c] -= kj * beta[c];
                if (lane == 0) arow[i] = kj;
            }
        }
        for (int t = tid; t < m * q; t += NT) Xb[t] += sK[t / q] * sdy[t % q];
        if (indep) {
            for (int k = wid; k < r; k += NW)
                for (int j = lane; j < m; j += 64) Ct[(size_t)k * m + j] -= sg[k] * sK[j];
            for (int j = tid; j < m; j += NT) {
                Ct[(size_t)r * m + j] = sK[j];
                C[(size_t)r * m + j] = sG[j];
            }
            if (tid == 0) {
                P[(size_t)r * rmax + r] = 1.0;
                Bf[(size_t)r * n + i] = 1.0;
            }
            r += 1;
        } else {
            for (int a = wid; a < r; a += NW)
                for (int k = lane; k < r; k += 64) P[(size_t)a * rmax + k] -= sz[a] * sz[k] / den;
            for (int k = tid; k < r; k += NT) Bf[(size_t)k * n + i] = sg[k];
        }
        __syncthreads();
    }
    if (tid == 0) {
        rank[b] = r;
        flags[b] = fl;
    }
}

size_t lds_bytes(int m, int rmax, int q) {
    return sizeof(double) * (3 * (size_t)m + 2 * (size_t)rmax + (size_t)q + 3 * NW);
}
// beta (n doubles) joins the LDS vectors while the total stays at 64 KiB, so
// that several workgroups still share a CU
bool beta_fits_lds(int n, int m, int rmax, int q) {
    return lds_bytes(m, rmax, q) + sizeof(double) * (size_t)n <= 64 * 1024;
}

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;

}  // namespace

// Scratch of rg_pinv_track_noalloc: a file-scope device array, so that entry
// point needs no allocation.  Every GPU the library runs on holds its own copy
// for the life of the process.  In host code the array's name is only a host
// stand-in; its device address, looked up once per device, is what kernels get.
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (nullptr on failure); must be
// called with device dev current.
void *scratch_address(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" size_t rg_pinv_track_workspace_bytes(int32_t B, int32_t n, int32_t m, int32_t r_max) {
    if (B < 1 || n < 0 || m < 1 || r_max < 1 || r_max > m) return 0;
    return sizeof(double) * (size_t)B * per_problem(n, m, r_max);
}

extern "C" rg_status rg_pinv_track_rhs(const double *A, const double *Y, int32_t B, int32_t n, int32_t m, int32_t q,
                                       int32_t r_max, double eps, double *Ap, double *X, int32_t *rank,
                                       uint32_t *flags, void *work, size_t work_bytes, void *stream) {
    if (B < 1 || n < 0 || m < 1 || q < 1 || r_max < 1 || r_max > m || std::isnan(eps)) return RG_E_INVALID;
    if (!X || !rank || !flags || !work) return RG_E_INVALID;
    if (n > 0 && (!A || !Y || !Ap)) return RG_E_INVALID;
    if (work_bytes < rg_pinv_track_workspace_bytes(B, n, m, r_max)) return RG_E_INVALID;
    const size_t lds0 = lds_bytes(m, r_max, q);
    if (lds0 > 160 * 1024) return RG_E_UNSUPPORTED;
    const bool beta_lds = beta_fits_lds(n, m, r_max, q);
    const size_t lds = lds0 + (beta_lds ? sizeof(double) * (size_t)n : 0);
    hipLaunchKernelGGL(k_pinv_track, dim3(B), dim3(NT), lds, (hipStream_t)stream, A, Y, n, m, q, r_max, eps, Ap, X,
                       rank, flags, (double *)work, per_problem(n, m, r_max), beta_lds);
    return hipGetLastError() == hipSuccess ? RG_OK : RG_E_DEVICE;
}

extern "C" rg_status rg_pinv_track(const double *A, const double *Y, int32_t B, int32_t n, int32_t m,
                                   int32_t r_max, double eps, double *Ap, double *X, int32_t *rank,
                                   uint32_t *flags, void *work, size_t work_bytes, void *stream) {
    return rg_pinv_track_rhs(A, Y, B, n, m, 1, r_max, eps, Ap, X, rank, flags, work, work_bytes, stream);
}

extern "C" size_t rg_pinv_track_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" rg_status rg_pinv_track_noalloc(const double *A, const double *Y, int32_t B, int32_t n, int32_t m,
                                           int32_t r_max, double eps, double *Ap, double *X, int32_t *rank,
                                           uint32_t *flags, void *stream) {
    if (B < 1 || n < 0 || m < 1 || r_max < 1 || r_max > m || std::isnan(eps)) return RG_E_INVALID;
    if (!X || !rank || !flags) return RG_E_INVALID;
    if (n > 0 && (!A || !Y || !Ap)) return RG_E_INVALID;
    const size_t need = rg_pinv_track_workspace_bytes(B, n, m, r_max);
    if (need > NOALLOC_SCRATCH_BYTES) return RG_E_UNSUPPORTED;
    if (lds_bytes(m, r_max, 1) > 160 * 1024) return RG_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RG_E_DEVICE;
    void *work = scratch_address(dev);
    if (!work) return RG_E_DEVICE;
    return rg_pinv_track(A, Y, B, n, m, r_max, eps, Ap, X, rank, flags, work, need, stream);
}
