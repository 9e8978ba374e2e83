// Internal declarations shared by the host API (rg_api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace rg {

// One record per stream, resident in device memory.
struct StreamMeta {
    int32_t m;          // regressors
    int32_t r_max;      // rank capacity (rows reserved for C and Ct)
    int32_t ldm;        // leading dimension of C and Ct rows (elements)
    int32_t r;          // current rank
    uint32_t flags;     // sticky RG_FLAG_* bits
    int32_t cls;        // kernel size class chosen at init (-1: generic kernel)
    int64_t state_off;  // element offset of C in the state region; Ct follows at +r_max*ldm
    int64_t p_off;      // offset of P^-1 (doubles, r_max x r_max, row-major) in the P region
    int64_t w_off;      // offset of w (doubles) in the w region
    int64_t x_off;      // offset of x in packed solution vectors
    int64_t rows_seen;  // rows applied since the last reset
    int64_t h_off;      // offset of H^-1 = (C C^T)^-1 (doubles, r_max x r_max) in the H region, or -1:
                        // streams with H^-1 keep the dual basis in factored form, Ct = H^-1 C, and
                        // their Ct rows in the state are not maintained
};

constexpr uint32_t FLAG_NONFINITE = 0x1u;
constexpr uint32_t FLAG_RANK_CAPACITY = 0x2u;
constexpr uint32_t FLAG_DENOMINATOR = 0x4u;
constexpr uint32_t OPT_NO_REPROJECT = 0x1u;
constexpr uint32_t OPT_ROW_BY_ROW = 0x8u;
constexpr uint32_t OPT_DEPENDENT_BLOCKS_ONLY = 0x10u;
constexpr uint32_t OPT_ORTHOGONAL = 0x20u;
constexpr uint32_t OPT_ORTHONORMAL = 0x40u;
constexpr uint32_t OPT_ONE_WG_PER_STREAM = 0x80u;
constexpr uint32_t OPT_EXPLICIT_REJECTIONS = 0x100u;

// Arguments of a push launch (by value).
template <typename T>
struct PushArgs {
    StreamMeta *meta;
    const int32_t *order;    // processing order (stream ids), length n_order
    int32_t n_order;
    uint32_t *counter;       // work-queue head, zeroed before the launch
    T *state;
    double *preg;            // P^-1 blocks (FP64 for both state types)
    double *hreg;            // H^-1 blocks of factored-form streams (FP64)
    double *wreg;
    const T *gamma;
    const T *y;
    const int64_t *row_ptr;  // nullable: single stream with k_single rows
    const int64_t *gamma_off;
    int64_t k_single;
    double eps;              // < 0: default of Section 3 at the current rank
    uint32_t opts;
    int32_t persistent;      // on-chip classes: persistent grid taking streams from the queue head
};

// Host-side launchers (defined in the kernel sources).
template <typename T>
hipError_t launch_push_generic(const PushArgs<T> &a, int grid, int m_max, int r_max_max, hipStream_t s);
// Dynamic LDS of the generic kernel, and whether it keeps each stream's state
// in LDS during a push (when that fits in 64 KiB per workgroup).
template <typename T>
size_t generic_lds_bytes(int m_max, int r_max_max, bool lds_state);
template <typename T>
bool generic_state_in_lds(int m_max, int r_max_max);
hipError_t launch_reset_counter(uint32_t *counter, hipStream_t s);
// LDS read-bandwidth probe (rg_probe.hip): blocks x 256 threads, each thread
// reads LDS_PROBE_BYTES_PER_THREAD_ITER bytes per iteration.
constexpr int LDS_PROBE_THREADS = 256;
constexpr int LDS_PROBE_BYTES_PER_THREAD_ITER = 8 * 16;
hipError_t launch_lds_probe(float *out, int blocks, int iters, hipStream_t s);
hipError_t launch_reset_streams(StreamMeta *meta, int B, hipStream_t s);
// One stream over the whole GPU (rg_big.hip): the stream of a single-stream
// handle that no on-chip class holds.  It keeps the dual basis in factored
// form (H^-1).  gam and y point at the first of the n rows of the push; M is
// the host copy of the stream's record.
size_t big_scratch_doubles(int m, int rmax);
template <typename T>
hipError_t launch_push_big(const PushArgs<T> &a, const StreamMeta &M, double *scratch, const T *gam, const T *y,
                           int64_t n, int num_cus, hipStream_t s);
// x = C^T (H^-1 w) of that stream over the whole GPU (scratch: its area).
template <typename T>
hipError_t launch_solution_big(const StreamMeta *meta, const StreamMeta &M, const T *state, const double *hreg,
                               const double *wreg, double *scratch, T *x, hipStream_t s);
template <typename T>
hipError_t launch_pinv(const StreamMeta *meta, int B, const T *state, const double *preg, const double *hreg,
                       const T *A, const int64_t *row_ptr, const int64_t *a_off, T *Ap, int m_max, int r_max_max,
                       hipStream_t s);
template <typename T>
hipError_t launch_solution(const StreamMeta *meta, int B, const T *state, const double *hreg, const double *wreg,
                           T *x, int r_max_max, hipStream_t s);
template <typename T>
hipError_t launch_adjoint(const StreamMeta *meta, int B, const T *state, const double *preg, const double *hreg,
                          const double *wreg, const T *A, const T *Y, const int64_t *row_ptr, const int64_t *a_off,
                          const T *g, T *dA, T *dY, int m_max, int r_max_max, hipStream_t s);
// Ct = H^-1 C of stream b (factored-form streams), r x m row-major into dst.
template <typename T>
hipError_t launch_ctilde(const StreamMeta *meta, int b, const T *state, const double *hreg, T *dst, int r,
                         hipStream_t s);

}  // namespace rg
