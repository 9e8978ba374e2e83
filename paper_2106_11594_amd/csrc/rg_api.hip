// Host side of librg.so: argument checks, the device workspace, scheduling
// order and kernel launches.  See include/rg.h for the contract.
#include "../../include/rg.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "rg_internal.h"
#include "rg_classes.h"

using rg::StreamMeta;

struct rg_ctx {
    int B = 0;
    int dtype = RG_F32;
    size_t esize = 4;
    hipStream_t stream = nullptr;
    uint32_t opts = 0;
    double eps = -1.0;
    int device = 0;
    int num_cus = 0;
    void *ws = nullptr;          // one device allocation for everything below
    size_t ws_bytes = 0;
    bool own_ws = true;          // false: the caller provided ws (rg_batch_init_ws)
    uint32_t known_flags = 0;    // OR of the stream flags the last synchronising call read
    StreamMeta *d_meta = nullptr;
    int32_t *d_order = nullptr;  // B entries: generic-class streams first, then each size class
    uint32_t *d_counter = nullptr;  // one queue head per kernel family (RG_MAX_FAMILIES)
    void *d_state = nullptr;
    double *d_p = nullptr;
    double *d_h = nullptr;       // H^-1 of the factored-form streams
    double *d_w = nullptr;
    double *d_big = nullptr;     // scratch of the multi-CU single-stream path (null if unused)
    std::vector<StreamMeta> h_meta;
    std::vector<int64_t> cost;
    // per-family segments of d_order
    std::vector<int> fam_begin, fam_count, fam_rows;
    hipStream_t aux[RG_MAX_FAMILIES] = {};
    hipEvent_t fork = nullptr, join[RG_MAX_FAMILIES] = {};
    int m_max_generic = 0, rmax_max_generic = 0;
    int m_max_all = 0, rmax_max_all = 0;
};

namespace {

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return RG_E_DEVICE;  \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    std::vector<StreamMeta> meta;
    size_t state_elems = 0, p_elems = 0, h_elems = 0, w_elems = 0, x_elems = 0;
};

// Kernel class of a stream (-1: generic kernel), and whether that class keeps
// the dual basis in factored form (the blocked on-chip classes do).  FP64
// streams of batches stay in the generic kernel, whose explicit Ct holds its
// rank decisions for kappa(C) beyond the factored form's reach; the stream of
// a one-stream FP64 handle takes the FP64 class when it fits (it would
// otherwise run over the whole GPU, also in factored form).
int stream_class(int32_t B, int m, int r_max, int dtype, uint32_t opts) {
    const bool generic = (opts & (RG_OPT_GENERIC_KERNEL | RG_OPT_ORTHOGONAL | RG_OPT_ORTHONORMAL)) != 0;
    if (generic || (dtype == RG_F64 && B > 1)) return -1;
    return rg::choose_class(m, r_max, dtype);
}

// A handle of one stream that no on-chip class holds runs it over the whole
// GPU (the multi-workgroup blocked path, factored form), whatever its size.
bool big_stream(int32_t B, int cls, int m, uint32_t opts) {
    (void)m;
    return B == 1 && cls < 0 && !(opts & (RG_OPT_GENERIC_KERNEL | RG_OPT_ORTHOGONAL | RG_OPT_ORTHONORMAL));
}

Layout plan_layout(int32_t B, const int32_t *m, const int32_t *r_max, size_t esize, int dtype, uint32_t opts) {
    Layout L;
    L.meta.resize(B);
    const size_t quantum = 16 / esize;  // keep every block 16-byte aligned
    for (int b = 0; b < B; ++b) {
        StreamMeta &M = L.meta[b];
        M.m = m[b];
        M.r_max = (r_max && r_max[b] > 0) ? std::min(r_max[b], m[b]) : m[b];
        M.ldm = (int32_t)align_up((size_t)M.m, quantum);
        M.r = 0;
        M.flags = 0;
        M.cls = stream_class(B, M.m, M.r_max, dtype, opts);
        M.h_off = -1;
        if (rg::class_factored(M.cls) || big_stream(B, M.cls, M.m, opts)) {
            M.h_off = (int64_t)L.h_elems;
            L.h_elems += align_up((size_t)M.r_max * M.r_max, 2);
        }
        M.state_off = (int64_t)L.state_elems;
        L.state_elems += align_up(2 * (size_t)M.r_max * M.ldm, quantum);
        M.p_off = (int64_t)L.p_elems;
        L.p_elems += align_up((size_t)M.r_max * M.r_max, 2);
        M.w_off = (int64_t)L.w_elems;
        L.w_elems += align_up((size_t)M.r_max, 2);
        M.x_off = (int64_t)L.x_elems;
        L.x_elems += (size_t)M.m;
        M.rows_seen = 0;
    }
    return L;
}

size_t ws_size(const Layout &L, int B, size_t esize, size_t big_doubles) {
    size_t off = align_up(sizeof(StreamMeta) * (size_t)B, 256);
    off += align_up(sizeof(int32_t) * (size_t)B, 256);
    off += 256;  // counters
    off += align_up(L.state_elems * esize, 256);
    off += align_up(L.p_elems * sizeof(double), 256);
    off += align_up(L.h_elems * sizeof(double), 256);
    off += align_up(L.w_elems * sizeof(double), 256);
    off += align_up(big_doubles * sizeof(double), 256);
    return off;
}

// Assign kernel families and upload the processing order (longest first).
rg_status upload_order(rg_ctx *h) {
    const int B = h->B;
    const int nfam = RG_MAX_FAMILIES;
    std::vector<std::vector<int32_t>> fam(nfam);
    for (int b = 0; b < B; ++b) {
        const int f = h->h_meta[b].cls + 1;  // family 0 = generic
        fam[f].push_back(b);
    }
    std::vector<int32_t> order;
    order.reserve(B);
    h->fam_begin.assign(nfam, 0);
    h->fam_count.assign(nfam, 0);
    h->fam_rows.assign(nfam, 0);
    for (int b = 0; b < B; ++b) {
        const int f = h->h_meta[b].cls + 1;
        h->fam_rows[f] = std::max(h->fam_rows[f], (int)h->h_meta[b].r_max);
    }
    for (int f = 0; f < nfam; ++f) {
        std::stable_sort(fam[f].begin(), fam[f].end(),
                         [&](int32_t a, int32_t c) { return h->cost[a] > h->cost[c]; });
        h->fam_begin[f] = (int)order.size();
        h->fam_count[f] = (int)fam[f].size();
        order.insert(order.end(), fam[f].begin(), fam[f].end());
    }
    HIPCHK(hipMemcpyAsync(h->d_order, order.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int f = 1; f < nfam; ++f)
        if (h->fam_count[f] > 0) HIPCHK(rg::prepare_class(f - 1, h->fam_rows[f]));
    // Forked streams only when two or more class families are active; with one
    // the family runs on the handle's stream.
    int nact = 0;
    for (int f = 1; f < nfam; ++f) nact += h->fam_count[f] > 0;
    if (nact >= 2) {
        if (!h->fork && hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess) return RG_E_DEVICE;
        for (int f = 1; f < nfam; ++f)
            if (h->fam_count[f] > 0 && !h->aux[f])
                if (hipStreamCreateWithFlags(&h->aux[f], hipStreamNonBlocking) != hipSuccess ||
                    hipEventCreateWithFlags(&h->join[f], hipEventDisableTiming) != hipSuccess)
                    return RG_E_DEVICE;
    }
    return RG_OK;
}

template <typename T>
rg_status push_impl(rg_ctx *h, const void *gamma, const void *y, const int64_t *row_ptr, const int64_t *goff,
                    int64_t k_single) {
    rg::PushArgs<T> a;
    a.meta = h->d_meta;
    a.state = (T *)h->d_state;
    a.preg = h->d_p;
    a.hreg = h->d_h;
    a.wreg = h->d_w;
    a.gamma = (const T *)gamma;
    a.y = (const T *)y;
    a.row_ptr = row_ptr;
    a.gamma_off = goff;
    a.k_single = k_single;
    a.eps = h->eps;
    a.opts = h->opts;
    a.persistent = (h->opts & RG_OPT_ONE_WG_PER_STREAM) ? 0 : 1;
    HIPCHK(rg::launch_reset_counter(h->d_counter, h->stream));
    // Size-class families run concurrently on forked streams (largest class
    // first), joined back into the handle's stream.
    int nact = 0;
    for (int f = 1; f < RG_MAX_FAMILIES; ++f) nact += h->fam_count[f] > 0;
    const bool serial = (h->opts & RG_OPT_SERIAL_CLASSES) != 0 || nact < 2;
    if (nact > 0 && !serial) HIPCHK(hipEventRecord(h->fork, h->stream));
    // Every family that was forked is joined back, also when a later launch
    // fails, so that the handle's stream always covers all work of the push.
    bool forked[RG_MAX_FAMILIES] = {};
    hipError_t err = hipSuccess;
    for (int f = RG_MAX_FAMILIES - 1; f >= 1 && err == hipSuccess; --f) {
        if (h->fam_count[f] == 0) continue;
        a.order = h->d_order + h->fam_begin[f];
        a.n_order = h->fam_count[f];
        a.counter = h->d_counter + f;
        if (serial) {
            err = rg::launch_push_class<T>(f - 1, a, h->fam_rows[f], h->stream);
            continue;
        }
        err = hipStreamWaitEvent(h->aux[f], h->fork, 0);
        if (err != hipSuccess) break;
        forked[f] = true;
        err = rg::launch_push_class<T>(f - 1, a, h->fam_rows[f], h->aux[f]);
    }
    for (int f = 1; f < RG_MAX_FAMILIES; ++f) {
        if (!forked[f]) continue;
        hipError_t e = hipEventRecord(h->join[f], h->aux[f]);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->join[f], 0);
        if (e != hipSuccess) (void)hipStreamSynchronize(h->aux[f]);
        if (err == hipSuccess) err = e;
    }
    if (err != hipSuccess) return RG_E_DEVICE;
    if (h->d_big) {
        // the multi-CU path enqueues one pass of kernels per block of rows, so
        // it needs the row count on the host: a batched push reads its extent
        const StreamMeta &M = h->h_meta[0];
        const T *g0 = (const T *)gamma, *y0 = (const T *)y;
        int64_t n = k_single;
        if (row_ptr) {
            int64_t rp[2], go = 0;
            HIPCHK(hipMemcpyAsync(rp, row_ptr, sizeof(rp), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipMemcpyAsync(&go, goff, sizeof(go), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            if (rp[1] < rp[0] || rp[0] < 0 || go < 0) return RG_E_INVALID;
            n = rp[1] - rp[0];
            g0 += go;
            y0 += rp[0];
        }
        HIPCHK(rg::launch_push_big<T>(a, M, h->d_big, g0, y0, n, h->num_cus, h->stream));
    } else if (h->fam_count[0] > 0) {
        a.order = h->d_order + h->fam_begin[0];
        a.n_order = h->fam_count[0];
        a.counter = h->d_counter;
        const size_t lds = rg::generic_lds_bytes<T>(
            h->m_max_generic, h->rmax_max_generic, rg::generic_state_in_lds<T>(h->m_max_generic, h->rmax_max_generic));
        int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / lds));
        int grid = std::min(h->fam_count[0], h->num_cus * per_cu);
        HIPCHK(rg::launch_push_generic<T>(a, grid, h->m_max_generic, h->rmax_max_generic, h->stream));
    }
    return RG_OK;
}

bool valid_handle(rg_handle h) { return h != nullptr && h->ws != nullptr; }

// Status of one stream's sticky flags (precedence: non-finite input, rank
// capacity, denominator).
rg_status flag_status(uint32_t f) {
    if (f & RG_FLAG_NONFINITE) return RG_E_NONFINITE;
    if (f & RG_FLAG_RANK_CAPACITY) return RG_E_RANK_CAPACITY;
    if (f) return RG_E_STATE;
    return RG_OK;
}

// Wait for every stream the handle enqueues on (its own and the forked class
// streams), so that nothing of it runs any more.
rg_status drain(rg_ctx *h) {
    rg_status st = RG_OK;
    if (hipStreamSynchronize(h->stream) != hipSuccess) st = RG_E_DEVICE;
    for (int f = 0; f < RG_MAX_FAMILIES; ++f)
        if (h->aux[f] && hipStreamSynchronize(h->aux[f]) != hipSuccess) st = RG_E_DEVICE;
    return st;
}

void release_streams(rg_ctx *h) {
    for (int f = 0; f < RG_MAX_FAMILIES; ++f) {
        if (h->aux[f]) (void)hipStreamDestroy(h->aux[f]);
        if (h->join[f]) (void)hipEventDestroy(h->join[f]);
        h->aux[f] = nullptr;
        h->join[f] = nullptr;
    }
    if (h->fork) (void)hipEventDestroy(h->fork);
    h->fork = nullptr;
}

}  // namespace

extern "C" {

void rg_default_options(rg_options *opt) {
    if (!opt) return;
    opt->dtype = RG_F32;
    opt->r_max = 0;
    opt->eps = -1.0;
    opt->stream = nullptr;
    opt->flags = 0;
}

const char *rg_status_string(rg_status s) {
    switch (s) {
        case RG_OK: return "ok";
        case RG_E_INVALID: return "invalid argument";
        case RG_E_NOMEM: return "out of memory";
        case RG_E_DEVICE: return "HIP runtime error";
        case RG_E_RANK_CAPACITY: return "rank capacity reached";
        case RG_E_NONFINITE: return "non-finite row or target";
        case RG_E_STATE: return "stream is flagged";
        case RG_E_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

int32_t rg_class_count(void) { return RG_NUM_CLASSES; }

rg_status rg_class_info(int32_t cls, int32_t *r_max_cap, int32_t *m_cap, int32_t *threads) {
    if (cls < 0 || cls > RG_CLASS_F64) return RG_E_INVALID;
    if (r_max_cap) *r_max_cap = rg::class_rmax(cls);
    if (m_cap) *m_cap = rg::class_mmax(cls);
    if (threads) *threads = rg::class_threads(cls);
    return RG_OK;
}

rg_status rg_class_fits(int32_t cls, int32_t m, int32_t r_max, int32_t *fits) {
    if (!fits || cls < 0 || cls > RG_CLASS_F64 || m <= 0 || r_max <= 0) return RG_E_INVALID;
    *fits = rg::class_fits(cls, m, r_max) ? 1 : 0;
    return RG_OK;
}

rg_status rg_set_class_rules(const int32_t *m_hi, const int32_t *r_max_hi, const int32_t *cls, int32_t n) {
    if (n < 0 || (n > 0 && (!m_hi || !r_max_hi || !cls))) return RG_E_INVALID;
    for (int k = 0; k < n; ++k)
        if (cls[k] < -1 || cls[k] >= RG_NUM_CLASSES) return RG_E_INVALID;
    rg::set_class_rules(m_hi, r_max_hi, cls, n);
    return RG_OK;
}

size_t rg_workspace_bytes(int32_t B, const int32_t *m, const int32_t *r_max, int32_t dtype) {
    if (B <= 0 || !m || (dtype != RG_F32 && dtype != RG_F64)) return 0;
    for (int b = 0; b < B; ++b)
        if (m[b] <= 0) return 0;
    const size_t es = dtype == RG_F64 ? 8 : 4;
    Layout L = plan_layout(B, m, r_max, es, dtype, 0);
    const StreamMeta &M0 = L.meta[0];
    const bool big = big_stream(B, M0.cls, M0.m, 0);
    return ws_size(L, B, es, big ? rg::big_scratch_doubles(M0.m, M0.r_max) : 0);
}

static rg_status batch_init(rg_handle *out, int32_t B, const int32_t *m, const int32_t *r_max,
                            const rg_options *opt, void *user_ws, size_t user_bytes) {
    if (!out) return RG_E_INVALID;
    *out = nullptr;
    if (B <= 0 || !m) return RG_E_INVALID;
    rg_options o;
    rg_default_options(&o);
    if (opt) o = *opt;
    if (o.dtype != RG_F32 && o.dtype != RG_F64) return RG_E_INVALID;
    if ((o.flags & RG_OPT_ORTHOGONAL) && (o.flags & RG_OPT_ORTHONORMAL)) return RG_E_INVALID;
    for (int b = 0; b < B; ++b) {
        if (m[b] <= 0) return RG_E_INVALID;
        if (r_max && r_max[b] > m[b]) return RG_E_INVALID;
    }
    rg_ctx *h = new (std::nothrow) rg_ctx();
    if (!h) return RG_E_NOMEM;
    h->B = B;
    h->dtype = o.dtype;
    h->esize = o.dtype == RG_F64 ? 8 : 4;
    h->stream = (hipStream_t)o.stream;
    h->opts = o.flags;
    h->eps = o.eps >= 0.0 ? o.eps : (o.dtype == RG_F32 ? 1e-3 : -1.0);
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
        delete h;
        return RG_E_DEVICE;
    }
    // kernel family per stream (the orthogonal factorization variants run in
    // the generic kernel only)
    Layout L = plan_layout(B, m, r_max, h->esize, h->dtype, o.flags);
    h->h_meta = L.meta;
    for (int b = 0; b < B; ++b) {
        StreamMeta &M = h->h_meta[b];
        if (M.cls < 0) {
            h->m_max_generic = std::max(h->m_max_generic, M.m);
            h->rmax_max_generic = std::max(h->rmax_max_generic, M.r_max);
        }
        h->m_max_all = std::max(h->m_max_all, M.m);
        h->rmax_max_all = std::max(h->rmax_max_all, M.r_max);
    }
    if (sizeof(double) * (2 * (size_t)h->m_max_generic + 3 * (size_t)h->rmax_max_generic + 8) > 160 * 1024 ||
        sizeof(double) * (5 * (size_t)h->m_max_all + 4 * (size_t)h->rmax_max_all) > 160 * 1024) {
        delete h;
        return RG_E_UNSUPPORTED;
    }
    // one large stream that no on-chip class holds runs over the whole GPU
    const StreamMeta &M0 = h->h_meta[0];
    const bool big = big_stream(B, M0.cls, M0.m, o.flags);
    const size_t big_doubles = big ? rg::big_scratch_doubles(M0.m, M0.r_max) : 0;
    h->ws_bytes = ws_size(L, B, h->esize, big_doubles);
    if (user_ws) {
        if (user_bytes < h->ws_bytes || ((uintptr_t)user_ws & 255u) != 0) {
            delete h;
            return RG_E_INVALID;
        }
        h->ws = user_ws;
        h->own_ws = false;
    } else if (hipMalloc(&h->ws, h->ws_bytes) != hipSuccess) {
        h->ws = nullptr;
        delete h;
        return RG_E_NOMEM;
    }
    char *p = (char *)h->ws;
    h->d_meta = (StreamMeta *)p;
    p += align_up(sizeof(StreamMeta) * (size_t)B, 256);
    h->d_order = (int32_t *)p;
    p += align_up(sizeof(int32_t) * (size_t)B, 256);
    h->d_counter = (uint32_t *)p;
    p += 256;
    h->d_state = p;
    p += align_up(L.state_elems * h->esize, 256);
    h->d_p = (double *)p;
    p += align_up(L.p_elems * sizeof(double), 256);
    h->d_h = (double *)p;
    p += align_up(L.h_elems * sizeof(double), 256);
    h->d_w = (double *)p;
    p += align_up(L.w_elems * sizeof(double), 256);
    if (big) h->d_big = (double *)p;
    rg_status st = RG_OK;
    if (hipMemsetAsync(h->ws, 0, h->ws_bytes, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->d_meta, h->h_meta.data(), sizeof(StreamMeta) * B, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess)
        st = RG_E_DEVICE;
    h->cost.resize(B);
    for (int b = 0; b < B; ++b) h->cost[b] = (int64_t)h->h_meta[b].m * h->h_meta[b].m * h->h_meta[b].r_max;
    if (st == RG_OK) st = upload_order(h);
    if (st != RG_OK) {
        (void)drain(h);
        release_streams(h);
        if (h->own_ws) (void)hipFree(h->ws);
        delete h;
        return st;
    }
    *out = h;
    return RG_OK;
}

rg_status rg_batch_init(rg_handle *out, int32_t B, const int32_t *m, const int32_t *r_max, const rg_options *opt) {
    return batch_init(out, B, m, r_max, opt, nullptr, 0);
}

rg_status rg_batch_init_ws(rg_handle *out, int32_t B, const int32_t *m, const int32_t *r_max,
                           const rg_options *opt, void *ws, size_t ws_bytes) {
    if (!ws) {
        if (out) *out = nullptr;
        return RG_E_INVALID;
    }
    return batch_init(out, B, m, r_max, opt, ws, ws_bytes);
}

rg_status rg_init(rg_handle *out, int32_t m, const rg_options *opt) {
    if (!out) return RG_E_INVALID;
    *out = nullptr;
    if (m <= 0) return RG_E_INVALID;
    rg_options o;
    rg_default_options(&o);
    if (opt) o = *opt;
    if (o.r_max > m) return RG_E_INVALID;
    int32_t rm = o.r_max > 0 ? o.r_max : m;
    return rg_batch_init(out, 1, &m, &rm, &o);
}

rg_status rg_batch_plan(rg_handle h, const int64_t *rows_hint) {
    if (!valid_handle(h)) return RG_E_INVALID;
    for (int b = 0; b < h->B; ++b) {
        const StreamMeta &M = h->h_meta[b];
        if (rows_hint && rows_hint[b] < 0) return RG_E_INVALID;
        h->cost[b] = rows_hint ? rows_hint[b] * (int64_t)M.m * M.r_max : (int64_t)M.m * M.m * M.r_max;
    }
    return upload_order(h);
}

rg_status rg_push_rows(rg_handle h, const void *gamma, const void *y, int64_t k) {
    if (!valid_handle(h) || h->B != 1 || k < 0) return RG_E_INVALID;
    if (k == 0) return RG_OK;
    if (!gamma || !y) return RG_E_INVALID;
    if (h->known_flags) return RG_E_STATE;
    return h->dtype == RG_F64 ? push_impl<double>(h, gamma, y, nullptr, nullptr, k)
                              : push_impl<float>(h, gamma, y, nullptr, nullptr, k);
}

rg_status rg_batch_push(rg_handle h, const void *gamma, const void *y, const int64_t *row_ptr,
                        const int64_t *gamma_off) {
    if (!valid_handle(h) || !gamma || !y || !row_ptr || !gamma_off) return RG_E_INVALID;
    return h->dtype == RG_F64 ? push_impl<double>(h, gamma, y, row_ptr, gamma_off, 0)
                              : push_impl<float>(h, gamma, y, row_ptr, gamma_off, 0);
}

rg_status rg_batch_solution(rg_handle h, void *x) {
    if (!valid_handle(h) || !x) return RG_E_INVALID;
    if (h->d_big) {
        const StreamMeta &M = h->h_meta[0];
        hipError_t e = h->dtype == RG_F64
                           ? rg::launch_solution_big<double>(h->d_meta, M, (const double *)h->d_state, h->d_h, h->d_w,
                                                             h->d_big, (double *)x, h->stream)
                           : rg::launch_solution_big<float>(h->d_meta, M, (const float *)h->d_state, h->d_h, h->d_w,
                                                            h->d_big, (float *)x, h->stream);
        return e == hipSuccess ? RG_OK : RG_E_DEVICE;
    }
    hipError_t e = h->dtype == RG_F64
                       ? rg::launch_solution<double>(h->d_meta, h->B, (const double *)h->d_state, h->d_h, h->d_w,
                                                     (double *)x, h->rmax_max_all, h->stream)
                       : rg::launch_solution<float>(h->d_meta, h->B, (const float *)h->d_state, h->d_h, h->d_w,
                                                    (float *)x, h->rmax_max_all, h->stream);
    return e == hipSuccess ? RG_OK : RG_E_DEVICE;
}

rg_status rg_solution(rg_handle h, void *x) {
    if (!valid_handle(h) || h->B != 1) return RG_E_INVALID;
    return rg_batch_solution(h, x);
}

static rg_status read_meta(rg_handle h, std::vector<StreamMeta> &dst) {
    dst.resize(h->B);
    HIPCHK(hipMemcpyAsync(dst.data(), h->d_meta, sizeof(StreamMeta) * h->B, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    uint32_t any = 0;
    for (int b = 0; b < h->B; ++b) any |= dst[b].flags;
    h->known_flags = any;
    return RG_OK;
}

rg_status rg_batch_rank(rg_handle h, int32_t *r) {
    if (!valid_handle(h) || !r) return RG_E_INVALID;
    std::vector<StreamMeta> M;
    rg_status st = read_meta(h, M);
    if (st != RG_OK) return st;
    for (int b = 0; b < h->B; ++b) r[b] = M[b].r;
    return RG_OK;
}

rg_status rg_batch_flags(rg_handle h, uint32_t *flags) {
    if (!valid_handle(h) || !flags) return RG_E_INVALID;
    std::vector<StreamMeta> M;
    rg_status st = read_meta(h, M);
    if (st != RG_OK) return st;
    for (int b = 0; b < h->B; ++b) flags[b] = M[b].flags;
    return RG_OK;
}

rg_status rg_batch_classes(rg_handle h, int32_t *cls) {
    if (!valid_handle(h) || !cls) return RG_E_INVALID;
    for (int b = 0; b < h->B; ++b) cls[b] = h->h_meta[b].cls;
    return RG_OK;
}

rg_status rg_probe_lds_read(void *out, int32_t blocks, int32_t iters, void *stream) {
    if (!out || blocks < 1 || iters < 1) return RG_E_INVALID;
    return rg::launch_lds_probe((float *)out, blocks, iters, (hipStream_t)stream) == hipSuccess ? RG_OK
                                                                                                 : RG_E_DEVICE;
}

rg_status rg_rank(rg_handle h, int32_t *r) {
    if (!valid_handle(h) || h->B != 1) return RG_E_INVALID;
    return rg_batch_rank(h, r);
}

rg_status rg_status_flags(rg_handle h, uint32_t *flags) {
    if (!valid_handle(h) || h->B != 1) return RG_E_INVALID;
    return rg_batch_flags(h, flags);
}

rg_status rg_reset(rg_handle h) {
    if (!valid_handle(h)) return RG_E_INVALID;
    if (rg::launch_reset_streams(h->d_meta, h->B, h->stream) != hipSuccess) return RG_E_DEVICE;
    h->known_flags = 0;
    return RG_OK;
}

rg_status rg_check(rg_handle h) {
    if (!valid_handle(h) || h->B != 1) return RG_E_INVALID;
    std::vector<StreamMeta> M;
    rg_status st = read_meta(h, M);
    return st != RG_OK ? st : flag_status(M[0].flags);
}

rg_status rg_batch_status(rg_handle h, int32_t *status) {
    if (!valid_handle(h) || !status) return RG_E_INVALID;
    std::vector<StreamMeta> M;
    rg_status st = read_meta(h, M);
    if (st != RG_OK) return st;
    for (int b = 0; b < h->B; ++b) status[b] = (int32_t)flag_status(M[b].flags);
    return RG_OK;
}

rg_status rg_batch_check_layout(rg_handle h, const int64_t *row_ptr, const int64_t *gamma_off, int64_t n_rows,
                                int64_t n_elems) {
    if (!valid_handle(h) || !row_ptr || !gamma_off || n_rows < 0 || n_elems < 0) return RG_E_INVALID;
    const int B = h->B;
    std::vector<int64_t> rp(B + 1), go(B);
    HIPCHK(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int64_t) * (B + 1), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(go.data(), gamma_off, sizeof(int64_t) * B, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (rp[0] != 0 || rp[B] != n_rows) return RG_E_INVALID;
    std::vector<std::pair<int64_t, int64_t>> spans;
    spans.reserve(B);
    for (int b = 0; b < B; ++b) {
        const int64_t nb = rp[b + 1] - rp[b];
        if (nb < 0) return RG_E_INVALID;
        if (nb == 0) continue;
        const int64_t len = nb * (int64_t)h->h_meta[b].m;
        if (go[b] < 0 || go[b] > n_elems - len) return RG_E_INVALID;
        spans.push_back({go[b], go[b] + len});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k].first < spans[k - 1].second) return RG_E_INVALID;
    return RG_OK;
}

rg_status rg_batch_get_state(rg_handle h, int32_t b, void *C, void *Ct, void *Pinv, double *w) {
    if (!valid_handle(h) || b < 0 || b >= h->B) return RG_E_INVALID;
    std::vector<StreamMeta> M;
    rg_status st = read_meta(h, M);
    if (st != RG_OK) return st;
    const StreamMeta &S = M[b];
    if (S.r == 0) return RG_OK;
    const size_t es = h->esize;
    char *base = (char *)h->d_state + (size_t)S.state_off * es;
    const size_t pitch = (size_t)S.ldm * es;
    if (C) HIPCHK(hipMemcpy2DAsync(C, (size_t)S.m * es, base, pitch, (size_t)S.m * es, S.r, hipMemcpyDeviceToDevice,
                                   h->stream));
    if (Ct && S.h_off >= 0)  // factored form: Ct = H^-1 C formed on the fly
        HIPCHK(h->dtype == RG_F64
                   ? rg::launch_ctilde<double>(h->d_meta, b, (const double *)h->d_state, h->d_h, (double *)Ct, S.r,
                                               h->stream)
                   : rg::launch_ctilde<float>(h->d_meta, b, (const float *)h->d_state, h->d_h, (float *)Ct, S.r,
                                              h->stream));
    else if (Ct)
        HIPCHK(hipMemcpy2DAsync(Ct, (size_t)S.m * es, base + (size_t)S.r_max * pitch, pitch, (size_t)S.m * es, S.r,
                                hipMemcpyDeviceToDevice, h->stream));
    if (Pinv)
        HIPCHK(hipMemcpy2DAsync(Pinv, (size_t)S.r * sizeof(double), h->d_p + S.p_off, (size_t)S.r_max * sizeof(double),
                                (size_t)S.r * sizeof(double), S.r, hipMemcpyDeviceToDevice, h->stream));
    if (w)
        HIPCHK(hipMemcpyAsync(w, h->d_w + S.w_off, sizeof(double) * S.r, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RG_OK;
}

rg_status rg_batch_adjoint(rg_handle h, const void *A, const void *Y, const int64_t *row_ptr, const int64_t *a_off,
                           const void *g, void *dA, void *dY) {
    if (!valid_handle(h) || !A || !Y || !row_ptr || !a_off || !g || !dA || !dY) return RG_E_INVALID;
    hipError_t e =
        h->dtype == RG_F64
            ? rg::launch_adjoint<double>(h->d_meta, h->B, (const double *)h->d_state, h->d_p, h->d_h, h->d_w,
                                         (const double *)A, (const double *)Y, row_ptr, a_off, (const double *)g,
                                         (double *)dA, (double *)dY, h->m_max_all, h->rmax_max_all, h->stream)
            : rg::launch_adjoint<float>(h->d_meta, h->B, (const float *)h->d_state, h->d_p, h->d_h, h->d_w,
                                        (const float *)A, (const float *)Y, row_ptr, a_off, (const float *)g,
                                        (float *)dA, (float *)dY, h->m_max_all, h->rmax_max_all, h->stream);
    return e == hipSuccess ? RG_OK : RG_E_DEVICE;
}

rg_status rg_batch_pinv(rg_handle h, const void *A, const int64_t *row_ptr, const int64_t *a_off, void *Ap) {
    if (!valid_handle(h) || !A || !row_ptr || !a_off || !Ap) return RG_E_INVALID;
    hipError_t e =
        h->dtype == RG_F64
            ? rg::launch_pinv<double>(h->d_meta, h->B, (const double *)h->d_state, h->d_p, h->d_h, (const double *)A, row_ptr,
                                      a_off, (double *)Ap, h->m_max_all, h->rmax_max_all, h->stream)
            : rg::launch_pinv<float>(h->d_meta, h->B, (const float *)h->d_state, h->d_p, h->d_h, (const float *)A, row_ptr,
                                     a_off, (float *)Ap, h->m_max_all, h->rmax_max_all, h->stream);
    return e == hipSuccess ? RG_OK : RG_E_DEVICE;
}

// Teardown order: wait for every stream the handle used (its own and the
// forked class streams), destroy those streams and events, and only then free
// the workspace, so that no enqueued kernel or event can outlive the memory.
rg_status rg_destroy(rg_handle h) {
    if (!h) return RG_E_INVALID;
    rg_status st = drain(h);
    release_streams(h);
    if (h->ws && h->own_ws && hipFree(h->ws) != hipSuccess) st = RG_E_DEVICE;
    h->ws = nullptr;
    delete h;
    return st;
}

}  // extern "C"
