// api.hip -- the exported C ABI (include/algdist.h): argument checks on the
// host, workspace management, and the launch schedule of each call.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>
#include <stdarg.h>

#include "device.h"
#include "internal.h"

using namespace ad;

namespace {

int fail(ad_handle h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(ad_handle h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return code;
}

bool k_ok(int K) { return K == 2 || K == 4 || K == 8 || K == 16 || K == 32 || K == 64; }
size_t dsize(int dtype) { return dtype == AD_F32 ? 4 : 8; }
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// the reason appended to a failed workspace reservation
const char* ws_why(int rc) {
    return rc == AD_EUNSUPPORTED
               ? ": the workspace would have to grow while the stream is capturing; make the "
                 "same call once uncaptured first"
               : "";
}

// Common CSR argument checks (host side: sizes and pointers only).
int check_csr(ad_handle h, const ad_csr* A) {
    if (!A) return fail(h, AD_EINVAL, "A is NULL");
    if (A->n < 0) return fail(h, AD_EINVAL, "n = %d < 0", A->n);
    if (A->nnz < 0 || A->nnz > 0x7fffffffLL)
        return fail(h, AD_ESTRUCT, "nnz = %lld outside [0, 2^31)", (long long)A->nnz);
    if (A->dtype != AD_F32 && A->dtype != AD_F64)
        return fail(h, AD_EDTYPE, "dtype %d is neither AD_F32 nor AD_F64", A->dtype);
    if (A->n > 0 && (!A->row_ptr || (A->nnz > 0 && (!A->col || !A->val))))
        return fail(h, AD_EINVAL, "null CSR array");
    if (A->n > 0 && A->nnz < A->n)
        return fail(h, AD_ESTRUCT, "nnz = %lld < n = %d: every row needs its diagonal",
                    (long long)A->nnz, A->n);
    return AD_OK;
}

int check_panel(ad_handle h, const void* X, const char* name, int n) {
    if (n > 0 && !X) return fail(h, AD_EINVAL, "%s is NULL", name);
    if (X && !aligned16(X)) return fail(h, AD_EINVAL, "%s is not 16-byte aligned", name);
    return AD_OK;
}

}  // namespace

// ---------------------------------------------------------------- static scratch
// Device memory of distance_ls_noalloc: the fused pass's per-workgroup
// partial sums of ls_val.  Each device holds its own copy of the array at
// its own address, resolved once per device in algdist_create; host code
// uses only that address (the array's name is a host-side stand-in).
constexpr size_t kStaticScratchBytes = size_t(1) << 20;  // 131072 FP64 partials
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};  // per-device address of `scratch`

// Resolves this device's copy of `scratch` (device must be current).
int resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return AD_EDEVICE;
    if (g_scratch[device]) return AD_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return AD_EDEVICE;
    g_scratch[device] = p;
    return AD_OK;
}
}  // namespace

namespace ad {
TimedScope::TimedScope(ad_handle h, const char* label, hipStream_t s) : h_(h), label_(label), s_(s) {
    if (!h_->timing) return;
    if (h_->events_used + 2 > h_->event_pool.size()) {
        for (int q = 0; q < 2; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            h_->event_pool.push_back(e);
        }
    }
    a_ = h_->event_pool[h_->events_used++];
    if (hipEventRecord(a_, s_) != hipSuccess) a_ = nullptr;
}

TimedScope::~TimedScope() {
    if (!a_) return;
    hipEvent_t b = h_->event_pool[h_->events_used++];
    if (hipEventRecord(b, s_) == hipSuccess) h_->timed.push_back({label_, a_, b});
}

int k_slot(int K) {
    for (int q = 1; q < kNumKSlots; ++q)
        if (K == (1 << q)) return q;
    return -1;
}

int nnz_bucket(int64_t nnz, int n) {
    const double r = n > 0 ? (double)nnz / n : 0.0;
    return r < 8 ? 0 : r < 16 ? 1 : r < 32 ? 2 : 3;
}

// bucket of a batch: stored entries per row over all members
int batch_bucket(int nmat, const ad_csr* As) {
    int64_t rows = 0, ents = 0;
    for (int m = 0; m < nmat; ++m) {
        rows += As[m].n;
        ents += As[m].nnz;
    }
    const double r = rows > 0 ? (double)ents / (double)rows : 0.0;
    return r < 8 ? 0 : r < 16 ? 1 : r < 32 ? 2 : 3;
}

LaunchCfg cfg_for(ad_handle h, int kernel, int dtype, int K, const ad_csr* A) {
    const int ks = k_slot(K);
    const int b = nnz_bucket(A->nnz, A->n);
    if (ks >= 0 && (dtype == AD_F32 || dtype == AD_F64) && h->has_tuned[kernel][dtype][ks][b])
        return h->tuned[kernel][dtype][ks][b];
    return LaunchCfg();
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

int ws_reserve(ad_handle h, size_t bytes, hipStream_t s) {
    const bool cap = stream_capturing(s);
    if (bytes <= h->ws_bytes) {
        if (cap) h->ws_pinned = true;  // the caller's graph now refers to this buffer
        return AD_OK;
    }
    // a buffer cannot move under a graph being captured
    if (cap) return AD_EUNSUPPORTED;
    if (h->ws_pinned) {
        // a captured graph may still replay on the old buffer: keep it
        if (h->ws) h->retired.push_back(h->ws);
        h->ws_pinned = false;
    } else {
        // earlier calls may still use the old buffer
        AD_HIP(hipDeviceSynchronize());
        if (h->ws) AD_HIP(hipFree(h->ws));
    }
    h->ws = nullptr;
    h->ws_bytes = 0;
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&h->ws, want) != hipSuccess) {
        h->ws = nullptr;
        return AD_ENOMEM;
    }
    h->ws_bytes = want;
    return AD_OK;
}
}  // namespace ad

extern "C" {

int algdist_version(void) { return ALGDIST_VERSION; }

int algdist_create(ad_handle* out, int device) {
    if (!out) return AD_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return AD_EDEVICE;
    ad_handle h = new ad_handle_s();
    h->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return AD_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) h->cu_count = prop.multiProcessorCount;
    if (hipMalloc((void**)&h->status, sizeof(unsigned)) != hipSuccess) {
        delete h;
        return AD_ENOMEM;
    }
    if (hipMemset(h->status, 0, sizeof(unsigned)) != hipSuccess ||
        resolve_scratch(device) != AD_OK) {
        (void)hipFree(h->status);
        delete h;
        return AD_EDEVICE;
    }
    *out = h;
    return AD_OK;
}

int algdist_destroy(ad_handle h) {
    if (!h) return AD_EINVAL;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    if (h->ws) (void)hipFree(h->ws);
    for (void* p : h->retired) (void)hipFree(p);
    if (h->status) (void)hipFree(h->status);
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
    batch_state_free(h);
    delete h;
    return AD_OK;
}

int algdist_status(ad_handle h, uint32_t* bits, int clear) {
    if (!h || !bits) return AD_EINVAL;
    AD_HIP(hipSetDevice(h->device));
    AD_HIP(hipDeviceSynchronize());
    unsigned v = 0;
    AD_HIP(hipMemcpy(&v, h->status, sizeof v, hipMemcpyDeviceToHost));
    *bits = v;
    if (clear) AD_HIP(hipMemset(h->status, 0, sizeof(unsigned)));
    return AD_OK;
}

const char* algdist_last_error(ad_handle h) { return h ? h->err.c_str() : "null handle"; }

int algdist_timing(ad_handle h, int enable) {
    if (!h) return AD_EINVAL;
    if (enable) {
        h->timed.clear();
        h->events_used = 0;
    }
    h->timing = enable != 0;
    return AD_OK;
}

const char* algdist_timing_report(ad_handle h) {
    if (!h) return "";
    h->report.clear();
    if (hipSetDevice(h->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return "";
    std::vector<std::string> labels;
    std::vector<int> count;
    std::vector<double> total;
    for (const auto& t : h->timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) continue;
        size_t q = 0;
        while (q < labels.size() && labels[q] != t.label) ++q;
        if (q == labels.size()) {
            labels.push_back(t.label);
            count.push_back(0);
            total.push_back(0.0);
        }
        ++count[q];
        total[q] += ms;
    }
    char line[160];
    for (size_t q = 0; q < labels.size(); ++q) {
        snprintf(line, sizeof line, "%s %d %.6f\n", labels[q].c_str(), count[q], total[q]);
        h->report += line;
    }
    return h->report.c_str();
}

static bool lpr_valid(int dtype, int K, int L) {
    return dtype == AD_F32 ? lpr_ok<float>(K, L) : lpr_ok<double>(K, L);
}

int algdist_set_launch(ad_handle h, const char* kernel, int32_t dtype, int32_t K, int32_t bucket,
                       int32_t lanes_per_row, int32_t rows_per_lane, int32_t xcd_map) {
    if (!h || !kernel) return AD_EINVAL;
    h->err.clear();
    int kn = -1;
    if (!strcmp(kernel, "jacobi")) kn = KN_JACOBI;
    else if (!strcmp(kernel, "gs_phase")) kn = KN_GS;
    else if (!strcmp(kernel, "algdist")) kn = KN_ALGDIST;
    else if (!strcmp(kernel, "ls_interp")) kn = KN_LS;
    else if (!strcmp(kernel, "batched")) kn = KN_BATCHED;
    else if (!strcmp(kernel, "distance_ls")) kn = KN_DLS;
    else if (!strcmp(kernel, "batched_distance")) kn = KN_BDIST;
    if (kn < 0) return fail(h, AD_EINVAL, "unknown kernel family '%s'", kernel);
    if (dtype != AD_F32 && dtype != AD_F64) return fail(h, AD_EDTYPE, "dtype %d", dtype);
    const int ks = k_slot(K);
    if (ks < 0) return fail(h, AD_EINVAL, "K = %d", K);
    if (bucket < -1 || bucket >= kNumBuckets) return fail(h, AD_EINVAL, "bucket %d", bucket);
    if (rows_per_lane < 1 || rows_per_lane > 1024) return fail(h, AD_EINVAL, "rows_per_lane %d", rows_per_lane);
    if (lanes_per_row != 0 && !lpr_valid(dtype, K, lanes_per_row))
        return fail(h, AD_EINVAL, "lanes_per_row %d unsupported for K = %d", lanes_per_row, K);
    LaunchCfg c;
    c.lpr = lanes_per_row;
    c.iter = kn == KN_LS ? 1 : rows_per_lane;
    if (xcd_map < 0 || xcd_map > 4096) return fail(h, AD_EINVAL, "xcd_map %d", xcd_map);
    c.xcd_map = xcd_map;
    for (int b = 0; b < kNumBuckets; ++b)
        if (bucket < 0 || bucket == b) {
            h->tuned[kn][dtype][ks][b] = c;
            h->has_tuned[kn][dtype][ks][b] = true;
        }
    return AD_OK;
}

int algdist_autotune(ad_handle h, const ad_csr* A, int32_t K, int32_t relax, const int32_t* color,
                     int32_t ncolors, const uint8_t* cf, int32_t caliber, const char* cache_json,
                     void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (relax != AD_JACOBI && relax != AD_MULTICOLOR_GS) return fail(h, AD_EINVAL, "relax = %d", relax);
    if (relax == AD_MULTICOLOR_GS && (ncolors < 1 || ncolors > 64 || (A->n > 0 && !color)))
        return fail(h, AD_EINVAL, "colours: ncolors = %d, color %p", ncolors, (const void*)color);
    if (A->n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    rc = autotune(h, A, K, relax, color, ncolors, cf, caliber, cache_json, (hipStream_t)stream);
    return rc ? fail(h, rc, "autotune") : AD_OK;
}

int algdist_autotune_batched(ad_handle h, int32_t nmat, const ad_csr* As, int32_t K,
                             int32_t sweeps, const char* cache_json, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    if (nmat < 1 || !As) return fail(h, AD_EINVAL, "nmat = %d or As is NULL", nmat);
    int rc;
    for (int m = 0; m < nmat; ++m) {
        if ((rc = check_csr(h, &As[m]))) return fail(h, rc, "matrix %d: %s", m, h->err.c_str());
        if (As[m].dtype != As[0].dtype) return fail(h, AD_EDTYPE, "matrix %d has another dtype", m);
    }
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (sweeps < 0) return fail(h, AD_EINVAL, "sweeps = %d < 0", sweeps);
    AD_HIP(hipSetDevice(h->device));
    rc = autotune_batched(h, nmat, As, K, sweeps, cache_json, (hipStream_t)stream);
    return rc ? fail(h, rc, "batched autotune") : AD_OK;
}

int csr_validate(ad_handle h, const ad_csr* A, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (A->n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    return launch_csr_validate(A, h->status, (hipStream_t)stream);
}

}  // extern "C"

namespace ad {

// Colour-phase Gauss-Seidel sweeps in the colour-major layout: stable
// colour partition (rowlist: permuted row -> natural row, seg), a
// colour-major copy of the CSR (rows of one colour contiguous, permuted
// columns), the start written in permuted order, ping-pong of two permuted
// panels, and the last sweep writing each row straight to its natural
// position in X.  Checkpoints are un-permuted.
int gs_sweeps(ad_handle h, const ad_csr* A, int K, uint64_t seed, const void* X0, int sweeps,
              const int32_t* color, int ncolors, void* X, void* ckpt, int ckpt_every,
              hipStream_t s, unsigned* color_status) {
    if (!color_status) color_status = h->status;
    const int dt = A->dtype;
    const int n = A->n;
    const size_t panel = (size_t)n * K * dsize(dt);
    const int nblk = color_partition_blocks(n);
    WsReq req;
    const size_t o_pa = req.add(panel);
    const size_t o_pb = req.add(panel);
    const size_t o_rl = req.add(sizeof(int32_t) * (size_t)n);
    const size_t o_inv = req.add(sizeof(int32_t) * (size_t)n);
    const size_t o_rpp = req.add(sizeof(int32_t) * ((size_t)n + 1));
    const size_t o_colp = req.add(sizeof(int32_t) * (size_t)A->nnz);
    const size_t o_valp = req.add(dsize(dt) * (size_t)A->nnz);
    const size_t o_seg = req.add(sizeof(int32_t) * (ncolors + 2));
    const size_t o_cnt = req.add(sizeof(int32_t) * 2 * (size_t)(ncolors + 1) * nblk);
    int rc;
    if ((rc = ws_reserve(h, req.off, s)))
        return fail(h, rc, "workspace of %zu bytes%s", req.off, ws_why(rc));
    char* ws = (char*)h->ws;
    void* P[2] = {ws + o_pa, ws + o_pb};
    int32_t* rowlist = (int32_t*)(ws + o_rl);
    int32_t* seg = (int32_t*)(ws + o_seg);
    PermCsr pc{n, rowlist, seg, (int32_t*)(ws + o_rpp), (int32_t*)(ws + o_colp), ws + o_valp};
    const bool fuse_start = !X0 && K * (int)dsize(dt) >= 16;
    {
        TimedScope ts(h, "color_partition", s);
        rc = launch_color_partition(n, color, ncolors, A->row_ptr, rowlist, (int32_t*)(ws + o_inv),
                                    seg, (int32_t*)(ws + o_cnt), nblk, (int32_t*)(ws + o_rpp),
                                    color_status, s);
        // the hash start is written by the entry copy when its rows are whole
        // 16-byte chunks; a given X0, or narrower rows, take their own launch
        if (!rc) rc = launch_perm_setup(dt, A, pc, (int32_t*)(ws + o_inv), s, K, seed,
                                        fuse_start ? P[0] : nullptr);
        if (rc) return fail(h, rc, "colour partition launch");
    }
    if (!fuse_start) {
        TimedScope ts(h, "tv_init", s);
        if ((rc = launch_start_perm(dt, n, K, rowlist, seed, X0, P[0], s)))
            return fail(h, rc, "start launch");
    }
    const LaunchCfg cfg = cfg_for(h, KN_GS, dt, K, A);
    for (int q = 0; q < sweeps; ++q) {
        void* Xold = P[q & 1];
        void* Xnew = P[(q + 1) & 1];
        if (ckpt && q % ckpt_every == 0) {
            TimedScope ts(h, "unpermute", s);
            rc = launch_unpermute(dt, n, K, rowlist, Xold,
                                  (char*)ckpt + (size_t)(q / ckpt_every) * panel, s);
            if (rc) return fail(h, rc, "checkpoint launch");
        }
        const bool last = q == sweeps - 1;
        for (int c = 0; c < ncolors; ++c) {
            TimedScope ts(h, "gs_phase", s);
            rc = launch_gs_phase_perm(dt, K, pc, c, ncolors, Xold, Xnew, last ? X : nullptr,
                                      (!last || c < ncolors - 1) ? 1 : 0, h->status, cfg, s);
            if (rc) return fail(h, rc, "relaxation launch");
        }
    }
    return AD_OK;
}

}  // namespace ad

extern "C" {

int setup_testvectors(ad_handle h, const ad_csr* A, int32_t K, uint64_t seed, const void* X0,
                      int32_t relax, int32_t sweeps, double omega, const int32_t* color,
                      int32_t ncolors, void* X, void* ckpt, int32_t ckpt_every, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (sweeps < 0) return fail(h, AD_EINVAL, "sweeps = %d < 0", sweeps);
    if (relax != AD_JACOBI && relax != AD_MULTICOLOR_GS)
        return fail(h, AD_EINVAL, "relax = %d is neither AD_JACOBI nor AD_MULTICOLOR_GS", relax);
    if (relax == AD_MULTICOLOR_GS && sweeps > 0) {
        if (ncolors < 1 || ncolors > 64)
            return fail(h, AD_EINVAL, "ncolors = %d outside [1, 64]", ncolors);
        if (A->n > 0 && !color) return fail(h, AD_EINVAL, "color is NULL");
    }
    if ((rc = check_panel(h, X, "X", A->n))) return rc;
    if ((rc = check_panel(h, X0, "X0", 0))) return rc;
    if (X0 && X0 == X) return fail(h, AD_EINVAL, "X0 and X alias");
    if (ckpt) {
        if (ckpt_every <= 0) return fail(h, AD_EINVAL, "ckpt_every = %d <= 0", ckpt_every);
        if ((rc = check_panel(h, ckpt, "ckpt", A->n))) return rc;
    }
    if (A->n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const int dt = A->dtype;
    const size_t panel = (size_t)A->n * K * dsize(dt);

    if (relax == AD_MULTICOLOR_GS && sweeps > 0)
        return gs_sweeps(h, A, K, seed, X0, sweeps, color, ncolors, X, ckpt, ckpt_every, s);

    // Jacobi (or no sweep).  Workspace: one extra panel for the ping-pong.
    WsReq req;
    const size_t o_pp = req.add(panel);
    if ((rc = ws_reserve(h, req.off, s)))
        return fail(h, rc, "workspace of %zu bytes%s", req.off, ws_why(rc));
    void* W = (char*)h->ws + o_pp;

    // Buffer of iterate q (0..sweeps): x^sweeps lands in X; a checkpointed
    // iterate lives in its checkpoint slot; the others alternate between X
    // and W so that every sweep reads and writes different buffers.
    const int ns = sweeps;
    std::vector<void*> buf(ns + 1);
    buf[ns] = X;
    for (int q = ns - 1; q >= 0; --q) {
        if (ckpt && q % ckpt_every == 0) buf[q] = (char*)ckpt + (size_t)(q / ckpt_every) * panel;
        else buf[q] = (buf[q + 1] == X) ? W : X;
    }
    if (X0 && ns > 0 && !ckpt) {
        buf[0] = (void*)X0;  // read-only start: sweep 0 reads it in place
    } else if (X0) {
        AD_HIP(hipMemcpyAsync(buf[0], X0, panel, hipMemcpyDeviceToDevice, s));
    } else {
        TimedScope ts(h, "tv_init", s);
        if ((rc = launch_tv_init(dt, 0, A->n, K, seed, buf[0], s))) return fail(h, rc, "tv_init launch");
    }
    if (ns == 0 && ckpt) AD_HIP(hipMemcpyAsync(ckpt, X, panel, hipMemcpyDeviceToDevice, s));

    const LaunchCfg cfg = cfg_for(h, KN_JACOBI, dt, K, A);
    for (int q = 0; q < ns; ++q) {
        TimedScope ts(h, "jacobi", s);
        rc = launch_jacobi(dt, K, A, buf[q], buf[q + 1], omega, h->status, cfg, s);
        if (rc) return fail(h, rc, "relaxation launch");
    }
    return AD_OK;
}

int algebraic_distance(ad_handle h, const ad_csr* A, int32_t K, const void* X, const double* w,
                       int32_t target, void* mu, double* p, double theta, const uint8_t* fmask,
                       uint8_t* strong, int32_t* nstrong, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (target != AD_TARGET_PLAIN && target != AD_TARGET_RESIDUAL)
        return fail(h, AD_EINVAL, "target = %d", target);
    if ((rc = check_panel(h, X, "X", A->n))) return rc;
    if (A->nnz > 0 && !mu) return fail(h, AD_EINVAL, "mu is NULL");
    if (strong && !(theta > 0.0 && theta < 1.0))
        return fail(h, AD_EINVAL, "theta = %g outside (0, 1)", theta);
    if (A->n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    const LaunchCfg cfg = cfg_for(h, KN_ALGDIST, A->dtype, K, A);
    TimedScope ts(h, "algdist", (hipStream_t)stream);
    rc = launch_algdist(A->dtype, K, A, X, w, target, mu, p, theta, fmask, strong, nstrong,
                        h->status, cfg, (hipStream_t)stream);
    return rc ? fail(h, rc, "algebraic_distance launch") : AD_OK;
}

int strength_graph(ad_handle h, const ad_csr* A, const void* mu, double theta,
                   const uint8_t* fmask, uint8_t* strong, int32_t* nstrong, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (!(theta > 0.0 && theta < 1.0)) return fail(h, AD_EINVAL, "theta = %g outside (0, 1)", theta);
    if (A->nnz > 0 && (!mu || !strong)) return fail(h, AD_EINVAL, "mu or strong is NULL");
    if (A->n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    TimedScope ts(h, "strength", (hipStream_t)stream);
    rc = launch_strength(A->dtype, A, mu, theta, fmask, strong, nstrong, (hipStream_t)stream);
    return rc ? fail(h, rc, "strength_graph launch") : AD_OK;
}

int ls_interp(ad_handle h, const ad_csr* A, int32_t K, const void* X, const double* w,
              const uint8_t* cf, const void* mu, int32_t caliber, int32_t target, int32_t* P_col,
              double* P_val, double* ls_val, int32_t* row_status, double* ls_sum, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (caliber < 1 || caliber > 8) return fail(h, AD_ECALIBER, "caliber = %d outside [1, 8]", caliber);
    if (caliber > K)
        return fail(h, AD_ECALIBER, "caliber = %d > K = %d: LS rows would not be unique", caliber, K);
    if (target != AD_TARGET_PLAIN && target != AD_TARGET_RESIDUAL)
        return fail(h, AD_EINVAL, "target = %d", target);
    if ((rc = check_panel(h, X, "X", A->n))) return rc;
    if (A->n > 0 && (!cf || !mu || !P_col || !P_val || !ls_val || !row_status))
        return fail(h, AD_EINVAL, "null output or input array");
    AD_HIP(hipSetDevice(h->device));
    const LaunchCfg cfg = cfg_for(h, KN_LS, A->dtype, K, A);
    double* bs = nullptr;
    if (ls_sum && A->n > 0) {
        const int nb = ls_interp_blocks(A->dtype, K, A->n, cfg);
        if ((rc = ws_reserve(h, sizeof(double) * (size_t)nb, (hipStream_t)stream)))
            return fail(h, rc, "workspace for %d block sums%s", nb, ws_why(rc));
        bs = (double*)h->ws;
    }
    TimedScope ts(h, "ls_interp", (hipStream_t)stream);
    rc = launch_ls_interp(A->dtype, K, caliber, A, X, w, cf, mu, target, P_col, P_val, ls_val,
                          row_status, bs, ls_sum, h->status, cfg, (hipStream_t)stream);
    return rc ? fail(h, rc, "ls_interp launch") : AD_OK;
}

}  // extern "C"

// distance_ls and distance_ls_noalloc: the block partial sums of ls_sum
// live in the handle's workspace (grown on demand) or, with noalloc, in this
// device's copy of the static scratch array.
static int distance_ls_impl(ad_handle h, const ad_csr* A, int32_t K, const void* X,
                            const double* w, int32_t target, void* mu, double theta,
                            const uint8_t* fmask, uint8_t* strong, int32_t* nstrong,
                            const uint8_t* cf, int32_t caliber, int32_t* P_col, double* P_val,
                            double* ls_val, int32_t* row_status, double* ls_sum, void* stream,
                            bool noalloc) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (target != AD_TARGET_PLAIN && target != AD_TARGET_RESIDUAL)
        return fail(h, AD_EINVAL, "target = %d", target);
    if (caliber < 1 || caliber > 8) return fail(h, AD_ECALIBER, "caliber = %d outside [1, 8]", caliber);
    if (caliber > K)
        return fail(h, AD_ECALIBER, "caliber = %d > K = %d: LS rows would not be unique", caliber, K);
    if ((rc = check_panel(h, X, "X", A->n))) return rc;
    if (A->nnz > 0 && !mu) return fail(h, AD_EINVAL, "mu is NULL");
    if (strong && !(theta > 0.0 && theta < 1.0))
        return fail(h, AD_EINVAL, "theta = %g outside (0, 1)", theta);
    if (A->n > 0 && (!cf || !P_col || !P_val || !ls_val || !row_status))
        return fail(h, AD_EINVAL, "null output or input array");
    AD_HIP(hipSetDevice(h->device));
    if (A->n == 0) return ls_sum ? launch_fill_f64(ls_sum, 1, 0.0, (hipStream_t)stream) : AD_OK;
    const LaunchCfg cfg = cfg_for(h, KN_DLS, A->dtype, K, A);
    double* bs = nullptr;
    if (ls_sum) {
        const int nb = dist_ls_blocks(A->dtype, K, A->n, cfg);
        const size_t need = sizeof(double) * (size_t)nb;
        if (noalloc) {
            if (need > kStaticScratchBytes)
                return fail(h, AD_ESTRUCT,
                            "%d rows need %zu bytes of block partial sums; the static scratch "
                            "holds %zu (%zu workgroups of the fused pass)",
                            A->n, need, kStaticScratchBytes, kStaticScratchBytes / sizeof(double));
            bs = (double*)g_scratch[h->device];
        } else {
            if ((rc = ws_reserve(h, need, (hipStream_t)stream)))
                return fail(h, rc, "workspace for %d block sums%s", nb, ws_why(rc));
            bs = (double*)h->ws;
        }
    }
    TimedScope ts(h, "distance_ls", (hipStream_t)stream);
    rc = launch_dist_ls(A->dtype, K, caliber, A, X, w, target, mu, theta, fmask, strong, nstrong,
                        cf, P_col, P_val, ls_val, row_status, bs, ls_sum, h->status, cfg,
                        (hipStream_t)stream);
    return rc ? fail(h, rc, "distance_ls launch") : AD_OK;
}

extern "C" {

int distance_ls(ad_handle h, const ad_csr* A, int32_t K, const void* X, const double* w,
                int32_t target, void* mu, double theta, const uint8_t* fmask, uint8_t* strong,
                int32_t* nstrong, const uint8_t* cf, int32_t caliber, int32_t* P_col,
                double* P_val, double* ls_val, int32_t* row_status, double* ls_sum, void* stream) {
    return distance_ls_impl(h, A, K, X, w, target, mu, theta, fmask, strong, nstrong, cf, caliber,
                            P_col, P_val, ls_val, row_status, ls_sum, stream, false);
}

int distance_ls_noalloc(ad_handle h, const ad_csr* A, int32_t K, const void* X, const double* w,
                        int32_t target, void* mu, double theta, const uint8_t* fmask,
                        uint8_t* strong, int32_t* nstrong, const uint8_t* cf, int32_t caliber,
                        int32_t* P_col, double* P_val, double* ls_val, int32_t* row_status,
                        double* ls_sum, void* stream) {
    return distance_ls_impl(h, A, K, X, w, target, mu, theta, fmask, strong, nstrong, cf, caliber,
                            P_col, P_val, ls_val, row_status, ls_sum, stream, true);
}

// Structure-only checks of A (values unused).
static int check_structure(ad_handle h, const ad_csr* A) {
    if (!A) return fail(h, AD_EINVAL, "A is NULL");
    if (A->n < 0) return fail(h, AD_EINVAL, "n = %d < 0", A->n);
    if (A->nnz < 0 || A->nnz > 0x7fffffffLL)
        return fail(h, AD_ESTRUCT, "nnz = %lld outside [0, 2^31)", (long long)A->nnz);
    if (A->n > 0 && (!A->row_ptr || (A->nnz > 0 && !A->col)))
        return fail(h, AD_EINVAL, "null CSR array");
    return AD_OK;
}

static int check_pattern(ad_handle h, int n, int64_t nnz_g, const int32_t* rpg,
                         const int32_t* cig) {
    if (nnz_g < 0 || nnz_g > 0x7fffffffLL)
        return fail(h, AD_ESTRUCT, "nnz_g = %lld outside [0, 2^31)", (long long)nnz_g);
    if (n > 0 && (!rpg || (nnz_g > 0 && !cig))) return fail(h, AD_EINVAL, "null pattern array");
    return AD_OK;
}

int power_graph_rows(ad_handle h, const ad_csr* A, int32_t d, int32_t* row_ptr_d, int64_t* nnz_d,
                     void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_structure(h, A);
    if (rc) return rc;
    if (d < 1) return fail(h, AD_EINVAL, "d = %d < 1", d);
    if (!row_ptr_d || !nnz_d) return fail(h, AD_EINVAL, "row_ptr_d or nnz_d is NULL");
    hipStream_t s = (hipStream_t)stream;
    AD_HIP(hipSetDevice(h->device));
    if (stream_capturing(s))
        return fail(h, AD_EUNSUPPORTED, "power_graph_rows synchronises the stream: not capturable");
    const size_t need = pow_rows_workspace(A->n);
    if ((rc = ws_reserve(h, need, s))) return fail(h, rc, "workspace of %zu bytes", need);
    int64_t tot = 0;
    int bad = 0;
    {
        TimedScope ts(h, "power_graph", s);
        rc = launch_pow_rows(A->n, d, A->row_ptr, A->col, row_ptr_d, h->ws, &tot, &bad, s);
    }
    if (rc) return fail(h, rc, "power_graph_rows launch");
    if (bad & 1) return fail(h, AD_EUNSUPPORTED, "a row of A^%d has more than 1024 entries", d);
    if (bad & 2) return fail(h, AD_EUNSUPPORTED, "A^%d has more than 2^31 - 1 entries", d);
    *nnz_d = tot;
    return AD_OK;
}

int power_graph_cols(ad_handle h, const ad_csr* A, int32_t d, const int32_t* row_ptr_d,
                     int32_t* col_d, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_structure(h, A);
    if (rc) return rc;
    if (d < 1) return fail(h, AD_EINVAL, "d = %d < 1", d);
    if (A->n > 0 && (!row_ptr_d || !col_d)) return fail(h, AD_EINVAL, "row_ptr_d or col_d is NULL");
    AD_HIP(hipSetDevice(h->device));
    TimedScope ts(h, "power_graph", (hipStream_t)stream);
    rc = launch_pow_cols(A->n, d, A->row_ptr, A->col, row_ptr_d, col_d, h->status,
                         (hipStream_t)stream);
    return rc ? fail(h, rc, "power_graph_cols launch") : AD_OK;
}

int algebraic_distance_graph(ad_handle h, const ad_csr* A, int64_t nnz_g, const int32_t* row_ptr_g,
                             const int32_t* col_g, int32_t K, const void* X, const double* w,
                             int32_t target, void* mu, double* p, double theta,
                             const uint8_t* fmask, uint8_t* strong, int32_t* nstrong,
                             void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if ((rc = check_pattern(h, A->n, nnz_g, row_ptr_g, col_g))) return rc;
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (target != AD_TARGET_PLAIN && target != AD_TARGET_RESIDUAL)
        return fail(h, AD_EINVAL, "target = %d", target);
    if ((rc = check_panel(h, X, "X", A->n))) return rc;
    if (nnz_g > 0 && !mu) return fail(h, AD_EINVAL, "mu is NULL");
    if (strong && !(theta > 0.0 && theta < 1.0))
        return fail(h, AD_EINVAL, "theta = %g outside (0, 1)", theta);
    if (A->n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    const ad_csr G{A->n, nnz_g, row_ptr_g, col_g, A->val, A->dtype};
    const LaunchCfg cfg = cfg_for(h, KN_ALGDIST, A->dtype, K, &G);
    TimedScope ts(h, "algdist_graph", (hipStream_t)stream);
    rc = launch_algdist(A->dtype, K, &G, X, w, target, mu, p, theta, fmask, strong, nstrong,
                        h->status, cfg, (hipStream_t)stream, A);
    return rc ? fail(h, rc, "algebraic_distance_graph launch") : AD_OK;
}

int ls_interp_search(ad_handle h, const ad_csr* A, int64_t nnz_g, const int32_t* row_ptr_g,
                     const int32_t* col_g, int32_t K, const void* X, const double* w,
                     const uint8_t* cf, int32_t caliber, double gamma, int32_t target,
                     int32_t* P_col, double* P_val, double* ls_val, int32_t* row_status,
                     void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if ((rc = check_pattern(h, A->n, nnz_g, row_ptr_g, col_g))) return rc;
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (caliber < 1 || caliber > 4)
        return fail(h, AD_ECALIBER, "caliber = %d outside [1, 4] for the set search", caliber);
    if (caliber > K)
        return fail(h, AD_ECALIBER, "caliber = %d > K = %d: LS rows would not be unique", caliber, K);
    if (!(gamma >= 0.0) || !(gamma < 1e6)) return fail(h, AD_EINVAL, "gamma = %g", gamma);
    if (target != AD_TARGET_PLAIN && target != AD_TARGET_RESIDUAL)
        return fail(h, AD_EINVAL, "target = %d", target);
    if ((rc = check_panel(h, X, "X", A->n))) return rc;
    if (A->n > 0 && (!cf || !P_col || !P_val || !ls_val || !row_status))
        return fail(h, AD_EINVAL, "null output or input array");
    if (A->n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    TimedScope ts(h, "ls_search", (hipStream_t)stream);
    rc = launch_ls_search(A->dtype, K, A, row_ptr_g, col_g, X, w, cf, caliber, gamma, target,
                          P_col, P_val, ls_val, row_status, h->status, (hipStream_t)stream);
    return rc ? fail(h, rc, "ls_interp_search launch") : AD_OK;
}

int relax_algdist_batched(ad_handle h, int32_t nmat, const ad_csr* As, int32_t K, uint64_t seed,
                          int32_t relax, int32_t sweeps, double omega, const double* w, void* X,
                          void* mu, double theta, uint8_t* strong, int32_t* nstrong,
                          void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    if (nmat < 1 || !As) return fail(h, AD_EINVAL, "nmat = %d or As is NULL", nmat);
    if (relax == AD_MULTICOLOR_GS)
        return fail(h, AD_EUNSUPPORTED,
                    "the batched path relaxes by damped Jacobi only (a batch carries no colouring)");
    if (relax != AD_JACOBI) return fail(h, AD_EINVAL, "relax = %d", relax);
    int rc;
    int64_t rows = 0, ents = 0;
    for (int m = 0; m < nmat; ++m) {
        if ((rc = check_csr(h, &As[m]))) return fail(h, rc, "matrix %d: %s", m, h->err.c_str());
        if (As[m].dtype != As[0].dtype) return fail(h, AD_EDTYPE, "matrix %d has another dtype", m);
        rows += As[m].n;
        ents += As[m].nnz;
    }
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (sweeps < 0) return fail(h, AD_EINVAL, "sweeps = %d < 0", sweeps);
    if (rows * K > ((int64_t)1 << 40)) return fail(h, AD_ESTRUCT, "batch too large");
    if ((rc = check_panel(h, X, "X", (int)(rows > 0)))) return rc;
    if (ents > 0 && !mu) return fail(h, AD_EINVAL, "mu is NULL");
    if (strong && !(theta > 0.0 && theta < 1.0))
        return fail(h, AD_EINVAL, "theta = %g outside (0, 1)", theta);
    if (rows == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    const int dt = As[0].dtype;
    const int ks = k_slot(K), b = batch_bucket(nmat, As);
    const LaunchCfg cfg = h->has_tuned[KN_BATCHED][dt][ks][b] ? h->tuned[KN_BATCHED][dt][ks][b]
                                                               : LaunchCfg();
    const LaunchCfg dcfg = h->has_tuned[KN_BDIST][dt][ks][b] ? h->tuned[KN_BDIST][dt][ks][b]
                                                             : LaunchCfg();
    TimedScope ts(h, "batched", (hipStream_t)stream);
    rc = launch_batched(h, nmat, As, K, seed, sweeps, omega, w, X, mu, theta, strong, nstrong, cfg,
                        dcfg, h->timing, (hipStream_t)stream);
    return rc ? fail(h, rc, "relax_algdist_batched launch") : AD_OK;
}

static int loss_grad_impl(ad_handle h, const ad_csr* A, int32_t K, int32_t relax,
                          const int32_t* color, int32_t ncolors, const void* ckpt,
                          int32_t ckpt_every, int32_t sweeps, double omega, const double* w,
                          const uint8_t* cf, const int32_t* P_col, const double* P_val,
                          int32_t caliber, const void* X_final, const double* dL,
                          double* grad_val, double* grad_omega, double* grad_w, void* stream,
                          const char* name) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (A->dtype != AD_F64) return fail(h, AD_EDTYPE, "the backward pass is FP64 only");
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (relax != AD_JACOBI && relax != AD_MULTICOLOR_GS)
        return fail(h, AD_EINVAL, "relax = %d is neither AD_JACOBI nor AD_MULTICOLOR_GS", relax);
    if (relax == AD_MULTICOLOR_GS && (ncolors < 1 || ncolors > 64 || (A->n > 0 && !color)))
        return fail(h, AD_EINVAL, "colours: ncolors = %d, color %p", ncolors, (const void*)color);
    if (sweeps < 0) return fail(h, AD_EINVAL, "sweeps = %d < 0", sweeps);
    if (ckpt_every < 1) return fail(h, AD_EINVAL, "ckpt_every = %d < 1", ckpt_every);
    if (caliber < 1 || caliber > 8) return fail(h, AD_ECALIBER, "caliber = %d outside [1, 8]", caliber);
    if (caliber > K)
        return fail(h, AD_ECALIBER, "caliber = %d > K = %d: LS rows would not be unique", caliber, K);
    if (!dL) return fail(h, AD_EINVAL, "dL is NULL");
    if (A->n > 0 && (!ckpt || !X_final || !cf || !P_col || !P_val || !grad_val))
        return fail(h, AD_EINVAL, "null input or output array");
    if ((rc = check_panel(h, ckpt, "ckpt", A->n)) || (rc = check_panel(h, X_final, "X_final", A->n)))
        return rc;
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    if (A->n == 0) {
        if (grad_omega && (rc = launch_fill_f64(grad_omega, 1, 0.0, s))) return rc;
        if (grad_w && (rc = launch_fill_f64(grad_w, K, 0.0, s))) return rc;
        return AD_OK;
    }
    TimedScope ts(h, "ls_loss_backward", s);
    rc = launch_ls_loss_backward(h, K, A, relax, color, ncolors, ckpt, ckpt_every, sweeps, omega, w,
                                 cf, P_col, P_val, caliber, X_final, dL, grad_val, grad_omega,
                                 grad_w, s);
    return rc ? fail(h, rc, "%s launch", name) : AD_OK;
}

int ls_interp_loss_backward(ad_handle h, const ad_csr* A, int32_t K, const void* ckpt,
                            int32_t ckpt_every, int32_t sweeps, double omega, const double* w,
                            const uint8_t* cf, const int32_t* P_col, const double* P_val,
                            int32_t caliber, const void* X_final, const double* dL,
                            double* grad_val, double* grad_omega, void* stream) {
    if (h && !grad_omega) {
        h->err.clear();
        return fail(h, AD_EINVAL, "grad_omega is NULL");
    }
    return loss_grad_impl(h, A, K, AD_JACOBI, nullptr, 0, ckpt, ckpt_every, sweeps, omega, w, cf,
                          P_col, P_val, caliber, X_final, dL, grad_val, grad_omega, nullptr, stream,
                          "ls_interp_loss_backward");
}

int ls_interp_loss_grad(ad_handle h, const ad_csr* A, int32_t K, int32_t relax,
                        const int32_t* color, int32_t ncolors, const void* ckpt,
                        int32_t ckpt_every, int32_t sweeps, double omega, const double* w,
                        const uint8_t* cf, const int32_t* P_col, const double* P_val,
                        int32_t caliber, const void* X_final, const double* dL, double* grad_val,
                        double* grad_omega, double* grad_w, void* stream) {
    return loss_grad_impl(h, A, K, relax, color, ncolors, ckpt, ckpt_every, sweeps, omega, w, cf,
                          P_col, P_val, caliber, X_final, dL, grad_val, grad_omega, grad_w, stream,
                          "ls_interp_loss_grad");
}

}  // extern "C"

// ---------------------------------------------------------------- compatible relaxation
namespace {

// Device buffers of one synchronous call, freed on every return path.
struct DevBufs {
    std::vector<void*> p;
    ~DevBufs() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    T* get(size_t count) {
        void* q = nullptr;
        if (hipMalloc(&q, count ? count * sizeof(T) : 16) != hipSuccess) return nullptr;
        p.push_back(q);
        return (T*)q;
    }
};

// One CR run: nu F-relaxation sweeps from the constant start on the F rows
// of cf; U (n x 2, column 0 the CR vector) receives u^nu and norms (device,
// 3 doubles) |F|, sum_F u^2, max_F |u|.  rho (host) = eq:meas1's estimate.
int cr_run(ad_handle h, const ad_csr* A, const int32_t* color, int ncolors, const uint8_t* cf,
           int nu, int* fcol, void* U0, void* U, double* part, double* norms, unsigned* cstat,
           double* rho, double* hnorms, hipStream_t s) {
    const int n = A->n;
    int rc = launch_cr_start(A->dtype, n, color, cf, fcol, U0, s);
    if (rc) return rc;
    {
        TimedScope ts(h, "cr_relax", s);
        if ((rc = gs_sweeps(h, A, 2, 0, U0, nu, fcol, ncolors, U, nullptr, 0, s, cstat))) return rc;
    }
    {
        TimedScope ts(h, "cr_norms", s);
        if ((rc = launch_cr_norms(A->dtype, n, cf, U, part, norms, s))) return rc;
    }
    AD_HIP(hipMemcpyAsync(hnorms, norms, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    *rho = (hnorms[0] > 0.0) ? pow(sqrt(hnorms[1]) / sqrt(hnorms[0]), 1.0 / (double)nu) : 0.0;
    return AD_OK;
}

int check_cr_args(ad_handle h, const ad_csr* A, const int32_t* color, int32_t ncolors,
                  const uint8_t* cf, int32_t nu) {
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (ncolors < 1 || ncolors > 64) return fail(h, AD_EINVAL, "ncolors = %d outside [1, 64]", ncolors);
    if (A->n > 0 && (!color || !cf)) return fail(h, AD_EINVAL, "color or cf is NULL");
    if (nu < 1) return fail(h, AD_EINVAL, "nu = %d < 1", nu);
    return AD_OK;
}

}  // namespace

extern "C" {

int cr_rate(ad_handle h, const ad_csr* A, const int32_t* color, int32_t ncolors, const uint8_t* cf,
            int32_t nu, void* u, double* rho, double* norms, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_cr_args(h, A, color, ncolors, cf, nu);
    if (rc) return rc;
    if (!rho) return fail(h, AD_EINVAL, "rho is NULL");
    double hn[3] = {0.0, 0.0, 0.0};
    *rho = 0.0;
    if (A->n == 0) {
        if (norms) memcpy(norms, hn, sizeof hn);
        return AD_OK;
    }
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const int n = A->n;
    const size_t vs = dsize(A->dtype);
    DevBufs b;
    int* fcol = b.get<int>(n);
    char* U0 = b.get<char>((size_t)n * 2 * vs);
    char* U = b.get<char>((size_t)n * 2 * vs);
    double* part = b.get<double>(3 * (size_t)cr_norm_blocks(n));
    double* nd = b.get<double>(3);
    unsigned* cstat = b.get<unsigned>(1);
    if (!fcol || !U0 || !U || !part || !nd || !cstat) return fail(h, AD_ENOMEM, "cr_rate buffers");
    if ((rc = cr_run(h, A, color, ncolors, cf, nu, fcol, U0, U, part, nd, cstat, rho, hn, s)))
        return fail(h, rc, "cr_rate");
    if (u) {
        // column 0 of the n x 2 panel
        AD_HIP(hipMemcpy2DAsync(u, vs, U, 2 * vs, vs, (size_t)n, hipMemcpyDeviceToDevice, s));
        AD_HIP(hipStreamSynchronize(s));
    }
    if (norms) memcpy(norms, hn, sizeof hn);
    return AD_OK;
}

int cr_candidates(ad_handle h, int32_t n, int32_t dtype, const uint8_t* cf, const void* u,
                  double tol, uint8_t* z, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    if (n < 0) return fail(h, AD_EINVAL, "n = %d", n);
    if (dtype != AD_F32 && dtype != AD_F64) return fail(h, AD_EDTYPE, "dtype %d", dtype);
    if (n > 0 && (!cf || !u || !z)) return fail(h, AD_EINVAL, "cf, u or z is NULL");
    if (n == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    DevBufs b;
    double* part = b.get<double>(3 * (size_t)cr_norm_blocks(n));
    double* nd = b.get<double>(3);
    char* U2 = b.get<char>((size_t)n * 2 * dsize(dtype));
    if (!part || !nd || !U2) return fail(h, AD_ENOMEM, "cr_candidates buffers");
    // the norm pass reads column 0 of an n x 2 panel
    const size_t vs = dsize(dtype);
    AD_HIP(hipMemcpy2DAsync(U2, 2 * vs, u, vs, vs, (size_t)n, hipMemcpyDeviceToDevice, s));
    int rc = launch_cr_norms(dtype, n, cf, U2, part, nd, s);
    if (!rc) rc = launch_cr_candidates(dtype, n, cf, u, 1, nd, tol, z, s);
    if (rc) return fail(h, rc, "cr_candidates launch");
    AD_HIP(hipStreamSynchronize(s));
    return AD_OK;
}

int independent_set(ad_handle h, const ad_csr* A, const uint8_t* strong, const uint8_t* z,
                    uint64_t seed, uint8_t* sel, int64_t* count, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_structure(h, A);
    if (rc) return rc;
    if (A->n > 0 && (!z || !sel || (A->nnz > 0 && !strong)))
        return fail(h, AD_EINVAL, "strong, z or sel is NULL");
    int64_t cnt = 0;
    if (A->n > 0) {
        AD_HIP(hipSetDevice(h->device));
        hipStream_t s = (hipStream_t)stream;
        const int n = A->n;
        const int64_t nnz = A->nnz;
        DevBufs b;
        int* cnt_c = b.get<int>(n);
        int64_t* cp = b.get<int64_t>((size_t)n + 1);
        int64_t* sc = (int64_t*)b.get<char>((size_t)scan_workspace_bytes(n));
        int* trow = b.get<int>((size_t)nnz);
        int* tent = b.get<int>((size_t)nnz);
        MisKey* key = b.get<MisKey>(n);
        int8_t* state = b.get<int8_t>(n);
        int* left = b.get<int>(1);
        if (!cnt_c || !cp || !sc || !trow || !tent || !key || !state || !left)
            return fail(h, AD_ENOMEM, "independent_set buffers");
        TimedScope ts(h, "independent_set", s);
        if ((rc = launch_csc_index(n, nnz, A->row_ptr, A->col, nullptr, cnt_c, cp, sc, trow, tent,
                                   nullptr, h->status, s)) ||
            (rc = run_independent_set(n, A->row_ptr, A->col, strong, cp, trow, tent,
                                      (const int*)sc, z, seed, key, state, left, sel, nullptr,
                                      &cnt, s)))
            return fail(h, rc, "independent_set");
    }
    if (count) *count = cnt;
    return AD_OK;
}

// Algorithm 1 with the strength graph and the independent set on the
// pattern G (nnz_g entries; mu per entry of G); CR relaxes with A.
static int cr_coarsening_on(ad_handle h, const ad_csr* A, int64_t nnz_g, const int32_t* rpg,
                            const int32_t* cig, const int32_t* color, int32_t ncolors,
                            const void* mu, double theta, int32_t nu, double delta,
                            int32_t max_stages, uint64_t seed, uint8_t* cf, double* rho,
                            int64_t* ncoarse, int32_t* nstages, void* stream) {
    int rc;
    if (!(theta > 0.0 && theta < 1.0)) return fail(h, AD_EINVAL, "theta = %g outside (0, 1)", theta);
    if (!(delta >= 0.0)) return fail(h, AD_EINVAL, "delta = %g", delta);
    if (max_stages < 0) return fail(h, AD_EINVAL, "max_stages = %d", max_stages);
    if (!rho || !ncoarse || !nstages) return fail(h, AD_EINVAL, "rho, ncoarse or nstages is NULL");
    if (nnz_g > 0 && !mu) return fail(h, AD_EINVAL, "mu is NULL");
    *nstages = 0;
    if (A->n == 0) {
        rho[0] = 0.0;
        ncoarse[0] = 0;
        return AD_OK;
    }
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const int n = A->n;
    const int64_t nnz = nnz_g;
    const ad_csr Gp{n, nnz_g, rpg, cig, nullptr, A->dtype};  // pattern only
    const size_t vs = dsize(A->dtype);
    DevBufs b;
    int* fcol = b.get<int>(n);
    char* U0 = b.get<char>((size_t)n * 2 * vs);
    char* U = b.get<char>((size_t)n * 2 * vs);
    double* part = b.get<double>(3 * (size_t)cr_norm_blocks(n));
    double* nd = b.get<double>(3);
    unsigned* cstat = b.get<unsigned>(1);
    uint8_t* z = b.get<uint8_t>(n);
    uint8_t* fm = b.get<uint8_t>(n);
    uint8_t* strong = b.get<uint8_t>((size_t)nnz);
    int* cnt_c = b.get<int>(n);
    int64_t* cp = b.get<int64_t>((size_t)n + 1);
    int64_t* sc = (int64_t*)b.get<char>((size_t)scan_workspace_bytes(n));
    int* trow = b.get<int>((size_t)nnz);
    int* tent = b.get<int>((size_t)nnz);
    MisKey* key = b.get<MisKey>(n);
    int8_t* state = b.get<int8_t>(n);
    int* left = b.get<int>(1);
    if (!fcol || !U0 || !U || !part || !nd || !cstat || !z || !fm || !strong || !cnt_c || !cp ||
        !sc || !trow || !tent || !key || !state || !left)
        return fail(h, AD_ENOMEM, "cr_coarsening buffers");
    {
        TimedScope ts(h, "cr_index", s);
        if ((rc = launch_csc_index(n, nnz, rpg, cig, nullptr, cnt_c, cp, sc, trow, tent, nullptr,
                                   h->status, s)))
            return fail(h, rc, "cr_coarsening: column index");
    }
    double r = 0.0, hn[3];
    if ((rc = cr_run(h, A, color, ncolors, cf, nu, fcol, U0, U, part, nd, cstat, &r, hn, s)))
        return fail(h, rc, "cr_coarsening: CR run");
    int64_t nc = n - (int64_t)hn[0];
    rho[0] = r;
    ncoarse[0] = nc;
    int stage = 0;
    while (r > delta && stage < max_stages) {
        {
            TimedScope ts(h, "cr_select", s);
            if ((rc = launch_cr_candidates(A->dtype, n, cf, U, 2, nd, 1.0 - r, z, s)) ||
                (rc = launch_cr_fmask(n, cf, fm, s)) ||
                (rc = launch_strength(A->dtype, &Gp, mu, theta, fm, strong, nullptr, s)))
                return fail(h, rc, "cr_coarsening: candidates / strength");
        }
        int64_t added = 0;
        {
            TimedScope ts(h, "independent_set", s);
            if ((rc = run_independent_set(n, rpg, cig, strong, cp, trow, tent, (const int*)sc, z,
                                          seed + (uint64_t)stage, key, state, left, nullptr, cf,
                                          &added, s)))
                return fail(h, rc, "cr_coarsening: independent set");
        }
        if (added == 0) break;  // no candidate: nothing can grow C
        ++stage;
        if ((rc = cr_run(h, A, color, ncolors, cf, nu, fcol, U0, U, part, nd, cstat, &r, hn, s)))
            return fail(h, rc, "cr_coarsening: CR run");
        nc += added;
        rho[stage] = r;
        ncoarse[stage] = nc;
    }
    *nstages = stage;
    return AD_OK;
}


int cr_coarsening(ad_handle h, const ad_csr* A, const int32_t* color, int32_t ncolors,
                  const void* mu, double theta, int32_t nu, double delta, int32_t max_stages,
                  uint64_t seed, uint8_t* cf, double* rho, int64_t* ncoarse, int32_t* nstages,
                  void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_cr_args(h, A, color, ncolors, cf, nu);
    if (rc) return rc;
    return cr_coarsening_on(h, A, A->nnz, A->row_ptr, A->col, color, ncolors, mu, theta, nu, delta,
                            max_stages, seed, cf, rho, ncoarse, nstages, stream);
}

int cr_coarsening_graph(ad_handle h, const ad_csr* A, int64_t nnz_g, const int32_t* row_ptr_g,
                        const int32_t* col_g, const int32_t* color, int32_t ncolors,
                        const void* mu_g, double theta, int32_t nu, double delta,
                        int32_t max_stages, uint64_t seed, uint8_t* cf, double* rho,
                        int64_t* ncoarse, int32_t* nstages, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_cr_args(h, A, color, ncolors, cf, nu);
    if (rc) return rc;
    if ((rc = check_pattern(h, A->n, nnz_g, row_ptr_g, col_g))) return rc;
    return cr_coarsening_on(h, A, nnz_g, row_ptr_g, col_g, color, ncolors, mu_g, theta, nu, delta,
                            max_stages, seed, cf, rho, ncoarse, nstages, stream);
}

}  // extern "C"

// ---------------------------------------------------------------- Galerkin operator, two-grid
namespace {

int check_interp(ad_handle h, const ad_csr* A, int32_t caliber, const int32_t* P_col,
                 const double* P_val, const uint8_t* cf) {
    int rc = check_csr(h, A);
    if (rc) return rc;
    if (caliber < 1 || caliber > 64) return fail(h, AD_ECALIBER, "caliber = %d outside [1, 64]", caliber);
    if (A->n > 0 && (!P_col || !P_val || !cf)) return fail(h, AD_EINVAL, "P_col, P_val or cf is NULL");
    if ((int64_t)A->n * caliber > INT32_MAX)
        return fail(h, AD_EUNSUPPORTED, "n * caliber beyond int32");
    return AD_OK;
}

struct GalerkinCtx {
    DevBufs b;
    GalerkinIn g;
    GalerkinWork w;
    bool ok = false;
    GalerkinCtx(const ad_csr* A, int32_t caliber, const int32_t* P_col, const double* P_val,
                const uint8_t* cf) {
        const int n = A->n;
        g = GalerkinIn{n, A->row_ptr, A->col, A->val, A->dtype, caliber, P_col, P_val, cf};
        w.flags = b.get<int>(n);
        w.scan = b.get<int64_t>((size_t)n + 1);
        w.scan_tmp = (int64_t*)b.get<char>((size_t)scan_workspace_bytes(n));
        w.cidx = b.get<int>(n);
        w.cnt = b.get<int>(n);
        w.pt = b.get<int64_t>((size_t)n + 1);
        w.ptkey = b.get<int64_t>((size_t)n * caliber);
        w.maxslots = b.get<int>(1);
        w.spill = b.get<int>(n);
        w.nspill = b.get<int>(1);
        ok = w.flags && w.scan && w.scan_tmp && w.cidx && w.cnt && w.pt && w.ptkey && w.maxslots &&
             w.spill && w.nspill;
    }
};

}  // namespace

extern "C" {

int galerkin_rows(ad_handle h, const ad_csr* A, int32_t caliber, const int32_t* P_col,
                  const double* P_val, const uint8_t* cf, int32_t* nc, int32_t* row_ptr_c,
                  int64_t* nnz_c, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_interp(h, A, caliber, P_col, P_val, cf);
    if (rc) return rc;
    if (!nc || !nnz_c || !row_ptr_c) return fail(h, AD_EINVAL, "nc, row_ptr_c or nnz_c is NULL");
    *nc = 0;
    *nnz_c = 0;
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    if (A->n == 0) return launch_fill_i32(row_ptr_c, 1, 0, s);
    GalerkinCtx c(A, caliber, P_col, P_val, cf);
    if (!c.ok) return fail(h, AD_ENOMEM, "galerkin_rows buffers");
    int ncl = 0;
    TimedScope ts(h, "galerkin", s);
    if ((rc = galerkin_prepare(c.g, c.w, &ncl, s)) ||
        (rc = galerkin_transpose(c.g, c.w, ncl, h->status, s)))
        return fail(h, rc, "galerkin_rows: coarse numbering / transpose");
    rc = galerkin_rows_run(c.g, c.w, ncl, row_ptr_c, nnz_c, s);
    if (rc == AD_EUNSUPPORTED)
        return fail(h, rc, "galerkin_rows: a coarse row has more than 64 contributing fine rows or "
                           "2048 products, or the operator has more than 2^31 entries");
    if (rc) return fail(h, rc, "galerkin_rows");
    *nc = ncl;
    return AD_OK;
}

int galerkin_cols(ad_handle h, const ad_csr* A, int32_t caliber, const int32_t* P_col,
                  const double* P_val, const uint8_t* cf, int32_t nc, const int32_t* row_ptr_c,
                  int32_t* col_c, double* val_c, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_interp(h, A, caliber, P_col, P_val, cf);
    if (rc) return rc;
    if (nc < 0 || nc > A->n) return fail(h, AD_EINVAL, "nc = %d", nc);
    if (nc > 0 && (!row_ptr_c || !col_c || !val_c))
        return fail(h, AD_EINVAL, "row_ptr_c, col_c or val_c is NULL");
    if (nc == 0) return AD_OK;
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    GalerkinCtx c(A, caliber, P_col, P_val, cf);
    if (!c.ok) return fail(h, AD_ENOMEM, "galerkin_cols buffers");
    int ncl = 0;
    TimedScope ts(h, "galerkin", s);
    if ((rc = galerkin_prepare(c.g, c.w, &ncl, s)) ||
        (rc = galerkin_transpose(c.g, c.w, ncl, h->status, s)))
        return fail(h, rc, "galerkin_cols: coarse numbering / transpose");
    if (ncl != nc) return fail(h, AD_EINVAL, "nc = %d but cf marks %d coarse points", nc, ncl);
    if ((rc = galerkin_cols_run(c.g, c.w, nc, row_ptr_c, col_c, val_c, s)))
        return fail(h, rc, "galerkin_cols");
    AD_HIP(hipStreamSynchronize(s));
    return AD_OK;
}

int two_grid_rate(ad_handle h, const ad_csr* A, const int32_t* color, int32_t ncolors,
                  int32_t caliber, const int32_t* P_col, const double* P_val, const uint8_t* cf,
                  int32_t nc, const int32_t* row_ptr_c, const int32_t* col_c, const double* val_c,
                  int32_t K, const void* E0, int32_t iters, int32_t pre, int32_t post,
                  double* hist, double* rho, void* stream) {
    if (!h) return AD_EINVAL;
    h->err.clear();
    int rc = check_interp(h, A, caliber, P_col, P_val, cf);
    if (rc) return rc;
    if (A->dtype != AD_F64) return fail(h, AD_EDTYPE, "the two-grid method runs in FP64");
    if (!k_ok(K)) return fail(h, AD_EINVAL, "K = %d: must be 2, 4, 8, 16, 32 or 64", K);
    if (ncolors < 1 || ncolors > 64 || (A->n > 0 && !color))
        return fail(h, AD_EINVAL, "colours: ncolors = %d, color %p", ncolors, (const void*)color);
    if (iters < 1 || pre < 0 || post < 0)
        return fail(h, AD_EINVAL, "iters = %d, pre = %d, post = %d", iters, pre, post);
    if (!rho) return fail(h, AD_EINVAL, "rho is NULL");
    if (nc < 1 || nc > kCoarseSolveMax || nc > A->n)
        return fail(h, AD_EUNSUPPORTED, "nc = %d outside [1, %d] (dense coarse solve)", nc,
                    kCoarseSolveMax);
    if (!row_ptr_c || !col_c || !val_c) return fail(h, AD_EINVAL, "coarse operator is NULL");
    if ((rc = check_panel(h, E0, "E0", A->n))) return rc;
    AD_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const int n = A->n;
    const size_t panel = (size_t)n * K;
    GalerkinCtx c(A, caliber, P_col, P_val, cf);
    double* E[2] = {c.b.get<double>(panel), c.b.get<double>(panel)};
    double* R = c.b.get<double>(panel);
    double* Rc = c.b.get<double>((size_t)nc * K);
    double* L = c.b.get<double>((size_t)nc * nc);
    double* Li = c.b.get<double>((size_t)nc * nc);
    double* LiT = c.b.get<double>((size_t)nc * nc);
    double* Wblk = (double*)c.b.get<char>(coarse_factor_workspace(nc));
    int* bad = c.b.get<int>(1);
    const int nb = two_grid_blocks(n, K);
    double* part = c.b.get<double>((size_t)nb * K);
    double* hd = c.b.get<double>((size_t)(iters + 1) * K);
    if (!c.ok || !E[0] || !E[1] || !R || !Rc || !L || !Li || !LiT || !Wblk || !bad || !part ||
        !hd)
        return fail(h, AD_ENOMEM, "two_grid_rate buffers");
    int ncl = 0;
    if ((rc = galerkin_prepare(c.g, c.w, &ncl, s)) ||
        (rc = galerkin_transpose(c.g, c.w, ncl, h->status, s)))
        return fail(h, rc, "two_grid_rate: coarse numbering / transpose");
    if (ncl != nc) return fail(h, AD_EINVAL, "nc = %d but cf marks %d coarse points", nc, ncl);
    {
        TimedScope ts(h, "coarse_factor", s);
        if ((rc = coarse_factor(nc, row_ptr_c, col_c, val_c, L, Li, LiT, Wblk, bad, s)))
            return fail(h, rc, "two_grid_rate: coarse factorisation");
    }
    int hbad = 0;
    AD_HIP(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    if (hbad) return fail(h, AD_ESTRUCT, "two_grid_rate: the coarse operator is not positive definite");
    AD_HIP(hipMemcpyAsync(E[0], E0, panel * sizeof(double), hipMemcpyDeviceToDevice, s));
    int cur = 0;
    if ((rc = a_norms_sq(c.g, K, E[0], part, hd, s))) return fail(h, rc, "two_grid_rate: norms");
    for (int it = 0; it < iters; ++it) {
        TimedScope ts(h, "two_grid_cycle", s);
        if (pre > 0) {
            if ((rc = gs_sweeps(h, A, K, 0, E[cur], pre, color, ncolors, E[cur ^ 1], nullptr, 0, s)))
                return fail(h, rc, "two_grid_rate: pre-smoothing");
            cur ^= 1;
        }
        if ((rc = coarse_correction(c.g, c.w, nc, K, Li, LiT, E[cur], R, Rc, s)))
            return fail(h, rc, "two_grid_rate: coarse-grid correction");
        if (post > 0) {
            if ((rc = gs_sweeps(h, A, K, 0, E[cur], post, color, ncolors, E[cur ^ 1], nullptr, 0, s)))
                return fail(h, rc, "two_grid_rate: post-smoothing");
            cur ^= 1;
        }
        if ((rc = a_norms_sq(c.g, K, E[cur], part, hd + (size_t)(it + 1) * K, s)))
            return fail(h, rc, "two_grid_rate: norms");
    }
    std::vector<double> hh((size_t)(iters + 1) * K);
    AD_HIP(hipMemcpyAsync(hh.data(), hd, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    for (double& v : hh) v = sqrt(v > 0.0 ? v : 0.0);
    for (int k = 0; k < K; ++k) {
        const double a = hh[(size_t)iters * K + k], b = hh[(size_t)(iters - 1) * K + k];
        rho[k] = b > 0.0 ? a / b : 0.0;
    }
    if (hist) memcpy(hist, hh.data(), hh.size() * sizeof(double));
    return AD_OK;
}

}  // extern "C"
