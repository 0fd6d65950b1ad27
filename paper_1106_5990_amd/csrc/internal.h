// internal.h -- host-side internals of libalgdist: the handle, its
// workspace, launch wrappers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>
#include <vector>

#include "algdist.h"
#include "device.h"

// One timed launch: HIP events recorded on the launch stream around it.
struct ad_timed_launch {
    const char* label;
    hipEvent_t a, b;
};

namespace ad {
// Launch knobs picked per call (the autotuner may override them).
struct LaunchCfg {
    int lpr = 0;      // lanes per row (0: the shape's default)
    int iter = 1;     // row-block steps per workgroup (rows per lane group per tile)
    int xcd_map = 1;  // 1: XCD-contiguous tile mapping
};
enum KernelId {
    KN_JACOBI = 0,
    KN_GS = 1,
    KN_ALGDIST = 2,
    KN_LS = 3,
    KN_BATCHED = 4,
    KN_DLS = 5,    // fused distances + LS rows
    KN_BDIST = 6,  // distance stage of the batched path
    KN_COUNT = 7
};
constexpr int kNumKSlots = 7;   // log2(K) for K = 2 .. 64
constexpr int kNumBuckets = 4;  // stored entries per row: < 8, < 16, < 32, >= 32
}  // namespace ad

struct ad_handle_s {
    int device = 0;
    unsigned* status = nullptr;  // sticky device status word
    void* ws = nullptr;          // workspace (grown on demand)
    size_t ws_bytes = 0;
    // true once a call has run while its stream was capturing: a caller's
    // graph may then refer to the current workspace, which is kept alive
    // (moved to `retired`) instead of being freed when it must grow
    bool ws_pinned = false;
    std::vector<void*> retired;  // device buffers freed by algdist_destroy
    std::string err;
    int cu_count = 256;
    // per-kernel timing (algdist_timing / algdist_timing_report)
    bool timing = false;
    std::vector<ad_timed_launch> timed;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
    std::string report;
    // launch configurations set by algdist_set_launch / algdist_autotune
    ad::LaunchCfg tuned[ad::KN_COUNT][2][ad::kNumKSlots][ad::kNumBuckets];
    bool has_tuned[ad::KN_COUNT][2][ad::kNumKSlots][ad::kNumBuckets] = {};
    void* batch = nullptr;  // state of the batched path (batched.hip)
};

namespace ad {

int k_slot(int K);                  // log2(K), or -1
int nnz_bucket(int64_t nnz, int n);  // 0..kNumBuckets-1
LaunchCfg cfg_for(ad_handle h, int kernel, int dtype, int K, const ad_csr* A);

// Compile-time dispatch over the supported K and lanes-per-row shapes.
template <typename T, typename F>
int with_k(int K, F&& f) {
    switch (K) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 32: return f(std::integral_constant<int, 32>{});
        case 64: return f(std::integral_constant<int, 64>{});
        default: return AD_EINVAL;
    }
}

template <typename T, int K, typename F>
int with_lpr(int lpr, F&& f) {
    if (lpr <= 0) lpr = lpr_default<T>(K);
#define AD_LPR_CASE(L)                                                   \
    case L:                                                              \
        if constexpr (lpr_ok<T>(K, L)) {                                 \
            f(std::integral_constant<int, L>{});                         \
            return AD_OK;                                                \
        } else {                                                         \
            return AD_EINVAL;                                            \
        }
    switch (lpr) {
        AD_LPR_CASE(1)
        AD_LPR_CASE(2)
        AD_LPR_CASE(4)
        AD_LPR_CASE(8)
        AD_LPR_CASE(16)
        AD_LPR_CASE(32)
        AD_LPR_CASE(64)
        default: return AD_EINVAL;
    }
#undef AD_LPR_CASE
}

// Workspace carve-up helper: returns aligned sub-buffers of the handle's
// workspace, growing it first if needed (growth synchronises the device).
struct WsReq {
    size_t off = 0;
    size_t add(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};
// Grows the workspace to at least `bytes`.  While `s` is capturing, growth
// is refused (AD_EUNSUPPORTED: a captured graph must not see its buffers
// move), and the current buffer is marked as referenced by a graph; a buffer
// so marked is retired, not freed, when a later uncaptured call grows it.
int ws_reserve(ad_handle h, size_t bytes, hipStream_t s);
// true when `s` is capturing into a graph
bool stream_capturing(hipStream_t s);

// Records HIP events around the launches made in its lifetime when the
// handle's timing is on (no-op otherwise).
class TimedScope {
   public:
    TimedScope(ad_handle h, const char* label, hipStream_t s);
    ~TimedScope();

   private:
    ad_handle h_;
    const char* label_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
};

// ---- util.hip
int launch_fill_f64(double* p, int64_t m, double v, hipStream_t s);
int launch_fill_i32(int32_t* p, int64_t m, int32_t v, hipStream_t s);
// out[0] = 0, out[q + 1] = cnt[0] + ... + cnt[q] (q < m); tmp holds
// scan_workspace_bytes(m) bytes
int64_t scan_workspace_bytes(int64_t m);
int launch_excl_scan(const int32_t* cnt, int64_t m, int64_t* out, int64_t* tmp, hipStream_t s);
int launch_narrow_i64(const int64_t* a, int64_t m, int32_t* b, hipStream_t s);

// ---- relax.hip
int launch_tv_init(int dtype, int64_t row0, int64_t nrows, int K, uint64_t seed, void* X,
                   hipStream_t s);
int launch_jacobi(int dtype, int K, const ad_csr* A, const void* Xin, void* Xout, double omega,
                  unsigned* status, const LaunchCfg& cfg, hipStream_t s);
// Builds the colour-sorted row list: rowlist[n], its inverse inv[n] (may be
// NULL) and seg[ncolors + 2]
// (seg[c]..seg[c+1] are the rows of colour c; seg[ncolors]..seg[ncolors+1]
// the rows with an invalid colour).  With rpp (n + 1 ints, may be NULL) it
// also writes the row pointers of the colour-major copy of the CSR whose
// row pointers are rp.  counts: 2 * (ncolors+1) * nblocks ints.
int launch_color_partition(int n, const int32_t* color, int ncolors, const int32_t* rp,
                           int32_t* rowlist, int32_t* inv, int32_t* seg, int32_t* counts,
                           int nblocks, int32_t* rpp, unsigned* status, hipStream_t s);
int color_partition_blocks(int n);
// Colour-major copy of a CSR for the colour phases: permuted row p is natural
// row rowlist[p]; its entries rpp[p]..rpp[p+1] keep their CSR order with
// columns mapped to permuted indices (colpp) and values copied (valpp).
struct PermCsr {
    int n;
    const int32_t* rowlist;  // n
    const int32_t* seg;      // ncolors + 2
    const int32_t* rpp;      // n + 1
    const int32_t* colpp;    // nnz
    const void* valpp;       // nnz values of the CSR's dtype
};
int launch_perm_setup(int dtype, const ad_csr* A, PermCsr& P, int32_t* inv, hipStream_t s,
                      int K = 0, uint64_t seed = 0, void* Xp = nullptr);
int launch_gs_phase_perm(int dtype, int K, const PermCsr& P, int c, int ncolors, const void* Xold,
                         void* Xnew, void* Xnat, int write_perm, unsigned* status,
                         const LaunchCfg& cfg, hipStream_t s);
int launch_start_perm(int dtype, int n, int K, const int32_t* rowlist, uint64_t seed,
                      const void* X0, void* Xp, hipStream_t s);
int launch_unpermute(int dtype, int n, int K, const int32_t* rowlist, const void* Xp, void* X,
                     hipStream_t s);

// ---- distance.hip
// true when algebraic_distance runs the edge-parallel kernel: default lanes
// per row (cfg.lpr <= 0), plain target, panel rows of at most 128 bytes.
bool algdist_uses_edge(int dtype, int K, int target, const LaunchCfg& cfg);
// Distances over the entries of A; the residual target is formed from At
// (NULL: A itself; another matrix when A is only a pattern, e.g. of A^d).
int launch_algdist(int dtype, int K, const ad_csr* A, const void* X, const double* w, int target,
                   void* mu, double* p, double theta, const uint8_t* fmask, uint8_t* strong,
                   int32_t* nstrong, unsigned* status, const LaunchCfg& cfg, hipStream_t s,
                   const ad_csr* At = nullptr);
int launch_strength(int dtype, const ad_csr* A, const void* mu, double theta,
                    const uint8_t* fmask, uint8_t* strong, int32_t* nstrong, hipStream_t s);
int launch_csr_validate(const ad_csr* A, unsigned* status, hipStream_t s);

// ---- interp.hip
int launch_ls_interp(int dtype, int K, int caliber, const ad_csr* A, const void* X,
                     const double* w, const uint8_t* cf, const void* mu, int target,
                     int32_t* P_col, double* P_val, double* ls_val, int32_t* row_status,
                     double* block_sums, double* ls_sum, unsigned* status,
                     const LaunchCfg& cfg, hipStream_t s);
int ls_interp_blocks(int dtype, int K, int n, const LaunchCfg& cfg);
int launch_dist_ls(int dtype, int K, int caliber, const ad_csr* A, const void* X, const double* w,
                   int target, void* mu, double theta, const uint8_t* fmask, uint8_t* strong,
                   int32_t* nstrong, const uint8_t* cf, int32_t* P_col, double* P_val,
                   double* ls_val, int32_t* row_status, double* block_sums, double* ls_sum,
                   unsigned* status, const LaunchCfg& cfg, hipStream_t s);
int dist_ls_blocks(int dtype, int K, int n, const LaunchCfg& cfg);

// ---- longrange.hip
// Row pointers of the pattern of A^d into rpd (n + 1 ints) from the
// structure of A; *host_tot receives the entry count and *host_bad a
// nonzero value (1: a row over the per-row cap, 2: past int32) -- both after
// synchronising s.  ws: pow_rows_workspace(n) bytes.
size_t pow_rows_workspace(int n);
int launch_pow_rows(int n, int d, const int* rp, const int* ci, int* rpd, void* ws,
                    int64_t* host_tot, int* host_bad, hipStream_t s);
int launch_pow_cols(int n, int d, const int* rp, const int* ci, const int* rpd, int* cid,
                    unsigned* status, hipStream_t s);
int launch_ls_search(int dtype, int K, const ad_csr* A, const int* rpg, const int* cig,
                     const void* X, const double* w, const uint8_t* cf, int caliber, double gamma,
                     int target, int32_t* P_col, double* P_val, double* ls_val,
                     int32_t* row_status, unsigned* status, hipStream_t s);

// ---- autotune.hip
int autotune(ad_handle h, const ad_csr* A, int K, int relax, const int32_t* color, int ncolors,
             const uint8_t* cf, int caliber, const char* cache, hipStream_t s);

// ---- batched.hip
int launch_batched(ad_handle h, int nmat, const ad_csr* As, int K, uint64_t seed, int sweeps,
                   double omega, const double* w, void* X, void* mu, double theta,
                   uint8_t* strong, int32_t* nstrong, const LaunchCfg& cfg,
                   const LaunchCfg& dcfg, bool direct, hipStream_t s);
void batch_state_free(ad_handle h);
int autotune_batched(ad_handle h, int nmat, const ad_csr* As, int K, int sweeps, const char* cache,
                     hipStream_t s);
int batch_bucket(int nmat, const ad_csr* As);

// ---- api.hip
// Colour-phase sweeps of setup_testvectors (arguments checked by the caller);
// color_status (null: the handle's) receives the partition's bad-colour flag.
int gs_sweeps(ad_handle h, const ad_csr* A, int K, uint64_t seed, const void* X0, int sweeps,
              const int32_t* color, int ncolors, void* X, void* ckpt, int ckpt_every,
              hipStream_t s, unsigned* color_status = nullptr);

// ---- coarsen.hip
int cr_norm_blocks(int n);
int launch_cr_start(int dtype, int n, const int* color, const uint8_t* cf, int* fcol, void* U0,
                    hipStream_t s);
int launch_cr_fmask(int n, const uint8_t* cf, uint8_t* fm, hipStream_t s);
int launch_cr_norms(int dtype, int n, const uint8_t* cf, const void* U, double* part,
                    double* norms, hipStream_t s);
int launch_cr_candidates(int dtype, int n, const uint8_t* cf, const void* U, int stride,
                         const double* norms, double tol, uint8_t* z, hipStream_t s);
// priority of a vertex in the independent set: (lam, h, index), loaded
// as one 16-byte record
struct alignas(16) MisKey {
    uint64_t h;
    int lam;
    int pad;
};
// asym: the flag launch_csc_index left (0: the pattern is structurally
// symmetric and column i lists row i's columns in order)
int run_independent_set(int n, const int* rp, const int* ci, const uint8_t* strong,
                        const int64_t* cp, const int* trow, const int* tent, const int* asym,
                        const uint8_t* z, uint64_t seed, MisKey* key, int8_t* state, int* left,
                        uint8_t* sel, uint8_t* cf, int64_t* count, hipStream_t s);

// ---- galerkin.hip
struct GalerkinIn {
    int n;
    const int* rp;
    const int* ci;
    const void* av;
    int dtype;
    int cal;
    const int* Pc;     // n x cal fine column indices, -1 padded
    const double* Pv;  // n x cal weights
    const uint8_t* cf;
};
struct GalerkinWork {
    int* flags;         // n
    int64_t* scan;      // n + 1 (also the coarse row counts' scan)
    int64_t* scan_tmp;  // scan_workspace_bytes(n)
    int* cidx;          // n
    int* cnt;           // n
    int64_t* pt;        // n + 1
    int64_t* ptkey;     // n * cal
    int* maxslots;      // 1
    int* spill;         // n: coarse rows left to the sort kernel
    int* nspill;        // 1
};
int galerkin_prepare(const GalerkinIn& g, GalerkinWork& w, int* nc_out, hipStream_t s);
int galerkin_transpose(const GalerkinIn& g, GalerkinWork& w, int nc, unsigned* status,
                       hipStream_t s);
int galerkin_rows_run(const GalerkinIn& g, GalerkinWork& w, int nc, int* rpc, int64_t* nnz_c,
                      hipStream_t s);
int galerkin_cols_run(const GalerkinIn& g, GalerkinWork& w, int nc, const int* rpc, int* colc,
                      double* valc, hipStream_t s);
size_t coarse_factor_workspace(int nc);  // bytes of coarse_factor's Wblk
int coarse_factor(int nc, const int* rpc, const int* colc, const double* valc, double* L,
                  double* Li, double* LiT, double* Wblk, int* bad, hipStream_t s);
int coarse_correction(const GalerkinIn& g, const GalerkinWork& w, int nc, int K, const double* Li,
                      const double* LiT, double* E, double* R, double* Rc, hipStream_t s);
int a_norms_sq(const GalerkinIn& g, int K, const double* E, double* part, double* out,
               hipStream_t s);
int two_grid_blocks(int n, int K);
constexpr int kCoarseSolveMax = 8192;

// ---- adjoint.hip
int launch_csc_index(int n, int64_t nnz, const int* rp, const int* ci, const double* av, int* cnt,
                     int64_t* cp, int64_t* sc, int* trow, int* tent, double* diag,
                     unsigned* status, hipStream_t s);
int launch_ls_loss_backward(ad_handle h, int K, const ad_csr* A, int relax, const int32_t* color,
                            int ncolors, const void* ckpt, int ce, int sweeps, double omega,
                            const double* w, const uint8_t* cf, const int32_t* P_col,
                            const double* P_val, int cal, const void* X_final, const double* dL,
                            double* grad_val, double* grad_omega, double* grad_w, hipStream_t s);

inline int grid_for_tiles(int64_t ntiles, int mode) {
    if (ntiles < 1) ntiles = 1;
    if (mode <= 0) return (int)ntiles;
    const int64_t span = mode == 1 ? 8 : 8 * (int64_t)mode;
    return (int)(span * ((ntiles + span - 1) / span));
}

}  // namespace ad

#define AD_HIP(call)                                       \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return AD_EDEVICE;           \
    } while (0)
