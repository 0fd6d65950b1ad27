// batched.hip -- many matrices through test-vector start, damped-Jacobi
// relaxation and the fused distance/strength step in ONE persistent launch.
//
// The host turns the batch into a task list, largest matrices first:
//   * a matrix of at most kWholeTiles tiles is one task: a single workgroup
//     runs its start, all sweeps and its distances, separated only by
//     workgroup barriers, while its panel and CSR stay in L2;
//   * a larger matrix is split into row tiles and contributes one task per
//     (stage, tile), stage 0 = start, 1..S = sweeps, S+1 = distances; a tile
//     of stage s waits until every tile of stage s-1 of the same matrix has
//     signalled completion on a per-(matrix, stage) counter.
// Workgroups take tasks from one atomic ticket in list order.  Every
// dependency of a task precedes it in that order, and a task is taken only
// by a running workgroup, so the earliest unfinished task can always
// proceed: the grid drains without any co-residency assumption.  Every wait
// is bounded (a spin limit that sets AD_STAT_TIMEOUT and gives up), so the
// kernel always exits.  Counters are cleared by a fill kernel launched just
// before it (both captured in a HIP graph for repeated calls).
//
// The rows are computed by the same per-row code as the single-matrix
// kernels (rowops.h), so a batch gives bitwise the results of running the
// block-diagonal concatenation of its matrices through those kernels.
#include <string.h>

#include <algorithm>
#include <vector>

#include "device.h"
#include "internal.h"
#include "rowops.h"

namespace ad {

constexpr int kWholeTiles = 4;       // matrices with <= this many tiles run whole
constexpr int kSpinLimit = 1 << 20;  // bounded wait: well under a second

struct BatchMat {
    const int* rp;
    const int* ci;
    const void* av;
    int n;
    int ntiles;
    int64_t row0;  // first row of the matrix in the concatenated panel
    int64_t e0;    // first entry of the matrix in the concatenated entry arrays
};

struct BatchTask {
    int m;      // matrix
    int stage;  // -1: whole matrix; 0: start; 1..S: sweep; S+1: distances
    int tile;
};

__device__ __forceinline__ bool wait_count(int* p, int target, unsigned* status) {
    int spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kSpinLimit) {
            flag(status, AD_STAT_TIMEOUT);
            return false;
        }
    }
    return true;
}

template <typename T, int K, int LPR, bool WEIGHTED>
__device__ __forceinline__ void batch_stage(const BatchMat& m, int stage, int r0, int r1,
                                            int sweeps, T omega, uint64_t seed, double theta,
                                            const double (&wd)[K / LPR], const T (&wt)[K / LPR],
                                            T* __restrict__ X, T* __restrict__ W,
                                            T* __restrict__ mu, uint8_t* __restrict__ strong,
                                            int* __restrict__ nstrong, unsigned* status) {
    using S = Shape<T, K, LPR>;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    // iterate q lives in X when sweeps - q is even, so x^S ends in X
    auto buf = [&](int q) -> T* { return (((sweeps - q) & 1) == 0 ? X : W) + (size_t)m.row0 * K; };
    const int* rp = m.rp;
    const int* ci = m.ci;
    const T* av = (const T*)m.av;
    if (stage == 0) {
        T* dst = buf(0);
        const int64_t c0 = (int64_t)r0 * K, c1 = (int64_t)r1 * K;
        const uint64_t base = (uint64_t)m.row0 * K;
        for (int64_t c = c0 + threadIdx.x; c < c1; c += kBlock)
            dst[c] = (T)uniform_pm1(splitmix64_at(seed, base + (uint64_t)c));
    } else if (stage <= sweeps) {
        const T* src = buf(stage - 1);
        T* dst = buf(stage);
        for (int i = r0 + wv * S::RPW + g; i < r1; i += S::RPB)
            jacobi_row<S, T, K>(i, l, rp, ci, av, src, dst, omega, status);
    } else {
        const T* Xf = buf(sweeps);
        for (int i = r0 + wv * S::RPW + g; i < r1; i += S::RPB)
            algdist_row<S, T, K, WEIGHTED>(i, l, rp, ci, av, Xf, wd, wt, true, mu + m.e0, nullptr, theta,
                                 nullptr, strong ? strong + m.e0 : nullptr,
                                 nstrong ? nstrong + m.row0 : nullptr, status);
    }
}

template <typename T, int K, int LPR, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void batched_kernel(
    const BatchMat* __restrict__ mats, const BatchTask* __restrict__ tasks, int ntasks,
    int* __restrict__ ctrl, int sweeps, T omega, uint64_t seed, double theta,
    const double* __restrict__ w, int tile_rows, T* __restrict__ X, T* __restrict__ W,
    T* __restrict__ mu, uint8_t* __restrict__ strong, int* __restrict__ nstrong,
    unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V;
    __shared__ int s_task;
    const int l = (threadIdx.x & (kWave - 1)) % LPR;
    double wd[V];
    T wt[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
        wd[q] = w ? w[l * V + q] : 1.0;
        wt[q] = (T)wd[q];
    }
    const int nst = sweeps + 2;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(&ctrl[0], 1);
        __syncthreads();
        const int t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const BatchTask tk = tasks[t];
        const BatchMat m = mats[tk.m];
        if (tk.stage < 0) {
            for (int st = 0; st < nst; ++st) {
                batch_stage<T, K, LPR, WEIGHTED>(m, st, 0, m.n, sweeps, omega, seed, theta, wd, wt, X, W, mu,
                                       strong, nstrong, status);
                __threadfence_block();
                __syncthreads();
            }
        } else {
            int* done = ctrl + 1 + (size_t)tk.m * nst;
            if (tk.stage > 0) {
                if (threadIdx.x == 0) wait_count(&done[tk.stage - 1], m.ntiles, status);
                __syncthreads();
                __threadfence();  // acquire: see the other workgroups' rows
            }
            const int r0 = tk.tile * tile_rows;
            const int r1 = min(m.n, r0 + tile_rows);
            batch_stage<T, K, LPR, WEIGHTED>(m, tk.stage, r0, r1, sweeps, omega, seed, theta, wd, wt, X, W,
                                   mu, strong, nstrong, status);
            __threadfence();  // release: this tile's rows before the signal
            __syncthreads();
            if (threadIdx.x == 0) atomicAdd(&done[tk.stage], 1);
        }
    }
}

__global__ __launch_bounds__(kBlock) void zero_ints_kernel(int* __restrict__ p, int64_t m) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < m) p[q] = 0;
}

// ---------------------------------------------------------------- host side
struct BatchPlan {
    std::vector<uint8_t> key;  // what the device tables and graph were built for
    int ntasks = 0;
    int grid = 0;
    int64_t nctrl = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Per-handle state of the batched path.  Its device buffer (ping-pong
// panel, counters, task tables) is its own allocation, so no other call can
// overwrite the tables a captured graph refers to.
struct BatchState {
    BatchPlan plan;
    void* dev = nullptr;
    size_t dev_bytes = 0;
    void* host_stage = nullptr;  // pinned staging for the task tables
    size_t host_bytes = 0;
    hipStream_t cap = nullptr;   // private stream used only for graph capture
};

static BatchState* state_of(ad_handle h) {
    if (!h->batch) h->batch = new BatchState();
    return (BatchState*)h->batch;
}

void batch_state_free(ad_handle h) {
    BatchState* b = (BatchState*)h->batch;
    if (!b) return;
    if (b->plan.exec) (void)hipGraphExecDestroy(b->plan.exec);
    if (b->plan.graph) (void)hipGraphDestroy(b->plan.graph);
    if (b->host_stage) (void)hipHostFree(b->host_stage);
    if (b->dev) (void)hipFree(b->dev);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    h->batch = nullptr;
}

template <typename T, int K, int LPR>
static int batched_launch(ad_handle h, const BatchMat* mats, const BatchTask* tasks, int ntasks,
                          int* ctrl, int64_t nctrl, int grid, int sweeps, double omega,
                          uint64_t seed, double theta, const double* w, int tile_rows, void* X,
                          void* W, void* mu, uint8_t* strong, int32_t* nstrong, hipStream_t s) {
    const int zb = (int)((nctrl + kBlock - 1) / kBlock);
    zero_ints_kernel<<<dim3(zb), dim3(kBlock), 0, s>>>(ctrl, nctrl);
    if (w)
        batched_kernel<T, K, LPR, true><<<dim3(grid), dim3(kBlock), 0, s>>>(
            mats, tasks, ntasks, ctrl, sweeps, (T)omega, seed, theta, w, tile_rows, (T*)X, (T*)W,
            (T*)mu, strong, nstrong, h->status);
    else
        batched_kernel<T, K, LPR, false><<<dim3(grid), dim3(kBlock), 0, s>>>(
            mats, tasks, ntasks, ctrl, sweeps, (T)omega, seed, theta, w, tile_rows, (T*)X, (T*)W,
            (T*)mu, strong, nstrong, h->status);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

template <typename T>
static int batched_dispatch(ad_handle h, int K, int lpr, const BatchMat* mats,
                            const BatchTask* tasks, int ntasks, int* ctrl, int64_t nctrl, int grid,
                            int sweeps, double omega, uint64_t seed, double theta, const double* w,
                            int tile_rows, void* X, void* W, void* mu, uint8_t* strong,
                            int32_t* nstrong, hipStream_t s) {
    int rc2 = AD_OK;
    const int rc = with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        return with_lpr<T, KK>(lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            rc2 = batched_launch<T, KK, L>(h, mats, tasks, ntasks, ctrl, nctrl, grid, sweeps, omega,
                                           seed, theta, w, tile_rows, X, W, mu, strong, nstrong, s);
        });
    });
    return rc ? rc : rc2;
}

template <typename T, int K, int LPR>
static int occupancy_of() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_kernel<T, K, LPR, false>, kBlock, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <typename T>
static int blocks_per_cu(int K, int lpr) {
    int out = 1;
    with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        return with_lpr<T, KK>(lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            out = occupancy_of<T, KK, L>();
        });
    });
    return out;
}

int launch_batched(ad_handle h, int nmat, const ad_csr* As, int K, uint64_t seed, int sweeps,
                   double omega, const double* w, void* X, void* mu, double theta,
                   uint8_t* strong, int32_t* nstrong, const LaunchCfg& cfg, hipStream_t s) {
    BatchState* bs = state_of(h);
    const int dt = As[0].dtype;
    const size_t vsz = dt == AD_F32 ? 4 : 8;
    const int lpr = cfg.lpr > 0 ? cfg.lpr
                                : (dt == AD_F32 ? lpr_default<float>(K) : lpr_default<double>(K));
    const int rpb = (kWave / lpr) * kWavesPerBlock;
    const int tile_rows = rpb * (cfg.iter > 0 ? cfg.iter : 16);

    // key: everything the tables, the grid and the captured graph depend on
    std::vector<uint8_t> key;
    auto put = [&](const void* p, size_t b) {
        const uint8_t* c = (const uint8_t*)p;
        key.insert(key.end(), c, c + b);
    };
    put(&nmat, sizeof nmat);
    put(As, sizeof(ad_csr) * (size_t)nmat);
    const void* ptrs[6] = {X, mu, strong, nstrong, w, (void*)s};
    put(ptrs, sizeof ptrs);
    put(&K, sizeof K);
    put(&seed, sizeof seed);
    put(&sweeps, sizeof sweeps);
    put(&omega, sizeof omega);
    put(&theta, sizeof theta);
    put(&lpr, sizeof lpr);
    put(&tile_rows, sizeof tile_rows);

    // offsets and tasks
    std::vector<BatchMat> mats((size_t)nmat);
    int64_t rows = 0, ents = 0;
    for (int m = 0; m < nmat; ++m) {
        mats[m].rp = As[m].row_ptr;
        mats[m].ci = As[m].col;
        mats[m].av = As[m].val;
        mats[m].n = As[m].n;
        mats[m].ntiles = (As[m].n + tile_rows - 1) / tile_rows;
        mats[m].row0 = rows;
        mats[m].e0 = ents;
        rows += As[m].n;
        ents += As[m].nnz;
    }
    const size_t panel = (size_t)rows * K * vsz;
    const int nst = sweeps + 2;
    const int64_t nctrl = 1 + (int64_t)nmat * nst;

    WsReq req;
    const size_t o_w = req.add(panel);
    const size_t o_ctrl = req.add(sizeof(int) * (size_t)nctrl);
    const size_t o_mats = req.add(sizeof(BatchMat) * (size_t)nmat);
    // task count is bounded by sum over tiled matrices of nst * ntiles + nmat
    int64_t maxtasks = 0;
    for (int m = 0; m < nmat; ++m)
        maxtasks += (mats[m].ntiles <= kWholeTiles) ? 1 : (int64_t)nst * mats[m].ntiles;
    const size_t o_tasks = req.add(sizeof(BatchTask) * (size_t)(maxtasks > 0 ? maxtasks : 1));
    const bool same = (key == bs->plan.key) && bs->dev_bytes >= req.off;
    int rc;
    if (!same && bs->dev_bytes < req.off) {
        AD_HIP(hipDeviceSynchronize());  // earlier launches may still use the old buffer
        if (bs->plan.exec) (void)hipGraphExecDestroy(bs->plan.exec);
        if (bs->plan.graph) (void)hipGraphDestroy(bs->plan.graph);
        bs->plan = BatchPlan();
        if (bs->dev) AD_HIP(hipFree(bs->dev));
        bs->dev = nullptr;
        bs->dev_bytes = 0;
        if (hipMalloc(&bs->dev, req.off) != hipSuccess) {
            bs->dev = nullptr;
            return AD_ENOMEM;
        }
        bs->dev_bytes = req.off;
    }
    char* ws = (char*)bs->dev;
    void* W = ws + o_w;
    int* ctrl = (int*)(ws + o_ctrl);
    BatchMat* dmats = (BatchMat*)(ws + o_mats);
    BatchTask* dtasks = (BatchTask*)(ws + o_tasks);

    if (!same) {
        // largest first (by entries), tiled matrices before whole ones
        std::vector<int> order((size_t)nmat);
        for (int m = 0; m < nmat; ++m) order[m] = m;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const bool ta = mats[a].ntiles > kWholeTiles, tb = mats[b].ntiles > kWholeTiles;
            if (ta != tb) return ta;
            return As[a].nnz > As[b].nnz;
        });
        std::vector<BatchTask> tasks;
        tasks.reserve((size_t)maxtasks);
        for (int m : order) {
            if (mats[m].n == 0) continue;
            if (mats[m].ntiles <= kWholeTiles) {
                tasks.push_back({m, -1, 0});
            } else {
                for (int st = 0; st < nst; ++st)
                    for (int t = 0; t < mats[m].ntiles; ++t) tasks.push_back({m, st, t});
            }
        }
        const size_t tb = sizeof(BatchMat) * mats.size() + sizeof(BatchTask) * tasks.size();
        if (bs->host_bytes < tb) {
            AD_HIP(hipDeviceSynchronize());  // the old staging buffer may still feed a copy
            if (bs->host_stage) AD_HIP(hipHostFree(bs->host_stage));
            bs->host_stage = nullptr;
            bs->host_bytes = 0;
            AD_HIP(hipHostMalloc(&bs->host_stage, tb + tb / 4, hipHostMallocDefault));
            bs->host_bytes = tb + tb / 4;
        } else {
            AD_HIP(hipStreamSynchronize(s));  // the previous upload has finished
        }
        memcpy(bs->host_stage, mats.data(), sizeof(BatchMat) * mats.size());
        memcpy((char*)bs->host_stage + sizeof(BatchMat) * mats.size(), tasks.data(),
               sizeof(BatchTask) * tasks.size());
        AD_HIP(hipMemcpyAsync(dmats, bs->host_stage, sizeof(BatchMat) * mats.size(),
                              hipMemcpyHostToDevice, s));
        AD_HIP(hipMemcpyAsync(dtasks, (char*)bs->host_stage + sizeof(BatchMat) * mats.size(),
                              sizeof(BatchTask) * tasks.size(), hipMemcpyHostToDevice, s));
        const int bpc = dt == AD_F32 ? blocks_per_cu<float>(K, lpr) : blocks_per_cu<double>(K, lpr);
        int grid = h->cu_count * bpc;
        if ((int64_t)grid > (int64_t)tasks.size()) grid = (int)tasks.size();
        if (grid < 1) grid = 1;
        if (bs->plan.exec) (void)hipGraphExecDestroy(bs->plan.exec);
        if (bs->plan.graph) (void)hipGraphDestroy(bs->plan.graph);
        bs->plan.exec = nullptr;
        bs->plan.graph = nullptr;
        bs->plan.key = key;
        bs->plan.ntasks = (int)tasks.size();
        bs->plan.grid = grid;
        bs->plan.nctrl = nctrl;
    }
    const BatchPlan& p = bs->plan;
    if (p.ntasks == 0) return AD_OK;

    auto launch_on = [&](hipStream_t st) {
        return dt == AD_F32
                   ? batched_dispatch<float>(h, K, lpr, dmats, dtasks, p.ntasks, ctrl, p.nctrl, p.grid,
                                             sweeps, omega, seed, theta, w, tile_rows, X, W, mu,
                                             strong, nstrong, st)
                   : batched_dispatch<double>(h, K, lpr, dmats, dtasks, p.ntasks, ctrl, p.nctrl, p.grid,
                                              sweeps, omega, seed, theta, w, tile_rows, X, W, mu,
                                              strong, nstrong, st);
    };
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    AD_HIP(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone || h->timing) return launch_on(s);  // caller records it
    if (!bs->plan.exec) {
        if (!bs->cap) AD_HIP(hipStreamCreateWithFlags(&bs->cap, hipStreamNonBlocking));
        AD_HIP(hipStreamBeginCapture(bs->cap, hipStreamCaptureModeThreadLocal));
        rc = launch_on(bs->cap);
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(bs->cap, &gr);
        if (rc) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (ec != hipSuccess) return AD_EDEVICE;
        bs->plan.graph = gr;
        AD_HIP(hipGraphInstantiate(&bs->plan.exec, gr, nullptr, nullptr, 0));
    }
    AD_HIP(hipGraphLaunch(bs->plan.exec, s));
    return AD_OK;
}

}  // namespace ad
