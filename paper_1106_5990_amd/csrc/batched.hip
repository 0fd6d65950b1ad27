// batched.hip -- many matrices through test-vector start, damped-Jacobi
// relaxation and the fused distance/strength step as one captured sequence.
//
// The batch is the block-diagonal matrix of its members, kept as separate
// CSR arrays with member-local column indices.  The host cuts every member
// into row tiles and uploads one table of (member, first row, end row); each
// stage is one launch over all tiles of all members, so a workgroup never
// waits on another one: the kernel boundary orders the stages.
//   launch 0       start panel of all rows (one counter stream over the batch),
//   launches 1..S  Jacobi sweeps, ping-pong between X and an internal panel,
//   launch S+1     distances with the strength row fused.
// The S + 2 launches are captured once in a HIP graph per argument set and
// replayed on later calls with the same arguments.
//
// Rows are computed by the per-row code of the single-matrix kernels
// (rowops.h) and the start uses the global row index, so a batch gives
// bitwise the results of those kernels on the concatenated matrix.
#include <string.h>

#include <algorithm>
#include <vector>

#include "device.h"
#include "internal.h"
#include "rowops.h"

namespace ad {

struct BatchMat {
    const int* rp;
    const int* ci;
    const void* av;
    int64_t row0;  // first row of the member in the concatenated panel
    int64_t e0;    // first entry of the member in the concatenated entry arrays
};

struct BatchTile {
    int m;   // member
    int r0;  // first member-local row
    int r1;  // end row (exclusive)
};

// Tile index of this workgroup, or -1.
__device__ __forceinline__ int64_t batch_tile(int64_t ntiles, int xcd) { return map_tile(ntiles, xcd); }

template <typename T, int K, int LPR>
__global__ __launch_bounds__(kBlock) void batch_jacobi_kernel(
    const BatchMat* __restrict__ mats, const BatchTile* __restrict__ tiles, int64_t ntiles,
    int iter, int xcd, const T* __restrict__ Xin, T* __restrict__ Xout, T omega,
    unsigned* status) {
    using S = Shape<T, K, LPR>;
    const int64_t t = batch_tile(ntiles, xcd);
    if (t < 0) return;
    const BatchTile tl = tiles[t];
    const BatchMat m = mats[tl.m];
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const T* xi = Xin + m.row0 * K;
    T* xo = Xout + m.row0 * K;
    __shared__ CsrStage<T> stg;
    for (int it = 0; it < iter; ++it) {
        const int iw = tl.r0 + it * S::RPB + wv * S::RPW;
        if (iw >= tl.r1) break;  // whole wavefront
        const int ie = (iw + S::RPW < tl.r1) ? iw + S::RPW : tl.r1;
        int64_t s0;
        int cnt;
        wave_lds_sync();
        stage_csr(stg, wv, lane, (int64_t)m.rp[iw], (int64_t)m.rp[ie], m.ci, (const T*)m.av, s0,
                  cnt);
        wave_lds_sync();
        const int i = iw + g;
        if (i >= tl.r1) continue;
        jacobi_row_staged<S, T, K>(i, l, m.rp, m.ci, (const T*)m.av, stg, wv, s0, cnt, xi, xo,
                                   omega, status);
    }
}

template <typename T, int K, int LPR, bool WEIGHTED, int UN>
__global__ __launch_bounds__(kBlock) void batch_algdist_kernel(
    const BatchMat* __restrict__ mats, const BatchTile* __restrict__ tiles, int64_t ntiles,
    int iter, int xcd, const T* __restrict__ X, const double* __restrict__ w, T* __restrict__ mu,
    double theta, uint8_t* __restrict__ strong, int* __restrict__ nstrong, unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V;
    const int64_t t = batch_tile(ntiles, xcd);
    if (t < 0) return;
    const BatchTile tl = tiles[t];
    const BatchMat m = mats[tl.m];
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    double wd[V];
    T wt[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
        wd[q] = WEIGHTED ? w[l * V + q] : 1.0;
        wt[q] = (T)wd[q];
    }
    const T* xm = X + m.row0 * K;
    T* mum = mu + m.e0;
    uint8_t* sm = strong ? strong + m.e0 : nullptr;
    int* nsm = nstrong ? nstrong + m.row0 : nullptr;
    for (int it = 0; it < iter; ++it) {
        const int iw = tl.r0 + it * S::RPB + wv * S::RPW;
        if (iw >= tl.r1) break;  // whole wavefront
        const bool ghost = iw + g >= tl.r1;
        if (ghost && CoopGather<T, V, LPR>::G == 1) break;  // ghosts only serve group loads
        algdist_row<S, T, K, WEIGHTED, UN>(ghost ? tl.r1 - 1 : iw + g, ghost, l, m.rp, m.ci,
                                       m.rp, m.ci, (const T*)m.av, xm, wd, wt, true, mum, nullptr,
                                       theta,
                                       nullptr, sm, nsm, status);
    }
}

// Distances in the edge-parallel form: a second tile table with tiles of
// kEdgeRows rows per wavefront.
template <typename T, int K, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void batch_algdist_edge_kernel(
    const BatchMat* __restrict__ mats, const BatchTile* __restrict__ tiles, int64_t ntiles,
    int xcd, const T* __restrict__ X, const double* __restrict__ w, T* __restrict__ mu,
    double theta, uint8_t* __restrict__ strong, int* __restrict__ nstrong, unsigned* status) {
    __shared__ EdgeLds<T> lds;
    const int64_t t = batch_tile(ntiles, xcd);
    if (t < 0) return;  // whole workgroup
    const BatchTile tl = tiles[t];
    const BatchMat m = mats[tl.m];
    const int r0 = tl.r0 + (threadIdx.x / kWave) * kEdgeRows;
    const int rl = r0 < tl.r1 ? min(kEdgeRows, tl.r1 - r0) : 0;
    algdist_edge_rows<T, K, WEIGHTED, true>(r0, rl, m.rp, m.ci, X + m.row0 * K, w, mu + m.e0,
                                            nullptr, theta, nullptr,
                                            strong ? strong + m.e0 : nullptr,
                                            nstrong ? nstrong + m.row0 : nullptr, lds, status);
}

constexpr int kEdgeTileRows = kEdgeRows * kWavesPerBlock;  // rows per distance tile (edge form)

// ---------------------------------------------------------------- host side
namespace {

struct BatchPlan {
    std::vector<uint8_t> key;  // arguments the tables and the graph were built for
    int64_t ntiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Per-handle state: the second panel, member and tile tables live in a
// buffer of their own, so no other call can overwrite what a captured graph
// refers to.
struct BatchState {
    BatchPlan plan;
    void* dev = nullptr;
    size_t dev_bytes = 0;
    void* host_stage = nullptr;  // pinned staging for the tables
    size_t host_bytes = 0;
    hipStream_t cap = nullptr;   // private stream used only for graph capture
    // true once a call ran inside a caller's stream capture: that graph refers
    // to `dev`, which is then never rewritten for another argument set
    bool pinned = false;
};

BatchState* state_of(ad_handle h) {
    if (!h->batch) h->batch = new BatchState();
    return (BatchState*)h->batch;
}

void drop_graph(BatchPlan& p) {
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    p.exec = nullptr;
    p.graph = nullptr;
}

struct Seq {
    ad_handle h;
    int dt, K, sweeps;
    int lpr, iter, xcd;     // relaxation shape
    int dlpr, dxcd, edge;   // distance shape (edge: the edge-parallel form)
    int64_t rows, ntiles, ndist;
    uint64_t seed;
    double omega, theta;
    const double* w;
    const BatchMat* mats;
    const BatchTile* tiles;   // relaxation tiles
    const BatchTile* dtiles;  // distance tiles
    int diter;                // row steps per distance tile (row-group form)
    bool long_rows;           // at least 16 stored entries per row on average
    void *X, *W, *mu;
    uint8_t* strong;
    int32_t* nstrong;
    unsigned* status;
};

template <typename T, int K, int LPR>
void seq_relax(const Seq& q, hipStream_t s) {
    // iterate k lives in X when sweeps - k is even, so the last one ends in X
    auto buf = [&](int k) -> T* { return (T*)((((q.sweeps - k) & 1) == 0) ? q.X : q.W); };
    const int grid = grid_for_tiles(q.ntiles, q.xcd);
    for (int k = 1; k <= q.sweeps; ++k) {
        TimedScope ts(q.h, "batch_jacobi", s);
        batch_jacobi_kernel<T, K, LPR><<<dim3(grid), dim3(kBlock), 0, s>>>(
            q.mats, q.tiles, q.ntiles, q.iter, q.xcd, buf(k - 1), buf(k), (T)q.omega, q.status);
    }
}

template <typename T, int K, int LPR>
void seq_dist_rows(const Seq& q, hipStream_t s) {
    TimedScope ts(q.h, "batch_algdist", s);
    const int grid = grid_for_tiles(q.ndist, q.dxcd);
    dist_unroll<T, K, LPR>(q.long_rows, [&](auto uc) {
        constexpr int UN = decltype(uc)::value;
        if (q.w)
            batch_algdist_kernel<T, K, LPR, true, UN><<<dim3(grid), dim3(kBlock), 0, s>>>(
                q.mats, q.dtiles, q.ndist, q.diter, q.dxcd, (const T*)q.X, q.w, (T*)q.mu, q.theta,
                q.strong, q.nstrong, q.status);
        else
            batch_algdist_kernel<T, K, LPR, false, UN><<<dim3(grid), dim3(kBlock), 0, s>>>(
                q.mats, q.dtiles, q.ndist, q.diter, q.dxcd, (const T*)q.X, nullptr, (T*)q.mu,
                q.theta, q.strong, q.nstrong, q.status);
    });
}

template <typename T, int K>
void seq_dist_edge(const Seq& q, hipStream_t s) {
    if constexpr (K * (int)sizeof(T) <= kEdgeMaxRowBytes) {
        TimedScope ts(q.h, "batch_algdist", s);
        const int grid = grid_for_tiles(q.ndist, q.dxcd);
        if (q.w)
            batch_algdist_edge_kernel<T, K, true><<<dim3(grid), dim3(kBlock), 0, s>>>(
                q.mats, q.dtiles, q.ndist, q.dxcd, (const T*)q.X, q.w, (T*)q.mu, q.theta,
                q.strong, q.nstrong, q.status);
        else
            batch_algdist_edge_kernel<T, K, false><<<dim3(grid), dim3(kBlock), 0, s>>>(
                q.mats, q.dtiles, q.ndist, q.dxcd, (const T*)q.X, nullptr, (T*)q.mu, q.theta,
                q.strong, q.nstrong, q.status);
    }
}

template <typename T>
int seq_dispatch(const Seq& q, hipStream_t s) {
    return with_k<T>(q.K, [&](auto kc) -> int {
        constexpr int KK = decltype(kc)::value;
        const int rc = with_lpr<T, KK>(q.lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            seq_relax<T, KK, L>(q, s);
        });
        if (rc) return rc;
        if (q.edge) {
            seq_dist_edge<T, KK>(q, s);
            return (int)AD_OK;
        }
        return with_lpr<T, KK>(q.dlpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            seq_dist_rows<T, KK, L>(q, s);
        });
    });
}

int run_seq(const Seq& q, hipStream_t s) {
    void* x0 = ((q.sweeps & 1) == 0) ? q.X : q.W;
    int rc;
    {
        TimedScope ts(q.h, "batch_tv_init", s);
        if ((rc = launch_tv_init(q.dt, 0, q.rows, q.K, q.seed, x0, s))) return rc;
    }
    if (q.ntiles == 0) return AD_OK;
    rc = q.dt == AD_F32 ? seq_dispatch<float>(q, s) : seq_dispatch<double>(q, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    return AD_OK;
}

}  // namespace

void batch_state_free(ad_handle h) {
    BatchState* b = (BatchState*)h->batch;
    if (!b) return;
    drop_graph(b->plan);
    if (b->host_stage) (void)hipHostFree(b->host_stage);
    if (b->dev) (void)hipFree(b->dev);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    h->batch = nullptr;
}

int launch_batched(ad_handle h, int nmat, const ad_csr* As, int K, uint64_t seed, int sweeps,
                   double omega, const double* w, void* X, void* mu, double theta,
                   uint8_t* strong, int32_t* nstrong, const LaunchCfg& cfg, const LaunchCfg& dcfg,
                   bool direct, hipStream_t s) {
    BatchState* bs = state_of(h);
    const int dt = As[0].dtype;
    const size_t vsz = dt == AD_F32 ? 4 : 8;
    auto resolve = [&](int l) {
        return l > 0 ? l : (dt == AD_F32 ? lpr_default<float>(K) : lpr_default<double>(K));
    };
    const int lpr = resolve(cfg.lpr);
    const int iter = cfg.iter > 0 ? cfg.iter : 1;
    const int xcd = cfg.xcd_map;
    const int64_t tile_rows = (int64_t)(kWave / lpr) * kWavesPerBlock * iter;
    const int edge = algdist_uses_edge(dt, K, AD_TARGET_PLAIN, dcfg) ? 1 : 0;
    const int dlpr = edge ? 0 : resolve(dcfg.lpr);
    const int diter = edge ? 1 : (dcfg.iter > 0 ? dcfg.iter : 1);
    const int dxcd = dcfg.xcd_map;
    const int64_t dist_rows =
        edge ? (int64_t)kEdgeTileRows : (int64_t)(kWave / dlpr) * kWavesPerBlock * diter;

    // key: everything the tables and the captured graph depend on
    std::vector<uint8_t> key;
    auto put = [&](const void* p, size_t b) {
        const uint8_t* c = (const uint8_t*)p;
        key.insert(key.end(), c, c + b);
    };
    put(&nmat, sizeof nmat);
    put(As, sizeof(ad_csr) * (size_t)nmat);
    const void* ptrs[5] = {X, mu, strong, nstrong, w};
    put(ptrs, sizeof ptrs);
    const int ints[9] = {K, sweeps, lpr, iter, xcd, edge, dlpr, diter, dxcd};
    put(ints, sizeof ints);
    const double dbl[2] = {omega, theta};
    put(dbl, sizeof dbl);
    put(&seed, sizeof seed);

    std::vector<BatchMat> mats((size_t)nmat);
    int64_t rows = 0, ents = 0, ntiles = 0, ndist = 0;
    for (int m = 0; m < nmat; ++m) {
        mats[m] = BatchMat{As[m].row_ptr, As[m].col, As[m].val, rows, ents};
        rows += As[m].n;
        ents += As[m].nnz;
        ntiles += (As[m].n + tile_rows - 1) / tile_rows;
        ndist += (As[m].n + dist_rows - 1) / dist_rows;
    }
    if (ntiles > ((int64_t)1 << 30) || ndist > ((int64_t)1 << 30)) return AD_ESTRUCT;  // grid limit

    WsReq req;
    const size_t o_w = req.add((size_t)rows * K * vsz);
    const size_t o_mats = req.add(sizeof(BatchMat) * (size_t)nmat);
    const size_t o_tiles = req.add(sizeof(BatchTile) * (size_t)(ntiles > 0 ? ntiles : 1));
    const size_t o_dtiles = req.add(sizeof(BatchTile) * (size_t)(ndist > 0 ? ndist : 1));
    const bool same = key == bs->plan.key && bs->dev_bytes >= req.off;
    const bool capturing = stream_capturing(s);
    if (!same) {
        // the tables are uploaded from the host: not inside a caller's capture
        if (capturing) return AD_EUNSUPPORTED;
        drop_graph(bs->plan);
        bs->plan.key.clear();
        if (bs->pinned) {
            // a caller's captured graph refers to the current buffer: keep it
            // alive and give this argument set a buffer of its own
            if (bs->dev) h->retired.push_back(bs->dev);
            bs->dev = nullptr;
            bs->dev_bytes = 0;
            bs->pinned = false;
        }
        if (bs->dev_bytes < req.off) {
            AD_HIP(hipDeviceSynchronize());  // earlier launches may still use the old buffer
            if (bs->dev) AD_HIP(hipFree(bs->dev));
            bs->dev = nullptr;
            bs->dev_bytes = 0;
            if (hipMalloc(&bs->dev, req.off) != hipSuccess) {
                bs->dev = nullptr;
                return AD_ENOMEM;
            }
            bs->dev_bytes = req.off;
        }
    }
    char* ws = (char*)bs->dev;
    BatchMat* dmats = (BatchMat*)(ws + o_mats);
    BatchTile* dtiles = (BatchTile*)(ws + o_tiles);
    BatchTile* ddtiles = (BatchTile*)(ws + o_dtiles);

    if (!same) {
        // relaxation tiles, then distance tiles, staged in one pinned buffer
        std::vector<BatchTile> tiles;
        tiles.reserve((size_t)(ntiles + ndist));
        auto cut = [&](int64_t rows_per_tile) {
            for (int m = 0; m < nmat; ++m)
                for (int64_t r = 0; r < As[m].n; r += rows_per_tile)
                    tiles.push_back(
                        BatchTile{m, (int)r, (int)std::min<int64_t>(As[m].n, r + rows_per_tile)});
        };
        cut(tile_rows);
        cut(dist_rows);
        const size_t mb = sizeof(BatchMat) * mats.size();
        const size_t tb = mb + sizeof(BatchTile) * tiles.size();
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
        memcpy(bs->host_stage, mats.data(), mb);
        memcpy((char*)bs->host_stage + mb, tiles.data(), sizeof(BatchTile) * tiles.size());
        AD_HIP(hipMemcpyAsync(dmats, bs->host_stage, mb, hipMemcpyHostToDevice, s));
        if (ntiles > 0)
            AD_HIP(hipMemcpyAsync(dtiles, (char*)bs->host_stage + mb,
                                  sizeof(BatchTile) * (size_t)ntiles, hipMemcpyHostToDevice, s));
        if (ndist > 0)
            AD_HIP(hipMemcpyAsync(ddtiles,
                                  (char*)bs->host_stage + mb + sizeof(BatchTile) * (size_t)ntiles,
                                  sizeof(BatchTile) * (size_t)ndist, hipMemcpyHostToDevice, s));
        bs->plan.key = key;
        bs->plan.ntiles = ntiles;
    }

    Seq q;
    q.h = h;
    q.dt = dt;
    q.K = K;
    q.sweeps = sweeps;
    q.lpr = lpr;
    q.iter = iter;
    q.xcd = xcd;
    q.dlpr = dlpr;
    q.dxcd = dxcd;
    q.edge = edge;
    q.rows = rows;
    q.ntiles = ntiles;
    q.ndist = ndist;
    q.long_rows = batch_bucket(nmat, As) >= 2;
    q.seed = seed;
    q.omega = omega;
    q.theta = theta;
    q.w = w;
    q.mats = dmats;
    q.tiles = dtiles;
    q.dtiles = ddtiles;
    q.diter = diter;
    q.X = X;
    q.W = ws + o_w;
    q.mu = mu;
    q.strong = strong;
    q.nstrong = nstrong;
    q.status = h->status;
    if (capturing) {
        bs->pinned = true;  // the caller's graph now refers to the tables and panel
        return run_seq(q, s);
    }
    if (direct) return run_seq(q, s);
    if (!bs->plan.exec) {
        if (!bs->cap) AD_HIP(hipStreamCreateWithFlags(&bs->cap, hipStreamNonBlocking));
        AD_HIP(hipStreamBeginCapture(bs->cap, hipStreamCaptureModeThreadLocal));
        const int rc = run_seq(q, bs->cap);
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(bs->cap, &gr);
        if (rc || ec != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc ? rc : AD_EDEVICE;
        }
        bs->plan.graph = gr;
        AD_HIP(hipGraphInstantiate(&bs->plan.exec, gr, nullptr, nullptr, 0));
    }
    AD_HIP(hipGraphLaunch(bs->plan.exec, s));
    return AD_OK;
}

}  // namespace ad
