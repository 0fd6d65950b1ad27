// autotune.hip -- launch-shape search for the kernel families.
//
// For one matrix (its dtype, K and stored-entries-per-row bucket) every
// valid shape of each family is timed with HIP events on scratch buffers:
//   lanes per row L (K / L panel entries per lane: the panel width a lane
//   owns; 64 / L rows per wavefront), rows per lane group per tile
//   (1, 2, 4), and the tile-to-XCD mapping (0: plain block order; 1: one
//   contiguous tile range per XCD; c in {4, 16, 64, 256}: chunks of 8c
//   tiles, c contiguous tiles per XCD in each); for the distances also
//   L = 0, the edge-parallel form (one lane per entry).
// The fastest shape per family is stored in the handle (the same slot
// algdist_set_launch writes) and, if a cache path is given, in a JSON file:
// one object per line,
//   {"kernel": "algdist", "dtype": 0, "K": 16, "bucket": 1, "lpr": 2, "iter": 1, "xcd": 1, "ms": 0.41}
// A cache entry for the key is used instead of timing.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace ad {

namespace {

const char* kFamilyName[KN_COUNT] = {"jacobi",  "gs_phase",    "algdist",         "ls_interp",
                                     "batched", "distance_ls", "batched_distance"};

struct Entry {
    std::string kernel;
    int dtype, K, bucket, lpr, iter, xcd;
    double ms;
};

std::vector<Entry> read_cache(const char* path) {
    std::vector<Entry> out;
    if (!path) return out;
    FILE* f = fopen(path, "r");
    if (!f) return out;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char name[64];
        Entry e;
        if (sscanf(line,
                   " {\"kernel\": \"%63[^\"]\", \"dtype\": %d, \"K\": %d, \"bucket\": %d, \"lpr\": %d, "
                   "\"iter\": %d, \"xcd\": %d, \"ms\": %lf}",
                   name, &e.dtype, &e.K, &e.bucket, &e.lpr, &e.iter, &e.xcd, &e.ms) == 8) {
            e.kernel = name;
            out.push_back(e);
        }
    }
    fclose(f);
    return out;
}

void write_cache(const char* path, const std::vector<Entry>& v) {
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const Entry& e : v)
        fprintf(f,
                "{\"kernel\": \"%s\", \"dtype\": %d, \"K\": %d, \"bucket\": %d, \"lpr\": %d, "
                "\"iter\": %d, \"xcd\": %d, \"ms\": %.6f}\n",
                e.kernel.c_str(), e.dtype, e.K, e.bucket, e.lpr, e.iter, e.xcd, e.ms);
    fclose(f);
    rename(tmp.c_str(), path);
}

// tile-to-XCD mappings tried (see map_tile)
constexpr int kXcdModes[6] = {0, 1, 4, 16, 64, 256};
// A shape replaces the current choice only when it is more than 2% faster:
// shapes within timing noise of each other then resolve to the first in
// enumeration order (fewer lanes per row, fewer row steps, plainer tile
// order) from run to run, instead of to whichever measured lower this time.
constexpr double kTuneMargin = 0.98;
constexpr int kTuneTrials = 5;

bool lpr_valid(int dtype, int K, int L) {
    return dtype == AD_F32 ? lpr_ok<float>(K, L) : lpr_ok<double>(K, L);
}

// average milliseconds of `reps` runs of fn (after one warm run)
template <typename F>
double time_ms(hipStream_t s, hipEvent_t a, hipEvent_t b, int reps, F&& fn, bool& ok) {
    ok = fn() == AD_OK;
    if (!ok) return 1e30;
    // the least of kTuneTrials timings of `reps` back-to-back runs: the
    // fastest of repeated measurements is the one least disturbed by clock
    // and queue noise
    double best = 1e30;
    for (int t = 0; t < kTuneTrials && ok; ++t) {
        (void)hipEventRecord(a, s);
        for (int r = 0; r < reps; ++r)
            if (fn() != AD_OK) ok = false;
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        best = ms / reps < best ? ms / reps : best;
    }
    return ok ? best : 1e30;
}

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        (void)hipDeviceSynchronize();  // scratch may still be in use by queued timing runs
        for (void* p : ptrs) (void)hipFree(p);
    }
    void* get(size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
};

}  // namespace

int autotune(ad_handle h, const ad_csr* A, int K, int relax, const int32_t* color, int ncolors,
             const uint8_t* cf, int caliber, const char* cache, hipStream_t s) {
    const int dt = A->dtype;
    const int ks = k_slot(K);
    const int bucket = nnz_bucket(A->nnz, A->n);
    std::vector<Entry> entries = read_cache(cache);
    const int fams[4] = {relax == AD_JACOBI ? KN_JACOBI : KN_GS, KN_ALGDIST, KN_LS, KN_DLS};
    const bool with_ls = cf != nullptr && caliber >= 1 && caliber <= K && caliber <= 8;
    bool need[4] = {true, true, with_ls, with_ls};
    for (int q = 0; q < 4; ++q)
        for (const Entry& e : entries)
            if (need[q] && e.kernel == kFamilyName[fams[q]] && e.dtype == dt && e.K == K &&
                e.bucket == bucket) {
                LaunchCfg c;
                c.lpr = e.lpr;
                c.iter = e.iter;
                c.xcd_map = e.xcd;
                h->tuned[fams[q]][dt][ks][bucket] = c;
                h->has_tuned[fams[q]][dt][ks][bucket] = true;
                need[q] = false;
            }
    if (!need[0] && !need[1] && !need[2] && !need[3]) return AD_OK;

    const size_t vs = dt == AD_F32 ? 4 : 8;
    const int n = A->n;
    const size_t panel = (size_t)n * K * vs;
    Scratch sc;
    void* X = sc.get(panel);
    void* X2 = sc.get(panel);
    void* mu = sc.get((size_t)A->nnz * vs);
    uint8_t* strong = (uint8_t*)sc.get((size_t)A->nnz);
    int32_t* ns = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
    if (!X || !X2 || !mu || !strong || !ns) return AD_ENOMEM;
    int rc = launch_tv_init(dt, 0, n, K, 1, X, s);
    if (rc) return rc;
    hipEvent_t ea, eb;
    AD_HIP(hipEventCreate(&ea));
    AD_HIP(hipEventCreate(&eb));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{ea, eb};

    // colour-major setup for the colour phases
    PermCsr pc{n, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (need[0] && relax == AD_MULTICOLOR_GS) {
        const int nblk = color_partition_blocks(n);
        int32_t* rowlist = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
        int32_t* inv = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
        int32_t* rpp = (int32_t*)sc.get(sizeof(int32_t) * ((size_t)n + 1));
        int32_t* colp = (int32_t*)sc.get(sizeof(int32_t) * (size_t)A->nnz);
        void* valp = sc.get(vs * (size_t)A->nnz);
        int32_t* seg = (int32_t*)sc.get(sizeof(int32_t) * (ncolors + 2));
        int32_t* cnt = (int32_t*)sc.get(sizeof(int32_t) * 2 * (size_t)(ncolors + 1) * nblk);
        if (!rowlist || !inv || !rpp || !colp || !valp || !seg || !cnt) return AD_ENOMEM;
        if ((rc = launch_color_partition(n, color, ncolors, A->row_ptr, rowlist, inv, seg, cnt,
                                         nblk, rpp, h->status, s)))
            return rc;
        pc = PermCsr{n, rowlist, seg, rpp, colp, valp};
        if ((rc = launch_perm_setup(dt, A, pc, inv, s))) return rc;
    }
    int32_t* Pc = nullptr;
    double *Pv = nullptr, *ls = nullptr, *bs = nullptr;
    int32_t* st = nullptr;
    if (with_ls) {
        Pc = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n * caliber);
        Pv = (double*)sc.get(sizeof(double) * (size_t)n * caliber);
        ls = (double*)sc.get(sizeof(double) * (size_t)n);
        st = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
        if (!Pc || !Pv || !ls || !st) return AD_ENOMEM;
    }

    const int iters[3] = {1, 2, 4};
    for (int q = 0; q < 4; ++q) {
        if (!need[q]) continue;
        const int fam = fams[q];
        double best = 1e30;
        LaunchCfg bestc;
        // lanes per row 0 is the default form: for distances the edge-parallel
        // kernel (one lane per entry), which ignores the row-step count
        for (int L = 0; L <= kWave; L = L ? 2 * L : 1) {
            if (L == 0 ? !(fam == KN_ALGDIST && algdist_uses_edge(dt, K, AD_TARGET_PLAIN, LaunchCfg()))
                       : !lpr_valid(dt, K, L))
                continue;
            for (int it : iters) {
                // LS rows and the edge-parallel distances ignore the row-step count
                if ((fam == KN_LS || L == 0) && it != 1) continue;
                for (int xcd : kXcdModes) {
                    LaunchCfg c;
                    c.lpr = L;
                    c.iter = it;
                    c.xcd_map = xcd;
                    bool ok = true;
                    double ms = 1e30;
                    if (fam == KN_JACOBI) {
                        ms = time_ms(s, ea, eb, 3, [&] {
                            return launch_jacobi(dt, K, A, X, X2, 0.7, h->status, c, s);
                        }, ok);
                    } else if (fam == KN_GS) {
                        ms = time_ms(s, ea, eb, 3, [&] {
                            int r = AD_OK;
                            for (int cc = 0; cc < ncolors && !r; ++cc)
                                r = launch_gs_phase_perm(dt, K, pc, cc, ncolors, X, X2, nullptr, 1,
                                                         h->status, c, s);
                            return r;
                        }, ok);
                        ms /= ncolors;
                    } else if (fam == KN_ALGDIST) {
                        ms = time_ms(s, ea, eb, 3, [&] {
                            return launch_algdist(dt, K, A, X, nullptr, AD_TARGET_PLAIN, mu, nullptr,
                                                  0.25, nullptr, strong, ns, h->status, c, s);
                        }, ok);
                    } else if (fam == KN_DLS) {
                        ms = time_ms(s, ea, eb, 3, [&] {
                            return launch_dist_ls(dt, K, caliber, A, X, nullptr, AD_TARGET_PLAIN,
                                                  mu, 0.25, nullptr, strong, ns, cf, Pc, Pv, ls,
                                                  st, nullptr, nullptr, h->status, c, s);
                        }, ok);
                    } else {
                        // distances once, then LS rows on them
                        if (launch_algdist(dt, K, A, X, nullptr, AD_TARGET_PLAIN, mu, nullptr, 0.25,
                                           nullptr, nullptr, nullptr, h->status, LaunchCfg(), s))
                            continue;
                        ms = time_ms(s, ea, eb, 3, [&] {
                            return launch_ls_interp(dt, K, caliber, A, X, nullptr, cf, mu,
                                                    AD_TARGET_PLAIN, Pc, Pv, ls, st, bs, nullptr,
                                                    h->status, c, s);
                        }, ok);
                    }
                    if (ok && ms < best * kTuneMargin) {
                        best = ms;
                        bestc = c;
                    }
                }
            }
        }
        if (best >= 1e30) continue;
        h->tuned[fam][dt][ks][bucket] = bestc;
        h->has_tuned[fam][dt][ks][bucket] = true;
        Entry e{kFamilyName[fam], dt, K, bucket, bestc.lpr, bestc.iter, bestc.xcd_map, best};
        bool replaced = false;
        for (Entry& x : entries)
            if (x.kernel == e.kernel && x.dtype == dt && x.K == K && x.bucket == bucket) {
                x = e;
                replaced = true;
            }
        if (!replaced) entries.push_back(e);
    }
    AD_HIP(hipStreamSynchronize(s));
    write_cache(cache, entries);
    return AD_OK;
}

// Batched sequence: the relaxation shape and the distance shape are picked
// separately.  Every valid relaxation shape (lanes per row, row steps per
// tile, XCD mapping) is timed on the batch itself with the default distance
// form, then every distance shape (the edge-parallel form or a row-group
// shape) with the chosen relaxation shape; each candidate's stage time comes
// from the library's per-launch HIP events (direct launches into scratch
// outputs).  Both are stored for the batch's entries-per-row bucket.
namespace {

// total ms of the launches labelled `label` recorded while fn ran
template <typename F>
double stage_ms(ad_handle h, hipStream_t s, const char* label, F&& fn, bool& ok) {
    const bool was = h->timing;
    const size_t t0 = h->timed.size();
    const int e0 = h->events_used;
    h->timing = true;
    ok = fn() == AD_OK;
    (void)hipStreamSynchronize(s);
    double ms = 0.0;
    for (size_t q = t0; q < h->timed.size(); ++q) {
        float x = 0.f;
        if (strcmp(h->timed[q].label, label) == 0 &&
            hipEventElapsedTime(&x, h->timed[q].a, h->timed[q].b) == hipSuccess)
            ms += x;
    }
    h->timed.resize(t0);
    h->events_used = e0;
    h->timing = was;
    return ok ? ms : 1e30;
}

}  // namespace

int autotune_batched(ad_handle h, int nmat, const ad_csr* As, int K, int sweeps, const char* cache,
                     hipStream_t s) {
    const int dt = As[0].dtype;
    const int ks = k_slot(K);
    const int bucket = batch_bucket(nmat, As);
    const int fams[2] = {KN_BATCHED, KN_BDIST};
    bool need[2] = {true, true};
    std::vector<Entry> entries = read_cache(cache);
    for (int f = 0; f < 2; ++f)
        for (const Entry& e : entries)
            if (need[f] && e.kernel == kFamilyName[fams[f]] && e.dtype == dt && e.K == K &&
                e.bucket == bucket) {
                LaunchCfg c;
                c.lpr = e.lpr;
                c.iter = e.iter;
                c.xcd_map = e.xcd;
                h->tuned[fams[f]][dt][ks][bucket] = c;
                h->has_tuned[fams[f]][dt][ks][bucket] = true;
                need[f] = false;
            }
    if (!need[0] && !need[1]) return AD_OK;
    int64_t rows = 0, ents = 0;
    for (int m = 0; m < nmat; ++m) {
        rows += As[m].n;
        ents += As[m].nnz;
    }
    if (rows == 0) return AD_OK;
    const size_t vs = dt == AD_F32 ? 4 : 8;
    Scratch sc;
    void* X = sc.get((size_t)rows * K * vs);
    void* mu = sc.get((size_t)ents * vs);
    uint8_t* strong = (uint8_t*)sc.get((size_t)ents);
    int32_t* ns = (int32_t*)sc.get(sizeof(int32_t) * (size_t)rows);
    if (!X || !mu || !strong || !ns) return AD_ENOMEM;
    LaunchCfg rcfg = h->has_tuned[KN_BATCHED][dt][ks][bucket] ? h->tuned[KN_BATCHED][dt][ks][bucket]
                                                              : LaunchCfg();
    LaunchCfg dcfg = h->has_tuned[KN_BDIST][dt][ks][bucket] ? h->tuned[KN_BDIST][dt][ks][bucket]
                                                            : LaunchCfg();
    const int iters[3] = {1, 2, 4};
    for (int f = 0; f < 2; ++f) {
        if (!need[f]) continue;
        const char* label = f == 0 ? "batch_jacobi" : "batch_algdist";
        double best = 1e30;
        LaunchCfg bestc;
        for (int L = 0; L <= kWave; L = L ? 2 * L : 1) {
            // relaxation: explicit shapes; distances: also 0, the edge-parallel form
            if (L == 0 ? (f == 0 || !algdist_uses_edge(dt, K, AD_TARGET_PLAIN, LaunchCfg()))
                       : !lpr_valid(dt, K, L))
                continue;
            for (int it : iters) {
                if (L == 0 && it != 1) continue;
                for (int xcd : kXcdModes) {
                    LaunchCfg c;
                    c.lpr = L;
                    c.iter = it;
                    c.xcd_map = xcd;
                    const LaunchCfg& rc_ = f == 0 ? c : rcfg;
                    const LaunchCfg& dc_ = f == 0 ? dcfg : c;
                    auto run = [&] {
                        return launch_batched(h, nmat, As, K, 1, sweeps, 2.0 / 3.0, nullptr, X, mu,
                                              0.25, strong, ns, rc_, dc_, true, s);
                    };
                    bool ok = true;
                    (void)stage_ms(h, s, label, run, ok);  // warm: tables, caches
                    if (!ok) continue;
                    double ms = 0.0;
                    for (int r = 0; r < 3 && ok; ++r) ms += stage_ms(h, s, label, run, ok);
                    if (ok && ms < best * kTuneMargin) {
                        best = ms;
                        bestc = c;
                    }
                }
            }
        }
        if (best >= 1e30) return AD_EDEVICE;
        (f == 0 ? rcfg : dcfg) = bestc;
        h->tuned[fams[f]][dt][ks][bucket] = bestc;
        h->has_tuned[fams[f]][dt][ks][bucket] = true;
        entries.push_back(Entry{kFamilyName[fams[f]], dt, K, bucket, bestc.lpr, bestc.iter,
                                bestc.xcd_map, best / 3.0});
    }
    AD_HIP(hipStreamSynchronize(s));
    write_cache(cache, entries);
    return AD_OK;
}

}  // namespace ad
