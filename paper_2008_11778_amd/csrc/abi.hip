// Host runtime and C ABI of the wave-equation calls.
//
// An Engine holds one or more inversion instances (each a geometry with all
// of its shots) and advances all of them together: every stepping launch
// covers the tiles of every active instance (a device tile table), and each
// instance derives its own time step, buffer parity and checkpoint slot from
// the launch's step counter, so instances with different grids, shot counts
// and record lengths share launches.  aafwi_ctx is an Engine with one
// instance whose inputs and outputs are caller buffers; aafwi_batch is an
// Engine with N instances that owns its model, data and gradient buffers (so
// the launch sequence can be captured once in a hipGraph and replayed).
//
// Forward pass: u^{n+1} = 2A u^n - B u^{n-1} + Kp (Lt u^n + src) for
// n = 0..nt-1 with (u^n, u^{n-1}) copied to checkpoint slot n/k when n % k == 0.
// Backward pass, segment by segment from the end of each record: recompute
// the segment's steps from its checkpoint storing q-hat^n, then run the
// adjoint steps of the segment backwards, imaging into per-shot
// accumulators; finally fold (sum over shots, transpose of the edge
// replication, scaling by 1/(A dt^2)).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"

namespace aafwi {
namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace aafwi

using aafwi::Error;

namespace {

// Host view of one instance.
struct InstHost {
    int nz = 0, nx = 0, nb = 0, nt = 0, S = 0, R = 0, nseg = 0;
    float h = 0, dt = 0;
    float mmin = 0;  // 1 / vmax_bound^2: the smallest m the scheme uses
    aafwi::WaveGrid g{};
    long long field = 0;
    int nrr = 0;
    std::vector<float> wavelet;
    // device memory
    float *K = nullptr, *E = nullptr;
    float* F[4] = {nullptr, nullptr, nullptr, nullptr};
    float* L[4] = {nullptr, nullptr, nullptr, nullptr};
    float *GI = nullptr, *ckpt = nullptr, *qseg = nullptr, *d = nullptr, *wav = nullptr, *mkeep = nullptr;
    float *m = nullptr, *grad = nullptr;  // caller buffers of batch instances
    const float* dobs = nullptr;
    int2* src = nullptr;
    int *rowmap = nullptr, *xmap = nullptr, *rnext = nullptr;
    bool have_ckpt = false;
    int tz[4] = {0, 0, 0, 0};  // per-instance strip heights (0: the engine's setting)
};

struct Engine {
    hipStream_t stream = nullptr;
    int k = 0;
    int k_ckpt = 0;       // checkpoint interval of the checkpointed layout
    bool keep_q = false;  // full storage: the kept forward writes q-hat of every step, no recompute
    bool is_batch = false;  // per-instance masks, caller buffers fixed at creation
    std::vector<InstHost> in;
    aafwi::Inst* dinst = nullptr;
    aafwi::TileRec* dtiles[4] = {nullptr, nullptr, nullptr, nullptr};
    int ntiles[4] = {0, 0, 0, 0};
    // two-step tables (64 output columns per wave) of forward, recompute, adjoint
    aafwi::TileRec* dtiles2[3] = {nullptr, nullptr, nullptr};
    int ntiles2[3] = {0, 0, 0};
    bool tb[3] = {false, false, false};  // forward / recompute / adjoint: two steps per launch
    int tz[4] = {0, 0, 0, 0};
    int order[4] = {0, 0, 0, 0};  // tile order: 0 = x-tiles of a strip adjacent, 1 = strips of a column adjacent
    int* active = nullptr;  // device [N], batches only
    std::vector<int> active_host;
    double* J = nullptr;    // device [N]
    double* fold_tmp = nullptr;  // device: one FP64 plane of the largest instance (shot sum before the fold)
    double* part = nullptr;
    int* flag = nullptr;
    int* same = nullptr;
    long long bytes = 0;
    std::vector<void*> allocs;
    std::map<void*, size_t> alloc_bytes;
    // timing
    int time_every = 0;
    long long launches[4] = {0, 0, 0, 0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];  // recorded, not yet read
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    double ev_ms[4] = {0.0, 0.0, 0.0, 0.0};  // summed durations of the pairs already read
    long long ev_n[4] = {0, 0, 0, 0};
    // graphs (batches)
    bool use_graphs = false;
    bool capturing = false;
    std::map<int, hipGraphExec_t> graphs;
};

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        aafwi::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        aafwi::set_last_error("host allocation failed");
        return AAFWI_E_NOMEM;
    } catch (...) {
        aafwi::set_last_error("unknown error");
        return AAFWI_E_INVALID;
    }
}

template <typename T>
T* dalloc(Engine* e, size_t count) {
    size_t bytes = sizeof(T) * (count ? count : 1);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{AAFWI_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    e->allocs.push_back(p);
    e->alloc_bytes[p] = bytes;
    e->bytes += (long long)bytes;
    return (T*)p;
}

template <typename T>
void dfree(Engine* e, T*& p) {
    if (!p) return;
    void* v = (void*)p;
    (void)hipFree(v);
    e->allocs.erase(std::remove(e->allocs.begin(), e->allocs.end(), v), e->allocs.end());
    auto it = e->alloc_bytes.find(v);
    if (it != e->alloc_bytes.end()) {
        e->bytes -= (long long)it->second;
        e->alloc_bytes.erase(it);
    }
    p = nullptr;
}

void free_engine(Engine* e) {
    if (!e) return;
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    for (void* p : e->allocs) (void)hipFree(p);
    for (auto& v : e->ev)
        for (auto& x : v) {
            (void)hipEventDestroy(x.first);
            (void)hipEventDestroy(x.second);
        }
    for (auto& x : e->ev_pool) {
        (void)hipEventDestroy(x.first);
        (void)hipEventDestroy(x.second);
    }
    delete e;
}

// Strip height: rows per wave; 0 picks about 8 strips per column of tiles.
int default_tz(int nzp) { return std::max(16, std::min((nzp + 7) / 8, 64)); }

void validate_geometry(const aafwi_geometry& G) {
    AAFWI_REQUIRE(G.nz >= 1 && G.nx >= 1, "create: nz and nx must be >= 1");
    AAFWI_REQUIRE(G.nb >= 1 && G.nb <= 4096, "create: nb must be in [1, 4096]");
    AAFWI_REQUIRE(G.nt >= 1, "create: nt must be >= 1");
    AAFWI_REQUIRE(G.nshots >= 1 && G.nrec >= 1, "create: nshots and nrec must be >= 1");
    AAFWI_REQUIRE(std::isfinite(G.h) && G.h > 0 && std::isfinite(G.dt) && G.dt > 0,
                  "create: h and dt must be positive");
    AAFWI_REQUIRE(std::isfinite(G.vref) && G.vref > 0, "create: vref must be positive");
    AAFWI_REQUIRE(std::isfinite(G.refl) && G.refl > 0, "create: refl must be positive");
    AAFWI_REQUIRE(std::isfinite(G.vmax_bound) && G.vmax_bound > 0, "create: vmax_bound must be positive");
    AAFWI_REQUIRE(G.src_iz && G.src_ix && G.rec_iz && G.rec_ix && G.wavelet, "create: NULL geometry array");
    AAFWI_REQUIRE(G.ckpt_every >= 0, "create: ckpt_every must be >= 0");
    const double cfl = (double)G.vmax_bound * G.dt / G.h;
    if (cfl > 0.55) throw Error{AAFWI_E_CFL, "create: vmax_bound*dt/h = " + std::to_string(cfl) + " exceeds 0.55"};
    const long long nzp = (long long)G.nz + 2LL * G.nb, nxp = (long long)G.nx + 2LL * G.nb;
    // byte offsets inside a plane (plus 16 rows of slack) must stay below 2^31
    AAFWI_REQUIRE(4LL * (nzp + 16) * ((nxp + 63) / 64 * 64) < (1LL << 31), "create: padded plane too large");
    AAFWI_REQUIRE(nzp < 65536, "create: too many padded rows");
    for (int s = 0; s < G.nshots; ++s)
        AAFWI_REQUIRE(G.src_iz[s] >= 0 && G.src_iz[s] < G.nz && G.src_ix[s] >= 0 && G.src_ix[s] < G.nx,
                      "create: source index outside the interior grid");
    for (long long i = 0; i < (long long)G.nshots * G.nrec; ++i)
        AAFWI_REQUIRE(G.rec_iz[i] >= 0 && G.rec_iz[i] < G.nz && G.rec_ix[i] >= 0 && G.rec_ix[i] < G.nx,
                      "create: receiver index outside the interior grid");
    for (int n = 0; n < G.nt; ++n) AAFWI_REQUIRE(std::isfinite(G.wavelet[n]), "create: wavelet must be finite");
}

void add_instance(Engine* e, const aafwi_geometry& G, const aafwi_batch_io* io) {
    validate_geometry(G);
    InstHost I;
    I.nz = G.nz; I.nx = G.nx; I.nb = G.nb; I.nt = G.nt; I.S = G.nshots; I.R = G.nrec;
    I.h = G.h; I.dt = G.dt;
    I.mmin = (float)(1.0 / ((double)G.vmax_bound * (double)G.vmax_bound));
    I.nseg = (G.nt + e->k - 1) / e->k;
    I.wavelet.assign(G.wavelet, G.wavelet + G.nt);
    aafwi::WaveGrid& g = I.g;
    g.nz = G.nz; g.nx = G.nx; g.nb = G.nb;
    g.nzp = G.nz + 2 * G.nb;
    g.nxp = G.nx + 2 * G.nb;
    g.pitch = (g.nxp + 63) / 64 * 64;
    g.plane = (long long)g.nzp * g.pitch;
    g.S = G.nshots;
    g.ntx = g.pitch / 64;
    const double smax = (G.refl >= 1.0f) ? 0.0 : 3.0 * G.vref * std::log(1.0 / (double)G.refl) / (2.0 * G.nb * G.h);
    g.scoef = (float)(smax * G.dt / 2.0);
    g.inv_nb = (float)(1.0 / G.nb);
    I.field = (long long)g.S * g.plane;

    // receiver maps
    std::vector<int> rowmap((size_t)g.S * g.nzp, -1);
    std::vector<int> nrows(g.S, 0);
    for (int s = 0; s < g.S; ++s)
        for (int r = 0; r < G.nrec; ++r) {
            const int zp = G.rec_iz[(long long)s * G.nrec + r] + G.nb;
            int& slot = rowmap[(size_t)s * g.nzp + zp];
            if (slot < 0) slot = nrows[s]++;
        }
    I.nrr = *std::max_element(nrows.begin(), nrows.end());
    std::vector<int> xmap((size_t)g.S * I.nrr * g.pitch, -1);
    std::vector<int> rnext((size_t)g.S * G.nrec, -1);
    for (int s = 0; s < g.S; ++s)
        for (int r = G.nrec - 1; r >= 0; --r) {
            const long long i = (long long)s * G.nrec + r;
            const int zp = G.rec_iz[i] + G.nb, xp = G.rec_ix[i] + G.nb;
            const int slot = rowmap[(size_t)s * g.nzp + zp];
            int& head = xmap[((size_t)s * I.nrr + slot) * g.pitch + xp];
            rnext[i] = head;  // chain in ascending receiver order
            head = r;
        }
    std::vector<int2> src(g.S);
    for (int s = 0; s < g.S; ++s) src[s] = make_int2(G.src_iz[s] + G.nb, G.src_ix[s] + G.nb);

    const size_t ndata = (size_t)g.S * G.nt * G.nrec;
    I.K = dalloc<float>(e, g.plane);
    I.E = dalloc<float>(e, g.plane);
    for (int i = 0; i < 4; ++i) {
        I.F[i] = dalloc<float>(e, I.field);
        I.L[i] = dalloc<float>(e, I.field);
    }
    I.GI = dalloc<float>(e, I.field);
    I.ckpt = dalloc<float>(e, (size_t)I.field * 2 * I.nseg);
    I.qseg = dalloc<float>(e, (size_t)I.field * e->k);
    I.d = (io && io->r) ? io->r : dalloc<float>(e, ndata);
    I.wav = dalloc<float>(e, G.nt);
    I.mkeep = dalloc<float>(e, (size_t)G.nz * G.nx);
    if (io) {
        I.m = io->m;
        I.dobs = io->d_obs;
        I.grad = io->grad;
    }
    I.src = dalloc<int2>(e, g.S);
    I.rowmap = dalloc<int>(e, rowmap.size());
    I.xmap = dalloc<int>(e, xmap.size());
    I.rnext = dalloc<int>(e, rnext.size());
    AAFWI_HIP(hipMemcpy(I.src, src.data(), sizeof(int2) * g.S, hipMemcpyHostToDevice));
    AAFWI_HIP(hipMemcpy(I.rowmap, rowmap.data(), sizeof(int) * rowmap.size(), hipMemcpyHostToDevice));
    AAFWI_HIP(hipMemcpy(I.xmap, xmap.data(), sizeof(int) * xmap.size(), hipMemcpyHostToDevice));
    AAFWI_HIP(hipMemcpy(I.rnext, rnext.data(), sizeof(int) * rnext.size(), hipMemcpyHostToDevice));
    AAFWI_HIP(hipMemcpy(I.wav, I.wavelet.data(), sizeof(float) * G.nt, hipMemcpyHostToDevice));
    // padding columns of every field read as zero forever (stores never reach them)
    for (int i = 0; i < 4; ++i) {
        AAFWI_HIP(hipMemset(I.F[i], 0, sizeof(float) * I.field));
        AAFWI_HIP(hipMemset(I.L[i], 0, sizeof(float) * I.field));
    }
    e->in.push_back(std::move(I));
}

// Tile table of one stepping kernel.  Workgroup i runs on XCD i % 8 and the
// kernels remap workgroup ids so that XCD x receives the x-th contiguous
// eighth of the table.  Each instance's tiles (shot-major, strip, x-tile) are
// cut into 8 contiguous chunks and chunk c of every instance is placed in
// region c, so every XCD holds the same share of every instance (instances
// whose records end early leave every XCD equally); regions are padded to
// equal length with no-op tiles (inst = -1).
std::vector<aafwi::TileRec> tile_table(Engine* e, int kid, bool two) {
    const int width = two ? aafwi::kTile2 : 64;
    constexpr int kX = 8, kWaves = 4;
    std::vector<std::vector<aafwi::TileRec>> region(kX);
    for (int i = 0; i < (int)e->in.size(); ++i) {
        const aafwi::WaveGrid& g = e->in[i].g;
        // one-step kernels keep a strip's receiver rows one per lane: at most 64 rows
        const int tz_set = e->in[i].tz[kid] ? e->in[i].tz[kid] : (e->tz[kid] ? e->tz[kid] : default_tz(g.nzp));
        const int tz = std::min(two ? tz_set : std::min(tz_set, 64), g.nzp);
        const int ntx = (g.nxp + width - 1) / width;
        std::vector<aafwi::TileRec> t;
        const int ord = e->order[kid];
        if (ord <= 1) {
            for (int s = 0; s < g.S; ++s) {
                if (ord == 0) {
                    for (int z0 = 0; z0 < g.nzp; z0 += tz)
                        for (int tx = 0; tx < ntx; ++tx)
                            t.push_back({i, s, tx * width, (z0 << 16) | std::min(z0 + tz, g.nzp)});
                } else {
                    for (int tx = 0; tx < ntx; ++tx)
                        for (int z0 = 0; z0 < g.nzp; z0 += tz)
                            t.push_back({i, s, tx * width, (z0 << 16) | std::min(z0 + tz, g.nzp)});
                }
            }
        } else {
            // groups of `ord` shots innermost: the same tile of several shots
            // runs at about the same time, so they share its Kp rows in L2
            for (int s0 = 0; s0 < g.S; s0 += ord)
                for (int z0 = 0; z0 < g.nzp; z0 += tz)
                    for (int tx = 0; tx < ntx; ++tx)
                        for (int s = s0; s < std::min(s0 + ord, g.S); ++s)
                            t.push_back({i, s, tx * width, (z0 << 16) | std::min(z0 + tz, g.nzp)});
        }
        const size_t n = t.size();
        for (int c = 0; c < kX; ++c)
            region[c].insert(region[c].end(), t.begin() + n * c / kX, t.begin() + n * (c + 1) / kX);
    }
    size_t L = 0;
    for (auto& r : region) L = std::max(L, r.size());
    L = (L + kWaves - 1) / kWaves * kWaves;
    std::vector<aafwi::TileRec> all;
    all.reserve(L * kX);
    for (int c = 0; c < kX; ++c) {
        all.insert(all.end(), region[c].begin(), region[c].end());
        all.resize((size_t)(c + 1) * L, aafwi::TileRec{-1, 0, 0, 0});
    }
    return all;
}

void upload_tiles(Engine* e, aafwi::TileRec*& dst, int& count, const std::vector<aafwi::TileRec>& all) {
    dfree(e, dst);
    dst = dalloc<aafwi::TileRec>(e, all.size());
    AAFWI_HIP(hipMemcpy(dst, all.data(), sizeof(aafwi::TileRec) * all.size(), hipMemcpyHostToDevice));
    count = (int)all.size();
}

void build_tiles(Engine* e, int kid) {
    upload_tiles(e, e->dtiles[kid], e->ntiles[kid], tile_table(e, kid, false));
    if (kid < 3) upload_tiles(e, e->dtiles2[kid], e->ntiles2[kid], tile_table(e, kid, true));
}

// Device descriptors of the instances (buffers, sizes, segment layout).
void upload_insts(Engine* e) {
    const int N = (int)e->in.size();
    std::vector<aafwi::Inst> tab(N);
    for (int i = 0; i < N; ++i) {
        const InstHost& I = e->in[i];
        aafwi::Inst& D = tab[i];
        D.g = I.g;
        D.K = I.K; D.E = I.E;
        for (int j = 0; j < 4; ++j) {
            D.F[j] = I.F[j];
            D.L[j] = I.L[j];
        }
        D.GI = I.GI;
        D.ckpt = I.ckpt; D.qseg = I.qseg; D.d = I.d; D.r = I.d; D.wav = I.wav;
        D.src = {I.src};
        D.rm = {I.rowmap, I.xmap, I.rnext, I.nrr, I.R};
        D.nt = I.nt; D.nseg = I.nseg; D.k = e->k;
        D.h2 = I.h * I.h;
        D.field = I.field;
    }
    AAFWI_HIP(hipMemcpy(e->dinst, tab.data(), sizeof(aafwi::Inst) * N, hipMemcpyHostToDevice));
}

void finalize(Engine* e) {
    const int N = (int)e->in.size();
    e->k_ckpt = e->k;
    e->dinst = dalloc<aafwi::Inst>(e, N);
    upload_insts(e);
    for (int kid = 0; kid < 4; ++kid) build_tiles(e, kid);
    // Default launch mode: two steps per launch once one time level pair of
    // every instance (the one-step working set) outgrows the 256 MB
    // Infinity Cache; below that, one-step kernels re-read their planes
    // from the cache and are faster.  The autotuner measures both.
    long long pair_bytes = 0;
    for (const InstHost& I : e->in) pair_bytes += 2LL * I.field * (long long)sizeof(float);
    for (bool& t : e->tb) t = pair_bytes > (256LL << 20);
    e->J = dalloc<double>(e, N);
    long long max_plane = 0;
    for (const InstHost& I : e->in) max_plane = std::max(max_plane, (long long)I.g.plane);
    e->fold_tmp = dalloc<double>(e, (size_t)max_plane);
    e->part = dalloc<double>(e, aafwi::kReduceBlocks);
    e->flag = dalloc<int>(e, 1);
    e->same = dalloc<int>(e, 1);
    AAFWI_HIP(hipMemset(e->flag, 0, sizeof(int)));
    AAFWI_HIP(hipMemset(e->J, 0, sizeof(double) * N));
    if (e->is_batch) {
        e->active = dalloc<int>(e, N);
        e->active_host.assign(N, 1);
        AAFWI_HIP(hipMemcpy(e->active, e->active_host.data(), sizeof(int) * N, hipMemcpyHostToDevice));
    }
    AAFWI_HIP(hipDeviceSynchronize());
}

// Reads every recorded pair whose end event has completed (all of them when
// ``wait``), adds its duration to the per-kernel sums and returns the pair to
// the pool, so that a run of any length is sampled over its whole span.
void harvest_events(Engine* e, bool wait) {
    if (wait) AAFWI_HIP(hipStreamSynchronize(e->stream));
    for (int id = 0; id < 4; ++id) {
        auto& v = e->ev[id];
        size_t keep = 0;
        for (size_t i = 0; i < v.size(); ++i) {
            if (!wait && hipEventQuery(v[i].second) != hipSuccess) {
                v[keep++] = v[i];
                continue;
            }
            float ms = 0.0f;
            AAFWI_HIP(hipEventElapsedTime(&ms, v[i].first, v[i].second));
            e->ev_ms[id] += ms;
            e->ev_n[id] += 1;
            e->ev_pool.push_back(v[i]);
        }
        v.resize(keep);
    }
    // a query of a pending event leaves "not ready" as the last error
    if (!wait) (void)hipGetLastError();
}

// Event pair around a stepping launch when sampling is on (not inside
// captures); when the pool is empty, the completed pairs are read first.
struct Timed {
    Engine* e;
    int id;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    Timed(Engine* e_, int id_) : e(e_), id(id_) {
        if (!e->capturing && e->time_every > 0 && (e->launches[id] % e->time_every) == 0) {
            if (e->ev_pool.empty()) harvest_events(e, false);
            if (!e->ev_pool.empty()) {
                ev = e->ev_pool.back();
                e->ev_pool.pop_back();
                AAFWI_HIP(hipEventRecord(ev.first, e->stream));
            }
        }
        e->launches[id] += 1;
    }
    ~Timed() {
        if (ev.first) {
            (void)hipEventRecord(ev.second, e->stream);
            e->ev[id].push_back(ev);
        }
    }
};

void step(Engine* e, int kid, const aafwi::StepArgs& a) {
    Timed t(e, kid);
    aafwi::launch_step(kid, e->stream, e->dtiles[kid], e->ntiles[kid], e->dinst, a);
}

void step2(Engine* e, int kid, const aafwi::StepArgs& a) {
    Timed t(e, kid);
    aafwi::launch_step2(kid, e->stream, e->dtiles2[kid], e->ntiles2[kid], e->dinst, a);
}

// Forward launch of the full-storage layout: it writes q-hat beside u^{n+1},
// the traffic of a recompute launch, so it takes the recompute kernel's launch
// mode, tile table and timing slot (the recompute pass itself never runs).
void step_keep_q(Engine* e, const aafwi::StepArgs& a) {
    constexpr int kid = AAFWI_K_REC_STEP;
    Timed t(e, kid);
    if (e->tb[kid])
        aafwi::launch_step2(AAFWI_K_FWD_STEP, e->stream, e->dtiles2[kid], e->ntiles2[kid], e->dinst, a);
    else
        aafwi::launch_step(AAFWI_K_FWD_STEP, e->stream, e->dtiles[kid], e->ntiles[kid], e->dinst, a);
}

void model_prep(Engine* e, int i, const float* m) {
    const InstHost& I = e->in[i];
    const double c2 = ((double)I.dt / (double)I.h) * ((double)I.dt / (double)I.h);
    aafwi::launch_model_prep(e->stream, I.g, (float)c2, I.mmin, m, I.K, e->flag, e->active, i);
}

int max_nt(const Engine* e) {
    int v = 0;
    for (auto& I : e->in) v = std::max(v, I.nt);
    return v;
}

// Forward pass of every (active) instance; models m[i], samples into d_ovr (if
// set) or the instances' own data buffers.
// Every instance holds its checkpoint and q-plane buffers (a failed layout
// switch that could not restore the previous layout leaves them unset).
void require_layout(const Engine* e) {
    for (const InstHost& I : e->in)
        if (!I.ckpt || !I.qseg) throw Error{AAFWI_E_STATE, "storage layout lost after a failed set_full_storage"};
}

void run_forward(Engine* e, const std::vector<const float*>& m, float* d_ovr, bool keep) {
    require_layout(e);
    const int N = (int)e->in.size();
    for (int i = 0; i < N; ++i) {
        model_prep(e, i, m[i]);
        for (int j = 0; j < 4; ++j) aafwi::launch_zero(e->stream, e->in[i].F[j], e->in[i].field);
    }
    aafwi::StepArgs a{0, 0, keep ? 1 : 0, d_ovr, nullptr, e->active};
    const int T = max_nt(e);
    const bool keep_q = keep && e->keep_q;
    a.keep_q = keep_q ? 1 : 0;
    const bool two = e->tb[keep_q ? AAFWI_K_REC_STEP : AAFWI_K_FWD_STEP];
    for (int n = 0; n < T; n += two ? 2 : 1) {
        a.n = n;
        if (keep_q)
            step_keep_q(e, a);
        else if (two)
            step2(e, AAFWI_K_FWD_STEP, a);
        else
            step(e, AAFWI_K_FWD_STEP, a);
    }
    if (keep)
        for (int i = 0; i < N; ++i)
            aafwi::launch_copy(e->stream, (long long)e->in[i].nz * e->in[i].nx, m[i], e->in[i].mkeep, e->active, i);
    for (int i = 0; i < N; ++i)
        if (e->active_host.empty() || e->active_host[i]) e->in[i].have_ckpt = keep;
}

int seg_len(const Engine* e, const InstHost& I, int J) {
    const int j = I.nseg - 1 - J;
    if (j < 0) return 0;
    return std::min(e->k, I.nt - j * e->k);
}

// Backward pass of every (active) instance from its kept checkpoints; the
// adjoint source is r_ovr (if set) or the instances' own residual buffers.
void run_backward(Engine* e, const float* r_ovr, const std::vector<float*>& grad) {
    require_layout(e);
    const int N = (int)e->in.size();
    int maxseg = 0;
    for (int i = 0; i < N; ++i) {
        InstHost& I = e->in[i];
        model_prep(e, i, I.mkeep);  // Kp of the kept run (a Born call may have replaced it)
        for (int j = 0; j < 4; ++j) aafwi::launch_zero(e->stream, I.L[j], I.field);
        aafwi::launch_zero(e->stream, I.GI, I.field);
        maxseg = std::max(maxseg, I.nseg);
    }
    aafwi::StepArgs a{0, 0, 0, nullptr, r_ovr, e->active};
    for (int J = 0; J < maxseg; ++J) {
        int len = 0;
        for (auto& I : e->in) len = std::max(len, seg_len(e, I, J));
        a.seg = J;
        // recompute and adjoint choose their launch mode independently: the
        // segment's q planes do not depend on it, and the adjoint keeps one
        // mode (one buffer convention) for the whole pass.  Full storage: the
        // kept forward already wrote the q planes of its one segment.
        if (!e->keep_q) {
            const bool two = e->tb[AAFWI_K_REC_STEP];
            for (int tt = 0; tt < len; tt += two ? 2 : 1) {
                a.n = tt;
                if (two)
                    step2(e, AAFWI_K_REC_STEP, a);
                else
                    step(e, AAFWI_K_REC_STEP, a);
            }
        }
        if (e->tb[AAFWI_K_ADJ_STEP]) {
            for (int tt = len - 1; tt >= 0; tt -= 2) {
                a.n = tt;
                step2(e, AAFWI_K_ADJ_STEP, a);
            }
        } else {
            for (int tt = len - 1; tt >= 0; --tt) {
                a.n = tt;
                step(e, AAFWI_K_ADJ_STEP, a);
            }
        }
    }
    for (int i = 0; i < N; ++i) {
        const InstHost& I = e->in[i];
        const double inv_dt2 = 1.0 / ((double)I.dt * (double)I.dt);
        aafwi::launch_fold(e->stream, I.g, (float)inv_dt2, I.GI, e->fold_tmp, I.mkeep, I.mmin, grad[i], e->active, i);
    }
}

void residuals(Engine* e, const std::vector<const float*>& d, const std::vector<const float*>& dobs,
               const std::vector<float*>& r) {
    for (int i = 0; i < (int)e->in.size(); ++i) {
        const InstHost& I = e->in[i];
        aafwi::launch_residual_misfit(e->stream, (long long)I.S * I.nt * I.R, d[i], dobs[i], r[i], e->part, e->J + i,
                                      e->active, i);
    }
}

// True when m is bitwise the model of instance 0's kept checkpoints (synchronises).
bool kept_model_is(Engine* e, const float* m) {
    InstHost& I = e->in[0];
    if (!I.have_ckpt) return false;
    aafwi::launch_compare(e->stream, (long long)I.nz * I.nx, m, I.mkeep, e->same);
    int v = 0;
    AAFWI_HIP(hipMemcpyAsync(&v, e->same, sizeof(int), hipMemcpyDeviceToHost, e->stream));
    AAFWI_HIP(hipStreamSynchronize(e->stream));
    return v == 1;
}

int timing_enable(Engine* e, int every) {
    harvest_events(e, true);
    for (int id = 0; id < 4; ++id) {
        e->ev_ms[id] = 0.0;
        e->ev_n[id] = 0;
        e->launches[id] = 0;
    }
    e->time_every = every;
    if (every > 0) {
        // timing-only events: no system-scope fence at record (its cache
        // writeback would be timed with the kernel); pairs are read once their
        // end event has completed and then recorded again
        while (e->ev_pool.size() < 4096) {
            hipEvent_t a, b;
            AAFWI_HIP(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
            AAFWI_HIP(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
            e->ev_pool.emplace_back(a, b);
        }
    }
    return AAFWI_OK;
}

int timing_read(Engine* e, int id, double* mean_ms, int64_t* count) {
    AAFWI_REQUIRE(mean_ms && count && id >= 0 && id < 4, "kernel_timing_read: bad argument");
    harvest_events(e, true);
    *count = (int64_t)e->ev_n[id];
    *mean_ms = e->ev_n[id] ? e->ev_ms[id] / (double)e->ev_n[id] : 0.0;
    return AAFWI_OK;
}

int set_tile(Engine* e, int kernel_id, int rows) {
    AAFWI_REQUIRE(rows >= 0 && rows <= 120, "set_tile: rows per wave must be in [0, 120]");
    AAFWI_REQUIRE(kernel_id >= -1 && kernel_id < 4, "set_tile: kernel_id must be -1 or a kernel id");
    AAFWI_HIP(hipStreamSynchronize(e->stream));
    for (int k = 0; k < 4; ++k)
        if (kernel_id == -1 || kernel_id == k) {
            e->tz[k] = rows;
            build_tiles(e, k);
        }
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
    return AAFWI_OK;
}

int set_tile_order(Engine* e, int kernel_id, int order) {
    AAFWI_REQUIRE(order >= 0 && order <= 64, "set_tile_order: order must be 0, 1 or a shot group size up to 64");
    AAFWI_REQUIRE(kernel_id >= -1 && kernel_id < 4, "set_tile_order: kernel_id must be -1 or a kernel id");
    AAFWI_HIP(hipStreamSynchronize(e->stream));
    for (int k = 0; k < 4; ++k)
        if (kernel_id == -1 || kernel_id == k) {
            e->order[k] = order;
            build_tiles(e, k);
        }
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
    return AAFWI_OK;
}

int set_time_blocking(Engine* e, int kernel_id, int enable) {
    AAFWI_REQUIRE(kernel_id >= -1 && kernel_id < 3, "set_time_blocking: kernel_id must be -1, 0, 1 or 2");
    AAFWI_HIP(hipStreamSynchronize(e->stream));
    for (int k = 0; k < 3; ++k)
        if (kernel_id == -1 || kernel_id == k) e->tb[k] = enable != 0;
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
    return AAFWI_OK;
}

// Switch between the checkpointed layout (checkpoints every k_ckpt steps, one
// segment of q planes, recomputed per segment) and full storage (q planes of
// every step, written by the kept forward).  Kept state is dropped either way.
// On an allocation failure the previous layout is restored and the error
// (AAFWI_E_NOMEM) rethrown.
int set_full_storage(Engine* e, bool on) {
    AAFWI_HIP(hipStreamSynchronize(e->stream));
    if (on == e->keep_q) return AAFWI_OK;
    auto release = [&]() {
        for (InstHost& I : e->in) {
            dfree(e, I.ckpt);
            dfree(e, I.qseg);
            I.have_ckpt = false;
        }
    };
    auto layout = [&](bool full) {
        e->k = full ? max_nt(e) : e->k_ckpt;
        for (InstHost& I : e->in) {
            I.nseg = (I.nt + e->k - 1) / e->k;
            I.ckpt = dalloc<float>(e, (size_t)I.field * 2 * I.nseg);
            I.qseg = dalloc<float>(e, (size_t)I.field * (full ? I.nt : e->k));
        }
    };
    release();
    try {
        layout(on);
    } catch (const Error&) {
        release();
        layout(e->keep_q);  // the memory just released holds it again
        upload_insts(e);
        throw;
    }
    e->keep_q = on;
    upload_insts(e);
    return AAFWI_OK;
}

// Run `body` directly, or (graphs on) capture it once under `key` and replay.
template <typename F>
void maybe_graph(Engine* e, int key, F&& body) {
    if (!e->use_graphs) {
        body();
        return;
    }
    auto it = e->graphs.find(key);
    if (it == e->graphs.end()) {
        hipGraph_t graph = nullptr;
        AAFWI_HIP(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
        e->capturing = true;
        try {
            body();
        } catch (...) {
            e->capturing = false;
            hipGraph_t g2 = nullptr;
            (void)hipStreamEndCapture(e->stream, &g2);
            if (g2) (void)hipGraphDestroy(g2);
            throw;
        }
        e->capturing = false;
        AAFWI_HIP(hipStreamEndCapture(e->stream, &graph));
        hipGraphExec_t exec = nullptr;
        const hipError_t err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        AAFWI_HIP(err);
        it = e->graphs.emplace(key, exec).first;
    }
    AAFWI_HIP(hipGraphLaunch(it->second, e->stream));
}

}  // namespace

// ---------------------------------------------------------------------------
// single context
// ---------------------------------------------------------------------------
struct aafwi_ctx {
    Engine* e = nullptr;
};

extern "C" const char* aafwi_last_error(void) { return aafwi::g_last_error.c_str(); }

extern "C" int aafwi_create(const aafwi_geometry* gp, aafwi_stream stream, aafwi_ctx** out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(gp != nullptr && out != nullptr, "create: NULL argument");
        *out = nullptr;
        validate_geometry(*gp);
        Engine* e = new Engine{};
        try {
            e->stream = (hipStream_t)stream;
            e->k = gp->ckpt_every > 0 ? std::min(gp->ckpt_every, gp->nt) : std::min(50, gp->nt);
            add_instance(e, *gp, nullptr);
            finalize(e);
        } catch (...) {
            free_engine(e);
            throw;
        }
        *out = new aafwi_ctx{e};
        return AAFWI_OK;
    });
}

extern "C" int aafwi_destroy(aafwi_ctx* c) {
    return guarded([&]() -> int {
        if (!c) return AAFWI_OK;
        (void)hipStreamSynchronize(c->e->stream);
        free_engine(c->e);
        delete c;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_device_bytes(const aafwi_ctx* c, int64_t* bytes) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && bytes, "device_bytes: NULL argument");
        *bytes = c->e->bytes;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_sync(aafwi_ctx* c) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "sync: NULL context");
        Engine* e = c->e;
        AAFWI_HIP(hipStreamSynchronize(e->stream));
        int f = 0;
        AAFWI_HIP(hipMemcpy(&f, e->flag, sizeof(int), hipMemcpyDeviceToHost));
        if (f) {
            AAFWI_HIP(hipMemset(e->flag, 0, sizeof(int)));
            throw Error{AAFWI_E_NONFINITE, "a model value was non-positive or non-finite"};
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_forward_model(aafwi_ctx* c, const float* m, float* d, int keep_ckpt) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && m && d, "forward_model: NULL argument");
        run_forward(c->e, {m}, d, keep_ckpt != 0);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_residual_misfit(aafwi_ctx* c, const float* d, const float* d_obs, float* r, double* J) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && d && d_obs && r && J, "residual_misfit: NULL argument");
        const InstHost& I = c->e->in[0];
        aafwi::launch_residual_misfit(c->e->stream, (long long)I.S * I.nt * I.R, d, d_obs, r, c->e->part, J, nullptr,
                                      0);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_adjoint_gradient(aafwi_ctx* c, const float* m, const float* d_obs, float* grad, double* J) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && m && d_obs && grad && J, "adjoint_gradient: NULL argument");
        Engine* e = c->e;
        InstHost& I = e->in[0];
        run_forward(e, {m}, I.d, true);
        aafwi::launch_residual_misfit(e->stream, (long long)I.S * I.nt * I.R, I.d, d_obs, I.d, e->part, J, nullptr, 0);
        run_backward(e, I.d, {grad});
        return AAFWI_OK;
    });
}

extern "C" int aafwi_adjoint_from_residual(aafwi_ctx* c, const float* r, float* grad) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && r && grad, "adjoint_from_residual: NULL argument");
        if (!c->e->in[0].have_ckpt)
            throw Error{AAFWI_E_STATE, "adjoint_from_residual: no kept checkpoints (call forward_model with keep_ckpt=1)"};
        run_backward(c->e, r, {grad});
        return AAFWI_OK;
    });
}

extern "C" int aafwi_born(aafwi_ctx* c, const float* m0, const float* dm, float* d_scat) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && m0 && dm && d_scat, "born: NULL argument");
        Engine* e = c->e;
        InstHost& I = e->in[0];
        // the kept checkpoints are untouched; Kp is rebuilt before any backward pass
        model_prep(e, 0, m0);
        aafwi::launch_born_prep(e->stream, I.g, I.mmin, m0, dm, I.E);
        for (int j = 0; j < 2; ++j) {
            aafwi::launch_zero(e->stream, I.F[j], I.field);
            aafwi::launch_zero(e->stream, I.L[j], I.field);
        }
        aafwi::StepArgs a{0, 0, 0, d_scat, nullptr, nullptr};
        for (int n = 0; n < I.nt; ++n) {
            a.n = n;
            step(e, AAFWI_K_BORN_STEP, a);
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_born_adjoint(aafwi_ctx* c, const float* m0, const float* y, float* image) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && m0 && y && image, "born_adjoint: NULL argument");
        Engine* e = c->e;
        if (!kept_model_is(e, m0)) run_forward(e, {m0}, e->in[0].d, true);
        run_backward(e, y, {image});
        return AAFWI_OK;
    });
}

extern "C" int aafwi_kernel_timing(aafwi_ctx* c, int every) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && every >= 0, "kernel_timing: bad argument");
        return timing_enable(c->e, every);
    });
}

extern "C" int aafwi_kernel_timing_read(aafwi_ctx* c, int id, double* mean_ms, int64_t* count) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "kernel_timing_read: NULL context");
        return timing_read(c->e, id, mean_ms, count);
    });
}

extern "C" int aafwi_set_tile(aafwi_ctx* c, int32_t kernel_id, int32_t rows) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "set_tile: NULL context");
        return set_tile(c->e, kernel_id, rows);
    });
}

extern "C" int aafwi_set_tile_order(aafwi_ctx* c, int32_t kernel_id, int32_t order) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "set_tile_order: NULL context");
        return set_tile_order(c->e, kernel_id, order);
    });
}

extern "C" int aafwi_set_time_blocking(aafwi_ctx* c, int enable) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "set_time_blocking: NULL context");
        return set_time_blocking(c->e, -1, enable);
    });
}

extern "C" int aafwi_set_time_blocking_kernel(aafwi_ctx* c, int32_t kernel_id, int enable) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "set_time_blocking_kernel: NULL context");
        return set_time_blocking(c->e, kernel_id, enable);
    });
}

extern "C" int aafwi_set_full_storage(aafwi_ctx* c, int enable) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "set_full_storage: NULL context");
        return set_full_storage(c->e, enable != 0);
    });
}

extern "C" int aafwi_get_full_storage(const aafwi_ctx* c, int* enabled) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && enabled, "get_full_storage: NULL argument");
        *enabled = c->e->keep_q ? 1 : 0;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_get_time_blocking(const aafwi_ctx* c, int* mask) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && mask, "get_time_blocking: NULL argument");
        *mask = (c->e->tb[0] ? 1 : 0) | (c->e->tb[1] ? 2 : 0) | (c->e->tb[2] ? 4 : 0);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_get_tile(const aafwi_ctx* c, int32_t kernel_id, int32_t* rows) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && rows && kernel_id >= 0 && kernel_id < 4, "get_tile: bad argument");
        const int tz = c->e->tz[kernel_id];
        *rows = std::min(tz ? tz : default_tz(c->e->in[0].g.nzp), c->e->in[0].g.nzp);
        return AAFWI_OK;
    });
}

// ---------------------------------------------------------------------------
// batches of uneven instances
// ---------------------------------------------------------------------------
struct aafwi_batch {
    Engine* e = nullptr;
};

namespace {
std::vector<const float*> batch_m(Engine* e) {
    std::vector<const float*> v;
    for (auto& I : e->in) v.push_back(I.m);
    return v;
}
}  // namespace

extern "C" int aafwi_batch_create(const aafwi_geometry* geoms, const aafwi_batch_io* io, int32_t ninst,
                                  int32_t ckpt_every, aafwi_stream stream, aafwi_batch** out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(geoms && io && out && ninst >= 1, "batch_create: bad argument");
        for (int i = 0; i < ninst; ++i)
            AAFWI_REQUIRE(io[i].m && io[i].d_obs && io[i].r && io[i].grad, "batch_create: NULL instance buffer");
        AAFWI_REQUIRE(ckpt_every >= 0, "batch_create: ckpt_every must be >= 0");
        *out = nullptr;
        int ntmax = 0;
        for (int i = 0; i < ninst; ++i) {
            validate_geometry(geoms[i]);
            ntmax = std::max(ntmax, geoms[i].nt);
        }
        Engine* e = new Engine{};
        try {
            e->stream = (hipStream_t)stream;
            e->is_batch = true;
            e->k = ckpt_every > 0 ? std::min(ckpt_every, ntmax) : std::min(50, ntmax);
            for (int i = 0; i < ninst; ++i) add_instance(e, geoms[i], &io[i]);
            finalize(e);
        } catch (...) {
            free_engine(e);
            throw;
        }
        *out = new aafwi_batch{e};
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_destroy(aafwi_batch* b) {
    return guarded([&]() -> int {
        if (!b) return AAFWI_OK;
        (void)hipStreamSynchronize(b->e->stream);
        free_engine(b->e);
        delete b;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_misfits(aafwi_batch* b, double* J) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b && J, "batch_misfits: NULL argument");
        AAFWI_HIP(hipMemcpyAsync(J, b->e->J, sizeof(double) * b->e->in.size(), hipMemcpyDeviceToDevice, b->e->stream));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_set_active(aafwi_batch* b, const uint8_t* active) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_set_active: NULL batch");
        const int N = (int)b->e->in.size();
        std::vector<int> v(N, 1);
        if (active)
            for (int i = 0; i < N; ++i) v[i] = active[i] ? 1 : 0;
        AAFWI_HIP(hipStreamSynchronize(b->e->stream));
        AAFWI_HIP(hipMemcpy(b->e->active, v.data(), sizeof(int) * N, hipMemcpyHostToDevice));
        b->e->active_host = v;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_forward(aafwi_batch* b, int keep_ckpt) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_forward: NULL batch");
        Engine* e = b->e;
        maybe_graph(e, keep_ckpt ? 1 : 0, [&]() {
            run_forward(e, batch_m(e), nullptr, keep_ckpt != 0);
            std::vector<const float*> d, dobs;
            std::vector<float*> r;
            for (auto& I : e->in) {
                d.push_back(I.d);
                dobs.push_back(I.dobs);
                r.push_back(I.d);
            }
            residuals(e, d, dobs, r);
        });
        // host-side state of the kept runs: a graph replay does not run the
        // body above, so it is set here for replays and direct calls alike
        for (int i = 0; i < (int)e->in.size(); ++i)
            if (e->active_host[i]) e->in[i].have_ckpt = keep_ckpt != 0;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_backward(aafwi_batch* b) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_backward: NULL batch");
        Engine* e = b->e;
        for (int i = 0; i < (int)e->in.size(); ++i)
            if (e->active_host[i] && !e->in[i].have_ckpt)
                throw Error{AAFWI_E_STATE, "batch_backward: an active instance has no kept checkpoints"};
        maybe_graph(e, 2, [&]() {
            std::vector<float*> grad;
            for (auto& I : e->in) grad.push_back(I.grad);
            run_backward(e, nullptr, grad);
        });
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_use_graphs(aafwi_batch* b, int enable) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_use_graphs: NULL batch");
        AAFWI_REQUIRE(!enable || b->e->stream != nullptr, "batch_use_graphs: graph capture needs a non-null stream");
        AAFWI_HIP(hipStreamSynchronize(b->e->stream));
        b->e->use_graphs = enable != 0;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_device_bytes(const aafwi_batch* b, int64_t* bytes) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b && bytes, "batch_device_bytes: NULL argument");
        *bytes = b->e->bytes;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_set_tile(aafwi_batch* b, int32_t kernel_id, int32_t rows) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_set_tile: NULL batch");
        return set_tile(b->e, kernel_id, rows);
    });
}

extern "C" int aafwi_batch_set_instance_tile(aafwi_batch* b, int32_t inst, int32_t kernel_id, int32_t rows) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_set_instance_tile: NULL batch");
        Engine* e = b->e;
        AAFWI_REQUIRE(inst >= 0 && inst < (int)e->in.size(), "batch_set_instance_tile: instance out of range");
        AAFWI_REQUIRE(rows >= 0 && rows <= 120, "batch_set_instance_tile: rows per wave must be in [0, 120]");
        AAFWI_REQUIRE(kernel_id >= -1 && kernel_id < 4, "batch_set_instance_tile: kernel_id must be -1 or a kernel id");
        AAFWI_HIP(hipStreamSynchronize(e->stream));
        for (int k = 0; k < 4; ++k)
            if (kernel_id == -1 || kernel_id == k) {
                e->in[inst].tz[k] = rows;
                build_tiles(e, k);
            }
        for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
        e->graphs.clear();
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_get_time_blocking(const aafwi_batch* b, int* mask) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b && mask, "batch_get_time_blocking: NULL argument");
        *mask = (b->e->tb[0] ? 1 : 0) | (b->e->tb[1] ? 2 : 0) | (b->e->tb[2] ? 4 : 0);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_set_time_blocking(aafwi_batch* b, int enable) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_set_time_blocking: NULL batch");
        return set_time_blocking(b->e, -1, enable);
    });
}

extern "C" int aafwi_batch_kernel_timing(aafwi_batch* b, int every) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b && every >= 0, "batch_kernel_timing: bad argument");
        return timing_enable(b->e, every);
    });
}

extern "C" int aafwi_batch_kernel_timing_read(aafwi_batch* b, int id, double* mean_ms, int64_t* count) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b, "batch_kernel_timing_read: NULL batch");
        return timing_read(b->e, id, mean_ms, count);
    });
}

// ---------------------------------------------------------------------------
// residual and misfit without any allocation
// ---------------------------------------------------------------------------
namespace {

// FP64 partial sums of the misfit reduction (one per reduction block), shared
// by every call on a device.  In host code this name is only a stand-in for
// the device array: its device address comes from hipGetSymbolAddress.
constexpr int kScratchDoubles = aafwi::kReduceBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
constexpr long long kMaxMisfitElems = 1LL << 40;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// (with that device current) and kept.
double* scratch_on_current_device() {
    int dev = -1;
    AAFWI_HIP(hipGetDevice(&dev));
    AAFWI_REQUIRE(dev >= 0 && dev < kMaxDevices, "residual_misfit_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        AAFWI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        AAFWI_REQUIRE(p != nullptr, "residual_misfit_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = (double*)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int aafwi_residual_misfit_noalloc(aafwi_stream stream, int64_t n, const float* d, const float* d_obs,
                                             float* r, double* J) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(d && d_obs && r && J, "residual_misfit_noalloc: NULL argument");
        AAFWI_REQUIRE(n >= 1, "residual_misfit_noalloc: n must be at least 1");
        AAFWI_REQUIRE(n <= kMaxMisfitElems, "residual_misfit_noalloc: n exceeds the 2^40-element limit");
        double* part = scratch_on_current_device();
        // the reduction writes every one of its kReduceBlocks partials before
        // the final sum reads them, so nothing left by an earlier call is read
        aafwi::launch_residual_misfit((hipStream_t)stream, (long long)n, d, d_obs, r, part, J, nullptr, 0);
        return AAFWI_OK;
    });
}
