// Host runtime and C ABI of the wave-equation calls: context creation
// (geometry validation, receiver maps, device scratch), the forward pass with
// checkpoints, the checkpointed backward pass (recompute + adjoint + imaging),
// Born modelling and its adjoint, and event timing of the stepping kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
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

struct aafwi_ctx {
    // geometry (host copy)
    int nz = 0, nx = 0, nb = 0, nt = 0, S = 0, R = 0, k = 0, nseg = 0;
    float h = 0, dt = 0, vref = 0, refl = 0, vmax = 0;
    std::vector<float> wavelet;
    aafwi::WaveGrid g{};
    aafwi::WaveGrid gk[4];  // per stepping kernel (tile height may differ)
    hipStream_t stream = nullptr;
    long long field = 0;  // S * plane floats

    // device scratch
    float* K = nullptr;      // Kp on the padded grid [plane]
    float* E = nullptr;      // Born dm/m0 [plane]
    float* F0 = nullptr;     // forward wavefields [S][plane] x 2
    float* F1 = nullptr;
    float* L0 = nullptr;     // adjoint (or scattered) wavefields [S][plane] x 2
    float* L1 = nullptr;
    float* GI = nullptr;     // per-shot image accumulators [S][plane]
    float* ckpt = nullptr;   // [nseg][2][S][plane]
    float* qseg = nullptr;   // [k][S][plane]
    float* dwork = nullptr;  // [S][nt][R]
    double* part = nullptr;  // reduction partials
    int* flag = nullptr;     // model-validity flag
    float* mkeep = nullptr;  // model of the kept checkpoints [nz][nx]
    int* same = nullptr;     // comparison flag
    int2* src = nullptr;     // [S]
    int* rowmap = nullptr;   // [S][nzp]
    int* xmap = nullptr;     // [S][nrr][pitch]
    int* rnext = nullptr;    // [S*R]
    int nrr = 0;
    long long bytes = 0;

    bool have_ckpt = false;

    // timing
    int time_every = 0;
    long long launches[4] = {0, 0, 0, 0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
};

namespace {

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

void dalloc(aafwi_ctx* c, void** p, size_t bytes) {
    if (bytes == 0) bytes = 4;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{AAFWI_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    c->bytes += (long long)bytes;
}

void free_ctx(aafwi_ctx* c) {
    if (!c) return;
    void* ps[] = {c->K, c->E, c->F0, c->F1, c->L0, c->L1, c->GI, c->ckpt, c->qseg,
                  c->dwork, c->part, c->flag, c->src, c->rowmap, c->xmap, c->rnext, c->mkeep, c->same};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    for (auto& v : c->ev)
        for (auto& e : v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    for (auto& e : c->ev_pool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete c;
}

// Strip height: rows per wave; 0 picks about 8 strips per column of tiles.
void apply_tile(aafwi::WaveGrid& g, int rows) {
    int tz = rows;
    if (tz == 0) tz = std::max(16, std::min((g.nzp + 7) / 8, 64));
    g.tz = std::min(tz, g.nzp);
    g.nzs = (g.nzp + g.tz - 1) / g.tz;
    g.ntiles = g.ntx * g.nzs * g.S;
}

aafwi::RecMaps maps(const aafwi_ctx* c) { return {c->rowmap, c->xmap, c->rnext, c->nrr, c->R}; }
aafwi::SrcNodes srcs(const aafwi_ctx* c) { return {c->src}; }

// Event pair around a launch of kernel `id` when sampling is on.
struct Timed {
    aafwi_ctx* c;
    int id;
    std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
    Timed(aafwi_ctx* c_, int id_) : c(c_), id(id_) {
        if (c->time_every > 0 && (c->launches[id] % c->time_every) == 0 && !c->ev_pool.empty()) {
            e = c->ev_pool.back();
            c->ev_pool.pop_back();
            AAFWI_HIP(hipEventRecord(e.first, c->stream));
        }
        c->launches[id] += 1;
    }
    ~Timed() {
        if (e.first) {
            (void)hipEventRecord(e.second, c->stream);
            c->ev[id].push_back(e);
        }
    }
};

void check_m(const aafwi_ctx* c, const void* p, const char* what) {
    if (!p) throw Error{AAFWI_E_INVALID, std::string(what) + " is NULL"};
}

void model_prep(aafwi_ctx* c, const float* m) {
    const double c2 = ((double)c->dt / (double)c->h) * ((double)c->dt / (double)c->h);
    aafwi::launch_model_prep(c->stream, c->g, (float)c2, m, c->K, c->flag);
}

float* ckpt_slot(aafwi_ctx* c, int j, int which) {
    return c->ckpt + ((long long)j * 2 + which) * c->field;
}

// Forward pass over all shots; samples into d (may be dwork).
void run_forward(aafwi_ctx* c, const float* m, float* d, bool keep) {
    model_prep(c, m);
    aafwi::launch_zero(c->stream, c->F0, c->field);
    aafwi::launch_zero(c->stream, c->F1, c->field);
    float* cur = c->F0;  // u^n
    float* prev = c->F1; // u^{n-1}
    for (int n = 0; n < c->nt; ++n) {
        float* cu = nullptr;
        float* cum = nullptr;
        if (keep && n % c->k == 0) {
            cu = ckpt_slot(c, n / c->k, 0);
            cum = ckpt_slot(c, n / c->k, 1);
        }
        {
            Timed t(c, AAFWI_K_FWD_STEP);
            aafwi::launch_fwd_step(c->stream, c->gk[AAFWI_K_FWD_STEP], c->K, cur, prev, prev, c->wavelet[n], srcs(c), maps(c), d, n,
                                   c->nt, cu, cum);
        }
        std::swap(cur, prev);
    }
    c->have_ckpt = keep;
    if (keep)
        AAFWI_HIP(hipMemcpyAsync(c->mkeep, m, sizeof(float) * (size_t)c->nz * c->nx, hipMemcpyDeviceToDevice,
                                 c->stream));
}

// True when m is bitwise the model of the kept checkpoints (synchronises).
bool kept_model_is(aafwi_ctx* c, const float* m) {
    if (!c->have_ckpt) return false;
    aafwi::launch_compare(c->stream, (long long)c->nz * c->nx, m, c->mkeep, c->same);
    int v = 0;
    AAFWI_HIP(hipMemcpyAsync(&v, c->same, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    AAFWI_HIP(hipStreamSynchronize(c->stream));
    return v == 1;
}

// Checkpointed backward pass for the residual r (the model is already in K).
void run_backward(aafwi_ctx* c, const float* r, float* grad) {
    aafwi::launch_zero(c->stream, c->L0, c->field);
    aafwi::launch_zero(c->stream, c->L1, c->field);
    aafwi::launch_zero(c->stream, c->GI, c->field);
    float* lam1 = c->L0;  // lam^{n+1}
    float* lam2 = c->L1;  // lam^{n+2}
    const float h2 = c->h * c->h;
    for (int j = c->nseg - 1; j >= 0; --j) {
        const int n0 = j * c->k, n1 = std::min(n0 + c->k, c->nt);
        // recompute u^{n0} .. u^{n1-1} from the checkpoint, storing q-hat^n
        const float* cur = ckpt_slot(c, j, 0);
        const float* prev = ckpt_slot(c, j, 1);
        bool prev_is_ck = true;
        float* work[2] = {c->F0, c->F1};
        int wi = 0;
        for (int n = n0; n < n1; ++n) {
            float* out;
            if (prev_is_ck) {
                out = work[wi];
                wi ^= 1;
            } else {
                out = const_cast<float*>(prev);
            }
            {
                Timed t(c, AAFWI_K_REC_STEP);
                aafwi::launch_rec_step(c->stream, c->gk[AAFWI_K_REC_STEP], c->K, cur, prev, out, c->wavelet[n], srcs(c),
                                       c->qseg + (long long)(n - n0) * c->field);
            }
            prev_is_ck = (cur == ckpt_slot(c, j, 0) || cur == ckpt_slot(c, j, 1));
            prev = cur;
            cur = out;
        }
        // adjoint steps n1-1 .. n0 with imaging
        for (int n = n1 - 1; n >= n0; --n) {
            {
                Timed t(c, AAFWI_K_ADJ_STEP);
                aafwi::launch_adj_step(c->stream, c->gk[AAFWI_K_ADJ_STEP], c->K, lam1, lam2, lam2, maps(c), r, n, c->nt, h2,
                                       c->qseg + (long long)(n - n0) * c->field, c->GI);
            }
            std::swap(lam1, lam2);
        }
    }
    const double inv_dt2 = 1.0 / ((double)c->dt * (double)c->dt);
    aafwi::launch_fold(c->stream, c->g, (float)inv_dt2, c->GI, grad);
}

}  // namespace

extern "C" const char* aafwi_last_error(void) { return aafwi::g_last_error.c_str(); }

extern "C" int aafwi_create(const aafwi_geometry* gp, aafwi_stream stream, aafwi_ctx** out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(gp != nullptr && out != nullptr, "create: NULL argument");
        *out = nullptr;
        const aafwi_geometry& G = *gp;
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
        if (cfl > 0.55)
            throw Error{AAFWI_E_CFL, "create: vmax_bound*dt/h = " + std::to_string(cfl) + " exceeds 0.55"};
        const long long nzp = (long long)G.nz + 2LL * G.nb, nxp = (long long)G.nx + 2LL * G.nb;
        // byte offsets of a plane (plus 16 rows of slack) must stay below 2^31
        AAFWI_REQUIRE(4LL * (nzp + 16) * ((nxp + 63) / 64 * 64) < (1LL << 31), "create: padded plane too large");
        for (int s = 0; s < G.nshots; ++s) {
            AAFWI_REQUIRE(G.src_iz[s] >= 0 && G.src_iz[s] < G.nz && G.src_ix[s] >= 0 && G.src_ix[s] < G.nx,
                          "create: source index outside the interior grid");
        }
        for (long long i = 0; i < (long long)G.nshots * G.nrec; ++i) {
            AAFWI_REQUIRE(G.rec_iz[i] >= 0 && G.rec_iz[i] < G.nz && G.rec_ix[i] >= 0 && G.rec_ix[i] < G.nx,
                          "create: receiver index outside the interior grid");
        }
        for (int n = 0; n < G.nt; ++n)
            AAFWI_REQUIRE(std::isfinite(G.wavelet[n]), "create: wavelet must be finite");

        aafwi_ctx* c = new aafwi_ctx{};
        try {
            c->nz = G.nz; c->nx = G.nx; c->nb = G.nb; c->nt = G.nt;
            c->S = G.nshots; c->R = G.nrec;
            c->h = G.h; c->dt = G.dt; c->vref = G.vref; c->refl = G.refl; c->vmax = G.vmax_bound;
            c->k = G.ckpt_every > 0 ? std::min(G.ckpt_every, G.nt) : std::min(50, G.nt);
            c->nseg = (G.nt + c->k - 1) / c->k;
            c->wavelet.assign(G.wavelet, G.wavelet + G.nt);
            c->stream = (hipStream_t)stream;

            aafwi::WaveGrid& g = c->g;
            g.nz = G.nz; g.nx = G.nx; g.nb = G.nb;
            g.nzp = (int)nzp; g.nxp = (int)nxp;
            g.pitch = (int)((nxp + 63) / 64 * 64);
            g.plane = (long long)g.nzp * g.pitch;
            g.S = G.nshots;
            g.ntx = g.pitch / 64;
            g.tz = 0;
            const double smax = (G.refl >= 1.0f) ? 0.0
                                                  : 3.0 * G.vref * std::log(1.0 / (double)G.refl) / (2.0 * G.nb * G.h);
            g.scoef = (float)(smax * G.dt / 2.0);
            g.inv_nb = (float)(1.0 / G.nb);
            c->field = (long long)g.S * g.plane;
            apply_tile(g, 0);
            for (auto& gk : c->gk) gk = g;

            // receiver maps
            std::vector<int> rowmap((size_t)g.S * g.nzp, -1);
            std::vector<int> nrows(g.S, 0);
            for (int s = 0; s < g.S; ++s)
                for (int r = 0; r < G.nrec; ++r) {
                    const int zp = G.rec_iz[(long long)s * G.nrec + r] + G.nb;
                    int& slot = rowmap[(size_t)s * g.nzp + zp];
                    if (slot < 0) slot = nrows[s]++;
                }
            c->nrr = *std::max_element(nrows.begin(), nrows.end());
            std::vector<int> xmap((size_t)g.S * c->nrr * g.pitch, -1);
            std::vector<int> rnext((size_t)g.S * G.nrec, -1);
            for (int s = 0; s < g.S; ++s)
                for (int r = G.nrec - 1; r >= 0; --r) {
                    const long long i = (long long)s * G.nrec + r;
                    const int zp = G.rec_iz[i] + G.nb, xp = G.rec_ix[i] + G.nb;
                    const int slot = rowmap[(size_t)s * g.nzp + zp];
                    int& head = xmap[((size_t)s * c->nrr + slot) * g.pitch + xp];
                    rnext[i] = head;  // chain (ascending receiver order)
                    head = r;
                }
            std::vector<int2> src(g.S);
            for (int s = 0; s < g.S; ++s) src[s] = make_int2(G.src_iz[s] + G.nb, G.src_ix[s] + G.nb);

            dalloc(c, (void**)&c->K, sizeof(float) * g.plane);
            dalloc(c, (void**)&c->E, sizeof(float) * g.plane);
            dalloc(c, (void**)&c->F0, sizeof(float) * c->field);
            dalloc(c, (void**)&c->F1, sizeof(float) * c->field);
            dalloc(c, (void**)&c->L0, sizeof(float) * c->field);
            dalloc(c, (void**)&c->L1, sizeof(float) * c->field);
            dalloc(c, (void**)&c->GI, sizeof(float) * c->field);
            dalloc(c, (void**)&c->ckpt, sizeof(float) * (size_t)c->field * 2 * c->nseg);
            dalloc(c, (void**)&c->qseg, sizeof(float) * (size_t)c->field * c->k);
            dalloc(c, (void**)&c->dwork, sizeof(float) * (size_t)g.S * G.nt * G.nrec);
            dalloc(c, (void**)&c->part, sizeof(double) * aafwi::kReduceBlocks);
            dalloc(c, (void**)&c->flag, sizeof(int));
            dalloc(c, (void**)&c->mkeep, sizeof(float) * (size_t)G.nz * G.nx);
            dalloc(c, (void**)&c->same, sizeof(int));
            dalloc(c, (void**)&c->src, sizeof(int2) * g.S);
            dalloc(c, (void**)&c->rowmap, sizeof(int) * rowmap.size());
            dalloc(c, (void**)&c->xmap, sizeof(int) * xmap.size());
            dalloc(c, (void**)&c->rnext, sizeof(int) * rnext.size());
            AAFWI_HIP(hipMemcpy(c->src, src.data(), sizeof(int2) * g.S, hipMemcpyHostToDevice));
            AAFWI_HIP(hipMemcpy(c->rowmap, rowmap.data(), sizeof(int) * rowmap.size(), hipMemcpyHostToDevice));
            AAFWI_HIP(hipMemcpy(c->xmap, xmap.data(), sizeof(int) * xmap.size(), hipMemcpyHostToDevice));
            AAFWI_HIP(hipMemcpy(c->rnext, rnext.data(), sizeof(int) * rnext.size(), hipMemcpyHostToDevice));
            AAFWI_HIP(hipMemset(c->flag, 0, sizeof(int)));
            // padding columns of every field stay zero forever
            AAFWI_HIP(hipMemset(c->F0, 0, sizeof(float) * c->field));
            AAFWI_HIP(hipMemset(c->F1, 0, sizeof(float) * c->field));
            AAFWI_HIP(hipMemset(c->L0, 0, sizeof(float) * c->field));
            AAFWI_HIP(hipMemset(c->L1, 0, sizeof(float) * c->field));
            AAFWI_HIP(hipDeviceSynchronize());
        } catch (...) {
            free_ctx(c);
            throw;
        }
        *out = c;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_destroy(aafwi_ctx* c) {
    return guarded([&]() -> int {
        if (!c) return AAFWI_OK;
        (void)hipStreamSynchronize(c->stream);
        free_ctx(c);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_device_bytes(const aafwi_ctx* c, int64_t* bytes) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && bytes, "device_bytes: NULL argument");
        *bytes = c->bytes;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_sync(aafwi_ctx* c) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "sync: NULL context");
        AAFWI_HIP(hipStreamSynchronize(c->stream));
        int f = 0;
        AAFWI_HIP(hipMemcpy(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost));
        if (f) {
            AAFWI_HIP(hipMemset(c->flag, 0, sizeof(int)));
            throw Error{AAFWI_E_NONFINITE, "a model value was non-positive or non-finite"};
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_forward_model(aafwi_ctx* c, const float* m, float* d, int keep_ckpt) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c, "forward_model: NULL context");
        check_m(c, m, "forward_model: m");
        check_m(c, d, "forward_model: d");
        run_forward(c, m, d, keep_ckpt != 0);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_residual_misfit(aafwi_ctx* c, const float* d, const float* d_obs, float* r, double* J) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && d && d_obs && r && J, "residual_misfit: NULL argument");
        aafwi::launch_residual_misfit(c->stream, (long long)c->S * c->nt * c->R, d, d_obs, r, c->part, J);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_adjoint_gradient(aafwi_ctx* c, const float* m, const float* d_obs, float* grad, double* J) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && m && d_obs && grad && J, "adjoint_gradient: NULL argument");
        run_forward(c, m, c->dwork, true);
        aafwi::launch_residual_misfit(c->stream, (long long)c->S * c->nt * c->R, c->dwork, d_obs, c->dwork, c->part,
                                      J);
        run_backward(c, c->dwork, grad);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_adjoint_from_residual(aafwi_ctx* c, const float* r, float* grad) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && r && grad, "adjoint_from_residual: NULL argument");
        if (!c->have_ckpt)
            throw Error{AAFWI_E_STATE, "adjoint_from_residual: no kept checkpoints (call forward_model with keep_ckpt=1)"};
        model_prep(c, c->mkeep);  // Kp of the kept run (a Born call may have replaced it)
        run_backward(c, r, grad);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_born(aafwi_ctx* c, const float* m0, const float* dm, float* d_scat) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && m0 && dm && d_scat, "born: NULL argument");
        // the kept checkpoints are untouched; Kp is rebuilt before any backward pass
        model_prep(c, m0);
        aafwi::launch_born_prep(c->stream, c->g, m0, dm, c->E);
        aafwi::launch_zero(c->stream, c->F0, c->field);
        aafwi::launch_zero(c->stream, c->F1, c->field);
        aafwi::launch_zero(c->stream, c->L0, c->field);
        aafwi::launch_zero(c->stream, c->L1, c->field);
        float *u = c->F0, *up = c->F1, *du = c->L0, *dup = c->L1;
        for (int n = 0; n < c->nt; ++n) {
            {
                Timed t(c, AAFWI_K_BORN_STEP);
                aafwi::launch_born_step(c->stream, c->gk[AAFWI_K_BORN_STEP], c->K, c->E, u, up, up, du, dup, dup, c->wavelet[n], srcs(c),
                                        maps(c), d_scat, n, c->nt);
            }
            std::swap(u, up);
            std::swap(du, dup);
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_born_adjoint(aafwi_ctx* c, const float* m0, const float* y, float* image) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && m0 && y && image, "born_adjoint: NULL argument");
        if (kept_model_is(c, m0)) {
            model_prep(c, m0);  // background forward already checkpointed
        } else {
            run_forward(c, m0, c->dwork, true);
        }
        run_backward(c, y, image);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_kernel_timing(aafwi_ctx* c, int every) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && every >= 0, "kernel_timing: bad argument");
        AAFWI_HIP(hipStreamSynchronize(c->stream));
        for (auto& v : c->ev) {
            for (auto& e : v) c->ev_pool.push_back(e);
            v.clear();
        }
        for (auto& l : c->launches) l = 0;
        c->time_every = every;
        if (every > 0) {
            while (c->ev_pool.size() < 8192) {
                hipEvent_t a, b;
                AAFWI_HIP(hipEventCreate(&a));
                AAFWI_HIP(hipEventCreate(&b));
                c->ev_pool.emplace_back(a, b);
            }
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_kernel_timing_read(aafwi_ctx* c, int id, double* mean_ms, int64_t* count) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && mean_ms && count && id >= 0 && id < 4, "kernel_timing_read: bad argument");
        AAFWI_HIP(hipStreamSynchronize(c->stream));
        double tot = 0.0;
        for (auto& e : c->ev[id]) {
            float ms = 0.0f;
            AAFWI_HIP(hipEventElapsedTime(&ms, e.first, e.second));
            tot += ms;
        }
        *count = (int64_t)c->ev[id].size();
        *mean_ms = c->ev[id].empty() ? 0.0 : tot / (double)c->ev[id].size();
        return AAFWI_OK;
    });
}

extern "C" int aafwi_set_tile(aafwi_ctx* c, int32_t kernel_id, int32_t rows) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && rows >= 0 && rows <= 64, "set_tile: rows per wave must be in [0, 64]");
        AAFWI_REQUIRE(kernel_id >= -1 && kernel_id < 4, "set_tile: kernel_id must be -1 or a kernel id");
        for (int k = 0; k < 4; ++k)
            if (kernel_id == -1 || kernel_id == k) apply_tile(c->gk[k], rows);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_get_tile(const aafwi_ctx* c, int32_t kernel_id, int32_t* rows) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(c && rows && kernel_id >= 0 && kernel_id < 4, "get_tile: bad argument");
        *rows = c->gk[kernel_id].tz;
        return AAFWI_OK;
    });
}
