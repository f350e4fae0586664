// Internal declarations shared by the translation units of libaafwi.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "aafwi.h"

namespace aafwi {

// Internal error carrier; converted to a status code at the C boundary.
struct Error {
    int code;
    std::string msg;
};

void set_last_error(const std::string& msg);

#define AAFWI_HIP(call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::aafwi::Error{AAFWI_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define AAFWI_REQUIRE(cond, msg)                                          \
    do {                                                                  \
        if (!(cond)) throw ::aafwi::Error{AAFWI_E_INVALID, (msg)};        \
    } while (0)

// Padded-grid layout of one wavefield plane: nzp rows of `pitch` floats; the
// columns [nxp, pitch) are padding that is never read as field values.
struct WaveGrid {
    int nz, nx, nb;
    int nzp, nxp, pitch;
    long long plane;  // nzp * pitch
    int S;            // shots (independent fields stacked plane after plane)
    int ntx;          // 64-column tiles per row
    int tz;           // rows per wave (z-strip height)
    int nzs;          // strips per column of tiles
    int ntiles;       // ntx * nzs * S wave-tiles
    float scoef;      // smax * dt / 2: sponge st = scoef * (xi_x^2 + xi_z^2)
    float inv_nb;
};

// Receiver lookup used for sampling (forward) and injection (adjoint):
// rowmap[s*nzp + z] is the receiver-row slot of padded row z for shot s (or
// -1); xmap[(s*nrr + slot)*pitch + x] is the first receiver index at that
// node (or -1); next[s*R + r] chains receivers sharing a node (-1 ends).
struct RecMaps {
    const int* rowmap;
    const int* xmap;
    const int* next;
    int nrr;
    int R;
};

// Source node of each shot as a padded (row, column) pair.
struct SrcNodes {
    const int2* node;
};

// Launchers (wave_kernels.hip).
void launch_model_prep(hipStream_t st, const WaveGrid& g, float c2, const float* m, float* K,
                       int* flag);
void launch_born_prep(hipStream_t st, const WaveGrid& g, const float* m0, const float* dm,
                      float* E);
void launch_zero(hipStream_t st, float* p, long long n);
void launch_compare(hipStream_t st, long long n, const float* a, const float* b, int* same);
void launch_fwd_step(hipStream_t st, const WaveGrid& g, const float* K, const float* u,
                     const float* uprev, float* out, float w, SrcNodes src, RecMaps rm,
                     float* d, int n, int nt, float* ck_u, float* ck_um);
void launch_rec_step(hipStream_t st, const WaveGrid& g, const float* K, const float* u,
                     const float* uprev, float* out, float w, SrcNodes src, float* q);
void launch_adj_step(hipStream_t st, const WaveGrid& g, const float* K, const float* l,
                     const float* lprev, float* out, RecMaps rm, const float* r, int n, int nt,
                     float h2, const float* q, float* gimg);
void launch_born_step(hipStream_t st, const WaveGrid& g, const float* K, const float* E,
                      const float* u, const float* uprev, float* uout, const float* du,
                      const float* duprev, float* duout, float w, SrcNodes src, RecMaps rm,
                      float* d, int n, int nt);
void launch_fold(hipStream_t st, const WaveGrid& g, float inv_dt2, const float* gimg, float* grad);
void launch_residual_misfit(hipStream_t st, long long n, const float* d, const float* dobs,
                            float* r, double* partials, double* J);

// Vector kernels (aa_kernels.hip).
void launch_dot(hipStream_t st, long long n, const float* x, const float* y, const float* z,
                double* partials, double* out);
void launch_blend(hipStream_t st, long long n, float lam, const float* pt, const float* pb,
                  float* out);
void launch_axpy(hipStream_t st, long long n, float a, const float* x, float* y);
void launch_scale(hipStream_t st, long long n, float a, const float* x, float* out);

constexpr int kReduceBlocks = 1024;  // fixed partial count: deterministic reductions
constexpr int kReduceThreads = 256;

}  // namespace aafwi
