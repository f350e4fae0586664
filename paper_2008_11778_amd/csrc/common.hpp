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

// One inversion instance (one geometry, all of its shots) as the stepping
// kernels see it: a device-resident table entry read with scalar loads.
struct Inst {
    WaveGrid g;
    const float* K;        // Kp on the padded grid [plane]
    const float* E;        // Born perturbation dm/m0 [plane]
    // Wavefields [S][plane].  One-step kernels ping-pong between F[0..1]
    // (forward), L[0..1] (adjoint) and, for Born, F[0..1] (background) and
    // L[0..1] (scattered): level n+1 overwrites level n-1 in place, which
    // only the owning point reads.  Two-step kernels keep level n in
    // F[n % 4] / L[n % 4], so a launch that advances two levels never
    // overwrites a level that a neighbouring tile may still read.
    float* F[4];
    float* L[4];
    float* GI;             // image accumulators [S][plane]
    float* ckpt;           // [nseg][2][S][plane]
    float* qseg;           // [k][S][plane]
    float* d;              // sampling target [S][nt][R] (instance-owned)
    const float* r;        // adjoint source [S][nt][R] (instance-owned)
    const float* wav;      // source wavelet [nt]
    SrcNodes src;
    RecMaps rm;
    int nt, nseg, k;
    float h2;
    long long field;       // S * plane floats
};

// One wave's work: 64 columns from x0 (one-step kernels) or 56 output
// columns from x0 (two-step kernels), rows [z0, z1) of shot s of instance
// inst.  z01 packs z0 << 16 | z1.
struct TileRec {
    int inst, s, x0, z01;
};

// Per-launch step selection.  Forward and Born: n is the time step.
// Recompute and adjoint: seg counts segments from the end of each instance's
// record and n is the step inside the segment.  Two-step launches cover
// steps {n, n+1} (forward, recompute) or {n, n-1} (adjoint), clipped to each
// instance's range.  Instances derive their own
// step index, buffer parity and checkpoint slot from these, so instances with
// different record lengths share one launch.
struct StepArgs {
    int n;
    int seg;
    int keep;              // forward: copy (u^n, u^{n-1}) to the checkpoint slot
    float* d_ovr;          // if set: sampling target for every instance (single context)
    const float* r_ovr;    // if set: adjoint source for every instance (single context)
    const int* active;     // per-instance mask (NULL = all active)
    int keep_q = 0;        // forward: write q-hat of step n to plane n of qseg (full storage, one segment)
};

// Forward-kernel modes: plain forward (sampling, checkpoint copies),
// recompute of a segment from its checkpoint (q-hat out, no sampling), and
// forward keeping q-hat of every step (sampling, no checkpoint copies).
constexpr int kModeFwd = 0, kModeRec = 1, kModeFwdQ = 2;

// Launchers (wave_kernels.hip).
// mmin = 1 / vmax_bound^2: the scheme runs on max(m, mmin) (its stable domain)
void launch_model_prep(hipStream_t st, const WaveGrid& g, float c2, float mmin, const float* m, float* K,
                       int* flag, const int* active, int inst);
void launch_born_prep(hipStream_t st, const WaveGrid& g, float mmin, const float* m0, const float* dm,
                      float* E);
void launch_zero(hipStream_t st, float* p, long long n);
void launch_compare(hipStream_t st, long long n, const float* a, const float* b, int* same);
// Stepping kernels over a tile table (kernel ids as AAFWI_K_*).
void launch_step(int kernel_id, hipStream_t st, const TileRec* tiles, int ntiles, const Inst* insts,
                 const StepArgs& a);
void launch_step2(int kernel_id, hipStream_t st, const TileRec* tiles, int ntiles, const Inst* insts,
                  const StepArgs& a);
constexpr int kTile2 = 64;  // output columns of a two-step wave tile (aligned like the one-step tiles)
// Per-instance kernels; `active`/`inst` make them no-ops for masked instances.
void launch_fold(hipStream_t st, const WaveGrid& g, float inv_dt2, const float* gimg, double* ssum, const float* m,
                 float mmin, float* grad, const int* active, int inst);
void launch_residual_misfit(hipStream_t st, long long n, const float* d, const float* dobs,
                            float* r, double* partials, double* J, const int* active, int inst);
void launch_copy(hipStream_t st, long long n, const float* src, float* dst, const int* active, int inst);

// Vector kernels (aa_kernels.hip).
void launch_dot(hipStream_t st, long long n, const float* x, const float* y, const float* z,
                double* partials, double* out);
void launch_blend(hipStream_t st, long long n, float lam, const float* pt, const float* pb,
                  float* out);
void launch_axpy(hipStream_t st, long long n, float a, const float* x, float* y);
void launch_scale(hipStream_t st, long long n, float a, const float* x, float* out);
void launch_floor(hipStream_t st, long long n, float floor, float* x);

constexpr int kReduceBlocks = 1024;  // fixed partial count: deterministic reductions
constexpr int kReduceThreads = 256;

}  // namespace aafwi
