// Stepping, imaging and reduction kernels of the acoustic FD hot path (gfx950).
//
// Every stepping kernel advances all shots by one leapfrog step of the scheme
//   u^{n+1} = 2A u^n - B u^{n-1} + Kp (Lt u^n + src),
// where Lt is the unscaled 8th-order Laplacian sum (Lap = Lt / h^2),
// Kp = A (dt/h)^2 / m_pad is stored per padded cell, and the sponge factors
// A = 1/(1+st), B = 2A - 1 are rebuilt from the cell index (no array read).
// In these units a point source w/h^2 enters as +w and a receiver residual r
// of the adjoint enters as -h^2 r (section "FWI and LSRTM", eq. FWD,
// eq. FWI_adj).
//
// Work decomposition: a wave owns a 64-column x tz-row tile of one shot.
// Each lane walks its column down the strip keeping the nine u^n values of
// the z-stencil in registers; the x-neighbours come from a 72-float LDS row
// (64 centre values + 4-cell halo each side) written and read by the same
// wave, so only wave-level ordering is needed.  Four independent waves form
// a workgroup; workgroup ids are remapped so that each XCD receives a
// contiguous run of tiles (shared halos and the shared Kp rows stay in one L2).
#include "common.hpp"

namespace aafwi {
namespace {

constexpr int kWaves = 4;
constexpr float kC0 = -205.0f / 72.0f;
constexpr float kC1 = 8.0f / 5.0f;
constexpr float kC2 = -1.0f / 5.0f;
constexpr float kC3 = 8.0f / 315.0f;
constexpr float kC4 = -1.0f / 560.0f;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hardware hands workgroup i to XCD i % 8; give XCD x a contiguous range of
// logical ids instead (a bijection on [0, n)).
__device__ __forceinline__ int xcd_remap(int i, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = i & 7, k = i >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ float sponge_st(int i, int n_int, int nb, float inv_nb, float coef) {
    const int d = (i < nb) ? (nb - i) : ((i >= nb + n_int) ? (i - (nb + n_int - 1)) : 0);
    const float xi = (float)d * inv_nb;
    return coef * xi * xi;
}

struct Tile {
    int s, x0, z0, z1, lane;
    bool live;
};

__device__ __forceinline__ Tile decode_tile(const WaveGrid& g) {
    Tile t;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = __builtin_amdgcn_readfirstlane(blk * kWaves + wave);
    t.live = tile < g.ntiles;
    const int tx = tile % g.ntx;
    const int rest = tile / g.ntx;
    const int zs = rest % g.nzs;
    t.s = rest / g.nzs;
    t.x0 = tx * 64;
    t.z0 = zs * g.tz;
    t.z1 = min(t.z0 + g.tz, g.nzp);
    t.lane = lane;
    return t;
}

// Column state of one field for a wave.  At the top of the iteration for row
// z the lane holds u at rows z-4 .. z+5 (q0..q9); the load of row z+6 is
// issued during the iteration and lands in q9 two iterations later, so each
// global load has two row-iterations of latency cover.
struct Column {
    float q0, q1, q2, q3, q4, q5, q6, q7, q8, q9;
};

// Branch-free guarded load: the address is clamped to the plane origin when
// the element is outside the grid, and the value replaced by zero.
__device__ __forceinline__ float ld_sel(const float* P, int off, bool ok) {
    const float v = P[ok ? off : 0];
    return ok ? v : 0.0f;
}

// Prime the queue with rows z0-4 .. z0+5 (o0 = z0*pitch + x).
__device__ __forceinline__ void prime(Column& c, const float* U, const WaveGrid& g, int z0, int o0, bool xin) {
    const int p = g.pitch;
    c.q0 = ld_sel(U, o0 - 4 * p, xin && z0 - 4 >= 0);
    c.q1 = ld_sel(U, o0 - 3 * p, xin && z0 - 3 >= 0);
    c.q2 = ld_sel(U, o0 - 2 * p, xin && z0 - 2 >= 0);
    c.q3 = ld_sel(U, o0 - 1 * p, xin && z0 - 1 >= 0);
    c.q4 = ld_sel(U, o0, xin && z0 < g.nzp);
    c.q5 = ld_sel(U, o0 + 1 * p, xin && z0 + 1 < g.nzp);
    c.q6 = ld_sel(U, o0 + 2 * p, xin && z0 + 2 < g.nzp);
    c.q7 = ld_sel(U, o0 + 3 * p, xin && z0 + 3 < g.nzp);
    c.q8 = ld_sel(U, o0 + 4 * p, xin && z0 + 4 < g.nzp);
    c.q9 = ld_sel(U, o0 + 5 * p, xin && z0 + 5 < g.nzp);
}

// Advance one row; `incoming` is u at row z+6.
__device__ __forceinline__ void shift(Column& c, float incoming) {
    c.q0 = c.q1; c.q1 = c.q2; c.q2 = c.q3; c.q3 = c.q4; c.q4 = c.q5;
    c.q5 = c.q6; c.q6 = c.q7; c.q7 = c.q8; c.q8 = c.q9; c.q9 = incoming;
}

// Per-row stream (one value per row of the strip) with two rows of prefetch.
struct Pipe {
    float v0, v1;  // rows z, z+1
};

__device__ __forceinline__ void pipe_init(Pipe& p, const float* P, const WaveGrid& g, int z0, int z1, int o0,
                                          bool ok) {
    p.v0 = ld_sel(P, o0, ok && z0 < z1);
    p.v1 = ld_sel(P, o0 + g.pitch, ok && z0 + 1 < z1);
}

__device__ __forceinline__ void pipe_shift(Pipe& p, float incoming) {
    p.v0 = p.v1;
    p.v1 = incoming;
}

// Unscaled 8th-order Laplacian at the lane's node: z-pairs from the queue,
// x-pairs from the LDS row (centre of lane l at row[4 + l]).
__device__ __forceinline__ float lap8(const Column& c, const float* row, int lane) {
    const float* r = row + 4 + lane;
    const float s1 = (c.q3 + c.q5) + (r[-1] + r[1]);
    const float s2 = (c.q2 + c.q6) + (r[-2] + r[2]);
    const float s3 = (c.q1 + c.q7) + (r[-3] + r[3]);
    const float s4 = (c.q0 + c.q8) + (r[-4] + r[4]);
    float acc = (2.0f * kC0) * c.q4;
    acc = fmaf(kC1, s1, acc);
    acc = fmaf(kC2, s2, acc);
    acc = fmaf(kC3, s3, acc);
    acc = fmaf(kC4, s4, acc);
    return acc;
}

// Halo column of lane l < 8 (lanes 0-3 left, 4-7 right) and its LDS slot.
struct Halo {
    int hx, slot;
    bool ok;
};

__device__ __forceinline__ Halo halo_cfg(int lane, int x0, int nxp) {
    Halo h;
    h.hx = (lane < 4) ? (x0 - 4 + lane) : (x0 + 60 + lane);
    h.ok = (lane < 8) && h.hx >= 0 && h.hx < nxp;
    h.slot = (lane < 4) ? lane : (64 + lane);
    return h;
}

// Stage row z of a field into LDS: centre values from the queue, halo value
// hv (prefetched) from lanes 0-7.
__device__ __forceinline__ void stage(float* row, const Column& c, float hv, int lane, const Halo& h) {
    wave_sync();
    row[4 + lane] = c.q4;
    if (lane < 8) row[h.slot] = hv;
    wave_sync();
}

// Receiver-row slots of the strip's rows, one per lane (strips are at most
// 64 rows); read back per row with a wave-uniform lane index.
__device__ __forceinline__ int strip_rowmap(const RecMaps& rm, const WaveGrid& g, const Tile& t) {
    const bool ok = t.lane < t.z1 - t.z0;
    const int i = t.s * g.nzp + t.z0 + t.lane;
    const int v = rm.rowmap[ok ? i : t.s * g.nzp];
    return ok ? v : -1;
}

// ---------------------------------------------------------------------------
// forward step (sampling, optional checkpoint copy) and recompute step (q out)
// ---------------------------------------------------------------------------
template <bool kRecompute>
__global__ __launch_bounds__(256) void k_fwd_step(WaveGrid g, const float* __restrict__ K,
                                                  const float* __restrict__ u, const float* uprev,
                                                  float* out, float w, SrcNodes src, RecMaps rm,
                                                  float* __restrict__ d, int n, int nt,
                                                  float* __restrict__ ck_u,
                                                  float* __restrict__ ck_um,
                                                  float* __restrict__ q) {
    __shared__ float lds[kWaves][2][72];
    const Tile t = decode_tile(g);
    if (!t.live) return;
    const int lane = t.lane;
    float* rowbuf = &lds[threadIdx.x >> 6][0][0];
    const int x = t.x0 + lane;
    const bool xin = x < g.nxp;
    const long long off0 = (long long)t.s * g.plane;
    const float* U = u + off0;
    const float* UP = uprev + off0;
    float* O = out + off0;
    float* CU = ck_u ? ck_u + off0 : nullptr;
    float* CUM = ck_um ? ck_um + off0 : nullptr;
    float* Q = kRecompute ? q + off0 : nullptr;
    const Halo hc = halo_cfg(lane, t.x0, g.nxp);
    const float sx = sponge_st(x, g.nx, g.nb, g.inv_nb, g.scoef);
    const int2 sn = src.node[t.s];
    const int my_rm = kRecompute ? -1 : strip_rowmap(rm, g, t);
    const int p = g.pitch;

    Column c;
    int o = t.z0 * p + x;             // this lane's node
    int oh = t.z0 * p + hc.hx;        // this lane's halo node (lanes 0-7)
    prime(c, U, g, t.z0, o, xin);
    Pipe pv, kv, hv;
    pipe_init(pv, UP, g, t.z0, t.z1, o, xin);
    pipe_init(kv, K, g, t.z0, t.z1, o, xin);
    pipe_init(hv, U, g, t.z0, t.z1, oh, hc.ok);
    for (int z = t.z0; z < t.z1; ++z, o += p, oh += p) {
        const float nq = ld_sel(U, o + 6 * p, xin && z + 6 < g.nzp);
        const bool more = z + 2 < t.z1;
        const float npv = ld_sel(UP, o + 2 * p, xin && more);
        const float nkv = ld_sel(K, o + 2 * p, xin && more);
        const float nhv = ld_sel(U, oh + 2 * p, hc.ok && more);
        float* row = rowbuf + (z & 1) * 72;
        stage(row, c, hv.v0, lane, hc);
        float acc = lap8(c, row, lane);
        if (z == sn.x && x == sn.y) acc += w;
        const float st = sx + sponge_st(z, g.nz, g.nb, g.inv_nb, g.scoef);
        const float A = __builtin_amdgcn_rcpf(1.0f + st);
        const float B = fmaf(2.0f, A, -1.0f);
        const float qh = kv.v0 * acc;
        const float un = fmaf(2.0f * A, c.q4, fmaf(-B, pv.v0, qh));
        if (xin) {
            if (CU) {
                CU[o] = c.q4;
                CUM[o] = pv.v0;
            }
            O[o] = un;
            if (kRecompute) Q[o] = qh;
        }
        if (!kRecompute) {
            const int slot = __builtin_amdgcn_readlane(my_rm, z - t.z0);
            if (slot >= 0 && xin) {
                int ri = rm.xmap[((long long)t.s * rm.nrr + slot) * p + x];
                while (ri >= 0) {
                    d[((long long)t.s * nt + n) * rm.R + ri] = un;
                    ri = rm.next[t.s * rm.R + ri];
                }
            }
        }
        shift(c, nq);
        pipe_shift(pv, npv);
        pipe_shift(kv, nkv);
        pipe_shift(hv, nhv);
    }
}

// ---------------------------------------------------------------------------
// adjoint step with receiver injection and zero-lag imaging g += lam^n * q^n
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_step(WaveGrid g, const float* __restrict__ K,
                                                  const float* __restrict__ l, const float* lprev,
                                                  float* out, RecMaps rm,
                                                  const float* __restrict__ r, int n, int nt,
                                                  float h2, const float* __restrict__ q,
                                                  float* __restrict__ gimg) {
    __shared__ float lds[kWaves][2][72];
    const Tile t = decode_tile(g);
    if (!t.live) return;
    const int lane = t.lane;
    float* rowbuf = &lds[threadIdx.x >> 6][0][0];
    const int x = t.x0 + lane;
    const bool xin = x < g.nxp;
    const long long off0 = (long long)t.s * g.plane;
    const float* U = l + off0;
    const float* UP = lprev + off0;
    float* O = out + off0;
    const float* Q = q + off0;
    float* GI = gimg + off0;
    const Halo hc = halo_cfg(lane, t.x0, g.nxp);
    const float sx = sponge_st(x, g.nx, g.nb, g.inv_nb, g.scoef);
    const int my_rm = strip_rowmap(rm, g, t);
    const int p = g.pitch;

    Column c;
    int o = t.z0 * p + x;
    int oh = t.z0 * p + hc.hx;
    prime(c, U, g, t.z0, o, xin);
    Pipe pv, kv, hv, qv, gv;
    pipe_init(pv, UP, g, t.z0, t.z1, o, xin);
    pipe_init(kv, K, g, t.z0, t.z1, o, xin);
    pipe_init(hv, U, g, t.z0, t.z1, oh, hc.ok);
    pipe_init(qv, Q, g, t.z0, t.z1, o, xin);
    pipe_init(gv, GI, g, t.z0, t.z1, o, xin);
    for (int z = t.z0; z < t.z1; ++z, o += p, oh += p) {
        const float nq = ld_sel(U, o + 6 * p, xin && z + 6 < g.nzp);
        const bool more = xin && (z + 2 < t.z1);
        const float npv = ld_sel(UP, o + 2 * p, more);
        const float nkv = ld_sel(K, o + 2 * p, more);
        const float nhv = ld_sel(U, oh + 2 * p, hc.ok && z + 2 < t.z1);
        const float nqv = ld_sel(Q, o + 2 * p, more);
        const float ngv = ld_sel(GI, o + 2 * p, more);
        float* row = rowbuf + (z & 1) * 72;
        stage(row, c, hv.v0, lane, hc);
        float acc = lap8(c, row, lane);
        const int slot = __builtin_amdgcn_readlane(my_rm, z - t.z0);
        if (slot >= 0 && xin) {
            int ri = rm.xmap[((long long)t.s * rm.nrr + slot) * p + x];
            float rs = 0.0f;
            while (ri >= 0) {
                rs += r[((long long)t.s * nt + n) * rm.R + ri];
                ri = rm.next[t.s * rm.R + ri];
            }
            acc = fmaf(-h2, rs, acc);
        }
        const float st = sx + sponge_st(z, g.nz, g.nb, g.inv_nb, g.scoef);
        const float A = __builtin_amdgcn_rcpf(1.0f + st);
        const float B = fmaf(2.0f, A, -1.0f);
        const float ln = fmaf(2.0f * A, c.q4, fmaf(-B, pv.v0, kv.v0 * acc));
        if (xin) {
            O[o] = ln;
            GI[o] = fmaf(ln, qv.v0, gv.v0);
        }
        shift(c, nq);
        pipe_shift(pv, npv);
        pipe_shift(kv, nkv);
        pipe_shift(hv, nhv);
        pipe_shift(qv, nqv);
        pipe_shift(gv, ngv);
    }
}

// ---------------------------------------------------------------------------
// Born pair step: background u0 and scattered du with source -E * qhat0,
// E = dm_pad / m0_pad (eq. Born: -m_r d^2u0/dt^2), sampling du.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_born_step(WaveGrid g, const float* __restrict__ K,
                                                   const float* __restrict__ E,
                                                   const float* __restrict__ u,
                                                   const float* uprev, float* uout,
                                                   const float* __restrict__ du,
                                                   const float* duprev, float* duout, float w,
                                                   SrcNodes src, RecMaps rm,
                                                   float* __restrict__ d, int n, int nt) {
    __shared__ float lds[kWaves][2][2][72];
    const Tile t = decode_tile(g);
    if (!t.live) return;
    const int lane = t.lane;
    const int wv = threadIdx.x >> 6;
    const int x = t.x0 + lane;
    const bool xin = x < g.nxp;
    const long long off0 = (long long)t.s * g.plane;
    const float* U = u + off0;
    const float* UP = uprev + off0;
    float* UO = uout + off0;
    const float* D = du + off0;
    const float* DP = duprev + off0;
    float* DO = duout + off0;
    const Halo hc = halo_cfg(lane, t.x0, g.nxp);
    const float sx = sponge_st(x, g.nx, g.nb, g.inv_nb, g.scoef);
    const int2 sn = src.node[t.s];
    const int my_rm = strip_rowmap(rm, g, t);
    const int p = g.pitch;

    Column c, e;
    int o = t.z0 * p + x;
    int oh = t.z0 * p + hc.hx;
    prime(c, U, g, t.z0, o, xin);
    prime(e, D, g, t.z0, o, xin);
    Pipe pv, dpv, kv, ev, hv, dhv;
    pipe_init(pv, UP, g, t.z0, t.z1, o, xin);
    pipe_init(dpv, DP, g, t.z0, t.z1, o, xin);
    pipe_init(kv, K, g, t.z0, t.z1, o, xin);
    pipe_init(ev, E, g, t.z0, t.z1, o, xin);
    pipe_init(hv, U, g, t.z0, t.z1, oh, hc.ok);
    pipe_init(dhv, D, g, t.z0, t.z1, oh, hc.ok);
    for (int z = t.z0; z < t.z1; ++z, o += p, oh += p) {
        const bool ahead = xin && z + 6 < g.nzp;
        const float nq = ld_sel(U, o + 6 * p, ahead);
        const float ne = ld_sel(D, o + 6 * p, ahead);
        const bool more = xin && (z + 2 < t.z1);
        const bool hmore = hc.ok && (z + 2 < t.z1);
        const float npv = ld_sel(UP, o + 2 * p, more);
        const float ndpv = ld_sel(DP, o + 2 * p, more);
        const float nkv = ld_sel(K, o + 2 * p, more);
        const float nev = ld_sel(E, o + 2 * p, more);
        const float nhv = ld_sel(U, oh + 2 * p, hmore);
        const float ndhv = ld_sel(D, oh + 2 * p, hmore);
        float* row0 = &lds[wv][z & 1][0][0];
        float* row1 = &lds[wv][z & 1][1][0];
        stage(row0, c, hv.v0, lane, hc);
        stage(row1, e, dhv.v0, lane, hc);
        float acc0 = lap8(c, row0, lane);
        const float acc1 = lap8(e, row1, lane);
        if (z == sn.x && x == sn.y) acc0 += w;
        const float st = sx + sponge_st(z, g.nz, g.nb, g.inv_nb, g.scoef);
        const float A = __builtin_amdgcn_rcpf(1.0f + st);
        const float B = fmaf(2.0f, A, -1.0f);
        const float qh0 = kv.v0 * acc0;
        const float un = fmaf(2.0f * A, c.q4, fmaf(-B, pv.v0, qh0));
        const float dn = fmaf(2.0f * A, e.q4, fmaf(-B, dpv.v0, fmaf(kv.v0, acc1, -ev.v0 * qh0)));
        if (xin) {
            UO[o] = un;
            DO[o] = dn;
        }
        const int slot = __builtin_amdgcn_readlane(my_rm, z - t.z0);
        if (slot >= 0 && xin) {
            int ri = rm.xmap[((long long)t.s * rm.nrr + slot) * p + x];
            while (ri >= 0) {
                d[((long long)t.s * nt + n) * rm.R + ri] = dn;
                ri = rm.next[t.s * rm.R + ri];
            }
        }
        shift(c, nq);
        shift(e, ne);
        pipe_shift(pv, npv);
        pipe_shift(dpv, ndpv);
        pipe_shift(kv, nkv);
        pipe_shift(ev, nev);
        pipe_shift(hv, nhv);
        pipe_shift(dhv, ndhv);
    }
}

// ---------------------------------------------------------------------------
// model preparation, Born perturbation, fold, misfit
// ---------------------------------------------------------------------------
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Kp = A c2 / m_pad on every padded cell, 0 in the pitch padding; raises flag
// for a non-positive or non-finite m.
__global__ void k_model_prep(WaveGrid g, float c2, const float* __restrict__ m, float* __restrict__ K,
                             int* __restrict__ flag) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.plane) return;
    const int zp = (int)(i / g.pitch), xp = (int)(i % g.pitch);
    if (xp >= g.nxp) {
        K[i] = 0.0f;
        return;
    }
    const int iz = clampi(zp - g.nb, 0, g.nz - 1), ix = clampi(xp - g.nb, 0, g.nx - 1);
    const float mv = m[(long long)iz * g.nx + ix];
    if (!(mv > 0.0f) || !isfinite(mv)) flag[0] = 1;
    const float st = sponge_st(zp, g.nz, g.nb, g.inv_nb, g.scoef) +
                     sponge_st(xp, g.nx, g.nb, g.inv_nb, g.scoef);
    const float A = __builtin_amdgcn_rcpf(1.0f + st);
    K[i] = A * c2 / mv;
}

__global__ void k_born_prep(WaveGrid g, const float* __restrict__ m0, const float* __restrict__ dm,
                            float* __restrict__ E) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.plane) return;
    const int zp = (int)(i / g.pitch), xp = (int)(i % g.pitch);
    if (xp >= g.nxp) {
        E[i] = 0.0f;
        return;
    }
    const long long j = (long long)clampi(zp - g.nb, 0, g.nz - 1) * g.nx + clampi(xp - g.nb, 0, g.nx - 1);
    E[i] = dm[j] / m0[j];
}

__global__ void k_zero(float* __restrict__ p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0f;
}

// grad[iz][ix] = sum_s sum over the padded cells copied from (iz, ix) of
// gimg_s * (1 + st) / dt^2  (the image holds lam * A dt^2 q; 1/A = 1 + st).
__global__ void k_fold(WaveGrid g, float inv_dt2, const float* __restrict__ gimg,
                       float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nz * g.nx) return;
    const int iz = i / g.nx, ix = i % g.nx;
    const int za = (iz == 0) ? 0 : iz + g.nb;
    const int zb = (iz == g.nz - 1) ? g.nzp - 1 : iz + g.nb;
    const int xa = (ix == 0) ? 0 : ix + g.nb;
    const int xb = (ix == g.nx - 1) ? g.nxp - 1 : ix + g.nb;
    double acc = 0.0;
    for (int s = 0; s < g.S; ++s) {
        const float* G = gimg + (long long)s * g.plane;
        for (int zp = za; zp <= zb; ++zp) {
            const float sz = sponge_st(zp, g.nz, g.nb, g.inv_nb, g.scoef);
            for (int xp = xa; xp <= xb; ++xp) {
                const double ia = 1.0 + (double)sz + (double)sponge_st(xp, g.nx, g.nb, g.inv_nb, g.scoef);
                acc += (double)G[(long long)zp * g.pitch + xp] * ia;
            }
        }
    }
    grad[i] = (float)(acc * (double)inv_dt2);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(kReduceThreads) void k_residual(long long n, const float* d,
                                                             const float* __restrict__ dobs,
                                                             float* r, double* __restrict__ part) {
    __shared__ double sh[kReduceThreads];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * kReduceThreads + threadIdx.x; i < n;
         i += (long long)kReduceBlocks * kReduceThreads) {
        const float rv = d[i] - dobs[i];
        r[i] = rv;
        acc += (double)rv * (double)rv;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kReduceThreads) void k_finish_sum(const double* __restrict__ part,
                                                               double scale, double* __restrict__ out) {
    __shared__ double sh[kReduceThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < kReduceBlocks; i += kReduceThreads) acc += part[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = s * scale;
}

inline int step_blocks(const WaveGrid& g) { return (g.ntiles + kWaves - 1) / kWaves; }

}  // namespace

void launch_model_prep(hipStream_t st, const WaveGrid& g, float c2, const float* m, float* K, int* flag) {
    const int blocks = (int)((g.plane + 255) / 256);
    hipLaunchKernelGGL(k_model_prep, dim3(blocks), dim3(256), 0, st, g, c2, m, K, flag);
    AAFWI_HIP(hipGetLastError());
}

void launch_born_prep(hipStream_t st, const WaveGrid& g, const float* m0, const float* dm, float* E) {
    const int blocks = (int)((g.plane + 255) / 256);
    hipLaunchKernelGGL(k_born_prep, dim3(blocks), dim3(256), 0, st, g, m0, dm, E);
    AAFWI_HIP(hipGetLastError());
}

void launch_zero(hipStream_t st, float* p, long long n) {
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((int)blocks), dim3(256), 0, st, p, n);
    AAFWI_HIP(hipGetLastError());
}

void launch_fwd_step(hipStream_t st, const WaveGrid& g, const float* K, const float* u,
                     const float* uprev, float* out, float w, SrcNodes src, RecMaps rm, float* d,
                     int n, int nt, float* ck_u, float* ck_um) {
    hipLaunchKernelGGL(k_fwd_step<false>, dim3(step_blocks(g)), dim3(64 * kWaves), 0, st, g, K, u,
                       uprev, out, w, src, rm, d, n, nt, ck_u, ck_um, (float*)nullptr);
    AAFWI_HIP(hipGetLastError());
}

void launch_rec_step(hipStream_t st, const WaveGrid& g, const float* K, const float* u,
                     const float* uprev, float* out, float w, SrcNodes src, float* q) {
    RecMaps none{nullptr, nullptr, nullptr, 0, 0};
    hipLaunchKernelGGL(k_fwd_step<true>, dim3(step_blocks(g)), dim3(64 * kWaves), 0, st, g, K, u,
                       uprev, out, w, src, none, (float*)nullptr, 0, 0, (float*)nullptr,
                       (float*)nullptr, q);
    AAFWI_HIP(hipGetLastError());
}

void launch_adj_step(hipStream_t st, const WaveGrid& g, const float* K, const float* l,
                     const float* lprev, float* out, RecMaps rm, const float* r, int n, int nt,
                     float h2, const float* q, float* gimg) {
    hipLaunchKernelGGL(k_adj_step, dim3(step_blocks(g)), dim3(64 * kWaves), 0, st, g, K, l, lprev,
                       out, rm, r, n, nt, h2, q, gimg);
    AAFWI_HIP(hipGetLastError());
}

void launch_born_step(hipStream_t st, const WaveGrid& g, const float* K, const float* E,
                      const float* u, const float* uprev, float* uout, const float* du,
                      const float* duprev, float* duout, float w, SrcNodes src, RecMaps rm,
                      float* d, int n, int nt) {
    hipLaunchKernelGGL(k_born_step, dim3(step_blocks(g)), dim3(64 * kWaves), 0, st, g, K, E, u,
                       uprev, uout, du, duprev, duout, w, src, rm, d, n, nt);
    AAFWI_HIP(hipGetLastError());
}

void launch_fold(hipStream_t st, const WaveGrid& g, float inv_dt2, const float* gimg, float* grad) {
    const int n = g.nz * g.nx;
    hipLaunchKernelGGL(k_fold, dim3((n + 255) / 256), dim3(256), 0, st, g, inv_dt2, gimg, grad);
    AAFWI_HIP(hipGetLastError());
}

void launch_residual_misfit(hipStream_t st, long long n, const float* d, const float* dobs, float* r,
                            double* partials, double* J) {
    hipLaunchKernelGGL(k_residual, dim3(kReduceBlocks), dim3(kReduceThreads), 0, st, n, d, dobs, r,
                       partials);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kReduceThreads), 0, st, (const double*)partials, 0.5,
                       J);
    AAFWI_HIP(hipGetLastError());
}

}  // namespace aafwi
