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
constexpr int kUFwd = 4;   // rows per register block: forward / recompute
constexpr int kUAdj = 4;   // adjoint + imaging
constexpr int kUBorn = 2;  // Born pair (two fields)
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
    int inst, s, x0, z0, z1, lane;
    bool live;
};

// The wave's entry of the tile table (wave-uniform, read with scalar loads).
__device__ __forceinline__ Tile decode_tile(const TileRec* __restrict__ tiles, int ntiles) {
    Tile t;
    t.lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = __builtin_amdgcn_readfirstlane(blk * kWaves + wave);
    t.live = tile < ntiles;
    if (!t.live) return t;
    const TileRec r = tiles[tile];
    t.inst = __builtin_amdgcn_readfirstlane(r.inst);
    if (t.inst < 0) {  // padding entry of the table
        t.live = false;
        return t;
    }
    t.s = __builtin_amdgcn_readfirstlane(r.s);
    t.x0 = __builtin_amdgcn_readfirstlane(r.x0);
    const int z01 = __builtin_amdgcn_readfirstlane(r.z01);
    t.z0 = z01 >> 16;
    t.z1 = z01 & 0xffff;
    return t;
}

// Buffer views.  Every field plane of one shot is addressed through a raw
// buffer resource (base in SGPRs, 32-bit byte offset per lane).  The hardware
// range check returns 0 for loads, and drops stores, at offsets at or beyond
// the plane size; lanes outside the grid carry an offset with bit 31 set, so
// they read zeros and write nothing.  That is also the zero field outside the
// padded grid that the stencil assumes (rows above and below the plane).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr unsigned kOut = 0x80000000u;

__device__ __forceinline__ Rsrc view(const float* base, long long plane) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(plane * 4), 0x00020000);
}
// The b32 builtins move raw 32-bit patterns: reinterpret, never convert.
__device__ __forceinline__ float bld(Rsrc r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void bst(Rsrc r, unsigned off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

// Streams touched once per pass (q-hat planes, checkpoint copies) carry the
// non-temporal cache policy, so they do not push out of the caches the
// planes that the next launch reads again (u^n, lam^n, the image).
constexpr int kStream = 2;  // cache-policy operand: non-temporal
__device__ __forceinline__ float bld_s(Rsrc r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kStream));
}
__device__ __forceinline__ void bst_s(Rsrc r, unsigned off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, kStream);
}

// Register blocking along z.  A lane advances U rows per block.  At the
// start of the block for rows zb .. zb+U-1 it holds the z-queue q[0..U+8) =
// u at rows zb-4 .. zb+U+3 and the per-row streams (u^{n-1}, Kp, halo, ...)
// of those U rows; it then issues every load of the next block (U new queue
// rows and U rows of each stream) before computing the current one, so a
// wave keeps U rows of loads in flight behind U rows of arithmetic.  The U
// rows are staged to LDS together (U x 72 floats per wave) behind one
// wave-level ordering point.
template <int U>
struct Queue {
    float q[U + 8];
};

template <int U>
__device__ __forceinline__ void queue_prime(Queue<U>& c, Rsrc R, unsigned o, unsigned rb) {
#pragma unroll
    for (int i = 0; i < U + 8; ++i) c.q[i] = bld(R, o + (unsigned)(i - 4) * rb);
}

// rows zb+U+4 .. zb+2U+3 (the queue's incoming rows for the next block)
template <int U>
__device__ __forceinline__ void queue_fetch(float (&nq)[U], Rsrc R, unsigned o, unsigned rb) {
#pragma unroll
    for (int i = 0; i < U; ++i) nq[i] = bld(R, o + (unsigned)(U + 4 + i) * rb);
}

template <int U>
__device__ __forceinline__ void queue_advance(Queue<U>& c, const float (&nq)[U]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) c.q[i] = c.q[i + U];
#pragma unroll
    for (int i = 0; i < U; ++i) c.q[8 + i] = nq[i];
}

// U rows of a per-row stream starting at byte offset o.
template <int U>
__device__ __forceinline__ void rows_fetch(float (&v)[U], Rsrc R, unsigned o, unsigned rb) {
#pragma unroll
    for (int i = 0; i < U; ++i) v[i] = bld(R, o + (unsigned)i * rb);
}

template <int U>
__device__ __forceinline__ void rows_fetch_s(float (&v)[U], Rsrc R, unsigned o, unsigned rb) {
#pragma unroll
    for (int i = 0; i < U; ++i) v[i] = bld_s(R, o + (unsigned)i * rb);
}

template <int U>
__device__ __forceinline__ void rows_copy(float (&dst)[U], const float (&src)[U]) {
#pragma unroll
    for (int i = 0; i < U; ++i) dst[i] = src[i];
}

// Unscaled 8th-order Laplacian at one point: z-pairs from the register
// column q (centred on the point), x-pairs from the LDS row r (centred on
// the point's lane).
// ZS: stride of the z-column in floats.
template <int ZS>
__device__ __forceinline__ float lap8g(const float* q, const float* r) {
    const float s1 = (q[-ZS] + q[ZS]) + (r[-1] + r[1]);
    const float s2 = (q[-2 * ZS] + q[2 * ZS]) + (r[-2] + r[2]);
    const float s3 = (q[-3 * ZS] + q[3 * ZS]) + (r[-3] + r[3]);
    const float s4 = (q[-4 * ZS] + q[4 * ZS]) + (r[-4] + r[4]);
    float acc = (2.0f * kC0) * q[0];
    acc = fmaf(kC1, s1, acc);
    acc = fmaf(kC2, s2, acc);
    acc = fmaf(kC3, s3, acc);
    acc = fmaf(kC4, s4, acc);
    return acc;
}

template <int U>
__device__ __forceinline__ float lap8(const Queue<U>& c, int j, const float* row, int lane) {
    return lap8g<1>(c.q + j + 4, row + 4 + lane);
}

// Per-lane addressing of a wave tile: node offset (bytes, row z0) and halo
// offset for lanes 0-7 (lanes 0-3 left halo, 4-7 right halo), with out-of-grid
// lanes pushed out of the buffer.
struct Lanes {
    int x;
    unsigned o, oh, rb;
    int hslot;
    bool xin, interior_x;
    float sx;
};

__device__ __forceinline__ Lanes lanes(const WaveGrid& g, const Tile& t) {
    Lanes L;
    L.x = t.x0 + t.lane;
    L.xin = L.x < g.nxp;
    L.rb = (unsigned)g.pitch * 4u;
    L.o = L.xin ? (unsigned)(t.z0 * g.pitch + L.x) * 4u : kOut;
    const int hx = (t.lane < 4) ? (t.x0 - 4 + t.lane) : (t.x0 + 60 + t.lane);
    const bool hok = (t.lane < 8) && hx >= 0 && hx < g.nxp;
    L.oh = hok ? (unsigned)(t.z0 * g.pitch + hx) * 4u : kOut;
    L.hslot = (t.lane < 4) ? t.lane : (64 + t.lane);
    // the whole 64-column tile lies inside the undamped interior columns
    L.interior_x = (t.x0 >= g.nb) && (t.x0 + 64 <= g.nb + g.nx);
    L.sx = sponge_st(L.x, g.nx, g.nb, g.inv_nb, g.scoef);
    return L;
}

// Stage the U rows of a block into LDS: centre values from the queue, halo
// values (prefetched) from lanes 0-7.
template <int U>
__device__ __forceinline__ void stage(float* rows, const Queue<U>& c, const float (&hv)[U], int lane, int hslot) {
    wave_sync();
#pragma unroll
    for (int j = 0; j < U; ++j) {
        rows[j * 72 + 4 + lane] = c.q[j + 4];
        if (lane < 8) rows[j * 72 + hslot] = hv[j];
    }
    wave_sync();
}

// Sponge factors (A, B) of row z for this lane; exactly (1, 1) when the whole
// tile row is in the undamped interior (a wave-uniform branch).
template <typename LanesT>
__device__ __forceinline__ void sponge_ab(const WaveGrid& g, const LanesT& L, int z, float& A, float& B) {
    const bool interior = L.interior_x && z >= g.nb && z < g.nb + g.nz;
    if (interior) {
        A = 1.0f;
        B = 1.0f;
    } else {
        const float st = L.sx + sponge_st(z, g.nz, g.nb, g.inv_nb, g.scoef);
        A = __builtin_amdgcn_rcpf(1.0f + st);
        B = fmaf(2.0f, A, -1.0f);
    }
}

// Global-address-space views of pointers read from the instance table.  The
// compiler cannot infer where such pointers point, and generic (FLAT)
// accesses would make every later wait in a stepping loop drain all
// outstanding loads and stores instead of only the ones it needs.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gc(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gm(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Sum of the residuals injected at this lane's node of row slot `slot`.
__device__ __forceinline__ float injected(const RecMaps& rm, const WaveGrid& g, int s, int slot, int x,
                                          const float* r, int nt, int n) {
    float rs = 0.0f;
    int ri = gc(rm.xmap)[((long long)s * rm.nrr + slot) * g.pitch + x];
    while (ri >= 0) {
        rs += gc(r)[((long long)s * nt + n) * rm.R + ri];
        ri = gc(rm.next)[s * rm.R + ri];
    }
    return rs;
}

// Store v as the trace sample of every receiver at this lane's node of row
// slot `slot`.
__device__ __forceinline__ void sample(const RecMaps& rm, const WaveGrid& g, int s, int slot, int x, float* d,
                                       int nt, int n, float v) {
    int ri = gc(rm.xmap)[((long long)s * rm.nrr + slot) * g.pitch + x];
    while (ri >= 0) {
        gm(d)[((long long)s * nt + n) * rm.R + ri] = v;
        ri = gc(rm.next)[s * rm.R + ri];
    }
}

// Receiver-row slots of the strip's rows, one per lane (strips are at most
// 64 rows); read back per row with a wave-uniform lane index.
__device__ __forceinline__ int strip_rowmap(const RecMaps& rm, const WaveGrid& g, const Tile& t) {
    const bool ok = t.lane < t.z1 - t.z0;
    const int i = t.s * g.nzp + t.z0 + t.lane;
    const int v = gc(rm.rowmap)[ok ? i : t.s * g.nzp];
    return ok ? v : -1;
}

// ---------------------------------------------------------------------------
// forward step (sampling, optional checkpoint copy), recompute step (q out),
// and forward step that samples and keeps q-hat of every step (full storage)
// ---------------------------------------------------------------------------
template <int U, int kMode>
__global__ __launch_bounds__(256) void k_fwd_step(const TileRec* __restrict__ tiles, int ntiles,
                                                  const Inst* __restrict__ insts, StepArgs a) {
    __shared__ float lds[kWaves][U * 72];
    const Tile t = decode_tile(tiles, ntiles);
    if (!t.live) return;
    if (a.active && !a.active[t.inst]) return;
    constexpr bool kRecompute = kMode == kModeRec, kKeepQ = kMode != kModeFwd, kSample = kMode != kModeRec;
    const Inst& I = insts[t.inst];
    const WaveGrid g = I.g;
    // step index, buffers and checkpoint slot of this instance
    int n;
    const float* u;
    const float* uprev;
    float* out;
    float* ck_u = nullptr;
    float* q = nullptr;
    if (!kRecompute) {
        n = a.n;
        if (n >= I.nt) return;
        u = I.F[n & 1];  // u^n
        out = I.F[(n + 1) & 1];  // u^{n-1}, overwritten by u^{n+1}
        uprev = out;
        if (kMode == kModeFwd && a.keep && n % I.k == 0) ck_u = I.ckpt + (long long)(n / I.k) * 2 * I.field;
        if (kKeepQ) q = I.qseg + (long long)n * I.field;  // one segment: its step index is n
    } else {
        const int j = I.nseg - 1 - a.seg;  // segment being recomputed
        const int tt = a.n;
        n = j * I.k + tt;
        if (j < 0 || n >= I.nt) return;
        const float* c0 = I.ckpt + (long long)j * 2 * I.field;  // u^{jk}, u^{jk-1}
        if (tt == 0) {
            u = c0;
            uprev = c0 + I.field;
            out = I.F[0];
        } else if (tt == 1) {
            u = I.F[0];
            uprev = c0;
            out = I.F[1];
        } else {
            u = I.F[(tt + 1) & 1];
            out = I.F[tt & 1];
            uprev = out;
        }
        q = I.qseg + (long long)tt * I.field;
    }
    const float w = I.wav[n];
    const int nt = I.nt;
    const RecMaps rm = I.rm;
    float* d = a.d_ovr ? a.d_ovr : I.d;
    const int lane = t.lane;
    float* rows = &lds[threadIdx.x >> 6][0];
    const long long off0 = (long long)t.s * g.plane;
    const Rsrc UR = view(u + off0, g.plane);
    const Rsrc UP = view(uprev + off0, g.plane);
    const Rsrc O = view(out + off0, g.plane);
    const Rsrc KR = view(I.K, g.plane);
    const bool ck = ck_u != nullptr;
    const Rsrc CU = view(ck ? ck_u + off0 : u, g.plane);
    const Rsrc CUM = view(ck ? ck_u + I.field + off0 : u, g.plane);
    const Rsrc QR = view(kKeepQ ? q + off0 : u, g.plane);
    const Lanes L = lanes(g, t);
    const int2 sn = I.src.node[t.s];
    const int my_rm = kSample ? strip_rowmap(rm, g, t) : -1;
    const unsigned rb = L.rb;

    unsigned o = L.o, oh = L.oh;
    Queue<U> c;
    queue_prime(c, UR, o, rb);
    float pv[U], kv[U], hv[U];
    rows_fetch(pv, UP, o, rb);
    rows_fetch(kv, KR, o, rb);
    rows_fetch(hv, UR, oh, rb);
    for (int zb = t.z0; zb < t.z1; zb += U, o += U * rb, oh += U * rb) {
        float nq[U], npv[U], nkv[U], nhv[U];
        queue_fetch(nq, UR, o, rb);
        rows_fetch(npv, UP, o + U * rb, rb);
        rows_fetch(nkv, KR, o + U * rb, rb);
        rows_fetch(nhv, UR, oh + U * rb, rb);
        stage(rows, c, hv, lane, L.hslot);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int z = zb + j;
            if (z >= t.z1) break;
            const unsigned oz = o + (unsigned)j * rb;
            float acc = lap8(c, j, rows + j * 72, lane);
            if (z == sn.x && L.x == sn.y) acc += w;
            float A, B;
            sponge_ab(g, L, z, A, B);
            const float qh = kv[j] * acc;
            const float un = fmaf(2.0f * A, c.q[j + 4], fmaf(-B, pv[j], qh));
            if (ck) {
                bst_s(CU, oz, c.q[j + 4]);
                bst_s(CUM, oz, pv[j]);
            }
            bst(O, oz, un);
            if (kKeepQ) bst_s(QR, oz, qh);
            if (kSample) {
                const int slot = __builtin_amdgcn_readlane(my_rm, z - t.z0);
                if (slot >= 0 && L.xin) sample(rm, g, t.s, slot, L.x, d, nt, n, un);
            }
        }
        queue_advance(c, nq);
        rows_copy(pv, npv);
        rows_copy(kv, nkv);
        rows_copy(hv, nhv);
    }
}

// ---------------------------------------------------------------------------
// adjoint step with receiver injection and zero-lag imaging g += lam^n * q^n
// ---------------------------------------------------------------------------
template <int U>
__global__ __launch_bounds__(256) void k_adj_step(const TileRec* __restrict__ tiles, int ntiles,
                                                  const Inst* __restrict__ insts, StepArgs a) {
    __shared__ float lds[kWaves][U * 72];
    const Tile t = decode_tile(tiles, ntiles);
    if (!t.live) return;
    if (a.active && !a.active[t.inst]) return;
    const Inst& I = insts[t.inst];
    const WaveGrid g = I.g;
    const int j = I.nseg - 1 - a.seg;
    const int tt = a.n;
    const int n = j * I.k + tt;
    if (j < 0 || n >= I.nt) return;
    // lam^{n+1} sits in L[(nt-1-n) & 1]; lam^n overwrites lam^{n+2} in the other
    const int par = (I.nt - 1 - n) & 1;
    const float* l = I.L[par];
    float* out = I.L[par ^ 1];
    const float* lprev = out;
    const float* r = a.r_ovr ? a.r_ovr : I.r;
    const float* q = I.qseg + (long long)tt * I.field;
    const int nt = I.nt;
    const RecMaps rm = I.rm;
    const float h2 = I.h2;
    const int lane = t.lane;
    float* rows = &lds[threadIdx.x >> 6][0];
    const long long off0 = (long long)t.s * g.plane;
    const Rsrc UR = view(l + off0, g.plane);
    const Rsrc UP = view(lprev + off0, g.plane);
    const Rsrc O = view(out + off0, g.plane);
    const Rsrc KR = view(I.K, g.plane);
    const Rsrc QR = view(q + off0, g.plane);
    const Rsrc GI = view(I.GI + off0, g.plane);
    const Lanes L = lanes(g, t);
    const int my_rm = strip_rowmap(rm, g, t);
    const unsigned rb = L.rb;

    unsigned o = L.o, oh = L.oh;
    Queue<U> c;
    queue_prime(c, UR, o, rb);
    float pv[U], kv[U], hv[U], qv[U], gv[U];
    rows_fetch(pv, UP, o, rb);
    rows_fetch(kv, KR, o, rb);
    rows_fetch(hv, UR, oh, rb);
    rows_fetch_s(qv, QR, o, rb);
    rows_fetch(gv, GI, o, rb);
    for (int zb = t.z0; zb < t.z1; zb += U, o += U * rb, oh += U * rb) {
        float nq[U], npv[U], nkv[U], nhv[U], nqv[U], ngv[U];
        queue_fetch(nq, UR, o, rb);
        rows_fetch(npv, UP, o + U * rb, rb);
        rows_fetch(nkv, KR, o + U * rb, rb);
        rows_fetch(nhv, UR, oh + U * rb, rb);
        rows_fetch_s(nqv, QR, o + U * rb, rb);
        rows_fetch(ngv, GI, o + U * rb, rb);
        stage(rows, c, hv, lane, L.hslot);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int z = zb + j;
            if (z >= t.z1) break;
            const unsigned oz = o + (unsigned)j * rb;
            float acc = lap8(c, j, rows + j * 72, lane);
            const int slot = __builtin_amdgcn_readlane(my_rm, z - t.z0);
            if (slot >= 0 && L.xin) acc = fmaf(-h2, injected(rm, g, t.s, slot, L.x, r, nt, n), acc);
            float A, B;
            sponge_ab(g, L, z, A, B);
            const float ln = fmaf(2.0f * A, c.q[j + 4], fmaf(-B, pv[j], kv[j] * acc));
            bst(O, oz, ln);
            bst(GI, oz, fmaf(ln, qv[j], gv[j]));
        }
        queue_advance(c, nq);
        rows_copy(pv, npv);
        rows_copy(kv, nkv);
        rows_copy(hv, nhv);
        rows_copy(qv, nqv);
        rows_copy(gv, ngv);
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch (forward, recompute, adjoint).
//
// A wave owns the 64 columns [x0, x0+64) (x0 a multiple of 64, so every row
// it streams is two whole cache lines) and rows [z0, z1); lane l is column
// x0 + l.  Step two (level n+1 -> n+2) of those points needs step one
// (n -> n+1) on the 4-cell frame around them: rows z0-4 .. z1+3 and columns
// x0-4 .. x0+67.  The 64 lanes evaluate step one on their own columns for
// rows z0-4 .. z1+3; the eight frame columns are evaluated in one extra pass
// per 4-row block, packed as (row, frame column) over lanes 0-31, from side
// loads of those columns (lanes 32-63 fetch the four columns beyond each
// side that the frame's stencil reaches).  Step two trails step one by one
// register block and reads the step-one values from registers (z) and from
// an LDS row (x).  Out-of-grid rows and columns come out zero by themselves:
// their loads, Kp included, read zero through the buffer range check.  Each
// time level is read and written once per launch instead of once per step;
// the price is the frame (tz+8 of tz rows, 8 side columns per 64).  Every
// point is evaluated with the one-step arithmetic in the same order, so both
// paths give bitwise identical fields, traces and images.
// ---------------------------------------------------------------------------
struct Lanes2 {
    int xc;            // main column x0 + lane
    bool xin;          // inside the padded grid
    unsigned base;     // byte offset of (row 0, xc), or out of the buffer
    int sr;            // side lanes: row of the 4-row block, (lane & 31) >> 3
    int fc;            // frame column of lane & 31
    bool fin;          // that frame column lies inside the grid
    unsigned sbase;    // byte offset of (row sr, side column), or out: frame column
                       // for lanes 0-31, outer column for lanes 32-63
    unsigned fbase;    // lanes 0-31: as sbase (u^{n-1} and Kp of the frame); 32-63: out
    int apos;          // side value's place in the 80-column step-one row (x0-8 at 0)
    int fpos;          // place of the frame column of lane & 31 in that row
    int bpos;          // place of the frame column of lane & 31 in the 72-column step-two row (x0-4 at 0)
    bool interior_x;   // the 64 main columns are all undamped
    bool interior_f;   // columns x0-4 .. x0+67 are all undamped
    float sx;          // sponge term of the main column
    float fsx;         // sponge term of the frame column of lane & 31
};

__device__ __forceinline__ Lanes2 lanes2(const WaveGrid& g, const Tile& t) {
    Lanes2 L;
    const int lane = t.lane, k = lane & 7;
    L.xc = t.x0 + lane;
    L.xin = L.xc < g.nxp;
    L.base = L.xin ? (unsigned)L.xc * 4u : kOut;
    L.sr = (lane & 31) >> 3;
    L.fc = k < 4 ? t.x0 - 4 + k : t.x0 + 60 + k;
    L.fin = L.fc >= 0 && L.fc < g.nxp;
    const int oc = k < 4 ? t.x0 - 8 + k : t.x0 + 64 + k;
    const int sc = lane < 32 ? L.fc : oc;
    const bool sin = sc >= 0 && sc < g.nxp;
    L.sbase = sin ? (unsigned)(L.sr * g.pitch + sc) * 4u : kOut;
    L.fbase = lane < 32 ? L.sbase : kOut;
    L.apos = sc - (t.x0 - 8);
    L.fpos = L.fc - (t.x0 - 8);
    L.bpos = L.fc - (t.x0 - 4);
    L.interior_x = (t.x0 >= g.nb) && (t.x0 + 64 <= g.nb + g.nx);
    L.interior_f = (t.x0 - 4 >= g.nb) && (t.x0 + 68 <= g.nb + g.nx);
    L.sx = sponge_st(L.xc, g.nx, g.nb, g.inv_nb, g.scoef);
    L.fsx = sponge_st(L.fc, g.nx, g.nb, g.inv_nb, g.scoef);
    return L;
}

// Byte offset of row z (may be negative: the unsigned sum then lies beyond
// the plane and reads as zero).
__device__ __forceinline__ unsigned row_off(int z, int pitch) { return (unsigned)(z * pitch * 4); }

// Receiver-row slots of the rows z0-4 .. z0+123 a two-step tile touches
// (strips of up to 120 rows), held one per lane in two registers (loaded
// once per tile) and read back with a wave-uniform lane index (readlane) or,
// for the packed frame rows, a per-lane one (bpermute): no memory access
// inside the row loop, whose prefetched loads would otherwise all be waited
// for.
struct FrameRows {
    int lo, hi;
};

__device__ __forceinline__ FrameRows frame_rowmap(const RecMaps& rm, const WaveGrid& g, const Tile& t) {
    FrameRows f;
    const int za = t.z0 - 4 + t.lane, zb = t.z0 + 60 + t.lane, zmax = min(t.z1 + 4, g.nzp);
    f.lo = (za >= 0 && za < zmax) ? gc(rm.rowmap)[t.s * g.nzp + za] : -1;
    f.hi = (zb < zmax) ? gc(rm.rowmap)[t.s * g.nzp + zb] : -1;
    return f;
}

__device__ __forceinline__ int frame_slot(const FrameRows& f, int z, int z0) {
    const int i = z - (z0 - 4);
    return i < 64 ? __builtin_amdgcn_readlane(f.lo, i) : __builtin_amdgcn_readlane(f.hi, i - 64);
}

// Per-lane row z (all lanes take part).
__device__ __forceinline__ int frame_slot_lane(const FrameRows& f, int z, int z0) {
    const int i = z - (z0 - 4);
    const int a = (i & 63) * 4;
    const int lo = __builtin_amdgcn_ds_bpermute(a, f.lo), hi = __builtin_amdgcn_ds_bpermute(a, f.hi);
    return (i >= 0 && i < 64) ? lo : (i >= 64 && i < 128) ? hi : -1;
}

// Register rings of the two-step kernels.  The loop over 4-row blocks is
// unrolled four times and every row block of every stream has a fixed ring
// slot: block k sits in slot k & 3 of a 4-deep ring and k & 1 of a 2-deep
// one.  The loads of block k+1 go to slots that block k does not touch and
// nothing moves between slots, so each block waits for its own rows right
// before using them, with the next block's loads still in flight.  (A queue
// shifted at the end of every block copies the rows just loaded, which waits
// for all of them there and leaves the wave with nothing in flight.)
template <int K>
struct Blk {
    static constexpr int prev = (K + 3) & 3, cur = K & 3, next = (K + 1) & 3, ahead = (K + 2) & 3;
    static constexpr int even = K & 1, odd = (K + 1) & 1;
};

// The 12-row z-window (rows za-4 .. za+7) from three ring slots.
__device__ __forceinline__ void window(float (&w)[12], const float (&a)[4], const float (&b)[4],
                                       const float (&c)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        w[i] = a[i];
        w[4 + i] = b[i];
        w[8 + i] = c[i];
    }
}

// LDS of a two-step wave: the step-one rows (4 x 80: columns x0-8 .. x0+71),
// the frame columns' z-window (12 rows x 8), the step-two rows (4 x 72:
// columns x0-4 .. x0+67).
constexpr int kRowA = 80, kRowB = 72, kLds2 = 4 * kRowA + 12 * 8 + 4 * kRowB;

// Stage the block's u^n (or lam^{n+1}) rows: main lanes' rows into the
// step-one rows, the side values (row sr of the block) beside them, and the
// frame columns' rows za-4 .. za+7 into the z-window.
__device__ __forceinline__ void stage_one(float* A, float* F, const float (&q)[12], float hp, float hc, float hn,
                                          int lane, const Lanes2& L) {
    wave_sync();
#pragma unroll
    for (int j = 0; j < 4; ++j) A[j * kRowA + 8 + lane] = q[j + 4];
    A[L.sr * kRowA + L.apos] = hc;
    if (lane < 32) {
        const int f = lane & 7;
        F[L.sr * 8 + f] = hp;
        F[(4 + L.sr) * 8 + f] = hc;
        F[(8 + L.sr) * 8 + f] = hn;
    }
    wave_sync();
}

// Stage the step-one rows that step two reads: main lanes' values and the
// frame values of lanes 0-31.
__device__ __forceinline__ void stage_two(float* Bv, const float (&v)[12], float bf, int lane, const Lanes2& L) {
    wave_sync();
#pragma unroll
    for (int j = 0; j < 4; ++j) Bv[j * kRowB + 4 + lane] = v[j + 4];
    if (lane < 32) Bv[L.sr * kRowB + L.bpos] = bf;
    wave_sync();
}

template <int V>
struct IC {
    static constexpr int value = V;
};

// Store with the row offset in the scalar offset operand; only for rows
// known to lie inside the plane (lanes pushed out of it keep their bit-31
// offset in voffset and still drop the store).
__device__ __forceinline__ void bst_row(Rsrc r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bst_row_s(Rsrc r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, kStream);
}

// Frame rows z0-4+i (i < 128) flagged in a two-word lane mask: whether rows
// i0 .. i0+7 are all unflagged.
__device__ __forceinline__ bool rows_clear(unsigned long long lo, unsigned long long hi, int i0) {
    unsigned long long w;
    if (i0 >= 64)
        w = hi >> (i0 - 64);
    else if (i0 == 0)
        w = lo;
    else
        w = (lo >> i0) | (hi << (64 - i0));
    return (w & 0xffull) == 0;
}

// Blocks whose eight rows (step one at za .. za+3, step two at za-4 .. za-1)
// lie inside the strip and the undamped interior, with no receiver or
// source row among them, take a branch-free path: A = B = 1 exactly, no
// per-row tests, the same arithmetic in the same order.
struct FastRows {
    int zlo, zhi;                // za-4 >= zlo and za+3 < zhi
    unsigned long long lo, hi;   // flagged frame rows
    bool on;                     // the tile qualifies at all
};

__device__ __forceinline__ FastRows fast_rows(const WaveGrid& g, const Tile& t, const Lanes2& L, const FrameRows& fr,
                                              int src_row, bool on) {
    FastRows f;
    f.zlo = max(t.z0, g.nb);
    f.zhi = min(t.z1, g.nb + g.nz);
    const int za = t.z0 - 4 + t.lane, zb = t.z0 + 60 + t.lane;
    f.lo = __builtin_amdgcn_ballot_w64(fr.lo >= 0 || za == src_row);
    f.hi = __builtin_amdgcn_ballot_w64(fr.hi >= 0 || zb == src_row);
    f.on = on && L.interior_f;
    return f;
}

__device__ __forceinline__ bool is_fast(const FastRows& f, int za, int z0) {
    return f.on && za - 4 >= f.zlo && za + 3 < f.zhi && rows_clear(f.lo, f.hi, za - z0);
}

// Sponge factors of a point off the main lanes (no interior shortcut: with
// both sponge terms zero the reciprocal is exactly 1, as on the shortcut).
__device__ __forceinline__ void sponge_pt(const WaveGrid& g, float sx, int z, float& A, float& B) {
    const float st = sx + sponge_st(z, g.nz, g.nb, g.inv_nb, g.scoef);
    A = __builtin_amdgcn_rcpf(1.0f + st);
    B = fmaf(2.0f, A, -1.0f);
}

template <int U, int kMode>
__global__ __launch_bounds__(256) void k_fwd_step2(const TileRec* __restrict__ tiles, int ntiles,
                                                   const Inst* __restrict__ insts, StepArgs a) {
    static_assert(U == 4, "the two-step register rings hold 4-row blocks");
    __shared__ float lds[kWaves][kLds2];
    const Tile t = decode_tile(tiles, ntiles);
    if (!t.live) return;
    if (a.active && !a.active[t.inst]) return;
    constexpr bool kRecompute = kMode == kModeRec, kKeepQ = kMode != kModeFwd, kSample = kMode != kModeRec;
    const Inst& I = insts[t.inst];
    const WaveGrid g = I.g;
    int n, tt = 0, cnt;
    const float* u;
    const float* uprev;
    if (!kRecompute) {
        n = a.n;
        if (n >= I.nt) return;
        cnt = min(2, I.nt - n);
        u = I.F[n & 3];
        uprev = I.F[(n + 3) & 3];
    } else {
        const int j = I.nseg - 1 - a.seg;
        tt = a.n;
        if (j < 0) return;
        const int len = min(I.k, I.nt - j * I.k);
        if (tt >= len) return;
        cnt = min(2, len - tt);
        n = j * I.k + tt;
        const float* c0 = I.ckpt + (long long)j * 2 * I.field;  // u^{jk}, u^{jk-1}
        u = tt == 0 ? c0 : I.F[n & 3];
        uprev = tt == 0 ? c0 + I.field : I.F[(n + 3) & 3];
    }
    const bool two = cnt == 2;
    float* out1 = I.F[(n + 1) & 3];
    float* out2 = I.F[(n + 2) & 3];
    // checkpoint slots reached by this launch: (u^n, u^{n-1}) and (u^{n+1}, u^n)
    float* ck0 = nullptr;
    float* ck1 = nullptr;
    if (kMode == kModeFwd && a.keep) {
        if (n % I.k == 0) ck0 = I.ckpt + (long long)(n / I.k) * 2 * I.field;
        if (two && (n + 1) % I.k == 0) ck1 = I.ckpt + (long long)((n + 1) / I.k) * 2 * I.field;
    }
    const float w0 = I.wav[n];
    const float w1 = two ? I.wav[n + 1] : 0.0f;
    const int nt = I.nt;
    const RecMaps rm = I.rm;
    float* d = a.d_ovr ? a.d_ovr : I.d;
    const int lane = t.lane;
    float* A_ = &lds[threadIdx.x >> 6][0];
    float* F_ = A_ + 4 * kRowA;
    float* B_ = F_ + 12 * 8;
    const long long off0 = (long long)t.s * g.plane;
    const Rsrc UR = view(u + off0, g.plane);
    const Rsrc UP = view(uprev + off0, g.plane);
    const Rsrc O1 = view(out1 + off0, g.plane);
    const Rsrc O2 = view(out2 + off0, g.plane);
    const Rsrc KR = view(I.K, g.plane);
    const Rsrc C0U = view(ck0 ? ck0 + off0 : u, g.plane);
    const Rsrc C0P = view(ck0 ? ck0 + I.field + off0 : u, g.plane);
    const Rsrc C1U = view(ck1 ? ck1 + off0 : u, g.plane);
    const Rsrc C1P = view(ck1 ? ck1 + I.field + off0 : u, g.plane);
    // q-hat planes: the segment's step tt (recompute) or step n (full storage, one segment)
    float* q0 = kKeepQ ? I.qseg + (long long)(kRecompute ? tt : n) * I.field + off0 : out1;
    const Rsrc Q0 = view(q0, g.plane);
    const Rsrc Q1 = view(kKeepQ && two ? q0 + I.field : out1, g.plane);
    const Lanes2 L = lanes2(g, t);
    const int2 sn = I.src.node[t.s];
    const unsigned rb = (unsigned)g.pitch * 4u;
    const unsigned own_mask = L.xin ? 0u : kOut;  // OR-ed into store offsets
    FrameRows fr{-1, -1};
    if (kSample) fr = frame_rowmap(rm, g, t);
    const FastRows fast = fast_rows(g, t, L, fr, sn.x, two && !ck0 && !ck1);

    const int za0 = t.z0 - 4;
    const int zend = two ? t.z1 + 4 : t.z1;
    int za = za0;
    unsigned o = L.base + row_off(za0, g.pitch);
    unsigned os = L.sbase + row_off(za0, g.pitch);
    unsigned of = L.fbase + row_off(za0, g.pitch);
    float c[4][4];   // u^n: blocks k-1, k, k+1 in use, k+2 arriving
    float b[4][4];   // u^{n+1} of step one: blocks k-2, k-1, k
    float kp[4][4];  // Kp: block k-1 (step two), k (step one), k+1 arriving
    float p[2][4];   // u^{n-1}: block k, k+1 arriving
    float hs[4];     // side lanes: u^n at row sr of blocks k-1, k, k+1 in use, k+2 arriving
    float ph[2], kh[2];  // lanes 0-31: u^{n-1}, Kp at the frame column, row sr of block k, k+1 arriving
    float bh[2];     // lanes 0-31: step one at the frame column, row sr of block k, and of block k-1
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        c[3][i] = bld(UR, o + (unsigned)(i - 4) * rb);
        c[0][i] = bld(UR, o + (unsigned)i * rb);
        c[1][i] = bld(UR, o + (unsigned)(4 + i) * rb);
        kp[3][i] = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r][i] = 0.0f;
    }
    hs[3] = bld(UR, os - 4u * rb);
    hs[0] = bld(UR, os);
    hs[1] = bld(UR, os + 4u * rb);
    rows_fetch(p[0], UP, o, rb);
    rows_fetch(kp[0], KR, o, rb);
    ph[0] = bld(UP, of);
    kh[0] = bld(KR, of);
    bh[0] = bh[1] = 0.0f;

    auto block = [&](auto KC) __attribute__((always_inline)) {
        using S = Blk<decltype(KC)::value>;
        // the next block's rows
#pragma unroll
        for (int i = 0; i < 4; ++i) c[S::ahead][i] = bld(UR, o + (unsigned)(8 + i) * rb);
        rows_fetch(p[S::odd], UP, o + 4 * rb, rb);
        rows_fetch(kp[S::next], KR, o + 4 * rb, rb);
        hs[S::ahead] = bld(UR, os + 8u * rb);
        ph[S::odd] = bld(UP, of + 4u * rb);
        kh[S::odd] = bld(KR, of + 4u * rb);
        float q[12];
        window(q, c[S::prev], c[S::cur], c[S::next]);
        stage_one(A_, F_, q, hs[S::prev], hs[S::cur], hs[S::next], lane, L);
        const float* fz = F_ + (4 + L.sr) * 8 + (lane & 7);  // frame z-column, centred
        const float* fx = A_ + L.sr * kRowA + L.fpos;        // frame x-row, centred
        if (is_fast(fast, za, t.z0)) {
            // with A = B = 1 the leapfrog update would otherwise fuse Kp*acc
            // into the subtraction and skip the rounding of q-hat
#pragma clang fp contract(off)
            const unsigned ow = o | own_mask;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float acc = lap8g<1>(q + j + 4, A_ + j * kRowA + 8 + lane);
                const float qh = kp[S::cur][j] * acc;
                const float un = fmaf(2.0f, q[j + 4], fmaf(-1.0f, p[S::even][j], qh));
                b[S::cur][j] = un;
                bst_row(O1, ow, (unsigned)j * rb, un);
                if (kKeepQ) bst_row_s(Q0, ow, (unsigned)j * rb, qh);
            }
            {
                const float acc = lap8g<8>(fz, fx);
                const float qh = kh[S::even] * acc;
                bh[S::even] = fmaf(2.0f, fz[0], fmaf(-1.0f, ph[S::even], qh));
            }
            float v[12];
            window(v, b[S::ahead], b[S::prev], b[S::cur]);
            stage_two(B_, v, bh[S::odd], lane, L);
            const unsigned ow2 = ow - 4u * rb;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float acc = lap8g<1>(v + j + 4, B_ + j * kRowB + 4 + lane);
                const float qh = kp[S::prev][j] * acc;
                const float un = fmaf(2.0f, v[j + 4], fmaf(-1.0f, q[j], qh));
                bst_row(O2, ow2, (unsigned)j * rb, un);
                if (kKeepQ) bst_row_s(Q1, ow2, (unsigned)j * rb, qh);
            }
            za += 4;
            o += 4 * rb;
            os += 4 * rb;
            of += 4 * rb;
            return;
        }
        // step one at rows za .. za+3, main lanes
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int z = za + j;
            float acc = lap8g<1>(q + j + 4, A_ + j * kRowA + 8 + lane);
            if (z == sn.x && L.xc == sn.y) acc += w0;
            float A, B;
            sponge_ab(g, L, z, A, B);
            const float qh = kp[S::cur][j] * acc;
            const float un = fmaf(2.0f * A, q[j + 4], fmaf(-B, p[S::even][j], qh));
            b[S::cur][j] = un;
            if (z >= t.z0 && z < t.z1) {
                const unsigned oz = (o + (unsigned)j * rb) | own_mask;
                if (ck0) {
                    bst_s(C0U, oz, q[j + 4]);
                    bst_s(C0P, oz, p[S::even][j]);
                }
                if (ck1) {
                    bst_s(C1U, oz, un);
                    bst_s(C1P, oz, q[j + 4]);
                }
                bst(O1, oz, un);
                if (kKeepQ) bst_s(Q0, oz, qh);
                if (kSample) {
                    const int slot = frame_slot(fr, z, t.z0);
                    if (slot >= 0 && L.xin) sample(rm, g, t.s, slot, L.xc, d, nt, n, un);
                }
            }
        }
        // step one at the frame columns, row za + sr (lanes 0-31; 32-63 repeat them)
        {
            const int z = za + L.sr;
            float acc = lap8g<8>(fz, fx);
            if (z == sn.x && L.fc == sn.y) acc += w0;
            float A, B;
            sponge_pt(g, L.fsx, z, A, B);
            const float qh = kh[S::even] * acc;
            bh[S::even] = fmaf(2.0f * A, fz[0], fmaf(-B, ph[S::even], qh));
        }
        // step two at rows za-4 .. za-1
        if (two && za - 4 >= t.z0) {
            float v[12];
            window(v, b[S::ahead], b[S::prev], b[S::cur]);
            stage_two(B_, v, bh[S::odd], lane, L);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int z = za - 4 + j;
                if (z >= t.z1) break;
                float acc = lap8g<1>(v + j + 4, B_ + j * kRowB + 4 + lane);
                if (z == sn.x && L.xc == sn.y) acc += w1;
                float A, B;
                sponge_ab(g, L, z, A, B);
                const float qh = kp[S::prev][j] * acc;
                const float un = fmaf(2.0f * A, v[j + 4], fmaf(-B, q[j], qh));
                const unsigned oz = (o + (unsigned)j * rb - 4u * rb) | own_mask;
                bst(O2, oz, un);
                if (kKeepQ) bst_s(Q1, oz, qh);
                if (kSample) {
                    const int slot = frame_slot(fr, z, t.z0);
                    if (slot >= 0 && L.xin) sample(rm, g, t.s, slot, L.xc, d, nt, n + 1, un);
                }
            }
        }
        za += 4;
        o += 4 * rb;
        os += 4 * rb;
        of += 4 * rb;
    };
    while (za < zend) {
        block(IC<0>{});
        if (za >= zend) break;
        block(IC<1>{});
        if (za >= zend) break;
        block(IC<2>{});
        if (za >= zend) break;
        block(IC<3>{});
    }
}

// Adjoint + imaging, steps n (lam^{n+1}, lam^{n+2} -> lam^n) and n-1; the
// image takes lam^n q^n then lam^{n-1} q^{n-1} at every owned point, in that
// order, in one read-modify-write.
template <int U>
__global__ __launch_bounds__(256) void k_adj_step2(const TileRec* __restrict__ tiles, int ntiles,
                                                   const Inst* __restrict__ insts, StepArgs a) {
    static_assert(U == 4, "the two-step register rings hold 4-row blocks");
    __shared__ float lds[kWaves][kLds2];
    const Tile t = decode_tile(tiles, ntiles);
    if (!t.live) return;
    if (a.active && !a.active[t.inst]) return;
    const Inst& I = insts[t.inst];
    const WaveGrid g = I.g;
    const int j0 = I.nseg - 1 - a.seg;
    if (j0 < 0) return;
    const int len = min(I.k, I.nt - j0 * I.k);
    if (a.n - 1 >= len) return;
    const int tt = min(a.n, len - 1);  // upper step of the pair inside the segment
    const bool two = tt == a.n && tt >= 1;
    const int n = j0 * I.k + tt;
    const float* l = I.L[(n + 1) & 3];
    const float* lprev = I.L[(n + 2) & 3];
    float* out1 = I.L[n & 3];
    float* out2 = I.L[(n + 3) & 3];
    const float* r = a.r_ovr ? a.r_ovr : I.r;
    const float* qa = I.qseg + (long long)tt * I.field;
    const float* qb = two ? qa - I.field : qa;
    const int nt = I.nt;
    const RecMaps rm = I.rm;
    const float h2 = I.h2;
    const int lane = t.lane;
    float* A_ = &lds[threadIdx.x >> 6][0];
    float* F_ = A_ + 4 * kRowA;
    float* B_ = F_ + 12 * 8;
    const long long off0 = (long long)t.s * g.plane;
    const Rsrc UR = view(l + off0, g.plane);
    const Rsrc UP = view(lprev + off0, g.plane);
    const Rsrc O1 = view(out1 + off0, g.plane);
    const Rsrc O2 = view(out2 + off0, g.plane);
    const Rsrc KR = view(I.K, g.plane);
    const Rsrc QA = view(qa + off0, g.plane);
    const Rsrc QB = view(qb + off0, g.plane);
    const Rsrc GI = view(I.GI + off0, g.plane);
    const Lanes2 L = lanes2(g, t);
    const unsigned rb = (unsigned)g.pitch * 4u;
    const unsigned own_mask = L.xin ? 0u : kOut;
    const FrameRows fr = frame_rowmap(rm, g, t);
    const FastRows fast = fast_rows(g, t, L, fr, -1, two);

    const int za0 = t.z0 - 4;
    const int zend = two ? t.z1 + 4 : t.z1;
    int za = za0;
    unsigned o = L.base + row_off(za0, g.pitch);
    unsigned os = L.sbase + row_off(za0, g.pitch);
    unsigned of = L.fbase + row_off(za0, g.pitch);
    float c[4][4];   // lam^{n+1}: blocks k-1, k, k+1 in use, k+2 arriving
    float b[4][4];   // lam^n of step one: blocks k-2, k-1, k
    float kp[4][4];  // Kp: block k-1 (step two), k (step one), k+1 arriving
    float p[2][4];   // lam^{n+2}: block k, k+1 arriving
    float hs[4];     // side lanes: lam^{n+1} at row sr of blocks k-1, k, k+1 in use, k+2 arriving
    float ph[2], kh[2];  // lanes 0-31: lam^{n+2}, Kp at the frame column
    float bh[2];     // lanes 0-31: step one at the frame column, blocks k and k-1
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        c[3][i] = bld(UR, o + (unsigned)(i - 4) * rb);
        c[0][i] = bld(UR, o + (unsigned)i * rb);
        c[1][i] = bld(UR, o + (unsigned)(4 + i) * rb);
        kp[3][i] = 0.0f;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) b[rr][i] = 0.0f;
    }
    hs[3] = bld(UR, os - 4u * rb);
    hs[0] = bld(UR, os);
    hs[1] = bld(UR, os + 4u * rb);
    rows_fetch(p[0], UP, o, rb);
    rows_fetch(kp[0], KR, o, rb);
    ph[0] = bld(UP, of);
    kh[0] = bld(KR, of);
    bh[0] = bh[1] = 0.0f;

    auto block = [&](auto KC) __attribute__((always_inline)) {
        using S = Blk<decltype(KC)::value>;
        // image operands of step two's rows za-4 .. za-1, issued before the
        // next block's rows so that waiting for them leaves those in flight
        float ia[4], ib[4], ig[4];
        if (two && za - 4 >= t.z0) {
            rows_fetch_s(ia, QA, o - 4 * rb, rb);
            rows_fetch_s(ib, QB, o - 4 * rb, rb);
            rows_fetch(ig, GI, o - 4 * rb, rb);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) ia[i] = ib[i] = ig[i] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) c[S::ahead][i] = bld(UR, o + (unsigned)(8 + i) * rb);
        rows_fetch(p[S::odd], UP, o + 4 * rb, rb);
        rows_fetch(kp[S::next], KR, o + 4 * rb, rb);
        hs[S::ahead] = bld(UR, os + 8u * rb);
        ph[S::odd] = bld(UP, of + 4u * rb);
        kh[S::odd] = bld(KR, of + 4u * rb);
        float q[12];
        window(q, c[S::prev], c[S::cur], c[S::next]);
        stage_one(A_, F_, q, hs[S::prev], hs[S::cur], hs[S::next], lane, L);
        const float* fz = F_ + (4 + L.sr) * 8 + (lane & 7);
        const float* fx = A_ + L.sr * kRowA + L.fpos;
        if (is_fast(fast, za, t.z0)) {
            // with A = B = 1 the leapfrog update would otherwise fuse Kp*acc
            // into the subtraction and skip the rounding of q-hat
#pragma clang fp contract(off)
            const unsigned ow = o | own_mask;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float acc = lap8g<1>(q + j + 4, A_ + j * kRowA + 8 + lane);
                const float ln = fmaf(2.0f, q[j + 4], fmaf(-1.0f, p[S::even][j], kp[S::cur][j] * acc));
                b[S::cur][j] = ln;
                bst_row(O1, ow, (unsigned)j * rb, ln);
            }
            {
                const float acc = lap8g<8>(fz, fx);
                bh[S::even] = fmaf(2.0f, fz[0], fmaf(-1.0f, ph[S::even], kh[S::even] * acc));
            }
            float v[12];
            window(v, b[S::ahead], b[S::prev], b[S::cur]);
            stage_two(B_, v, bh[S::odd], lane, L);
            const unsigned ow2 = ow - 4u * rb;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float acc = lap8g<1>(v + j + 4, B_ + j * kRowB + 4 + lane);
                const float lm = fmaf(2.0f, v[j + 4], fmaf(-1.0f, q[j], kp[S::prev][j] * acc));
                bst_row(O2, ow2, (unsigned)j * rb, lm);
                bst_row(GI, ow2, (unsigned)j * rb, fmaf(lm, ib[j], fmaf(v[j + 4], ia[j], ig[j])));
            }
            za += 4;
            o += 4 * rb;
            os += 4 * rb;
            of += 4 * rb;
            return;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int z = za + j;
            float acc = lap8g<1>(q + j + 4, A_ + j * kRowA + 8 + lane);
            const int slot = frame_slot(fr, z, t.z0);
            if (slot >= 0 && L.xin) acc = fmaf(-h2, injected(rm, g, t.s, slot, L.xc, r, nt, n), acc);
            float A, B;
            sponge_ab(g, L, z, A, B);
            const float ln = fmaf(2.0f * A, q[j + 4], fmaf(-B, p[S::even][j], kp[S::cur][j] * acc));
            b[S::cur][j] = ln;
            if (z >= t.z0 && z < t.z1) {
                const unsigned oz = (o + (unsigned)j * rb) | own_mask;
                bst(O1, oz, ln);
                if (!two) bst(GI, oz, fmaf(ln, bld_s(QA, oz), bld(GI, oz)));
            }
        }
        // step one at the frame columns, row za + sr (lanes 0-31; 32-63 repeat them)
        {
            const int z = za + L.sr;
            float acc = lap8g<8>(fz, fx);
            const int slot = frame_slot_lane(fr, z, t.z0);
            if (slot >= 0 && L.fin) acc = fmaf(-h2, injected(rm, g, t.s, slot, L.fc, r, nt, n), acc);
            float A, B;
            sponge_pt(g, L.fsx, z, A, B);
            bh[S::even] = fmaf(2.0f * A, fz[0], fmaf(-B, ph[S::even], kh[S::even] * acc));
        }
        if (two && za - 4 >= t.z0) {
            float v[12];
            window(v, b[S::ahead], b[S::prev], b[S::cur]);
            stage_two(B_, v, bh[S::odd], lane, L);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int z = za - 4 + j;
                if (z >= t.z1) break;
                float acc = lap8g<1>(v + j + 4, B_ + j * kRowB + 4 + lane);
                const int slot = frame_slot(fr, z, t.z0);
                if (slot >= 0 && L.xin) acc = fmaf(-h2, injected(rm, g, t.s, slot, L.xc, r, nt, n - 1), acc);
                float A, B;
                sponge_ab(g, L, z, A, B);
                const float lm = fmaf(2.0f * A, v[j + 4], fmaf(-B, q[j], kp[S::prev][j] * acc));
                const unsigned oz = (o + (unsigned)j * rb - 4u * rb) | own_mask;
                bst(O2, oz, lm);
                bst(GI, oz, fmaf(lm, ib[j], fmaf(v[j + 4], ia[j], ig[j])));
            }
        }
        za += 4;
        o += 4 * rb;
        os += 4 * rb;
        of += 4 * rb;
    };
    while (za < zend) {
        block(IC<0>{});
        if (za >= zend) break;
        block(IC<1>{});
        if (za >= zend) break;
        block(IC<2>{});
        if (za >= zend) break;
        block(IC<3>{});
    }
}

// ---------------------------------------------------------------------------
// Born pair step: background u0 and scattered du with source -E * qhat0,
// E = dm_pad / m0_pad (eq. Born: -m_r d^2u0/dt^2), sampling du.
// ---------------------------------------------------------------------------
template <int U>
__global__ __launch_bounds__(256) void k_born_step(const TileRec* __restrict__ tiles, int ntiles,
                                                   const Inst* __restrict__ insts, StepArgs a) {
    __shared__ float lds[kWaves][2][U * 72];
    const Tile t = decode_tile(tiles, ntiles);
    if (!t.live) return;
    if (a.active && !a.active[t.inst]) return;
    const Inst& I = insts[t.inst];
    const WaveGrid g = I.g;
    const int n = a.n;
    if (n >= I.nt) return;
    const float* u = I.F[n & 1];
    float* uout = I.F[(n + 1) & 1];
    const float* uprev = uout;
    const float* du = I.L[n & 1];
    float* duout = I.L[(n + 1) & 1];
    const float* duprev = duout;
    const float w = I.wav[n];
    const int nt = I.nt;
    const RecMaps rm = I.rm;
    float* d = a.d_ovr ? a.d_ovr : I.d;
    const int lane = t.lane;
    const int wv = threadIdx.x >> 6;
    const long long off0 = (long long)t.s * g.plane;
    const Rsrc UR = view(u + off0, g.plane);
    const Rsrc UP = view(uprev + off0, g.plane);
    const Rsrc UO = view(uout + off0, g.plane);
    const Rsrc DR = view(du + off0, g.plane);
    const Rsrc DP = view(duprev + off0, g.plane);
    const Rsrc DO = view(duout + off0, g.plane);
    const Rsrc KR = view(I.K, g.plane);
    const Rsrc ER = view(I.E, g.plane);
    const Lanes L = lanes(g, t);
    const int2 sn = I.src.node[t.s];
    const int my_rm = strip_rowmap(rm, g, t);
    const unsigned rb = L.rb;

    unsigned o = L.o, oh = L.oh;
    Queue<U> c, e;
    queue_prime(c, UR, o, rb);
    queue_prime(e, DR, o, rb);
    float pv[U], dpv[U], kv[U], ev[U], hv[U], dhv[U];
    rows_fetch(pv, UP, o, rb);
    rows_fetch(dpv, DP, o, rb);
    rows_fetch(kv, KR, o, rb);
    rows_fetch(ev, ER, o, rb);
    rows_fetch(hv, UR, oh, rb);
    rows_fetch(dhv, DR, oh, rb);
    for (int zb = t.z0; zb < t.z1; zb += U, o += U * rb, oh += U * rb) {
        float nq[U], ne[U], npv[U], ndpv[U], nkv[U], nev[U], nhv[U], ndhv[U];
        queue_fetch(nq, UR, o, rb);
        queue_fetch(ne, DR, o, rb);
        rows_fetch(npv, UP, o + U * rb, rb);
        rows_fetch(ndpv, DP, o + U * rb, rb);
        rows_fetch(nkv, KR, o + U * rb, rb);
        rows_fetch(nev, ER, o + U * rb, rb);
        rows_fetch(nhv, UR, oh + U * rb, rb);
        rows_fetch(ndhv, DR, oh + U * rb, rb);
        stage(&lds[wv][0][0], c, hv, lane, L.hslot);
        stage(&lds[wv][1][0], e, dhv, lane, L.hslot);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int z = zb + j;
            if (z >= t.z1) break;
            const unsigned oz = o + (unsigned)j * rb;
            float acc0 = lap8(c, j, &lds[wv][0][j * 72], lane);
            const float acc1 = lap8(e, j, &lds[wv][1][j * 72], lane);
            if (z == sn.x && L.x == sn.y) acc0 += w;
            float A, B;
            sponge_ab(g, L, z, A, B);
            const float qh0 = kv[j] * acc0;
            const float un = fmaf(2.0f * A, c.q[j + 4], fmaf(-B, pv[j], qh0));
            const float dn = fmaf(2.0f * A, e.q[j + 4], fmaf(-B, dpv[j], fmaf(kv[j], acc1, -ev[j] * qh0)));
            bst(UO, oz, un);
            bst(DO, oz, dn);
            const int slot = __builtin_amdgcn_readlane(my_rm, z - t.z0);
            if (slot >= 0 && L.xin) sample(rm, g, t.s, slot, L.x, d, nt, n, dn);
        }
        queue_advance(c, nq);
        queue_advance(e, ne);
        rows_copy(pv, npv);
        rows_copy(dpv, ndpv);
        rows_copy(kv, nkv);
        rows_copy(ev, nev);
        rows_copy(hv, nhv);
        rows_copy(dhv, ndhv);
    }
}

// ---------------------------------------------------------------------------
// model preparation, Born perturbation, fold, misfit
// ---------------------------------------------------------------------------
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Kp = A c2 / m_pad on every padded cell, 0 in the pitch padding; raises flag
// for a non-positive or non-finite m.
// The scheme is stable only for velocities up to the geometry's bound, so it
// runs on m_eff = max(m, mmin), mmin = 1 / vmax_bound^2; the gradient and Born
// modelling take the derivative of that map (zero below the floor).
__global__ void k_model_prep(WaveGrid g, float c2, float mmin, const float* __restrict__ m, float* __restrict__ K,
                             int* __restrict__ flag, const int* __restrict__ active, int inst) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.plane || (active && !active[inst])) return;
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
    K[i] = A * c2 / fmaxf(mv, mmin);
}

__global__ void k_born_prep(WaveGrid g, float mmin, const float* __restrict__ m0, const float* __restrict__ dm,
                            float* __restrict__ E) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.plane) return;
    const int zp = (int)(i / g.pitch), xp = (int)(i % g.pitch);
    if (xp >= g.nxp) {
        E[i] = 0.0f;
        return;
    }
    const long long j = (long long)clampi(zp - g.nb, 0, g.nz - 1) * g.nx + clampi(xp - g.nb, 0, g.nx - 1);
    E[i] = m0[j] >= mmin ? dm[j] / m0[j] : 0.0f;  // dm moves m_eff only at or above the floor
}

__global__ void k_copy(long long n, const float* __restrict__ src, float* __restrict__ dst,
                       const int* __restrict__ active, int inst) {
    if (active && !active[inst]) return;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_zero(float* __restrict__ p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0f;
}

// grad[iz][ix] = sum over the padded cells copied from (iz, ix) of
// (sum_s gimg_s) * (1 + st) / dt^2  (the image holds lam * A dt^2 q; 1/A = 1 + st).
// Two passes in FP64, each in a fixed order: the shot sum at every padded
// cell (one coalesced sweep over the S planes), then the fold of the sponge
// cells onto the interior edge cells they copy (at most (nb+1)^2 cells for a
// corner, read from the small summed plane).
__global__ void k_shot_sum(WaveGrid g, const float* __restrict__ gimg, double* __restrict__ ssum,
                           const int* __restrict__ active, int inst) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.plane || (active && !active[inst])) return;
    double acc = 0.0;
    for (int s = 0; s < g.S; ++s) acc += (double)gimg[(long long)s * g.plane + i];
    ssum[i] = acc;
}

__global__ void k_fold(WaveGrid g, float inv_dt2, const double* __restrict__ ssum, const float* __restrict__ m,
                       float mmin, float* __restrict__ grad, const int* __restrict__ active, int inst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nz * g.nx || (active && !active[inst])) return;
    const int iz = i / g.nx, ix = i % g.nx;
    const int za = (iz == 0) ? 0 : iz + g.nb;
    const int zb = (iz == g.nz - 1) ? g.nzp - 1 : iz + g.nb;
    const int xa = (ix == 0) ? 0 : ix + g.nb;
    const int xb = (ix == g.nx - 1) ? g.nxp - 1 : ix + g.nb;
    double acc = 0.0;
    for (int zp = za; zp <= zb; ++zp) {
        const float sz = sponge_st(zp, g.nz, g.nb, g.inv_nb, g.scoef);
        for (int xp = xa; xp <= xb; ++xp) {
            const double ia = 1.0 + (double)sz + (double)sponge_st(xp, g.nx, g.nb, g.inv_nb, g.scoef);
            acc += ssum[(long long)zp * g.pitch + xp] * ia;
        }
    }
    // chain rule through m_eff = max(m, mmin): no gradient below the floor (the
    // derivative from above at the floor itself, where projected iterates sit)
    grad[i] = m[i] >= mmin ? (float)(acc * (double)inv_dt2) : 0.0f;
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
                                                             float* r, double* __restrict__ part,
                                                             const int* __restrict__ active, int inst) {
    __shared__ double sh[kReduceThreads];
    if (active && !active[inst]) return;
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
                                                               double scale, double* __restrict__ out,
                                                               const int* __restrict__ active, int inst) {
    __shared__ double sh[kReduceThreads];
    if (active && !active[inst]) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < kReduceBlocks; i += kReduceThreads) acc += part[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = s * scale;
}

// same[0] = 1 iff a and b are bitwise equal (n elements).
__global__ void k_compare(long long n, const float* __restrict__ a, const float* __restrict__ b,
                          int* __restrict__ same) {
    __shared__ int diff;
    if (threadIdx.x == 0) diff = 0;
    __syncthreads();
    int local = 0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x)
        local |= (__builtin_bit_cast(unsigned, a[i]) != __builtin_bit_cast(unsigned, b[i]));
    if (local) diff = 1;
    __syncthreads();
    if (threadIdx.x == 0) same[0] = diff ? 0 : 1;
}

}  // namespace

void launch_model_prep(hipStream_t st, const WaveGrid& g, float c2, float mmin, const float* m, float* K, int* flag,
                       const int* active, int inst) {
    const int blocks = (int)((g.plane + 255) / 256);
    hipLaunchKernelGGL(k_model_prep, dim3(blocks), dim3(256), 0, st, g, c2, mmin, m, K, flag, active, inst);
    AAFWI_HIP(hipGetLastError());
}

void launch_born_prep(hipStream_t st, const WaveGrid& g, float mmin, const float* m0, const float* dm, float* E) {
    const int blocks = (int)((g.plane + 255) / 256);
    hipLaunchKernelGGL(k_born_prep, dim3(blocks), dim3(256), 0, st, g, mmin, m0, dm, E);
    AAFWI_HIP(hipGetLastError());
}

void launch_compare(hipStream_t st, long long n, const float* a, const float* b, int* same) {
    hipLaunchKernelGGL(k_compare, dim3(1), dim3(1024), 0, st, n, a, b, same);
    AAFWI_HIP(hipGetLastError());
}

void launch_copy(hipStream_t st, long long n, const float* src, float* dst, const int* active, int inst) {
    long long blocks = (n + 255) / 256;
    blocks = blocks > 4096 ? 4096 : (blocks < 1 ? 1 : blocks);
    hipLaunchKernelGGL(k_copy, dim3((int)blocks), dim3(256), 0, st, n, src, dst, active, inst);
    AAFWI_HIP(hipGetLastError());
}

void launch_zero(hipStream_t st, float* p, long long n) {
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((int)blocks), dim3(256), 0, st, p, n);
    AAFWI_HIP(hipGetLastError());
}

void launch_step(int kernel_id, hipStream_t st, const TileRec* tiles, int ntiles, const Inst* insts,
                 const StepArgs& a) {
    const dim3 grid((ntiles + kWaves - 1) / kWaves), block(64 * kWaves);
    switch (kernel_id) {
        case AAFWI_K_FWD_STEP:
            if (a.keep_q)
                hipLaunchKernelGGL((k_fwd_step<kUFwd, kModeFwdQ>), grid, block, 0, st, tiles, ntiles, insts, a);
            else
                hipLaunchKernelGGL((k_fwd_step<kUFwd, kModeFwd>), grid, block, 0, st, tiles, ntiles, insts, a);
            break;
        case AAFWI_K_REC_STEP:
            hipLaunchKernelGGL((k_fwd_step<kUFwd, kModeRec>), grid, block, 0, st, tiles, ntiles, insts, a);
            break;
        case AAFWI_K_ADJ_STEP:
            hipLaunchKernelGGL(k_adj_step<kUAdj>, grid, block, 0, st, tiles, ntiles, insts, a);
            break;
        default:
            hipLaunchKernelGGL(k_born_step<kUBorn>, grid, block, 0, st, tiles, ntiles, insts, a);
            break;
    }
    AAFWI_HIP(hipGetLastError());
}

void launch_step2(int kernel_id, hipStream_t st, const TileRec* tiles, int ntiles, const Inst* insts,
                  const StepArgs& a) {
    const dim3 grid((ntiles + kWaves - 1) / kWaves), block(64 * kWaves);
    switch (kernel_id) {
        case AAFWI_K_FWD_STEP:
            if (a.keep_q)
                hipLaunchKernelGGL((k_fwd_step2<kUFwd, kModeFwdQ>), grid, block, 0, st, tiles, ntiles, insts, a);
            else
                hipLaunchKernelGGL((k_fwd_step2<kUFwd, kModeFwd>), grid, block, 0, st, tiles, ntiles, insts, a);
            break;
        case AAFWI_K_REC_STEP:
            hipLaunchKernelGGL((k_fwd_step2<kUFwd, kModeRec>), grid, block, 0, st, tiles, ntiles, insts, a);
            break;
        case AAFWI_K_ADJ_STEP:
            hipLaunchKernelGGL(k_adj_step2<kUAdj>, grid, block, 0, st, tiles, ntiles, insts, a);
            break;
        default:
            throw Error{AAFWI_E_INVALID, "launch_step2: no two-step Born kernel"};
    }
    AAFWI_HIP(hipGetLastError());
}

void launch_fold(hipStream_t st, const WaveGrid& g, float inv_dt2, const float* gimg, double* ssum, const float* m,
                 float mmin, float* grad, const int* active, int inst) {
    hipLaunchKernelGGL(k_shot_sum, dim3((unsigned)((g.plane + 255) / 256)), dim3(256), 0, st, g, gimg, ssum, active,
                       inst);
    AAFWI_HIP(hipGetLastError());
    const int n = g.nz * g.nx;
    hipLaunchKernelGGL(k_fold, dim3((n + 255) / 256), dim3(256), 0, st, g, inv_dt2, (const double*)ssum, m, mmin,
                       grad, active, inst);
    AAFWI_HIP(hipGetLastError());
}

void launch_residual_misfit(hipStream_t st, long long n, const float* d, const float* dobs, float* r,
                            double* partials, double* J, const int* active, int inst) {
    hipLaunchKernelGGL(k_residual, dim3(kReduceBlocks), dim3(kReduceThreads), 0, st, n, d, dobs, r, partials,
                       active, inst);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kReduceThreads), 0, st, (const double*)partials, 0.5, J,
                       active, inst);
    AAFWI_HIP(hipGetLastError());
}

}  // namespace aafwi
