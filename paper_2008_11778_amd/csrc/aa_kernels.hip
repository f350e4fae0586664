// Anderson-acceleration step for gradient descent (Algorithm 2, Steps 1-3,
// eq. Ak, eq. AAopt2, eq. solveGamma, eq. AA2_update) and the FP64 vector
// reductions used by the line search.
//
// With f_i = -eta g_i the least-squares problem min ||A_k gamma - f_k|| has
// A_k = -eta [g_{i+1} - g_i], so gamma = argmin ||dG gamma - g_k|| with
// dG = [g_{i+1} - g_i] does not depend on eta.  The device keeps a ring of
// the last M+1 accepted (p_i, g_i) in FP32, the FP64 Gram matrix of the
// consecutive gradient differences (each difference formed exactly in FP64
// from two FP32 values) and the right-hand side dG^T g_k.  Each step adds
// one Gram row/column in a single pass over the window, then one workgroup
// decomposes the Gram matrix (Jacobi in parallel ordering, FP64): the oldest
// columns are dropped while cond_2(A_k) = sqrt(lmax/lmin) exceeds cond_max,
// and gamma = V diag(1/l) V^T rhs.  The mixing pass forms, per element in FP64,
//   p_bar   = p_k - eta g_k
//   p_tilde = p_bar - sum_i gamma_i [(p_{i+1} - p_i) - eta (g_{i+1} - g_i)].
//
// Second solver (the update the paper's Algorithm 2, Step 2 names): a QR
// factorisation dG = Q R kept up to date as columns enter and leave the
// window, with Q (n x m, FP64) on the device and R (m x m) in the state.  A
// new difference column is orthogonalised against Q by classical
// Gram-Schmidt with one reorthogonalisation; dropping the oldest column
// leaves R upper Hessenberg, which Givens rotations G restore, and Q becomes
// the leading columns of Q G^T (applied as one small matrix product per
// element).  gamma = R^{-1} Q^T g_k by back substitution.  The conditioning
// of R is that of dG, so the solve is not squared as in the Gram form; the
// drop rule is the same (cond_2(R) = sqrt(lmax/lmin) of R^T R).
#include <cmath>
#include <algorithm>
#include <new>
#include <vector>

#include "common.hpp"

namespace aafwi {

constexpr int kAACap = 32;  // ring capacity bound: M + 1 <= 32

struct AAState {
    int head, count, slot_new, mk;
    double cond;
    double gram[kAACap * kAACap];
    double rhs[kAACap];
    double gamma[kAACap];
    // QR solver
    int rot_in, rot_out;          // pending Q <- Q W, W: rot_in x rot_out (0: none)
    double R[kAACap * kAACap];    // upper triangular, row-major, stride kAACap
    double W[kAACap * kAACap];
    double c1[kAACap], c2[kAACap];
    double nrm2;
};

namespace {

__device__ __forceinline__ double wave_reduce(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void aa_prepare_body(AAState* s, int cap) {
    if (s->count == cap) {
        // drop the oldest iterate and its gradient difference
        const int ndg = s->count - 1;
        for (int i = 0; i + 1 < ndg; ++i)
            for (int j = 0; j + 1 < ndg; ++j) s->gram[i * kAACap + j] = s->gram[(i + 1) * kAACap + j + 1];
        s->head = (s->head + 1) % cap;
        s->count -= 1;
    }
    s->slot_new = (s->head + s->count) % cap;
}

__global__ void k_aa_prepare(AAState* s, int cap) {
    if (threadIdx.x != 0) return;
    aa_prepare_body(s, cap);
}

// One pass: copy (p_new, g_new) into the ring and accumulate, per block,
//   cross[i] = dnew . dG_i (i < cnt-1), cross[cnt-1] = dnew . dnew,
//   rhs[i]   = dG_i . g_new (i < cnt-1), rhs[cnt-1] = dnew . g_new,
// with dnew = g_new - g_{cnt-1}.
template <int CAP>
__device__ __forceinline__ void aa_dots_body(long long n, const float* __restrict__ p_new,
                                             const float* __restrict__ g_new, float* __restrict__ ring_p,
                                             float* __restrict__ ring_g, int cap, const AAState* __restrict__ s,
                                             const float* __restrict__ w, double* __restrict__ part, int blk) {
    const int cnt = s->count, head = s->head, slot_new = s->slot_new;
    double cross[CAP], rhs[CAP];
#pragma unroll
    for (int i = 0; i < CAP; ++i) cross[i] = rhs[i] = 0.0;
    for (long long e = (long long)blk * kReduceThreads + threadIdx.x; e < n;
         e += (long long)kReduceBlocks * kReduceThreads) {
        const float gn = g_new[e];
        ring_p[(long long)slot_new * n + e] = p_new[e];
        ring_g[(long long)slot_new * n + e] = gn;
        if (cnt == 0) continue;
        float gv[CAP];
#pragma unroll
        for (int i = 0; i < CAP; ++i)
            gv[i] = (i < cnt) ? ring_g[(long long)((head + i) % cap) * n + e] : 0.0f;
        double glast = 0.0;
#pragma unroll
        for (int i = 0; i < CAP; ++i)
            if (i == cnt - 1) glast = (double)gv[i];
        const double wv = w ? (double)w[e] : 1.0;
        const double dnew = (double)gn - glast;
        const double wd = wv * dnew, wg = wv * (double)gn;
#pragma unroll
        for (int i = 0; i + 1 < CAP; ++i) {
            if (i + 1 < cnt) {
                const double dg = (double)gv[i + 1] - (double)gv[i];
                cross[i] += wd * dg;
                rhs[i] += dg * wg;
            }
        }
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            if (i == cnt - 1) {
                cross[i] += wd * dnew;
                rhs[i] += dnew * wg;
            }
        }
    }
    __shared__ double sh[kReduceThreads / 64][2 * CAP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
        const double a = wave_reduce(cross[i]);
        const double b = wave_reduce(rhs[i]);
        if (lane == 0) {
            sh[wv][i] = a;
            sh[wv][CAP + i] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * CAP) {
        double t = 0.0;
        for (int w = 0; w < kReduceThreads / 64; ++w) t += sh[w][threadIdx.x];
        part[(long long)blk * 2 * CAP + threadIdx.x] = t;
    }
}

template <int CAP>
__global__ __launch_bounds__(kReduceThreads) void k_aa_dots(long long n, const float* __restrict__ p_new,
                                                            const float* __restrict__ g_new,
                                                            float* __restrict__ ring_p,
                                                            float* __restrict__ ring_g, int cap,
                                                            const AAState* __restrict__ s,
                                                            const float* __restrict__ w,
                                                            double* __restrict__ part) {
    aa_dots_body<CAP>(n, p_new, g_new, ring_p, ring_g, cap, s, w, part, blockIdx.x);
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fixed-order sum of the kReduceBlocks partial rows (row stride `stride`
// doubles, the first NV used) by one wavefront: lane l adds rows
// R l .. R l + R - 1 in order (R = kReduceBlocks / 64), then a butterfly
// combines the lanes, so every lane returns the same NV sums.
template <int NV>
__device__ __forceinline__ void wave_partial_sums(const double* __restrict__ part, int stride, double (&acc)[NV]) {
    static_assert(kReduceBlocks % 64 == 0, "partial rows split evenly over the lanes");
    constexpr int R = kReduceBlocks / 64;
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int j = 0; j < R; ++j) {
        const double* row = part + (long long)(l * R + j) * stride;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += row[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = wave_reduce(acc[v]);
}

// Jacobi eigen-decomposition of the symmetric n x n matrix S (row stride
// kAACap, n <= 31), overwritten by its diagonalisation; V receives the
// vectors.  Parallel ordering: the indices (plus a dummy one when n is odd)
// are paired round-robin, so each round holds n/2 disjoint (p, q) pairs and a
// sweep of n - 1 rounds meets every pair once.  Rotations of disjoint pairs
// commute, so a round applies all of its rotations at once: each lane
// computes the angle of one pair from the same matrix, then the column, row
// and vector updates are spread over the wavefront (one element pair per
// lane and pass).  The angle and the threshold are those of the classical
// cyclic method.  Called by all 64 lanes of a single-wave block, S and V in
// LDS.

__device__ void jacobi_eig_wave(double* S, double* V, int n) {
    __shared__ double rc[kAACap / 2], rs[kAACap / 2];
    __shared__ int rp[kAACap / 2], rq[kAACap / 2];
    const int k = threadIdx.x;
    if (k < n)
        for (int i = 0; i < n; ++i) V[k * kAACap + i] = (i == k) ? 1.0 : 0.0;
    wave_sync_lds();
    const int N = n + (n & 1);  // players, with index n as the dummy when n is odd
    const int half = N / 2;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        if (k < n)
            for (int j = 0; j < n; ++j) {
                const double v = S[k * kAACap + j];
                if (j == k)
                    diag = v * v;
                else
                    off += v * v;
            }
        // butterfly sums: every lane holds the same value, so all take the same exit
        off = wave_reduce(off);  // both triangles
        diag = wave_reduce(diag);
        if (off <= 2e-32 * diag || off == 0.0) break;
        for (int r = 0; r < N - 1; ++r) {
            if (k < half) {
                // circle method: position 0 holds index 0, positions 1 .. N-1 rotate by r
                const int a = (k == 0) ? 0 : 1 + (k - 1 + r) % (N - 1);
                const int b = 1 + (N - 2 - k + r) % (N - 1);  // position N-1-k
                int p = min(a, b), q = max(a, b);
                double c = 1.0, sn = 0.0;
                if (q >= n) {
                    p = q = -1;  // paired with the dummy: no rotation
                } else {
                    const double apq = S[p * kAACap + q];
                    if (apq != 0.0) {
                        const double app = S[p * kAACap + p], aqq = S[q * kAACap + q];
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t =
                            (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                    }
                }
                rp[k] = p;
                rq[k] = q;
                rc[k] = c;
                rs[k] = sn;
            }
            wave_sync_lds();
            for (int it = k; it < n * half; it += 64) {  // columns p, q of every pair
                const int i = it % n, m = it / n;
                const int p = rp[m], q = rq[m];
                if (p < 0) continue;
                const double c = rc[m], sn = rs[m];
                const double sip = S[i * kAACap + p], siq = S[i * kAACap + q];
                S[i * kAACap + p] = c * sip - sn * siq;
                S[i * kAACap + q] = sn * sip + c * siq;
            }
            wave_sync_lds();
            for (int it = k; it < n * half; it += 64) {  // rows p, q of every pair
                const int j = it % n, m = it / n;
                const int p = rp[m], q = rq[m];
                if (p < 0) continue;
                const double c = rc[m], sn = rs[m];
                const double spj = S[p * kAACap + j], sqj = S[q * kAACap + j];
                S[p * kAACap + j] = c * spj - sn * sqj;
                S[q * kAACap + j] = sn * spj + c * sqj;
            }
            wave_sync_lds();
            if (k < half && rp[k] >= 0) S[rp[k] * kAACap + rq[k]] = S[rq[k] * kAACap + rp[k]] = 0.0;
            for (int it = k; it < n * half; it += 64) {  // vectors
                const int i = it % n, m = it / n;
                const int p = rp[m], q = rq[m];
                if (p < 0) continue;
                const double c = rc[m], sn = rs[m];
                const double vip = V[i * kAACap + p], viq = V[i * kAACap + q];
                V[i * kAACap + p] = c * vip - sn * viq;
                V[i * kAACap + q] = sn * vip + c * viq;
            }
            wave_sync_lds();
        }
    }
}

template <int CAP>
__device__ void aa_solve_body(AAState* s, const double* __restrict__ part, int cap, double cond_max) {
    __shared__ double sums[2 * CAP];
    __shared__ double S[kAACap * kAACap];
    __shared__ double V[kAACap * kAACap];
    const int t = threadIdx.x;
    {
        double acc[2 * CAP];
        wave_partial_sums<2 * CAP>(part, 2 * CAP, acc);
        if (t == 0)
#pragma unroll
            for (int v = 0; v < 2 * CAP; ++v) sums[v] = acc[v];
    }
    __shared__ int ctl[2];  // lane 0 -> wave: columns left (ndg), done flag
    __syncthreads();
    // lane 0 keeps the window bookkeeping; the eigen-decompositions use the wave
    int ndg = 0;
    double cond = 1.0;
    if (t == 0) {
        const int cnt = s->count;  // before the push
        if (cnt >= 1) {
            const int k = cnt - 1;  // index of the new difference column
            for (int i = 0; i < k; ++i) {
                s->gram[k * kAACap + i] = sums[i];
                s->gram[i * kAACap + k] = sums[i];
            }
            s->gram[k * kAACap + k] = sums[k];
            for (int i = 0; i <= k; ++i) s->rhs[i] = sums[CAP + i];
        }
        s->count = cnt + 1;
        ndg = s->count - 1;
        ctl[0] = ndg;
    }
    wave_sync_lds();
    while (ctl[0] > 0) {
        const int nd = ctl[0];
        if (t == 0)
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < nd; ++j) S[i * kAACap + j] = s->gram[i * kAACap + j];
        wave_sync_lds();
        jacobi_eig_wave(S, V, nd);
        wave_sync_lds();
        if (t == 0) {
            double lmax = 0.0, lmin = INFINITY;
            for (int i = 0; i < nd; ++i) {
                lmax = fmax(lmax, S[i * kAACap + i]);
                lmin = fmin(lmin, S[i * kAACap + i]);
            }
            cond = (lmin > 0.0) ? sqrt(lmax / lmin) : INFINITY;
            ctl[1] = cond <= cond_max;
            if (ctl[1]) {
                for (int i = 0; i < nd; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < nd; ++j) {
                        double vr = 0.0;
                        for (int k = 0; k < nd; ++k) vr += V[k * kAACap + j] * s->rhs[k];
                        acc += V[i * kAACap + j] * vr / S[j * kAACap + j];
                    }
                    s->gamma[i] = acc;
                }
            } else {
                // drop the oldest column for good
                for (int i = 0; i + 1 < nd; ++i) {
                    for (int j = 0; j + 1 < nd; ++j) s->gram[i * kAACap + j] = s->gram[(i + 1) * kAACap + j + 1];
                    s->rhs[i] = s->rhs[i + 1];
                }
                s->head = (s->head + 1) % cap;
                s->count -= 1;
                ctl[0] = nd - 1;
                cond = 1.0;
            }
        }
        wave_sync_lds();
        if (ctl[1]) break;
    }
    if (t == 0) {
        ndg = ctl[0];
        s->mk = ndg;
        s->cond = (ndg > 0) ? cond : 0.0;
    }
}

template <int CAP>
__global__ __launch_bounds__(64) void k_aa_solve(AAState* s, const double* __restrict__ part, int cap,
                                                 double cond_max) {
    aa_solve_body<CAP>(s, part, cap, cond_max);
}

template <int CAP>
__device__ __forceinline__ void aa_mix_body(long long e, long long n, const float* __restrict__ p_k,
                                            const float* __restrict__ g_k, float eta, float beta,
                                            const float* __restrict__ ring_p, const float* __restrict__ ring_g,
                                            int cap, const AAState* __restrict__ s, float* __restrict__ p_bar,
                                            float* __restrict__ p_tilde) {
    const int mk = s->mk, head = s->head;
    const double et = (double)eta;
    const double eb = (double)eta * (double)beta;
    const double pb = (double)p_k[e] - et * (double)g_k[e];
    double pt = (double)p_k[e] - eb * (double)g_k[e];
    if (mk > 0) {
        float pv[CAP], gv[CAP];
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            const bool ok = i <= mk;
            const long long o = (long long)((head + i) % cap) * n + e;
            pv[i] = ok ? ring_p[o] : 0.0f;
            gv[i] = ok ? ring_g[o] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i + 1 < CAP; ++i) {
            if (i < mk) {
                const double dGi = ((double)pv[i + 1] - (double)pv[i]) - eb * ((double)gv[i + 1] - (double)gv[i]);
                pt -= s->gamma[i] * dGi;
            }
        }
    }
    p_bar[e] = (float)pb;
    p_tilde[e] = (float)pt;
}

template <int CAP>
__global__ __launch_bounds__(256) void k_aa_mix(long long n, const float* __restrict__ p_k,
                                                const float* __restrict__ g_k, float eta, float beta,
                                                const float* __restrict__ ring_p,
                                                const float* __restrict__ ring_g, int cap,
                                                const AAState* __restrict__ s, float* __restrict__ p_bar,
                                                float* __restrict__ p_tilde) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    aa_mix_body<CAP>(e, n, p_k, g_k, eta, beta, ring_p, ring_g, cap, s, p_bar, p_tilde);
}

// ---------------------------------------------------------------------------
// QR solver kernels
// ---------------------------------------------------------------------------
// Delete column 0 of the m-column factor (R, rhs): R[:, 1:] is upper
// Hessenberg; rotations on rows (i, i+1) zero its subdiagonal.  W (m_in x m)
// accumulates Q's pending transform: W <- (W G^T)[:, :m-1].
__device__ void qr_drop_first(AAState* s, int m, double* rhs) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j + 1 < m; ++j) s->R[i * kAACap + j] = s->R[i * kAACap + j + 1];
    const int m_in = s->rot_in;
    for (int i = 0; i + 1 < m; ++i) {
        const double a = s->R[i * kAACap + i], b = s->R[(i + 1) * kAACap + i];
        const double r = hypot(a, b);
        const double c = r > 0.0 ? a / r : 1.0, sn = r > 0.0 ? b / r : 0.0;
        for (int j = i; j + 1 < m; ++j) {
            const double x = s->R[i * kAACap + j], y = s->R[(i + 1) * kAACap + j];
            s->R[i * kAACap + j] = c * x + sn * y;
            s->R[(i + 1) * kAACap + j] = -sn * x + c * y;
        }
        s->R[(i + 1) * kAACap + i] = 0.0;
        if (rhs) {
            const double x = rhs[i], y = rhs[i + 1];
            rhs[i] = c * x + sn * y;
            rhs[i + 1] = -sn * x + c * y;
        }
        for (int k = 0; k < m_in; ++k) {  // columns i, i+1 of W times G_i^T
            const double x = s->W[k * kAACap + i], y = s->W[k * kAACap + i + 1];
            s->W[k * kAACap + i] = c * x + sn * y;
            s->W[k * kAACap + i + 1] = -sn * x + c * y;
        }
    }
    for (int i = 0; i + 1 < m; ++i) s->R[i * kAACap + (m - 1)] = 0.0;
    for (int j = 0; j < m; ++j) s->R[(m - 1) * kAACap + j] = 0.0;
    s->rot_out = m - 1;
}

__device__ void qr_begin_transform(AAState* s, int m) {
    s->rot_in = m;
    s->rot_out = m;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) s->W[i * kAACap + j] = (i == j) ? 1.0 : 0.0;
}

// Before the push: a full ring drops its oldest iterate and difference column.
__global__ void k_qr_prepare(AAState* s, int cap) {
    if (threadIdx.x != 0) return;
    s->rot_in = s->rot_out = 0;
    if (s->count == cap) {
        const int m = s->count - 1;
        qr_begin_transform(s, m);
        qr_drop_first(s, m, nullptr);
        s->head = (s->head + 1) % cap;
        s->count -= 1;
    }
    s->slot_new = (s->head + s->count) % cap;
}

// Q[:, j] <- sum_i Q[:, i] W[i][j], j < rot_out (no-op without a pending transform).
template <int CAP>
__global__ __launch_bounds__(256) void k_qr_rotate(long long n, double* __restrict__ Q, const AAState* __restrict__ s) {
    const int m_in = s->rot_in, m_out = s->rot_out;
    if (m_in == 0) return;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double row[CAP];
#pragma unroll
    for (int i = 0; i < CAP; ++i) row[i] = i < m_in ? Q[(long long)i * n + e] : 0.0;
    for (int j = 0; j < m_out; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < CAP; ++i)
            if (i < m_in) acc += row[i] * s->W[i * kAACap + j];
        Q[(long long)j * n + e] = acc;
    }
}

// Block partials of up to CAP dot products (written to part[block][i]).
template <int CAP>
__device__ __forceinline__ void store_partials(double (&v)[CAP], int ncol, double* part) {
    __shared__ double sh[kReduceThreads / 64][CAP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
        const double a = wave_reduce(v[i]);
        if (lane == 0) sh[wv][i] = a;
    }
    __syncthreads();
    if ((int)threadIdx.x < ncol) {
        double t = 0.0;
        for (int w = 0; w < kReduceThreads / 64; ++w) t += sh[w][threadIdx.x];
        part[(long long)blockIdx.x * 2 * kAACap + threadIdx.x] = t;
    }
}

// Push (p_new, g_new) into the ring; a = g_new - g_last (FP64) into Q[:, m];
// partials of Q[:, i] . a, i < m.
template <int CAP>
__global__ __launch_bounds__(kReduceThreads) void k_qr_append(long long n, const float* __restrict__ p_new,
                                                              const float* __restrict__ g_new,
                                                              float* __restrict__ ring_p, float* __restrict__ ring_g,
                                                              int cap, double* __restrict__ Q,
                                                              const AAState* __restrict__ s,
                                                              const float* __restrict__ w,
                                                              double* __restrict__ part) {
    const int cnt = s->count, slot_new = s->slot_new;
    const int m = cnt - 1;  // existing difference columns (if cnt >= 1)
    const int last = (s->head + cnt - 1 + cap) % cap;
    double v[CAP];
#pragma unroll
    for (int i = 0; i < CAP; ++i) v[i] = 0.0;
    for (long long e = (long long)blockIdx.x * kReduceThreads + threadIdx.x; e < n;
         e += (long long)kReduceBlocks * kReduceThreads) {
        const float gn = g_new[e];
        ring_p[(long long)slot_new * n + e] = p_new[e];
        if (cnt >= 1) {
            const double sw = w ? sqrt((double)w[e]) : 1.0;
            const double a = sw * ((double)gn - (double)ring_g[(long long)last * n + e]);
            Q[(long long)m * n + e] = a;
#pragma unroll
            for (int i = 0; i < CAP; ++i)
                if (i < m) v[i] += Q[(long long)i * n + e] * a;
        }
        ring_g[(long long)slot_new * n + e] = gn;
    }
    store_partials<CAP>(v, CAP, part);
}

// a <- a - Q[:, :m] c (c = c1 or c2); partials of Q[:, i] . a (i < m), or of
// a . a when `norm` is set.
template <int CAP>
__global__ __launch_bounds__(kReduceThreads) void k_qr_subtract(long long n, double* __restrict__ Q,
                                                                const AAState* __restrict__ s, int second,
                                                                double* __restrict__ part) {
    const int m = s->count - 1;
    double v[CAP];
#pragma unroll
    for (int i = 0; i < CAP; ++i) v[i] = 0.0;
    if (m >= 0) {
        const double* c = second ? s->c2 : s->c1;
        double cc[CAP];
#pragma unroll
        for (int i = 0; i < CAP; ++i) cc[i] = i < m ? c[i] : 0.0;
        for (long long e = (long long)blockIdx.x * kReduceThreads + threadIdx.x; e < n;
             e += (long long)kReduceBlocks * kReduceThreads) {
            double a = Q[(long long)m * n + e];
            double q[CAP];
#pragma unroll
            for (int i = 0; i < CAP; ++i) q[i] = i < m ? Q[(long long)i * n + e] : 0.0;
#pragma unroll
            for (int i = 0; i < CAP; ++i)
                if (i < m) a -= cc[i] * q[i];
            Q[(long long)m * n + e] = a;
            if (!second) {
#pragma unroll
                for (int i = 0; i < CAP; ++i)
                    if (i < m) v[i] += q[i] * a;
            } else {
                v[0] += a * a;
            }
        }
    }
    store_partials<CAP>(v, CAP, part);
}

// Q[:, m] <- a / rho; partials of Q[:, i] . (W^(1/2) g_k) for i <= m.
template <int CAP>
__global__ __launch_bounds__(kReduceThreads) void k_qr_scale_rhs(long long n, double* __restrict__ Q,
                                                                 const float* __restrict__ g_k,
                                                                 const AAState* __restrict__ s,
                                                                 const float* __restrict__ w,
                                                                 double* __restrict__ part) {
    const int m = s->count - 1;
    const double rho = sqrt(s->nrm2);
    const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
    double v[CAP];
#pragma unroll
    for (int i = 0; i < CAP; ++i) v[i] = 0.0;
    for (long long e = (long long)blockIdx.x * kReduceThreads + threadIdx.x; e < n;
         e += (long long)kReduceBlocks * kReduceThreads) {
        const double g = (w ? sqrt((double)w[e]) : 1.0) * (double)g_k[e];
        if (m >= 0) {
            const double q = Q[(long long)m * n + e] * inv;
            Q[(long long)m * n + e] = q;
        }
#pragma unroll
        for (int i = 0; i < CAP; ++i)
            if (i <= m) v[i] += Q[(long long)i * n + e] * g;
    }
    store_partials<CAP>(v, CAP, part);
}

// Fixed-order sum of the block partials (first kAACap values of each row)
// into c1, c2, nrm2 or rhs; one wavefront.
__global__ __launch_bounds__(64) void k_qr_reduce(const double* __restrict__ part, int which, AAState* s) {
    double acc[kAACap];
    wave_partial_sums<kAACap>(part, 2 * kAACap, acc);
    if (threadIdx.x != 0) return;
    if (which == 2) {
        s->nrm2 = acc[0];
        return;
    }
    double* dst = which == 0 ? s->c1 : which == 1 ? s->c2 : s->rhs;
#pragma unroll
    for (int v = 0; v < kAACap; ++v) dst[v] = acc[v];
}

// Finish the push (new column of R), apply the drop rule, solve R gamma = Q^T g_k.
__global__ __launch_bounds__(64) void k_qr_solve(AAState* s, int cap, double cond_max) {
    __shared__ double S[kAACap * kAACap];
    __shared__ double V[kAACap * kAACap];
    __shared__ int ctl[2];  // lane 0 -> wave: columns left (m), done flag
    const int t = threadIdx.x;
    double cond = 1.0;
    if (t == 0) {
        const int cnt = s->count;
        int m = 0;
        if (cnt >= 1) {
            const int k = cnt - 1;  // the new column
            for (int i = 0; i < k; ++i) {
                s->R[i * kAACap + k] = s->c1[i] + s->c2[i];
                s->R[k * kAACap + i] = 0.0;
            }
            s->R[k * kAACap + k] = sqrt(s->nrm2);
            m = k + 1;
        }
        s->count = cnt + 1;
        qr_begin_transform(s, m);
        s->rot_in = 0;  // no transform unless a column is dropped below
        ctl[0] = m;
        ctl[1] = 0;
    }
    wave_sync_lds();
    while (ctl[0] > 0) {
        const int m = ctl[0];
        if (t == 0)  // singular values of R from the eigenvalues of R^T R
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) {
                    double acc = 0.0;
                    for (int k = 0; k <= (i < j ? i : j); ++k) acc += s->R[k * kAACap + i] * s->R[k * kAACap + j];
                    S[i * kAACap + j] = acc;
                }
        wave_sync_lds();
        jacobi_eig_wave(S, V, m);
        wave_sync_lds();
        if (t == 0) {
            double lmax = 0.0, lmin = INFINITY;
            for (int i = 0; i < m; ++i) {
                lmax = fmax(lmax, S[i * kAACap + i]);
                lmin = fmin(lmin, S[i * kAACap + i]);
            }
            cond = (lmin > 0.0) ? sqrt(lmax / lmin) : INFINITY;
            ctl[1] = cond <= cond_max;
            if (ctl[1]) {
                for (int i = m - 1; i >= 0; --i) {
                    double acc = s->rhs[i];
                    for (int j = i + 1; j < m; ++j) acc -= s->R[i * kAACap + j] * s->gamma[j];
                    s->gamma[i] = acc / s->R[i * kAACap + i];
                }
            } else {
                if (s->rot_in == 0) qr_begin_transform(s, m);
                qr_drop_first(s, m, s->rhs);  // rhs becomes (G Q^T g_k) of the remaining columns
                s->head = (s->head + 1) % cap;
                s->count -= 1;
                ctl[0] = m - 1;
                cond = 1.0;
            }
        }
        wave_sync_lds();
        if (ctl[1]) break;
    }
    if (t == 0) {
        s->mk = ctl[0];
        s->cond = (ctl[0] > 0) ? cond : 0.0;
    }
}

template <int CAP>
void aa_launch_qr(hipStream_t st, long long n, const float* p, const float* g, float eta, float beta,
                  const float* w, float* ring_p, float* ring_g, int cap, AAState* s, double* part,
                  double cond_max, double* Q, float* pbar, float* ptilde) {
    const dim3 red(kReduceBlocks), rt(kReduceThreads), el((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_qr_prepare, dim3(1), dim3(64), 0, st, s, cap);
    hipLaunchKernelGGL(k_qr_rotate<CAP>, el, dim3(256), 0, st, n, Q, (const AAState*)s);
    hipLaunchKernelGGL(k_qr_append<CAP>, red, rt, 0, st, n, p, g, ring_p, ring_g, cap, Q, (const AAState*)s, w, part);
    hipLaunchKernelGGL(k_qr_reduce, dim3(1), dim3(64), 0, st, (const double*)part, 0, s);
    hipLaunchKernelGGL(k_qr_subtract<CAP>, red, rt, 0, st, n, Q, (const AAState*)s, 0, part);
    hipLaunchKernelGGL(k_qr_reduce, dim3(1), dim3(64), 0, st, (const double*)part, 1, s);
    hipLaunchKernelGGL(k_qr_subtract<CAP>, red, rt, 0, st, n, Q, (const AAState*)s, 1, part);
    hipLaunchKernelGGL(k_qr_reduce, dim3(1), dim3(64), 0, st, (const double*)part, 2, s);
    hipLaunchKernelGGL(k_qr_scale_rhs<CAP>, red, rt, 0, st, n, Q, g, (const AAState*)s, w, part);
    hipLaunchKernelGGL(k_qr_reduce, dim3(1), dim3(64), 0, st, (const double*)part, 3, s);
    hipLaunchKernelGGL(k_qr_solve, dim3(1), dim3(64), 0, st, s, cap, cond_max);
    hipLaunchKernelGGL(k_qr_rotate<CAP>, el, dim3(256), 0, st, n, Q, (const AAState*)s);
    hipLaunchKernelGGL(k_aa_mix<CAP>, el, dim3(256), 0, st, n, p, g, eta, beta, (const float*)ring_p,
                       (const float*)ring_g, cap, (const AAState*)s, pbar, ptilde);
    AAFWI_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kReduceThreads) void k_dot(long long n, const float* __restrict__ x,
                                                        const float* __restrict__ y,
                                                        const float* __restrict__ z,
                                                        double* __restrict__ part) {
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * kReduceThreads + threadIdx.x; i < n;
         i += (long long)kReduceBlocks * kReduceThreads) {
        const double yv = z ? ((double)y[i] - (double)z[i]) : (double)y[i];
        acc += (double)x[i] * yv;
    }
    __shared__ double sh[kReduceThreads / 64];
    const double w = wave_reduce(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kReduceThreads / 64; ++i) t += sh[i];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kReduceThreads) void k_sum_partials(const double* __restrict__ part,
                                                                 double* __restrict__ out) {
    __shared__ double sh[kReduceThreads / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < kReduceBlocks; i += kReduceThreads) acc += part[i];
    const double w = wave_reduce(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kReduceThreads / 64; ++i) t += sh[i];
        out[0] = t;
    }
}

// Element-wise kernels: outputs may alias inputs (same index only).
__global__ void k_blend(long long n, float lam, const float* pt, const float* pb, float* out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l = (double)lam;
    out[i] = (float)(l * (double)pt[i] + (1.0 - l) * (double)pb[i]);
}

__global__ void k_scale(long long n, float a, const float* x, float* out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = a * x[i];
}

// x = max(x, floor) in place: an iterate kept in the model's stable domain.
__global__ void k_floor(long long n, float floor, float* x) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] = fmaxf(x[i], floor);
}

// out = -Lap_h img on an nz x nx image (8th-order second differences, zero
// outside the image): the Laplacian-filtered RTM image.
__global__ void k_laplacian_filter(int nz, int nx, float inv_h2, const float* __restrict__ img,
                                   float* __restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, z = blockIdx.y;
    if (x >= nx) return;
    const float c[5] = {-205.0f / 72.0f, 8.0f / 5.0f, -1.0f / 5.0f, 8.0f / 315.0f, -1.0f / 560.0f};
    const long long o = (long long)z * nx + x;
    float acc = 2.0f * c[0] * img[o];
#pragma unroll
    for (int j = 1; j <= 4; ++j) {
        const float zl = z - j >= 0 ? img[o - (long long)j * nx] : 0.0f;
        const float zr = z + j < nz ? img[o + (long long)j * nx] : 0.0f;
        const float xl = x - j >= 0 ? img[o - j] : 0.0f;
        const float xr = x + j < nx ? img[o + j] : 0.0f;
        acc = fmaf(c[j], (zl + zr) + (xl + xr), acc);
    }
    out[o] = -acc * inv_h2;
}

__global__ void k_axpy(long long n, float a, const float* x, float* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = fmaf(a, x[i], y[i]);
}

template <int CAP>
void aa_launch(hipStream_t st, long long n, const float* p, const float* g, float eta, float beta, const float* w,
               float* ring_p, float* ring_g, int cap, AAState* s, double* part, double cond_max, float* pbar,
               float* ptilde) {
    hipLaunchKernelGGL(k_aa_prepare, dim3(1), dim3(64), 0, st, s, cap);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_aa_dots<CAP>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, st, n, p, g, ring_p,
                       ring_g, cap, (const AAState*)s, w, part);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_aa_solve<CAP>, dim3(1), dim3(64), 0, st, s, (const double*)part, cap, cond_max);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_aa_mix<CAP>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, eta, beta,
                       (const float*)ring_p, (const float*)ring_g, cap, (const AAState*)s, pbar, ptilde);
    AAFWI_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Batched step: the Gram/mixing step of many independent instances (each its
// own n, window and eta; one M) in four launches.  Instance i's work runs the
// single-instance arithmetic on its own state with the same partial-sum
// count, so its results are bitwise those of aafwi_aa_step.
// ---------------------------------------------------------------------------
struct BAAInst {
    long long n;
    const float* p;
    const float* g;
    float* pbar;
    float* ptilde;
    float* ring_p;
    float* ring_g;
    AAState* s;
    double* part;
    float eta;
    int active;
};

__global__ void k_baa_prepare(const BAAInst* __restrict__ in, int count, int cap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || !in[i].active) return;
    aa_prepare_body(in[i].s, cap);
}

template <int CAP>
__global__ __launch_bounds__(kReduceThreads) void k_baa_dots(const BAAInst* __restrict__ in, int cap) {
    const BAAInst& I = in[blockIdx.y];
    if (!I.active) return;  // uniform over the block
    aa_dots_body<CAP>(I.n, I.p, I.g, I.ring_p, I.ring_g, cap, I.s, nullptr, I.part, blockIdx.x);
}

template <int CAP>
__global__ __launch_bounds__(64) void k_baa_solve(const BAAInst* __restrict__ in, int cap, double cond_max) {
    const BAAInst& I = in[blockIdx.x];
    if (!I.active) return;
    aa_solve_body<CAP>(I.s, I.part, cap, cond_max);
}

template <int CAP>
__global__ __launch_bounds__(256) void k_baa_mix(const BAAInst* __restrict__ in, int cap) {
    const BAAInst& I = in[blockIdx.y];
    if (!I.active) return;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I.n) return;
    aa_mix_body<CAP>(e, I.n, I.p, I.g, I.eta, 1.0f, I.ring_p, I.ring_g, cap, I.s, I.pbar, I.ptilde);
}

template <int CAP>
void baa_launch(hipStream_t st, const BAAInst* tab, int count, long long max_n, int cap, double cond_max) {
    hipLaunchKernelGGL(k_baa_prepare, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, st, tab, count, cap);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_baa_dots<CAP>, dim3(kReduceBlocks, (unsigned)count), dim3(kReduceThreads), 0, st, tab, cap);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_baa_solve<CAP>, dim3((unsigned)count), dim3(64), 0, st, tab, cap, cond_max);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_baa_mix<CAP>, dim3((unsigned)((max_n + 255) / 256), (unsigned)count), dim3(256), 0, st,
                       tab, cap);
    AAFWI_HIP(hipGetLastError());
}

}  // namespace

void launch_dot(hipStream_t st, long long n, const float* x, const float* y, const float* z,
                double* partials, double* out) {
    hipLaunchKernelGGL(k_dot, dim3(kReduceBlocks), dim3(kReduceThreads), 0, st, n, x, y, z, partials);
    AAFWI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kReduceThreads), 0, st, (const double*)partials, out);
    AAFWI_HIP(hipGetLastError());
}

void launch_blend(hipStream_t st, long long n, float lam, const float* pt, const float* pb, float* out) {
    hipLaunchKernelGGL(k_blend, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, lam, pt, pb, out);
    AAFWI_HIP(hipGetLastError());
}

void launch_scale(hipStream_t st, long long n, float a, const float* x, float* out) {
    hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, out);
    AAFWI_HIP(hipGetLastError());
}

void launch_floor(hipStream_t st, long long n, float floor, float* x) {
    hipLaunchKernelGGL(k_floor, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, floor, x);
    AAFWI_HIP(hipGetLastError());
}

void launch_axpy(hipStream_t st, long long n, float a, const float* x, float* y) {
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, y);
    AAFWI_HIP(hipGetLastError());
}

}  // namespace aafwi

// ---------------------------------------------------------------------------
// C ABI: AA state and vector helpers
// ---------------------------------------------------------------------------
struct aafwi_aa {
    long long n;
    int M, cap, capT;  // cap = M + 1 slots; capT = kernel template bound
    double cond_max;
    hipStream_t stream;
    float* ring_p;
    float* ring_g;
    aafwi::AAState* state;
    double* part;
    int solver;        // AAFWI_AA_GRAM or AAFWI_AA_QR
    double* Q;         // QR solver: n x M, FP64 (allocated on first use)
    float beta;        // damping of the mixed step (1 = none)
    const float* w;    // least-squares weights (device, n), or NULL
};

namespace {

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const aafwi::Error& e) {
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

void aa_free(aafwi_aa* a) {
    if (!a) return;
    if (a->ring_p) (void)hipFree(a->ring_p);
    if (a->ring_g) (void)hipFree(a->ring_g);
    if (a->state) (void)hipFree(a->state);
    if (a->part) (void)hipFree(a->part);
    if (a->Q) (void)hipFree(a->Q);
    delete a;
}

}  // namespace

extern "C" int aafwi_aa_create(int64_t n, int32_t M, double cond_max, aafwi_stream stream, aafwi_aa** out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(out != nullptr, "aa_create: out is NULL");
        *out = nullptr;
        AAFWI_REQUIRE(n > 0, "aa_create: n must be positive");
        AAFWI_REQUIRE(M >= 1 && M + 1 <= aafwi::kAACap, "aa_create: M must be in [1, 31]");
        AAFWI_REQUIRE(cond_max >= 1.0, "aa_create: cond_max must be >= 1");
        aafwi_aa* a = new aafwi_aa{};
        a->n = n;
        a->M = M;
        a->cap = M + 1;
        a->capT = a->cap <= 4 ? 4 : a->cap <= 8 ? 8 : a->cap <= 16 ? 16 : 32;
        a->cond_max = cond_max;
        a->stream = (hipStream_t)stream;
        a->beta = 1.0f;
        try {
            auto alloc = [&](void** p, size_t bytes) {
                if (hipMalloc(p, bytes) != hipSuccess)
                    throw aafwi::Error{AAFWI_E_NOMEM, "aa_create: device allocation failed"};
            };
            alloc((void**)&a->ring_p, sizeof(float) * (size_t)n * a->cap);
            alloc((void**)&a->ring_g, sizeof(float) * (size_t)n * a->cap);
            alloc((void**)&a->state, sizeof(aafwi::AAState));
            alloc((void**)&a->part, sizeof(double) * aafwi::kReduceBlocks * 2 * aafwi::kAACap);
            AAFWI_HIP(hipMemsetAsync(a->state, 0, sizeof(aafwi::AAState), a->stream));
        } catch (...) {
            aa_free(a);
            throw;
        }
        *out = a;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_aa_reset(aafwi_aa* a) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(a != nullptr, "aa_reset: NULL state");
        AAFWI_HIP(hipMemsetAsync(a->state, 0, sizeof(aafwi::AAState), a->stream));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_aa_destroy(aafwi_aa* a) {
    return guarded([&]() -> int {
        if (!a) return AAFWI_OK;
        (void)hipStreamSynchronize(a->stream);
        aa_free(a);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_aa_step(aafwi_aa* a, const float* p_k, const float* g_k, float eta, float* p_bar,
                             float* p_tilde, double* gamma, int32_t* mk) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(a != nullptr, "aa_step: NULL state");
        AAFWI_REQUIRE(p_k && g_k && p_bar && p_tilde, "aa_step: NULL vector");
        AAFWI_REQUIRE(std::isfinite(eta) && eta >= 0.0f, "aa_step: eta must be finite and >= 0");
        if (a->solver == AAFWI_AA_QR) {
            switch (a->capT) {
                case 4: aafwi::aa_launch_qr<4>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, a->Q, p_bar, p_tilde); break;
                case 8: aafwi::aa_launch_qr<8>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, a->Q, p_bar, p_tilde); break;
                case 16: aafwi::aa_launch_qr<16>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, a->Q, p_bar, p_tilde); break;
                default: aafwi::aa_launch_qr<32>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, a->Q, p_bar, p_tilde); break;
            }
        } else {
            switch (a->capT) {
                case 4: aafwi::aa_launch<4>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, p_bar, p_tilde); break;
                case 8: aafwi::aa_launch<8>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, p_bar, p_tilde); break;
                case 16: aafwi::aa_launch<16>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, p_bar, p_tilde); break;
                default: aafwi::aa_launch<32>(a->stream, a->n, p_k, g_k, eta, a->beta, a->w, a->ring_p, a->ring_g, a->cap, a->state, a->part, a->cond_max, p_bar, p_tilde); break;
            }
        }
        if (gamma)
            AAFWI_HIP(hipMemcpyAsync(gamma, a->state->gamma, sizeof(double) * a->M, hipMemcpyDeviceToDevice,
                                     a->stream));
        if (mk)
            AAFWI_HIP(hipMemcpyAsync(mk, &a->state->mk, sizeof(int32_t), hipMemcpyDeviceToDevice, a->stream));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_aa_set_solver(aafwi_aa* a, int solver) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(a != nullptr, "aa_set_solver: NULL state");
        AAFWI_REQUIRE(solver == AAFWI_AA_GRAM || solver == AAFWI_AA_QR, "aa_set_solver: unknown solver");
        AAFWI_HIP(hipStreamSynchronize(a->stream));
        if (solver == AAFWI_AA_QR && !a->Q) {
            if (hipMalloc((void**)&a->Q, sizeof(double) * (size_t)a->n * a->M) != hipSuccess) {
                (void)hipGetLastError();
                a->Q = nullptr;
                throw aafwi::Error{AAFWI_E_NOMEM, "aa_set_solver: device allocation failed"};
            }
        }
        a->solver = solver;
        AAFWI_HIP(hipMemsetAsync(a->state, 0, sizeof(aafwi::AAState), a->stream));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_aa_set_damping(aafwi_aa* a, float beta) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(a != nullptr, "aa_set_damping: NULL state");
        AAFWI_REQUIRE(std::isfinite(beta) && beta > 0.0f, "aa_set_damping: beta must be finite and positive");
        a->beta = beta;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_aa_set_weights(aafwi_aa* a, const float* w) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(a != nullptr, "aa_set_weights: NULL state");
        AAFWI_HIP(hipStreamSynchronize(a->stream));
        a->w = w;
        AAFWI_HIP(hipMemsetAsync(a->state, 0, sizeof(aafwi::AAState), a->stream));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_aa_last_cond(aafwi_aa* a, double* cond_dev) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(a && cond_dev, "aa_last_cond: NULL argument");
        AAFWI_HIP(hipMemcpyAsync(cond_dev, &a->state->cond, sizeof(double), hipMemcpyDeviceToDevice, a->stream));
        return AAFWI_OK;
    });
}


extern "C" int aafwi_blend(aafwi_stream stream, int64_t n, float lambda, const float* p_tilde, const float* p_bar,
                           float* out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(n > 0 && p_tilde && p_bar && out, "blend: bad argument");
        aafwi::launch_blend((hipStream_t)stream, n, lambda, p_tilde, p_bar, out);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_dot(aafwi_stream stream, int64_t n, const float* x, const float* y, double* out,
                         double* workspace) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(n > 0 && x && y && out && workspace, "dot: bad argument");
        aafwi::launch_dot((hipStream_t)stream, n, x, y, nullptr, workspace, out);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_dot_diff(aafwi_stream stream, int64_t n, const float* g, const float* a, const float* b,
                              double* out, double* workspace) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(n > 0 && g && a && b && out && workspace, "dot_diff: bad argument");
        aafwi::launch_dot((hipStream_t)stream, n, g, a, b, workspace, out);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_scale(aafwi_stream stream, int64_t n, float a, const float* x, float* out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(n > 0 && x && out, "scale: bad argument");
        aafwi::launch_scale((hipStream_t)stream, n, a, x, out);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_floor(aafwi_stream stream, int64_t n, float floor, float* x) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(n > 0 && x, "floor: bad argument");
        AAFWI_REQUIRE(std::isfinite(floor), "floor: floor must be finite");
        aafwi::launch_floor((hipStream_t)stream, n, floor, x);
        return AAFWI_OK;
    });
}

extern "C" int aafwi_laplacian_filter(aafwi_stream stream, int32_t nz, int32_t nx, float h, const float* image,
                                      float* out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(nz >= 1 && nx >= 1 && image && out && image != out, "laplacian_filter: bad argument");
        AAFWI_REQUIRE(std::isfinite(h) && h > 0.0f, "laplacian_filter: h must be positive");
        AAFWI_REQUIRE(nz < 65536, "laplacian_filter: too many rows");
        const float inv_h2 = (float)(1.0 / ((double)h * (double)h));
        hipLaunchKernelGGL(aafwi::k_laplacian_filter, dim3((nx + 255) / 256, nz), dim3(256), 0, (hipStream_t)stream,
                           nz, nx, inv_h2, image, out);
        AAFWI_HIP(hipGetLastError());
        return AAFWI_OK;
    });
}

extern "C" int aafwi_axpy(aafwi_stream stream, int64_t n, float a, const float* x, float* y) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(n > 0 && x && y, "axpy: bad argument");
        aafwi::launch_axpy((hipStream_t)stream, n, a, x, y);
        return AAFWI_OK;
    });
}

// ---------------------------------------------------------------------------
// C ABI: batched Anderson step
// ---------------------------------------------------------------------------
struct aafwi_batch_aa {
    int count, M, cap, capT;
    double cond_max;
    hipStream_t stream;
    std::vector<long long> n;
    long long max_n;
    float* ring;  // per instance: ring_p then ring_g, n_i * cap floats each
    std::vector<long long> ring_off;
    aafwi::AAState* states;
    double* part;  // per instance: kReduceBlocks * 2 * kAACap doubles
    aafwi::BAAInst* dtab;
    std::vector<aafwi::BAAInst> htab;
};

namespace {
void baa_free(aafwi_batch_aa* b) {
    if (!b) return;
    if (b->ring) (void)hipFree(b->ring);
    if (b->states) (void)hipFree(b->states);
    if (b->part) (void)hipFree(b->part);
    if (b->dtab) (void)hipFree(b->dtab);
    delete b;
}
}  // namespace

extern "C" int aafwi_batch_aa_create(int32_t count, const int64_t* n, int32_t M, double cond_max,
                                     aafwi_stream stream, aafwi_batch_aa** out) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(out != nullptr, "batch_aa_create: out is NULL");
        *out = nullptr;
        AAFWI_REQUIRE(count >= 1 && count <= 65535, "batch_aa_create: count must be in [1, 65535]");
        AAFWI_REQUIRE(n != nullptr, "batch_aa_create: n is NULL");
        AAFWI_REQUIRE(M >= 1 && M + 1 <= aafwi::kAACap, "batch_aa_create: M must be in [1, 31]");
        AAFWI_REQUIRE(cond_max >= 1.0, "batch_aa_create: cond_max must be >= 1");
        aafwi_batch_aa* b = new aafwi_batch_aa{};
        b->count = count;
        b->M = M;
        b->cap = M + 1;
        b->capT = b->cap <= 4 ? 4 : b->cap <= 8 ? 8 : b->cap <= 16 ? 16 : 32;
        b->cond_max = cond_max;
        b->stream = (hipStream_t)stream;
        b->max_n = 0;
        long long total = 0;
        for (int i = 0; i < count; ++i) {
            if (n[i] <= 0) {
                delete b;
                throw aafwi::Error{AAFWI_E_INVALID, "batch_aa_create: every n must be positive"};
            }
            b->n.push_back(n[i]);
            b->ring_off.push_back(total);
            total += 2LL * n[i] * b->cap;
            b->max_n = std::max(b->max_n, (long long)n[i]);
        }
        try {
            auto alloc = [&](void** p, size_t bytes) {
                if (hipMalloc(p, bytes) != hipSuccess) {
                    (void)hipGetLastError();
                    *p = nullptr;
                    throw aafwi::Error{AAFWI_E_NOMEM, "batch_aa_create: device allocation failed"};
                }
            };
            alloc((void**)&b->ring, sizeof(float) * (size_t)total);
            alloc((void**)&b->states, sizeof(aafwi::AAState) * (size_t)count);
            alloc((void**)&b->part, sizeof(double) * aafwi::kReduceBlocks * 2 * aafwi::kAACap * (size_t)count);
            alloc((void**)&b->dtab, sizeof(aafwi::BAAInst) * (size_t)count);
            AAFWI_HIP(hipMemsetAsync(b->states, 0, sizeof(aafwi::AAState) * (size_t)count, b->stream));
        } catch (...) {
            baa_free(b);
            throw;
        }
        b->htab.resize(count);
        *out = b;
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_aa_step(aafwi_batch_aa* b, const float* const* p_k, const float* const* g_k,
                                   const float* eta, float* const* p_bar, float* const* p_tilde,
                                   const uint8_t* active) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b != nullptr, "batch_aa_step: NULL state");
        AAFWI_REQUIRE(p_k && g_k && eta && p_bar && p_tilde, "batch_aa_step: NULL argument array");
        for (int i = 0; i < b->count; ++i) {
            const bool on = active ? active[i] != 0 : true;
            if (on) {
                AAFWI_REQUIRE(p_k[i] && g_k[i] && p_bar[i] && p_tilde[i], "batch_aa_step: NULL vector");
                AAFWI_REQUIRE(std::isfinite(eta[i]) && eta[i] >= 0.0f, "batch_aa_step: eta must be finite and >= 0");
            }
            aafwi::BAAInst& I = b->htab[i];
            I.n = b->n[i];
            I.p = p_k[i];
            I.g = g_k[i];
            I.pbar = p_bar[i];
            I.ptilde = p_tilde[i];
            I.ring_p = b->ring + b->ring_off[i];
            I.ring_g = b->ring + b->ring_off[i] + b->n[i] * b->cap;
            I.s = b->states + i;
            I.part = b->part + (size_t)i * aafwi::kReduceBlocks * 2 * aafwi::kAACap;
            I.eta = eta[i];
            I.active = on ? 1 : 0;
        }
        // pageable source: the copy has consumed htab when the call returns
        AAFWI_HIP(hipMemcpyAsync(b->dtab, b->htab.data(), sizeof(aafwi::BAAInst) * b->count, hipMemcpyHostToDevice,
                                 b->stream));
        switch (b->capT) {
            case 4: aafwi::baa_launch<4>(b->stream, b->dtab, b->count, b->max_n, b->cap, b->cond_max); break;
            case 8: aafwi::baa_launch<8>(b->stream, b->dtab, b->count, b->max_n, b->cap, b->cond_max); break;
            case 16: aafwi::baa_launch<16>(b->stream, b->dtab, b->count, b->max_n, b->cap, b->cond_max); break;
            default: aafwi::baa_launch<32>(b->stream, b->dtab, b->count, b->max_n, b->cap, b->cond_max); break;
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_aa_reset(aafwi_batch_aa* b, const uint8_t* which) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b != nullptr, "batch_aa_reset: NULL state");
        for (int i = 0; i < b->count; ++i)
            if (!which || which[i])
                AAFWI_HIP(hipMemsetAsync(b->states + i, 0, sizeof(aafwi::AAState), b->stream));
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_aa_state(aafwi_batch_aa* b, double* gamma, int32_t* mk) {
    return guarded([&]() -> int {
        AAFWI_REQUIRE(b != nullptr, "batch_aa_state: NULL state");
        for (int i = 0; i < b->count; ++i) {
            if (gamma)
                AAFWI_HIP(hipMemcpyAsync(gamma + (size_t)i * b->M, b->states[i].gamma, sizeof(double) * b->M,
                                         hipMemcpyDeviceToDevice, b->stream));
            if (mk)
                AAFWI_HIP(hipMemcpyAsync(mk + i, &b->states[i].mk, sizeof(int32_t), hipMemcpyDeviceToDevice,
                                         b->stream));
        }
        return AAFWI_OK;
    });
}

extern "C" int aafwi_batch_aa_destroy(aafwi_batch_aa* b) {
    return guarded([&]() -> int {
        if (!b) return AAFWI_OK;
        (void)hipStreamSynchronize(b->stream);
        baa_free(b);
        return AAFWI_OK;
    });
}
