// SDMM (Sec. 4.4, Algorithm 1) with S = 3: L1 = Psi^dagger, L2 = Phi, L3 = I,
// f1 = ||W .||_1, f2 = indicator of the l2 ball of radius eps around y,
// f3 = indicator of the positive orthant; x-update by conjugate gradient on
// Q = Phi^dagger Phi + 2 I (Parseval Psi, Sec. 4.4).
//
// Everything is enqueued on the caller's stream; inner products, norms and
// the CG scalars alpha, beta are double precision and stay on the device.
// Reductions are deterministic: each block writes a partial sum to a slot,
// and every consumer block adds the slot's partials in the same fixed order.
// Visibility-length vectors (y, z2, Phi x) are kept in plan order, so Phi and
// Phi^dagger inside the loop avoid the permutation to the caller's order.
//
// The CG of step 5 is warm-started from the previous xhat, so its initial
// residual is b - Phi^dagger Phi xhat - 2 xhat with b = x1 + x2 + x3 and
// x2 = Phi^dagger w2.  Since Phi xhat is at hand (step 8 forms it, s2, for the
// l2-ball prox), the state keeps rhs = b - Phi^dagger Phi xhat =
// x1 + x3 + Phi^dagger (w2 - s2): one Phi^dagger per iteration instead of a
// Phi/Phi^dagger pair plus Phi^dagger w2, and the difference is taken in the
// visibility domain.  The initialisation sets it for the starting xhat;
// b itself is formed only for the exported state (rhs + Phi^dagger s2).
#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>

#include "common.hpp"

namespace riop {


constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

// Partial-sum slots (each kRedBlocks doubles).
enum Slot { SLOT_RR0 = 0, SLOT_RR1, SLOT_PQ, SLOT_E, SLOT_NU, SLOT_MAX, SLOT_F1, kSlots };
// Scalar slots.
// SC_GAMMA is the penalty of the SDMM state; SC_GAMMA_Q receives riop_gamma's
// value, so that a query between SDMM steps leaves the running state alone.
// SC_RR0 is the squared norm of CG's initial residual, SC_CGIT the CG
// iterations that changed the iterate in the current solve.
enum Scalar { SC_GAMMA = 0, SC_F1ACC, SC_F1PREV, SC_EPS, SC_RRFINAL, SC_ITER, SC_GAMMA_Q, SC_P2SCALE, SC_RR0, SC_CGIT,
              kScalars };

__device__ inline double block_sum(double v) {
    __shared__ double red[kRedThreads];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline double block_max(double v) {
    __shared__ double red[kRedThreads];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Sum of one slot's partials, in a fixed order, computed by the whole block.
__device__ inline double slot_sum(const double *partials, int slot) {
    __shared__ double tot;
    double v = 0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) v += partials[slot * kRedBlocks + i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) tot = s;
    __syncthreads();
    return tot;
}

#define GRID_LOOP(i, n) for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

// Grid-stride loop over kU elements per thread per step: a thread's elements
// are i0, i0 + stride, ..., the same order as GRID_LOOP, so per-thread sums are
// unchanged.  The kernels below read all kU elements of a step before writing
// any: their arrays may alias as far as the compiler knows, so it would not
// move a later element's loads above an earlier one's stores, and one element
// per thread in flight is too little to cover HBM latency.
constexpr int kU = 4;
#define CHUNK_LOOP(i0, st, n)                                                                  \
    for (long st = (long)gridDim.x * blockDim.x, i0 = (long)blockIdx.x * blockDim.x + threadIdx.x; \
         i0 < (n); i0 += kU * st)
#define FOR_U(u) _Pragma("unroll") for (int u = 0; u < kU; ++u)

template <typename R> __device__ inline double abs2(C<R> z) { return (double)z.x * z.x + (double)z.y * z.y; }

// r = b - (Qx_partial + 2 x); p = r; slot <- sum |r|^2 (ax null: Qx_partial = 0);
// the CG iteration count restarts.
template <typename R>
__global__ void cg_init(const C<R> *b, const C<R> *x, const C<R> *ax, C<R> *r, C<R> *p, long N, double *partials,
                        int slot, double *scalars) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scalars[SC_CGIT] = 0.0;
    double acc = 0;
    CHUNK_LOOP(i0, st, N) {
        C<R> xv[kU], av[kU], bv[kU];
        FOR_U(u) if (i0 + u * st < N) {
            xv[u] = x[i0 + u * st];
            av[u] = ax ? ax[i0 + u * st] : mk<R>(0, 0);
            bv[u] = b[i0 + u * st];
        }
        FOR_U(u) if (i0 + u * st < N) {
            const long i = i0 + u * st;
            const C<R> ri = mk<R>(bv[u].x - (av[u].x + R(2) * xv[u].x), bv[u].y - (av[u].y + R(2) * xv[u].y));
            r[i] = ri;
            p[i] = ri;
            acc += abs2<R>(ri);
        }
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[slot * kRedBlocks + blockIdx.x] = s;
}

// qp <- qp + 2 p ; slot <- sum Re(conj(p) qp)
template <typename R> __global__ void cg_pq(const C<R> *p, C<R> *qp, long N, double *partials, int slot) {
    double acc = 0;
    CHUNK_LOOP(i0, st, N) {
        C<R> pv[kU], qv[kU];
        FOR_U(u) if (i0 + u * st < N) {
            pv[u] = p[i0 + u * st];
            qv[u] = qp[i0 + u * st];
        }
        FOR_U(u) if (i0 + u * st < N) {
            const C<R> pi = pv[u];
            C<R> q = qv[u];
            q.x += R(2) * pi.x;
            q.y += R(2) * pi.y;
            qp[i0 + u * st] = q;
            acc += (double)pi.x * q.x + (double)pi.y * q.y;
        }
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[slot * kRedBlocks + blockIdx.x] = s;
}

// alpha = rr_old / pq ; x += alpha p ; r -= alpha qp ; slot_new <- sum |r|^2.
// With tol2 > 0, CG stops (alpha = 0 from then on, the iterate frozen) once
// |r|^2 <= tol2 |r_0|^2, r_0 the initial residual (first = 1 records |r_0|^2).
template <typename R>
__global__ void cg_update(C<R> *x, C<R> *r, const C<R> *p, const C<R> *qp, long N, double *partials, int slot_old,
                          int slot_pq, int slot_new, double *scalars, double tol2, int first) {
    // The first chunk's loads are issued before the partial sums are read,
    // so that the two latencies overlap.
    const long st = (long)gridDim.x * blockDim.x;
    long i0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
    C<R> pv[kU], qv[kU], xv[kU], rv[kU];
    auto load = [&](long b) {
        FOR_U(u) if (b + u * st < N) {
            const long i = b + u * st;
            pv[u] = p[i];
            qv[u] = qp[i];
            xv[u] = x[i];
            rv[u] = r[i];
        }
    };
    load(i0);
    const double rr = slot_sum(partials, slot_old);
    const double pq = slot_sum(partials, slot_pq);
    const double rr0 = first ? rr : scalars[SC_RR0];
    const bool converged = tol2 > 0.0 && rr <= tol2 * rr0;
    const double alpha = (rr == 0.0 || pq == 0.0 || converged) ? 0.0 : rr / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (first) scalars[SC_RR0] = rr;
        if (alpha != 0.0) scalars[SC_CGIT] += 1.0;
    }
    double acc = 0;
    for (bool head = true; i0 < N; i0 += kU * st, head = false) {
        if (!head) load(i0);
        FOR_U(u) if (i0 + u * st < N) {
            const long i = i0 + u * st;
            C<R> xi = xv[u], ri = rv[u];
            xi.x = (R)((double)xi.x + alpha * pv[u].x);
            xi.y = (R)((double)xi.y + alpha * pv[u].y);
            ri.x = (R)((double)ri.x - alpha * qv[u].x);
            ri.y = (R)((double)ri.y - alpha * qv[u].y);
            x[i] = xi;
            r[i] = ri;
            acc += abs2<R>(ri);
        }
    }
    __syncthreads();
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[slot_new * kRedBlocks + blockIdx.x] = s;
}

// beta = rr_new / rr_old ; p = r + beta p
template <typename R>
__global__ void cg_direction(const C<R> *r, C<R> *p, long N, const double *partials, int slot_old, int slot_new) {
    const double rr_old = slot_sum(partials, slot_old);
    const double rr_new = slot_sum(partials, slot_new);
    const double beta = rr_old == 0.0 ? 0.0 : rr_new / rr_old;
    CHUNK_LOOP(i0, st, N) {
        C<R> rv[kU], pv[kU];
        FOR_U(u) if (i0 + u * st < N) {
            rv[u] = r[i0 + u * st];
            pv[u] = p[i0 + u * st];
        }
        FOR_U(u) if (i0 + u * st < N) {
            p[i0 + u * st] = mk<R>((R)((double)rv[u].x + beta * pv[u].x), (R)((double)rv[u].y + beta * pv[u].y));
        }
    }
}

// An exactly zero residual stops CG: the update kernels above turn 0/0 into
// alpha = beta = 0, so the iterate no longer changes.

__global__ void slot_to_scalar(const double *partials, int slot, double *scalars, int which) {
    const double s = slot_sum(partials, slot);
    if (threadIdx.x == 0) scalars[which] = s;
}

// out = a + 2 b
template <typename R> __global__ void add_2x(const C<R> *a, const C<R> *b, C<R> *out, long N) {
    GRID_LOOP(i, N) {
        const C<R> ai = a[i], bi = b[i];
        out[i] = mk<R>(ai.x + R(2) * bi.x, ai.y + R(2) * bi.y);
    }
}

// slot <- max |v|
template <typename R> __global__ void max_abs(const C<R> *v, long n, double *partials, int slot) {
    double m = 0;
    GRID_LOOP(i, n) m = fmax(m, sqrt(abs2<R>(v[i])));
    const double s = block_max(m);
    if (threadIdx.x == 0) partials[slot * kRedBlocks + blockIdx.x] = s;
}

__global__ void gamma_from_max(const double *partials, int slot, double beta, double *scalars, int which) {
    double m = 0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) m = fmax(m, partials[slot * kRedBlocks + i]);
    m = block_max(m);
    if (threadIdx.x == 0) scalars[which] = beta * m;
}

__global__ void set_scalar(double *scalars, int which, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) scalars[which] = v;
}

// Gather / scatter between caller order and plan order.
template <typename R> __global__ void gather_perm(const C<R> *src, const int *perm, C<R> *dst, long M) {
    GRID_LOOP(i, M) dst[i] = src[perm[i]];
}
template <typename R> __global__ void scatter_perm(const C<R> *src, const int *perm, C<R> *dst, long M) {
    GRID_LOOP(i, M) dst[perm[i]] = src[i];
}

// prox2 pass 1: slot_e <- sum |s + z2 - y|^2, slot_nu <- sum |y - s|^2
template <typename R>
__global__ void prox2_norms(const C<R> *s, const C<R> *z2, const C<R> *y, long M, double *partials) {
    double e = 0, nu = 0;
    CHUNK_LOOP(i0, st, M) {
        C<R> sv[kU], zv[kU], yv[kU];
        FOR_U(u) if (i0 + u * st < M) {
            sv[u] = s[i0 + u * st];
            zv[u] = z2[i0 + u * st];
            yv[u] = y[i0 + u * st];
        }
        FOR_U(u) if (i0 + u * st < M) {
            const C<R> si = sv[u], zi = zv[u], yi = yv[u];
            const double dr = (double)si.x + zi.x - yi.x, di = (double)si.y + zi.y - yi.y;
            e += dr * dr + di * di;
            const double fr = (double)yi.x - si.x, fi = (double)yi.y - si.y;
            nu += fr * fr + fi * fi;
        }
    }
    const double se = block_sum(e);
    const double sn = block_sum(nu);
    if (threadIdx.x == 0) {
        partials[SLOT_E * kRedBlocks + blockIdx.x] = se;
        partials[SLOT_NU * kRedBlocks + blockIdx.x] = sn;
    }
}

// prox2 pass 2, its scale: min(1, eps / ||s + z2 - y||).  The rest of the
// pass (v = s + z2; r2 = y + (v - y) scale; z2 <- v - r2; the values
// (r2 - z2) - s for Phi^dagger) runs inside the gridding kernel.
__global__ void prox2_scale(const double *partials, double *scalars) {
    const double e = sqrt(slot_sum(partials, SLOT_E));
    const double eps = scalars[SC_EPS];
    if (threadIdx.x == 0) scalars[SC_P2SCALE] = e > eps ? eps / e : 1.0;
}

// prox3 and the right-hand side: v = xhat + z3; r3 = max(Re v, 0);
// z3 <- v - r3; rhs = x1 + x2 + (r3 - z3), where the x2 passed in is
// Phi^dagger (w2 - Phi xhat), so rhs is the sum less Phi^dagger Phi xhat.
template <typename R>
__global__ void prox3_rhs(const C<R> *xh, C<R> *z3, const C<R> *x1, const C<R> *x2, C<R> *rhs, long N) {
    CHUNK_LOOP(i0, st, N) {
        C<R> xv[kU], zv[kU], av[kU], bv[kU];
        FOR_U(u) if (i0 + u * st < N) {
            const long i = i0 + u * st;
            xv[u] = xh[i];
            zv[u] = z3[i];
            av[u] = x1[i];
            bv[u] = x2[i];
        }
        FOR_U(u) if (i0 + u * st < N) {
            const long i = i0 + u * st;
            const R vr = xv[u].x + zv[u].x, vi = xv[u].y + zv[u].y;
            const R r3 = vr > R(0) ? vr : R(0);
            const C<R> zn = mk<R>(vr - r3, vi);
            z3[i] = zn;
            rhs[i] = mk<R>(av[u].x + bv[u].x + (r3 - zn.x), av[u].y + bv[u].y - zn.y);
        }
    }
}

// out = v (reals)
template <typename R> __global__ void fill_real(R *out, long n, R v) {
    GRID_LOOP(i, n) out[i] = v;
}

// out = a + sb b (sb = +1 or -1)
template <typename R> __global__ void lin2(const C<R> *a, const C<R> *b, R sb, C<R> *out, long N) {
    GRID_LOOP(i, N) {
        const C<R> x = a[i], y = b[i];
        out[i] = mk<R>(x.x + sb * y.x, x.y + sb * y.y);
    }
}

// First stage of f1 over the analysis blocks' partials: block b sums every
// (kRedBlocks * kRedThreads)-th partial from its own offset into slot SLOT_F1.
__global__ void f1_partials(const double *f1part, int f1_count, double *partials) {
    double v = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < f1_count; i += kRedBlocks * kRedThreads) v += f1part[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) partials[SLOT_F1 * kRedBlocks + blockIdx.x] = s;
}

// history[t] = {f1, zeta, nu, final CG rr, CG iterations} with t the device
// iteration counter (so a captured graph can be replayed); f1_prev <- f1;
// t <- t + 1.
__global__ void record_stats(const double *partials, double *scalars, double *hist, int cap, int rr_slot) {
    const double nu2 = slot_sum(partials, SLOT_NU);
    const double rr = slot_sum(partials, rr_slot);
    const double f1 = slot_sum(partials, SLOT_F1);
    if (threadIdx.x == 0) {
        const int t = (int)scalars[SC_ITER];
        scalars[SC_F1ACC] = f1;
        const double prev = scalars[SC_F1PREV];
        const double zeta = prev == 0.0 ? INFINITY : fabs(f1 - prev) / fabs(prev);
        if (t < cap) {
            double *h = hist + (long)kHistStride * t;
            h[0] = f1;
            h[1] = zeta;
            h[2] = sqrt(nu2) / scalars[SC_EPS];
            h[3] = rr;
            h[4] = scalars[SC_CGIT];
        }
        scalars[SC_F1PREV] = f1;
        scalars[SC_RRFINAL] = rr;
        scalars[SC_ITER] = (double)(t + 1);
    }
}

// ---------------------------------------------------------------------------
// Block SDMM (Sec. 4.5): one l2 ball per data block, blk[i] the block of
// plan-order visibility i.

constexpr int kMaxBlocks = 1024;

// Per reduction block, for every data block b: sum |s + z2 - y|^2 and
// sum |y - s|^2 over its visibilities, accumulated in LDS (a wavefront whose
// live visibilities share one block adds its wave sum with one atomic).
template <typename R>
__global__ void prox2_norms_blocks(const C<R> *s, const C<R> *z2, const C<R> *y, const int *blk, long M, int nb,
                                   double *bpart) {
    extern __shared__ double sh[];  // 2 nb
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) sh[i] = 0.0;
    __syncthreads();
    for (long i0 = (long)blockIdx.x * blockDim.x; i0 < M; i0 += (long)gridDim.x * blockDim.x) {
        const long i = i0 + threadIdx.x;
        const bool live = i < M;
        int b = -1;
        double e = 0.0, nu = 0.0;
        if (live) {
            b = blk[i];
            const C<R> si = s[i], zi = z2[i], yi = y[i];
            const double dr = (double)si.x + zi.x - yi.x, di = (double)si.y + zi.y - yi.y;
            const double fr = (double)yi.x - si.x, fi = (double)yi.y - si.y;
            e = dr * dr + di * di;
            nu = fr * fr + fi * fi;
        }
        const int bref = __shfl(b, 0);
        if (__all(!live || b == bref) && bref >= 0) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                e += __shfl_xor(e, o);
                nu += __shfl_xor(nu, o);
            }
            if ((threadIdx.x & 63) == 0) {
                atomicAdd(&sh[2 * bref], e);
                atomicAdd(&sh[2 * bref + 1], nu);
            }
        } else if (live) {
            atomicAdd(&sh[2 * b], e);
            atomicAdd(&sh[2 * b + 1], nu);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) bpart[(long)blockIdx.x * 2 * nb + i] = sh[i];
}

// Per data block: scale = min(1, eps_b / ||v_b - y_b||), nu_b = ||y_b - s_b|| / eps_b
// (partials summed in a fixed order); the largest nu_b, squared, becomes the
// only nonzero partial of SLOT_NU (the history's nu, with SC_EPS = 1).
__global__ void block_scales(const double *bpart, int nb, const double *beps, double *bscale, double *bnu,
                             double *partials) {
    double m = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        double e2 = 0.0, n2 = 0.0;
        for (int w = 0; w < kRedBlocks; ++w) {
            e2 += bpart[(long)w * 2 * nb + 2 * b];
            n2 += bpart[(long)w * 2 * nb + 2 * b + 1];
        }
        const double e = sqrt(e2), eps = beps[b];
        bscale[b] = e > eps ? eps / e : 1.0;
        bnu[b] = sqrt(n2) / eps;
        m = fmax(m, bnu[b]);
    }
    m = block_max(m);
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) partials[SLOT_NU * kRedBlocks + i] = i ? 0.0 : m * m;
}

// The balls' projections and duals, and the values for Phi^dagger:
// v = s + z2, r = y + (v - y) scale_b, z2 <- v - r, d = r - z2 - s.
template <typename R>
__global__ void prox2_apply_blocks(const C<R> *s, C<R> *z2, const C<R> *y, const int *blk, const double *bscale,
                                   C<R> *d, long M) {
    GRID_LOOP(i, M) {
        const C<R> si = s[i], zi = z2[i], yi = y[i];
        const double sc = bscale[blk[i]];
        const double vr = (double)si.x + zi.x, vi = (double)si.y + zi.y;
        const double rr = yi.x + (vr - yi.x) * sc, ri = yi.y + (vi - yi.y) * sc;
        const double znr = vr - rr, zni = vi - ri;
        z2[i] = mk<R>((R)znr, (R)zni);
        d[i] = mk<R>((R)(rr - znr - si.x), (R)(ri - zni - si.y));
    }
}

// blk[i] = block_of[perm[i]]; flag <- 1 if a block index is outside [0, nb).
__global__ void gather_blocks(const int *block_of, const int *perm, long M, int nb, int *blk, int *flag) {
    GRID_LOOP(i, M) {
        const int b = block_of[perm[i]];
        if (b < 0 || b >= nb) atomicOr(flag, 1);
        blk[i] = b < 0 ? 0 : (b >= nb ? nb - 1 : b);
    }
}

// ---------------------------------------------------------------------------
// Weighted TV prior (Sec. 3.3 eq. tvproblem, Sec. 5): the prox of
// lam ||W grad .||_1 by fast gradient projection on the dual (Beck &
// Teboulle), forward differences with zero last-row / last-column
// differences; complex images are real vectors of twice the length.
// gradT(p, q) below is the adjoint of the gradient (minus the divergence).

enum Prior { PRIOR_SARA = 0, PRIOR_TV = 1 };

template <typename R> __device__ inline C<R> grad_adj_at(const C<R> *p, const C<R> *q, int i, int j, int n) {
    const long k = (long)i * n + j;
    C<R> v = mk<R>(0, 0);
    if (i >= 1) v = cadd<R>(v, p[k - n]);
    if (i < n - 1) v = csub<R>(v, p[k]);
    if (j >= 1) v = cadd<R>(v, q[k - 1]);
    if (j < n - 1) v = csub<R>(v, q[k]);
    return v;
}

// b = xhat + z1 (the point the prox is taken at); the dual starts at zero.
template <typename R>
__global__ void tv_begin(const C<R> *xh, const C<R> *z1, C<R> *b, C<R> *p, C<R> *q, C<R> *r, C<R> *s, long N) {
    GRID_LOOP(i, N) {
        b[i] = cadd<R>(xh[i], z1[i]);
        const C<R> z = mk<R>(0, 0);
        p[i] = z;
        q[i] = z;
        r[i] = z;
        s[i] = z;
    }
}

// u = b - lam gradT(r, s)
template <typename R> __global__ void tv_u(const C<R> *b, const C<R> *r, const C<R> *s, C<R> *u, int n,
                                           const double *lamp) {
    const R lam = (R)*lamp;
    GRID_LOOP(k, (long)n * n) {
        const int i = (int)(k / n), j = (int)(k - (long)i * n);
        const C<R> g = grad_adj_at<R>(r, s, i, j, n);
        u[k] = mk<R>(b[k].x - lam * g.x, b[k].y - lam * g.y);
    }
}

// (p, q) <- projection onto |(p, q)_ij| <= w_ij of (r, s) + grad(u) / (8 lam);
// (r, s) <- (p, q) + c ((p, q) - (p, q)_previous).
template <typename R>
__global__ void tv_dual(const C<R> *u, const R *w, C<R> *p, C<R> *q, C<R> *r, C<R> *s, int n, const double *lamp,
                        double c) {
    const double lam = *lamp;
    const R step = lam > 0 ? (R)(1.0 / (8.0 * lam)) : R(0);
    const R cc = (R)c;
    GRID_LOOP(k, (long)n * n) {
        const int i = (int)(k / n), j = (int)(k - (long)i * n);
        const C<R> uk = u[k];
        const C<R> gx = i < n - 1 ? csub<R>(u[k + n], uk) : mk<R>(0, 0);
        const C<R> gy = j < n - 1 ? csub<R>(u[k + 1], uk) : mk<R>(0, 0);
        C<R> pn = mk<R>(r[k].x + step * gx.x, r[k].y + step * gx.y);
        C<R> qn = mk<R>(s[k].x + step * gy.x, s[k].y + step * gy.y);
        const R wk = w ? w[k] : R(1);
        if (wk > R(0)) {
            const R mag = sqrt(pn.x * pn.x + pn.y * pn.y + qn.x * qn.x + qn.y * qn.y);
            if (mag > wk) {
                const R f = wk / mag;
                pn = cscale<R>(pn, f);
                qn = cscale<R>(qn, f);
            }
        } else {
            pn = mk<R>(0, 0);
            qn = mk<R>(0, 0);
        }
        const C<R> po = p[k], qo = q[k];
        r[k] = mk<R>(pn.x + cc * (pn.x - po.x), pn.y + cc * (pn.y - po.y));
        s[k] = mk<R>(qn.x + cc * (qn.x - qo.x), qn.y + cc * (qn.y - qo.y));
        p[k] = pn;
        q[k] = qn;
    }
}

// r1 = b - lam gradT(p, q); z1 <- b - r1; x1 = r1 - z1 (Algorithm 1 steps 7-9, L1 = I).
template <typename R>
__global__ void tv_finish(const C<R> *b, const C<R> *p, const C<R> *q, C<R> *z1, C<R> *x1, int n, const double *lamp) {
    const R lam = (R)*lamp;
    GRID_LOOP(k, (long)n * n) {
        const int i = (int)(k / n), j = (int)(k - (long)i * n);
        const C<R> g = grad_adj_at<R>(p, q, i, j, n);
        const C<R> bk = b[k];
        const C<R> r1 = mk<R>(bk.x - lam * g.x, bk.y - lam * g.y);
        const C<R> zn = csub<R>(bk, r1);
        z1[k] = zn;
        x1[k] = csub<R>(r1, zn);
    }
}

// SLOT_F1 partials of f1 = sum_ij w_ij |(grad x)_ij|.
template <typename R> __global__ void tv_norm_partials(const C<R> *x, const R *w, int n, double *partials) {
    double acc = 0.0;
    GRID_LOOP(k, (long)n * n) {
        const int i = (int)(k / n), j = (int)(k - (long)i * n);
        const C<R> xk = x[k];
        const C<R> gx = i < n - 1 ? csub<R>(x[k + n], xk) : mk<R>(0, 0);
        const C<R> gy = j < n - 1 ? csub<R>(x[k + 1], xk) : mk<R>(0, 0);
        const double m = sqrt(abs2<R>(gx) + abs2<R>(gy));
        acc += w ? (double)w[k] * m : m;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[SLOT_F1 * kRedBlocks + blockIdx.x] = t;
}

// slot <- sum_ij |(grad x)_ij|^2
template <typename R> __global__ void tv_sum_mag2(const C<R> *x, int n, double *partials, int slot) {
    double acc = 0.0;
    GRID_LOOP(k, (long)n * n) {
        const int i = (int)(k / n), j = (int)(k - (long)i * n);
        const C<R> xk = x[k];
        const C<R> gx = i < n - 1 ? csub<R>(x[k + n], xk) : mk<R>(0, 0);
        const C<R> gy = j < n - 1 ? csub<R>(x[k + 1], xk) : mk<R>(0, 0);
        acc += abs2<R>(gx) + abs2<R>(gy);
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[slot * kRedBlocks + blockIdx.x] = t;
}

// RWTV weights: w_ij = delta / (delta + |(grad x)_ij|).
template <typename R> __global__ void tv_reweight(const C<R> *x, R *w, int n, double delta) {
    GRID_LOOP(k, (long)n * n) {
        const int i = (int)(k / n), j = (int)(k - (long)i * n);
        const C<R> xk = x[k];
        const C<R> gx = i < n - 1 ? csub<R>(x[k + n], xk) : mk<R>(0, 0);
        const C<R> gy = j < n - 1 ? csub<R>(x[k + 1], xk) : mk<R>(0, 0);
        w[k] = (R)(delta / (delta + sqrt(abs2<R>(gx) + abs2<R>(gy))));
    }
}

// Reweighted l1 (Sec. 3.3): w_j = delta / (delta + |alpha_j|).
template <typename R> __global__ void reweight_weights(const C<R> *alpha, R *w, long D, double delta) {
    GRID_LOOP(i, D) w[i] = (R)(delta / (delta + sqrt(abs2<R>(alpha[i]))));
}

// slot <- sum |a|^2
template <typename R> __global__ void sum_abs2(const C<R> *a, long n, double *partials, int slot) {
    double acc = 0;
    GRID_LOOP(i, n) acc += abs2<R>(a[i]);
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[slot * kRedBlocks + blockIdx.x] = s;
}

// slot_d <- sum |x - xp|^2, slot_x <- sum |x|^2
template <typename R>
__global__ void diff_norms(const C<R> *x, const C<R> *xp, long n, double *partials, int slot_d, int slot_x) {
    double d = 0, t = 0;
    GRID_LOOP(i, n) {
        const C<R> a = x[i], b = xp[i];
        const double dr = (double)a.x - b.x, di = (double)a.y - b.y;
        d += dr * dr + di * di;
        t += abs2<R>(a);
    }
    const double sd = block_sum(d);
    const double st = block_sum(t);
    if (threadIdx.x == 0) {
        partials[slot_d * kRedBlocks + blockIdx.x] = sd;
        partials[slot_x * kRedBlocks + blockIdx.x] = st;
    }
}

// ---------------------------------------------------------------------------
// Host side.

// Launch of a vector / reduction kernel, timed as the "vector" kind.
#define VEC_LAUNCH(p, ...)                          \
    do {                                            \
        TimedScope ts_((p), KK_VECTOR, s);          \
        hipLaunchKernelGGL(__VA_ARGS__);            \
    } while (0)

static dim3 RB() { return dim3(kRedBlocks); }
static dim3 RT() { return dim3(kRedThreads); }

static void ensure_work(riop_plan *p) {
    SdmmWork &w = p->sd;
    if (w.ready) return;
    const size_t cb = cbytes(p);
    const size_t N = (size_t)p->n * p->n, D = (size_t)p->q * N, M = (size_t)std::max<int64_t>(1, p->M);
    w.xhat.alloc(cb * N);
    w.rhs.alloc(cb * N);
    w.r.alloc(cb * N);
    w.p.alloc(cb * N);
    w.qp.alloc(cb * N);
    w.tmpN.alloc(cb * N);
    w.x1.alloc(cb * N);
    w.z3loc.alloc(cb * N);
    w.z1loc.alloc(cb * D);
    w.w1.alloc(cb * D);
    w.ysort.alloc(cb * M);
    w.z2loc.alloc(cb * M);
    w.s2.alloc(cb * M);
    w.partials.alloc(sizeof(double) * kSlots * kRedBlocks);
    w.f1_count = psi_adj_blocks(p);
    w.f1part.alloc(sizeof(double) * (size_t)std::max(1, w.f1_count));
    w.scalars.alloc(sizeof(double) * kScalars);
    w.ready = true;
}

template <typename R> static void gram_sorted(riop_plan *p, const void *x, void *out, hipStream_t s) {
    // out = Phi^dagger Phi x = Z^T D F^dagger (G^T G) F D Z x, with G^T G fused.
    launch_phi_fft_forward<R>(p, x, s);
    launch_gram<R>(p, p->grid.ptr, p->grid2.ptr, s);
    launch_phi_fft_adjoint<R>(p, out, s, p->grid2.ptr);
}

// out = Phi^dagger y for y in plan order.
template <typename R> static void phi_adj_sorted(riop_plan *p, const void *y, void *out, hipStream_t s) {
    launch_grid<R>(p, y, 0, s);
    launch_phi_fft_adjoint<R>(p, out, s);
}

// s2 = Phi x in plan order.
template <typename R> static void phi_into_s2(riop_plan *p, const void *x, hipStream_t s) {
    launch_phi_fft_forward<R>(p, x, s);
    launch_degrid<R>(p, p->sd.s2.ptr, 0, s);
}

// Device memory CG works in: residual, direction and Q times the direction
// (N complex each), the partial-sum slots (kSlots * kRedBlocks doubles) and
// the scalar slots (kScalars doubles).
template <typename R> struct CgWork {
    C<R> *r, *p, *qp;
    double *partials, *scalars;
};

template <typename R> static CgWork<R> plan_cg_work(riop_plan *p) {
    SdmmWork &w = p->sd;
    return CgWork<R>{w.r.as<C<R>>(), w.p.as<C<R>>(), w.qp.as<C<R>>(), w.partials.as<double>(), w.scalars.as<double>()};
}

// CG on Q from x.  b_less_gram: b already has Phi^dagger Phi x subtracted.
// Besides the plan's operator buffers it touches only `w`.
template <typename R>
static void cg_run(riop_plan *p, const void *b, void *x, int n_iter, double tol, int *final_slot, hipStream_t s,
                   const CgWork<R> &w, bool b_less_gram = false) {
    const long N = (long)p->n * p->n;
    double *part = w.partials;
    double *sc = w.scalars;
    const double tol2 = tol > 0 ? tol * tol : 0.0;
    if (!b_less_gram) gram_sorted<R>(p, x, w.qp, s);
    VEC_LAUNCH(p, cg_init<R>, RB(), RT(), 0, s, static_cast<const C<R> *>(b), static_cast<const C<R> *>(x),
                       b_less_gram ? (const C<R> *)nullptr : (const C<R> *)w.qp, w.r, w.p, N, part, (int)SLOT_RR0,
                       sc);
    RIOP_HIP(hipGetLastError());
    // Where the FFT's column passes can, they apply the direction update
    // (before transforming p) and form q + 2 p with its p.q partials (after);
    // otherwise the vector kernels do.  The direction of the last iteration is
    // never needed and is not formed.
    const bool fold = fft_folds_cg(p, kRedBlocks);
    int cur = SLOT_RR0;
    for (int k = 0; k < n_iter; ++k) {
        const int nxt = cur == SLOT_RR0 ? SLOT_RR1 : SLOT_RR0;
        CgFuse<R> cg;
        cg.part = part;
        cg.nred = kRedBlocks;
        cg.slot_pq = SLOT_PQ;
        if (k > 0) {  // p = r + beta p, beta = rr[cur] / rr[previous]
            if (fold) {
                cg.r = w.r;
                cg.slot_old = nxt;
                cg.slot_new = cur;
            } else {
                VEC_LAUNCH(p, cg_direction<R>, RB(), RT(), 0, s, (const C<R> *)w.r, w.p, N, (const double *)part,
                           nxt, cur);
            }
        }
        if (fold) cg.p = w.p;
        const bool d_done = launch_phi_fft_forward<R>(p, w.p, s, fold ? &cg : nullptr);
        launch_gram<R>(p, p->grid.ptr, p->grid2.ptr, s);
        const bool q_done = launch_phi_fft_adjoint<R>(p, w.qp, s, p->grid2.ptr, fold ? &cg : nullptr);
        RIOP_REQUIRE(d_done == (fold && k > 0) && q_done == fold, RIOP_EDEVICE, "CG step folding mismatch");
        if (!fold) VEC_LAUNCH(p, cg_pq<R>, RB(), RT(), 0, s, (const C<R> *)w.p, w.qp, N, part, (int)SLOT_PQ);
        VEC_LAUNCH(p, cg_update<R>, RB(), RT(), 0, s, static_cast<C<R> *>(x), w.r, (const C<R> *)w.p,
                           (const C<R> *)w.qp, N, part, cur, (int)SLOT_PQ, nxt, sc, tol2, k == 0 ? 1 : 0);
        RIOP_HIP(hipGetLastError());
        cur = nxt;
    }
    *final_slot = cur;
}

// gamma = beta ||L1^dagger Phi^dagger y||_inf with L1 = Psi^dagger (SARA) or I (TV).
template <typename R> static void gamma_run(riop_plan *p, const void *y_sorted_or_user, int user, double beta,
                                            hipStream_t s, int which, int prior = PRIOR_SARA) {
    ensure_work(p);
    SdmmWork &w = p->sd;
    const long N = (long)p->n * p->n, D = (long)p->q * N;
    launch_grid<R>(p, y_sorted_or_user, user, s);
    launch_phi_fft_adjoint<R>(p, w.tmpN.ptr, s);
    if (prior == PRIOR_TV) {
        VEC_LAUNCH(p, max_abs<R>, RB(), RT(), 0, s, w.tmpN.as<C<R>>(), N, w.partials.as<double>(), (int)SLOT_MAX);
    } else {
        launch_psi_adj<R>(p, w.tmpN.ptr, w.w1.ptr, s);
        VEC_LAUNCH(p, max_abs<R>, RB(), RT(), 0, s, w.w1.as<C<R>>(), D, w.partials.as<double>(), (int)SLOT_MAX);
    }
    VEC_LAUNCH(p, gamma_from_max, dim3(1), RT(), 0, s, (const double *)w.partials.as<double>(), (int)SLOT_MAX,
                       beta, w.scalars.as<double>(), which);
    RIOP_HIP(hipGetLastError());
}

// Algorithm 1, steps 1-3 (or a resumed state), penalty and data in plan order.
template <typename R>
static void sdmm_init(riop_plan *p, const void *y, double eps, const riop_sdmm_params *prm, const void *x0,
                      hipStream_t s, int prior = PRIOR_SARA, int tv_inner = 0) {
    ensure_work(p);
    SdmmWork &w = p->sd;
    const long N = (long)p->n * p->n, M = (long)p->M;
    // Length of the l1 term's variables: q N coefficients (SARA) or N pixels (TV).
    const long D = prior == PRIOR_TV ? N : (long)p->q * N;
    if (prior == PRIOR_TV) {
        for (DevBuf *b : {&w.tvb, &w.tvu, &w.tvp, &w.tvq, &w.tvr, &w.tvs}) b->reserve(cbytes(p) * (size_t)N);
    }
    if (w.prior != prior || w.tv_inner != tv_inner) ++w.epoch;
    w.prior = prior;
    w.tv_inner = tv_inner;
    const size_t cb = cbytes(p);
    double *sc = w.scalars.as<double>();
    // The history buffer only grows, so that its address (held by graphs
    // captured from riop_sdmm_step) changes only when more iterations must be
    // kept; every change of what a captured step depends on moves the epoch.
    const size_t need = sizeof(double) * kHistStride * (size_t)std::max(1, prm->T);
    if (!w.history.ptr || w.history.bytes < need) {
        w.history.alloc(need);
        ++w.epoch;
    }
    w.hist_cap = (int)std::min<size_t>(w.history.bytes / (sizeof(double) * kHistStride), 1u << 30);
    if (w.n_cg != prm->n_cg || w.weights != prm->weights || w.cg_tol != prm->cg_tol || w.nblocks != 0) ++w.epoch;
    w.nblocks = 0;  // a blocked run sets it after this initialisation
    w.n_cg = prm->n_cg;
    w.weights = prm->weights;
    w.cg_tol = prm->cg_tol;
    C<R> *xh = w.xhat.as<C<R>>();
    // Caller inputs: NaN or Inf sets the plan's non-finite flag.
    check_finite_input(p, y, 2 * M, s);
    check_finite_input(p, x0, 2 * N, s);
    check_finite_input(p, prm->weights, D, s);
    if (prm->resume) {
        check_finite_input(p, prm->z1, 2 * D, s);
        check_finite_input(p, prm->z2, 2 * M, s);
        check_finite_input(p, prm->z3, 2 * N, s);
        check_finite_input(p, prm->rhs, 2 * N, s);
    }

    if (M > 0)
        VEC_LAUNCH(p, gather_perm<R>, RB(), RT(), 0, s, static_cast<const C<R> *>(y), p->perm.as<int>(),
                   w.ysort.as<C<R>>(), M);
    VEC_LAUNCH(p, set_scalar, dim3(1), dim3(1), 0, s, sc, (int)SC_EPS, eps);
    VEC_LAUNCH(p, set_scalar, dim3(1), dim3(1), 0, s, sc, (int)SC_ITER, 0.0);
    if (prm->gamma > 0) {
        VEC_LAUNCH(p, set_scalar, dim3(1), dim3(1), 0, s, sc, (int)SC_GAMMA, prm->gamma);
    } else {
        gamma_run<R>(p, w.ysort.ptr, 0, prm->beta, s, (int)SC_GAMMA, prior);
    }
    if (prm->resume) {
        RIOP_REQUIRE(x0 && prm->z1 && prm->z2 && prm->z3 && prm->rhs, RIOP_EINVAL,
                     "resume needs x, z1, z2, z3 and rhs");
        RIOP_HIP(hipMemcpyAsync(xh, x0, cb * N, hipMemcpyDeviceToDevice, s));
        RIOP_HIP(hipMemcpyAsync(w.z1loc.ptr, prm->z1, cb * D, hipMemcpyDeviceToDevice, s));
        RIOP_HIP(hipMemcpyAsync(w.z3loc.ptr, prm->z3, cb * N, hipMemcpyDeviceToDevice, s));
        RIOP_HIP(hipMemcpyAsync(w.rhs.ptr, prm->rhs, cb * N, hipMemcpyDeviceToDevice, s));
        if (M > 0)
            VEC_LAUNCH(p, gather_perm<R>, RB(), RT(), 0, s, static_cast<const C<R> *>(prm->z2),
                       p->perm.as<int>(), w.z2loc.as<C<R>>(), M);
        VEC_LAUNCH(p, set_scalar, dim3(1), dim3(1), 0, s, sc, (int)SC_F1PREV, prm->f1_prev);
        // rhs <- b - Phi^dagger Phi xhat
        phi_into_s2<R>(p, xh, s);
        phi_adj_sorted<R>(p, w.s2.ptr, w.tmpN.ptr, s);
        VEC_LAUNCH(p, lin2<R>, RB(), RT(), 0, s, (const C<R> *)w.rhs.as<C<R>>(), (const C<R> *)w.tmpN.as<C<R>>(),
                   R(-1), w.rhs.as<C<R>>(), N);
    } else {
        // z_i = 0, r_i = L_i x0, x_i = L_i^dagger r_i.
        launch_fill_zero<R>(w.z1loc.ptr, D, s);
        launch_fill_zero<R>(w.z2loc.ptr, std::max<long>(1, M), s);
        launch_fill_zero<R>(w.z3loc.ptr, N, s);
        if (x0) {
            RIOP_HIP(hipMemcpyAsync(xh, x0, cb * N, hipMemcpyDeviceToDevice, s));
            if (prior == PRIOR_TV) {  // L1 = I: x1 = x0
                RIOP_HIP(hipMemcpyAsync(w.x1.ptr, x0, cb * N, hipMemcpyDeviceToDevice, s));
            } else {
                launch_psi_adj<R>(p, xh, w.w1.ptr, s);
                launch_psi<R>(p, w.w1.ptr, w.x1.ptr, s);
            }
            // x2 = Phi^dagger Phi x0 cancels against the warm start: rhs = x1 + x0.
            phi_into_s2<R>(p, xh, s);
            VEC_LAUNCH(p, lin2<R>, RB(), RT(), 0, s, (const C<R> *)w.x1.as<C<R>>(), (const C<R> *)xh, R(1),
                       w.rhs.as<C<R>>(), N);
        } else {
            launch_fill_zero<R>(xh, N, s);
            launch_fill_zero<R>(w.rhs.ptr, N, s);
            launch_fill_zero<R>(w.s2.ptr, std::max<long>(1, M), s);  // Phi 0 (for the exported b)
        }
        VEC_LAUNCH(p, set_scalar, dim3(1), dim3(1), 0, s, sc, (int)SC_F1PREV, 0.0);
    }
    RIOP_HIP(hipGetLastError());
    w.initialised = true;
}

// Enqueue `iters` iterations of Algorithm 1 (steps 5-9 and the halting
// quantities).  No host synchronisation and no allocation: safe to capture
// in a HIP graph and to replay.
template <typename R> static void sdmm_step(riop_plan *p, int iters, hipStream_t s) {
    SdmmWork &w = p->sd;
    RIOP_REQUIRE(w.initialised, RIOP_EINVAL, "SDMM state not initialised");
    const long N = (long)p->n * p->n, M = (long)p->M;
    double *part = w.partials.as<double>();
    double *sc = w.scalars.as<double>();
    C<R> *xh = w.xhat.as<C<R>>();
    Prox1<R> px{w.z1loc.as<C<R>>(), w.w1.as<C<R>>(), static_cast<const R *>(w.weights), sc + SC_GAMMA,
                w.f1part.as<double>()};
    for (int t = 0; t < iters; ++t) {
        // Step 5: x = Q^{-1} sum_i x_i by CG, warm-started from the previous x
        // (rhs holds the sum less Phi^dagger Phi x).
        int rr_slot = SLOT_RR0;
        cg_run<R>(p, w.rhs.ptr, xh, w.n_cg, w.cg_tol, &rr_slot, s, plan_cg_work<R>(p), true);
        if (w.prior == PRIOR_TV) {
            // Steps 7-9, i = 1 with L1 = I: r1 = prox of gamma ||W grad .||_1 at
            // xhat + z1 by fast gradient projection on the dual; x1 = r1 - z1.
            const long N = (long)p->n * p->n;
            const int n = p->n;
            const R *tw = static_cast<const R *>(w.weights);
            VEC_LAUNCH(p, tv_begin<R>, RB(), RT(), 0, s, (const C<R> *)xh, (const C<R> *)w.z1loc.as<C<R>>(),
                       w.tvb.as<C<R>>(), w.tvp.as<C<R>>(), w.tvq.as<C<R>>(), w.tvr.as<C<R>>(), w.tvs.as<C<R>>(), N);
            double tk = 1.0;
            for (int k = 0; k < w.tv_inner; ++k) {
                const double tn = (1.0 + std::sqrt(1.0 + 4.0 * tk * tk)) / 2.0;
                VEC_LAUNCH(p, tv_u<R>, RB(), RT(), 0, s, (const C<R> *)w.tvb.as<C<R>>(),
                           (const C<R> *)w.tvr.as<C<R>>(), (const C<R> *)w.tvs.as<C<R>>(), w.tvu.as<C<R>>(), n,
                           (const double *)(sc + SC_GAMMA));
                VEC_LAUNCH(p, tv_dual<R>, RB(), RT(), 0, s, (const C<R> *)w.tvu.as<C<R>>(), tw, w.tvp.as<C<R>>(),
                           w.tvq.as<C<R>>(), w.tvr.as<C<R>>(), w.tvs.as<C<R>>(), n, (const double *)(sc + SC_GAMMA),
                           (tk - 1.0) / tn);
                tk = tn;
            }
            VEC_LAUNCH(p, tv_finish<R>, RB(), RT(), 0, s, (const C<R> *)w.tvb.as<C<R>>(),
                       (const C<R> *)w.tvp.as<C<R>>(), (const C<R> *)w.tvq.as<C<R>>(), w.z1loc.as<C<R>>(),
                       w.x1.as<C<R>>(), n, (const double *)(sc + SC_GAMMA));
            VEC_LAUNCH(p, tv_norm_partials<R>, RB(), RT(), 0, s, (const C<R> *)xh, tw, n, part);
        } else {
            // Steps 7-9, i = 1: soft threshold fused into Psi^dagger; x1 = Psi (r1 - z1).
            launch_psi_adj_prox<R>(p, xh, px, s);
            launch_psi<R>(p, w.w1.ptr, w.x1.ptr, s);
        }
        // i = 2: projection onto the l2 ball around y; x2 = Phi^dagger (r2 - z2),
        // taken as Phi^dagger (r2 - z2 - Phi xhat) for the next warm start.
        phi_into_s2<R>(p, xh, s);
        if (w.nblocks == 0) {
            VEC_LAUNCH(p, prox2_norms<R>, RB(), RT(), 0, s, w.s2.as<C<R>>(), w.z2loc.as<C<R>>(),
                       w.ysort.as<C<R>>(), M, part);
            VEC_LAUNCH(p, prox2_scale, dim3(1), RT(), 0, s, (const double *)part, sc);
            launch_grid_prox2<R>(p, w.s2.ptr, w.z2loc.ptr, w.ysort.ptr, sc + SC_P2SCALE, s);
        } else {
            // Block SDMM (Sec. 4.5): one ball per data block; steps 7-9 of
            // every block i + 2 at once, sum_i Phi_i^dagger (r_i - z_i) as one
            // Phi^dagger of the concatenated values.
            const int nb = w.nblocks;
            VEC_LAUNCH(p, prox2_norms_blocks<R>, RB(), RT(), sizeof(double) * 2 * nb, s,
                       (const C<R> *)w.s2.as<C<R>>(), (const C<R> *)w.z2loc.as<C<R>>(),
                       (const C<R> *)w.ysort.as<C<R>>(), (const int *)w.blk.as<int>(), M, nb, w.bpart.as<double>());
            VEC_LAUNCH(p, block_scales, dim3(1), RT(), 0, s, (const double *)w.bpart.as<double>(), nb,
                       (const double *)w.beps.as<double>(), w.bscale.as<double>(), w.bnu.as<double>(), part);
            VEC_LAUNCH(p, prox2_apply_blocks<R>, RB(), RT(), 0, s, (const C<R> *)w.s2.as<C<R>>(),
                       w.z2loc.as<C<R>>(), (const C<R> *)w.ysort.as<C<R>>(), (const int *)w.blk.as<int>(),
                       (const double *)w.bscale.as<double>(), p->vis.as<C<R>>(), M);
            launch_grid<R>(p, p->vis.ptr, 0, s);
        }
        launch_phi_fft_adjoint<R>(p, w.tmpN.ptr, s);
        // i = 3 and the next right-hand side.
        VEC_LAUNCH(p, prox3_rhs<R>, RB(), RT(), 0, s, (const C<R> *)xh, w.z3loc.as<C<R>>(), w.x1.as<C<R>>(),
                   w.tmpN.as<C<R>>(), w.rhs.as<C<R>>(), N);
        if (w.prior != PRIOR_TV)
            VEC_LAUNCH(p, f1_partials, RB(), RT(), 0, s, (const double *)w.f1part.as<double>(), w.f1_count, part);
        VEC_LAUNCH(p, record_stats, dim3(1), RT(), 0, s, (const double *)part, sc, w.history.as<double>(),
                   w.hist_cap, rr_slot);
        RIOP_HIP(hipGetLastError());
    }
}

// Copy the state out, read the statistics (synchronises).  stop_iter: the
// iteration at which early stopping ended the run (0: none).
template <typename R>
static void sdmm_finish(riop_plan *p, const riop_sdmm_params *prm, void *x_out, riop_sdmm_stats *stats,
                        double *history, hipStream_t s, int stop_iter = 0) {
    SdmmWork &w = p->sd;
    RIOP_REQUIRE(w.initialised, RIOP_EINVAL, "SDMM state not initialised");
    const long N = (long)p->n * p->n, D = (long)p->q * N, M = (long)p->M;
    const size_t cb = cbytes(p);
    double *sc = w.scalars.as<double>();
    if (x_out) RIOP_HIP(hipMemcpyAsync(x_out, w.xhat.ptr, cb * N, hipMemcpyDeviceToDevice, s));
    const long D1 = w.prior == PRIOR_TV ? N : D;  // the l1 term's dual: q N (SARA) or N (TV)
    if (prm && prm->z1) RIOP_HIP(hipMemcpyAsync(prm->z1, w.z1loc.ptr, cb * D1, hipMemcpyDeviceToDevice, s));
    if (prm && prm->z3) RIOP_HIP(hipMemcpyAsync(prm->z3, w.z3loc.ptr, cb * N, hipMemcpyDeviceToDevice, s));
    if (prm && prm->rhs) {  // b = rhs + Phi^dagger Phi xhat
        phi_adj_sorted<R>(p, w.s2.ptr, w.tmpN.ptr, s);
        VEC_LAUNCH(p, lin2<R>, RB(), RT(), 0, s, (const C<R> *)w.rhs.as<C<R>>(), (const C<R> *)w.tmpN.as<C<R>>(),
                   R(1), static_cast<C<R> *>(prm->rhs), N);
    }
    if (prm && prm->z2 && M > 0)
        VEC_LAUNCH(p, scatter_perm<R>, RB(), RT(), 0, s, (const C<R> *)w.z2loc.as<C<R>>(), p->perm.as<int>(),
                   static_cast<C<R> *>(prm->z2), M);
    double scal[kScalars] = {};
    RIOP_HIP(hipMemcpyAsync(scal, sc, sizeof(scal), hipMemcpyDeviceToHost, s));
    RIOP_HIP(hipStreamSynchronize(s));
    mark_done(p, s);
    const int iters = (int)scal[SC_ITER];
    const int kept = std::min(iters, w.hist_cap);
    const int K = kHistStride;
    std::vector<double> hist(K * (size_t)std::max(1, kept), 0.0);
    if (kept > 0) {
        RIOP_HIP(hipMemcpyAsync(hist.data(), w.history.ptr, sizeof(double) * K * kept, hipMemcpyDeviceToHost, s));
        RIOP_HIP(hipStreamSynchronize(s));
    }
    if (history) std::copy(hist.begin(), hist.begin() + (size_t)K * kept, history);
    int bad = 0;  // first iteration (1-based) whose f1 or nu is not finite
    for (int t = 0; t < kept && !bad; ++t)
        if (!std::isfinite(hist[(size_t)K * t]) || !std::isfinite(hist[(size_t)K * t + 2])) bad = t + 1;
    if (stats) {
        stats->iters = iters;
        stats->gamma = scal[SC_GAMMA];
        stats->f1 = kept ? hist[(size_t)K * (kept - 1)] : 0.0;
        stats->zeta = kept ? hist[(size_t)K * (kept - 1) + 1] : INFINITY;
        stats->nu = kept ? hist[(size_t)K * (kept - 1) + 2] : 0.0;
        stats->cg_iters = kept ? (int32_t)hist[(size_t)K * (kept - 1) + 4] : 0;
        stats->status_iter = bad ? bad : stop_iter;
    }
    report_nonfinite(p, s);
    if (bad) throw Error{RIOP_ENONFINITE, "non-finite value reached a norm in SDMM (see stats.status_iter)"};
}

template <typename R>
static void sdmm_run(riop_plan *p, const void *y, double eps, const riop_sdmm_params *prm, void *x_inout,
                     riop_sdmm_stats *stats, hipStream_t s, int prior = PRIOR_SARA, int tv_inner = 0) {
    sdmm_init<R>(p, y, eps, prm, x_inout, s, prior, tv_inner);
    // Inputs holding NaN or Inf end the call before any iteration.
    try {
        report_nonfinite(p, s);
    } catch (const Error &) {
        if (stats) {
            *stats = riop_sdmm_stats{};
            stats->zeta = INFINITY;
        }
        throw;
    }
    const int T = std::max(0, prm->T);
    int stop_iter = 0;
    if (!prm->early_stop) {
        sdmm_step<R>(p, T, s);
    } else {
        double h[kHistStride];
        for (int t = 0; t < T; ++t) {
            sdmm_step<R>(p, 1, s);
            RIOP_HIP(hipMemcpyAsync(h, p->sd.history.as<double>() + (size_t)kHistStride * t, sizeof h,
                                    hipMemcpyDeviceToHost, s));
            RIOP_HIP(hipStreamSynchronize(s));
            if (!std::isfinite(h[0]) || !std::isfinite(h[2])) break;  // reported by sdmm_finish
            // Halting rule (Sec. 4.4): relative change of f1 below xi and the
            // data residual within [1 - tau, 1 + tau] of eps.
            if (h[1] < prm->xi && h[2] >= 1.0 - prm->tau && h[2] <= 1.0 + prm->tau) {
                stop_iter = t + 1;
                break;
            }
        }
    }
    sdmm_finish<R>(p, prm, x_inout, stats, prm->history, s, stop_iter);
}

// Block SDMM (Sec. 4.5, eqs. blocks, dbp1, dbp2): Algorithm 1 with S = R + 2.
// Q and the l1 and positivity steps are those of the plain run; the data
// term is one l2 ball per block.
template <typename R>
static void sdmm_blocks_run(riop_plan *p, const void *y, int nb, const int32_t *block_of, const double *eps,
                            const riop_sdmm_params *prm, void *x_inout, riop_sdmm_stats *stats, double *nu_out,
                            hipStream_t s) {
    ensure_work(p);
    SdmmWork &w = p->sd;
    const long M = (long)p->M;
    w.blk.reserve(sizeof(int) * (size_t)std::max<long>(1, M));
    w.beps.reserve(sizeof(double) * kMaxBlocks);
    w.bscale.reserve(sizeof(double) * kMaxBlocks);
    w.bnu.reserve(sizeof(double) * kMaxBlocks);
    w.bpart.reserve(sizeof(double) * 2 * (size_t)kMaxBlocks * kRedBlocks);
    w.bflag.reserve(sizeof(int));
    RIOP_HIP(hipMemsetAsync(w.bflag.ptr, 0, sizeof(int), s));
    if (M > 0)
        VEC_LAUNCH(p, gather_blocks, RB(), RT(), 0, s, (const int *)block_of, (const int *)p->perm.as<int>(), M, nb,
                   w.blk.as<int>(), w.bflag.as<int>());
    RIOP_HIP(hipMemcpyAsync(w.beps.ptr, eps, sizeof(double) * nb, hipMemcpyHostToDevice, s));
    int bad = 0;
    RIOP_HIP(hipMemcpyAsync(&bad, w.bflag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    RIOP_HIP(hipStreamSynchronize(s));
    RIOP_REQUIRE(!bad, RIOP_EINVAL, "block_of holds a block index outside [0, nblocks)");
    // eps enters through the blocks; the history's nu is already the largest
    // per-block ratio, so the state's eps slot holds 1.
    sdmm_init<R>(p, y, 1.0, prm, x_inout, s);
    w.nblocks = nb;
    ++w.epoch;
    report_nonfinite(p, s);
    const int T = std::max(0, prm->T);
    int stop_iter = 0;
    if (!prm->early_stop) {
        sdmm_step<R>(p, T, s);
    } else {
        double h[kHistStride];
        for (int t = 0; t < T; ++t) {
            sdmm_step<R>(p, 1, s);
            RIOP_HIP(hipMemcpyAsync(h, w.history.as<double>() + (size_t)kHistStride * t, sizeof h,
                                    hipMemcpyDeviceToHost, s));
            RIOP_HIP(hipStreamSynchronize(s));
            if (!std::isfinite(h[0]) || !std::isfinite(h[2])) break;
            if (h[1] < prm->xi && h[2] >= 1.0 - prm->tau && h[2] <= 1.0 + prm->tau) {
                stop_iter = t + 1;
                break;
            }
        }
    }
    if (nu_out) RIOP_HIP(hipMemcpyAsync(nu_out, w.bnu.ptr, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    sdmm_finish<R>(p, prm, x_inout, stats, prm->history, s, stop_iter);
}

// Sum of one partial-sum slot, read back to the host (synchronises).
static double slot_to_host(riop_plan *p, int slot, hipStream_t s) {
    VEC_LAUNCH(p, slot_to_scalar, dim3(1), RT(), 0, s, (const double *)p->sd.partials.as<double>(), slot,
               p->sd.scalars.as<double>(), (int)SC_RRFINAL);
    RIOP_HIP(hipGetLastError());
    double v = 0;
    RIOP_HIP(hipMemcpyAsync(&v, p->sd.scalars.as<double>() + SC_RRFINAL, sizeof v, hipMemcpyDeviceToHost, s));
    RIOP_HIP(hipStreamSynchronize(s));
    return v;
}

// Reweighted l1 (Sec. 3.3, the sequence of weighted problems of eq. delta):
// pass 0 with W = I, then up to rw->outer passes with
// w = delta / (delta + |Psi^dagger x_prev|), each a fresh run of Algorithm 1
// from the previous solution with the first pass's penalty.
template <typename R>
static void reweighted_run(riop_plan *p, const void *y, double eps, const riop_sdmm_params *inner,
                           const riop_reweight_params *rw, void *x, void *weights_out, riop_sdmm_stats *stats,
                           int32_t *passes_out, hipStream_t s, int prior = PRIOR_SARA, int tv_inner = 0) {
    ensure_work(p);
    SdmmWork &w = p->sd;
    const long N = (long)p->n * p->n;
    const long D = prior == PRIOR_TV ? N : (long)p->q * N;  // one weight per coefficient or per pixel
    const size_t cb = cbytes(p);
    w.rw_w.reserve(rbytes(p) * (size_t)D);
    w.xprev.reserve(cb * (size_t)N);
    riop_sdmm_params prm = *inner;
    prm.weights = nullptr;
    prm.resume = 0;
    prm.z1 = prm.z2 = prm.z3 = prm.rhs = nullptr;
    prm.history = nullptr;
    riop_sdmm_stats st{};
    double *part = w.partials.as<double>();
    sdmm_run<R>(p, y, eps, &prm, x, &st, s, prior, tv_inner);
    prm.gamma = st.gamma;
    int passes = 1;
    double delta = 0.0;
    for (int k = 0; k < rw->outer; ++k) {
        // Weights from the current solution's coefficients (SARA) or gradient
        // magnitudes (TV); delta_1 defaults to the RMS of the same quantity.
        if (prior == PRIOR_TV) {
            if (k == 0 && rw->delta0 <= 0) {
                VEC_LAUNCH(p, tv_sum_mag2<R>, RB(), RT(), 0, s, (const C<R> *)x, p->n, part, (int)SLOT_MAX);
                const double ms = slot_to_host(p, SLOT_MAX, s) / (double)D;
                delta = ms > 0 ? std::sqrt(ms) : 1.0;
            } else {
                delta = k == 0 ? rw->delta0 : std::max(rw->rho * delta, rw->delta_min);
            }
            VEC_LAUNCH(p, tv_reweight<R>, RB(), RT(), 0, s, (const C<R> *)x, w.rw_w.as<R>(), p->n, delta);
        } else {
            launch_psi_adj<R>(p, x, w.w1.ptr, s);
            if (k == 0) {
                if (rw->delta0 > 0) {
                    delta = rw->delta0;
                } else {
                    VEC_LAUNCH(p, sum_abs2<R>, RB(), RT(), 0, s, (const C<R> *)w.w1.as<C<R>>(), D, part,
                               (int)SLOT_MAX);
                    const double ms = slot_to_host(p, SLOT_MAX, s) / (double)D;
                    delta = ms > 0 ? std::sqrt(ms) : 1.0;
                }
            } else {
                delta = std::max(rw->rho * delta, rw->delta_min);
            }
            VEC_LAUNCH(p, reweight_weights<R>, RB(), RT(), 0, s, (const C<R> *)w.w1.as<C<R>>(), w.rw_w.as<R>(),
                       D, delta);
        }
        RIOP_HIP(hipMemcpyAsync(w.xprev.ptr, x, cb * N, hipMemcpyDeviceToDevice, s));
        prm.weights = w.rw_w.ptr;
        sdmm_run<R>(p, y, eps, &prm, x, &st, s, prior, tv_inner);
        ++passes;
        if (rw->tol > 0) {
            VEC_LAUNCH(p, diff_norms<R>, RB(), RT(), 0, s, (const C<R> *)x, (const C<R> *)w.xprev.as<C<R>>(), N,
                       part, (int)SLOT_E, (int)SLOT_NU);
            const double d2 = slot_to_host(p, SLOT_E, s), x2 = slot_to_host(p, SLOT_NU, s);
            const double change = x2 > 0 ? std::sqrt(d2 / x2) : 0.0;
            if (change <= rw->tol) break;
        }
    }
    if (weights_out) {
        if (passes == 1) {  // only the unweighted pass ran: W = I
            VEC_LAUNCH(p, fill_real<R>, RB(), RT(), 0, s, static_cast<R *>(weights_out), D, R(1));
        } else {
            RIOP_HIP(hipMemcpyAsync(weights_out, w.rw_w.ptr, rbytes(p) * (size_t)D, hipMemcpyDeviceToDevice, s));
        }
    }
    RIOP_HIP(hipStreamSynchronize(s));
    mark_done(p, s);
    if (stats) *stats = st;
    if (passes_out) *passes_out = passes;
}

template <typename R> static void apply_q_run(riop_plan *p, const void *x, void *out, hipStream_t s) {
    const long N = (long)p->n * p->n;
    ensure_work(p);
    check_finite_input(p, x, 2 * N, s);
    gram_sorted<R>(p, x, p->sd.tmpN.ptr, s);
    VEC_LAUNCH(p, add_2x<R>, RB(), RT(), 0, s, p->sd.tmpN.as<C<R>>(), static_cast<const C<R> *>(x),
                       static_cast<C<R> *>(out), N);
    RIOP_HIP(hipGetLastError());
}

// CG with its workspace in `w`; reads back the final <r, r> and the
// iteration count when asked (synchronises then).
template <typename R>
static void cg_with(riop_plan *p, const void *b, void *x, int n_iter, double tol, double *rr_out, int32_t *iters_out,
                    hipStream_t s, const CgWork<R> &w) {
    const long N = (long)p->n * p->n;
    check_finite_input(p, b, 2 * N, s);
    check_finite_input(p, x, 2 * N, s);
    int slot = SLOT_RR0;
    cg_run<R>(p, b, x, n_iter, tol, &slot, s, w);
    if (rr_out || iters_out) {
        VEC_LAUNCH(p, slot_to_scalar, dim3(1), RT(), 0, s, (const double *)w.partials, slot, w.scalars,
                   (int)SC_RRFINAL);
        RIOP_HIP(hipGetLastError());
        double sc[kScalars];
        RIOP_HIP(hipMemcpyAsync(sc, w.scalars, sizeof sc, hipMemcpyDeviceToHost, s));
        report_nonfinite(p, s);
        if (rr_out) *rr_out = sc[SC_RRFINAL];
        if (iters_out) *iters_out = n_iter > 0 ? (int32_t)sc[SC_CGIT] : 0;
    }
    mark_done(p, s);
}

template <typename R> static void cg_entry(riop_plan *p, const void *b, void *x, int n_iter, double tol,
                                           double *rr_out, int32_t *iters_out, hipStream_t s) {
    ensure_work(p);
    cg_with<R>(p, b, x, n_iter, tol, rr_out, iters_out, s, plan_cg_work<R>(p));
}

// ---------------------------------------------------------------------------
// Allocation-free CG: the workspace lives in a static device array, one copy
// per device the library runs on (held until the process ends).  Its device
// address is taken once per device with hipGetSymbolAddress; host code never
// uses the array's name as an address.

constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device (set up on first use).
static void *scratch_on_current_device() {
    int dev = -1;
    RIOP_HIP(hipGetDevice(&dev));
    RIOP_REQUIRE(dev >= 0 && dev < kMaxDevices, RIOP_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        RIOP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        RIOP_REQUIRE(ptr, RIOP_EDEVICE, "scratch symbol has no device address");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of scratch a plan's CG needs: partial-sum and scalar slots, then
// r, p, Q p.
static size_t cg_scratch_bytes(const riop_plan *p) {
    const size_t vec = align256(cbytes(p) * (size_t)p->n * p->n);
    return align256(sizeof(double) * kSlots * kRedBlocks) + align256(sizeof(double) * kScalars) + 3 * vec;
}

template <typename R>
static void cg_noalloc_entry(riop_plan *p, const void *b, void *x, int n_iter, double tol, double *rr_out,
                             int32_t *iters_out, hipStream_t s) {
    const size_t need = cg_scratch_bytes(p);
    if (need > kScratchBytes)
        throw Error{RIOP_ENOTSUP, "riop_cg_noalloc: the plan's CG workspace needs " + std::to_string(need) +
                                      " bytes, more than the " + std::to_string(kScratchBytes) +
                                      "-byte static scratch (use riop_cg)"};
    unsigned char *base = static_cast<unsigned char *>(scratch_on_current_device());
    const size_t vec = align256(cbytes(p) * (size_t)p->n * p->n);
    CgWork<R> w;
    w.partials = reinterpret_cast<double *>(base);
    base += align256(sizeof(double) * kSlots * kRedBlocks);
    w.scalars = reinterpret_cast<double *>(base);
    base += align256(sizeof(double) * kScalars);
    w.r = reinterpret_cast<C<R> *>(base);
    w.p = reinterpret_cast<C<R> *>(base + vec);
    w.qp = reinterpret_cast<C<R> *>(base + 2 * vec);
    // Every slot CG reads is written earlier in the same call (cg_init and the
    // first update set the residual norms, the iteration count and the
    // reference norm), so nothing from an earlier call is read.
    cg_with<R>(p, b, x, n_iter, tol, rr_out, iters_out, s, w);
}

template <typename R> static void gamma_entry(riop_plan *p, const void *y, double beta, double *g, hipStream_t s) {
    ensure_work(p);
    check_finite_input(p, y, 2 * p->M, s);
    gamma_run<R>(p, y, 1, beta, s, (int)SC_GAMMA_Q);
    RIOP_HIP(hipMemcpyAsync(g, p->sd.scalars.as<double>() + SC_GAMMA_Q, sizeof(double), hipMemcpyDeviceToHost, s));
    report_nonfinite(p, s);
    mark_done(p, s);
}

}  // namespace riop

using namespace riop;

template <typename F> static riop_status guarded2(F &&f) {
    try {
        clear_error();
        f();
        return RIOP_OK;
    } catch (const Error &e) {
        set_error("%s", e.msg.c_str());
        return e.status;
    } catch (...) {
        set_error("unexpected failure");
        return RIOP_EDEVICE;
    }
}

static void check_plan2(const riop_plan *p) {
    RIOP_REQUIRE(p, RIOP_EINVAL, "plan is NULL");
    int dev = -1;
    RIOP_HIP(hipGetDevice(&dev));
    RIOP_REQUIRE(dev == p->device, RIOP_EINVAL, "plan belongs to another device than the current one");
}

extern "C" {

riop_status riop_apply_q(riop_plan *p, const void *x, void *out, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(x && out && x != out, RIOP_EINVAL, "x and out must be distinct non-NULL pointers");
        if (p->prec == RIOP_F64)
            apply_q_run<double>(p, x, out, static_cast<hipStream_t>(stream));
        else
            apply_q_run<float>(p, x, out, static_cast<hipStream_t>(stream));
        mark_done(p, static_cast<hipStream_t>(stream));
    });
}

riop_status riop_cg(riop_plan *p, const void *b, void *x, int32_t n_iter, double tol, double *rr_out,
                    int32_t *iters_out, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(b && x && b != x, RIOP_EINVAL, "b and x must be distinct non-NULL pointers");
        RIOP_REQUIRE(n_iter >= 0, RIOP_EINVAL, "n_iter must be >= 0");
        RIOP_REQUIRE(tol >= 0 && std::isfinite(tol), RIOP_EINVAL, "tol must be finite and >= 0");
        if (p->prec == RIOP_F64)
            cg_entry<double>(p, b, x, n_iter, tol, rr_out, iters_out, static_cast<hipStream_t>(stream));
        else
            cg_entry<float>(p, b, x, n_iter, tol, rr_out, iters_out, static_cast<hipStream_t>(stream));
    });
}

riop_status riop_cg_noalloc(riop_plan *p, const void *b, void *x, int32_t n_iter, double tol, double *rr_out,
                            int32_t *iters_out, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(b && x && b != x, RIOP_EINVAL, "b and x must be distinct non-NULL pointers");
        RIOP_REQUIRE(n_iter >= 0, RIOP_EINVAL, "n_iter must be >= 0");
        RIOP_REQUIRE(tol >= 0 && std::isfinite(tol), RIOP_EINVAL, "tol must be finite and >= 0");
        if (p->prec == RIOP_F64)
            cg_noalloc_entry<double>(p, b, x, n_iter, tol, rr_out, iters_out, static_cast<hipStream_t>(stream));
        else
            cg_noalloc_entry<float>(p, b, x, n_iter, tol, rr_out, iters_out, static_cast<hipStream_t>(stream));
    });
}

riop_status riop_gamma(riop_plan *p, const void *y, double beta, double *gamma, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(gamma && (y || p->M == 0), RIOP_EINVAL, "NULL argument");
        if (p->prec == RIOP_F64)
            gamma_entry<double>(p, y, beta, gamma, static_cast<hipStream_t>(stream));
        else
            gamma_entry<float>(p, y, beta, gamma, static_cast<hipStream_t>(stream));
    });
}

riop_status riop_sdmm(riop_plan *p, const void *y, double eps, const riop_sdmm_params *prm, void *x_inout,
                      riop_sdmm_stats *stats, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(prm, RIOP_EINVAL, "params is NULL");
        RIOP_REQUIRE(y || p->M == 0, RIOP_EINVAL, "y is NULL");
        RIOP_REQUIRE(eps > 0 && std::isfinite(eps), RIOP_EINVAL, "eps must be positive and finite");
        RIOP_REQUIRE(prm->T >= 0 && prm->n_cg >= 0, RIOP_EINVAL, "T and n_cg must be >= 0");
        RIOP_REQUIRE(prm->gamma > 0 || prm->beta > 0, RIOP_EINVAL, "need gamma > 0 or beta > 0");
        RIOP_REQUIRE(prm->cg_tol >= 0 && std::isfinite(prm->cg_tol), RIOP_EINVAL, "cg_tol must be finite and >= 0");
        if (p->prec == RIOP_F64)
            sdmm_run<double>(p, y, eps, prm, x_inout, stats, static_cast<hipStream_t>(stream));
        else
            sdmm_run<float>(p, y, eps, prm, x_inout, stats, static_cast<hipStream_t>(stream));
    });
}

riop_status riop_sdmm_tv(riop_plan *p, const void *y, double eps, const riop_sdmm_params *prm, int32_t n_inner,
                         const riop_reweight_params *rw, void *x_inout, void *weights_out, riop_sdmm_stats *stats,
                         int32_t *passes, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(prm, RIOP_EINVAL, "params is NULL");
        RIOP_REQUIRE(y || p->M == 0, RIOP_EINVAL, "y is NULL");
        RIOP_REQUIRE(eps > 0 && std::isfinite(eps), RIOP_EINVAL, "eps must be positive and finite");
        RIOP_REQUIRE(prm->T >= 0 && prm->n_cg >= 0 && n_inner >= 0, RIOP_EINVAL, "T, n_cg and n_inner must be >= 0");
        RIOP_REQUIRE(prm->gamma > 0 || prm->beta > 0, RIOP_EINVAL, "need gamma > 0 or beta > 0");
        RIOP_REQUIRE(prm->cg_tol >= 0 && std::isfinite(prm->cg_tol), RIOP_EINVAL, "cg_tol must be finite and >= 0");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        if (rw) {
            RIOP_REQUIRE(x_inout, RIOP_EINVAL, "a reweighted run needs x_inout");
            RIOP_REQUIRE(!prm->weights && !prm->resume && !prm->z1 && !prm->z2 && !prm->z3 && !prm->rhs &&
                             !prm->history,
                         RIOP_EINVAL, "the reweighted run owns the weights and state: weights, resume, state and "
                                      "history pointers must be zero");
            RIOP_REQUIRE(rw->outer >= 0 && rw->rho > 0 && rw->rho <= 1 && rw->delta_min >= 0 && rw->tol >= 0 &&
                             std::isfinite(rw->delta0) && std::isfinite(rw->delta_min) && std::isfinite(rw->tol),
                         RIOP_EINVAL, "reweighting: outer >= 0, 0 < rho <= 1, delta_min >= 0, tol >= 0, finite delta0");
            if (p->prec == RIOP_F64)
                reweighted_run<double>(p, y, eps, prm, rw, x_inout, weights_out, stats, passes, st, PRIOR_TV, n_inner);
            else
                reweighted_run<float>(p, y, eps, prm, rw, x_inout, weights_out, stats, passes, st, PRIOR_TV, n_inner);
        } else {
            RIOP_REQUIRE(!weights_out, RIOP_EINVAL, "weights_out is for reweighted runs");
            if (p->prec == RIOP_F64)
                sdmm_run<double>(p, y, eps, prm, x_inout, stats, st, PRIOR_TV, n_inner);
            else
                sdmm_run<float>(p, y, eps, prm, x_inout, stats, st, PRIOR_TV, n_inner);
            if (passes) *passes = 1;
        }
    });
}

riop_status riop_sdmm_blocks(riop_plan *p, const void *y, int32_t nblocks, const int32_t *block_of, const double *eps,
                             const riop_sdmm_params *prm, void *x_inout, riop_sdmm_stats *stats, double *nu_out,
                             void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(prm && eps, RIOP_EINVAL, "params and eps are required");
        RIOP_REQUIRE(nblocks >= 1 && nblocks <= kMaxBlocks, RIOP_EINVAL, "nblocks must be in [1, 1024]");
        RIOP_REQUIRE((y && block_of) || p->M == 0, RIOP_EINVAL, "y and block_of are required");
        for (int b = 0; b < nblocks; ++b)
            RIOP_REQUIRE(eps[b] > 0 && std::isfinite(eps[b]), RIOP_EINVAL, "every eps must be positive and finite");
        RIOP_REQUIRE(prm->T >= 0 && prm->n_cg >= 0, RIOP_EINVAL, "T and n_cg must be >= 0");
        RIOP_REQUIRE(prm->gamma > 0 || prm->beta > 0, RIOP_EINVAL, "need gamma > 0 or beta > 0");
        RIOP_REQUIRE(prm->cg_tol >= 0 && std::isfinite(prm->cg_tol), RIOP_EINVAL, "cg_tol must be finite and >= 0");
        RIOP_REQUIRE(!prm->resume, RIOP_ENOTSUP, "block SDMM starts from x^(0); resume is not supported");
        if (p->prec == RIOP_F64)
            sdmm_blocks_run<double>(p, y, nblocks, block_of, eps, prm, x_inout, stats, nu_out,
                                    static_cast<hipStream_t>(stream));
        else
            sdmm_blocks_run<float>(p, y, nblocks, block_of, eps, prm, x_inout, stats, nu_out,
                                   static_cast<hipStream_t>(stream));
    });
}

riop_status riop_sdmm_reweighted(riop_plan *p, const void *y, double eps, const riop_sdmm_params *prm,
                                 const riop_reweight_params *rw, void *x_inout, void *weights_out,
                                 riop_sdmm_stats *stats, int32_t *passes, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(prm && rw && x_inout, RIOP_EINVAL, "params, reweighting params and x_inout are required");
        RIOP_REQUIRE(y || p->M == 0, RIOP_EINVAL, "y is NULL");
        RIOP_REQUIRE(eps > 0 && std::isfinite(eps), RIOP_EINVAL, "eps must be positive and finite");
        RIOP_REQUIRE(prm->T >= 0 && prm->n_cg >= 0, RIOP_EINVAL, "T and n_cg must be >= 0");
        RIOP_REQUIRE(prm->gamma > 0 || prm->beta > 0, RIOP_EINVAL, "need gamma > 0 or beta > 0");
        RIOP_REQUIRE(prm->cg_tol >= 0 && std::isfinite(prm->cg_tol), RIOP_EINVAL, "cg_tol must be finite and >= 0");
        RIOP_REQUIRE(!prm->weights && !prm->resume && !prm->z1 && !prm->z2 && !prm->z3 && !prm->rhs && !prm->history,
                     RIOP_EINVAL, "the reweighted run owns the weights and state: weights, resume, state and history "
                                  "pointers must be zero");
        RIOP_REQUIRE(rw->outer >= 0 && rw->rho > 0 && rw->rho <= 1 && rw->delta_min >= 0 && rw->tol >= 0 &&
                         std::isfinite(rw->delta0) && std::isfinite(rw->delta_min) && std::isfinite(rw->tol),
                     RIOP_EINVAL, "reweighting: outer >= 0, 0 < rho <= 1, delta_min >= 0, tol >= 0, finite delta0");
        if (p->prec == RIOP_F64)
            reweighted_run<double>(p, y, eps, prm, rw, x_inout, weights_out, stats, passes,
                                   static_cast<hipStream_t>(stream));
        else
            reweighted_run<float>(p, y, eps, prm, rw, x_inout, weights_out, stats, passes,
                                  static_cast<hipStream_t>(stream));
    });
}

riop_status riop_sdmm_init(riop_plan *p, const void *y, double eps, const riop_sdmm_params *prm, const void *x0,
                           void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(prm, RIOP_EINVAL, "params is NULL");
        RIOP_REQUIRE(y || p->M == 0, RIOP_EINVAL, "y is NULL");
        RIOP_REQUIRE(eps > 0 && std::isfinite(eps), RIOP_EINVAL, "eps must be positive and finite");
        RIOP_REQUIRE(prm->T >= 0 && prm->n_cg >= 0, RIOP_EINVAL, "T and n_cg must be >= 0");
        RIOP_REQUIRE(prm->gamma > 0 || prm->beta > 0, RIOP_EINVAL, "need gamma > 0 or beta > 0");
        RIOP_REQUIRE(prm->cg_tol >= 0 && std::isfinite(prm->cg_tol), RIOP_EINVAL, "cg_tol must be finite and >= 0");
        if (p->prec == RIOP_F64)
            sdmm_init<double>(p, y, eps, prm, x0, static_cast<hipStream_t>(stream));
        else
            sdmm_init<float>(p, y, eps, prm, x0, static_cast<hipStream_t>(stream));
        mark_done(p, static_cast<hipStream_t>(stream));
    });
}

riop_status riop_sdmm_step(riop_plan *p, int32_t iterations, void *stream) {
    return guarded2([&] {
        check_plan2(p);
        RIOP_REQUIRE(iterations >= 0, RIOP_EINVAL, "iterations must be >= 0");
        if (p->prec == RIOP_F64)
            sdmm_step<double>(p, iterations, static_cast<hipStream_t>(stream));
        else
            sdmm_step<float>(p, iterations, static_cast<hipStream_t>(stream));
        mark_done(p, static_cast<hipStream_t>(stream));
    });
}

riop_status riop_sdmm_finish(riop_plan *p, const riop_sdmm_params *prm, void *x_out, riop_sdmm_stats *stats,
                             void *stream) {
    return guarded2([&] {
        check_plan2(p);
        double *hist = prm ? prm->history : nullptr;
        if (p->prec == RIOP_F64)
            sdmm_finish<double>(p, prm, x_out, stats, hist, static_cast<hipStream_t>(stream));
        else
            sdmm_finish<float>(p, prm, x_out, stats, hist, static_cast<hipStream_t>(stream));
    });
}

}  // extern "C"
