// SARA dictionary Psi = (1/sqrt q) [Dirac, Db1, ..., Db8] (Sec. 3.3) and its
// adjoint, as periodised orthonormal 2-D DWTs in the Mallat layout.
//
// Analysis, one launch per level for all selected Daubechies bases at once
// (the bases are independent and computed in parallel, as in Sec. 5): a
// workgroup owns a TO x TO tile of each of the four sub-bands, stages the
// (2 TO + Lf - 2)^2 input region (periodic) in LDS, filters rows then columns
// and writes LL to the next level's input (or the coefficient plane at the
// last level) and LH / HL / HH to their Mallat positions.
//
// The final coefficients can go through an epilogue instead of a plain store:
// the SDMM update of the l1 term (Algorithm 1 steps 7-9 for i = 1,
// soft threshold of eq. prox1), which also accumulates f1 = sum w |alpha|.
//
// Synthesis is the exact transpose, columns then rows; its last level sums all
// bases and the Dirac plane for one output tile, so Psi alpha is written once.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace riop {

constexpr int kMaxTaps = 16;
constexpr int kTO = 16;  // output tile side per sub-band (analysis) / half the output tile (synthesis)


template <typename R> struct AnaArgs {
    const C<R> *in;     // level input: x (level 1, shared) or per-basis LL slot
    long in_bstride;    // complex elements between bases' inputs (0 when shared)
    C<R> *ll_out;       // next-level LL slot (per basis) or nullptr at the last level
    long ll_bstride;
    C<R> *alpha;        // coefficient planes (q x n x n)
    const R *filt;      // [9][2][kMaxTaps] low / high pass
    int basis[8];       // Daubechies order of each launched basis
    int plane[8];       // plane index of each launched basis
    int n, s, TO, last;
    R scale;            // 1/sqrt(q) applied to final coefficients
    int prox;
    Prox1<R> px;
};

template <typename R>
__device__ inline void emit_coef(const AnaArgs<R> &a, long j, C<R> c, double &f1) {
    c = cscale<R>(c, a.scale);
    if (!a.prox) {
        a.alpha[j] = c;
        return;
    }
    const R w = a.px.weights ? a.px.weights[j] : R(1);
    const R lam = (R)(*a.px.gamma) * w;
    const C<R> z = a.px.z1[j];
    const C<R> v = cadd<R>(c, z);
    const R mag = sqrt(v.x * v.x + v.y * v.y);
    const R sc = mag > lam ? R(1) - lam / mag : R(0);
    const C<R> r = cscale<R>(v, sc);
    const C<R> zn = csub<R>(v, r);
    a.px.z1[j] = zn;
    a.px.w1[j] = csub<R>(r, zn);
    f1 += (double)w * sqrt((double)c.x * c.x + (double)c.y * c.y);
}

// Block sum of f1 into this block's own partial slot (no atomics; the
// consumer adds the slots in a fixed order).
template <typename R> __device__ inline void block_add_f1(double f1, double *part) {
    __shared__ double red[256];
    red[threadIdx.x] = f1;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Prox epilogue with its operands already loaded (see emit_coef).
template <typename R>
__device__ inline void emit_coef_pre(const AnaArgs<R> &a, long j, C<R> c, C<R> z, R w, double &f1) {
    c = cscale<R>(c, a.scale);
    if (!a.prox) {
        a.alpha[j] = c;
        return;
    }
    const R lam = (R)(*a.px.gamma) * w;
    const C<R> v = cadd<R>(c, z);
    const R mag = sqrt(v.x * v.x + v.y * v.y);
    const R sc = mag > lam ? R(1) - lam / mag : R(0);
    const C<R> r = cscale<R>(v, sc);
    const C<R> zn = csub<R>(v, r);
    a.px.z1[j] = zn;
    a.px.w1[j] = csub<R>(r, zn);
    f1 += (double)w * sqrt((double)c.x * c.x + (double)c.y * c.y);
}

// One level of the analysis for one basis (blockIdx.y) and one TO x TO tile
// of each sub-band (blockIdx.x); 256 threads, seen as 4 rows of 64.
template <typename R, int TO>
__global__ void __launch_bounds__(256) dwt_analysis(AnaArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    const int bi = blockIdx.y;
    const int b = a.basis[bi];
    const int Lf = 2 * b;
    // Filter taps, zero past Lf: single precision keeps them in (scalar)
    // registers; double precision would need 64 scalar registers for them and
    // reads an LDS copy instead.
    __shared__ R taps[2][kMaxTaps];
    R h[kMaxTaps], g[kMaxTaps];
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int m = 0; m < kMaxTaps; ++m) {
            h[m] = m < Lf ? a.filt[(b * 2 + 0) * kMaxTaps + m] : R(0);
            g[m] = m < Lf ? a.filt[(b * 2 + 1) * kMaxTaps + m] : R(0);
        }
    } else {
        if (threadIdx.x < 2 * kMaxTaps) {
            const int e = threadIdx.x / kMaxTaps, m = threadIdx.x % kMaxTaps;
            taps[e][m] = m < Lf ? a.filt[(b * 2 + e) * kMaxTaps + m] : R(0);
        }
    }
#define TAP_H(m) (sizeof(R) == 4 ? h[m] : taps[0][m])
#define TAP_G(m) (sizeof(R) == 4 ? g[m] : taps[1][m])
    const int s = a.s, half = s >> 1;
    const int tiles = half / TO;
    const int k0 = (blockIdx.x / tiles) * TO, l0 = (blockIdx.x % tiles) * TO;
    const int IR = 2 * TO + Lf - 2;
    constexpr int IRM = 2 * TO + kMaxTaps - 2;  // LDS row stride
    C<R> *reg = reinterpret_cast<C<R> *>(smem_raw);  // [IRM][IRM]
    C<R> *rlo = reg + IRM * IRM;                     // [IRM][TO]
    C<R> *rhi = rlo + IRM * TO;
    const C<R> *in = a.in + bi * a.in_bstride;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;

    // Prox operands of this thread's outputs, loaded before the filtering.
    const int n = a.n;
    const long pbase = (long)a.plane[bi] * n * n;
    constexpr int PER = (TO * TO + 255) / 256;
    C<R> zq[PER][4];
    R wq[PER][4];
    long jq[PER][4];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + 256 * u;
        const int k = idx / TO, l = idx % TO;  // TO is a constant power of two
        const int gk = k0 + k, gl = l0 + l;
        jq[u][0] = pbase + (long)gk * n + gl;
        jq[u][1] = pbase + (long)gk * n + half + gl;
        jq[u][2] = pbase + (long)(half + gk) * n + gl;
        jq[u][3] = pbase + (long)(half + gk) * n + half + gl;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            zq[u][t] = mk<R>(0, 0);
            wq[u][t] = R(1);
        }
        if (a.prox && idx < TO * TO) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t == 0 && !a.last) continue;  // LL goes to the next level
                zq[u][t] = a.px.z1[jq[u][t]];
                if (a.px.weights) wq[u][t] = a.px.weights[jq[u][t]];
            }
        }
    }

    // Periodic extension (on the smallest levels the region can exceed 2s).
    // The region is at most 2 TO + 14 <= 64 wide, so thread (ty, tx) stages
    // column tx of rows ty, ty + 4, ...: all its loads are issued before any
    // is stored, so their latencies overlap.
    // (Single precision; double-precision rows would spill registers and
    // are staged one at a time.)
    if constexpr (sizeof(R) == 4) {
        constexpr int RPT = (IRM + 3) / 4;
        C<R> st[RPT];
        const bool col = tx < IR;
        const long gc = (2 * l0 + tx) % s;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = ty + 4 * i;
            if (col && r < IR) st[i] = in[(long)((2 * k0 + r) % s) * s + gc];
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = ty + 4 * i;
            if (col && r < IR) reg[r * IRM + tx] = st[i];
        }
    } else {
        for (int r = ty; r < IR; r += 4) {
            int gr = 2 * k0 + r;
            while (gr >= s) gr -= s;
            for (int c = tx; c < IR; c += 64) {
                int gc = 2 * l0 + c;
                while (gc >= s) gc -= s;
                reg[r * IRM + c] = in[(long)gr * s + gc];
            }
        }
    }
    __syncthreads();
    // Rows (axis 1): rlo[r][l] = sum_m h[m] in[r][2l + m], rhi with g.
    for (int idx = threadIdx.x; idx < IR * TO; idx += 256) {
        const int r = idx / TO, l = idx % TO;
        R lr = 0, li = 0, hr = 0, hi = 0;
        const C<R> *row = reg + r * IRM + 2 * l;
#pragma unroll
        for (int m = 0; m < kMaxTaps; ++m) {
            if (m < Lf) {
                const C<R> v = row[m];
                lr += TAP_H(m) * v.x;
                li += TAP_H(m) * v.y;
                hr += TAP_G(m) * v.x;
                hi += TAP_G(m) * v.y;
            }
        }
        rlo[r * TO + l] = mk<R>(lr, li);
        rhi[r * TO + l] = mk<R>(hr, hi);
    }
    __syncthreads();
    // Columns (axis 0).
    double f1 = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + 256 * u;
        if (idx >= TO * TO) break;
        const int k = idx / TO, l = idx % TO;
        R llr = 0, lli = 0, hlr = 0, hli = 0, lhr = 0, lhi = 0, hhr = 0, hhi = 0;
#pragma unroll
        for (int m = 0; m < kMaxTaps; ++m) {
            if (m < Lf) {
                const C<R> vl = rlo[(2 * k + m) * TO + l];
                const C<R> vh = rhi[(2 * k + m) * TO + l];
                llr += TAP_H(m) * vl.x;
                lli += TAP_H(m) * vl.y;
                hlr += TAP_G(m) * vl.x;
                hli += TAP_G(m) * vl.y;
                lhr += TAP_H(m) * vh.x;
                lhi += TAP_H(m) * vh.y;
                hhr += TAP_G(m) * vh.x;
                hhi += TAP_G(m) * vh.y;
            }
        }
        const int gk = k0 + k, gl = l0 + l;
        if (a.last) emit_coef_pre<R>(a, jq[u][0], mk<R>(llr, lli), zq[u][0], wq[u][0], f1);
        else a.ll_out[bi * a.ll_bstride + (long)gk * half + gl] = mk<R>(llr, lli);
        emit_coef_pre<R>(a, jq[u][1], mk<R>(lhr, lhi), zq[u][1], wq[u][1], f1);
        emit_coef_pre<R>(a, jq[u][2], mk<R>(hlr, hli), zq[u][2], wq[u][2], f1);
        emit_coef_pre<R>(a, jq[u][3], mk<R>(hhr, hhi), zq[u][3], wq[u][3], f1);
    }
    if (a.prox) block_add_f1<R>(f1, a.px.f1_part);
#undef TAP_H
#undef TAP_G
}

// Dirac plane: alpha_0 = x / sqrt(q) (or its prox epilogue).
template <typename R> __global__ void dirac_analysis(AnaArgs<R> a, const C<R> *x) {
    const long N = (long)a.n * a.n;
    double f1 = 0.0;
    const long base = (long)a.plane[0] * N;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
        emit_coef<R>(a, base + i, x[i], f1);
    if (a.prox) block_add_f1<R>(f1, a.px.f1_part);
}

template <typename R> struct SynArgs {
    const C<R> *alpha;  // coefficient planes (q x n x n)
    const C<R> *ll_in;  // per-basis LL slot for this level (nullptr at the coarsest level)
    long ll_in_bstride;
    C<R> *ll_out;       // per-basis output slot (levels > 1)
    long ll_out_bstride;
    C<R> *x;            // final image (level 1)
    const R *filt;
    int basis[8];
    int plane[8];
    int nbases;
    int dirac_plane;    // -1 if the Dirac basis is not selected
    int n, s, TO, coarsest;
    R scale;
};

// The four sub-band regions of one synthesis tile, KR <= TO + 7 square: at
// most 3 entries per thread for 256 threads, held in registers between their
// loads and their LDS stores.
constexpr int kSynEPT = ((kTO + kMaxTaps / 2 - 1) * (kTO + kMaxTaps / 2 - 1) + 255) / 256;
template <typename R> struct SynRegion {
    C<R> ll[kSynEPT], lh[kSynEPT], hl[kSynEPT], hh[kSynEPT];
};

// Issues the loads of basis slot bi's regions for the (2 TO)^2 output tile at (i0, j0).
template <typename R>
__device__ inline void syn_load(const SynArgs<R> &a, int bi, int i0, int j0, SynRegion<R> &v) {
    const int Lf = 2 * a.basis[bi];
    const int half = a.s >> 1, KR = a.TO + Lf / 2 - 1;
    const int kst = i0 / 2 - Lf / 2 + 1, lst = j0 / 2 - Lf / 2 + 1;
    const int n = a.n;
    const C<R> *plane = a.alpha + (long)a.plane[bi] * n * n;
    const C<R> *llsrc = a.coarsest ? nullptr : a.ll_in + bi * a.ll_in_bstride;
#pragma unroll
    for (int q = 0; q < kSynEPT; ++q) {
        const int idx = threadIdx.x + q * blockDim.x;
        if (idx < KR * KR) {
            const int r = idx / KR, c = idx - r * KR;
            int k = (kst + r) % half, l = (lst + c) % half;
            if (k < 0) k += half;
            if (l < 0) l += half;
            v.ll[q] = a.coarsest ? plane[(long)k * n + l] : llsrc[(long)k * half + l];
            v.lh[q] = plane[(long)k * n + half + l];
            v.hl[q] = plane[(long)(half + k) * n + l];
            v.hh[q] = plane[(long)(half + k) * n + half + l];
        }
    }
}

// Column then row synthesis of one (2 TO)^2 output tile of basis slot bi from
// its loaded regions; adds the result into acc (thread-owned outputs
// idx = threadIdx.x + k*blockDim).
template <typename R>
__device__ inline void syn_tile(const SynArgs<R> &a, int bi, const SynRegion<R> *v, int i0, int j0, C<R> *smem,
                                C<R> (&acc)[4]) {
    const int b = a.basis[bi];
    const int Lf = 2 * b;
    const R *h = a.filt + (b * 2 + 0) * kMaxTaps;
    const R *g = a.filt + (b * 2 + 1) * kMaxTaps;
    const int TO = a.TO, TS = 2 * TO;
    const int KR = TO + Lf / 2 - 1;
    C<R> *LL = smem, *LH = LL + KR * KR, *HL = LH + KR * KR, *HH = HL + KR * KR;
    C<R> *lo1 = HH + KR * KR, *hi1 = lo1 + TS * KR;
    __syncthreads();  // the previous tile's readers of smem are done
    if (v) {
#pragma unroll
        for (int q = 0; q < kSynEPT; ++q) {
            const int idx = threadIdx.x + q * blockDim.x;
            if (idx < KR * KR) {
                LL[idx] = v->ll[q];
                LH[idx] = v->lh[q];
                HL[idx] = v->hl[q];
                HH[idx] = v->hh[q];
            }
        }
    } else {  // regions read straight into LDS (double precision)
        const int half = a.s >> 1, n = a.n;
        const int kst = i0 / 2 - Lf / 2 + 1, lst = j0 / 2 - Lf / 2 + 1;
        const C<R> *plane = a.alpha + (long)a.plane[bi] * n * n;
        const C<R> *llsrc = a.coarsest ? nullptr : a.ll_in + bi * a.ll_in_bstride;
        for (int idx = threadIdx.x; idx < KR * KR; idx += blockDim.x) {
            const int r = idx / KR, c = idx - r * KR;
            int k = (kst + r) % half, l = (lst + c) % half;
            if (k < 0) k += half;
            if (l < 0) l += half;
            LL[idx] = a.coarsest ? plane[(long)k * n + l] : llsrc[(long)k * half + l];
            LH[idx] = plane[(long)k * n + half + l];
            HL[idx] = plane[(long)(half + k) * n + l];
            HH[idx] = plane[(long)(half + k) * n + half + l];
        }
    }
    __syncthreads();
    // Columns (axis 0): lo1[ii][c] from (LL, HL), hi1[ii][c] from (LH, HH).
    // Output rows 2 r and 2 r + 1 read the same Lf / 2 input rows (even and
    // odd taps), so one thread forms both from one set of LDS reads.
    for (int w = threadIdx.x; w < (TS / 2) * KR; w += blockDim.x) {
        const int rp = w / KR, c = w - rp * KR;
        R lr0 = 0, li0 = 0, hr0 = 0, hi0 = 0, lr1 = 0, li1 = 0, hr1 = 0, hi1_ = 0;
        const int base = rp + Lf / 2 - 1;
        for (int t = 0; t < Lf / 2; ++t) {
            const int r = base - t;
            const C<R> vll = LL[r * KR + c], vhl = HL[r * KR + c];
            const C<R> vlh = LH[r * KR + c], vhh = HH[r * KR + c];
            const int m0 = 2 * t, m1 = 2 * t + 1;
            lr0 += h[m0] * vll.x + g[m0] * vhl.x;
            li0 += h[m0] * vll.y + g[m0] * vhl.y;
            hr0 += h[m0] * vlh.x + g[m0] * vhh.x;
            hi0 += h[m0] * vlh.y + g[m0] * vhh.y;
            lr1 += h[m1] * vll.x + g[m1] * vhl.x;
            li1 += h[m1] * vll.y + g[m1] * vhl.y;
            hr1 += h[m1] * vlh.x + g[m1] * vhh.x;
            hi1_ += h[m1] * vlh.y + g[m1] * vhh.y;
        }
        lo1[(2 * rp) * KR + c] = mk<R>(lr0, li0);
        hi1[(2 * rp) * KR + c] = mk<R>(hr0, hi0);
        lo1[(2 * rp + 1) * KR + c] = mk<R>(lr1, li1);
        hi1[(2 * rp + 1) * KR + c] = mk<R>(hr1, hi1_);
    }
    __syncthreads();
    // Rows (axis 1), output columns 2 c and 2 c + 1 of a row per thread and
    // step from the same Lf / 2 inputs (see syn_out for the ownership).
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int w = threadIdx.x + k * blockDim.x;
        if (w >= TS * TS / 2) break;
        const int ii = w / (TS / 2), cp = w - ii * (TS / 2);
        const int base = cp + Lf / 2 - 1;
        R xr0 = 0, xi0 = 0, xr1 = 0, xi1 = 0;
        for (int t = 0; t < Lf / 2; ++t) {
            const int c = base - t;
            const C<R> vl = lo1[ii * KR + c], vh = hi1[ii * KR + c];
            const int m0 = 2 * t, m1 = 2 * t + 1;
            xr0 += h[m0] * vl.x + g[m0] * vh.x;
            xi0 += h[m0] * vl.y + g[m0] * vh.y;
            xr1 += h[m1] * vl.x + g[m1] * vh.x;
            xi1 += h[m1] * vl.y + g[m1] * vh.y;
        }
        acc[2 * k].x += xr0;
        acc[2 * k].y += xi0;
        acc[2 * k + 1].x += xr1;
        acc[2 * k + 1].y += xi1;
    }
}

// Output owned by accumulator q of this thread in a (2 TO)^2 synthesis tile:
// step q / 2 of the row pass, column parity q % 2 (false past the tile).
__device__ inline bool syn_out(int q, int TS, int &ii, int &jj) {
    const int w = threadIdx.x + (q >> 1) * blockDim.x;
    if (w >= TS * TS / 2) return false;
    ii = w / (TS / 2);
    jj = 2 * (w - ii * (TS / 2)) + (q & 1);
    return true;
}

// Levels > 1: one basis per blockIdx.y, writes the finer LL slot.
template <typename R> __global__ void __launch_bounds__(256) dwt_synthesis(SynArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int bi = blockIdx.y;
    const int TS = 2 * a.TO, tiles = a.s / TS;
    const int i0 = (blockIdx.x / tiles) * TS, j0 = (blockIdx.x % tiles) * TS;
    C<R> acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = mk<R>(0, 0);
    if constexpr (sizeof(R) == 4) {
        SynRegion<R> v;
        syn_load<R>(a, bi, i0, j0, v);
        syn_tile<R>(a, bi, &v, i0, j0, smem, acc);
    } else {
        syn_tile<R>(a, bi, nullptr, i0, j0, smem, acc);
    }
    C<R> *out = a.ll_out + bi * a.ll_out_bstride;
    for (int q = 0; q < 4; ++q) {
        int ii, jj;
        if (syn_out(q, TS, ii, jj)) out[(long)(i0 + ii) * a.s + j0 + jj] = acc[q];
    }
}

// Level 1: sum of all bases (and the Dirac plane) for one output tile.
template <typename R> __global__ void __launch_bounds__(256) dwt_synthesis_final(SynArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int TS = 2 * a.TO, tiles = a.s / TS;
    const int i0 = (blockIdx.x / tiles) * TS, j0 = (blockIdx.x % tiles) * TS;
    C<R> acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = mk<R>(0, 0);
    if constexpr (sizeof(R) == 4) {
        // The next basis's regions load while the current one is filtered
        // (single precision: double-precision regions would spill).
        SynRegion<R> v, vn;
        if (a.nbases > 0) syn_load<R>(a, 0, i0, j0, v);
        for (int bi = 0; bi < a.nbases; ++bi) {
            if (bi + 1 < a.nbases) syn_load<R>(a, bi + 1, i0, j0, vn);
            syn_tile<R>(a, bi, &v, i0, j0, smem, acc);
            v = vn;
        }
    } else {
        for (int bi = 0; bi < a.nbases; ++bi) syn_tile<R>(a, bi, nullptr, i0, j0, smem, acc);
    }
    const int n = a.n;
    for (int q = 0; q < 4; ++q) {
        int ii, jj;
        if (!syn_out(q, TS, ii, jj)) continue;
        const long o = (long)(i0 + ii) * n + j0 + jj;
        C<R> v = acc[q];
        if (a.dirac_plane >= 0) v = cadd<R>(v, a.alpha[(long)a.dirac_plane * n * n + o]);
        a.x[o] = cscale<R>(v, a.scale);
    }
}

template <typename R> __global__ void dirac_only_synthesis(const C<R> *alpha, int plane, C<R> *x, long N, R scale) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
        x[i] = cscale<R>(alpha[(long)plane * N + i], scale);
}

// ---------------------------------------------------------------------------
// Host side.

// Tile side: the largest power of two dividing the sub-band side, at most kTO.
static int tile_side(int half) { return std::min(kTO, half & -half); }

static size_t ll_offset(int n, int level) {
    // Slot of the LL produced by level `level` (1-based): sum of sizes of the earlier slots.
    size_t off = 0;
    for (int j = 1; j < level; ++j) {
        const size_t s = (size_t)(n >> j);
        off += s * s;
    }
    return off;
}

static int dirac_blocks(int n) { return (int)std::min<long>(((long)n * n + 255) / 256, 4096); }

int psi_adj_blocks(const riop_plan *p) {
    const int n = p->n;
    int nb = 0, total = 0;
    for (int i = 0; i < p->q; ++i) {
        if (p->bases[i] == 0) total += dirac_blocks(n);
        else ++nb;
    }
    if (nb == 0) return total;
    for (int lev = 1; lev <= p->L; ++lev) {
        const int half = (n >> (lev - 1)) >> 1, tiles = half / tile_side(half);
        total += tiles * tiles * nb;
    }
    return total;
}

template <typename R> static size_t ana_lds(int TO) {
    const int IR = 2 * TO + kMaxTaps - 2;
    return sizeof(C<R>) * (size_t)(IR * IR + 2 * IR * TO);
}
template <typename R> static size_t syn_lds(int TO) {
    const int KR = TO + kMaxTaps / 2 - 1;
    return sizeof(C<R>) * (size_t)(4 * KR * KR + 2 * 2 * TO * KR);
}

template <typename R>
static void psi_adj_impl(riop_plan *p, const void *x, void *alpha, const Prox1<R> *px, hipStream_t st) {
    const int n = p->n, L = p->L;
    AnaArgs<R> a{};
    a.alpha = static_cast<C<R> *>(alpha);
    a.filt = p->filters.as<R>();
    a.n = n;
    a.scale = (R)p->scale_q;
    a.prox = px != nullptr;
    if (px) a.px = *px;
    int nb = 0, dirac_plane = -1;
    for (int i = 0; i < p->q; ++i) {
        if (p->bases[i] == 0) {
            dirac_plane = i;
        } else {
            a.basis[nb] = p->bases[i];
            a.plane[nb] = i;
            ++nb;
        }
    }
    if (dirac_plane >= 0) {
        AnaArgs<R> d = a;
        d.plane[0] = dirac_plane;
        const int blocks = dirac_blocks(n);
        TimedScope ts(p, KK_PSI_ADJ, st);
        hipLaunchKernelGGL(dirac_analysis<R>, dim3(blocks), dim3(256), 0, st, d, static_cast<const C<R> *>(x));
        RIOP_HIP(hipGetLastError());
        if (a.prox) a.px.f1_part += blocks;
    }
    if (nb == 0) return;
    C<R> *ll = p->ll.as<C<R>>();
    for (int lev = 1; lev <= L; ++lev) {
        const int s = n >> (lev - 1), half = s >> 1;
        a.s = s;
        a.TO = tile_side(half);
        a.last = lev == L;
        if (lev == 1) {
            a.in = static_cast<const C<R> *>(x);
            a.in_bstride = 0;
        } else {
            a.in = ll + ll_offset(n, lev - 1);
            a.in_bstride = (long)p->ll_stride;
        }
        a.ll_out = a.last ? nullptr : ll + ll_offset(n, lev);
        a.ll_bstride = (long)p->ll_stride;
        const int tiles = half / a.TO;
        TimedScope ts(p, KK_PSI_ADJ, st);
        const dim3 grid(tiles * tiles, nb);
        AnaArgs<R> al = a;
        a.px.f1_part += a.prox ? (long)tiles * tiles * nb : 0;
        switch (al.TO) {
            case 16: hipLaunchKernelGGL((dwt_analysis<R, 16>), grid, dim3(256), ana_lds<R>(16), st, al); break;
            case 8: hipLaunchKernelGGL((dwt_analysis<R, 8>), grid, dim3(256), ana_lds<R>(8), st, al); break;
            case 4: hipLaunchKernelGGL((dwt_analysis<R, 4>), grid, dim3(256), ana_lds<R>(4), st, al); break;
            case 2: hipLaunchKernelGGL((dwt_analysis<R, 2>), grid, dim3(256), ana_lds<R>(2), st, al); break;
            default: hipLaunchKernelGGL((dwt_analysis<R, 1>), grid, dim3(256), ana_lds<R>(1), st, al); break;
        }
        RIOP_HIP(hipGetLastError());
    }
}

template <typename R> void launch_psi_adj(riop_plan *p, const void *x, void *alpha, hipStream_t st) {
    psi_adj_impl<R>(p, x, alpha, nullptr, st);
}

template <typename R>
void launch_psi_adj_prox(riop_plan *p, const void *x, const Prox1<R> &px, hipStream_t st) {
    psi_adj_impl<R>(p, x, p->sd.w1.ptr /* unused for prox stores */, &px, st);
}

template <typename R> void launch_psi(riop_plan *p, const void *alpha, void *x, hipStream_t st) {
    const int n = p->n, L = p->L;
    SynArgs<R> a{};
    a.alpha = static_cast<const C<R> *>(alpha);
    a.filt = p->filters.as<R>();
    a.n = n;
    a.scale = (R)p->scale_q;
    a.x = static_cast<C<R> *>(x);
    a.dirac_plane = -1;
    int nb = 0;
    for (int i = 0; i < p->q; ++i) {
        if (p->bases[i] == 0) {
            a.dirac_plane = i;
        } else {
            a.basis[nb] = p->bases[i];
            a.plane[nb] = i;
            ++nb;
        }
    }
    a.nbases = nb;
    if (nb == 0) {
        const long N = (long)n * n;
        const int blocks = (int)std::min<long>((N + 255) / 256, 4096);
        TimedScope ts(p, KK_PSI, st);
        hipLaunchKernelGGL(dirac_only_synthesis<R>, dim3(blocks), dim3(256), 0, st, a.alpha, a.dirac_plane,
                           a.x, N, a.scale);
        RIOP_HIP(hipGetLastError());
        return;
    }
    C<R> *ll = p->ll.as<C<R>>();
    for (int lev = L; lev >= 1; --lev) {
        const int s = n >> (lev - 1), half = s >> 1;
        a.s = s;
        a.TO = tile_side(half);
        a.coarsest = lev == L;
        a.ll_in = a.coarsest ? nullptr : ll + ll_offset(n, lev);
        a.ll_in_bstride = (long)p->ll_stride;
        const int TS = 2 * a.TO, tiles = s / TS;
        TimedScope ts(p, KK_PSI, st);
        if (lev > 1) {
            a.ll_out = ll + ll_offset(n, lev - 1);
            a.ll_out_bstride = (long)p->ll_stride;
            hipLaunchKernelGGL(dwt_synthesis<R>, dim3(tiles * tiles, nb), dim3(256), syn_lds<R>(a.TO), st, a);
        } else {
            hipLaunchKernelGGL(dwt_synthesis_final<R>, dim3(tiles * tiles), dim3(256), syn_lds<R>(a.TO), st, a);
        }
        RIOP_HIP(hipGetLastError());
    }
}

// Daubechies filters for the device, built on the host (see plan.cpp).
template void launch_psi_adj<float>(riop_plan *, const void *, void *, hipStream_t);
template void launch_psi_adj<double>(riop_plan *, const void *, void *, hipStream_t);
template void launch_psi<float>(riop_plan *, const void *, void *, hipStream_t);
template void launch_psi<double>(riop_plan *, const void *, void *, hipStream_t);
template void launch_psi_adj_prox<float>(riop_plan *, const void *, const Prox1<float> &, hipStream_t);
template void launch_psi_adj_prox<double>(riop_plan *, const void *, const Prox1<double> &, hipStream_t);

}  // namespace riop
