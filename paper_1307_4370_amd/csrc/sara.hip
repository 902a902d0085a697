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

template <typename R> __device__ inline void block_add_f1(double f1, double *acc) {
    __shared__ double red[256];
    red[threadIdx.x] = f1;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(acc, red[0]);
}

template <typename R>
__global__ void __launch_bounds__(256) dwt_analysis(AnaArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    const int bi = blockIdx.y;
    const int b = a.basis[bi];
    const int Lf = 2 * b;
    const R *h = a.filt + (b * 2 + 0) * kMaxTaps;
    const R *g = a.filt + (b * 2 + 1) * kMaxTaps;
    const int s = a.s, half = s >> 1, TO = a.TO;
    const int tiles = half / TO;
    const int k0 = (blockIdx.x / tiles) * TO, l0 = (blockIdx.x % tiles) * TO;
    const int IR = 2 * TO + Lf - 2;
    C<R> *reg = reinterpret_cast<C<R> *>(smem_raw);
    C<R> *rlo = reg + IR * IR;
    C<R> *rhi = rlo + IR * TO;
    const C<R> *in = a.in + bi * a.in_bstride;

    for (int idx = threadIdx.x; idx < IR * IR; idx += blockDim.x) {
        const int r = idx / IR, c = idx - r * IR;
        const int gr = (2 * k0 + r) % s, gc = (2 * l0 + c) % s;
        reg[idx] = in[(long)gr * s + gc];
    }
    __syncthreads();
    // Rows (axis 1): rlo[r][l] = sum_m h[m] in[r][2l + m], rhi with g.
    for (int idx = threadIdx.x; idx < IR * TO; idx += blockDim.x) {
        const int r = idx / TO, l = idx - r * TO;
        R lr = 0, li = 0, hr = 0, hi = 0;
        const C<R> *row = reg + r * IR + 2 * l;
        for (int m = 0; m < Lf; ++m) {
            const C<R> v = row[m];
            lr += h[m] * v.x;
            li += h[m] * v.y;
            hr += g[m] * v.x;
            hi += g[m] * v.y;
        }
        rlo[idx] = mk<R>(lr, li);
        rhi[idx] = mk<R>(hr, hi);
    }
    __syncthreads();
    // Columns (axis 0).
    double f1 = 0.0;
    C<R> *alpha = a.alpha + (long)a.plane[bi] * a.n * a.n;
    const long pbase = (long)a.plane[bi] * a.n * a.n;
    for (int idx = threadIdx.x; idx < TO * TO; idx += blockDim.x) {
        const int k = idx / TO, l = idx - k * TO;
        R llr = 0, lli = 0, hlr = 0, hli = 0, lhr = 0, lhi = 0, hhr = 0, hhi = 0;
        for (int m = 0; m < Lf; ++m) {
            const C<R> vl = rlo[(2 * k + m) * TO + l];
            const C<R> vh = rhi[(2 * k + m) * TO + l];
            llr += h[m] * vl.x;
            lli += h[m] * vl.y;
            hlr += g[m] * vl.x;
            hli += g[m] * vl.y;
            lhr += h[m] * vh.x;
            lhi += h[m] * vh.y;
            hhr += g[m] * vh.x;
            hhi += g[m] * vh.y;
        }
        const int gk = k0 + k, gl = l0 + l;
        const int n = a.n;
        if (a.last) {
            emit_coef<R>(a, pbase + (long)gk * n + gl, mk<R>(llr, lli), f1);
        } else {
            a.ll_out[bi * a.ll_bstride + (long)gk * half + gl] = mk<R>(llr, lli);
        }
        emit_coef<R>(a, pbase + (long)gk * n + half + gl, mk<R>(lhr, lhi), f1);
        emit_coef<R>(a, pbase + (long)(half + gk) * n + gl, mk<R>(hlr, hli), f1);
        emit_coef<R>(a, pbase + (long)(half + gk) * n + half + gl, mk<R>(hhr, hhi), f1);
    }
    (void)alpha;
    if (a.prox) block_add_f1<R>(f1, a.px.f1_acc);
}

// Dirac plane: alpha_0 = x / sqrt(q) (or its prox epilogue).
template <typename R> __global__ void dirac_analysis(AnaArgs<R> a, const C<R> *x) {
    const long N = (long)a.n * a.n;
    double f1 = 0.0;
    const long base = (long)a.plane[0] * N;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
        emit_coef<R>(a, base + i, x[i], f1);
    if (a.prox) block_add_f1<R>(f1, a.px.f1_acc);
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

// Column then row synthesis of one (2 TO)^2 output tile of basis slot bi;
// adds the result into acc (thread-owned outputs idx = threadIdx.x + k*blockDim).
template <typename R>
__device__ inline void syn_tile(const SynArgs<R> &a, int bi, int i0, int j0, C<R> *smem, C<R> (&acc)[4]) {
    const int b = a.basis[bi];
    const int Lf = 2 * b;
    const R *h = a.filt + (b * 2 + 0) * kMaxTaps;
    const R *g = a.filt + (b * 2 + 1) * kMaxTaps;
    const int s = a.s, half = s >> 1, TO = a.TO, TS = 2 * TO;
    const int KR = TO + Lf / 2 - 1;
    const int kst = i0 / 2 - Lf / 2 + 1, lst = j0 / 2 - Lf / 2 + 1;
    C<R> *LL = smem, *LH = LL + KR * KR, *HL = LH + KR * KR, *HH = HL + KR * KR;
    C<R> *lo1 = HH + KR * KR, *hi1 = lo1 + TS * KR;
    const int n = a.n;
    const C<R> *plane = a.alpha + (long)a.plane[bi] * n * n;
    const C<R> *llsrc = a.coarsest ? nullptr : a.ll_in + bi * a.ll_in_bstride;
    __syncthreads();
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
    __syncthreads();
    // Columns (axis 0): lo1[ii][c] from (LL, HL), hi1[ii][c] from (LH, HH).
    for (int idx = threadIdx.x; idx < TS * KR; idx += blockDim.x) {
        const int ii = idx / KR, c = idx - ii * KR;
        R lr = 0, li = 0, hr = 0, hi = 0;
        const int par = ii & 1, base = ii / 2 + Lf / 2 - 1;
        for (int t = 0; t < Lf / 2; ++t) {
            const int m = par + 2 * t;
            const int r = base - t;
            const C<R> vll = LL[r * KR + c], vhl = HL[r * KR + c];
            const C<R> vlh = LH[r * KR + c], vhh = HH[r * KR + c];
            lr += h[m] * vll.x + g[m] * vhl.x;
            li += h[m] * vll.y + g[m] * vhl.y;
            hr += h[m] * vlh.x + g[m] * vhh.x;
            hi += h[m] * vlh.y + g[m] * vhh.y;
        }
        lo1[idx] = mk<R>(lr, li);
        hi1[idx] = mk<R>(hr, hi);
    }
    __syncthreads();
    // Rows (axis 1).
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int idx = threadIdx.x + q * blockDim.x;
        if (idx >= TS * TS) break;
        const int ii = idx / TS, jj = idx - ii * TS;
        const int par = jj & 1, base = jj / 2 + Lf / 2 - 1;
        R xr = 0, xi = 0;
        for (int t = 0; t < Lf / 2; ++t) {
            const int m = par + 2 * t;
            const int c = base - t;
            const C<R> vl = lo1[ii * KR + c], vh = hi1[ii * KR + c];
            xr += h[m] * vl.x + g[m] * vh.x;
            xi += h[m] * vl.y + g[m] * vh.y;
        }
        acc[q].x += xr;
        acc[q].y += xi;
    }
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
    syn_tile<R>(a, bi, i0, j0, smem, acc);
    C<R> *out = a.ll_out + bi * a.ll_out_bstride;
    for (int q = 0; q < 4; ++q) {
        const int idx = threadIdx.x + q * blockDim.x;
        if (idx >= TS * TS) break;
        const int ii = idx / TS, jj = idx - ii * TS;
        out[(long)(i0 + ii) * a.s + j0 + jj] = acc[q];
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
    for (int bi = 0; bi < a.nbases; ++bi) syn_tile<R>(a, bi, i0, j0, smem, acc);
    const int n = a.n;
    for (int q = 0; q < 4; ++q) {
        const int idx = threadIdx.x + q * blockDim.x;
        if (idx >= TS * TS) break;
        const int ii = idx / TS, jj = idx - ii * TS;
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
        const long N = (long)n * n;
        const int blocks = (int)std::min<long>((N + 255) / 256, 4096);
        TimedScope ts(p, KK_PSI_ADJ, st);
        hipLaunchKernelGGL(dirac_analysis<R>, dim3(blocks), dim3(256), 0, st, d, static_cast<const C<R> *>(x));
        RIOP_HIP(hipGetLastError());
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
        hipLaunchKernelGGL(dwt_analysis<R>, dim3(tiles * tiles, nb), dim3(256), ana_lds<R>(a.TO), st, a);
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
