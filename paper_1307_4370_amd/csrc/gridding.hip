// Interpolation matrix G of the measurement operator (Sec. 5, eq. opmodel) and
// its transpose, applied on the fly from each visibility's Kaiser-Bessel window.
//
// Plan layout (built here, once per coverage): every visibility's first window
// cell (a0, b0) = (floor(g - J/2) + 1) mod K and fractional offset
// rho = g - J/2 - floor(g - J/2) in [0, 1), with g = u K / (2 pi) computed in
// double precision, binned by the T x T grid tile holding (a0, b0) with a
// stable counting sort (tile, then caller index).
//
// Degridding (G): one workgroup per work unit (a tile and a chunk of its
// visibilities) stages the (T + J - 1)^2 grid region its windows can touch in
// LDS, then each thread interpolates one visibility at a time from LDS.
// Gridding (G^T): the same work units accumulate their visibilities' J x J
// contributions into an LDS copy of the region with LDS atomics, then add the
// region into the grid with one global atomic per cell.
//
// Kernel weights: for tap j the weight phi(rho + J/2 - 1 - j) is a polynomial
// in s = 2 rho - 1 fitted at plan time; phi is even, so taps j and J-1-j share
// the even and odd parts E(s^2), O(s^2): w_j = E + s O, w_{J-1-j} = E - s O.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace riop {

template <typename R> struct KDeg;
template <> struct KDeg<float> { static constexpr int D = 8; };
template <> struct KDeg<double> { static constexpr int D = 14; };

// ---------------------------------------------------------------------------
// Binning kernels.

template <typename R>
__global__ void bin_kernel(const R *__restrict__ uv, int64_t M, int K, int J, int T, int tps,
                           double gscale, int *__restrict__ tile_of, uint32_t *__restrict__ cell_of,
                           R *__restrict__ frac_of, int *__restrict__ flag) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double u = (double)uv[2 * m], v = (double)uv[2 * m + 1];
    const double lim = M_PI * (1.0 + 9.5367431640625e-07);
    if (!(fabs(u) <= lim) || !(fabs(v) <= lim)) {  // also catches NaN
        atomicOr(flag, 1);
        tile_of[m] = 0;
        cell_of[m] = 0;
        frac_of[2 * m] = 0;
        frac_of[2 * m + 1] = 0;
        return;
    }
    const double hu = u * gscale - 0.5 * J, hv = v * gscale - 0.5 * J;
    const double fu = floor(hu), fv = floor(hv);
    int a0 = ((int)fu + 1) % K, b0 = ((int)fv + 1) % K;
    if (a0 < 0) a0 += K;
    if (b0 < 0) b0 += K;
    tile_of[m] = (a0 / T) * tps + (b0 / T);
    cell_of[m] = (uint32_t)a0 | ((uint32_t)b0 << 16);
    frac_of[2 * m] = (R)(hu - fu);
    frac_of[2 * m + 1] = (R)(hv - fv);
}

constexpr int kBinChunk = 16384;  // visibilities per binning block

__global__ void hist_kernel(const int *__restrict__ tile_of, int64_t M, int ntiles, int nblk,
                            int *__restrict__ counts) {
    extern __shared__ int hist[];
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) hist[t] = 0;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kBinChunk;
    const int64_t hi = min<int64_t>(M, lo + kBinChunk);
    for (int64_t m = lo + threadIdx.x; m < hi; m += blockDim.x) atomicAdd(&hist[tile_of[m]], 1);
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) counts[(int64_t)t * nblk + blockIdx.x] = hist[t];
}

// Exclusive scan of int32 in three launches (block scan, scan of block sums, add).
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 4;

__global__ void scan_blocks(const int *__restrict__ in, int *__restrict__ out, int64_t n,
                            int *__restrict__ sums) {
    __shared__ int s[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanPer + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer];
    int tot = 0;
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        tot += v[i];
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int run = s[threadIdx.x] - tot;
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void scan_sums(int *__restrict__ sums, int nsums) {
    // Single block: sequential over chunks of kScanBlock.
    __shared__ int s[kScanBlock];
    int carry = 0;
    for (int base = 0; base < nsums; base += kScanBlock) {
        const int i = base + threadIdx.x;
        const int v = i < nsums ? sums[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nsums) sums[i] = carry + s[threadIdx.x] - v;
        const int total = s[kScanBlock - 1];
        __syncthreads();
        carry += total;
    }
}

__global__ void scan_add(int *__restrict__ out, int64_t n, const int *__restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanPer + (int64_t)threadIdx.x * kScanPer;
    const int add = sums[blockIdx.x];
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) out[base + i] += add;
}

__global__ void tile_start_kernel(const int *__restrict__ offsets, int ntiles, int nblk, int64_t M,
                                  int *__restrict__ tile_start) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles) tile_start[t] = offsets[(int64_t)t * nblk];
    if (t == ntiles) tile_start[t] = (int)M;
}

// Stable scatter: one wavefront per binning block walks its chunk in order,
// ranking equal tiles among the 64 lanes of each step.
template <typename R>
__global__ void __launch_bounds__(64) scatter_kernel(const int *__restrict__ tile_of,
                                                     const uint32_t *__restrict__ cell_of,
                                                     const R *__restrict__ frac_of, int64_t M,
                                                     int ntiles, int nblk,
                                                     const int *__restrict__ offsets,
                                                     int *__restrict__ perm, uint32_t *__restrict__ cell,
                                                     R *__restrict__ frac) {
    extern __shared__ int cursor[];
    for (int t = threadIdx.x; t < ntiles; t += 64) cursor[t] = offsets[(int64_t)t * nblk + blockIdx.x];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kBinChunk;
    const int64_t hi = min<int64_t>(M, lo + kBinChunk);
    const int lane = threadIdx.x;
    for (int64_t s = lo; s < hi; s += 64) {
        const int64_t m = s + lane;
        const int t = m < hi ? tile_of[m] : -1;
        int before = 0, after = 0;
        for (int l = 0; l < 64; ++l) {
            const int tl = __shfl(t, l, 64);
            before += (l < lane && tl == t) ? 1 : 0;
            after += (l > lane && tl == t) ? 1 : 0;
        }
        int pos = 0;
        if (t >= 0) pos = cursor[t] + before;
        __syncthreads();
        if (t >= 0) {
            if (after == 0) cursor[t] = pos + 1;
            perm[pos] = (int)m;
            cell[pos] = cell_of[m];
            frac[2 * (int64_t)pos] = frac_of[2 * m];
            frac[2 * (int64_t)pos + 1] = frac_of[2 * m + 1];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Kernel weights.

// Per-tap-pair polynomial coefficients, passed by value in the kernel
// arguments so they live in scalar registers / the constant cache.
template <typename R> struct KCoef {
    R c[8][2][KDeg<R>::D / 2 + 1];  // [tap pair][even, odd][power of s^2]
};

template <typename R, int J>
__device__ inline void kb_weights(R rho, const KCoef<R> &kc, R (&w)[J]) {
    constexpr int D = KDeg<R>::D;
    constexpr int NEV = D / 2 + 1;   // even coefficients s^0, s^2, ..., s^(2*(NEV-1))
    constexpr int NOD = (D + 1) / 2; // odd coefficients s^1, s^3, ...
    const R s = R(2) * rho - R(1);
    const R u = s * s;
#pragma unroll
    for (int jp = 0; jp < J / 2; ++jp) {
        const R *ce = kc.c[jp][0];
        const R *co = kc.c[jp][1];
        R e = ce[NEV - 1];
#pragma unroll
        for (int k = NEV - 2; k >= 0; --k) e = e * u + ce[k];
        R o = co[NOD - 1];
#pragma unroll
        for (int k = NOD - 2; k >= 0; --k) o = o * u + co[k];
        w[jp] = e + s * o;
        w[J - 1 - jp] = e - s * o;
    }
}

// ---------------------------------------------------------------------------
// Degridding and gridding.

template <typename R> struct GridArgs {
    C<R> *grid;
    const WorkUnit *units;
    const uint32_t *cell;
    const R *frac;
    const int *perm;
    KCoef<R> kc;
    C<R> *vout;        // degrid output
    const C<R> *vin;   // grid input
    int K, T, tps;
    int order_user;
};

constexpr int kUnit = 2048;           // visibilities per work unit
constexpr int kDegridThreads = 256;
constexpr int kPerThread = kUnit / kDegridThreads;

template <typename R, int J, bool USER>
__device__ inline void degrid_one(const GridArgs<R> &a, const C<R> *reg, int W, int ta, int tb, int v) {
    const uint32_t cv = a.cell[v];
    const int la = (int)(cv & 0xffffu) - ta, lb = (int)(cv >> 16) - tb;
    R wu_[J], wv_[J];
    kb_weights<R, J>(a.frac[2 * (int64_t)v], a.kc, wu_);
    kb_weights<R, J>(a.frac[2 * (int64_t)v + 1], a.kc, wv_);
    R ar = 0, ai = 0;
    const C<R> *base = reg + la * W + lb;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        R rr = 0, ri = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const C<R> g = base[i * W + j];
            rr += wv_[j] * g.x;
            ri += wv_[j] * g.y;
        }
        ar += wu_[i] * rr;
        ai += wu_[i] * ri;
        // Scheduling fence: one window row of loads in flight at a time.
        __builtin_amdgcn_sched_barrier(0);
    }
    const int64_t dst = USER ? (int64_t)a.perm[v] : (int64_t)v;
    a.vout[dst] = mk<R>(ar, ai);
}

// Each thread handles a fixed number of visibilities, each in its own guarded
// block: a rolled loop gets rotated so that all J*J window loads of the next
// visibility stay live across the back edge, which halves occupancy.
template <typename R, int J, bool USER>
__global__ void __launch_bounds__(kDegridThreads) degrid_kernel(GridArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    C<R> *reg = reinterpret_cast<C<R> *>(smem_raw);
    const WorkUnit wu = a.units[blockIdx.x];
    const int W = a.T + J - 1;
    const int ta = (wu.tile / a.tps) * a.T, tb = (wu.tile % a.tps) * a.T;
    const int K = a.K;
    for (int idx = threadIdx.x; idx < W * W; idx += blockDim.x) {
        const int i = idx / W, j = idx - (idx / W) * W;
        int gi = ta + i, gj = tb + j;
        if (gi >= K) gi -= K;
        if (gj >= K) gj -= K;
        reg[idx] = a.grid[(int64_t)gi * K + gj];
    }
    __syncthreads();
    const int end = wu.start + wu.count;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int v = wu.start + threadIdx.x + k * kDegridThreads;
        if (v < end) degrid_one<R, J, USER>(a, reg, W, ta, tb, v);
    }
}

template <typename R, int J, bool USER>
__device__ inline void grid_one(const GridArgs<R> &a, R *acc_r, R *acc_i, int W, int ta, int tb, int v) {
    const uint32_t cv = a.cell[v];
    const int la = (int)(cv & 0xffffu) - ta, lb = (int)(cv >> 16) - tb;
    R wu_[J], wv_[J];
    kb_weights<R, J>(a.frac[2 * (int64_t)v], a.kc, wu_);
    kb_weights<R, J>(a.frac[2 * (int64_t)v + 1], a.kc, wv_);
    const C<R> val = a.vin[USER ? (int64_t)a.perm[v] : (int64_t)v];
    const int base = la * W + lb;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const R cr = wu_[i] * val.x, ci = wu_[i] * val.y;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            atomicAdd(&acc_r[base + i * W + j], cr * wv_[j]);
            atomicAdd(&acc_i[base + i * W + j], ci * wv_[j]);
        }
    }
}

template <typename R, int J, bool USER>
__global__ void __launch_bounds__(kDegridThreads) grid_kernel(GridArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    const WorkUnit wu = a.units[blockIdx.x];
    const int W = a.T + J - 1;
    R *acc_r = reinterpret_cast<R *>(smem_raw);
    R *acc_i = acc_r + W * W;
    for (int idx = threadIdx.x; idx < W * W; idx += blockDim.x) {
        acc_r[idx] = 0;
        acc_i[idx] = 0;
    }
    __syncthreads();
    const int ta = (wu.tile / a.tps) * a.T, tb = (wu.tile % a.tps) * a.T;
    const int end = wu.start + wu.count;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int v = wu.start + threadIdx.x + k * kDegridThreads;
        if (v < end) grid_one<R, J, USER>(a, acc_r, acc_i, W, ta, tb, v);
    }
    __syncthreads();
    const int K = a.K;
    for (int idx = threadIdx.x; idx < W * W; idx += blockDim.x) {
        const R vr = acc_r[idx], vi = acc_i[idx];
        if (vr == R(0) && vi == R(0)) continue;
        const int i = idx / W, j = idx - (idx / W) * W;
        int gi = ta + i, gj = tb + j;
        if (gi >= K) gi -= K;
        if (gj >= K) gj -= K;
        R *g = reinterpret_cast<R *>(a.grid + (int64_t)gi * K + gj);
        unsafeAtomicAdd(g, vr);
        unsafeAtomicAdd(g + 1, vi);
    }
}

// Fused G^T G: each work unit stages its input region, and for each of its
// visibilities computes the weights once, interpolates s = sum w X and spreads
// s w back into an LDS accumulator; the accumulator is added into the output
// grid (zeroed beforehand) with one global atomic per cell.
template <typename R, int J>
__device__ inline void gram_one(const GridArgs<R> &a, const C<R> *reg, R *acc_r, R *acc_i, int W, int ta, int tb,
                                int v) {
    const uint32_t cv = a.cell[v];
    const int la = (int)(cv & 0xffffu) - ta, lb = (int)(cv >> 16) - tb;
    R wu_[J], wv_[J];
    kb_weights<R, J>(a.frac[2 * (int64_t)v], a.kc, wu_);
    kb_weights<R, J>(a.frac[2 * (int64_t)v + 1], a.kc, wv_);
    R sr = 0, si = 0;
    const C<R> *base = reg + la * W + lb;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        R rr = 0, ri = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const C<R> g = base[i * W + j];
            rr += wv_[j] * g.x;
            ri += wv_[j] * g.y;
        }
        sr += wu_[i] * rr;
        si += wu_[i] * ri;
        __builtin_amdgcn_sched_barrier(0);
    }
    const int o = la * W + lb;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const R cr = wu_[i] * sr, ci = wu_[i] * si;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            atomicAdd(&acc_r[o + i * W + j], cr * wv_[j]);
            atomicAdd(&acc_i[o + i * W + j], ci * wv_[j]);
        }
    }
}

template <typename R, int J>
__global__ void __launch_bounds__(kDegridThreads) gram_kernel(GridArgs<R> a, const C<R> *__restrict__ gin) {
    extern __shared__ unsigned char smem_raw[];
    const WorkUnit wu = a.units[blockIdx.x];
    const int W = a.T + J - 1;
    C<R> *reg = reinterpret_cast<C<R> *>(smem_raw);
    R *acc_r = reinterpret_cast<R *>(reg + W * W);
    R *acc_i = acc_r + W * W;
    const int ta = (wu.tile / a.tps) * a.T, tb = (wu.tile % a.tps) * a.T;
    const int K = a.K;
    for (int idx = threadIdx.x; idx < W * W; idx += blockDim.x) {
        const int i = idx / W, j = idx - (idx / W) * W;
        int gi = ta + i, gj = tb + j;
        if (gi >= K) gi -= K;
        if (gj >= K) gj -= K;
        reg[idx] = gin[(int64_t)gi * K + gj];
        acc_r[idx] = 0;
        acc_i[idx] = 0;
    }
    __syncthreads();
    const int end = wu.start + wu.count;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int v = wu.start + threadIdx.x + k * kDegridThreads;
        if (v < end) gram_one<R, J>(a, reg, acc_r, acc_i, W, ta, tb, v);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < W * W; idx += blockDim.x) {
        const R vr = acc_r[idx], vi = acc_i[idx];
        if (vr == R(0) && vi == R(0)) continue;
        const int i = idx / W, j = idx - (idx / W) * W;
        int gi = ta + i, gj = tb + j;
        if (gi >= K) gi -= K;
        if (gj >= K) gj -= K;
        R *g = reinterpret_cast<R *>(a.grid + (int64_t)gi * K + gj);
        unsafeAtomicAdd(g, vr);
        unsafeAtomicAdd(g + 1, vi);
    }
}

template <typename R> __global__ void fill_zero_kernel(C<R> *buf, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n; k += stride) buf[k] = mk<R>(0, 0);
}

// ---------------------------------------------------------------------------
// Host side.

template <typename R> void launch_fill_zero(void *buf, size_t n, hipStream_t st) {
    if (n == 0) return;
    const int threads = 256;
    const int64_t blocks = std::min<int64_t>((int64_t)((n + threads - 1) / threads), 8192);
    hipLaunchKernelGGL(fill_zero_kernel<R>, dim3((unsigned)blocks), dim3(threads), 0, st,
                       static_cast<C<R> *>(buf), (int64_t)n);
    RIOP_HIP(hipGetLastError());
}

template <typename R> static void build_layout_t(riop_plan *p, const void *uv, hipStream_t st) {
    const int64_t M = p->M;
    const int K = p->K, T = p->tile, tps = p->tiles_per_side, ntiles = p->ntiles;
    p->perm.alloc(sizeof(int32_t) * M);
    p->cell.alloc(sizeof(uint32_t) * M);
    p->frac.alloc(sizeof(R) * 2 * M);
    p->tile_start.alloc(sizeof(int32_t) * (ntiles + 1));
    DevBuf tile_of, cell_of, frac_of, flag, counts, offsets, sums;
    const int nblk = (int)std::max<int64_t>(1, (M + kBinChunk - 1) / kBinChunk);
    const int64_t ncounts = (int64_t)ntiles * nblk;
    tile_of.alloc(sizeof(int) * M);
    cell_of.alloc(sizeof(uint32_t) * M);
    frac_of.alloc(sizeof(R) * 2 * M);
    flag.alloc(sizeof(int));
    counts.alloc(sizeof(int) * ncounts);
    offsets.alloc(sizeof(int) * ncounts);
    const int64_t per_blk = (int64_t)kScanBlock * kScanPer;
    const int nsums = (int)((ncounts + per_blk - 1) / per_blk);
    sums.alloc(sizeof(int) * nsums);
    RIOP_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(int), st));
    if (M > 0) {
        const int threads = 256;
        hipLaunchKernelGGL(bin_kernel<R>, dim3((unsigned)((M + threads - 1) / threads)), dim3(threads), 0, st,
                           static_cast<const R *>(uv), M, K, p->J, T, tps, (double)K / (2.0 * M_PI),
                           tile_of.as<int>(), cell_of.as<uint32_t>(), frac_of.as<R>(), flag.as<int>());
        RIOP_HIP(hipGetLastError());
    }
    const size_t lds_tiles = sizeof(int) * ntiles;
    hipLaunchKernelGGL(hist_kernel, dim3(nblk), dim3(256), lds_tiles, st, tile_of.as<int>(), M, ntiles, nblk,
                       counts.as<int>());
    RIOP_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_blocks, dim3(nsums), dim3(kScanBlock), 0, st, counts.as<int>(), offsets.as<int>(),
                       ncounts, sums.as<int>());
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanBlock), 0, st, sums.as<int>(), nsums);
    hipLaunchKernelGGL(scan_add, dim3(nsums), dim3(kScanBlock), 0, st, offsets.as<int>(), ncounts,
                       sums.as<int>());
    hipLaunchKernelGGL(tile_start_kernel, dim3((ntiles + 1 + 255) / 256), dim3(256), 0, st, offsets.as<int>(),
                       ntiles, nblk, M, p->tile_start.as<int>());
    RIOP_HIP(hipGetLastError());
    if (M > 0) {
        hipLaunchKernelGGL(scatter_kernel<R>, dim3(nblk), dim3(64), lds_tiles, st, tile_of.as<int>(),
                           cell_of.as<uint32_t>(), frac_of.as<R>(), M, ntiles, nblk, offsets.as<int>(),
                           p->perm.as<int>(), p->cell.as<uint32_t>(), p->frac.as<R>());
        RIOP_HIP(hipGetLastError());
    }
    int hflag = 0;
    std::vector<int> ts(ntiles + 1);
    RIOP_HIP(hipMemcpyAsync(&hflag, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOP_HIP(hipMemcpyAsync(ts.data(), p->tile_start.ptr, sizeof(int) * (ntiles + 1), hipMemcpyDeviceToHost, st));
    RIOP_HIP(hipStreamSynchronize(st));
    RIOP_REQUIRE(hflag == 0, RIOP_EINVAL, "uv coordinates must be finite and inside [-pi, pi]");

    // Work units: chunks of at most kUnit visibilities of one tile.
    const int unit = kUnit;
    std::vector<WorkUnit> units;
    int maxc = 0;
    for (int t = 0; t < ntiles; ++t) {
        const int s = ts[t], e = ts[t + 1];
        for (int c = s; c < e; c += unit) {
            const int cnt = std::min(unit, e - c);
            units.push_back(WorkUnit{t, c, cnt, 0});
            maxc = std::max(maxc, cnt);
        }
    }
    p->nunits = (int)units.size();
    p->max_unit = maxc;
    p->units.alloc(sizeof(WorkUnit) * std::max<size_t>(1, units.size()));
    if (!units.empty())
        RIOP_HIP(hipMemcpyAsync(p->units.ptr, units.data(), sizeof(WorkUnit) * units.size(),
                                hipMemcpyHostToDevice, st));
    RIOP_HIP(hipStreamSynchronize(st));
}

void build_layout(riop_plan *p, const void *uv, hipStream_t st) {
    if (p->prec == RIOP_F64)
        build_layout_t<double>(p, uv, st);
    else
        build_layout_t<float>(p, uv, st);
}

template <typename R> static GridArgs<R> grid_args(riop_plan *p) {
    GridArgs<R> a{};
    a.grid = p->grid.as<C<R>>();
    a.units = p->units.as<WorkUnit>();
    a.cell = p->cell.as<uint32_t>();
    a.frac = p->frac.as<R>();
    a.perm = p->perm.as<int>();
    const std::vector<double> &hc = p->kcoef_host;
    for (int jp = 0; jp < p->J / 2; ++jp)
        for (int e = 0; e < 2; ++e)
            for (int k = 0; k < KDeg<R>::D / 2 + 1; ++k)
                a.kc.c[jp][e][k] = (R)hc[(size_t)(jp * 2 + e) * kMaxPoly + k];
    a.K = p->K;
    a.T = p->tile;
    a.tps = p->tiles_per_side;
    return a;
}

#define RIOP_J_CASES(MACRO) MACRO(2) MACRO(4) MACRO(6) MACRO(8) MACRO(10) MACRO(12) MACRO(14) MACRO(16)

template <typename R> void launch_degrid(riop_plan *p, void *y, int order_user, hipStream_t st) {
    if (p->nunits == 0) return;
    GridArgs<R> a = grid_args<R>(p);
    a.vout = static_cast<C<R> *>(y);
    a.order_user = order_user;
    const int W = p->tile + p->J - 1;
    const size_t lds = sizeof(C<R>) * W * W;
    TimedScope ts(p, KK_DEGRID, st);
    switch (p->J) {
#define DG(JJ) \
    case JJ:                                                                                          \
        if (order_user)                                                                               \
            hipLaunchKernelGGL((degrid_kernel<R, JJ, true>), dim3(p->nunits), dim3(kDegridThreads), lds, st, a); \
        else                                                                                          \
            hipLaunchKernelGGL((degrid_kernel<R, JJ, false>), dim3(p->nunits), dim3(kDegridThreads), lds, st, a); \
        break;
        RIOP_J_CASES(DG)
#undef DG
        default: throw Error{RIOP_ENOTSUP, "unsupported kernel width"};
    }
    RIOP_HIP(hipGetLastError());
}

template <typename R> void launch_grid(riop_plan *p, const void *y, int order_user, hipStream_t st) {
    {
        TimedScope tz(p, KK_GRID_ZERO, st);
        launch_fill_zero<R>(p->grid.ptr, (size_t)p->K * p->K, st);
    }
    if (p->nunits == 0) return;
    GridArgs<R> a = grid_args<R>(p);
    a.vin = static_cast<const C<R> *>(y);
    a.order_user = order_user;
    const int W = p->tile + p->J - 1;
    const size_t lds = sizeof(R) * 2 * W * W;
    TimedScope ts(p, KK_GRID, st);
    switch (p->J) {
#define GK(JJ) \
    case JJ:                                                                                          \
        if (order_user)                                                                               \
            hipLaunchKernelGGL((grid_kernel<R, JJ, true>), dim3(p->nunits), dim3(kDegridThreads), lds, st, a); \
        else                                                                                          \
            hipLaunchKernelGGL((grid_kernel<R, JJ, false>), dim3(p->nunits), dim3(kDegridThreads), lds, st, a); \
        break;
        RIOP_J_CASES(GK)
#undef GK
        default: throw Error{RIOP_ENOTSUP, "unsupported kernel width"};
    }
    RIOP_HIP(hipGetLastError());
}

template <typename R> void launch_gram(riop_plan *p, const void *in_grid, void *out_grid, hipStream_t st) {
    {
        TimedScope tz(p, KK_GRID_ZERO, st);
        launch_fill_zero<R>(out_grid, (size_t)p->K * p->K, st);
    }
    if (p->nunits == 0) return;
    GridArgs<R> a = grid_args<R>(p);
    a.grid = static_cast<C<R> *>(out_grid);
    const int W = p->tile + p->J - 1;
    const size_t lds = (sizeof(C<R>) + 2 * sizeof(R)) * W * W;
    const C<R> *gin = static_cast<const C<R> *>(in_grid);
    TimedScope ts(p, KK_GRAM, st);
    switch (p->J) {
#define GR(JJ) \
    case JJ: hipLaunchKernelGGL((gram_kernel<R, JJ>), dim3(p->nunits), dim3(kDegridThreads), lds, st, a, gin); break;
        RIOP_J_CASES(GR)
#undef GR
        default: throw Error{RIOP_ENOTSUP, "unsupported kernel width"};
    }
    RIOP_HIP(hipGetLastError());
}

template void launch_gram<float>(riop_plan *, const void *, void *, hipStream_t);
template void launch_gram<double>(riop_plan *, const void *, void *, hipStream_t);
template void launch_degrid<float>(riop_plan *, void *, int, hipStream_t);
template void launch_degrid<double>(riop_plan *, void *, int, hipStream_t);
template void launch_grid<float>(riop_plan *, const void *, int, hipStream_t);
template void launch_grid<double>(riop_plan *, const void *, int, hipStream_t);
template void launch_fill_zero<float>(void *, size_t, hipStream_t);
template void launch_fill_zero<double>(void *, size_t, hipStream_t);

}  // namespace riop
