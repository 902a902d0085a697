// Interpolation matrix G of the measurement operator (Sec. 5, eq. opmodel) and
// its transpose, applied on the fly from each visibility's Kaiser-Bessel window.
//
// Plan layout (built here, once per coverage): every visibility's first window
// cell (a0, b0) = (floor(g - J/2) + 1) mod K and fractional offset
// rho = g - J/2 - floor(g - J/2) in [0, 1), with g = u K / (2 pi) computed in
// double precision.  Visibilities are sorted by T x T grid tile, then by cell
// inside the tile (row-major), then by caller index (a stable radix sort of
// the key); cell_start[key] gives the plan-order range of every cell
// (key = tile * T^2 + local row * T + local col).
//
// Degridding (G): one workgroup per work unit (a tile and a chunk of its
// visibilities) stages the (T + J - 1)^2 grid region its windows can touch in
// LDS, then each thread interpolates one visibility at a time from LDS.
// Neighbouring threads hold neighbouring cells, which keeps LDS bank conflicts
// low.
//
// Gridding (G^T): one workgroup per sort tile.  Its visibilities are one
// contiguous plan-order range and their windows reach only the tile and the
// first J - 1 rows / columns of its neighbours below and to the right.  The
// workgroup accumulates them into that (T + J - 1)-sided region, held in
// double precision in LDS (runs of visibilities that share a window row and an
// 8-aligned column block are summed in registers, on the matrix cores where
// possible, and closed with LDS double atomic adds: floating-point LDS
// atomics in single precision are slow on this GPU), then stores its own
// cells to the grid and the rest to its halo cells; a second kernel adds each
// tile's three incoming halos.  No zeroing of the grid, no global atomics,
// and every visibility is read once.
//
// Kernel weights: for tap j the weight phi(rho + J/2 - 1 - j) is a polynomial
// in s = 2 rho - 1 fitted at plan time; phi is even, so taps j and J-1-j share
// the even and odd parts E(s^2), O(s^2): w_j = E + s O, w_{J-1-j} = E - s O.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace riop {

template <typename R> struct KDeg;
template <> struct KDeg<float> { static constexpr int D = 7; };
template <> struct KDeg<double> { static constexpr int D = 14; };

// ---------------------------------------------------------------------------
// Binning kernels.

template <typename R>
__global__ void bin_kernel(const R *__restrict__ uv, int64_t M, int K, int J, int T, int tps,
                           double gscale, uint32_t *__restrict__ key_of, uint32_t *__restrict__ cell_of,
                           R *__restrict__ frac_of, int *__restrict__ flag) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double u = (double)uv[2 * m], v = (double)uv[2 * m + 1];
    const double lim = M_PI * (1.0 + 9.5367431640625e-07);
    if (!(fabs(u) <= lim) || !(fabs(v) <= lim)) {  // also catches NaN
        atomicOr(flag, 1);
        key_of[m] = 0;
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
    const int tile = (a0 / T) * tps + (b0 / T);
    key_of[m] = (uint32_t)(tile * T * T + (a0 % T) * T + (b0 % T));
    cell_of[m] = (uint32_t)a0 | ((uint32_t)b0 << 16);
    frac_of[2 * m] = (R)(hu - fu);
    frac_of[2 * m + 1] = (R)(hv - fv);
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

// Stable LSD radix sort of (key, caller index) pairs, 8 bits per pass, so
// that the plan order is by key and, within a key, by caller index, in O(M)
// work for any coverage.  A block owns kSortTile consecutive elements.
//   rs_hist:    its digit counts, stored digit-major (count[d * nblk + b]), so
//               that one exclusive scan gives every (digit, block) its first
//               output position;
//   rs_scatter: its elements in position order, 256 at a time; lanes of one
//               wavefront with equal digits are matched through eight ballots
//               (one per digit bit), ranked by lane, and placed after the
//               earlier wavefronts' and earlier rounds' elements of that digit.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;

__global__ void __launch_bounds__(kSortThreads) rs_hist(const uint32_t *__restrict__ keys, int64_t M, int shift,
                                                        int nblk, int *__restrict__ count) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < M) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    count[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads) rs_scatter(const uint32_t *__restrict__ keys_in,
                                                           const int *__restrict__ vals_in, int64_t M, int shift,
                                                           int nblk, const int *__restrict__ offset,
                                                           uint32_t *__restrict__ keys_out,
                                                           int *__restrict__ vals_out) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ int run[256];            // next output position of each digit
    __shared__ int wcnt[kWaves][256];   // this round's count of each digit per wavefront
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    run[tid] = offset[(int64_t)tid * nblk + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;  // lanes under this one
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + tid;
        const bool valid = i < M;
        const uint32_t key = valid ? keys_in[i] : 0u;
        const int val = valid ? (vals_in ? vals_in[i] : (int)i) : 0;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        int tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            tot += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += tot;
        __syncthreads();
    }
}

// start[k] = first plan-order position whose key is >= k (binary search over
// the sorted keys), for k = 0 .. nkeys.
__global__ void key_starts(const uint32_t *__restrict__ sorted, int64_t M, int64_t nkeys, int *__restrict__ start) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nkeys) return;
    int64_t lo = 0, hi = M;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)sorted[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    start[k] = (int)lo;
}

template <typename R>
__global__ void gather_layout(const int *__restrict__ perm, const uint32_t *__restrict__ cell_of,
                              const R *__restrict__ frac_of, int64_t M, uint32_t *__restrict__ cell,
                              R *__restrict__ frac) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int m = perm[i];
    cell[i] = cell_of[m];
    frac[2 * i] = frac_of[2 * (int64_t)m];
    frac[2 * i + 1] = frac_of[2 * (int64_t)m + 1];
}

__global__ void tile_start_from_keys(const int *__restrict__ start, int ntiles, int T2, int *__restrict__ ts) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= ntiles) ts[t] = start[(int64_t)t * T2];
}

// ---------------------------------------------------------------------------
// Kernel weights.

// Weights of the J taps at fractional offset rho, with the coefficient table
// read through a pointer (global, wave-uniform: scalar loads), laid out
// [pair][even/odd][KS].
template <typename R, int J>
__device__ inline void kb_weights_ptr(R rho, const R *__restrict__ kc, R (&w)[J]) {
    constexpr int D = KDeg<R>::D;
    constexpr int NEV = D / 2 + 1, NOD = (D + 1) / 2, KS = D / 2 + 1;
    const R s = R(2) * rho - R(1);
    const R u = s * s;
#pragma unroll
    for (int jp = 0; jp < J / 2; ++jp) {
        const R *ce = kc + (jp * 2 + 0) * KS;
        const R *co = kc + (jp * 2 + 1) * KS;
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
    const R *kc;       // kernel coefficients [pair][even/odd][D/2 + 1]
    C<R> *vout;        // degrid output
    const C<R> *vin;   // grid input
    int K, T, tps;
    int order_user;
};

constexpr int kUnit = 1024;           // visibilities per work unit
constexpr int kDegridThreads = 256;
constexpr int kPerThread = kUnit / kDegridThreads;

template <typename R, int J, bool USER>
__device__ inline void degrid_one(const GridArgs<R> &a, const R *kc, const C<R> *reg, int W, int ta, int tb,
                                  int v) {
    const uint32_t cv = a.cell[v];
    const R fu = a.frac[2 * (int64_t)v], fv = a.frac[2 * (int64_t)v + 1];
    const int la = (int)(cv & 0xffffu) - ta, lb = (int)(cv >> 16) - tb;
    R wu_[J], wv_[J];
    kb_weights_ptr<R, J>(fu, kc, wu_);
    kb_weights_ptr<R, J>(fv, kc, wv_);
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
    // Region rows by wavefront (a wave-uniform row and row address), columns
    // by lane (no divisions).
    for (int i = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); i < W; i += kDegridThreads >> 6) {
        int gi = ta + i;
        if (gi >= K) gi -= K;
        const C<R> *grow = a.grid + (int64_t)gi * K;
        C<R> *lrow = reg + i * W;
        for (int j = threadIdx.x & 63; j < W; j += 64) {
            int gj = tb + j;
            if (gj >= K) gj -= K;
            lrow[j] = grow[gj];
        }
    }
    // Single precision: the coefficient table (32 values at J = 8) in
    // registers for the whole block, so no visibility reloads it.
    constexpr int KS = KDeg<R>::D / 2 + 1, NKC = (J / 2) * 2 * KS;
    const R *kc = a.kc;
    R kcr[sizeof(R) == 4 ? NKC : 1];
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int i = 0; i < NKC; ++i) kcr[i] = a.kc[i];
        kc = kcr;
    }
    __syncthreads();
    const int end = wu.start + wu.count;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int v = wu.start + threadIdx.x + k * kDegridThreads;
        if (v < end) degrid_one<R, J, USER>(a, kc, reg, W, ta, tb, v);
    }
}

// ---------------------------------------------------------------------------
// Gridding: one workgroup per sort tile.

// Windows up to 8 wide are accumulated with matrix instructions
// (v_mfma_f32_16x16x4_f32, v_mfma_f64_16x16x4_f64: the same operand layouts;
// the accumulator rows differ, see the run close), wider ones with vector FMAs.
template <typename R> __host__ __device__ constexpr bool grid_mfma(int J) { return J <= 8; }

typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
__device__ inline mfma_f4 mfma_16x16x4(float a, float b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline mfma_d4 mfma_16x16x4(double a, double b, mfma_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row length of a wavefront's tap-major staging arrays.  Vector path: odd,
// so the eight-address broadcast reads fall in distinct banks.  Matrix path:
// 4 mod 32, so the operand reads (16 rows x 4 entries per instruction) hit 64
// distinct banks.  Either way the staging stores (consecutive lanes) are
// conflict-free.
// Entries per staged slice: 32 on the double-precision matrix path (one lane
// per entry and axis, which halves the staging area so that two workgroups
// fit per CU), 64 otherwise (one lane per entry).
template <typename R> __host__ __device__ constexpr int slice_len(int J) {
    return grid_mfma<R>(J) && sizeof(R) == 8 ? 32 : 64;
}
template <typename R> __host__ __device__ constexpr int slice_row(int J) {
    return grid_mfma<R>(J) ? (slice_len<R>(J) == 32 ? 36 : 68) : 65;
}

// LDS bytes of one wavefront's staging area.
template <typename R> __host__ __device__ constexpr int grid_stage_bytes(int J) {
    return ((int)sizeof(C<R>) * (grid_mfma<R>(J) ? 8 : J) + (int)sizeof(R) * 8 * ((J + 7) / 8 + 1)) * slice_row<R>(J);
}

// Region of a T x T tile: the cells its visibilities' windows reach, rows
// 0 .. T + J - 2 and columns 0 .. T + 8 NB - 1 (the run blocks are 8 NB + 8
// wide and start at a multiple of 8 below T), held as two double planes.
__host__ __device__ constexpr int region_rows(int T, int J) { return T + J - 1; }
__host__ __device__ constexpr int region_stride(int T, int J) { return T + 8 * ((J + 7) / 8); }

// Wavefronts per workgroup: of 6, 4 and 2, the count that keeps the most
// wavefronts resident per CU (160 KB of LDS, 32 x 32 tile), preferring more
// wavefronts per tile on ties (shorter heavy tiles).
template <typename R> __host__ __device__ constexpr int grid_waves(int J) {
    const int tile = 2 * 8 * region_rows(32, J) * region_stride(32, J) + 1024;
    const int st = grid_stage_bytes<R>(J);
    const int w6 = 6 * (163840 / (6 * st + tile)), w4 = 4 * (163840 / (4 * st + tile)), w2 = 2 * (163840 / (2 * st + tile));
    return (w6 >= w4 && w6 >= w2 && w6 > 0) ? 6 : (w4 >= w2 && w4 > 0) ? 4 : 2;
}

template <typename R> static size_t grid_lds(int T, int J, int waves) {
    return sizeof(double) * 2 * (size_t)region_rows(T, J) * region_stride(T, J) +
           (size_t)grid_stage_bytes<R>(J) * waves + sizeof(R) * (size_t)J * (KDeg<R>::D / 2 + 1);
}

// Halo of a tile: the region cells outside it, which belong to the tiles to
// the right (right strip, T x (J-1)), below and below-right (bottom strip,
// (J-1) x (T+J-1)).
__host__ __device__ constexpr int halo_cells(int T, int J) { return T * (J - 1) + (J - 1) * (T + J - 1); }
// Halo buffer layout.  Right strips first, by grid row: row i of tile (dr,
// dc) at ((dr T + i) tps + dc) (J - 1), so that the left parts one grid row
// receives are one contiguous run of tps (J - 1) cells.  Then the bottom
// strips (with the corner), tile by tile: (J - 1) rows of T + J - 1 cells at
// ntiles T (J - 1) + t (J - 1)(T + J - 1).
__host__ __device__ inline int64_t halo_right(int T, int J, int tps, int dr, int i, int dc) {
    return ((int64_t)(dr * T + i) * tps + dc) * (J - 1);
}
__host__ __device__ inline int64_t halo_bottom(int T, int J, int tps, int t) {
    return (int64_t)tps * tps * T * (J - 1) + (int64_t)t * (J - 1) * (T + J - 1);
}

template <typename R> struct TileArgs {
    C<R> *grid;               // own T x T cells of every tile
    C<R> *halo;               // halo_cells(T, J) per tile
    const uint32_t *cell;     // plan order: a0 | b0 << 16
    const R *frac;            // plan order: rho_u, rho_v
    const int *perm;          // plan order -> caller order
    const WorkUnit *order;    // tiles, heaviest first: (tile, first visibility, count)
    const C<R> *vin;          // values to grid
    const R *__restrict__ kc; // kernel coefficients [pair][even/odd][D/2 + 1]
    int K, T, tps;            // grid side, tile side, tiles per side
    // Fused l2-ball prox (P2 kernels, plan order): the values gridded are
    // d2 = r2 - z2' - s with v = s + z2, r2 = y + (v - y) scale, z2' = v - r2,
    // and z2' replaces z2.
    const C<R> *p2s, *p2y;
    C<R> *p2z;
    const double *p2scale;    // min(1, eps / ||v - y||), one value
};

// Own cells of tile t to the grid, the rest of its region to its halo cells.
// T is a power of two (shifts and masks); the bottom strip's row is found by
// a single-precision reciprocal, exact here: cell index and strip width are
// small integers, so (c + 1/2) / W stays at least 1 / (2 W) away from the
// integers.
template <typename R, int J>
__device__ inline void store_region(const TileArgs<R> &a, const double *tre, const double *tim, int t, int tid,
                                    int nthreads) {
    const int T = a.T, K = a.K, RS = region_stride(T, J), lt = __builtin_ctz(T);
    const int ta = (t / a.tps) * T, tb = (t % a.tps) * T;
    C<R> *gbase = a.grid + (int64_t)ta * K + tb;  // T rows of K cells: 32-bit offsets below
    // Two horizontally adjacent cells per step (T and RS are even): 16-byte
    // LDS reads of each plane.
    for (int c2 = tid; c2 < T * T / 2; c2 += nthreads) {
        const int c = 2 * c2, r = c >> lt, col = c & (T - 1);
        const double2 re = *reinterpret_cast<const double2 *>(tre + r * RS + col);
        const double2 im = *reinterpret_cast<const double2 *>(tim + r * RS + col);
        C<R> *g = gbase + r * K + col;
        g[0] = mk<R>((R)re.x, (R)im.x);
        g[1] = mk<R>((R)re.y, (R)im.y);
    }
    // Right strip: J - 1 cells of each row, rows tps (J - 1) apart.
    C<R> *right = a.halo + halo_right(T, J, a.tps, t / a.tps, 0, t % a.tps);
    const int rstride = a.tps * (J - 1);
    for (int c = tid; c < T * (J - 1); c += nthreads) {
        const int r = c / (J - 1), jj = c - r * (J - 1);
        right[(int64_t)r * rstride + jj] = mk<R>((R)tre[r * RS + T + jj], (R)tim[r * RS + T + jj]);
    }
    C<R> *bottom = a.halo + halo_bottom(T, J, a.tps, t);
    const int W = T + J - 1;
    const float inv = 1.0f / (float)W;
    for (int c = tid; c < (J - 1) * W; c += nthreads) {  // bottom strip with the corner
        const int q = (int)(((float)c + 0.5f) * inv);
        const int r = T + q, col = c - q * W;
        bottom[c] = mk<R>((R)tre[r * RS + col], (R)tim[r * RS + col]);
    }
}

// A tile's visibilities are one contiguous plan-order range; its wavefronts
// take equal contiguous shares of it and work independently, at most 64
// visibilities (a slice) at a time.
//
// Staging: lane t of the wavefront takes visibility t of the slice and writes
// its J row weights times the value, and its J column weights shifted by the
// window's column offset inside an 8-aligned column block (zeros around them),
// to the wavefront's own LDS area.
//
// Accumulation: the wavefront walks the slice one visibility per step.  In
// plan order, visibilities of one window row and one column block are
// consecutive, so such a run is summed in registers and added to the region
// only where it ends (a bit mask built by one ballot per slice), with LDS
// double-precision atomic adds: the region is held in double for both
// precisions (on this GPU the double LDS atomic is several times faster than
// the single one).  Matrix path: each group of 4 staged visibilities is one
// 16 x 16 x 4 product, A = window rows (real, imaginary) x entries, B =
// entries x column slots.  Vector path: lane (i, j) holds window rows i + 8p
// and column slots j + 8q.  No workgroup barrier inside the loop: a wavefront
// reads only what it staged itself.
//
// The workgroup finally stores its own T x T cells to the grid and the rest
// of the region to its halo cells; the adjoint FFT's row pass adds the halos
// of the three neighbours a tile receives from as it loads the grid (or
// grid_merge does, where that pass is not the specialised one).
// WAVES: grid_waves<R>(J), or 2 for tiles whose region leaves too little LDS.
// P2: the values are formed from the l2-ball prox's inputs (see TileArgs), in
// double precision, at staging (the second pass of the prox of f2, Sec. 4.4).
template <typename R, int J, bool USER, int WAVES, bool P2>
__global__ void __launch_bounds__(64 * WAVES) grid_tile(TileArgs<R> a) {
    constexpr int kWaves = WAVES, kThreads = 64 * kWaves;
    constexpr int NB = (J + 7) / 8;  // row slots per lane (vector path)
    constexpr int QB = NB + 1;       // column slots per lane
    constexpr int NC = 8 * QB;       // staged column-weight rows
    constexpr bool MF = grid_mfma<R>(J);
    constexpr int JR = MF ? 8 : J;   // staged row-weight rows
    constexpr int SR = slice_row<R>(J);
    constexpr int SL = slice_len<R>(J);
    constexpr int BATCH = sizeof(R) == 8 ? (J > 12 ? 2 : 4) : (J > 8 ? 4 : 8);
    // Kernel coefficients through scalar loads where they fit in scalar
    // registers alongside everything else, else from an LDS copy.
    constexpr bool kScalarCoef = sizeof(R) == 4 && J <= 12;
    constexpr bool kUnroll = !(sizeof(R) == 8 && J > 12);
    constexpr int KS = KDeg<R>::D / 2 + 1;
    extern __shared__ unsigned char smem_raw[];
    const int T = a.T, K = a.K, tps = a.tps;
    const int RR = region_rows(T, J), RS = region_stride(T, J), PS = RR * RS;
    double *tre = reinterpret_cast<double *>(smem_raw);                   // [RR][RS] real parts
    double *tim = tre + PS;                                               // [RR][RS] imaginary parts
    C<R> *wuv_all = reinterpret_cast<C<R> *>(tim + PS);                   // [waves][JR][SR]: wu_i * value
    R *wv_all = reinterpret_cast<R *>(wuv_all + (size_t)kWaves * JR * SR);  // [waves][NC][SR]
    R *kcl = wv_all + (size_t)kWaves * NC * SR;                           // [J/2][2][KS]
    const int tid = threadIdx.x;
    if constexpr (!kScalarCoef)
        for (int i = tid; i < (J / 2) * 2 * KS; i += kThreads) kcl[i] = a.kc[i];

    const WorkUnit wk = a.order[blockIdx.x];
    const int t = wk.tile, v0 = wk.start, total = wk.count;
    if (total == 0) {  // an empty tile: zeros for its cells and its halo cells, no region
        const int ta0 = (t / tps) * T, tb0 = (t % tps) * T, lt = __builtin_ctz(T);
        for (int c = tid; c < T * T; c += kThreads) {
            const int r = c >> lt;
            a.grid[(int64_t)(ta0 + r) * K + tb0 + (c & (T - 1))] = mk<R>(0, 0);
        }
        C<R> *right = a.halo + halo_right(T, J, tps, t / tps, 0, t % tps);
        for (int c = tid; c < T * (J - 1); c += kThreads) {
            const int r = c / (J - 1);
            right[(int64_t)r * tps * (J - 1) + c - r * (J - 1)] = mk<R>(0, 0);
        }
        C<R> *bottom = a.halo + halo_bottom(T, J, tps, t);
        for (int c = tid; c < (J - 1) * (T + J - 1); c += kThreads) bottom[c] = mk<R>(0, 0);
        return;
    }
    const int ta = (t / tps) * T, tb = (t % tps) * T;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, li = lane >> 3, lj = lane & 7;
    // 32-entry slices: lane = entry + 32 axis stages one axis of one entry
    // (axis 0: u, with the value; axis 1: v).  64-entry slices: lane = entry,
    // both axes.
    constexpr bool SPLIT = SL == 32;
    const int e = SPLIT ? (lane & 31) : lane, ax = SPLIT ? (lane >> 5) : 0;
    // This wavefront's share of the tile's visibilities (tile-relative).
    const int f_begin = (int)(((int64_t)wave * total) / kWaves);
    const int f_end = (int)(((int64_t)(wave + 1) * total) / kWaves);

    // The visibility this lane stages next: cell, offsets and value.
    uint32_t cv = 0;
    R fu = 0, fv = 0;
    C<R> val = mk<R>(0, 0);
    C<R> ps = mk<R>(0, 0), pz = mk<R>(0, 0), py = mk<R>(0, 0);  // P2 inputs
    auto load = [&](int f) {
        if (f < f_end) {
            const int v = v0 + f;
            cv = a.cell[v];
            if constexpr (SPLIT) {
                fu = a.frac[2 * (int64_t)v + ax];  // this lane's axis
            } else {
                fu = a.frac[2 * (int64_t)v];
                fv = a.frac[2 * (int64_t)v + 1];
            }
            if (ax == 0) {
                if constexpr (P2) {
                    ps = a.p2s[v];
                    pz = a.p2z[v];
                    py = a.p2y[v];
                } else {
                    val = a.vin[USER ? (int64_t)a.perm[v] : (int64_t)v];
                }
            }
        }
    };
    const double p2sc = P2 ? *a.p2scale : 1.0;
    // The first slice's loads are in flight while the region is cleared.
    load(f_begin + e);
    {  // 16-byte stores (the region starts the LDS block; PS is even)
        double2 *t2 = reinterpret_cast<double2 *>(tre);
        for (int c = tid; c < PS; c += kThreads) t2[c] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    C<R> *wuv = wuv_all + wave * JR * SR;
    R *wv = wv_all + wave * NC * SR;
    // Matrix path: row-weight rows J .. 7 are never staged and stay zero.
    if constexpr (MF)
        for (int i = J * SR + lane; i < JR * SR; i += 64) wuv[i] = mk<R>(0, 0);

    // Vector path state.
    int ic[NB], jc[QB];
#pragma unroll
    for (int p = 0; p < NB; ++p) ic[p] = min(li + 8 * p, J - 1) * SR;
#pragma unroll
    for (int q = 0; q < QB; ++q) jc[q] = (lj + 8 * q) * SR;
    C<R> acc[NB][QB];
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
        for (int q = 0; q < QB; ++q) acc[p][q] = mk<R>(0, 0);
    // Closing a run adds its sums to the region cells its window block covers.
    auto close_run = [&](int pos) {
        const int la = pos >> 8, cb = (pos & 255) << 3;
#pragma unroll
        for (int p = 0; p < NB; ++p)
#pragma unroll
            for (int q = 0; q < QB; ++q) {
                const int i = li + 8 * p;
                if (i < J) {
                    const int c = (la + i) * RS + cb + lj + 8 * q;
                    __hip_atomic_fetch_add(tre + c, (double)acc[p][q].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add(tim + c, (double)acc[p][q].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                acc[p][q] = mk<R>(0, 0);
            }
    };
    // Matrix path state: lane l holds D[4 (l / 16) + r][l % 16], i.e. window
    // rows 2 (l / 16) and 2 (l / 16) + 1 (real, imaginary) of column slot l % 16.
    typedef R mf4 __attribute__((ext_vector_type(4)));
    mf4 dacc = {R(0), R(0), R(0), R(0)};
    const int mk_ = lane >> 4, mi = lane & 15;
    const int abase = 2 * ((mi >> 1) * SR + mk_) + (mi & 1);  // real-part index into wuv
    const int bbase = mi * SR + mk_;                          // index into wv
    const int coff = 2 * mk_ * RS + mi;                       // this lane's first cell of a run block
    auto close_run_mf = [&](int pos) {
        if constexpr (sizeof(R) == 4) {
            // f32 product: lane (mk_, mi) holds rows 4 mk_ .. 4 mk_ + 3, i.e.
            // window rows 2 mk_ + h (h = 0, 1), real and imaginary.
            const int c = (pos >> 8) * RS + ((pos & 255) << 3) + coff;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (2 * mk_ + h < J) {
                    __hip_atomic_fetch_add(tre + c + h * RS, (double)dacc[2 * h], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add(tim + c + h * RS, (double)dacc[2 * h + 1], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        } else {
            // f64 product: lane (mk_, mi) holds rows 4 r + mk_ (r = 0..3), i.e.
            // window rows 2 r + (mk_ >> 1) of one part (mk_ & 1: imaginary).
            double *plane = (mk_ & 1) ? tim : tre;
            const int c = ((pos >> 8) + (mk_ >> 1)) * RS + ((pos & 255) << 3) + mi;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (2 * r + (mk_ >> 1) < J)
                    __hip_atomic_fetch_add(plane + c + 2 * r * RS, (double)dacc[r], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        dacc = mf4{R(0), R(0), R(0), R(0)};
    };
    int cur = -1;  // packed window row and column block of the open run (-1: none yet)

    for (int base = f_begin; base < f_end; base += SL) {
        const int nlive = min(SL, f_end - base);
        const bool live = e < nlive;
        if constexpr (P2) {
            if (live && ax == 0) {
                const double vr = (double)ps.x + pz.x, vi = (double)ps.y + pz.y;
                const double rr = py.x + (vr - py.x) * p2sc, ri = py.y + (vi - py.y) * p2sc;
                const double znr = vr - rr, zni = vi - ri;
                a.p2z[v0 + base + e] = mk<R>((R)znr, (R)zni);
                val = mk<R>((R)(rr - znr - ps.x), (R)(ri - zni - ps.y));
            }
        }
        // Staging.  Lanes past the end stage zero values, so the
        // accumulation below runs over all 64 entries without bound tests.
        if (!live) val = mk<R>(0, 0);
        const int la = (int)(cv & 0xffffu) - ta, lb = (int)(cv >> 16) - tb;  // in [0, T)
        const int pos = (live && ax == 0) ? (la << 8) | (lb >> 3) : -1;
        const int db = lb & 7;
        if constexpr (SPLIT) {
            R w_[J];
            if constexpr (kScalarCoef) kb_weights_ptr<R, J>(fu, a.kc, w_);
            else kb_weights_ptr<R, J>(fu, kcl, w_);
            if (ax == 0) {
#pragma unroll
                for (int i = 0; i < J; ++i) wuv[i * SR + e] = mk<R>(w_[i] * val.x, w_[i] * val.y);
            } else {
                // Column weights at rows db .. db + J - 1, zeros in the other
                // rows: all rows cleared at fixed offsets, then the weights
                // written over them (one wavefront's LDS writes land in order).
#pragma unroll
                for (int r = 0; r < NC; ++r) wv[r * SR + e] = R(0);
                R *wcol = wv + db * SR + e;
#pragma unroll
                for (int j = 0; j < J; ++j) wcol[j * SR] = w_[j];
            }
        } else {
            R wu_[J], wv_[J];
            if constexpr (kScalarCoef) {
                kb_weights_ptr<R, J>(fu, a.kc, wu_);
                kb_weights_ptr<R, J>(fv, a.kc, wv_);
            } else {
                kb_weights_ptr<R, J>(fu, kcl, wu_);
                kb_weights_ptr<R, J>(fv, kcl, wv_);
            }
#pragma unroll
            for (int i = 0; i < J; ++i) wuv[i * SR + lane] = mk<R>(wu_[i] * val.x, wu_[i] * val.y);
            // Column weights at rows db .. db + J - 1, zeros in the other
            // rows: all rows cleared at fixed offsets, then the weights
            // written over them (one wavefront's LDS writes land in order).
#pragma unroll
            for (int r = 0; r < NC; ++r) wv[r * SR + lane] = R(0);
            R *wcol = wv + db * SR + lane;
#pragma unroll
            for (int j = 0; j < J; ++j) wcol[j * SR] = wv_[j];
        }
        // Run starts: entries whose window row or column block differs from
        // the previous entry's (lane 0 compares with the open run).
        const int prev = __builtin_amdgcn_update_dpp(cur, pos, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
        const uint64_t starts = __ballot(live && ax == 0 && pos != prev);
        __builtin_amdgcn_wave_barrier();
        // The next slice's visibility: global loads in flight during the accumulation.
        load(base + SL + e);

        if constexpr (MF) {
            // Groups of 4 entries; a group holding run starts is split into
            // products over the entries of each run (B masked by entry).
            const R *wuf = reinterpret_cast<const R *>(wuv);
            if (nlive == SL) {
#pragma unroll
                for (int g = 0; g < SL / 4; ++g) {
                    const R av = wuf[abase + 8 * g];
                    const R bv = wv[bbase + 4 * g];
                    const unsigned s4 = (unsigned)(starts >> (4 * g)) & 0xFu;
                    if (__builtin_expect(s4 == 0, 1)) {
                        dacc = mfma_16x16x4(av, bv, dacc);
                    } else {
                        unsigned m = s4;
                        int lo = 0;
                        while (m) {
                            const int b = __builtin_ctz(m);
                            m &= m - 1;
                            if (b > lo) {
                                const R bm = (mk_ >= lo && mk_ < b) ? bv : R(0);
                                dacc = mfma_16x16x4(av, bm, dacc);
                            }
                            if (cur >= 0) close_run_mf(cur);
                            cur = __builtin_amdgcn_readlane(pos, 4 * g + b);
                            lo = b;
                        }
                        const R bm = mk_ >= lo ? bv : R(0);
                        dacc = mfma_16x16x4(av, bm, dacc);
                    }
                }
            } else {  // a partial slice: its groups past the last live entry are all zero
                const int ng = (nlive + 3) >> 2;
#pragma unroll 1
                for (int g = 0; g < ng; ++g) {
                    const R av = wuf[abase + 8 * g];
                    const R bv = wv[bbase + 4 * g];
                    const unsigned s4 = (unsigned)(starts >> (4 * g)) & 0xFu;
                    if (__builtin_expect(s4 == 0, 1)) {
                        dacc = mfma_16x16x4(av, bv, dacc);
                    } else {
                        unsigned m = s4;
                        int lo = 0;
                        while (m) {
                            const int b = __builtin_ctz(m);
                            m &= m - 1;
                            if (b > lo) {
                                const R bm = (mk_ >= lo && mk_ < b) ? bv : R(0);
                                dacc = mfma_16x16x4(av, bm, dacc);
                            }
                            if (cur >= 0) close_run_mf(cur);
                            cur = __builtin_amdgcn_readlane(pos, 4 * g + b);
                            lo = b;
                        }
                        const R bm = mk_ >= lo ? bv : R(0);
                        dacc = mfma_16x16x4(av, bm, dacc);
                    }
                }
            }
        } else {
            // One staged visibility per step; unrolled over the slice
            // (constant bit tests, immediate offsets) where registers allow,
            // with the reads of the next batch issued before the current
            // batch is used.
            auto fetch_batch = [&](int kb, C<R> (&us)[BATCH][NB], R (&ws)[BATCH][QB]) {
#pragma unroll
                for (int k = 0; k < BATCH; ++k) {
#pragma unroll
                    for (int p = 0; p < NB; ++p) us[k][p] = wuv[ic[p] + kb + k];
#pragma unroll
                    for (int q = 0; q < QB; ++q) ws[k][q] = wv[jc[q] + kb + k];
                }
            };
            auto use_batch = [&](int kb, const C<R> (&us)[BATCH][NB], const R (&ws)[BATCH][QB]) {
#pragma unroll
                for (int k = 0; k < BATCH; ++k) {
                    if (__builtin_expect((starts >> (kb + k)) & 1, 0)) {
                        if (cur >= 0) close_run(cur);
                        cur = __builtin_amdgcn_readlane(pos, kb + k);
                    }
#pragma unroll
                    for (int p = 0; p < NB; ++p)
#pragma unroll
                        for (int q = 0; q < QB; ++q) {
                            acc[p][q].x += us[k][p].x * ws[k][q];
                            acc[p][q].y += us[k][p].y * ws[k][q];
                        }
                }
            };
            if constexpr (kUnroll) {
                C<R> u0[BATCH][NB], u1[BATCH][NB];
                R w0[BATCH][QB], w1[BATCH][QB];
                fetch_batch(0, u0, w0);
#pragma unroll
                for (int kb = 0; kb < 64; kb += 2 * BATCH) {
                    fetch_batch(kb + BATCH, u1, w1);
                    use_batch(kb, u0, w0);
                    if (kb + 2 * BATCH < 64) fetch_batch(kb + 2 * BATCH, u0, w0);
                    use_batch(kb + BATCH, u1, w1);
                }
            } else {
#pragma unroll 1
                for (int kb = 0; kb < 64; kb += BATCH) {
                    C<R> u0[BATCH][NB];
                    R w0[BATCH][QB];
                    fetch_batch(kb, u0, w0);
                    use_batch(kb, u0, w0);
                }
            }
        }
        // The next slice's staging overwrites this one.
        __builtin_amdgcn_wave_barrier();
    }
    if (cur >= 0) {
        if constexpr (MF) close_run_mf(cur);
        else close_run(cur);
    }
    __syncthreads();
    store_region<R, J>(a, tre, tim, t, tid, kThreads);
}

// Adds to each tile's first J-1 rows and columns what the tiles above, to
// the left and above-left left in their halo cells (periodic in the tile
// grid), in that fixed order.  One thread per border cell.  The adjoint FFT's
// specialised row pass performs the same additions, in the same order, on
// load; this kernel serves the other FFT lengths.
template <typename R>
__global__ void grid_merge(C<R> *grid, const C<R> *halo, int K, int T, int J, int tps) {
    const int per = (J - 1) * (2 * T - J + 1);  // border cells per tile
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)tps * tps * per) return;
    const int d = (int)(g / per), e = (int)(g % per);
    int i, j;
    if (e < (J - 1) * T) {
        i = e / T;
        j = e % T;
    } else {
        const int e2 = e - (J - 1) * T;
        i = J - 1 + e2 / (J - 1);
        j = e2 % (J - 1);
    }
    const int dr = d / tps, dc = d % tps;
    const int up = ((dr + tps - 1) % tps) * tps + dc;
    const int left = dr * tps + (dc + tps - 1) % tps;
    const int ul = ((dr + tps - 1) % tps) * tps + (dc + tps - 1) % tps;
    const int64_t cell = (int64_t)(dr * T + i) * K + dc * T + j;
    C<R> v = grid[cell];
    if (i < J - 1) v = cadd<R>(v, halo[halo_bottom(T, J, tps, up) + i * (T + J - 1) + j]);
    if (j < J - 1) v = cadd<R>(v, halo[halo_right(T, J, tps, dr, i, left % tps) + j]);
    if (i < J - 1 && j < J - 1) v = cadd<R>(v, halo[halo_bottom(T, J, tps, ul) + i * (T + J - 1) + T + j]);
    grid[cell] = v;
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

// Exclusive scan of n ints in place of `out` (may equal `in`), with `sums`
// holding ceil(n / (kScanBlock kScanPer)) ints.
static void scan_exclusive(const int *in, int *out, int64_t n, int *sums, hipStream_t st) {
    const int64_t per_blk = (int64_t)kScanBlock * kScanPer;
    const int nsums = (int)((n + per_blk - 1) / per_blk);
    hipLaunchKernelGGL(scan_blocks, dim3(nsums), dim3(kScanBlock), 0, st, in, out, n, sums);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanBlock), 0, st, sums, nsums);
    hipLaunchKernelGGL(scan_add, dim3(nsums), dim3(kScanBlock), 0, st, out, n, (const int *)sums);
    RIOP_HIP(hipGetLastError());
}

template <typename R> static void build_layout_t(riop_plan *p, const void *uv, hipStream_t st) {
    const int64_t M = p->M;
    const int K = p->K, T = p->tile, tps = p->tiles_per_side, ntiles = p->ntiles, J = p->J;
    const int64_t nkeys = (int64_t)K * K;
    p->perm.alloc(sizeof(int32_t) * M);
    p->cell.alloc(sizeof(uint32_t) * M);
    p->frac.alloc(sizeof(R) * 2 * M);
    p->tile_start.alloc(sizeof(int32_t) * (ntiles + 1));
    p->cell_start.alloc(sizeof(int32_t) * (nkeys + 1));
    DevBuf key_a, key_b, val_b, cell_of, frac_of, flag, counts, sums;
    key_a.alloc(sizeof(uint32_t) * M);
    key_b.alloc(sizeof(uint32_t) * M);
    val_b.alloc(sizeof(int) * M);
    cell_of.alloc(sizeof(uint32_t) * M);
    frac_of.alloc(sizeof(R) * 2 * M);
    flag.alloc(sizeof(int));
    const int64_t nblk = std::max<int64_t>(1, (M + kSortTile - 1) / kSortTile);
    const int64_t ncount = 256 * nblk;
    const int64_t per_blk = (int64_t)kScanBlock * kScanPer;
    counts.alloc(sizeof(int) * ncount);
    sums.alloc(sizeof(int) * ((std::max(ncount, nkeys + 1) + per_blk - 1) / per_blk));
    RIOP_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(int), st));
    const int threads = 256;
    const unsigned gM = (unsigned)std::max<int64_t>(1, (M + threads - 1) / threads);
    int *start = p->cell_start.as<int>();
    if (M > 0) {
        hipLaunchKernelGGL(bin_kernel<R>, dim3(gM), dim3(threads), 0, st, static_cast<const R *>(uv), M, K, J, T, tps,
                           (double)K / (2.0 * M_PI), key_a.as<uint32_t>(), cell_of.as<uint32_t>(), frac_of.as<R>(),
                           flag.as<int>());
        RIOP_HIP(hipGetLastError());
        // Stable radix sort of (key, caller index): as many 8-bit passes as
        // the largest key needs; the first pass takes the index implicitly.
        int bits = 1;
        while (bits < 32 && ((int64_t)1 << bits) < nkeys) ++bits;
        const int passes = (bits + 7) / 8;
        uint32_t *kin = key_a.as<uint32_t>(), *kout = key_b.as<uint32_t>();
        int *vin = nullptr, *vout = passes % 2 ? p->perm.as<int>() : val_b.as<int>();
        for (int ps = 0; ps < passes; ++ps) {
            hipLaunchKernelGGL(rs_hist, dim3((unsigned)nblk), dim3(kSortThreads), 0, st, (const uint32_t *)kin, M,
                               8 * ps, (int)nblk, counts.as<int>());
            scan_exclusive(counts.as<int>(), counts.as<int>(), ncount, sums.as<int>(), st);
            hipLaunchKernelGGL(rs_scatter, dim3((unsigned)nblk), dim3(kSortThreads), 0, st, (const uint32_t *)kin,
                               (const int *)vin, M, 8 * ps, (int)nblk, (const int *)counts.as<int>(), kout, vout);
            RIOP_HIP(hipGetLastError());
            std::swap(kin, kout);
            vin = vout;
            vout = vout == p->perm.as<int>() ? val_b.as<int>() : p->perm.as<int>();
        }
        // kin holds the sorted keys, vin == perm.
        RIOP_REQUIRE(vin == p->perm.as<int>(), RIOP_EDEVICE, "radix sort buffer parity");
        hipLaunchKernelGGL(key_starts, dim3((unsigned)((nkeys + 1 + threads - 1) / threads)), dim3(threads), 0, st,
                           (const uint32_t *)kin, M, nkeys, start);
        hipLaunchKernelGGL(gather_layout<R>, dim3(gM), dim3(threads), 0, st, (const int *)p->perm.as<int>(),
                           cell_of.as<uint32_t>(), frac_of.as<R>(), M, p->cell.as<uint32_t>(), p->frac.as<R>());
        RIOP_HIP(hipGetLastError());
    } else {
        hipLaunchKernelGGL(key_starts, dim3((unsigned)((nkeys + 1 + threads - 1) / threads)), dim3(threads), 0, st,
                           (const uint32_t *)key_a.as<uint32_t>(), (int64_t)0, nkeys, start);
        RIOP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(tile_start_from_keys, dim3((ntiles + 1 + 255) / 256), dim3(256), 0, st, (const int *)start,
                       ntiles, T * T, p->tile_start.as<int>());
    RIOP_HIP(hipGetLastError());
    int hflag = 0;
    std::vector<int> ts(ntiles + 1);
    RIOP_HIP(hipMemcpyAsync(&hflag, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOP_HIP(hipMemcpyAsync(ts.data(), p->tile_start.ptr, sizeof(int) * (ntiles + 1), hipMemcpyDeviceToHost, st));
    RIOP_HIP(hipStreamSynchronize(st));
    RIOP_REQUIRE(hflag == 0, RIOP_EINVAL, "uv coordinates must be finite and inside [-pi, pi]");

    // Degridding work units: chunks of at most kUnit visibilities of one tile.
    std::vector<WorkUnit> units;
    int maxc = 0;
    for (int t = 0; t < ntiles; ++t) {
        const int s0 = ts[t], e0 = ts[t + 1];
        for (int c = s0; c < e0; c += kUnit) {
            const int cnt = std::min(kUnit, e0 - c);
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

    // Gridding: sort tiles, heaviest first, each with its visibility range.
    std::vector<std::pair<int, int>> work(ntiles);
    for (int t = 0; t < ntiles; ++t) work[t] = {ts[t + 1] - ts[t], t};
    std::stable_sort(work.begin(), work.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    std::vector<WorkUnit> order(ntiles);
    for (int k = 0; k < ntiles; ++k) {
        const int t = work[k].second;
        order[k] = WorkUnit{t, ts[t], ts[t + 1] - ts[t], 0};
    }
    p->tile_order.alloc(sizeof(WorkUnit) * ntiles);
    RIOP_HIP(hipMemcpyAsync(p->tile_order.ptr, order.data(), sizeof(WorkUnit) * ntiles, hipMemcpyHostToDevice, st));
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
    a.kc = p->kcoef_compact.as<R>();
    a.K = p->K;
    a.T = p->tile;
    a.tps = p->tiles_per_side;
    return a;
}

#define RIOP_J_CASES(MACRO) MACRO(2) MACRO(4) MACRO(6) MACRO(8) MACRO(10) MACRO(12) MACRO(14) MACRO(16)

template <typename R>
static void launch_degrid_from(riop_plan *p, const void *grid, void *y, int order_user, hipStream_t st) {
    if (p->nunits == 0) return;
    GridArgs<R> a = grid_args<R>(p);
    a.grid = const_cast<C<R> *>(static_cast<const C<R> *>(grid));
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

template <typename R> void launch_degrid(riop_plan *p, void *y, int order_user, hipStream_t st) {
    launch_degrid_from<R>(p, p->grid.ptr, y, order_user, st);
}

void check_grid_lds(riop_plan *p) {
    const size_t lds = p->prec == RIOP_F64 ? grid_lds<double>(p->tile, p->J, 2) : grid_lds<float>(p->tile, p->J, 2);
    RIOP_REQUIRE(lds <= p->lds_max, RIOP_ENOTSUP, "gridding tile too large for LDS; use a smaller tile");
}

template <typename R>
static void launch_tiles(riop_plan *p, const void *vals, int order_user, void *out_grid, hipStream_t st,
                         const TileArgs<R> *p2 = nullptr) {
    TileArgs<R> a{};
    a.grid = static_cast<C<R> *>(out_grid);
    a.halo = p->halo.as<C<R>>();
    a.cell = p->cell.as<uint32_t>();
    a.frac = p->frac.as<R>();
    a.perm = p->perm.as<int>();
    a.order = p->tile_order.as<WorkUnit>();
    a.vin = static_cast<const C<R> *>(vals);
    a.kc = p->kcoef_compact.as<R>();
    a.K = p->K;
    a.T = p->tile;
    a.tps = p->tiles_per_side;
    if (p2) {
        RIOP_REQUIRE(!order_user, RIOP_EINVAL, "the fused prox gridding is plan order only");
        a.p2s = p2->p2s;
        a.p2z = p2->p2z;
        a.p2y = p2->p2y;
        a.p2scale = p2->p2scale;
    }
    int waves = grid_waves<R>(p->J);
    if (grid_lds<R>(p->tile, p->J, waves) > p->lds_max) waves = 2;
    const size_t lds = grid_lds<R>(p->tile, p->J, waves);
    RIOP_REQUIRE(lds <= p->lds_max, RIOP_ENOTSUP, "gridding tile too large for LDS");
    TimedScope ts(p, p2 ? KK_GRID_PROX2 : KK_GRID, st);
    const dim3 g(p->ntiles);
    switch (p->J) {
#define GK(JJ)                                                                                            \
    case JJ: {                                                                                            \
        constexpr int WD = grid_waves<R>(JJ);                                                             \
        if (waves == WD) {                                                                                \
            if (p2) hipLaunchKernelGGL((grid_tile<R, JJ, false, WD, true>), g, dim3(64 * WD), lds, st, a);  \
            else if (order_user) hipLaunchKernelGGL((grid_tile<R, JJ, true, WD, false>), g, dim3(64 * WD), lds, st, a); \
            else hipLaunchKernelGGL((grid_tile<R, JJ, false, WD, false>), g, dim3(64 * WD), lds, st, a);    \
        } else {                                                                                          \
            if (p2) hipLaunchKernelGGL((grid_tile<R, JJ, false, 2, true>), g, dim3(128), lds, st, a);        \
            else if (order_user) hipLaunchKernelGGL((grid_tile<R, JJ, true, 2, false>), g, dim3(128), lds, st, a); \
            else hipLaunchKernelGGL((grid_tile<R, JJ, false, 2, false>), g, dim3(128), lds, st, a);          \
        }                                                                                                 \
        break;                                                                                            \
    }
        RIOP_J_CASES(GK)
#undef GK
        default: throw Error{RIOP_ENOTSUP, "unsupported kernel width"};
    }
    RIOP_HIP(hipGetLastError());
    // The halos are added by the adjoint FFT's first pass as it loads the grid.
    p->halo_pending = out_grid;
}

template <typename R> void launch_grid_merge(riop_plan *p, void *grid, hipStream_t st) {
    const int64_t cells = (int64_t)p->ntiles * (p->J - 1) * (2 * p->tile - p->J + 1);
    if (cells > 0) {
        TimedScope ts(p, KK_GRID, st);
        const int threads = 256;
        hipLaunchKernelGGL(grid_merge<R>, dim3((unsigned)((cells + threads - 1) / threads)), dim3(threads), 0, st,
                           static_cast<C<R> *>(grid), (const C<R> *)p->halo.as<C<R>>(), p->K, p->tile, p->J,
                           p->tiles_per_side);
        RIOP_HIP(hipGetLastError());
    }
}

template <typename R> void launch_grid(riop_plan *p, const void *y, int order_user, hipStream_t st) {
    launch_tiles<R>(p, y, order_user, p->grid.ptr, st);
}

// Gridding of the l2-ball prox's output, formed inside the gridding kernel
// from s, z2 (updated in place) and y, all in plan order.
template <typename R>
void launch_grid_prox2(riop_plan *p, const void *s, void *z2, const void *y, const double *scale, hipStream_t st) {
    TileArgs<R> q{};
    q.p2s = static_cast<const C<R> *>(s);
    q.p2z = static_cast<C<R> *>(z2);
    q.p2y = static_cast<const C<R> *>(y);
    q.p2scale = scale;
    launch_tiles<R>(p, nullptr, 0, p->grid.ptr, st, &q);
}

// out_grid = G^T G in_grid: the precomputed planes when the plan holds them,
// else degridding into plan-order scratch, then gridding.
template <typename R> void launch_gram(riop_plan *p, const void *in_grid, void *out_grid, hipStream_t st) {
    if (p->gram.ptr) {
        launch_gram_apply<R>(p, in_grid, out_grid, st);
        return;
    }
    launch_degrid_from<R>(p, in_grid, p->vis.ptr, 0, st);
    launch_tiles<R>(p, p->vis.ptr, 0, out_grid, st);
}

template void launch_gram<float>(riop_plan *, const void *, void *, hipStream_t);
template void launch_gram<double>(riop_plan *, const void *, void *, hipStream_t);
template void launch_degrid<float>(riop_plan *, void *, int, hipStream_t);
template void launch_degrid<double>(riop_plan *, void *, int, hipStream_t);
template void launch_grid<float>(riop_plan *, const void *, int, hipStream_t);
template void launch_grid<double>(riop_plan *, const void *, int, hipStream_t);
template void launch_grid_prox2<float>(riop_plan *, const void *, void *, const void *, const double *, hipStream_t);
template void launch_grid_prox2<double>(riop_plan *, const void *, void *, const void *, const double *, hipStream_t);
template void launch_grid_merge<float>(riop_plan *, void *, hipStream_t);
template void launch_grid_merge<double>(riop_plan *, void *, hipStream_t);
template void launch_fill_zero<float>(void *, size_t, hipStream_t);
template void launch_fill_zero<double>(void *, size_t, hipStream_t);

}  // namespace riop
