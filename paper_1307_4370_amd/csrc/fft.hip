// Oversampled unitary 2-D DFT F of the measurement operator (Sec. 5) on the
// K x K grid, K = 2n, with the zero padding Z and gridding correction D folded
// into its first pass and their transposes into the last pass of the adjoint.
//
// Each pass is a batch of 1-D length-K transforms done by one kernel:
// Stockham auto-sort, mixed radix (2, 3, 4, 8), data in registers within a
// stage and exchanged through LDS between stages.  A thread owns the E
// elements jt + e K/E (e = 0..E-1) of its transform at the start and end of
// every stage, so global loads and stores are strided by K/E and coalesce.
//
// Pruning: the forward transforms read only the n nonzero inputs of the padded
// line, the adjoint transforms write only the n outputs that survive the crop.
//
// Passes (grid stored row-major [k1][k2], k1 <-> u, k2 <-> v):
//   Phi      : columns of x (n transforms, strided)  -> tmp [K][n]
//              rows of tmp   (K transforms, contiguous) -> grid [K][K]
//   Phi^dag  : rows of grid  (K transforms, keep n outputs) -> tmp [K][n]
//              columns of tmp (n transforms, keep n outputs) -> x
#include "common.hpp"

namespace riop {

template <typename R> struct FftArgs {
    const C<R> *in;
    C<R> *out;
    const C<R> *tw;      // N twiddles exp(-2 pi i m / N)
    const R *dax;        // factor along the transform axis (n entries), nullable
    const R *dbt;        // factor along the batch axis (nbatch entries), nullable
    long in_ts, in_es;   // strides (in complex elements) between transforms / elements
    long out_ts, out_es;
    // Adjoint row pass of the power-of-two kernel: gridding halos to add on
    // load (nullptr: none), with the gridding tile side, J and tiles per side.
    const C<R> *halo;
    int hT, hJ, htps;
    // CG steps folded into the column passes (power-of-two kernel).  Forward:
    // with cg_r set, the input p is replaced by r + beta p first and written
    // back, beta = sum(cg_part[cg_new]) / sum(cg_part[cg_old]).  Adjoint: with
    // cg_p set, the output q becomes q + 2 p and each block leaves its part of
    // sum Re(conj(p) q) in cg_part[cg_pq] (cg_nred doubles per slot).
    const C<R> *cg_r, *cg_p;
    double *cg_part;
    int cg_nred, cg_old, cg_new, cg_pq;
    int N, nbatch, C, n;
    int pad_in, crop_out;
    int factors_at_input;
    int nstages;
    int radix[kMaxStages];
    R scale;
};

// y_r = sum_s x_s w^(r s), w = exp(SGN 2 pi i / RR)
template <typename R, int RR, int SGN> struct Dft;

template <typename R, int SGN> struct Dft<R, 2, SGN> {
    __device__ static void run(C<R> *x) {
        C<R> a = x[0], b = x[1];
        x[0] = cadd<R>(a, b);
        x[1] = csub<R>(a, b);
    }
};

// multiply by SGN * i
template <typename R, int SGN> __device__ inline C<R> mul_si(C<R> a) {
    return SGN > 0 ? mk<R>(-a.y, a.x) : mk<R>(a.y, -a.x);
}

template <typename R, int SGN> struct Dft<R, 4, SGN> {
    __device__ static void run(C<R> *x) {
        C<R> a = cadd<R>(x[0], x[2]), b = csub<R>(x[0], x[2]);
        C<R> c = cadd<R>(x[1], x[3]), d = mul_si<R, SGN>(csub<R>(x[1], x[3]));
        x[0] = cadd<R>(a, c);
        x[2] = csub<R>(a, c);
        x[1] = cadd<R>(b, d);
        x[3] = csub<R>(b, d);
    }
};

template <typename R, int SGN> struct Dft<R, 8, SGN> {
    __device__ static void run(C<R> *x) {
        C<R> e[4] = {x[0], x[2], x[4], x[6]};
        C<R> o[4] = {x[1], x[3], x[5], x[7]};
        Dft<R, 4, SGN>::run(e);
        Dft<R, 4, SGN>::run(o);
        const R h = R(0.70710678118654752440084436210484903928);
        // w8^1 = (1 + SGN i)/sqrt2, w8^2 = SGN i, w8^3 = (-1 + SGN i)/sqrt2
        C<R> t1 = mk<R>(h * (o[1].x - SGN * o[1].y), h * (o[1].y + SGN * o[1].x));
        C<R> t2 = mul_si<R, SGN>(o[2]);
        C<R> t3 = mk<R>(h * (-o[3].x - SGN * o[3].y), h * (-o[3].y + SGN * o[3].x));
        x[0] = cadd<R>(e[0], o[0]);
        x[4] = csub<R>(e[0], o[0]);
        x[1] = cadd<R>(e[1], t1);
        x[5] = csub<R>(e[1], t1);
        x[2] = cadd<R>(e[2], t2);
        x[6] = csub<R>(e[2], t2);
        x[3] = cadd<R>(e[3], t3);
        x[7] = csub<R>(e[3], t3);
    }
};

template <typename R, int SGN> struct Dft<R, 3, SGN> {
    __device__ static void run(C<R> *x) {
        const R s3 = R(0.86602540378443864676372317075293618347);
        C<R> t = cadd<R>(x[1], x[2]);
        C<R> u = csub<R>(x[1], x[2]);
        C<R> m = mk<R>(x[0].x - R(0.5) * t.x, x[0].y - R(0.5) * t.y);
        C<R> v = mul_si<R, SGN>(cscale<R>(u, s3));
        x[0] = cadd<R>(x[0], t);
        x[1] = cadd<R>(m, v);
        x[2] = csub<R>(m, v);
    }
};

// One Stockham stage of radix RR on the thread's E registers.
template <typename R, int E, int RR, int SGN>
__device__ inline void stage(C<R> (&v)[E], int jt, int NE, int N, int Ns, const C<R> *tw) {
    constexpr int B = E / RR;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = jt + b * NE;
        const int k = j % Ns;
        C<R> x[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r) x[r] = v[b + r * B];
        if (Ns > 1) {
            // One table twiddle per butterfly, w = exp(SGN 2 pi i k / (Ns RR));
            // the others are its powers (products at most three deep), which
            // spares the memory pipeline RR - 2 gathers per butterfly.
            C<R> w[RR];
            w[1] = tw[k * (N / (Ns * RR))];
            if (SGN > 0) w[1].y = -w[1].y;
            if constexpr (RR > 2) w[2] = cmul<R>(w[1], w[1]);
            if constexpr (RR > 3) w[3] = cmul<R>(w[2], w[1]);
            if constexpr (RR > 4) {
                w[4] = cmul<R>(w[2], w[2]);
                w[5] = cmul<R>(w[4], w[1]);
                w[6] = cmul<R>(w[4], w[2]);
                w[7] = cmul<R>(w[4], w[3]);
            }
#pragma unroll
            for (int r = 1; r < RR; ++r) x[r] = cmul<R>(x[r], w[r]);
        }
        Dft<R, RR, SGN>::run(x);
#pragma unroll
        for (int r = 0; r < RR; ++r) v[b + r * B] = x[r];
    }
}

// LDS slot of line position a.  SWZ (lines a multiple of 32 long): the low
// five bits are XORed with bits 3..7, which spreads both the stride-RR
// writes and the unit-stride reads of every exchange over all banks.
template <bool SWZ> __device__ inline int lds_slot(int a) { return SWZ ? a ^ ((a >> 3) & 31) : a; }

template <typename R, int E, bool SWZ = false>
__device__ inline void exchange(C<R> (&v)[E], C<R> *lds, int ls, int jt, int NE, int Ns, int RR) {
    // v[b + r*B] holds output r of butterfly j = jt + b*NE, destined for
    // position (j - k) * RR + k + r * Ns with k = j mod Ns.
    const int B = E / RR;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int b = e % B, r = e / B;
        const int j = jt + b * NE;
        const int k = j % Ns;
        lds[lds_slot<SWZ>((j - k) * RR + k + r * Ns) * ls] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[lds_slot<SWZ>(jt + e * NE) * ls];
}

// Sum of one double per thread over the block, returned to every thread.
// `red` holds at least ceil(blockDim.x / 64) doubles of LDS; brackets its use
// with barriers.  blockDim.x is a power of two; blocks narrower than a
// wavefront (the column pass of 16-point lines has 32 threads) shuffle only
// within their own lanes.
__device__ inline double block_sum_all(double v, double *red) {
    const int width = blockDim.x < 64 ? (int)blockDim.x : 64;
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Map line index i of a padded length-N line to its source index in [0, n),
// or -1 inside the zero band: pixel j sits at line index (j - n/2) mod N.
__device__ inline int band_index(int i, int N, int n) {
    const int h = n >> 1;
    if (i < h) return i + h;
    if (i >= N - h) return i - (N - h);
    return -1;
}

// Row passes run 256-thread blocks, at least 4 (radix-2^k lines) or 2 (wider
// register sets) resident per CU.
template <typename R, int E> constexpr int fft_row_blocks() { return E == 8 ? 4 : 2; }
// Column blocks: up to 1024 threads, 512 for the 24-element lines, whose
// register sets would otherwise spill at 1024 threads (128 registers).
template <int E> constexpr int fft_col_threads() { return E == 24 ? 512 : 1024; }

template <typename R, int E, int SGN, bool COLS>
__global__ void __launch_bounds__(COLS ? fft_col_threads<E>() : 256, COLS ? 1 : (fft_row_blocks<R, E>()))
    fft_pass(FftArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    const int N = a.N;
    const int NE = N / E;
    int c, jt;
    if (COLS) {
        c = threadIdx.x % a.C;
        jt = threadIdx.x / a.C;
    } else {
        c = threadIdx.x / NE;
        jt = threadIdx.x % NE;
    }
    // Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
    // range of transforms so neighbouring columns share its L2.
    int blk = blockIdx.x;
    if (COLS) {
        const int nb = gridDim.x, qq = nb >> 3, rr = nb & 7, x = blk & 7;
        blk = x * qq + min(x, rr) + (blk >> 3);
    }
    const long t = (long)blk * a.C + c;
    const bool active = t < a.nbatch;
    C<R> *lds = COLS ? smem + c : smem + (long)c * N;
    const int ls = COLS ? a.C : 1;

    C<R> v[E];
    const R tf = (active && a.dbt && a.factors_at_input) ? a.dbt[t] : R(1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = jt + e * NE;
        const int j = a.pad_in ? band_index(i, N, a.n) : i;
        C<R> z = mk<R>(0, 0);
        if (active && j >= 0) {
            z = a.in[t * a.in_ts + (long)j * a.in_es];
            if (a.factors_at_input) {
                R f = a.scale * tf;
                if (a.dax) f *= a.dax[j];
                z = cscale<R>(z, f);
            }
        }
        v[e] = z;
    }

    int Ns = 1;
    for (int s = 0; s < a.nstages; ++s) {
        const int RR = a.radix[s];
        if (s > 0) exchange<R, E>(v, lds, ls, jt, NE, Ns, a.radix[s - 1]);
        if (s > 0) Ns *= a.radix[s - 1];
        switch (RR) {
            case 8: if constexpr (E % 8 == 0) stage<R, E, 8, SGN>(v, jt, NE, N, Ns, a.tw); break;
            case 4: if constexpr (E % 4 == 0) stage<R, E, 4, SGN>(v, jt, NE, N, Ns, a.tw); break;
            case 3: if constexpr (E % 3 == 0) stage<R, E, 3, SGN>(v, jt, NE, N, Ns, a.tw); break;
            default: if constexpr (E % 2 == 0) stage<R, E, 2, SGN>(v, jt, NE, N, Ns, a.tw); break;
        }
    }

    if (!active) return;
    const R tf_out = (a.dbt && !a.factors_at_input) ? a.dbt[t] : R(1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = jt + e * NE;
        const int j = a.crop_out ? band_index(i, N, a.n) : i;
        if (j < 0) continue;
        C<R> z = v[e];
        if (!a.factors_at_input) {
            R f = a.scale * tf_out;
            if (a.dax) f *= a.dax[j];
            z = cscale<R>(z, f);
        }
        a.out[t * a.out_ts + (long)j * a.out_es] = z;
    }
}

// ---------------------------------------------------------------------------
// Power-of-two lengths, N = 2^LOGN, 16 <= N <= 16384: the same pass with the
// stage sequence fixed at compile time (radix 8 while 8 divides what is left,
// then one radix-4 or radix-2 stage), so every index, stride and twiddle step
// is a constant and k = j mod Ns is a mask.

template <int N, int Ns> __host__ __device__ constexpr int p2_radix() {
    return (N / Ns) % 8 == 0 ? 8 : (N / Ns) % 4 == 0 ? 4 : 2;
}
template <typename R, int E, int SGN, int N, int Ns>
__device__ inline void p2_stages(C<R> (&v)[E], int jt, C<R> *lds, int ls, const C<R> *tw) {
    constexpr int RR = p2_radix<N, Ns>(), NE = N / E;
    stage<R, E, RR, SGN>(v, jt, NE, N, Ns, tw);
    if constexpr (Ns * RR < N) {
        exchange<R, E, (N % 32 == 0)>(v, lds, ls, jt, NE, Ns, RR);
        p2_stages<R, E, SGN, N, Ns * RR>(v, jt, lds, ls, tw);
    }
}

// The operator's four passes are fixed by (SGN, COLS), and the p2 kernel
// specialises to them: forward passes read the padded line, whose n = N/2
// inputs sit at line positions [0, N/4) and [3N/4, N), i.e. elements e < 2
// and e >= 6 of every thread (elements 2..5 are zero and not loaded);
// adjoint passes write only those positions; column passes carry the
// gridding correction and 1/K (forward: on input, adjoint: on output).  Rows
// are contiguous (element stride 1), columns adjacent (transform stride 1),
// so every element offset is a 32-bit index.
template <typename R, int LOGN, int SGN, bool COLS>
__global__ void __launch_bounds__(COLS ? 1024 : 256, COLS ? 1 : (fft_row_blocks<R, 8>()))
fft_pass_p2(FftArgs<R> a) {
    constexpr int N = 1 << LOGN, E = 8, NE = N / E;
    constexpr bool FWD = SGN < 0;
    extern __shared__ unsigned char smem_raw[];
    C<R> *smem = reinterpret_cast<C<R> *>(smem_raw);
    int c, jt;
    if (COLS) {
        c = threadIdx.x % a.C;
        jt = threadIdx.x / a.C;
    } else {
        c = threadIdx.x / NE;
        jt = threadIdx.x % NE;
    }
    int blk = blockIdx.x;
    if (COLS) {  // contiguous transform ranges per XCD (blocks are dealt round-robin to the 8 XCDs)
        const int nb = gridDim.x, qq = nb >> 3, rr = nb & 7, x = blk & 7;
        blk = x * qq + min(x, rr) + (blk >> 3);
    }
    const long t = (long)blk * a.C + c;
    const bool active = t < a.nbatch;
    C<R> *lds = COLS ? smem + c : smem + (long)c * N;
    const int ls = COLS ? a.C : 1;
    // Pixel index of band element e (e < 2 or e >= 6) of this thread.
    auto band = [&](int e) { return e < 2 ? jt + e * NE + N / 4 : jt + e * NE - 3 * N / 4; };

    const C<R> *src = COLS ? a.in + t : a.in + t * a.in_ts;
    const int ies = COLS ? (int)a.in_es : 1;
    C<R> v[E];
    if constexpr (FWD) {
        const R f0 = (COLS && active) ? a.scale * a.dbt[t] : R(1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            v[e] = mk<R>(0, 0);
            if ((e < 2 || e >= 6) && active) v[e] = src[band(e) * ies];
        }
        if constexpr (COLS) {
            if (a.cg_r) {
                // CG direction p = r + beta p, beta = rr_new / rr_old (0 when
                // rr_old = 0), reduced while the line's loads are in flight.
                C<R> rv[E];
#pragma unroll
                for (int e = 0; e < E; ++e)
                    rv[e] = ((e < 2 || e >= 6) && active) ? a.cg_r[t + (long)band(e) * ies] : mk<R>(0, 0);
                // Each wavefront sums the partials itself (no barrier): lane
                // strides, then an XOR butterfly, whose partner lanes add the
                // same two values, so every wavefront gets the identical sums.
                const int width = blockDim.x < 64 ? (int)blockDim.x : 64;
                double so = 0.0, sn = 0.0;
                for (int i = threadIdx.x & 63; i < a.cg_nred; i += width) {
                    so += a.cg_part[a.cg_old * a.cg_nred + i];
                    sn += a.cg_part[a.cg_new * a.cg_nred + i];
                }
                for (int o = width >> 1; o > 0; o >>= 1) {
                    so += __shfl_xor(so, o);
                    sn += __shfl_xor(sn, o);
                }
                const double beta = so == 0.0 ? 0.0 : sn / so;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if ((e < 2 || e >= 6) && active) {
                        const C<R> z = v[e];
                        v[e] = mk<R>((R)((double)rv[e].x + beta * z.x), (R)((double)rv[e].y + beta * z.y));
                        const_cast<C<R> *>(a.in)[t + (long)band(e) * ies] = v[e];
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e)
                if ((e < 2 || e >= 6) && active) v[e] = cscale<R>(v[e], f0 * a.dax[band(e)]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = active ? src[(jt + e * NE) * ies] : mk<R>(0, 0);
        if constexpr (!COLS) {
            // Gridding halos: a tile's first J - 1 rows and columns receive
            // what the tiles above, to the left and above-left left in their
            // halo cells, added in that order.  The row's left and above-left
            // parts (J - 1 values per tile) are first gathered into this
            // row's LDS line at a stride W = 8 or 16 per tile, which the
            // first exchange overwrites only after its leading barrier; host
            // side: 2 W tps <= N, so each thread gathers at most 4.
            if (a.halo) {
                const int T = a.hT, J1 = a.hJ - 1, tps = a.htps, lt = __builtin_ctz(T);
                const int lw = J1 <= 8 ? 3 : 4, NL = tps << lw;
                // Halo layout (gridding): the right strips by grid row, so
                // the left parts of row k1 are one contiguous run of
                // tps (J - 1) cells; then the bottom strips (with the corner)
                // tile by tile, BC = (J - 1)(T + J - 1) cells each.
                const int BC = J1 * (T + J1);
                const int k1 = (int)t, dr = k1 >> lt, i = k1 & (T - 1);
                const int upr = dr == 0 ? tps - 1 : dr - 1;
                const C<R> *hrow = a.halo + (long)k1 * tps * J1;                            // left parts
                const C<R> *hup = a.halo + (long)tps * tps * T * J1 + (long)upr * tps * BC +
                                  i * (T + J1);                                             // above, above-left
                // The above tile's part (rows i < J - 1), loaded with the
                // line so that the latencies overlap.
                C<R> up[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int k2 = jt + e * NE, dc = k2 >> lt, j = k2 & (T - 1);
                    up[e] = (active && i < J1) ? hup[dc * BC + j] : mk<R>(0, 0);
                }
                C<R> hl[4], hu[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int f = jt + q * NE, dc = f >> lw, j = f & ((1 << lw) - 1);
                    const int lc = dc == 0 ? tps - 1 : dc - 1;
                    const bool use = active && f < NL && j < J1;
                    hl[q] = use ? hrow[lc * J1 + j] : mk<R>(0, 0);
                    hu[q] = (use && i < J1) ? hup[lc * BC + T + j] : mk<R>(0, 0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int f = jt + q * NE;
                    if (f < NL) {
                        lds[f] = hl[q];
                        lds[NL + f] = hu[q];
                    }
                }
                __syncthreads();
                if (active) {
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int k2 = jt + e * NE, dc = k2 >> lt, j = k2 & (T - 1);
                        if (i < J1) v[e] = cadd<R>(v[e], up[e]);
                        if (j < J1) v[e] = cadd<R>(v[e], lds[(dc << lw) + j]);
                        if (i < J1 && j < J1) v[e] = cadd<R>(v[e], lds[NL + (dc << lw) + j]);
                    }
                }
            }
        }
    }
    p2_stages<R, E, SGN, N, 1>(v, jt, lds, ls, a.tw);
    C<R> *dst = COLS ? a.out + t : a.out + t * a.out_ts;
    const int oes = COLS ? (int)a.out_es : 1;
    if constexpr (FWD) {
        if (!active) return;
#pragma unroll
        for (int e = 0; e < E; ++e) dst[(jt + e * NE) * oes] = v[e];
    } else {
        double acc = 0.0;  // CG: sum Re(conj(p) q) over this thread's outputs
        if (active) {
            const R f0 = COLS ? a.scale * a.dbt[t] : R(1);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e >= 2 && e < 6) continue;
                const int j = band(e);
                C<R> z = v[e];
                if constexpr (COLS) {
                    z = cscale<R>(z, f0 * a.dax[j]);
                    if (a.cg_p) {  // q + 2 p
                        const C<R> pv = a.cg_p[t + (long)j * oes];
                        z.x += R(2) * pv.x;
                        z.y += R(2) * pv.y;
                        acc += (double)pv.x * z.x + (double)pv.y * z.y;
                    }
                }
                dst[j * oes] = z;
            }
        }
        if constexpr (COLS) {
            if (a.cg_p) {
                acc = block_sum_all(acc, reinterpret_cast<double *>(smem));
                double *slot = a.cg_part + (long)a.cg_pq * a.cg_nred;
                if (threadIdx.x == 0) slot[blockIdx.x] = acc;
                if (blockIdx.x == 0)  // entries past the grid's blocks
                    for (int i = gridDim.x + threadIdx.x; i < a.cg_nred; i += blockDim.x) slot[i] = 0.0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host side.

static int elems_per_thread(const FftPlan &f) { return f.E; }

// Transforms per column-pass block: as many as 64 KB of LDS and 1024 threads
// allow, at most 16.
static int col_block_transforms(const FftPlan &f, size_t cbytes) {
    const int threads = f.E == 24 ? fft_col_threads<24>() : fft_col_threads<8>();
    const int Cb = (int)std::min<size_t>((64 * 1024) / (cbytes * (size_t)f.N), threads / (f.N / f.E));
    return std::max(1, std::min(Cb, 16));
}

void build_fft_plan(riop_plan *p, hipStream_t st) {
    FftPlan &f = p->fft;
    const int N = p->K;
    f.N = N;
    int m = N, threes = 0;
    while (m % 3 == 0) {
        m /= 3;
        ++threes;
    }
    RIOP_REQUIRE((m & (m - 1)) == 0 && m >= 8, RIOP_ENOTSUP,
                 "grid side K = 2n must be 2^a 3^b with 2^a >= 8");
    f.nstages = 0;
    int rest = m;
    while (rest >= 8) {
        f.radix[f.nstages++] = 8;
        rest /= 8;
    }
    if (rest == 4) f.radix[f.nstages++] = 4;
    if (rest == 2) f.radix[f.nstages++] = 2;
    for (int i = 0; i < threes; ++i) f.radix[f.nstages++] = 3;
    RIOP_REQUIRE(f.nstages <= kMaxStages, RIOP_ENOTSUP, "too many FFT stages");
    f.E = threes ? 24 : 8;
    RIOP_REQUIRE(N % f.E == 0, RIOP_ENOTSUP, "grid side not divisible by the FFT thread width");
    // One line per row-pass block of at most 256 threads, E points each, and
    // the line held in LDS.
    RIOP_REQUIRE(N / f.E <= 256, RIOP_ENOTSUP,
                 "grid side K = 2n too large for the FFT passes (K <= 2048 for powers of two, "
                 "K <= 6144 with factors of 3)");
    RIOP_REQUIRE(cbytes(p) * (size_t)N <= p->lds_max, RIOP_ENOTSUP, "one FFT line does not fit in LDS");

    // Twiddles exp(-2 pi i m / N) from double-precision sin/cos.
    const size_t cb = cbytes(p);
    std::vector<double> tw(2 * (size_t)N);
    for (int k = 0; k < N; ++k) {
        // Reduce the angle to [0, pi/4]-ish accuracy by exact symmetries is not
        // needed: cos/sin of 2 pi k / N in double are accurate to ~1 ulp.
        const double ang = -2.0 * M_PI * (double)k / (double)N;
        tw[2 * k] = cos(ang);
        tw[2 * k + 1] = sin(ang);
    }
    f.twiddle.alloc(cb * N);
    if (p->prec == RIOP_F64) {
        RIOP_HIP(hipMemcpyAsync(f.twiddle.ptr, tw.data(), cb * N, hipMemcpyHostToDevice, st));
    } else {
        std::vector<float> t32(2 * (size_t)N);
        for (size_t i = 0; i < t32.size(); ++i) t32[i] = (float)tw[i];
        RIOP_HIP(hipMemcpyAsync(f.twiddle.ptr, t32.data(), cb * N, hipMemcpyHostToDevice, st));
    }
    RIOP_HIP(hipStreamSynchronize(st));
}

template <typename R, int SGN, bool COLS>
static bool launch_pass(riop_plan *p, FftArgs<R> a, int kind, hipStream_t st) {
    const FftPlan &f = p->fft;
    a.N = f.N;
    a.nstages = f.nstages;
    for (int i = 0; i < f.nstages; ++i) a.radix[i] = f.radix[i];
    a.tw = f.twiddle.as<C<R>>();
    const int E = elems_per_thread(f);
    const int NE = f.N / E;
    const size_t lds_budget = 64 * 1024;
    const size_t line = sizeof(C<R>) * (size_t)f.N;
    int Cb;
    if (COLS) {
        Cb = col_block_transforms(f, sizeof(C<R>));
    } else {
        Cb = std::max(1, 256 / NE);
        Cb = (int)std::max<size_t>(1, std::min<size_t>(Cb, lds_budget / line));
    }
    RIOP_REQUIRE(COLS || Cb * NE <= 256, RIOP_ENOTSUP, "FFT row block too large");
    a.C = Cb;
    const int threads = Cb * NE;
    RIOP_REQUIRE(threads <= 1024, RIOP_ENOTSUP, "FFT block too large");
    const int N = f.N;
    const bool pow2 = (N & (N - 1)) == 0 && N >= 16 && N <= 16384;
    const int blocks = (a.nbatch + Cb - 1) / Cb;
    const size_t lds = line * Cb;
    // CG steps ride only on the power-of-two column kernel, with at most one
    // partial per block.
    bool fused = false;
    if (a.cg_r || a.cg_p) {
        fused = COLS && pow2 && E == 8 && blocks <= a.cg_nred && (threads & (threads - 1)) == 0;
        if (!fused) a.cg_r = a.cg_p = nullptr;
    }
    TimedScope ts(p, kind, st);
    if (pow2 && E == 8) {
        // The specialised kernel's layout and band assumptions (see above).
        const bool fwd = SGN < 0;
        RIOP_REQUIRE(2 * a.n == N && a.pad_in == (fwd ? 1 : 0) && a.crop_out == (fwd ? 0 : 1) &&
                         (COLS ? (a.in_ts == 1 && a.out_ts == 1 && a.dax && a.dbt)
                               : (a.in_es == 1 && a.out_es == 1 && !a.dax && !a.dbt && a.scale == R(1))),
                     RIOP_EINVAL, "FFT pass layout not supported by the power-of-two kernel");
        switch (N) {
#define P2(LG)                                                                                        \
    case 1 << LG:                                                                                     \
        hipLaunchKernelGGL((fft_pass_p2<R, LG, SGN, COLS>), dim3(blocks), dim3(threads), lds, st, a); \
        break;
            P2(4) P2(5) P2(6) P2(7) P2(8) P2(9) P2(10) P2(11) P2(12) P2(13) P2(14)
#undef P2
        }
    } else if (E == 8) {
        hipLaunchKernelGGL((fft_pass<R, 8, SGN, COLS>), dim3(blocks), dim3(threads), lds, st, a);
    } else {
        hipLaunchKernelGGL((fft_pass<R, 24, SGN, COLS>), dim3(blocks), dim3(threads), lds, st, a);
    }
    RIOP_HIP(hipGetLastError());
    return fused;
}

bool fft_folds_cg(const riop_plan *p, int nred) {
    const FftPlan &f = p->fft;
    const int N = f.N;
    if ((N & (N - 1)) != 0 || N < 16 || N > 16384 || f.E != 8) return false;
    const int Cb = col_block_transforms(f, cbytes(p));
    return (p->n + Cb - 1) / Cb <= nred;
}

template <typename R>
bool launch_phi_fft_forward(riop_plan *p, const void *x, hipStream_t st, const CgFuse<R> *cg) {
    const int n = p->n, K = p->K;
    const R *d = p->deapod.as<R>();
    // Pass 1: columns q of x, transform over p; pad, correct by d(p) d(q), scale 1/K.
    FftArgs<R> a{};
    a.in = static_cast<const C<R> *>(x);
    a.out = p->tmp.as<C<R>>();
    a.in_ts = 1;
    a.in_es = n;
    a.out_ts = 1;
    a.out_es = n;
    a.nbatch = n;
    a.n = n;
    a.pad_in = 1;
    a.crop_out = 0;
    a.dax = d;
    a.dbt = d;
    a.factors_at_input = 1;
    a.scale = R(1) / R(K);
    if (cg && cg->r) {
        a.cg_r = cg->r;
        a.cg_part = cg->part;
        a.cg_nred = cg->nred;
        a.cg_old = cg->slot_old;
        a.cg_new = cg->slot_new;
    }
    const bool fused = launch_pass<R, -1, true>(p, a, KK_FFT_FWD_COL, st);
    // Pass 2: rows k1 of tmp, transform over q (padded) -> grid row k1.
    FftArgs<R> b{};
    b.in = p->tmp.as<C<R>>();
    b.out = p->grid.as<C<R>>();
    b.in_ts = n;
    b.in_es = 1;
    b.out_ts = K;
    b.out_es = 1;
    b.nbatch = K;
    b.n = n;
    b.pad_in = 1;
    b.crop_out = 0;
    b.factors_at_input = 1;
    b.scale = R(1);
    launch_pass<R, -1, false>(p, b, KK_FFT_FWD_ROW, st);
    return fused;
}

template <typename R>
bool launch_phi_fft_adjoint(riop_plan *p, void *x, hipStream_t st, const void *grid, const CgFuse<R> *cg) {
    const int n = p->n, K = p->K;
    const R *d = p->deapod.as<R>();
    // Pass 1: rows k1 of grid, inverse transform over k2, keep the n cropped outputs.
    FftArgs<R> a{};
    a.in = grid ? static_cast<const C<R> *>(grid) : p->grid.as<C<R>>();
    // A grid just written by gridding still lacks its tiles' halos: the
    // specialised row pass adds them on load, otherwise they are merged first.
    if (p->halo_pending) {
        const int N = p->fft.N;
        const bool p2 = (N & (N - 1)) == 0 && N >= 16 && N <= 16384 && p->fft.E == 8;
        const int w = p->J - 1 <= 8 ? 8 : 16;
        if (p2 && p->halo_pending == a.in && 2 * w * p->tiles_per_side <= N) {
            a.halo = p->halo.as<C<R>>();
            a.hT = p->tile;
            a.hJ = p->J;
            a.htps = p->tiles_per_side;
        } else {
            launch_grid_merge<R>(p, p->halo_pending, st);
        }
        p->halo_pending = nullptr;
    }
    a.out = p->tmp.as<C<R>>();
    a.in_ts = K;
    a.in_es = 1;
    a.out_ts = n;
    a.out_es = 1;
    a.nbatch = K;
    a.n = n;
    a.pad_in = 0;
    a.crop_out = 1;
    a.factors_at_input = 0;
    a.scale = R(1);
    launch_pass<R, +1, false>(p, a, KK_FFT_ADJ_ROW, st);
    // Pass 2: columns q of tmp, inverse over k1, crop to p, correct by d(p) d(q), 1/K.
    FftArgs<R> b{};
    b.in = p->tmp.as<C<R>>();
    b.out = static_cast<C<R> *>(x);
    b.in_ts = 1;
    b.in_es = n;
    b.out_ts = 1;
    b.out_es = n;
    b.nbatch = n;
    b.n = n;
    b.pad_in = 0;
    b.crop_out = 1;
    b.dax = d;
    b.dbt = d;
    b.factors_at_input = 0;
    b.scale = R(1) / R(K);
    if (cg && cg->p) {
        b.cg_p = cg->p;
        b.cg_part = cg->part;
        b.cg_nred = cg->nred;
        b.cg_pq = cg->slot_pq;
    }
    return launch_pass<R, +1, true>(p, b, KK_FFT_ADJ_COL, st);
}

template bool launch_phi_fft_forward<float>(riop_plan *, const void *, hipStream_t, const CgFuse<float> *);
template bool launch_phi_fft_forward<double>(riop_plan *, const void *, hipStream_t, const CgFuse<double> *);
template bool launch_phi_fft_adjoint<float>(riop_plan *, void *, hipStream_t, const void *, const CgFuse<float> *);
template bool launch_phi_fft_adjoint<double>(riop_plan *, void *, hipStream_t, const void *,
                                             const CgFuse<double> *);

}  // namespace riop
