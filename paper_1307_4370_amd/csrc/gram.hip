// Precomputed Gram operator H = G^T G of the interpolation matrix, the
// acceleration of the CG x-update the paper proposes (Sec. 4.5 and Sec. 7:
// store G^T G so that CG no longer forms the M-length vector G F D Z p at
// every iteration).
//
// H is real, symmetric and banded: H[c, c + d] is nonzero only for offsets
// d = (da, db) with |da|, |db| < J (grid indices periodic mod K).  The plan
// stores one K x K plane per offset of the half set
//     da = 0, 0 <= db < J   and   1 <= da < J, -J < db < J
// (J + (J - 1)(2J - 1) planes: 113 for J = 8), H_d[c] = H[c, c + d]; the other
// half follows from symmetry, H[c, c - d] = H_d[c - d].
//
// Build: H_d[c] = sum_m w_m(c) w_m(c + d), w_m the separable Kaiser-Bessel
// window weights of visibility m (the plan's own polynomials, so H is the Gram
// of exactly the G that degridding and gridding apply).  One wavefront per
// visibility stages its J x J window weights in LDS and walks the list of
// (cell, partner, offset) triples with both cells inside the window, adding
// products with double-precision atomics into double planes (summed in no
// fixed order); the planes are then rounded to the plan's type.
//
// Apply: out[c] = sum_{d in half} H_d[c] in[c + d] + sum_{d in half, d != 0}
// H_d[c - d] in[c - d], one thread per cell, planes read with unit stride.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace riop {

int gram_planes(int J) { return J + (J - 1) * (2 * J - 1); }

// Offset (da, db) of plane k.
static void gram_offset(int J, int k, int *da, int *db) {
    if (k < J) {
        *da = 0;
        *db = k;
    } else {
        const int r = k - J;
        *da = 1 + r / (2 * J - 1);
        *db = r % (2 * J - 1) - (J - 1);
    }
}

constexpr int kGramWaves = 4;  // wavefronts per build block

template <typename R>
__global__ void __launch_bounds__(64 * kGramWaves)
    gram_build(const uint32_t *__restrict__ cell, const R *__restrict__ frac, const R *__restrict__ kc, long M, int K,
               int J, int nks, const int3 *__restrict__ triples, int ntriples, double *__restrict__ H) {
    __shared__ double wsh[kGramWaves][16 * 16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *wv = wsh[wave];
    const long K2 = (long)K * K;
    const long nwaves = (long)gridDim.x * kGramWaves;
    for (long v = (long)blockIdx.x * kGramWaves + wave; v < M; v += nwaves) {
        const uint32_t cv = cell[v];
        const int a0 = (int)(cv & 0xffffu), b0 = (int)(cv >> 16);
        // 1-D weights of tap t: phi(rho + J/2 - 1 - t) from the pair polynomials
        // (tap t and J - 1 - t share the even part E and odd part O in s = 2 rho - 1).
        double wu = 0.0, wvv = 0.0;
        if (lane < 2 * J) {
            const int axis = lane / J, t = lane % J;
            const R rho = frac[2 * v + axis];
            const R s = R(2) * rho - R(1), u = s * s;
            const int jp = t < J / 2 ? t : J - 1 - t;
            const R *ce = kc + (jp * 2 + 0) * nks;
            const R *co = kc + (jp * 2 + 1) * nks;
            R e = ce[nks - 1], o = co[nks - 1];
            for (int k = nks - 2; k >= 0; --k) {
                e = e * u + ce[k];
                o = o * u + co[k];
            }
            const R wt = t < J / 2 ? e + s * o : e - s * o;
            if (axis == 0) wu = (double)wt;
            else wvv = (double)wt;
        }
        // Window weights w(i, j) = wu_i wv_j into LDS (every lane takes part
        // in each shuffle, so the sources are always active).
        for (int base = 0; base < J * J; base += 64) {
            const int c = base + lane;
            const bool in = c < J * J;
            const int i = in ? c / J : 0, j = in ? c - (c / J) * J : 0;
            const double a = __shfl(wu, i), b = __shfl(wvv, J + j);
            if (in) wv[c] = a * b;
        }
        __builtin_amdgcn_wave_barrier();
        for (int t = lane; t < ntriples; t += 64) {
            const int3 tr = triples[t];  // (cell, partner, plane), cells as i * J + j
            const int i = tr.x / J, j = tr.x - (tr.x / J) * J;
            int ga = a0 + i, gb = b0 + j;
            if (ga >= K) ga -= K;
            if (gb >= K) gb -= K;
            atomicAdd(&H[(long)tr.z * K2 + (long)ga * K + gb], wv[tr.x] * wv[tr.y]);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename R> __global__ void gram_round(const double *__restrict__ Hd, R *__restrict__ H, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        H[i] = (R)Hd[i];
}

__global__ void fill_zero_f64(double *p, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
}

template <typename R>
__global__ void gram_apply(const R *__restrict__ H, const int2 *__restrict__ offs, int nplanes, const C<R> *in,
                           C<R> *out, int K) {
    const long K2 = (long)K * K;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < K2; c += (long)gridDim.x * blockDim.x) {
        const int k1 = (int)(c / K), k2 = (int)(c - (long)k1 * K);
        double ar = 0.0, ai = 0.0;
        for (int d = 0; d < nplanes; ++d) {
            const int2 o = offs[d];
            int f1 = k1 + o.x, f2 = k2 + o.y;
            f1 -= f1 >= K ? K : 0;
            f2 += f2 < 0 ? K : 0;
            f2 -= f2 >= K ? K : 0;
            const long cf = (long)f1 * K + f2;
            const R hf = H[(long)d * K2 + c];
            const C<R> xf = in[cf];
            ar += (double)hf * xf.x;
            ai += (double)hf * xf.y;
            if (d) {
                int b1 = k1 - o.x, b2 = k2 - o.y;
                b1 += b1 < 0 ? K : 0;
                b2 += b2 < 0 ? K : 0;
                b2 -= b2 >= K ? K : 0;
                const long cb = (long)b1 * K + b2;
                const R hb = H[(long)d * K2 + cb];
                const C<R> xb = in[cb];
                ar += (double)hb * xb.x;
                ai += (double)hb * xb.y;
            }
        }
        out[c] = mk<R>((R)ar, (R)ai);
    }
}

template <typename R> static void gram_build_t(riop_plan *p, hipStream_t st) {
    const int J = p->J, K = p->K, np_ = gram_planes(J);
    const long K2 = (long)K * K;
    RIOP_REQUIRE(J <= 16, RIOP_ENOTSUP, "Gram build supports J <= 16");
    // (cell, partner, plane) triples with both cells inside the J x J window.
    std::vector<int3> tri;
    std::vector<int2> offs(np_);
    for (int k = 0; k < np_; ++k) {
        int da, db;
        gram_offset(J, k, &da, &db);
        offs[k] = make_int2(da, db);
        for (int i = 0; i + da < J; ++i)
            for (int j = std::max(0, -db); j < J && j + db < J; ++j)
                tri.push_back(make_int3(i * J + j, (i + da) * J + (j + db), k));
    }
    DevBuf tri_d, Hd;
    tri_d.alloc(sizeof(int3) * tri.size());
    RIOP_HIP(hipMemcpyAsync(tri_d.ptr, tri.data(), sizeof(int3) * tri.size(), hipMemcpyHostToDevice, st));
    p->gram_offs.alloc(sizeof(int2) * np_);
    RIOP_HIP(hipMemcpyAsync(p->gram_offs.ptr, offs.data(), sizeof(int2) * np_, hipMemcpyHostToDevice, st));
    Hd.alloc(sizeof(double) * np_ * K2);
    hipLaunchKernelGGL(fill_zero_f64, dim3(4096), dim3(256), 0, st, Hd.as<double>(), (long)np_ * K2);
    if (p->M > 0) {
        const long blocks = std::min<long>((p->M + kGramWaves - 1) / kGramWaves, 16384);
        hipLaunchKernelGGL((gram_build<R>), dim3((unsigned)blocks), dim3(64 * kGramWaves), 0, st,
                           (const uint32_t *)p->cell.as<uint32_t>(), (const R *)p->frac.as<R>(),
                           (const R *)p->kcoef_compact.as<R>(), (long)p->M, K, J, p->n_even,
                           (const int3 *)tri_d.as<int3>(), (int)tri.size(), Hd.as<double>());
    }
    p->gram.alloc(sizeof(R) * np_ * K2);
    hipLaunchKernelGGL((gram_round<R>), dim3(4096), dim3(256), 0, st, (const double *)Hd.as<double>(), p->gram.as<R>(),
                       (long)np_ * K2);
    RIOP_HIP(hipGetLastError());
    RIOP_HIP(hipStreamSynchronize(st));  // the temporaries go out of scope
    p->gram_nplanes = np_;
}

void gram_build_plan(riop_plan *p, hipStream_t st) {
    RIOP_REQUIRE(p->n_even == p->n_odd || p->n_even == p->n_odd + 1, RIOP_EDEVICE, "kernel polynomial layout");
    if (p->prec == RIOP_F64)
        gram_build_t<double>(p, st);
    else
        gram_build_t<float>(p, st);
}

template <typename R> void launch_gram_apply(riop_plan *p, const void *in_grid, void *out_grid, hipStream_t st) {
    const long K2 = (long)p->K * p->K;
    const int threads = 256;
    const long blocks = std::min<long>((K2 + threads - 1) / threads, 16384);
    TimedScope ts(p, KK_GRAM, st);
    hipLaunchKernelGGL((gram_apply<R>), dim3((unsigned)blocks), dim3(threads), 0, st, (const R *)p->gram.as<R>(),
                       (const int2 *)p->gram_offs.as<int2>(), p->gram_nplanes, static_cast<const C<R> *>(in_grid),
                       static_cast<C<R> *>(out_grid), p->K);
    RIOP_HIP(hipGetLastError());
}

template void launch_gram_apply<float>(riop_plan *, const void *, void *, hipStream_t);
template void launch_gram_apply<double>(riop_plan *, const void *, void *, hipStream_t);

}  // namespace riop
