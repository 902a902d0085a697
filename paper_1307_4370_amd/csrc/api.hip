// C entry points, plan construction and the host-side tables of the library:
//   * Kaiser-Bessel kernel (Beatty-Nishimura-Pauly width rule for oversampling
//     2) fitted per tap by a polynomial in the fractional offset, and the
//     gridding correction d = 1 / phihat (Sec. 5: D with d = 1/g-hat);
//   * Daubechies DbN scaling filters by spectral factorisation of Daubechies'
//     half-band polynomial, roots found with the Durand-Kerner iteration.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <new>

#include "common.hpp"

namespace riop {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// Device-memory accounting and the RIOP_DEVICE_MEMORY_LIMIT hook.

static std::atomic<size_t> g_held{0};

size_t device_bytes_held() { return g_held.load(); }

void account_alloc(size_t bytes) {
    size_t limit = 0;
    if (const char *e = std::getenv("RIOP_DEVICE_MEMORY_LIMIT")) limit = (size_t)std::strtoull(e, nullptr, 10);
    const size_t now = g_held.fetch_add(bytes) + bytes;
    if (limit && now > limit) {
        g_held.fetch_sub(bytes);
        throw Error{RIOP_ENOMEM, "device allocation refused: RIOP_DEVICE_MEMORY_LIMIT (" + std::to_string(limit) +
                                     " bytes) would be exceeded"};
    }
}

void account_free(size_t bytes) { g_held.fetch_sub(bytes); }

// ---------------------------------------------------------------------------
// Finiteness of caller inputs.  A NaN or an infinity fails x - x == 0.

template <typename R> __global__ void finite_check_kernel(const R *__restrict__ v, int64_t n, int *flag) {
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += 4 * stride) {
        R a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = i + u * stride < n ? v[i + u * stride] : R(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) bad |= !(a[u] - a[u] == R(0));
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

void check_finite_input(riop_plan *p, const void *v, int64_t nreal, hipStream_t st) {
    if (!v || nreal <= 0) return;
    const int threads = 256;
    const int64_t blocks = std::min<int64_t>((nreal + 4 * threads - 1) / (4 * threads), 2048);
    if (p->prec == RIOP_F64)
        hipLaunchKernelGGL(finite_check_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, st,
                           static_cast<const double *>(v), nreal, p->nonfinite.as<int>());
    else
        hipLaunchKernelGGL(finite_check_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, st,
                           static_cast<const float *>(v), nreal, p->nonfinite.as<int>());
    RIOP_HIP(hipGetLastError());
}

void report_nonfinite(riop_plan *p, hipStream_t st) {
    int flag = 0;
    RIOP_HIP(hipMemcpyAsync(&flag, p->nonfinite.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOP_HIP(hipStreamSynchronize(st));
    if (flag) {
        RIOP_HIP(hipMemsetAsync(p->nonfinite.ptr, 0, sizeof(int), st));
        RIOP_HIP(hipStreamSynchronize(st));
        throw Error{RIOP_ENONFINITE, "a NaN or Inf was found in an input of this plan's calls"};
    }
}

void mark_done(riop_plan *p, hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (p->done) RIOP_HIP(hipEventRecord(p->done, st));
}

// ---------------------------------------------------------------------------
// Event timing.

Timing::~Timing() {
    for (auto &e : pending) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

hipEvent_t Timing::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    RIOP_HIP(hipEventCreate(&e));
    return e;
}

void Timing::flush() {
    for (auto &e : pending) {
        RIOP_HIP(hipEventSynchronize(e.second.second));
        float ms = 0;
        RIOP_HIP(hipEventElapsedTime(&ms, e.second.first, e.second.second));
        total_ms[e.first] += ms;
        launches[e.first] += 1;
        pool.push_back(e.second.first);
        pool.push_back(e.second.second);
    }
    pending.clear();
}

TimedScope::TimedScope(riop_plan *p_, int kind_, hipStream_t s_) : p(p_), kind(kind_), s(s_) {
    if (!p->timing.on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    a = p->timing.get();
    RIOP_HIP(hipEventRecord(a, s));
}

TimedScope::~TimedScope() {
    if (!a) return;
    try {
        hipEvent_t b = p->timing.get();
        (void)hipEventRecord(b, s);
        p->timing.pending.push_back({kind, {a, b}});
    } catch (...) {
    }
}

static const char *kKindNames[KK_COUNT] = {"fft_fwd_col", "fft_fwd_row", "fft_adj_row", "fft_adj_col",
                                           "degrid",      "grid",        "grid_zero",   "psi_adj",
                                           "psi",         "vector",      "grid_prox2",  "gram"};

// ---------------------------------------------------------------------------
// Kaiser-Bessel kernel on the host.

static double bessel_i0(double z) {
    // Power series sum_k (z/2)^(2k) / (k!)^2; all terms positive.
    const double q = 0.25 * z * z;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

static double kb_phi(double t, int J, double beta, double i0b) {
    const double r = 1.0 - (2.0 * t / J) * (2.0 * t / J);
    if (r < 0) return 0.0;
    return bessel_i0(beta * std::sqrt(r)) / i0b;
}

static double kb_phihat(double l, int J, int K, double beta, double i0b) {
    const double s = M_PI * J * l / K;
    const double w = std::sqrt(beta * beta - s * s);
    return J * std::sinh(w) / (w * i0b);
}

void build_kernel_tables(riop_plan *p) {
    const int J = p->J, K = p->K, n = p->n;
    const double alpha = 2.0;
    const double beta = M_PI * std::sqrt((J / alpha) * (J / alpha) * (alpha - 0.5) * (alpha - 0.5) - 0.8);
    const double i0b = bessel_i0(beta);
    p->kb_beta = beta;
    const int D = p->prec == RIOP_F64 ? 14 : 7;
    p->kdeg = D;
    p->n_even = D / 2 + 1;
    p->n_odd = (D + 1) / 2;
    // Chebyshev interpolation of f(s) = phi((s + 1)/2 + J/2 - 1 - jp) on [-1, 1].
    std::vector<double> coef((size_t)(J / 2) * 2 * kMaxPoly, 0.0);
    double worst = 0.0;
    for (int jp = 0; jp < J / 2; ++jp) {
        auto f = [&](double s) { return kb_phi((s + 1.0) / 2.0 + J / 2.0 - 1.0 - jp, J, beta, i0b); };
        std::vector<double> fx(D + 1), cheb(D + 1, 0.0);
        for (int i = 0; i <= D; ++i) fx[i] = f(std::cos(M_PI * (i + 0.5) / (D + 1)));
        for (int k = 0; k <= D; ++k) {
            double acc = 0;
            for (int i = 0; i <= D; ++i) acc += fx[i] * std::cos(M_PI * k * (i + 0.5) / (D + 1));
            cheb[k] = acc * 2.0 / (D + 1);
        }
        cheb[0] *= 0.5;
        // Chebyshev -> monomial in s through T_{k+1} = 2 s T_k - T_{k-1}.
        std::vector<double> mono(D + 1, 0.0), tkm1(D + 1, 0.0), tk(D + 1, 0.0), tkp1(D + 1, 0.0);
        tkm1[0] = 1.0;
        mono[0] += cheb[0];
        if (D >= 1) {
            tk[1] = 1.0;
            mono[1] += cheb[1];
        }
        for (int k = 1; k < D; ++k) {
            std::fill(tkp1.begin(), tkp1.end(), 0.0);
            for (int i = 0; i < D; ++i) tkp1[i + 1] += 2.0 * tk[i];
            for (int i = 0; i <= D; ++i) tkp1[i] -= tkm1[i];
            for (int i = 0; i <= D; ++i) mono[i] += cheb[k + 1] * tkp1[i];
            tkm1 = tk;
            tk = tkp1;
        }
        double *ce = &coef[(size_t)(jp * 2 + 0) * kMaxPoly];
        double *co = &coef[(size_t)(jp * 2 + 1) * kMaxPoly];
        for (int i = 0; i <= D; ++i) (i % 2 == 0 ? ce[i / 2] : co[i / 2]) = mono[i];
        // Verify both taps of the pair (s and -s) on a dense grid, evaluating the
        // split form in the plan's precision.
        for (int i = 0; i <= 4000; ++i) {
            const double s = -1.0 + i / 2000.0;
            double ev, od;
            if (p->prec == RIOP_F64) {
                double u = s * s, e = ce[p->n_even - 1], o = co[p->n_odd - 1];
                for (int k = p->n_even - 2; k >= 0; --k) e = e * u + ce[k];
                for (int k = p->n_odd - 2; k >= 0; --k) o = o * u + co[k];
                ev = e;
                od = o;
            } else {
                float sf = (float)s, u = sf * sf, e = (float)ce[p->n_even - 1], o = (float)co[p->n_odd - 1];
                for (int k = p->n_even - 2; k >= 0; --k) e = e * u + (float)ce[k];
                for (int k = p->n_odd - 2; k >= 0; --k) o = o * u + (float)co[k];
                ev = e;
                od = o;
            }
            worst = std::max(worst, std::fabs(ev + s * od - f(s)));
            worst = std::max(worst, std::fabs(ev - s * od - f(-s)));
        }
    }
    p->kfit_err = worst;
    const double target = p->prec == RIOP_F64 ? 1e-13 : 1e-7;
    RIOP_REQUIRE(worst <= target, RIOP_ENOTSUP, "kernel polynomial fit not accurate enough for this width");
    // Gridding correction d(l) for l = p - n/2.
    std::vector<double> d(n);
    for (int i = 0; i < n; ++i) d[i] = 1.0 / kb_phihat(i - n / 2, J, K, beta, i0b);
    const size_t rb = rbytes(p);
    // Device table [pair][even/odd][D/2 + 1] in the plan's type, read by the
    // gridding, degridding and Gram kernels.
    const int KS = D / 2 + 1;
    std::vector<double> compact((size_t)(J / 2) * 2 * KS, 0.0);
    for (int jp = 0; jp < J / 2; ++jp)
        for (int e = 0; e < 2; ++e)
            for (int k = 0; k < KS; ++k) compact[(size_t)(jp * 2 + e) * KS + k] = coef[(size_t)(jp * 2 + e) * kMaxPoly + k];
    p->kcoef_compact.alloc(rb * compact.size());
    if (p->prec == RIOP_F64) {
        RIOP_HIP(hipMemcpy(p->kcoef_compact.ptr, compact.data(), rb * compact.size(), hipMemcpyHostToDevice));
    } else {
        std::vector<float> c32(compact.begin(), compact.end());
        RIOP_HIP(hipMemcpy(p->kcoef_compact.ptr, c32.data(), rb * c32.size(), hipMemcpyHostToDevice));
    }
    p->deapod.alloc(rb * n);
    if (p->prec == RIOP_F64) {
        RIOP_HIP(hipMemcpy(p->deapod.ptr, d.data(), rb * n, hipMemcpyHostToDevice));
    } else {
        std::vector<float> d32(d.begin(), d.end());
        RIOP_HIP(hipMemcpy(p->deapod.ptr, d32.data(), rb * n, hipMemcpyHostToDevice));
    }
}

// ---------------------------------------------------------------------------
// Daubechies filters.

using cd = std::complex<double>;

// All roots of sum_k a[k] z^k (a[deg] != 0) by the Durand-Kerner iteration.
static std::vector<cd> poly_roots(const std::vector<double> &a) {
    const int deg = (int)a.size() - 1;
    std::vector<cd> z(deg);
    const cd seed(0.4, 0.9);
    for (int i = 0; i < deg; ++i) z[i] = std::pow(seed, i);
    auto eval = [&](cd x) {
        cd v = a[deg];
        for (int k = deg - 1; k >= 0; --k) v = v * x + a[k];
        return v;
    };
    for (int it = 0; it < 5000; ++it) {
        double moved = 0;
        for (int i = 0; i < deg; ++i) {
            cd den = a[deg];
            for (int j = 0; j < deg; ++j)
                if (j != i) den *= (z[i] - z[j]);
            const cd step = eval(z[i]) / den;
            z[i] -= step;
            moved = std::max(moved, std::abs(step));
        }
        if (moved < 1e-16) break;
    }
    // Newton polish.
    for (int i = 0; i < deg; ++i) {
        for (int it = 0; it < 4; ++it) {
            cd v = a[deg], dv = 0;
            for (int k = deg - 1; k >= 0; --k) {
                dv = dv * z[i] + v;
                v = v * z[i] + a[k];
            }
            if (std::abs(dv) > 0) z[i] -= v / dv;
        }
    }
    return z;
}

static std::vector<double> daubechies(int N) {
    if (N == 1) return {M_SQRT1_2, M_SQRT1_2};
    // P(y) = sum_{k<N} C(N-1+k, k) y^k with y = (2 - z - 1/z)/4; multiply by
    // z^(N-1) to get an ordinary polynomial Q(z) of degree 2N-2.
    std::vector<double> Pc(N);
    for (int k = 0; k < N; ++k) {
        double c = 1;
        for (int i = 1; i <= k; ++i) c = c * (N - 1 + i) / i;
        Pc[k] = c;
    }
    // y as a Laurent polynomial: coefficients of z^-1, z^0, z^1.
    std::vector<double> Q(2 * N - 1, 0.0);  // index e + (N-1) for power e in [-(N-1), N-1]
    std::vector<double> yk(2 * N - 1, 0.0);
    yk[N - 1] = 1.0;  // y^0
    for (int k = 0; k < N; ++k) {
        for (int e = 0; e < 2 * N - 1; ++e) Q[e] += Pc[k] * yk[e];
        std::vector<double> nx(2 * N - 1, 0.0);
        for (int e = 0; e < 2 * N - 1; ++e) {
            if (yk[e] == 0) continue;
            if (e - 1 >= 0) nx[e - 1] += -0.25 * yk[e];
            nx[e] += 0.5 * yk[e];
            if (e + 1 < 2 * N - 1) nx[e + 1] += -0.25 * yk[e];
        }
        yk = nx;
    }
    std::vector<cd> roots = poly_roots(Q);
    std::vector<cd> inside;
    for (const cd &r : roots)
        if (std::abs(r) < 1.0) inside.push_back(r);
    RIOP_REQUIRE((int)inside.size() == N - 1, RIOP_EDEVICE, "Daubechies factorisation failed");
    // H(z) = (1 + z)^N prod (z - r), increasing powers.
    std::vector<cd> H(1, cd(1.0));
    auto mul = [&](cd root) {  // multiply by (z - root)
        std::vector<cd> out(H.size() + 1, cd(0.0));
        for (size_t i = 0; i < H.size(); ++i) {
            out[i + 1] += H[i];
            out[i] -= root * H[i];
        }
        H = out;
    };
    for (int i = 0; i < N; ++i) mul(cd(-1.0));
    for (const cd &r : inside) mul(r);
    std::vector<double> h(2 * N);
    double sum = 0;
    for (int i = 0; i < 2 * N; ++i) {
        h[i] = H[2 * N - 1 - i].real();  // reverse: Daubechies' orientation
        sum += h[i];
    }
    for (double &v : h) v *= M_SQRT2 / sum;
    // Self-check: double-shift orthonormality.
    for (int m = 0; m < N; ++m) {
        double s = 0;
        for (int k = 0; k + 2 * m < 2 * N; ++k) s += h[k] * h[k + 2 * m];
        RIOP_REQUIRE(std::fabs(s - (m == 0 ? 1.0 : 0.0)) < 1e-12, RIOP_EDEVICE, "Daubechies filter check failed");
    }
    return h;
}

void build_filters(riop_plan *p) {
    constexpr int kTaps = 16;
    std::vector<double> f(9 * 2 * kTaps, 0.0);
    for (int b = 1; b <= 8; ++b) {
        if (!(p->mask >> b & 1)) continue;
        std::vector<double> h = daubechies(b);
        const int L = 2 * b;
        for (int m = 0; m < L; ++m) {
            f[(b * 2 + 0) * kTaps + m] = h[m];
            f[(b * 2 + 1) * kTaps + m] = ((m & 1) ? -1.0 : 1.0) * h[L - 1 - m];
        }
        p->flen[b] = L;
    }
    const size_t rb = rbytes(p);
    p->filters.alloc(rb * f.size());
    if (p->prec == RIOP_F64) {
        RIOP_HIP(hipMemcpy(p->filters.ptr, f.data(), rb * f.size(), hipMemcpyHostToDevice));
    } else {
        std::vector<float> f32(f.begin(), f.end());
        RIOP_HIP(hipMemcpy(p->filters.ptr, f32.data(), rb * f32.size(), hipMemcpyHostToDevice));
    }
}

static int default_tile(int K, int J) {
    int t = K >= 256 ? 32 : (K >= 64 ? 16 : 8);
    while (t < J) t *= 2;
    return t;
}

static void validate(const riop_desc *d) {
    RIOP_REQUIRE(d, RIOP_EINVAL, "desc is NULL");
    RIOP_REQUIRE(d->oversample == 2, RIOP_ENOTSUP, "only oversampling 2 is supported");
    RIOP_REQUIRE(d->n >= 8 && d->n <= 3072 && d->n % 2 == 0, RIOP_ESHAPE, "n must be even, 8..3072");
    RIOP_REQUIRE(d->M >= 0 && d->M < (int64_t(1) << 31), RIOP_ESHAPE, "M must be in [0, 2^31)");
    RIOP_REQUIRE(d->J >= 2 && d->J <= 16 && d->J % 2 == 0, RIOP_EINVAL, "J must be even, 2..16");
    RIOP_REQUIRE(2 * d->n >= 2 * d->J, RIOP_ESHAPE, "grid too small for the kernel width");
    RIOP_REQUIRE(d->levels >= 1 && d->levels <= 12, RIOP_EINVAL, "levels must be 1..12");
    RIOP_REQUIRE(d->n % (1 << d->levels) == 0, RIOP_ESHAPE, "n must be divisible by 2^levels");
    RIOP_REQUIRE(d->dict_mask != 0 && d->dict_mask < (1u << 9), RIOP_EINVAL, "dict_mask must be in [1, 2^9)");
    RIOP_REQUIRE(d->prec == RIOP_F32 || d->prec == RIOP_F64, RIOP_EINVAL, "prec must be RIOP_F32 or RIOP_F64");
    for (int i = 0; i < 7; ++i) RIOP_REQUIRE(d->reserved[i] == 0, RIOP_EINVAL, "reserved fields must be zero");
    if (d->tile) {
        const int t = d->tile;
        RIOP_REQUIRE(t >= 8 && t <= 64 && (t & (t - 1)) == 0 && (2 * d->n) % t == 0, RIOP_EINVAL,
                     "tile must be a power of two in [8, 64] dividing 2n");
    }
}

}  // namespace riop

using namespace riop;

template <typename F> static riop_status guarded(F &&f) {
    try {
        clear_error();
        f();
        return RIOP_OK;
    } catch (const Error &e) {
        set_error("%s", e.msg.c_str());
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return RIOP_ENOMEM;
    } catch (...) {
        set_error("unexpected failure");
        return RIOP_EDEVICE;
    }
}

static hipStream_t S(void *s) { return static_cast<hipStream_t>(s); }

static void check_plan(const riop_plan *p) {
    RIOP_REQUIRE(p, RIOP_EINVAL, "plan is NULL");
    int dev = -1;
    RIOP_HIP(hipGetDevice(&dev));
    RIOP_REQUIRE(dev == p->device, RIOP_EINVAL, "plan belongs to another device than the current one");
}

extern "C" {

const char *riop_last_error(void) { return g_err.c_str(); }

const char *riop_version(void) { return "riop 0.1.0 gfx950"; }

riop_status riop_plan_create(const riop_desc *desc, const void *uv, void *stream, riop_plan **out) {
    if (!out) {
        set_error("out is NULL");
        return RIOP_EINVAL;
    }
    *out = nullptr;
    riop_plan *p = nullptr;
    riop_status st = guarded([&] {
        validate(desc);
        RIOP_REQUIRE(desc->M == 0 || uv, RIOP_EINVAL, "uv is NULL");
        p = new riop_plan();
        p->desc = *desc;
        RIOP_HIP(hipGetDevice(&p->device));
        p->n = desc->n;
        p->K = 2 * desc->n;
        p->J = desc->J;
        p->L = desc->levels;
        p->M = desc->M;
        p->prec = desc->prec;
        p->mask = desc->dict_mask;
        p->q = 0;
        for (int b = 0; b < 9; ++b)
            if (p->mask >> b & 1) p->bases[p->q++] = b;
        p->scale_q = 1.0 / std::sqrt((double)p->q);
        p->tile = desc->tile ? desc->tile : default_tile(p->K, p->J);
        RIOP_REQUIRE(p->tile >= p->J && p->K % p->tile == 0, RIOP_EINVAL,
                     "gridding tile must be at least J and divide 2n");
        {
            int v = 0;
            RIOP_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
            p->lds_max = (size_t)std::max(v, 0);
        }
        check_grid_lds(p);
        p->tiles_per_side = p->K / p->tile;
        p->ntiles = p->tiles_per_side * p->tiles_per_side;
        const hipStream_t s = S(stream);
        build_fft_plan(p, s);
        build_kernel_tables(p);
        build_filters(p);
        const size_t cb = cbytes(p);
        const size_t N = (size_t)p->n * p->n;
        p->tmp.alloc(cb * (size_t)p->K * p->n);
        p->grid.alloc(cb * (size_t)p->K * p->K);
        p->grid2.alloc(cb * (size_t)p->K * p->K);
        p->halo.alloc(cb * (size_t)p->ntiles * grid_halo_cells(p->tile, p->J));
        p->vis.alloc(cb * (size_t)std::max<int64_t>(1, p->M));
        p->img.alloc(cb * N);
        size_t lls = 0;
        for (int j = 1; j < p->L; ++j) lls += (size_t)(p->n >> j) * (p->n >> j);
        p->ll_stride = std::max<size_t>(1, lls);
        p->ll.alloc(cb * p->ll_stride * 8);
        build_layout(p, uv, s);
        p->nonfinite.alloc(sizeof(int));
        RIOP_HIP(hipMemsetAsync(p->nonfinite.ptr, 0, sizeof(int), s));
        RIOP_HIP(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
        RIOP_HIP(hipStreamSynchronize(s));
        p->device_bytes = 0;
        for (const DevBuf *b : {&p->perm, &p->cell, &p->frac, &p->tile_start, &p->units, &p->cell_start,
                                &p->tile_order, &p->halo, &p->kcoef_compact, &p->deapod,
                                &p->fft.twiddle, &p->tmp, &p->grid, &p->grid2, &p->vis, &p->img, &p->filters, &p->ll})
            p->device_bytes += (int64_t)b->bytes;
    });
    if (st != RIOP_OK) {
        delete p;
        return st;
    }
    *out = p;
    return RIOP_OK;
}

riop_status riop_plan_destroy(riop_plan *plan) {
    if (!plan) return RIOP_OK;
    return guarded([&] {
        // Wait for the work the plan's own calls enqueued (its last uncaptured
        // call's stream), not for the whole device.
        if (plan->done) {
            (void)hipEventSynchronize(plan->done);
            (void)hipEventDestroy(plan->done);
            plan->done = nullptr;
        }
        delete plan;
    });
}

riop_status riop_gram_build(riop_plan *p, void *stream) {
    return guarded([&] {
        check_plan(p);
        p->gram.release();
        p->gram_offs.release();
        p->gram_nplanes = 0;
        gram_build_plan(p, S(stream));
        mark_done(p, S(stream));
    });
}

riop_status riop_gram_release(riop_plan *p) {
    return guarded([&] {
        check_plan(p);
        if (p->done) RIOP_HIP(hipEventSynchronize(p->done));
        p->gram.release();
        p->gram_offs.release();
        p->gram_nplanes = 0;
    });
}

riop_status riop_plan_sync(riop_plan *p, void *stream) {
    return guarded([&] {
        check_plan(p);
        report_nonfinite(p, static_cast<hipStream_t>(stream));
    });
}

int64_t riop_device_bytes(void) { return (int64_t)device_bytes_held(); }

double riop_noise_bound(int64_t M, double sigma) {
    // ||n||^2 / (sigma^2 / 2) follows a chi^2 law with 2M degrees of freedom
    // (mean 2M, standard deviation 2 sqrt(M)); eps bounds it two standard
    // deviations above the mean.
    if (M < 0 || !(sigma >= 0)) return NAN;
    const double m = (double)M;
    return std::sqrt((2.0 * m + 4.0 * std::sqrt(m)) * sigma * sigma / 2.0);
}

riop_status riop_plan_info(const riop_plan *p, riop_info *info) {
    return guarded([&] {
        RIOP_REQUIRE(p && info, RIOP_EINVAL, "NULL argument");
        info->n = p->n;
        info->K = p->K;
        info->J = p->J;
        info->levels = p->L;
        info->q = p->q;
        info->prec = p->prec;
        info->M = p->M;
        info->tile = p->tile;
        info->ntiles = p->ntiles;
        info->nunits = p->nunits;
        info->kernel_degree = p->kdeg;
        info->kb_beta = p->kb_beta;
        info->kernel_fit_err = p->kfit_err;
        int64_t extra = 0;
        for (const DevBuf *b : {&p->sd.xhat, &p->sd.rhs, &p->sd.r, &p->sd.p, &p->sd.qp, &p->sd.tmpN, &p->sd.x1,
                                &p->sd.z3loc, &p->sd.z1loc, &p->sd.w1, &p->sd.ysort, &p->sd.z2loc, &p->sd.s2,
                                &p->sd.partials, &p->sd.scalars, &p->sd.history, &p->gram, &p->gram_offs})
            extra += (int64_t)b->bytes;
        info->device_bytes = p->device_bytes + extra;
    });
}

riop_status riop_timing_enable(riop_plan *p, int32_t on) {
    return guarded([&] {
        check_plan(p);
        p->timing.flush();
        p->timing.on = on != 0;
        for (int k = 0; k < KK_COUNT; ++k) {
            p->timing.total_ms[k] = 0;
            p->timing.launches[k] = 0;
        }
    });
}

riop_status riop_timing_read(riop_plan *p, int32_t kind, double *total_ms, int64_t *launches) {
    return guarded([&] {
        check_plan(p);
        RIOP_REQUIRE(kind >= 0 && kind < KK_COUNT, RIOP_EINVAL, "kernel kind out of range");
        p->timing.flush();
        if (total_ms) *total_ms = p->timing.total_ms[kind];
        if (launches) *launches = p->timing.launches[kind];
    });
}

int32_t riop_timing_kinds(void) { return KK_COUNT; }

const char *riop_timing_name(int32_t kind) { return kind >= 0 && kind < KK_COUNT ? kKindNames[kind] : ""; }

riop_status riop_plan_layout(const riop_plan *p, int32_t *perm, uint32_t *cell, int32_t *tile_start,
                             void *stream) {
    return guarded([&] {
        check_plan(p);
        const hipStream_t s = S(stream);
        if (perm && p->M)
            RIOP_HIP(hipMemcpyAsync(perm, p->perm.ptr, sizeof(int32_t) * p->M, hipMemcpyDeviceToDevice, s));
        if (cell && p->M)
            RIOP_HIP(hipMemcpyAsync(cell, p->cell.ptr, sizeof(uint32_t) * p->M, hipMemcpyDeviceToDevice, s));
        if (tile_start)
            RIOP_HIP(hipMemcpyAsync(tile_start, p->tile_start.ptr, sizeof(int32_t) * (p->ntiles + 1),
                                    hipMemcpyDeviceToDevice, s));
    });
}

}  // extern "C"

namespace riop {

template <typename R> void phi_impl(riop_plan *p, const void *x, void *y, int user, hipStream_t s) {
    launch_phi_fft_forward<R>(p, x, s);
    launch_degrid<R>(p, y, user, s);
}
template <typename R> void phi_adj_impl(riop_plan *p, const void *y, void *x, int user, hipStream_t s) {
    launch_grid<R>(p, y, user, s);
    launch_phi_fft_adjoint<R>(p, x, s);
}

}  // namespace riop

extern "C" {

#define RIOP_DISPATCH(p, FN, ...) \
    ((p)->prec == RIOP_F64 ? FN<double>(__VA_ARGS__) : FN<float>(__VA_ARGS__))

riop_status riop_phi(riop_plan *p, const void *x, void *y, void *stream) {
    return guarded([&] {
        check_plan(p);
        RIOP_REQUIRE(x && (y || p->M == 0), RIOP_EINVAL, "NULL data pointer");
        RIOP_REQUIRE(x != y, RIOP_EINVAL, "x and y must not alias");
        check_finite_input(p, x, 2 * (int64_t)p->n * p->n, S(stream));
        RIOP_DISPATCH(p, phi_impl, p, x, y, 1, S(stream));
        mark_done(p, S(stream));
    });
}

riop_status riop_phi_adj(riop_plan *p, const void *y, void *x, void *stream) {
    return guarded([&] {
        check_plan(p);
        RIOP_REQUIRE(x && (y || p->M == 0), RIOP_EINVAL, "NULL data pointer");
        RIOP_REQUIRE(x != y, RIOP_EINVAL, "x and y must not alias");
        check_finite_input(p, y, 2 * p->M, S(stream));
        RIOP_DISPATCH(p, phi_adj_impl, p, y, x, 1, S(stream));
        mark_done(p, S(stream));
    });
}

riop_status riop_phi_sorted(riop_plan *p, const void *x, void *y, void *stream) {
    return guarded([&] {
        check_plan(p);
        RIOP_REQUIRE(x && (y || p->M == 0), RIOP_EINVAL, "NULL data pointer");
        RIOP_REQUIRE(x != y, RIOP_EINVAL, "x and y must not alias");
        check_finite_input(p, x, 2 * (int64_t)p->n * p->n, S(stream));
        RIOP_DISPATCH(p, phi_impl, p, x, y, 0, S(stream));
        mark_done(p, S(stream));
    });
}

riop_status riop_phi_adj_sorted(riop_plan *p, const void *y, void *x, void *stream) {
    return guarded([&] {
        check_plan(p);
        RIOP_REQUIRE(x && (y || p->M == 0), RIOP_EINVAL, "NULL data pointer");
        RIOP_REQUIRE(x != y, RIOP_EINVAL, "x and y must not alias");
        check_finite_input(p, y, 2 * p->M, S(stream));
        RIOP_DISPATCH(p, phi_adj_impl, p, y, x, 0, S(stream));
        mark_done(p, S(stream));
    });
}

riop_status riop_psi_adj(riop_plan *p, const void *x, void *alpha, void *stream) {
    return guarded([&] {
        check_plan(p);
        RIOP_REQUIRE(x && alpha, RIOP_EINVAL, "NULL data pointer");
        RIOP_REQUIRE(x != alpha, RIOP_EINVAL, "x and alpha must not alias");
        check_finite_input(p, x, 2 * (int64_t)p->n * p->n, S(stream));
        RIOP_DISPATCH(p, launch_psi_adj, p, x, alpha, S(stream));
        mark_done(p, S(stream));
    });
}

riop_status riop_psi(riop_plan *p, const void *alpha, void *x, void *stream) {
    return guarded([&] {
        check_plan(p);
        RIOP_REQUIRE(x && alpha, RIOP_EINVAL, "NULL data pointer");
        RIOP_REQUIRE(x != alpha, RIOP_EINVAL, "x and alpha must not alias");
        check_finite_input(p, alpha, 2 * (int64_t)p->q * p->n * p->n, S(stream));
        RIOP_DISPATCH(p, launch_psi, p, alpha, x, S(stream));
        mark_done(p, S(stream));
    });
}

}  // extern "C"
