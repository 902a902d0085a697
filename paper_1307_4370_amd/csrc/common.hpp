// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/riop.h"

namespace riop {

// ---------------------------------------------------------------------------
// Complex values: interleaved (re, im) of the plan's real type.
template <typename R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename R> using C = typename cplx_t<R>::type;

template <typename R> __host__ __device__ inline C<R> mk(R re, R im) {
    C<R> z;
    z.x = re;
    z.y = im;
    return z;
}
template <typename R> __device__ inline C<R> cadd(C<R> a, C<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R> __device__ inline C<R> csub(C<R> a, C<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R> __device__ inline C<R> cmul(C<R> a, C<R> b) {
    return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R> __device__ inline C<R> cscale(C<R> a, R s) { return mk<R>(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------
// Error handling: every entry point converts failures into a riop_status and a
// thread-local message.
void set_error(const char *fmt, ...);
void clear_error();

struct Error {
    riop_status status;
    std::string msg;
};

#define RIOP_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            throw ::riop::Error{e_ == hipErrorOutOfMemory ? RIOP_ENOMEM : RIOP_EDEVICE,        \
                                std::string(#call) + ": " + hipGetErrorString(e_)};           \
        }                                                                                     \
    } while (0)

#define RIOP_REQUIRE(cond, status, msg)                                                       \
    do {                                                                                      \
        if (!(cond)) throw ::riop::Error{status, msg};                                        \
    } while (0)

// Device memory held by the library's allocations in this process, and the
// limit on it: the environment variable RIOP_DEVICE_MEMORY_LIMIT (bytes,
// read at every allocation; unset or 0 = no limit).  An allocation that would
// pass the limit fails with RIOP_ENOMEM exactly as a failed hipMalloc does.
size_t device_bytes_held();
void account_alloc(size_t bytes);    // throws RIOP_ENOMEM past the limit
void account_free(size_t bytes);

// Device allocation owned by a plan.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 256;
        account_alloc(b);
        const hipError_t e = hipMalloc(&ptr, b);
        if (e != hipSuccess) {
            ptr = nullptr;
            account_free(b);
            throw Error{e == hipErrorOutOfMemory ? RIOP_ENOMEM : RIOP_EDEVICE,
                        std::string("hipMalloc: ") + hipGetErrorString(e)};
        }
        bytes = b;
    }
    // Keeps the current buffer (and its address) when it is at least b bytes.
    void reserve(size_t b) {
        if (!ptr || bytes < b) alloc(b);
    }
    void release() {
        if (ptr) {
            (void)hipFree(ptr);
            account_free(bytes);
        }
        ptr = nullptr;
        bytes = 0;
    }
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

// One gridding work unit: a tile and a contiguous chunk of its visibilities.
struct WorkUnit {
    int32_t tile;
    int32_t start;  // plan-order index of the first visibility
    int32_t count;
    int32_t pad;
};

constexpr int kMaxStages = 10;
constexpr int kMaxPoly = 24;  // coefficients per even/odd part

// FFT plan for one transform length.
struct FftPlan {
    int N = 0;
    int E = 0;              // elements per thread
    int nstages = 0;
    int radix[kMaxStages] = {};
    DevBuf twiddle;         // N complex: exp(-2 pi i m / N)
};

// Kernel kinds for event timing.
enum KernelKind {
    KK_FFT_FWD_COL = 0, KK_FFT_FWD_ROW, KK_FFT_ADJ_ROW, KK_FFT_ADJ_COL,
    KK_DEGRID, KK_GRID, KK_GRID_ZERO, KK_PSI_ADJ, KK_PSI, KK_VECTOR, KK_GRID_PROX2, KK_GRAM, KK_COUNT
};

struct Timing {
    bool on = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[KK_COUNT] = {};
    int64_t launches[KK_COUNT] = {};
    ~Timing();
    hipEvent_t get();
    void flush();
};

// Device-side SDMM workspace (allocated on first use).
struct SdmmWork {
    bool ready = false;
    DevBuf xhat, rhs, r, p, qp, tmpN, x1, z3loc;
    DevBuf z1loc, w1;       // q*N complex
    DevBuf ysort, z2loc, s2; // M complex, plan order
    DevBuf partials;        // doubles for block reductions
    DevBuf f1part;          // per analysis block partials of f1 (psi_adj_blocks doubles)
    int f1_count = 0;
    DevBuf scalars;         // doubles: scalar slots
    // Block SDMM (R data blocks): each visibility's block in plan order
    // (int32 M), per-block eps, ball scale and nu (R doubles each), and the
    // reduction blocks' partial norms (kRedBlocks * 2R doubles).
    int nblocks = 0;
    DevBuf blk, beps, bscale, bnu, bpart, bflag;
    // Prior of the l1 step: 0 = analysis l1 over the SARA dictionary (L1 =
    // Psi^dagger), 1 = weighted TV (L1 = I, prox by fast gradient projection
    // on the dual with tv_inner iterations; buffers N complex each).
    int prior = 0;
    int tv_inner = 0;
    DevBuf tvb, tvu, tvp, tvq, tvr, tvs;
    DevBuf rw_w;            // reweighted l1: the current weights (q*N reals)
    DevBuf xprev;           // reweighted l1: the previous pass's solution (N complex)
    DevBuf history;         // doubles, kHistStride per iteration
    int hist_cap = 0;       // iterations the history buffer holds (grows only)
    int n_cg = 0;
    double cg_tol = 0.0;
    const void *weights = nullptr;
    bool initialised = false;
    // Incremented whenever something a captured iteration depends on changes
    // (a workspace address, n_cg, the weights pointer): a graph captured from
    // riop_sdmm_step is valid while the epoch it was captured at is current.
    uint64_t epoch = 0;
};

// Doubles per iteration in the SDMM history: f1, zeta, nu, final CG <r, r>,
// CG iterations used.
constexpr int kHistStride = 5;

}  // namespace riop

struct riop_plan {
    riop_desc desc{};
    int device = 0;
    int n = 0, K = 0, J = 0, L = 0, q = 0, prec = 0;
    int64_t M = 0;
    uint32_t mask = 0;
    int bases[9] = {};
    double scale_q = 1.0;  // 1/sqrt(q)

    // Visibility layout (plan order).
    int tile = 0, tiles_per_side = 0, ntiles = 0;
    size_t lds_max = 65536;     // LDS bytes one workgroup may use on the plan's device
    riop::DevBuf perm;        // int32[M]
    riop::DevBuf cell;        // uint32[M]: a0 | b0 << 16
    riop::DevBuf frac;        // R[2M]: (rho_u, rho_v)
    riop::DevBuf tile_start;  // int32[ntiles + 1]
    riop::DevBuf units;       // WorkUnit[nunits] (degridding)
    riop::DevBuf cell_start;  // int32[K^2 + 1]: plan-order start of each cell key
    riop::DevBuf tile_order;  // WorkUnit[ntiles]: tiles with their visibility ranges, heaviest first (gridding)
    riop::DevBuf halo;        // per tile: region cells outside the tile (gridding)
    void *halo_pending = nullptr;  // grid last written by gridding, its tiles' halos not yet added
    int nunits = 0;
    int max_unit = 0;

    // Kaiser-Bessel kernel: per tap pair even/odd polynomial coefficients.
    double kb_beta = 0;
    int kdeg = 0;                // degree of the per-tap polynomial in s
    int n_even = 0, n_odd = 0;   // coefficients in the even / odd parts
    double kfit_err = 0;
    riop::DevBuf kcoef_compact;  // R[J/2][2][D/2 + 1] compact copy
    riop::DevBuf deapod;         // R[n]: d(p - n/2)

    // FFT.
    riop::FftPlan fft;

    // Workspaces.
    riop::DevBuf tmp;    // K x n complex
    riop::DevBuf grid;   // K x K complex
    riop::DevBuf grid2;  // K x K complex: output grid of the fused Gram kernel
    riop::DevBuf vis;    // M complex, plan order scratch
    riop::DevBuf img;    // n x n complex scratch

    // SARA.
    riop::DevBuf filters;   // R[9][16] low-pass filters (index = basis)
    int flen[9] = {};
    riop::DevBuf ll;        // per-basis low-low scratch (analysis / synthesis)
    size_t ll_stride = 0;   // complex entries per basis in `ll`

    // Precomputed Gram operator G^T G (optional): one K x K plane of the
    // plan's real type per offset of the half set, and the offsets (int2).
    riop::DevBuf gram, gram_offs;
    int gram_nplanes = 0;

    riop::SdmmWork sd;
    riop::Timing timing;
    int64_t device_bytes = 0;

    // Sticky flag set on the device when a caller input holds a NaN or Inf
    // (int, device); read and cleared by the next call that synchronises.
    riop::DevBuf nonfinite;
    // Recorded on the stream of the plan's last (uncaptured) call, so that
    // destroying the plan waits for its own work only (created with the plan).
    hipEvent_t done = nullptr;

    riop_plan() = default;
    riop_plan(const riop_plan &) = delete;
    riop_plan &operator=(const riop_plan &) = delete;
    ~riop_plan() {
        if (done) (void)hipEventDestroy(done);
    }
};

namespace riop {

inline size_t cbytes(const riop_plan *p) { return p->prec == RIOP_F64 ? 16 : 8; }
inline size_t rbytes(const riop_plan *p) { return p->prec == RIOP_F64 ? 8 : 4; }

// Launch helpers implemented in the kernel translation units.  All take the
// plan's real type as a template parameter and enqueue on `st`.
// CG steps the column FFT passes can fold in (CG on Q = Phi^dagger Phi + 2 I,
// Sec. 4.4): before a forward transform of p, the direction update
// p <- r + beta p with beta = sum(part[slot_new]) / sum(part[slot_old]) (0 when
// the old sum is 0); after an adjoint transform into q, q <- q + 2 p with the
// per-block partials of sum Re(conj(p) q) left in part[slot_pq].  `part` holds
// nred doubles per slot.
template <typename R> struct CgFuse {
    const C<R> *r = nullptr;  // residual (direction update), nullable
    const C<R> *p = nullptr;  // direction (p.q), nullable
    double *part = nullptr;
    int nred = 0, slot_old = 0, slot_new = 0, slot_pq = 0;
};
// Whether the column passes fold in the CG steps of CgFuse with nred partials
// per slot (the power-of-two kernel with at most nred column blocks).
bool fft_folds_cg(const riop_plan *p, int nred);
// Forward FFT passes; returns whether cg->r's direction update was folded in
// (false: the caller must apply it first; nothing was done).
template <typename R>
bool launch_phi_fft_forward(riop_plan *p, const void *x, hipStream_t st, const CgFuse<R> *cg = nullptr);
// Adjoint FFT passes; `grid` selects the input grid (nullptr: the plan's grid).
// Returns whether cg->p's q + 2 p and p.q partials were folded in.
template <typename R>
bool launch_phi_fft_adjoint(riop_plan *p, void *x, hipStream_t st, const void *grid = nullptr,
                            const CgFuse<R> *cg = nullptr);
// out_grid = G^T G in_grid (fused degrid + grid, the Gram part of Phi^dagger Phi).
// Throws RIOP_ENOTSUP if the plan's gridding tile needs more LDS than the device has.
void check_grid_lds(riop_plan *p);
// Complex halo cells of one gridding tile (right strip and bottom strip).
inline int grid_halo_cells(int T, int J) { return T * (J - 1) + (J - 1) * (T + J - 1); }
template <typename R> void launch_gram(riop_plan *p, const void *in_grid, void *out_grid, hipStream_t st);
// Precomputed G^T G: planes per offset for width J, build (synchronises) and apply.
int gram_planes(int J);
void gram_build_plan(riop_plan *p, hipStream_t st);
template <typename R> void launch_gram_apply(riop_plan *p, const void *in_grid, void *out_grid, hipStream_t st);
// Adds the gridding halos into `grid` (needed only where the adjoint FFT does
// not add them while loading; see launch_phi_fft_adjoint).
template <typename R> void launch_grid_merge(riop_plan *p, void *grid, hipStream_t st);
template <typename R>
void launch_degrid(riop_plan *p, void *y, int order_user, hipStream_t st);
template <typename R>
void launch_grid(riop_plan *p, const void *y, int order_user, hipStream_t st);
template <typename R>
void launch_grid_prox2(riop_plan *p, const void *s, void *z2, const void *y, const double *scale, hipStream_t st);
template <typename R> void launch_fill_zero(void *buf, size_t ncomplex, hipStream_t st);
template <typename R> void launch_psi_adj(riop_plan *p, const void *x, void *alpha, hipStream_t st);
template <typename R> void launch_psi(riop_plan *p, const void *alpha, void *x, hipStream_t st);

// SDMM l1 step fused into the last analysis pass (Algorithm 1, steps 7-9, i = 1).
template <typename R> struct Prox1 {
    C<R> *z1;          // dual variable, updated in place
    C<R> *w1;          // r1 - z1 (new), input of the synthesis
    const R *weights;  // diagonal of W, nullable (W = I)
    const double *gamma;
    double *f1_part;   // one partial of f1 = sum w |Psi^dagger x| per analysis block
};
// Number of analysis blocks (all levels and the Dirac plane) of one Psi^dagger.
int psi_adj_blocks(const riop_plan *p);
template <typename R>
void launch_psi_adj_prox(riop_plan *p, const void *x, const Prox1<R> &px, hipStream_t st);

// Brackets the kernel launches of its lifetime with timing events when the
// plan's timing is enabled.
struct TimedScope {
    riop_plan *p;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    TimedScope(riop_plan *p_, int kind_, hipStream_t s_);
    ~TimedScope();
};

// Launch a check of nreal reals at v (caller input) that sets the plan's
// sticky non-finite flag; v may be NULL.
void check_finite_input(riop_plan *p, const void *v, int64_t nreal, hipStream_t st);
// Synchronise `st`; if the plan's non-finite flag is set, clear it and throw
// RIOP_ENONFINITE.
void report_nonfinite(riop_plan *p, hipStream_t st);
// Record the plan's completion event on `st` (not while `st` is capturing).
void mark_done(riop_plan *p, hipStream_t st);

void build_fft_plan(riop_plan *p, hipStream_t st);
void build_layout(riop_plan *p, const void *uv, hipStream_t st);
void build_kernel_tables(riop_plan *p);
void build_filters(riop_plan *p);

}  // namespace riop
