// libspd host runtime and C ABI (see include/spd.h).
//
// Drivers for Algorithm 1 of the paper (Cholesky with mixed-precision
// iterative refinement, Section 3.1): the blocked low-precision factorisation
// with one panel of lookahead on a second stream, the substitutions, and the
// binary64 refinement loop with its stopping/divergence rules and the
// precision fallback chain (the convergence condition of Eq. (4) is what the
// divergence test guards against).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "spd.h"

#define SPD_TILE_H 128
#define SPD_IB_H 32
#define SPD_INFO_NONE_H 0x7fffffffffffffffULL

struct spd_factor_s {
    int device = 0;
    int64_t n = 0, npad = 0;
    int prec = -1;
    int elem = 0;            // bytes per factor element (4 or 8)
    int nb = 0;              // panel width
    size_t cap_L = 0;        // allocated bytes of L / W / Winv
    void *L = nullptr;       // npad x npad, column-major, lower used
    void *W = nullptr;       // nt blocks NB x NB: inverses of the diagonal blocks
    void *Winv = nullptr;    // npad/32 blocks 32 x 32: inverses of the 32-wide diagonal sub-blocks
    double *d = nullptr;     // n: equilibration
    int64_t cap_d = 0;
    double mu = 1.0;
    int half = HALF_NONE;    // operand rounding of the trailing update (BF16 / FP16 factors)
    int group = 4;           // panels per trailing-update group, binary32/64 (SPD_GROUP overrides)
    int group_half = 8;      // the same for binary16/bfloat16 operands, even, <= 8 (SPD_GROUP_HALF overrides)
    bool small_main = false; // a group's thin trailing updates on 64-tiles too (SPD_SMALL_MAIN=1)
    bool pinned = false;     // schedule fixed by the environment or the tuner: no cache lookup
    int upd_slots = 0;       // cap on the main-stream update's workgroups (SPD_UPD_SLOTS; 0: one per tile)
    bool imported = false;   // the factor came from spd_factor_import (not the method's own factorisation)
    bool info_pending = false;  // spd_posv's factorisation: info not read back yet (read with the first residual)
    void *Lh = nullptr;      // two panel copies in that precision (npad x NB halves each)
    size_t cap_Lh = 0;
    unsigned long long *info_dev = nullptr;
    unsigned long long *info_host = nullptr;  // pinned
    // solve workspace
    void *Y = nullptr, *Z = nullptr;
    size_t cap_YZ = 0;
    double *smax = nullptr;
    int64_t cap_smax = 0;
    // triangular solve state
    void *WB = nullptr;          // inverses of the big diagonal blocks
    size_t cap_WB = 0;
    void *Tb = nullptr;          // scratch of their construction
    size_t cap_Tb = 0;
    void *tP = nullptr;          // partial products
    size_t cap_tP = 0;
    int *tctl = nullptr;         // work-queue head + per-row counters
    int cap_tctl = 0;
    int *terr = nullptr;         // sticky error flag (device)
    unsigned long long wait_ticks = 100000000ULL;  // bounded waits of the solves: 1 s of the 100 MHz clock
    int *terr_host = nullptr;    // pinned mirror
    // refinement workspace
    double *R = nullptr;
    size_t cap_R = 0;
    double *P = nullptr;
    size_t cap_P = 0;
    double *norms = nullptr, *norms_host = nullptr;
    int64_t cap_norms = 0;
    hipStream_t side = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};

// Device memory of spd_residual_noalloc: partial sums, norms, eta and (when
// the caller passes no R) the residual itself.  Each device holds its own copy
// until the process ends; host code uses only the address
// hipGetSymbolAddress returns for it (per device), never the name.
static __device__ __align__(256) char scratch[SPD_NOALLOC_SCRATCH_BYTES];

namespace {

// ---- optional kernel timing (spd_profile_*) ----
struct ProfRec {
    hipEvent_t a, b;
    int kind;
    double flops, bytes;
};
struct ProfTotals {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
ProfTotals g_prof_tot[SPD_K_COUNT];

bool prof_enabled()
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    return g_prof_on;
}

// Returns an event recorded before the launch (or nullptr when disabled).
hipEvent_t prof_begin(hipStream_t st)
{
    if (!g_prof_on) return nullptr;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    hipEventRecord(e, st);
    return e;
}

void prof_end(hipEvent_t a, hipStream_t st, int kind, double flops, double bytes)
{
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return;
    }
    hipEventRecord(b, st);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_pending.push_back({a, b, kind, flops, bytes});
}

// algorithmic work of one trailing-update launch over tile columns [lo, hi)
// Algorithmic work of one trailing-update launch: flops of the lower tiles
// (diagonal tiles count their lower half), bytes = each C tile read and
// written once in the factor type (elem) plus its two operand panels
// (op_elem bytes per element).
void update_work(int t, int lo, int hi, int nbk, int elem, int op_elem, double *flops, double *bytes)
{
    const double T = SPD_TILE_H;
    double f = 0, b = 0;
    for (int c = lo; c < hi; ++c) {
        const double off = t - c - 1;  // off-diagonal tiles in this tile column
        f += off * 2.0 * T * T * nbk + T * (T + 1) * nbk;
        b += (off + 1) * (2.0 * T * T * elem + 2.0 * T * nbk * op_elem);
    }
    *flops = f;
    *bytes = b;
}

spd_status map_err(hipError_t e)
{
    if (e == hipSuccess) return SPD_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SPD_ERR_OUT_OF_MEMORY;
    return SPD_ERR_DEVICE;
}

#define HIP_TRY(x)                                   \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) return map_err(e_);    \
    } while (0)
#define SPD_TRY(x)                                   \
    do {                                             \
        spd_status s_ = (x);                         \
        if (s_ != SPD_OK) return s_;                 \
    } while (0)

spd_opts defaults()
{
    spd_opts o;
    o.tol = 1e-14;
    o.max_iter = 10;
    o.fallback = 1;
    o.equilibrate = 1;
    o.theta = 0.1;
    return o;
}

bool opts_valid(const spd_opts &o)
{
    return o.tol >= 0.0 && o.max_iter >= 0 && o.theta > 0.0 && o.theta <= 1.0;
}

// grow a device buffer (contents not preserved)
spd_status grow(void **p, size_t *cap, size_t bytes, bool zero, hipStream_t st)
{
    if (*cap >= bytes && *p) return SPD_OK;
    if (*p) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    HIP_TRY(hipMalloc(p, bytes ? bytes : 16));
    *cap = bytes;
    if (zero) HIP_TRY(hipMemsetAsync(*p, 0, bytes, st));
    return SPD_OK;
}

spd_status ensure_stream_objs(spd_factor_t F)
{
    if (!F->side) HIP_TRY(hipStreamCreateWithFlags(&F->side, hipStreamNonBlocking));
    for (auto &e : F->ev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (!F->info_dev) HIP_TRY(hipMalloc(&F->info_dev, sizeof(unsigned long long)));
    if (!F->info_host) HIP_TRY(hipHostMalloc(&F->info_host, sizeof(unsigned long long), hipHostMallocDefault));
    return SPD_OK;
}

const char *prec_tag(int p) { return p == SPD_BF16 ? "bf16" : p == SPD_FP16 ? "fp16" : p == SPD_FP32 ? "fp32" : "fp64"; }

double fp16_scale(double theta)
{
    // largest power of two <= theta * 65504
    int e;
    std::frexp(theta * 65504.0, &e);
    return std::ldexp(1.0, e - 1);
}

// ---------------------------------------------------------------------------
// Blocked right-looking factorisation, panels of NB columns, trailing
// updates per group of G panels, one group of lookahead:
//   side stream: the panel chain (each panel's columns updated by the
//                group's earlier panels, its diagonal factor, its panel
//                solve) and the update of the next group's columns;
//   main stream: the update of the remaining trailing columns.
template <typename T>
spd_status factor_blocked(spd_factor_t F, hipStream_t st)
{
    const int64_t NB = spd::Panel<T>::NB, npad = F->npad, nt = npad / NB;
    T *H = (T *)F->L;
    T *Wi = (T *)F->Winv;
    const int64_t wi_blk = (NB / SPD_IB_H) * SPD_IB_H * SPD_IB_H;
    hipEvent_t evU = F->ev[0], evP = F->ev[1];
    // Panels are factored one by one (NB wide) but the trailing update is
    // applied per group of G panels (K = G NB), which cuts the C-tile
    // traffic per flop G-fold.  Lookahead is one group.  With half-precision
    // operands the update is bound by that traffic up to K ~ 1000 (the
    // binary32 C tile against 2.5 PFLOP/s), so their groups are wider and
    // their trailing update runs on 256 x 256 tiles (npad is then a multiple
    // of 256 and G even, so every group's trailing region is whole tiles).
    const int half = (sizeof(T) == 4) ? F->half : HALF_NONE;
    const int64_t G = half ? F->group_half : F->group;
    const int64_t ng = (nt + G - 1) / G;
    const int op_elem = half ? 2 : (int)sizeof(T);
    // half-precision operand copies of panels k mod 16 (two groups), written
    // by the panel solve and read by the updates
    const int64_t lh_slot = npad * NB;  // halves per copy
    auto lh = [&](int64_t k) -> void * {
        return half ? (void *)((char *)F->Lh + (size_t)(k & 15) * lh_slot * 2) : nullptr;
    };
    // H -= L_{.,[p0,p1)} L_{.,[p0,p1)}^T on tile columns [lo, hi) of the
    // region starting at row/column r0
    // the main stream's updates use at most F->upd_slots workgroups (looping
    // over tiles), so that the panel chain always finds free slots
    auto update = [&](int64_t p0, int64_t p1, int64_t r0, int lo, int hi, hipStream_t s, int prio, int kind) {
        const int cap = (s == st && kind == SPD_K_UPDATE) ? F->upd_slots : 0;
        const int t = (int)((npad - r0) / SPD_TILE_H);
        if (t <= 0 || lo >= hi) return;
        hipEvent_t pe = prof_begin(s);
        const int64_t rem = npad - r0;
        // a group's trailing update on the main stream: 256 x 256 tiles, all
        // its panels in one pass.  The side stream's update of the next
        // group's columns lies on the panel chain's path, which bounds a
        // half-precision factorisation: 128-tiles, four times the workgroups
        // at two per compute unit, finish it sooner (binary16 at n = 16384:
        // 11.77 -> 11.55 ms per solve).
        if (half && s == st && p1 - p0 > 1 && rem % 256 == 0 && lo % 2 == 0 && hi % 2 == 0) {
            const int sk0 = (int)((r0 - (p0 + 1) * NB) / SPD_IB_H);
            spd::launch_syrk_update_h256((float *)H, npad, F->Lh, (int)(p0 & 15), lh_slot / 8, sk0, (int)(p1 - p0),
                                         half, r0, (int)(rem / 256), lo / 2, hi / 2, F->info_dev, s, prio, cap);
        } else if (half) {
            // copy of panel p starts at row (p + 1) NB
            const int sk0 = (int)((r0 - (p0 + 1) * NB) / SPD_IB_H);
            spd::launch_syrk_update_half((float *)H, npad, F->Lh, (int)(p0 & 15), lh_slot / 8, sk0, (int)(p1 - p0),
                                         half, r0, t, lo, hi, F->info_dev, s, prio, cap);
        } else {
            // a group's trailing update keeps 128-tiles (64-tiles for the
            // chain's single tile columns): one kernel instance per role
            spd::launch_syrk_update<T>(H, npad, p0 * NB, (int)((p1 - p0) * NB), r0, t, lo, hi, F->info_dev, s, prio,
                                       cap, kind == SPD_K_CHAIN_UPDATE || F->small_main);
        }
        if (pe) {
            double fl, by;
            update_work(t, lo, hi, (int)((p1 - p0) * NB), (int)sizeof(T), op_elem, &fl, &by);
            prof_end(pe, s, kind, fl, by);
        }
    };
    // the panel chain of group g, left-looking inside the group: panel k's
    // columns take the updates of the group's earlier panels in one launch
    // (K up to (G - 1) NB, one tile column), then its diagonal block is
    // factored and the rows below it solved
    auto chain = [&](int64_t g, hipStream_t s) {
        const int64_t p0 = g * G, p1 = std::min<int64_t>((g + 1) * G, nt);
        for (int64_t k = p0; k < p1; ++k) {
            const int64_t r = k * NB;
            if (k > p0) update(p0, k, r, 0, (int)(NB / SPD_TILE_H), s, 1, SPD_K_CHAIN_UPDATE);
            spd::launch_potrf_diag<T>(H + r + r * npad, npad, r, Wi + k * wi_blk, F->info_dev, s);
            spd::launch_trsm_panel<T>(H, npad, r, r + NB, npad - r - NB, Wi + k * wi_blk, F->info_dev, s, lh(k),
                                      half);
        }
    };

    // Per group g: the side stream runs the group's panel chain, then the
    // update of the next group's columns by the group's panels (recorded as
    // evU), then the next group's chain; the main stream, after evU, updates
    // the rest of the trailing columns (recorded as evR), which overlaps the
    // next chain.  The next group's columns take that update only after the
    // main stream's update of the previous group is done (evR), since both
    // write them.  Successive chains are thus joined on one stream, with no
    // hop between streams on the path that bounds the last groups.
    hipEvent_t evR = F->ev[2];
    chain(0, st);
    if (ng > 1) {
        HIP_TRY(hipEventRecord(evP, st));
        HIP_TRY(hipStreamWaitEvent(F->side, evP, 0));
        for (int64_t g = 0; g + 1 < ng; ++g) {
            const int64_t p0 = g * G, p1 = std::min<int64_t>(p0 + G, nt), r0 = p1 * NB;
            const int t = (int)((npad - r0) / SPD_TILE_H);
            int next = (int)((std::min<int64_t>(p1 + G, nt) - p1) * (NB / SPD_TILE_H));
            if (half) next = std::min(t, (next + 1) & ~1);  // whole 256-tile columns on both sides of the split
            if (g > 0) HIP_TRY(hipStreamWaitEvent(F->side, evR, 0));
            update(p0, p1, r0, 0, next, F->side, 1, SPD_K_UPDATE);
            HIP_TRY(hipEventRecord(evU, F->side));
            // enqueued before the chain, so that the main stream never waits on the host
            HIP_TRY(hipStreamWaitEvent(st, evU, 0));
            update(p0, p1, r0, next, t, st, 0, SPD_K_UPDATE);
            HIP_TRY(hipEventRecord(evR, st));
            chain(g + 1, F->side);
        }
        HIP_TRY(hipEventRecord(evP, F->side));
        HIP_TRY(hipStreamWaitEvent(st, evP, 0));
    }
    HIP_TRY(hipGetLastError());
    spd::launch_trtri_blocks<T>(H, npad, nt, Wi, (T *)F->W, st);
    spd::launch_build_winv<T>(H, npad, npad, (const T *)F->W, (T *)F->WB, (T *)F->Tb, st);
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

// sizes and buffers of a factor of order n at precision prec (L, W, Winv
// zeroed when (re)allocated), the solve structures, d; mu and the operand
// rounding from prec
spd_status prepare_factor(spd_factor_t F, int64_t n, int prec, double theta, hipStream_t st)
{
    const int64_t old_npad = F->npad;
    const int old_elem = F->elem;
    F->n = n;
    F->prec = prec;
    F->elem = (prec == SPD_FP64) ? 8 : 4;
    F->nb = (prec == SPD_FP64) ? spd::Panel<double>::NB : spd::Panel<float>::NB;
    // half-precision operands: whole 256 x 256 tiles in every group's trailing region
    const int64_t pad = (prec == SPD_FP16 || prec == SPD_BF16) ? 256 : F->nb;
    F->npad = ((n + pad - 1) / pad) * pad;
    if (F->npad == 0) F->npad = pad;
    const int64_t npad = F->npad;
    SPD_TRY(ensure_stream_objs(F));
    // one allocation for L, W and Winv (all zeroed when (re)allocated)
    const size_t bL = (size_t)npad * npad * F->elem;
    const size_t bW = (size_t)npad * F->nb * F->elem;
    const size_t bWi = (size_t)npad * SPD_IB_H * F->elem;
    size_t cap = F->cap_L;
    void *base = F->L;
    SPD_TRY(grow(&base, &cap, bL + bW + bWi, true, st));
    F->L = base;
    F->cap_L = cap;
    F->W = (char *)base + bL;
    F->Winv = (char *)base + bL + bW;
    size_t capw = F->cap_WB;
    const size_t bWB = (size_t)spd::solve_winv_elems(npad) * F->elem;
    SPD_TRY(grow(&F->WB, &capw, bWB, true, st));
    F->cap_WB = capw;
    // The factorisation writes only the lower parts of W, Winv and WB; the
    // zeros above rely on these buffers being zero there.  Buffers kept from
    // a factor of another layout (npad or element size: a precision switch
    // on the handle) hold that factor's values at those places: clear them.
    if (old_npad != npad || old_elem != F->elem) {
        spd::launch_zero((double *)F->W, (int64_t)((bW + bWi) / sizeof(double)), st);
        spd::launch_zero((double *)F->WB, (int64_t)(bWB / sizeof(double)), st);
    }
    size_t capt = F->cap_Tb;
    SPD_TRY(grow(&F->Tb, &capt, (size_t)spd::solve_tmp_elems(npad) * F->elem, false, st));
    F->cap_Tb = capt;
    size_t capd = (size_t)F->cap_d * sizeof(double);
    SPD_TRY(grow((void **)&F->d, &capd, (size_t)std::max<int64_t>(n, 1) * sizeof(double), false, st));
    F->cap_d = (int64_t)(capd / sizeof(double));

    F->mu = (prec == SPD_FP16) ? fp16_scale(theta) : 1.0;
    F->half = (prec == SPD_FP16) ? HALF_F16 : (prec == SPD_BF16) ? HALF_BF16 : HALF_NONE;
    if (F->half) {
        size_t caph = F->cap_Lh;
        SPD_TRY(grow(&F->Lh, &caph, (size_t)16 * npad * F->nb * 2, false, st));
        F->cap_Lh = caph;
    }
    return SPD_OK;
}

spd_status do_factor(spd_factor_t F, const double *A, int64_t n, int64_t lda, int prec, const spd_opts &o,
                     hipStream_t st, int64_t *info, bool sync = true)
{
    F->info_pending = false;
    SPD_TRY(prepare_factor(F, n, prec, o.theta, st));
    F->imported = false;
    if (!F->pinned) {
        // the autotuner's schedule for this precision and size, when there is one
        spd::TuneVal tv;
        if (spd::tune_lookup(spd::tune_key(prec_tag(prec), spd::tune_bucket(n)), &tv)) {
            if (prec == SPD_FP16 || prec == SPD_BF16) {
                F->group_half = tv.a;
            } else {
                F->group = tv.a;
                F->small_main = tv.c != 0;
            }
            F->upd_slots = tv.b;
        }
    }
    if (F->terr) HIP_TRY(hipMemsetAsync(F->terr, 0, sizeof(int), st));  // a new factor starts with no timeout
    const int64_t npad = F->npad;
    const int equil = (prec != SPD_FP64 && o.equilibrate) ? 1 : 0;
    *F->info_host = SPD_INFO_NONE_H;
    HIP_TRY(hipMemcpyAsync(F->info_dev, F->info_host, sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    if (n > 0) spd::launch_equil(A, lda, n, F->d, equil, st);
    const double tri = (double)n * (n + 1) / 2;
    hipEvent_t pe = prof_begin(st);
    if (prec == SPD_FP64)
        spd::launch_convert<double>(A, lda, n, npad, F->d, 1.0, (double *)F->L, npad, st);
    else
        spd::launch_convert<float>(A, lda, n, npad, F->d, F->mu, (float *)F->L, npad, st);
    if (pe) prof_end(pe, st, SPD_K_CONVERT, tri, tri * (8.0 + F->elem));
    if (prec == SPD_FP64)
        SPD_TRY(factor_blocked<double>(F, st));
    else
        SPD_TRY(factor_blocked<float>(F, st));
    *info = 0;
    if (!sync) {
        // the caller reads info back later (resolve_info, or with the first residual)
        HIP_TRY(hipGetLastError());
        F->info_pending = true;
        return SPD_OK;
    }
    HIP_TRY(hipMemcpyAsync(F->info_host, F->info_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const unsigned long long v = *F->info_host;
    *info = (v == SPD_INFO_NONE_H) ? 0 : (int64_t)v;
    return *info ? SPD_ERR_NOT_SPD : SPD_OK;
}

// A factor L of A supplied by the caller (binary64, lower triangle of an
// n x n column-major array) taken as the handle's factor at precision prec
// (binary32: rounded once; binary64: as is), with D = I and mu = 1; the
// block inverses the solves use are formed from it.
template <typename T>
void import_factor(spd_factor_t F, const double *L, int64_t ldl, hipStream_t st)
{
    const int64_t n = F->n, npad = F->npad, nt = npad / spd::Panel<T>::NB;
    spd::launch_equil(L, ldl, n, F->d, 0, st);  // d = 1
    spd::launch_convert<T>(L, ldl, n, npad, F->d, 1.0, (T *)F->L, npad, st);
    spd::launch_inv32_blocks<T>((const T *)F->L, npad, npad, (T *)F->Winv, F->info_dev, st);
    spd::launch_trtri_blocks<T>((const T *)F->L, npad, nt, (const T *)F->Winv, (T *)F->W, st);
    spd::launch_build_winv<T>((const T *)F->L, npad, npad, (const T *)F->W, (T *)F->WB, (T *)F->Tb, st);
}

spd_status do_import(spd_factor_t F, const double *L, int64_t n, int64_t ldl, int prec, hipStream_t st,
                     int64_t *info)
{
    F->info_pending = false;
    SPD_TRY(prepare_factor(F, n, prec, 0.1, st));
    F->imported = true;
    if (F->terr) HIP_TRY(hipMemsetAsync(F->terr, 0, sizeof(int), st));
    *F->info_host = SPD_INFO_NONE_H;
    HIP_TRY(hipMemcpyAsync(F->info_dev, F->info_host, sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    if (n > 0) {
        if (prec == SPD_FP64)
            import_factor<double>(F, L, ldl, st);
        else
            import_factor<float>(F, L, ldl, st);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(F->info_host, F->info_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const unsigned long long v = *F->info_host;
    *info = (v == SPD_INFO_NONE_H) ? 0 : (int64_t)v;
    return *info ? SPD_ERR_NOT_SPD : SPD_OK;
}

spd_status ensure_trsv_ws(spd_factor_t F, hipStream_t st)
{
    size_t cap = F->cap_tP;
    SPD_TRY(grow(&F->tP, &cap, (size_t)spd::trsv_scratch_elems(F->npad) * F->elem, false, st));
    F->cap_tP = cap;
    const int nctl = 2 * spd::trsv_ctl_ints(F->npad);  // one set per direction
    if (F->cap_tctl < nctl) {
        if (F->tctl) {
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipFree(F->tctl));
            F->tctl = nullptr;
        }
        HIP_TRY(hipMalloc(&F->tctl, nctl * sizeof(int)));
        F->cap_tctl = nctl;
    }
    if (!F->terr) {
        HIP_TRY(hipMalloc(&F->terr, sizeof(int)));
        HIP_TRY(hipMemsetAsync(F->terr, 0, sizeof(int), st));
    }
    if (!F->terr_host) HIP_TRY(hipHostMalloc(&F->terr_host, sizeof(int), hipHostMallocDefault));
    return SPD_OK;
}

spd_status ensure_solve_ws(spd_factor_t F, int64_t m, hipStream_t st)
{
    SPD_TRY(ensure_trsv_ws(F, st));
    const size_t b = (size_t)F->npad * m * F->elem;
    size_t cap = F->cap_YZ;
    void *base = F->Y;
    SPD_TRY(grow(&base, &cap, 2 * b, false, st));
    F->Y = base;
    F->Z = (char *)base + F->npad * m * F->elem;  // Z follows Y for this m
    F->cap_YZ = cap;
    size_t capm = (size_t)F->cap_smax * sizeof(double);
    SPD_TRY(grow((void **)&F->smax, &capm, (size_t)m * sizeof(double), false, st));
    F->cap_smax = (int64_t)(capm / sizeof(double));
    return SPD_OK;
}

// Low-precision solve of (D R / s) and X (+)= s mu D Y: Algorithm 1's first solve,
// and its correction solve with the update of x.
// The scaling launch also clears the triangular solves' counters and, when
// given, zero_next[0, nzero) (the next residual's norms).
template <typename T>
void solve_apply(spd_factor_t F, const double *R, int64_t ldr, int64_t m, const double *smax, double *X, int64_t ldx,
                 int accumulate, double *zmax, double *zero_next, int64_t nzero, hipStream_t st)
{
    const int64_t npad = F->npad;
    T *Y = (T *)F->Y;
    T *Z = (T *)((char *)F->Y + npad * m * sizeof(T));
    spd::launch_rhs_scale<T>(R, ldr, F->n, npad, (int)m, F->d, smax, Y, npad, zero_next, nzero, F->tctl,
                             2 * spd::trsv_ctl_ints(npad), st);
    hipEvent_t pe = prof_begin(st);
    spd::launch_trsv<T>((const T *)F->L, npad, (const T *)F->WB, npad, (int)m, Y, Z, npad, (T *)F->tP, F->tctl,
                        true, F->terr, F->wait_ticks, st);
    if (pe)
        prof_end(pe, st, SPD_K_TRSV, 2.0 * (double)npad * npad * m,
                 (double)sizeof(T) * ((double)npad * (npad + 1) + 4.0 * npad * m));
    spd::launch_update_x<T>(X, ldx, F->n, (int)m, Y, npad, F->d, F->mu, smax, accumulate, zmax, st);
}

spd_status do_solve(spd_factor_t F, const double *B, int64_t ldb, int64_t m, double *X, int64_t ldx,
                    hipStream_t st)
{
    if (F->n == 0 || m == 0) return SPD_OK;
    SPD_TRY(ensure_solve_ws(F, m, st));
    spd::launch_zero(F->smax, m, st);
    spd::launch_rhs_max(B, ldb, F->n, (int)m, F->d, F->smax, st);
    if (F->elem == 8)
        solve_apply<double>(F, B, ldb, m, F->smax, X, ldx, 0, nullptr, nullptr, 0, st);
    else
        solve_apply<float>(F, B, ldb, m, F->smax, X, ldx, 0, nullptr, nullptr, 0, st);
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

spd_status ensure_refine_ws(spd_factor_t F, int64_t m, hipStream_t st)
{
    size_t cap = F->cap_R;
    SPD_TRY(grow((void **)&F->R, &cap, (size_t)F->n * m * sizeof(double), false, st));
    F->cap_R = cap;
    cap = F->cap_P;
    SPD_TRY(grow((void **)&F->P, &cap, (size_t)spd::resid_scratch(F->n, (int)m) * sizeof(double), false, st));
    F->cap_P = cap;
    const int64_t nn = 1 + 5 * m;
    if (F->cap_norms < nn) {
        if (F->norms) {
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipFree(F->norms));
            HIP_TRY(hipHostFree(F->norms_host));
            F->norms = F->norms_host = nullptr;
        }
        HIP_TRY(hipMalloc(&F->norms, 2 * nn * sizeof(double)));  // two sets, used in turn
        HIP_TRY(hipHostMalloc(&F->norms_host, nn * sizeof(double), hipHostMallocDefault));
        F->cap_norms = nn;
    }
    return SPD_OK;
}

int next_prec(int p) { return (p == SPD_BF16 || p == SPD_FP16) ? SPD_FP32 : SPD_FP64; }

// The stopping rule (Algorithm 1's while-test read as "until x is accurate to
// binary64 level"; the divergence test guards Eq. (4)).  Per column, after
// correction k (z_k solved from the residual of x_k, backward error eta_k,
// x_{k+1} = x_k + z_k): zeta_k = ||z_k|| / ||x_{k+1}|| and the observed
// contraction rho_k = zeta_k / zeta_{k-1}.  z_k tracks the error of x_k; with
// geometric contraction x_{k+1} keeps about rho_k/(1-rho_k) zeta_k of it,
// while residuals rounded at binary64 level resolve x only to about
// (zeta_k/eta_k) u.  A column is done once eta_{k+1} <= tol and
//   eta_{k+1} = 0 or zeta_k <= u; or rho_k < 1/2 and rho_k/(1-rho_k) eta_k <= u;
//   or rho_k >= 1/2 and eta_k <= 4u (no contraction left from a rounding-level
//   residual).
// The backward error alone does not decide: it reaches 1e-14, even 4u, while x
// still misses 10 cond u along the eigenvectors of the smallest eigenvalues.
// The method's own binary64 factor is backward stable: its first solve is
// accepted at eta <= tol.  The iterate handed to the loop counts as a first
// solve (zeta_0 = 1).
constexpr double U64 = 0x1p-53;
constexpr double ETA_FLOOR = 0x1p-51;

bool column_done(double eta_new, double zeta, double zeta_prev, double eta_in, int k, bool stable, double tol)
{
    if (!(eta_new <= tol)) return false;
    if (eta_new == 0.0 || zeta <= U64) return true;
    if (k == 0) return stable;
    const double rho = zeta / zeta_prev;
    return (rho < 0.5) ? (rho / (1.0 - rho)) * eta_in <= U64 : eta_in <= ETA_FLOOR;
}

// Reads back the info word of a factorisation that did not (spd_posv's):
// SPD_ERR_NOT_SPD, with *info the 1-based failing column, when it broke down.
spd_status resolve_info(spd_factor_t F, hipStream_t st, int64_t *info)
{
    *info = 0;
    if (!F->info_pending) return SPD_OK;
    HIP_TRY(hipMemcpyAsync(F->info_host, F->info_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    F->info_pending = false;
    const unsigned long long v = *F->info_host;
    if (v == SPD_INFO_NONE_H) return SPD_OK;
    *info = (int64_t)v;
    return SPD_ERR_NOT_SPD;
}

// One refinement run at the handle's current precision, from the iterate in
// X (taken as the result of one low-precision solve).  Returns SPD_OK (every
// column done), SPD_ERR_NO_CONVERGENCE (diverged, or max_iter corrections
// without success); device errors propagate.
spd_status refine_once(spd_factor_t F, const double *A, int64_t lda, const double *B, int64_t ldb, int64_t m,
                       double *X, int64_t ldx, const spd_opts &o, spd_report *rep, hipStream_t st)
{
    const int64_t n = F->n;
    SPD_TRY(ensure_solve_ws(F, m, st));
    SPD_TRY(ensure_refine_ws(F, m, st));
    const int64_t nn = 1 + 5 * m;  // ||A||, then per column max|r|, max|x|, max|b|, max|D r|, max|z|
    std::vector<double> eta(m), eprev(m), zeta(m, 1.0), zprev(m, 1.0);
    std::vector<char> done(m, 0);
    const bool stable = (F->prec == SPD_FP64 && !F->imported);
    rep->iters_low = 1;  // the iterate came from one low-precision solve
    rep->iters_high = 0;
    double eta0 = 0.0, anorm = 0.0;
    int stalls = 0;
    spd_status result = SPD_ERR_NO_CONVERGENCE;
    // Two sets of norms used in turn: the residual of iteration k accumulates
    // into set k % 2, which the scaling launch of the correction before it
    // cleared (the correction writes its max|z| there too), while that
    // correction reads its scale from the other set.
    double *nset[2] = {F->norms, F->norms + nn};
    int cur = 0;
    spd::launch_zero(nset[0], nn, st);
    for (;;) {
        const int first = (rep->iters_high == 0);
        double *norms = nset[cur];
        hipEvent_t pr = prof_begin(st);
        spd::launch_residual(A, lda, n, X, ldx, B, ldb, (int)m, F->R, n, F->d, norms, first, F->P, st);
        if (pr)
            prof_end(pr, st, SPD_K_RESIDUAL, 2.0 * n * n * m,
                     8.0 * ((double)n * (n + 1) / 2 + 3.0 * n * m));
        const bool check_info = F->info_pending;
        spd::launch_publish(norms, nn, F->terr, check_info ? F->info_dev : nullptr, F->norms_host, F->terr_host,
                            check_info ? F->info_host : nullptr, st);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return map_err(e);
        if (check_info) {
            // the factorisation's own outcome comes first: a broken-down factor
            // made this residual meaningless
            F->info_pending = false;
            const unsigned long long v = *F->info_host;
            if (v != SPD_INFO_NONE_H) {
                rep->info = (int64_t)v;
                return SPD_ERR_NOT_SPD;
            }
        }
        if (*F->terr_host) return SPD_ERR_DEVICE;  // a triangular-solve wait timed out
        const int k = rep->iters_high;  // corrections applied so far
        rep->iters_high++;
        if (first) anorm = F->norms_host[0];
        bool finite = std::isfinite(anorm), all = true;
        double worst = 0.0;
        for (int64_t c = 0; c < m; ++c) {
            const double rn = F->norms_host[1 + c], xn = F->norms_host[1 + m + c], bn = F->norms_host[1 + 2 * m + c];
            const double den = anorm * xn + bn;
            double v = (den > 0.0) ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
            if (!(rn == rn) || !(xn == xn)) v = NAN;
            eta[c] = v;
            if (!std::isfinite(v)) finite = false;
            if (v > worst) worst = v;
            if (k > 0) {
                const double zn = F->norms_host[1 + 4 * m + c];
                zeta[c] = (zn == 0.0) ? 0.0 : zn / xn;
            }
            if (!done[c]) done[c] = column_done(v, zeta[c], zprev[c], eprev[c], k, stable, o.tol);
            all = all && done[c];
        }
        rep->eta = finite ? worst : NAN;
        if (!finite) break;                                  // diverged
        if (all && worst <= o.tol) { result = SPD_OK; break; }
        if (k == 0) {
            eta0 = worst;
        } else {
            bool all_slow = true;
            for (int64_t c = 0; c < m; ++c)
                if (!(eta[c] > 0.9 * eprev[c])) all_slow = false;
            stalls = all_slow ? stalls + 1 : 0;
            if (worst > o.tol && (worst > eta0 || stalls >= 2)) break;  // diverged / stagnated
        }
        if (rep->iters_low > o.max_iter) break;  // out of corrections: no convergence
        eprev = eta;
        zprev = zeta;
        // correction: Z = low-precision solve of D R / s, X += s mu D Z
        double *next = nset[cur ^ 1];
        const double *dmax = norms + 1 + 3 * m;
        double *zmax = next + 1 + 4 * m;
        if (F->elem == 8)
            solve_apply<double>(F, F->R, n, m, dmax, X, ldx, 1, zmax, next, nn, st);
        else
            solve_apply<float>(F, F->R, n, m, dmax, X, ldx, 1, zmax, next, nn, st);
        e = hipGetLastError();
        if (e != hipSuccess) return map_err(e);
        cur ^= 1;
        rep->iters_low++;
    }
    return result;
}

bool valid_prec(int p) { return p >= SPD_BF16 && p <= SPD_FP64; }

// ---- batched solver state (per device; kept until the process ends) ----
constexpr int kMaxDevices = 64;
constexpr int kBatchMaxGrid = 1024;
// persistent grid sizes tried by the batched autotuner (four wavefronts per
// workgroup: the kernels are built for that size)
constexpr int kBatchGrids[] = {256, 512, 768, 1024};
struct BatchEntry {
    int32_t *order = nullptr;  // work order (and, after it, the queue counter)
    int *queue = nullptr;
    int grid = 256, waves = 4;
};
struct BatchCtx {
    void *ws = nullptr;
    // the workspace is shared by every call on the device: a call on another
    // stream first waits for the previous call's launch (not under capture)
    hipEvent_t last = nullptr;
    hipStream_t last_stream = nullptr;
    std::map<int64_t, BatchEntry> per_batch;
    float *picker = nullptr;  // perceptron parameters (device), kept until the process ends
    bool picker_on = false;
    float *mlp_scratch = nullptr;  // gradient partials of spd_mlp_grad
    size_t cap_mlp = 0;
};
std::mutex g_batch_mu;
BatchCtx g_batch[kMaxDevices];

}  // namespace

// ---------------------------------------------------------------------------
// Algorithm 2 (Section 3.2): conjugate gradients on the binary32 operator A~
// with binary64 vectors and scalars, restarted from a binary64 residual.
struct spd_cg_s {
    int64_t n = 0, ldt = 0, k = -1;  // k >= 0: band |i - j| <= k; k < 0: dense
    float *At = nullptr;             // dense ldt x ldt, or (2k + 1) rows of length ldt
    size_t cap_At = 0;               // bytes allocated for At
    int m = 0;                       // right-hand sides the workspace is sized for
    double *R = nullptr, *P = nullptr, *Z = nullptr, *part = nullptr, *vpart = nullptr, *sc = nullptr;
    double *norms = nullptr, *rscr = nullptr;
    double *Xs = nullptr;            // x at the start of the inner phase (its change is the correction)
    float *Pf = nullptr;
    float *Zp = nullptr;             // k-slice partials of the dense multi-column product
    int *flags = nullptr;            // act[2][m] (parity slots), go[m], cnt[m]
    double *norms_host = nullptr;
    int *flags_host = nullptr;
    hipStream_t gstream = nullptr;   // capture stream for the banded iteration graph
};

namespace {

void cg_free_ws(spd_cg_t H)
{
    hipFree(H->R); hipFree(H->P); hipFree(H->Z); hipFree(H->part); hipFree(H->vpart); hipFree(H->sc); hipFree(H->Xs);
    hipFree(H->norms); hipFree(H->rscr); hipFree(H->Pf); hipFree(H->Zp); hipFree(H->flags);
    if (H->norms_host) hipHostFree(H->norms_host);
    if (H->flags_host) hipHostFree(H->flags_host);
    H->R = H->P = H->Z = H->part = H->vpart = H->sc = H->norms = H->rscr = H->Xs = nullptr;
    H->Pf = nullptr;
    H->Zp = nullptr;
    H->flags = nullptr;
    H->norms_host = nullptr;
    H->flags_host = nullptr;
    H->m = 0;
}

spd_status cg_ensure_ws(spd_cg_t H, int m, hipStream_t st)
{
    if (H->m >= m) return SPD_OK;
    HIP_TRY(hipStreamSynchronize(st));
    cg_free_ws(H);
    const int64_t n = H->n, ldt = H->ldt;
    const size_t nm = (size_t)n * m * sizeof(double);
    HIP_TRY(hipMalloc(&H->R, nm));
    HIP_TRY(hipMalloc(&H->P, nm));
    HIP_TRY(hipMalloc(&H->Z, nm));
    HIP_TRY(hipMalloc(&H->Xs, nm));
    // product partials: sized for the most per column any m' <= m uses (the
    // workspace is reused for fewer right-hand sides)
    const int64_t mvp = std::max(spd::cg_mv_parts(n, ldt, H->k, m), spd::cg_mv_parts(n, ldt, H->k, 1));
    HIP_TRY(hipMalloc(&H->part, (size_t)mvp * m * sizeof(double)));
    HIP_TRY(hipMalloc(&H->vpart, (size_t)spd::cg_vec_parts(n) * m * sizeof(double)));
    HIP_TRY(hipMalloc(&H->sc, (size_t)4 * m * sizeof(double)));
    HIP_TRY(hipMalloc(&H->norms, (size_t)(1 + 5 * m) * sizeof(double)));
    HIP_TRY(hipMalloc(&H->rscr, (size_t)spd::resid_scratch(n, m) * sizeof(double)));
    HIP_TRY(hipMalloc(&H->Pf, (size_t)spd::cg_pf_elems(ldt, m) * sizeof(float)));
    if (H->k < 0 && spd::cg_zp_elems(n, m) > 0)
        HIP_TRY(hipMalloc(&H->Zp, (size_t)spd::cg_zp_elems(n, m) * sizeof(float)));
    HIP_TRY(hipMalloc(&H->flags, (size_t)4 * m * sizeof(int)));
    HIP_TRY(hipHostMalloc(&H->norms_host, (size_t)(1 + 5 * m) * sizeof(double), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&H->flags_host, (size_t)4 * m * sizeof(int), hipHostMallocDefault));
    H->m = m;
    return SPD_OK;
}

spd_status cg_refine(spd_cg_t H, const double *A, int64_t lda, const double *B, int64_t ldb, int m, double *X,
                     int64_t ldx, const spd_cg_opts &o, spd_report *rep, hipStream_t st)
{
    const int64_t n = H->n, ldt = H->ldt, k = H->k;
    SPD_TRY(cg_ensure_ws(H, m, st));
    // Pf's padding (rows n..ldt-1, columns m.. of the last block) must read as zero
    spd::launch_zero((double *)H->Pf, spd::cg_pf_elems(ldt, m) / 2, st);
    const int64_t nmv = spd::cg_mv_parts(n, ldt, k, m), nv = spd::cg_vec_parts(n);
    int *act = H->flags, *go = H->flags + 2 * m, *cnt = H->flags + 3 * m;  // act: two parity slots
    int *go_h = H->flags_host + 2 * m;
    const double it2 = o.inner_tol * o.inner_tol;
    const int nn = 1 + 5 * m;  // as refine_once: the last m hold each column's change over its phase
    // iterations launched between host checks: a dense product is long
    // enough that one check per iteration costs nothing
    const int S = (k < 0) ? 2 : 16;
    const double band_w = (k < 0) ? (double)n : (double)(2 * k + 1);
    const double mv_flops = 2.0 * band_w * n * m, mv_bytes = 4.0 * band_w * n + 20.0 * n * m;
    // one CG iteration: product, x/r update, p update (parity slot par); with
    // profiling on, the product alone is bracketed by the caller
    auto launch_iteration = [&](int par, hipStream_t q) {
        spd::launch_cg_mv(H->At, ldt, n, k, m, H->Pf, H->P, H->Z, H->part, nmv, act + par * m, H->Zp, q);
        spd::launch_cg_xr(n, m, H->part, nmv, H->sc, par, H->P, H->Z, X, ldx, H->R, H->vpart, nv, act, q);
        spd::launch_cg_p(n, m, H->vpart, nv, H->sc, par, H->R, H->P, H->Pf, ldt, act, cnt, o.max_inner, q);
    };
    // Banded iterations are launch-bound: the S iterations between host
    // checks are captured once per call into a graph (all arguments are fixed
    // for the call) and replayed.  Not while kernel profiling is on (its
    // events bracket single launches), and any capture failure falls back to
    // direct launches.
    hipGraphExec_t gexec = nullptr;
    if (k >= 0 && !prof_enabled()) {
        bool ok = H->gstream || hipStreamCreateWithFlags(&H->gstream, hipStreamNonBlocking) == hipSuccess;
        hipGraph_t g = nullptr;
        if (ok) ok = hipStreamBeginCapture(H->gstream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            for (int s = 0; s < S; ++s) launch_iteration(s & 1, H->gstream);
            ok = hipStreamEndCapture(H->gstream, &g) == hipSuccess && g;
        }
        if (ok) ok = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) hipGraphDestroy(g);
        if (!ok) {
            gexec = nullptr;
            (void)hipGetLastError();
        }
    }
    struct GraphGuard {
        hipGraphExec_t &e;
        ~GraphGuard() { if (e) hipGraphExecDestroy(e); }
    } gguard{gexec};
    std::vector<double> eta1(m, 0.0), prev(m, 0.0), zeta(m, 1.0), zprev(m, 1.0);
    std::vector<int> done(m, 0), stalls(m, 0);
    std::vector<double> eta(m, 0.0);
    double anorm = 0.0;
    spd_status result = SPD_ERR_NO_CONVERGENCE;
    rep->iters_low = rep->iters_high = 0;
    for (int outer = 0;; ++outer) {
        spd::launch_zero(outer == 0 ? H->norms : H->norms + 1, outer == 0 ? nn - m : nn - m - 1, st);
        spd::launch_residual(A, lda, n, X, ldx, B, ldb, m, H->R, n, nullptr, H->norms, outer == 0, H->rscr, st);
        HIP_TRY(hipMemcpyAsync(H->norms_host, H->norms, nn * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        rep->iters_high++;
        if (outer == 0) anorm = H->norms_host[0];
        bool bad = !(anorm == anorm), all_done = true;
        double worst = 0.0;
        for (int c = 0; c < m; ++c) {
            const double rn = H->norms_host[1 + c], xn = H->norms_host[1 + m + c], bn = H->norms_host[1 + 2 * m + c];
            const double den = anorm * xn + bn;
            double e = (den > 0.0) ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
            if (!(rn == rn) || !(xn == xn)) e = NAN;
            if (!done[c]) {
                eta[c] = e;
                if (outer > 0) {  // the column ran the last inner phase
                    const double dn = H->norms_host[1 + 4 * m + c];
                    zprev[c] = zeta[c];
                    zeta[c] = (dn == 0.0) ? 0.0 : dn / xn;
                }
                if (!std::isfinite(e)) {
                    bad = true;
                } else if (e <= o.tol) {
                    done[c] = column_done(e, zeta[c], zprev[c], prev[c], outer, false, o.tol);
                } else if (outer > 0) {
                    stalls[c] = (e > 0.9 * prev[c]) ? stalls[c] + 1 : 0;
                    if (e > eta1[c] || stalls[c] >= 2) bad = true;
                }
                if (outer == 0) eta1[c] = e;
                prev[c] = e;
            }
            if (!done[c]) all_done = false;
            if (!(eta[c] <= worst)) worst = eta[c];
        }
        rep->eta = worst;
        if (bad) break;
        if (all_done) { result = SPD_OK; break; }
        if (outer >= o.max_outer) break;
        // inner phase for the columns not done, from x saved in Xs
        for (int c = 0; c < m; ++c) go_h[c] = !done[c];
        HIP_TRY(hipMemcpyAsync(go, go_h, m * sizeof(int), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpy2DAsync(H->Xs, n * sizeof(double), X, ldx * sizeof(double), n * sizeof(double), m,
                                 hipMemcpyDeviceToDevice, st));
        spd::launch_cg_start(n, m, H->R, H->P, H->Pf, ldt, H->vpart, nv, go, st);
        spd::launch_cg_begin(H->vpart, nv, H->sc, act, go, cnt, it2, o.max_inner, m, st);
        int launched = 0;
        for (;;) {
            if (gexec) {
                HIP_TRY(hipGraphLaunch(gexec, st));
            } else {
                for (int s = 0; s < S; ++s) {  // S is even: iteration parity = s & 1
                    hipEvent_t pe = prof_begin(st);
                    launch_iteration(s & 1, st);
                    if (pe) prof_end(pe, st, SPD_K_CG_MV, mv_flops, mv_bytes);
                }
            }
            launched += S;
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(H->flags_host, H->flags, 4 * m * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            bool any = false;
            for (int c = 0; c < m; ++c) any |= H->flags_host[c] != 0;  // slot 0 after an even count
            if (!any || launched > o.max_inner + S) break;
        }
        int longest = 0;
        for (int c = 0; c < m; ++c)
            if (go_h[c]) longest = std::max(longest, H->flags_host[3 * m + c]);
        rep->iters_low += longest;
        // each column's change of x over the phase (columns that sat out: 0)
        spd::launch_zero(H->norms + 1 + 4 * m, m, st);
        spd::launch_col_maxdiff(X, ldx, H->Xs, n, n, m, H->norms + 1 + 4 * m, st);
    }
    return result;
}

}  // namespace

extern "C" {

void spd_opts_default(spd_opts *o)
{
    if (o) *o = defaults();
}

const char *spd_status_str(spd_status s)
{
    switch (s) {
    case SPD_OK: return "SPD_OK";
    case SPD_ERR_INVALID_ARG: return "SPD_ERR_INVALID_ARG";
    case SPD_ERR_NOT_SPD: return "SPD_ERR_NOT_SPD";
    case SPD_ERR_NO_CONVERGENCE: return "SPD_ERR_NO_CONVERGENCE";
    case SPD_ERR_DEVICE: return "SPD_ERR_DEVICE";
    case SPD_ERR_OUT_OF_MEMORY: return "SPD_ERR_OUT_OF_MEMORY";
    case SPD_ERR_UNSUPPORTED: return "SPD_ERR_UNSUPPORTED";
    }
    return "SPD_ERR_UNKNOWN";
}

const char *spd_version(void) { return "libspd 0.1 (gfx950)"; }

void spd_profile_enable(int on)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
}

void spd_profile_reset(void)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &r : g_prof_pending) {
        hipEventSynchronize(r.b);
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    for (auto &t : g_prof_tot) t = ProfTotals();
}

spd_status spd_profile_query(int kernel, int64_t *launches, double *total_ms, double *total_flops,
                             double *total_bytes)
{
    if (kernel < 0 || kernel >= SPD_K_COUNT) return SPD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &r : g_prof_pending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e == hipSuccess) {
            ProfTotals &t = g_prof_tot[r.kind];
            t.launches++;
            t.ms += ms;
            t.flops += r.flops;
            t.bytes += r.bytes;
        }
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    const ProfTotals &t = g_prof_tot[kernel];
    if (launches) *launches = t.launches;
    if (total_ms) *total_ms = t.ms;
    if (total_flops) *total_flops = t.flops;
    if (total_bytes) *total_bytes = t.bytes;
    return SPD_OK;
}

}  // extern "C"

namespace {

// spd_factor's body; with sync false the info word is left to be read back
// with the first residual (spd_posv), and SPD_OK means only "launched"
spd_status factor_entry(const double *A, int64_t n, int64_t lda, spd_prec prec, const spd_opts *o,
                        void *hip_stream, spd_factor_t *F, int64_t *info, bool sync)
{
    if (!F || !info || n < 0 || lda < std::max<int64_t>(1, n) || (n > 0 && !A) || !valid_prec(prec))
        return SPD_ERR_INVALID_ARG;
    const spd_opts op = o ? *o : defaults();
    if (!opts_valid(op)) return SPD_ERR_INVALID_ARG;
    *info = 0;
    bool created = false;
    if (!*F) {
        *F = new (std::nothrow) spd_factor_s();
        if (!*F) return SPD_ERR_OUT_OF_MEMORY;
        created = true;
        (*F)->pinned = std::getenv("SPD_GROUP") || std::getenv("SPD_GROUP_HALF") || std::getenv("SPD_UPD_SLOTS") ||
                       std::getenv("SPD_SMALL_MAIN");
        if (const char *e = std::getenv("SPD_GROUP")) (*F)->group = std::max(1, std::min(8, std::atoi(e)));
        if (const char *e = std::getenv("SPD_SMALL_MAIN")) (*F)->small_main = std::atoi(e) != 0;
        if (const char *e = std::getenv("SPD_GROUP_HALF"))
            (*F)->group_half = std::max(2, std::min(8, std::atoi(e) & ~1));
        if (const char *e = std::getenv("SPD_UPD_SLOTS")) (*F)->upd_slots = std::max(0, std::atoi(e));
        if (hipGetDevice(&(*F)->device) != hipSuccess) {
            delete *F;
            *F = nullptr;
            return SPD_ERR_DEVICE;
        }
    }
    spd_status s = do_factor(*F, A, n, lda, prec, op, (hipStream_t)hip_stream, info, sync);
    if (s != SPD_OK && s != SPD_ERR_NOT_SPD && created) {
        spd_factor_destroy(*F);
        *F = nullptr;
    }
    return s;
}

}  // namespace

extern "C" {

spd_status spd_factor(const double *A, int64_t n, int64_t lda, spd_prec prec, const spd_opts *o, void *hip_stream,
                      spd_factor_t *F, int64_t *info)
{
    return factor_entry(A, n, lda, prec, o, hip_stream, F, info, true);
}

spd_status spd_factor_import(const double *L, int64_t n, int64_t ldl, spd_prec prec, void *hip_stream,
                             spd_factor_t *F, int64_t *info)
{
    if (!F || !info || n < 0 || ldl < std::max<int64_t>(1, n) || (n > 0 && !L) ||
        (prec != SPD_FP32 && prec != SPD_FP64))
        return SPD_ERR_INVALID_ARG;
    *info = 0;
    bool created = false;
    if (!*F) {
        *F = new (std::nothrow) spd_factor_s();
        if (!*F) return SPD_ERR_OUT_OF_MEMORY;
        created = true;
        if (hipGetDevice(&(*F)->device) != hipSuccess) {
            delete *F;
            *F = nullptr;
            return SPD_ERR_DEVICE;
        }
    }
    spd_status s = do_import(*F, L, n, ldl, prec, (hipStream_t)hip_stream, info);
    if (s != SPD_OK && s != SPD_ERR_NOT_SPD && created) {
        spd_factor_destroy(*F);
        *F = nullptr;
    }
    return s;
}

spd_status spd_solve(spd_factor_t F, const double *B, int64_t ldb, int64_t nrhs, double *X, int64_t ldx,
                     void *hip_stream)
{
    if (!F || F->prec < 0 || nrhs < 0) return SPD_ERR_INVALID_ARG;
    const int64_t n = F->n;
    if (ldb < std::max<int64_t>(1, n) || ldx < std::max<int64_t>(1, n)) return SPD_ERR_INVALID_ARG;
    if (n > 0 && nrhs > 0 && (!B || !X)) return SPD_ERR_INVALID_ARG;
    return do_solve(F, B, ldb, nrhs, X, ldx, (hipStream_t)hip_stream);
}

}  // extern "C"

namespace {

// spd_refine's body after argument checks: refinement from the iterate in X,
// escalating precision when the rule of Eq. (4) fails (op.fallback)
spd_status refine_loop(spd_factor_t F, const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrhs,
                       double *X, int64_t ldx, const spd_opts &op, spd_report *rep, hipStream_t st)
{
    const int64_t n = F->n;
    std::memset(rep, 0, sizeof(*rep));
    rep->prec_used = F->prec;
    if (n == 0 || nrhs == 0) {
        int64_t info = 0;
        spd_status s = resolve_info(F, st, &info);
        rep->info = info;
        rep->status = s;
        rep->eta = 0.0;
        return s;
    }
    for (;;) {
        spd_status s = refine_once(F, A, lda, B, ldb, nrhs, X, ldx, op, rep, st);
        rep->prec_used = F->prec;
        if (s != SPD_ERR_NO_CONVERGENCE || !op.fallback || F->prec == SPD_FP64) {
            rep->status = s;
            return s;
        }
        // escalate: re-factor at the next precision and restart from solve(B)
        rep->fallbacks++;
        int64_t info = 0;
        int p = next_prec(F->prec);
        for (;;) {
            s = do_factor(F, A, n, lda, p, op, st, &info);
            if (s == SPD_ERR_NOT_SPD && p != SPD_FP64) {
                rep->fallbacks++;
                p = next_prec(p);
                continue;
            }
            break;
        }
        rep->prec_used = F->prec;
        rep->info = info;
        if (s != SPD_OK) {
            rep->status = s;
            return s;
        }
        s = do_solve(F, B, ldb, nrhs, X, ldx, st);
        if (s != SPD_OK) {
            rep->status = s;
            return s;
        }
    }
}

}  // namespace

extern "C" {

spd_status spd_refine(spd_factor_t F, const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrhs,
                      double *X, int64_t ldx, const spd_opts *o, spd_report *rep, void *hip_stream)
{
    if (!F || F->prec < 0 || !rep || nrhs < 0) return SPD_ERR_INVALID_ARG;
    const int64_t n = F->n;
    if (lda < std::max<int64_t>(1, n) || ldb < std::max<int64_t>(1, n) || ldx < std::max<int64_t>(1, n))
        return SPD_ERR_INVALID_ARG;
    if (n > 0 && nrhs > 0 && (!A || !B || !X)) return SPD_ERR_INVALID_ARG;
    const spd_opts op = o ? *o : defaults();
    if (!opts_valid(op)) return SPD_ERR_INVALID_ARG;
    return refine_loop(F, A, lda, B, ldb, nrhs, X, ldx, op, rep, (hipStream_t)hip_stream);
}

spd_status spd_autotune(int64_t n, spd_prec prec, void *hip_stream, spd_tune_result *out)
{
    if (n < 1 || n > (int64_t)1 << 20 || !valid_prec(prec) || !out) return SPD_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    const int64_t nb = spd::tune_bucket(n);
    const std::string key = spd::tune_key(prec_tag(prec), nb);
    spd::TuneVal tv;
    if (int src = spd::tune_lookup(key, &tv)) {
        out->group = tv.a;
        out->upd_slots = tv.b;
        out->ms = tv.ms;
        out->from_cache = src;
        out->n = nb;
        out->small_tiles = tv.c;
        return SPD_OK;
    }
    // time the factorisation of a test matrix of the bucket's order under
    // every candidate schedule (the schedule changes no result)
    const bool half = (prec == SPD_FP16 || prec == SPD_BF16);
    // (panels per group, workgroup cap, thin group updates on 64-row tiles)
    struct Cand {
        int g, cap, small;
    };
    std::vector<Cand> cand;
    if (half) {
        for (int g : {2, 4, 8})
            for (int c : {0, 192, 224}) cand.push_back({g, c, 0});
    } else if (prec == SPD_FP32) {
        // 64-row tiles apply to uncapped launches only
        for (int g : {2, 4, 6, 8}) {
            cand.push_back({g, 0, 0});
            cand.push_back({g, 0, 1});
            cand.push_back({g, 448, 0});
        }
    } else {
        for (int g : {2, 4, 6, 8}) cand.push_back({g, 0, 0});
    }
    hipStream_t st = (hipStream_t)hip_stream;
    double *A = nullptr;
    HIP_TRY(hipMalloc(&A, (size_t)nb * nb * sizeof(double)));
    spd::launch_tune_matrix(A, nb, st);
    spd_factor_t F = new (std::nothrow) spd_factor_s();
    if (!F) {
        hipFree(A);
        return SPD_ERR_OUT_OF_MEMORY;
    }
    F->pinned = true;
    spd_status result = SPD_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) result = map_err(he);
    if (result == SPD_OK && hipGetDevice(&F->device) != hipSuccess) result = SPD_ERR_DEVICE;
    const spd_opts op = defaults();
    double best = 1e30;
    int64_t info = 0;
    for (size_t i = 0; i < cand.size() && result == SPD_OK; ++i) {
        (half ? F->group_half : F->group) = cand[i].g;
        F->upd_slots = cand[i].cap;
        F->small_main = cand[i].small != 0;
        double t = 1e30;
        for (int r = 0; r < 3 && result == SPD_OK; ++r) {  // first run warms up
            hipEventRecord(e0, st);
            result = do_factor(F, A, nb, nb, prec, op, st, &info);
            hipEventRecord(e1, st);
            float ms = 0.f;
            if (result == SPD_OK && hipEventSynchronize(e1) == hipSuccess &&
                hipEventElapsedTime(&ms, e0, e1) == hipSuccess && r > 0)
                t = std::min(t, (double)ms);
        }
        if (result == SPD_OK && t < best) {
            best = t;
            tv.a = cand[i].g;
            tv.b = cand[i].cap;
            tv.c = cand[i].small;
            tv.ms = t;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    spd_factor_destroy(F);
    hipFree(A);
    if (result != SPD_OK) return result;
    spd::tune_store(key, tv);
    out->group = tv.a;
    out->upd_slots = tv.b;
    out->ms = tv.ms;
    out->from_cache = 0;
    out->n = nb;
    out->small_tiles = tv.c;
    return SPD_OK;
}

void spd_autotune_clear(void) { spd::tune_clear(); }

spd_status spd_factor_set_wait_limit(spd_factor_t F, double seconds)
{
    if (!F || !(seconds >= 0.0) || seconds > 1e6) return SPD_ERR_INVALID_ARG;
    F->wait_ticks = (unsigned long long)(seconds * 1e8);  // wall_clock64: 100 MHz
    return SPD_OK;
}

spd_status spd_posv(const double *A, int64_t n, int64_t lda, const double *B, int64_t ldb, int64_t nrhs, double *X,
                    int64_t ldx, spd_prec prec, const spd_opts *o, spd_report *rep, void *hip_stream,
                    spd_factor_t *F)
{
    if (!rep || !F) return SPD_ERR_INVALID_ARG;
    std::memset(rep, 0, sizeof(*rep));
    const spd_opts op = o ? *o : defaults();
    if (!opts_valid(op) || !valid_prec(prec) || nrhs < 0) return SPD_ERR_INVALID_ARG;
    if (ldb < std::max<int64_t>(1, n) || ldx < std::max<int64_t>(1, n)) return SPD_ERR_INVALID_ARG;
    if (n > 0 && nrhs > 0 && (!B || !X)) return SPD_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    int p = prec;
    int fallbacks = 0;
    spd_status s;
    // The factorisation's info word is read back with the first residual
    // (no host round trip between factor, solve and refinement); a breakdown
    // then restarts at the next precision as a synchronous check would.
    for (;;) {
        int64_t info = 0;
        s = factor_entry(A, n, lda, (spd_prec)p, &op, hip_stream, F, &info, false);
        if (s == SPD_OK) s = do_solve(*F, B, ldb, nrhs, X, ldx, st);
        if (s == SPD_OK) {
            s = refine_loop(*F, A, lda, B, ldb, nrhs, X, ldx, op, rep, st);
        } else {
            std::memset(rep, 0, sizeof(*rep));
            rep->status = s;
        }
        if (*F && (*F)->info_pending) {
            // an error came before the read-back: settle it here
            int64_t v = 0;
            if (resolve_info(*F, st, &v) == SPD_ERR_NOT_SPD && s == SPD_OK) s = SPD_ERR_NOT_SPD;
            rep->info = v;
        }
        rep->prec_used = p;
        if (s == SPD_ERR_NOT_SPD && op.fallback && p != SPD_FP64) {
            ++fallbacks;
            p = next_prec(p);
            continue;
        }
        break;
    }
    if (s == SPD_ERR_NOT_SPD) rep->status = s;
    if (*F && s != SPD_ERR_NOT_SPD) rep->prec_used = (*F)->prec;
    rep->fallbacks += fallbacks;
    return s;
}

}  // extern "C"

namespace {
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// this device's copy of `scratch` (looked up once per device, with it current)
spd_status noalloc_scratch(char **ptr)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return SPD_ERR_DEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return SPD_ERR_DEVICE;
        g_scratch_ptr[dev] = (char *)p;
    }
    *ptr = g_scratch_ptr[dev];
    return SPD_OK;
}
}  // namespace

extern "C" {

spd_status spd_residual_noalloc(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx,
                                const double *B, int64_t ldb, int64_t nrhs, double *R, int64_t ldr, double *eta,
                                void *hip_stream)
{
    if (n < 0 || nrhs < 0 || lda < std::max<int64_t>(1, n) || ldx < std::max<int64_t>(1, n) ||
        ldb < std::max<int64_t>(1, n) || (R && ldr < std::max<int64_t>(1, n)))
        return SPD_ERR_INVALID_ARG;
    if (n > 0 && nrhs > 0 && (!A || !X || !B)) return SPD_ERR_INVALID_ARG;
    if (n > INT32_MAX || nrhs > INT32_MAX) return SPD_ERR_INVALID_ARG;
    // layout in the scratch array, each part 256-byte aligned; sizes beyond
    // the array are rejected before any device work
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int64_t nn = 1 + 4 * nrhs;
    const size_t bP = (n > 0 && nrhs > 0) ? up((size_t)spd::resid_scratch(n, (int)nrhs) * sizeof(double)) : 0;
    const size_t bR = R ? 0 : up((size_t)n * nrhs * sizeof(double));
    const size_t bN = up((size_t)nn * sizeof(double)), bE = up((size_t)nrhs * sizeof(double));
    if (bP + bR + bN + bE > (size_t)SPD_NOALLOC_SCRATCH_BYTES) return SPD_ERR_INVALID_ARG;
    if (n == 0 || nrhs == 0) {
        for (int64_t c = 0; eta && c < nrhs; ++c) eta[c] = 0.0;
        return SPD_OK;
    }
    char *base = nullptr;
    SPD_TRY(noalloc_scratch(&base));
    hipStream_t st = (hipStream_t)hip_stream;
    double *P = (double *)base;
    double *Rw = R ? R : (double *)(base + bP);
    const int64_t ldrw = R ? ldr : n;
    double *norms = (double *)(base + bP + bR);
    double *etad = (double *)(base + bP + bR + bN);
    spd::launch_zero(norms, nn, st);
    spd::launch_residual(A, lda, n, X, ldx, B, ldb, (int)nrhs, Rw, ldrw, nullptr, norms, 1, P, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && eta) {
        spd::launch_eta_from_norms(norms, (int)nrhs, etad, st);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(eta, etad, (size_t)nrhs * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    return map_err(e);
}

spd_status spd_residual(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx, const double *B,
                        int64_t ldb, int64_t nrhs, double *R, int64_t ldr, double *eta, void *hip_stream)
{
    if (n < 0 || nrhs < 0 || lda < std::max<int64_t>(1, n) || ldx < std::max<int64_t>(1, n) ||
        ldb < std::max<int64_t>(1, n) || (R && ldr < std::max<int64_t>(1, n)))
        return SPD_ERR_INVALID_ARG;
    if (n > 0 && nrhs > 0 && (!A || !X || !B)) return SPD_ERR_INVALID_ARG;
    if (n == 0 || nrhs == 0) {
        for (int64_t c = 0; eta && c < nrhs; ++c) eta[c] = 0.0;
        return SPD_OK;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t nn = 1 + 4 * nrhs;
    const size_t bP = (size_t)spd::resid_scratch(n, (int)nrhs) * sizeof(double);
    const size_t bR = R ? 0 : (size_t)n * nrhs * sizeof(double);
    char *scratch = nullptr;
    HIP_TRY(hipMalloc(&scratch, bP + bR + nn * sizeof(double)));
    double *P = (double *)scratch;
    double *Rw = R ? R : (double *)(scratch + bP);
    const int64_t ldrw = R ? ldr : n;
    double *norms = (double *)(scratch + bP + bR);
    spd::launch_zero(norms, nn, st);
    spd::launch_residual(A, lda, n, X, ldx, B, ldb, (int)nrhs, Rw, ldrw, nullptr, norms, 1, P, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && eta) {
        double *h = new (std::nothrow) double[nn];
        if (!h) {
            hipStreamSynchronize(st);
            hipFree(scratch);
            return SPD_ERR_OUT_OF_MEMORY;
        }
        e = hipMemcpyAsync(h, norms, nn * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        for (int64_t c = 0; e == hipSuccess && c < nrhs; ++c) {
            const double rn = h[1 + c], xn = h[1 + nrhs + c], bn = h[1 + 2 * nrhs + c];
            const double den = h[0] * xn + bn;
            double v = (den > 0.0) ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
            if (!(rn == rn) || !(xn == xn) || !(h[0] == h[0])) v = NAN;
            eta[c] = v;
        }
        delete[] h;
    } else if (e == hipSuccess) {
        e = hipStreamSynchronize(st);
    }
    hipError_t e2 = hipFree(scratch);
    if (e == hipSuccess) e = e2;
    return map_err(e);
}

static spd_status solve_batched_impl(int64_t batch, const int32_t *n, const int32_t *nrhs, const int64_t *a_off,
                              const double *A, const int64_t *b_off, const double *B, double *X, spd_prec *prec,
                              const spd_opts *o, spd_report *reps, void *hip_stream, int64_t *ticks)
{
    if (batch < 0) return SPD_ERR_INVALID_ARG;
    if (batch == 0) return SPD_OK;
    if (!n || !nrhs || !a_off || !A || !b_off || !B || !X || !prec || !reps) return SPD_ERR_INVALID_ARG;
    if (batch > (int64_t)INT32_MAX) return SPD_ERR_INVALID_ARG;
    const spd_opts op = o ? *o : defaults();
    if (!opts_valid(op)) return SPD_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return SPD_ERR_DEVICE;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    const bool capturing = (cs != hipStreamCaptureStatusNone);

    std::lock_guard<std::mutex> g(g_batch_mu);
    BatchCtx &c = g_batch[dev];
    auto it = c.per_batch.find(batch);
    if (it == c.per_batch.end() && capturing) return SPD_ERR_UNSUPPORTED;
    if (!c.ws) {
        // every candidate's grid fits; never freed, so captured graphs stay valid
        const size_t bytes = (size_t)kBatchMaxGrid * spd::batch_ws_stride();
        HIP_TRY(hipMalloc(&c.ws, bytes));
    }
    if (!capturing) {
        if (!c.last) HIP_TRY(hipEventCreateWithFlags(&c.last, hipEventDisableTiming));
        else if (c.last_stream != st) HIP_TRY(hipStreamWaitEvent(st, c.last, 0));
    }
    spd::BatchLaunch l;
    l.batch = batch;
    l.n = n;
    l.nrhs = nrhs;
    l.a_off = a_off;
    l.b_off = b_off;
    l.A = A;
    l.B = B;
    l.X = X;
    l.prec = (int32_t *)prec;
    l.reps = reps;
    l.tol = op.tol;
    l.mu16 = fp16_scale(op.theta);
    l.max_iter = op.max_iter;
    l.fallback = op.fallback;
    l.equilibrate = op.equilibrate;
    l.ws = c.ws;
    l.picker = c.picker_on ? c.picker : nullptr;
    l.ticks = ticks;
    if (it == c.per_batch.end()) {
        BatchEntry e;
        HIP_TRY(hipMalloc(&e.order, (size_t)batch * sizeof(int32_t) + 256));
        e.queue = (int *)((char *)e.order + (size_t)batch * sizeof(int32_t) + 128);
        // autotune: time every launch shape on this batch, keep the fastest;
        // the requested precisions are restored before each run (prec is in/out)
        int32_t *saved = nullptr;
        HIP_TRY(hipMalloc(&saved, (size_t)batch * sizeof(int32_t)));
        HIP_TRY(hipMemcpyAsync(saved, prec, (size_t)batch * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        hipEvent_t ea, eb;
        HIP_TRY(hipEventCreate(&ea));
        HIP_TRY(hipEventCreate(&eb));
        float best = 1e30f;
        hipError_t err = hipSuccess;
        // a grid chosen for this batch size earlier (the cache file) is reused
        spd::TuneVal tv;
        const std::string key = spd::tune_key("batched", batch);
        const bool cached = spd::tune_lookup(key, &tv) != 0;
        for (int cand : kBatchGrids) {
            if (cached && cand != tv.a) continue;
            l.grid = (int)std::min<int64_t>(cand, batch);
            l.waves = 4;
            l.order = e.order;
            l.queue = e.queue;
            if (err == hipSuccess)
                err = hipMemcpyAsync(prec, saved, (size_t)batch * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
            if (err == hipSuccess) err = hipEventRecord(ea, st);
            if (err == hipSuccess) err = spd::launch_batch(l, st);
            if (err == hipSuccess) err = hipEventRecord(eb, st);
            if (err == hipSuccess) err = hipEventSynchronize(eb);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, ea, eb);
            if (err == hipSuccess && ms < best) {
                best = ms;
                e.grid = l.grid;
                e.waves = l.waves;
                tv.a = cand;
                tv.ms = ms;
            }
        }
        if (err == hipSuccess && !cached) spd::tune_store(key, tv);
        if (err == hipSuccess)
            err = hipMemcpyAsync(prec, saved, (size_t)batch * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
        if (err == hipSuccess) err = hipStreamSynchronize(st);
        hipEventDestroy(ea);
        hipEventDestroy(eb);
        hipFree(saved);
        if (err != hipSuccess) {
            hipFree(e.order);
            return map_err(err);
        }
        it = c.per_batch.emplace(batch, e).first;
    }
    l.grid = it->second.grid;
    l.waves = it->second.waves;
    l.order = it->second.order;
    l.queue = it->second.queue;
    HIP_TRY(spd::launch_batch(l, st));
    if (!capturing) {
        HIP_TRY(hipEventRecord(c.last, st));
        c.last_stream = st;
    }
    return SPD_OK;
}

spd_status spd_solve_batched(int64_t batch, const int32_t *n, const int32_t *nrhs, const int64_t *a_off,
                             const double *A, const int64_t *b_off, const double *B, double *X, spd_prec *prec,
                             const spd_opts *o, spd_report *reps, void *hip_stream)
{
    return solve_batched_impl(batch, n, nrhs, a_off, A, b_off, B, X, prec, o, reps, hip_stream, nullptr);
}

spd_status spd_solve_batched_timed(int64_t batch, const int32_t *n, const int32_t *nrhs, const int64_t *a_off,
                                   const double *A, const int64_t *b_off, const double *B, double *X, spd_prec *prec,
                                   const spd_opts *o, spd_report *reps, int64_t *ticks, void *hip_stream)
{
    if (!ticks && batch > 0) return SPD_ERR_INVALID_ARG;
    return solve_batched_impl(batch, n, nrhs, a_off, A, b_off, B, X, prec, o, reps, hip_stream, ticks);
}

spd_status spd_picker_set(const float *params, void *hip_stream)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return SPD_ERR_DEVICE;
    std::lock_guard<std::mutex> g(g_batch_mu);
    BatchCtx &c = g_batch[dev];
    if (!params) {
        c.picker_on = false;
        return SPD_OK;
    }
    if (!c.picker) HIP_TRY(hipMalloc(&c.picker, SPD_PICKER_NPARAM * sizeof(float)));
    HIP_TRY(hipMemcpyAsync(c.picker, params, SPD_PICKER_NPARAM * sizeof(float), hipMemcpyDeviceToDevice,
                           (hipStream_t)hip_stream));
    c.picker_on = true;
    return SPD_OK;
}

spd_status spd_picker_features(int64_t batch, const int32_t *n, const int32_t *nrhs, const int64_t *a_off,
                               const double *A, float *feat, void *hip_stream)
{
    if (batch < 0) return SPD_ERR_INVALID_ARG;
    if (batch == 0) return SPD_OK;
    if (!n || !nrhs || !a_off || !A || !feat) return SPD_ERR_INVALID_ARG;
    spd::launch_features(batch, n, nrhs, a_off, A, feat, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

spd_status spd_mlp_forward(const float *params, const float *X, int64_t N, float *logits, void *hip_stream)
{
    if (N < 0 || (N > 0 && (!params || !X || !logits))) return SPD_ERR_INVALID_ARG;
    spd::launch_mlp_forward(params, X, N, logits, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

spd_status spd_mlp_grad(const float *params, const float *X, const int32_t *y, int64_t N, float *grad,
                        float *loss, void *hip_stream)
{
    if (N <= 0 || !params || !X || !y || !grad) return SPD_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return SPD_ERR_DEVICE;
    std::lock_guard<std::mutex> g(g_batch_mu);
    BatchCtx &c = g_batch[dev];
    void *p = c.mlp_scratch;
    size_t cap = c.cap_mlp;
    SPD_TRY(grow(&p, &cap, (size_t)spd::mlp_grad_scratch(N) * sizeof(float), false, st));
    c.mlp_scratch = (float *)p;
    c.cap_mlp = cap;
    spd::launch_mlp_grad(params, X, y, N, grad, loss, c.mlp_scratch, st);
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

spd_status spd_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count, int32_t step, float lr,
                        float beta1, float beta2, float eps, void *hip_stream)
{
    if (count < 0 || step < 1 || (count > 0 && (!params || !grad || !m || !v))) return SPD_ERR_INVALID_ARG;
    spd::launch_adam(params, grad, m, v, count, step, lr, beta1, beta2, eps, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

spd_status spd_batched_config(int64_t batch, int32_t *grid, int32_t *waves)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return SPD_ERR_DEVICE;
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto it = g_batch[dev].per_batch.find(batch);
    if (it == g_batch[dev].per_batch.end()) return SPD_ERR_INVALID_ARG;
    if (grid) *grid = it->second.grid;
    if (waves) *waves = it->second.waves;
    return SPD_OK;
}

void spd_factor_destroy(spd_factor_t F)
{
    if (!F) return;
    if (F->side) hipStreamSynchronize(F->side);
    hipFree(F->L);
    hipFree(F->Lh);
    hipFree(F->d);
    hipFree(F->Y);
    hipFree(F->smax);
    hipFree(F->R);
    hipFree(F->P);
    hipFree(F->norms);
    hipFree(F->info_dev);
    hipFree(F->WB);
    hipFree(F->Tb);
    hipFree(F->tP);
    hipFree(F->tctl);
    hipFree(F->terr);
    if (F->terr_host) hipHostFree(F->terr_host);
    if (F->norms_host) hipHostFree(F->norms_host);
    if (F->info_host) hipHostFree(F->info_host);
    for (auto &e : F->ev)
        if (e) hipEventDestroy(e);
    if (F->side) hipStreamDestroy(F->side);
    delete F;
}

spd_status spd_factor_query(spd_factor_t F, int64_t *n, int32_t *prec, int32_t *nb)
{
    if (!F) return SPD_ERR_INVALID_ARG;
    if (n) *n = F->n;
    if (prec) *prec = F->prec;
    if (nb) *nb = F->nb;
    return SPD_OK;
}

spd_status spd_factor_export(spd_factor_t F, double *Lout, int64_t ldl, double *dout, double *mu, void *hip_stream)
{
    if (!F || F->prec < 0) return SPD_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    if (Lout) {
        if (ldl < std::max<int64_t>(1, F->n)) return SPD_ERR_INVALID_ARG;
        if (F->elem == 8)
            spd::launch_export<double>((const double *)F->L, F->npad, F->n, Lout, ldl, st);
        else
            spd::launch_export<float>((const float *)F->L, F->npad, F->n, Lout, ldl, st);
    }
    if (dout && F->n > 0)
        HIP_TRY(hipMemcpyAsync(dout, F->d, F->n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (mu) *mu = F->mu;
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

void spd_cg_opts_default(spd_cg_opts *o)
{
    if (!o) return;
    o->tol = 1e-14;
    o->inner_tol = 1e-6;
    o->max_outer = 30;
    o->max_inner = 2000;
}

spd_status spd_cg_prepare(const double *A, int64_t n, int64_t lda, int64_t half_band, void *hip_stream,
                          spd_cg_t *H)
{
    if (!H || n < 0 || lda < std::max<int64_t>(1, n) || (n > 0 && !A)) return SPD_ERR_INVALID_ARG;
    if (half_band >= 0 && !spd::cg_band_ok(half_band)) return SPD_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)hip_stream;
    spd_cg_t h = *H;
    if (!h) {
        h = new (std::nothrow) spd_cg_s;
        if (!h) return SPD_ERR_OUT_OF_MEMORY;
        *H = h;
    }
    const int64_t ldt = spd::cg_ldt(n);
    const int64_t k = (half_band >= 0 && half_band < n - 1) ? half_band : -1;  // a band covering A is A
    const size_t bytes = ((k >= 0) ? (size_t)(2 * k + 1) * ldt : (size_t)ldt * ldt) * sizeof(float);
    if (h->n != n || h->ldt != ldt || h->k != k) {  // the workspace is laid out for n and k
        HIP_TRY(hipStreamSynchronize(st));
        cg_free_ws(h);
    }
    if (h->cap_At < bytes) {  // the operator's buffer is kept when large enough
        HIP_TRY(hipStreamSynchronize(st));
        hipFree(h->At);
        h->At = nullptr;
        h->cap_At = 0;
        HIP_TRY(hipMalloc(&h->At, bytes));
        h->cap_At = bytes;
    }
    h->n = n;
    h->ldt = ldt;
    h->k = k;
    if (h->k >= 0)
        spd::launch_cg_band(A, lda, n, h->k, h->At, h->ldt, st);
    else
        spd::launch_cg_dense(A, lda, n, h->At, h->ldt, st);
    HIP_TRY(hipGetLastError());
    return SPD_OK;
}

spd_status spd_cg_refine(spd_cg_t H, const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrhs,
                         double *X, int64_t ldx, const spd_cg_opts *o, spd_report *rep, void *hip_stream)
{
    if (!H || !rep) return SPD_ERR_INVALID_ARG;
    const int64_t n = H->n;
    spd_cg_opts oo;
    spd_cg_opts_default(&oo);
    if (o) oo = *o;
    if (nrhs < 0 || nrhs > 65535 || lda < std::max<int64_t>(1, n) || ldb < std::max<int64_t>(1, n) ||
        ldx < std::max<int64_t>(1, n) || !(oo.tol >= 0.0) || !(oo.inner_tol >= 0.0) || oo.max_outer < 0 ||
        oo.max_inner < 0)
        return SPD_ERR_INVALID_ARG;
    if (n > 0 && nrhs > 0 && (!A || !B || !X)) return SPD_ERR_INVALID_ARG;
    std::memset(rep, 0, sizeof(*rep));
    rep->prec_used = SPD_FP32;
    if (n == 0 || nrhs == 0) return SPD_OK;
    const spd_status s = cg_refine(H, A, lda, B, ldb, (int)nrhs, X, ldx, oo, rep, (hipStream_t)hip_stream);
    rep->status = s;
    return s;
}

void spd_cg_destroy(spd_cg_t H)
{
    if (!H) return;
    hipDeviceSynchronize();
    cg_free_ws(H);
    hipFree(H->At);
    if (H->gstream) hipStreamDestroy(H->gstream);
    delete H;
}

}  // extern "C"
