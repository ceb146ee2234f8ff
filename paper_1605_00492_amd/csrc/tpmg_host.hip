// Host side of libtpmg: argument validation, workspace layout, hierarchy
// setup, the V-cycle and CG drivers, and the C interface declared in tpmg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpmg.h"
#include "tpmg_internal.h"

using namespace tpmg;

namespace {

thread_local std::string g_last_error;

constexpr size_t kAlign = 256;

// Pinned host blocks for the scalars a solve reads back (Scalars followed by
// kMultiMax + 2 doubles), kept for reuse by later hierarchies: pinning host
// memory costs more than the rest of the host side of a set-up.
constexpr size_t kPinnedBytes = sizeof(Scalars) + (kMultiMax + 2) * sizeof(double);
std::mutex g_pinned_mu;
std::vector<void *> g_pinned_free;

void *pinned_take()
{
    {
        std::lock_guard<std::mutex> lock(g_pinned_mu);
        if (!g_pinned_free.empty()) {
            void *p = g_pinned_free.back();
            g_pinned_free.pop_back();
            return p;
        }
    }
    void *p = nullptr;
    return hipHostMalloc(&p, kPinnedBytes, hipHostMallocDefault) == hipSuccess ? p : nullptr;
}

void pinned_give(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    g_pinned_free.push_back(p);
}

struct LevelBufs {
    int n = 0, plane = 0;
    void *c = nullptr;                       // [3][nz * plane], tiled storage
    void *mu = nullptr, *wh = nullptr, *wz = nullptr;  // [nz]
    void *b = nullptr, *A = nullptr, *B = nullptr, *E = nullptr;  // level vectors
};

struct EventPool {
    std::vector<hipEvent_t> start, stop;
    int used = 0;
    double acc_ms = 0.0;
    int64_t launches = 0;
};

}  // namespace

struct tpmg_hierarchy {
    tpmg_desc d{};
    std::vector<double> dz;  // host copy of the spacings (empty = uniform)
    int L = 0, nz = 0;
    size_t ncell = 0;        // cells on level 0
    bool mixed = false;
    LevelBufs l64[TPMG_MAX_LEVELS], l32[TPMG_MAX_LEVELS];
    double *ainv64 = nullptr;
    float *ainv32 = nullptr;
    int m_coarse = 0;
    // FP64 vectors for the outer iteration and layout staging
    double *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    double *stage0 = nullptr, *stage1 = nullptr;  // stage0 heads 3 contiguous cell vectors
    float *r32 = nullptr, *z32 = nullptr;
    double *partials = nullptr;
    Scalars *sc = nullptr;
    int *bad = nullptr;
    void *scal[2] = {nullptr, nullptr};  // per-level scalars mu, wh, wz of all levels: FP64, FP32
    Scalars *sc_host = nullptr;  // pinned, followed by kMultiMax + 2 doubles (dots_host)
    double *dots_host = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
    bool prof = false, prof_levels = false;
    EventPool pools[TPMG_K_COUNT + TPMG_MAX_LEVELS];  // kernel classes, then one per level
    // damping of the sweeps of the next V-cycle: d.omega, except inside a
    // solve whose options make the preconditioner vary between iterations
    double omega_run = 0.0;
};

namespace {

tpmg_status fail(tpmg_hierarchy *h, tpmg_status s, const std::string &msg)
{
    if (h) h->err = msg;
    g_last_error = msg;
    return s;
}

tpmg_status hip_fail(tpmg_hierarchy *h, hipError_t e, const char *where)
{
    std::string msg = std::string(where) + ": " + hipGetErrorString(e);
    return fail(h, TPMG_ERR_DEVICE, msg);
}

#define HIP_TRY(h, expr)                                    \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail((h), e_, #expr); \
    } while (0)

tpmg_status validate_desc(const tpmg_desc *d)
{
    if (!d) return fail(nullptr, TPMG_ERR_INVALID_ARG, "desc is NULL");
    if (d->nlevels < 1 || d->nlevels > TPMG_MAX_LEVELS)
        return fail(nullptr, TPMG_ERR_SHAPE, "nlevels out of range");
    if (d->nz < 1 || d->nz > TPMG_MAX_NZ) return fail(nullptr, TPMG_ERR_SHAPE, "nz out of range");
    if (d->n < 1 || d->n > 16384) return fail(nullptr, TPMG_ERR_SHAPE, "n out of range");
    if (d->n % (1 << (d->nlevels - 1)) != 0)
        return fail(nullptr, TPMG_ERR_SHAPE, "n must be divisible by 2^(nlevels-1)");
    const double dof = (double)d->n * d->n * d->nz;
    // reductions use one partial per workgroup of 256 columns x (4 to 16)
    // cells; kernels address each FP64 level array with 32-bit byte offsets
    if (dof / (256.0 * 4.0) > (double)kMaxPartials * 0.9 || dof * 8.0 >= 4294967296.0)
        return fail(nullptr, TPMG_ERR_SHAPE, "grid too large");
    if (!(d->a_h >= 0.0) || !(d->a_z >= 0.0) || !std::isfinite(d->a_h) || !std::isfinite(d->a_z))
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "a_h and a_z must be finite and >= 0");
    if (d->nu_pre < 1 || d->nu_post < 1 || d->nu_pre > 64 || d->nu_post > 64)
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "nu_pre and nu_post must be in [1, 64]");
    if (!(d->omega > 0.0 && d->omega <= 1.0))
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "omega must be in (0, 1]");
    if (d->coarse != TPMG_COARSE_DIRECT && d->coarse != TPMG_COARSE_SMOOTH)
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "bad coarse mode");
    if (d->coarse == TPMG_COARSE_SMOOTH && (d->n_coarse < 1 || d->n_coarse > 64))
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "n_coarse must be in [1, 64]");
    if (d->precision != TPMG_FP64 && d->precision != TPMG_MIXED_FP32_VCYCLE)
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "bad precision");
    if (d->coarse == TPMG_COARSE_DIRECT) {
        const long nc = d->n >> (d->nlevels - 1);
        if (nc * nc * (long)d->nz > TPMG_MAX_DIRECT_DOF)
            return fail(nullptr, TPMG_ERR_SHAPE, "coarsest level too large for the direct solve");
    }
    int M, CPW, P;
    bool shape_ok = true;
    for (int mode : {SWEEP_ZERO, SWEEP_GENERAL, SWEEP_PROLONG})
        shape_ok = shape_ok && sweep_shape(d->nz, false, mode, &M, &CPW, &P) && sweep_shape(d->nz, true, mode, &M, &CPW, &P);
    if (!shape_ok)
        return fail(nullptr, TPMG_ERR_SHAPE, "nz not supported");
    if (d->dz)
        for (int k = 0; k < d->nz; ++k)
            if (!(d->dz[k] > 0.0) || !std::isfinite(d->dz[k]))
                return fail(nullptr, TPMG_ERR_NOT_SPD, "dz must be positive and finite");
    return TPMG_OK;
}

// Carve the workspace.  With h == nullptr only the size is computed.
size_t plan_workspace(const tpmg_desc &d, tpmg_hierarchy *h)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = (off + kAlign - 1) / kAlign * kAlign;
        void *p = h ? (void *)(h->ws + off) : nullptr;
        off += bytes;
        return p;
    };
    const bool mixed = d.precision == TPMG_MIXED_FP32_VCYCLE;
    const size_t nz = (size_t)d.nz;
    for (int pass = 0; pass < (mixed ? 2 : 1); ++pass) {
        const size_t S = pass == 0 ? sizeof(double) : sizeof(float);
        // mu, wh, wz of every level in one block, uploaded by one copy
        char *scal = (char *)take((size_t)d.nlevels * 3 * nz * S);
        if (h) h->scal[pass] = scal;
        for (int l = 0; l < d.nlevels; ++l) {
            const int n = d.n >> l;
            const size_t cells = (size_t)n * n * nz;
            LevelBufs tmp;
            LevelBufs &B = h ? (pass == 0 ? h->l64[l] : h->l32[l]) : tmp;
            B.n = n;
            B.plane = n * n;
            B.c = take(3 * cells * S);
            if (h) {
                B.mu = scal + (size_t)(3 * l + 0) * nz * S;
                B.wh = scal + (size_t)(3 * l + 1) * nz * S;
                B.wz = scal + (size_t)(3 * l + 2) * nz * S;
            }
            B.A = take(cells * S);
            B.B = take(cells * S);
            if (l > 0) {
                B.b = take(cells * S);
                B.E = take(cells * S);
            }
        }
    }
    const size_t ncell = (size_t)d.n * d.n * nz;
    if (d.coarse == TPMG_COARSE_DIRECT) {
        const size_t nc = (size_t)(d.n >> (d.nlevels - 1));
        const size_t m = nc * nc * nz;
        void *a64 = take(m * m * sizeof(double));
        void *a32 = mixed ? take(m * m * sizeof(float)) : nullptr;
        if (h) {
            h->ainv64 = (double *)a64;
            h->ainv32 = (float *)a32;
            h->m_coarse = (int)m;
        }
    }
    double *vec[5];
    for (int i = 0; i < 5; ++i) vec[i] = (double *)take(ncell * sizeof(double));
    double *stage = (double *)take(3 * ncell * sizeof(double));
    float *r32 = mixed ? (float *)take(ncell * sizeof(float)) : nullptr;
    float *z32 = mixed ? (float *)take(ncell * sizeof(float)) : nullptr;
    double *partials = (double *)take((2 * (size_t)kMaxPartials + 2 * kReduceSegs) * sizeof(double));
    Scalars *sc = (Scalars *)take(sizeof(Scalars));
    int *bad = (int *)take(sizeof(int) * 4);
    if (h) {
        h->r = vec[0];
        h->z = vec[1];
        h->p0 = vec[2];
        h->p1 = vec[3];
        h->q = vec[4];
        h->stage0 = stage;
        h->stage1 = stage + ncell;
        h->r32 = r32;
        h->z32 = z32;
        h->partials = partials;
        h->sc = sc;
        h->bad = bad;
    }
    return (off + kAlign - 1) / kAlign * kAlign;
}

template <typename T>
Level<T> level_view(const tpmg_hierarchy *h, int l)
{
    const LevelBufs &B = (sizeof(T) == 8) ? h->l64[l] : h->l32[l];
    Level<T> L;
    L.n = B.n;
    L.nz = h->nz;
    L.plane = B.plane;
    L.c = (const T *)B.c;
    L.mu = (const T *)B.mu;
    L.wh = (const T *)B.wh;
    L.wz = (const T *)B.wz;
    static const char *ef = getenv("TPMG_FULL_CHUNKS");
    L.full_chunks = !(ef && atoi(ef) == 0);
    return L;
}

template <typename T>
const LevelBufs &bufs(const tpmg_hierarchy *h, int l)
{
    return (sizeof(T) == 8) ? h->l64[l] : h->l32[l];
}

// ---- profiling --------------------------------------------------------------

// Event pool of the kernels that run on V-cycle level l.
constexpr int kLevelPool = TPMG_K_COUNT;
constexpr int kPools = TPMG_K_COUNT + TPMG_MAX_LEVELS;

struct Timed {
    tpmg_hierarchy *h;
    int cls;
    hipStream_t s;
    bool on;
    Timed(const tpmg_hierarchy *hc, int c, hipStream_t st) : h(const_cast<tpmg_hierarchy *>(hc)), cls(c), s(st)
    {
        on = h->prof && cls >= 0 && (cls < kLevelPool || h->prof_levels);
        if (!on) return;
        EventPool &P = h->pools[cls];
        if (P.used == (int)P.start.size()) {
            // pool full: fold the recorded pairs into the running total
            for (int i = 0; i < P.used; ++i) {
                float ms = 0;
                (void)hipEventSynchronize(P.stop[i]);
                (void)hipEventElapsedTime(&ms, P.start[i], P.stop[i]);
                P.acc_ms += ms;
            }
            P.used = 0;
        }
        (void)hipEventRecord(P.start[P.used], s);
    }
    ~Timed()
    {
        if (!on) return;
        EventPool &P = h->pools[cls];
        (void)hipEventRecord(P.stop[P.used], s);
        ++P.used;
        ++P.launches;
    }
};

// ---- V-cycle ----------------------------------------------------------------

template <typename T>
tpmg_status sweep(const tpmg_hierarchy *h, int l, int mode, const T *u, const T *b, T *out, const T *ec,
                  hipStream_t s)
{
    int cls = -1;
    if (l == 0) cls = mode == SWEEP_ZERO ? TPMG_K_SWEEP0 : (mode == SWEEP_GENERAL ? TPMG_K_SWEEP : TPMG_K_PROLSWEEP);
    Timed t(h, cls, s), tl(h, kLevelPool + l, s);
    HIP_TRY(const_cast<tpmg_hierarchy *>(h),
            launch_sweep<T>(level_view<T>(h, l), mode, u, b, out, ec, (T)h->omega_run, s));
    return TPMG_OK;
}

template <typename T>
tpmg_status coarse_solve(const tpmg_hierarchy *h, const T *b, T *out, hipStream_t s)
{
    const int l = h->L - 1;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (h->d.coarse == TPMG_COARSE_DIRECT) {
        const T *ainv = (sizeof(T) == 8) ? (const T *)h->ainv64 : (const T *)h->ainv32;
        Timed tl(h, kLevelPool + l, s);
        HIP_TRY(hm, launch_coarse_gemv<T>(ainv, h->m_coarse, b, out, s));
        return TPMG_OK;
    }
    const LevelBufs &B = bufs<T>(h, l);
    T *A = (T *)B.A, *Bb = (T *)B.B;
    const int nsw = h->d.n_coarse;
    const T *prev = nullptr;
    for (int i = 0; i < nsw; ++i) {
        T *dst = (i == nsw - 1) ? out : ((i % 2 == 0) ? A : Bb);
        tpmg_status st = sweep<T>(h, l, i == 0 ? SWEEP_ZERO : SWEEP_GENERAL, prev, b, dst, nullptr, s);
        if (st != TPMG_OK) return st;
        prev = dst;
    }
    return TPMG_OK;
}

// z = V_l b (zero initial guess), Sec. 3 cycle M1-M5 applied recursively.
template <typename T>
tpmg_status vcycle_level(const tpmg_hierarchy *h, int l, const T *b, T *out, hipStream_t s)
{
    if (l == h->L - 1) return coarse_solve<T>(h, b, out, s);
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    const LevelBufs &B = bufs<T>(h, l);
    const LevelBufs &C = bufs<T>(h, l + 1);
    T *cur = (T *)B.A, *other = (T *)B.B;
    tpmg_status st = sweep<T>(h, l, SWEEP_ZERO, nullptr, b, cur, nullptr, s);  // M1
    if (st != TPMG_OK) return st;
    for (int i = 1; i < h->d.nu_pre; ++i) {
        if ((st = sweep<T>(h, l, SWEEP_GENERAL, cur, b, other, nullptr, s)) != TPMG_OK) return st;
        std::swap(cur, other);
    }
    {
        Timed t(h, l == 0 ? TPMG_K_RESTRICT : -1, s), tl(h, kLevelPool + l, s);  // M2
        HIP_TRY(hm, launch_resid_restrict<T>(level_view<T>(h, l), cur, b, (T *)C.b, s));
    }
    if ((st = vcycle_level<T>(h, l + 1, (const T *)C.b, (T *)C.E, s)) != TPMG_OK) return st;  // M3
    const T *src = cur;
    for (int i = 0; i < h->d.nu_post; ++i) {  // M4 (fused into the first sweep), M5
        T *dst = (i == h->d.nu_post - 1) ? out : ((i % 2 == 0) ? other : cur);
        st = (i == 0) ? sweep<T>(h, l, SWEEP_PROLONG, src, b, dst, (const T *)C.E, s)
                      : sweep<T>(h, l, SWEEP_GENERAL, src, b, dst, nullptr, s);
        if (st != TPMG_OK) return st;
        src = dst;
    }
    return TPMG_OK;
}

template <typename T>
tpmg_status vcycle(const tpmg_hierarchy *h, const T *b, T *out, hipStream_t s)
{
    Timed t(h, TPMG_K_VCYCLE, s);
    return vcycle_level<T>(h, 0, b, out, s);
}

// ---- host factorisation of the coarsest operator (direct mode) -----------------

// Dense H on the coarsest level, rows and columns in the level's storage
// order (so the dense inverse applies directly to stored vectors), assembled
// from the level's face coefficients and scalars.
void assemble_dense(const std::vector<double> &c, const std::vector<double> &mu, const std::vector<double> &wh,
                    const std::vector<double> &wz, int n, int nz, std::vector<double> &A)
{
    const int plane = n * n;
    const size_t m = (size_t)plane * nz;
    A.assign(m * m, 0.0);
    const size_t fs = (size_t)plane * nz;
    auto idx = [&](int i, int j, int k) -> size_t {
        i = (i % n + n) % n;
        j = (j % n + n) % n;
        return cell_index((size_t)j * n + i, k, plane, nz);
    };
    auto couple = [&](size_t p, size_t q, double w) {
        A[p * m + p] += w;
        A[q * m + q] += w;
        A[p * m + q] -= w;
        A[q * m + p] -= w;
    };
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const size_t p = idx(i, j, k);
                A[p * m + p] += mu[k];
                couple(p, idx(i + 1, j, k), wh[k] * c[p]);
                couple(p, idx(i, j + 1, k), wh[k] * c[fs + p]);
                if (k + 1 < nz) couple(p, idx(i, j, k + 1), wz[k] * c[2 * fs + p]);
            }
}

// A^{-1} of a dense SPD matrix via Cholesky A = C C^T, W = C^{-1}, A^{-1} = W^T W.
bool spd_inverse(std::vector<double> &A, size_t m, std::vector<double> &Ainv)
{
    for (size_t j = 0; j < m; ++j) {
        double *Aj = &A[j * m];
        double d = Aj[j];
        for (size_t p = 0; p < j; ++p) d -= Aj[p] * Aj[p];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        Aj[j] = d;
        for (size_t i = j + 1; i < m; ++i) {
            double *Ai = &A[i * m];
            double s = Ai[j];
            for (size_t p = 0; p < j; ++p) s -= Ai[p] * Aj[p];
            Ai[j] = s / d;
        }
    }
    // rows of W = C^{-1}: W[c][i] for i >= c holds (C^{-1})_{i c}
    std::vector<double> W(m * m, 0.0);
    for (size_t c = 0; c < m; ++c) {
        double *w = &W[c * m];
        for (size_t i = c; i < m; ++i) {
            const double *Ci = &A[i * m];
            double s = (i == c) ? 1.0 : 0.0;
            for (size_t p = c; p < i; ++p) s -= Ci[p] * w[p];
            w[i] = s / Ci[i];
        }
    }
    Ainv.assign(m * m, 0.0);
    for (size_t a = 0; a < m; ++a)
        for (size_t b = a; b < m; ++b) {
            const double *wa = &W[a * m], *wb = &W[b * m];
            double s = 0.0;
            for (size_t i = std::max(a, b); i < m; ++i) s += wa[i] * wb[i];
            Ainv[a * m + b] = s;
            Ainv[b * m + a] = s;
        }
    return true;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

tpmg_status check_handle(const tpmg_hierarchy *h)
{
    if (!h) return fail(nullptr, TPMG_ERR_INVALID_ARG, "hierarchy is NULL");
    return TPMG_OK;
}

tpmg_status check_fp32(const tpmg_hierarchy *h, int fp32)
{
    if (fp32 != 0 && fp32 != 1) return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG, "fp32 must be 0 or 1");
    if (fp32 && !h->mixed)
        return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG,
                    "fp32 requires a TPMG_MIXED_FP32_VCYCLE hierarchy");
    return TPMG_OK;
}

tpmg_status check_layout(const tpmg_hierarchy *h, int layout)
{
    if (layout != TPMG_LAYOUT_LEVEL_MAJOR && layout != TPMG_LAYOUT_COLUMN_MAJOR)
        return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG, "bad layout");
    return TPMG_OK;
}

tpmg_status check_ptrs(const tpmg_hierarchy *h, std::initializer_list<const void *> ps)
{
    for (const void *p : ps) {
        if (!p) return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG, "NULL buffer");
        if (!aligned16(p)) return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG, "buffer not 16-byte aligned");
    }
    return TPMG_OK;
}

// Reduce the partials of the last launch into the scalars.
tpmg_status finalize(tpmg_hierarchy *h, int G, int nvals, int stage, int flexible, hipStream_t s)
{
    HIP_TRY(h, launch_finalize(h->partials, G, nvals, h->sc, stage, flexible, h->partials + 2 * (size_t)kMaxPartials,
                               s));
    return TPMG_OK;
}

tpmg_status read_scalars(tpmg_hierarchy *h, hipStream_t s)
{
    HIP_TRY(h, hipMemcpyAsync(h->sc_host, h->sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    return TPMG_OK;
}

// z = V r in the hierarchy's precision (mixed: r32 must already hold fl32(r)).
tpmg_status precondition(tpmg_hierarchy *h, hipStream_t s)
{
    if (h->mixed) return vcycle<float>(h, h->r32, h->z32, s);
    return vcycle<double>(h, h->r, h->z, s);
}

// The component entry points take the caller's level-major vectors and stage
// them in the level's storage order through the CG vectors r, z, p0, p1
// (free outside tpmg_solve; each holds a level-0 FP64 vector).
tpmg_status stage_in(const tpmg_hierarchy *h, const void *src, void *dst, int level, int elem, hipStream_t s)
{
    HIP_TRY(const_cast<tpmg_hierarchy *>(h),
            launch_cells_in(src, TPMG_LAYOUT_LEVEL_MAJOR, dst, nullptr, h->l64[level].plane, h->nz, elem, s));
    return TPMG_OK;
}

tpmg_status stage_out(const tpmg_hierarchy *h, const void *src, void *dst, int level, int elem, hipStream_t s)
{
    HIP_TRY(const_cast<tpmg_hierarchy *>(h),
            launch_cells_out(src, dst, TPMG_LAYOUT_LEVEL_MAJOR, h->l64[level].plane, h->nz, elem, s));
    return TPMG_OK;
}

template <typename T>
tpmg_status smooth_impl(const tpmg_hierarchy *h, int level, const void *u, const void *b, void *out,
                               hipStream_t s)
{
    tpmg_status st;
    T *us = (T *)h->r, *bs = (T *)h->z, *os = (T *)h->p0;
    if (u && (st = stage_in(h, u, us, level, sizeof(T), s)) != TPMG_OK) return st;
    if ((st = stage_in(h, b, bs, level, sizeof(T), s)) != TPMG_OK) return st;
    if ((st = sweep<T>(h, level, u ? SWEEP_GENERAL : SWEEP_ZERO, u ? us : nullptr, bs, os, nullptr, s)) != TPMG_OK)
        return st;
    return stage_out(h, os, out, level, sizeof(T), s);
}

template <typename T>
tpmg_status resid_restrict_impl(const tpmg_hierarchy *h, int level, const void *u, const void *b, void *bc,
                                hipStream_t s)
{
    tpmg_status st;
    T *us = (T *)h->r, *bs = (T *)h->z, *os = (T *)h->p0;
    if ((st = stage_in(h, u, us, level, sizeof(T), s)) != TPMG_OK) return st;
    if ((st = stage_in(h, b, bs, level, sizeof(T), s)) != TPMG_OK) return st;
    HIP_TRY(const_cast<tpmg_hierarchy *>(h), launch_resid_restrict<T>(level_view<T>(h, level), us, bs, os, s));
    return stage_out(h, os, bc, level + 1, sizeof(T), s);
}

template <typename T>
tpmg_status prolong_smooth_impl(const tpmg_hierarchy *h, int level, const void *u, const void *ec, const void *b,
                                void *out, hipStream_t s)
{
    tpmg_status st;
    T *us = (T *)h->r, *es = (T *)h->z, *bs = (T *)h->p0, *os = (T *)h->p1;
    if ((st = stage_in(h, u, us, level, sizeof(T), s)) != TPMG_OK) return st;
    if ((st = stage_in(h, ec, es, level + 1, sizeof(T), s)) != TPMG_OK) return st;
    if ((st = stage_in(h, b, bs, level, sizeof(T), s)) != TPMG_OK) return st;
    if ((st = sweep<T>(h, level, SWEEP_PROLONG, us, bs, os, es, s)) != TPMG_OK) return st;
    return stage_out(h, os, out, level, sizeof(T), s);
}

template <typename T>
tpmg_status coarse_solve_impl(const tpmg_hierarchy *h, const void *b, void *u, hipStream_t s)
{
    tpmg_status st;
    const int l = h->L - 1;
    T *bs = (T *)h->r, *os = (T *)h->z;
    if ((st = stage_in(h, b, bs, l, sizeof(T), s)) != TPMG_OK) return st;
    if ((st = coarse_solve<T>(h, bs, os, s)) != TPMG_OK) return st;
    return stage_out(h, os, u, l, sizeof(T), s);
}

// Sum of the recorded event pairs of one pool (synchronises them).
tpmg_status read_pool(tpmg_hierarchy *h, int pool, double *total_ms, int64_t *launches)
{
    EventPool &P = h->pools[pool];
    for (int i = 0; i < P.used; ++i) {
        float ms = 0;
        HIP_TRY(h, hipEventSynchronize(P.stop[i]));
        HIP_TRY(h, hipEventElapsedTime(&ms, P.start[i], P.stop[i]));
        P.acc_ms += ms;
    }
    P.used = 0;
    *total_ms = P.acc_ms;
    *launches = P.launches;
    return TPMG_OK;
}

// ---- staging memory of tpmg_apply_operator_static -------------------------------
// A file-scope device array, so that the entry point needs neither an
// allocation nor the hierarchy's own staging vectors.  Every GPU the library
// runs on holds its own copy until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is passed to
// kernels.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
tpmg_status static_scratch(tpmg_hierarchy *h, void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(h, e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(h, TPMG_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(h, e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(h, TPMG_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TPMG_OK;
}

}  // namespace

// =============================================================================
// C interface
// =============================================================================

extern "C" {

tpmg_status tpmg_workspace_bytes(const tpmg_desc *desc, size_t *bytes)
{
    tpmg_status st = validate_desc(desc);
    if (st != TPMG_OK) return st;
    if (!bytes) return fail(nullptr, TPMG_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = plan_workspace(*desc, nullptr);
    return TPMG_OK;
}

tpmg_status tpmg_setup_hierarchy(const tpmg_desc *desc, const double *c_dev, int32_t layout, void *workspace_dev,
                                 size_t workspace_bytes, void *stream, tpmg_hierarchy **out)
{
    tpmg_status st = validate_desc(desc);
    if (st != TPMG_OK) return st;
    if (!out) return fail(nullptr, TPMG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (layout != TPMG_LAYOUT_LEVEL_MAJOR && layout != TPMG_LAYOUT_COLUMN_MAJOR)
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "bad layout");
    if (!c_dev || !aligned16(c_dev)) return fail(nullptr, TPMG_ERR_INVALID_ARG, "c is NULL or misaligned");
    const size_t need = plan_workspace(*desc, nullptr);
    if (!workspace_dev || workspace_bytes < need || ((uintptr_t)workspace_dev % kAlign) != 0)
        return fail(nullptr, TPMG_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");

    tpmg_hierarchy *h = new tpmg_hierarchy();
    h->d = *desc;
    h->omega_run = desc->omega;
    if (desc->dz) h->dz.assign(desc->dz, desc->dz + desc->nz);
    h->d.dz = nullptr;
    h->L = desc->nlevels;
    h->nz = desc->nz;
    h->ncell = (size_t)desc->n * desc->n * desc->nz;
    h->mixed = desc->precision == TPMG_MIXED_FP32_VCYCLE;
    h->ws = (char *)workspace_dev;
    h->ws_bytes = workspace_bytes;
    plan_workspace(*desc, h);
    hipStream_t s = as_stream(stream);

    auto bail = [&](tpmg_status code) {
        g_last_error = h->err;
        (void)hipStreamSynchronize(s);  // copies from host buffers of this call may be in flight
        pinned_give(h->sc_host);
        delete h;
        return code;
    };
    h->sc_host = (Scalars *)pinned_take();
    if (!h->sc_host) return bail(fail(h, TPMG_ERR_DEVICE, "hipHostMalloc failed"));
    h->dots_host = reinterpret_cast<double *>(reinterpret_cast<char *>(h->sc_host) + sizeof(Scalars));

    // per-level scalars: s_k, t_{k+1/2}
    const int nz = desc->nz;
    std::vector<double> sk(nz, 1.0), tk(nz, 1.0);
    {
        double mean = 0.0;
        for (int k = 0; k < nz; ++k) mean += desc->dz ? desc->dz[k] : 1.0;
        mean /= nz;
        for (int k = 0; k < nz; ++k) sk[k] = (desc->dz ? desc->dz[k] : 1.0) / mean;
        for (int k = 0; k + 1 < nz; ++k) tk[k] = 0.5 * (sk[k] + sk[k + 1]);
    }
    std::vector<std::vector<double>> mu(h->L), wh(h->L), wz(h->L);
    // the blocks uploaded to h->scal (level l: mu, wh, wz), alive until the
    // synchronisation below
    std::vector<double> s64((size_t)h->L * 3 * nz);
    std::vector<float> s32(h->mixed ? s64.size() : 0);
    for (int l = 0; l < h->L; ++l) {
        const double f = std::ldexp(1.0, 2 * l);
        mu[l].resize(nz);
        wh[l].resize(nz);
        wz[l].resize(nz);
        for (int k = 0; k < nz; ++k) {
            mu[l][k] = f * sk[k];
            wh[l][k] = desc->a_h * sk[k];
            wz[l][k] = (k + 1 < nz) ? f * desc->a_z / tk[k] : 0.0;
            const size_t o = (size_t)3 * l * nz + k;
            s64[o] = mu[l][k];
            s64[o + nz] = wh[l][k];
            s64[o + 2 * nz] = wz[l][k];
        }
    }
    for (size_t i = 0; i < s32.size(); ++i) s32[i] = (float)s64[i];
    hipError_t e;
    if ((e = hipMemcpyAsync(h->scal[0], s64.data(), s64.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (h->mixed && (e = hipMemcpyAsync(h->scal[1], s32.data(), s32.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess))
        return bail(hip_fail(h, e, "copy level scalars"));
    const int plane0 = desc->n * desc->n;
    if ((e = launch_fill((double *)h->bad, 0.0, 1, s)) != hipSuccess ||
        (e = launch_copy_coeffs(c_dev, layout, (double *)h->l64[0].c, h->mixed ? (float *)h->l32[0].c : nullptr,
                                plane0, nz, h->bad, s)) != hipSuccess)
        return bail(hip_fail(h, e, "copy coefficients"));
    for (int l = 0; l + 1 < h->L; ++l)
        if ((e = launch_coarsen(level_view<double>(h, l), (double *)h->l64[l + 1].c,
                                h->mixed ? (float *)h->l32[l + 1].c : nullptr, s)) != hipSuccess)
            return bail(hip_fail(h, e, "coarsen"));
    int bad = 0;
    if ((e = hipMemcpyAsync(&bad, h->bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(hip_fail(h, e, "setup"));
    if (bad) return bail(fail(h, TPMG_ERR_NOT_SPD, std::to_string(bad) + " face coefficient(s) not positive and finite"));

    if (desc->coarse == TPMG_COARSE_DIRECT) {
        const int l = h->L - 1;
        const int n = h->l64[l].n;
        const size_t cells = (size_t)n * n * nz;
        std::vector<double> c(3 * cells);
        if ((e = hipMemcpy(c.data(), h->l64[l].c, 3 * cells * 8, hipMemcpyDeviceToHost)) != hipSuccess)
            return bail(hip_fail(h, e, "read coarsest coefficients"));
        std::vector<double> A, Ainv;
        assemble_dense(c, mu[l], wh[l], wz[l], n, nz, A);
        if (!spd_inverse(A, cells, Ainv)) return bail(fail(h, TPMG_ERR_NOT_SPD, "coarsest operator not SPD"));
        if ((e = hipMemcpy(h->ainv64, Ainv.data(), cells * cells * 8, hipMemcpyHostToDevice)) != hipSuccess)
            return bail(hip_fail(h, e, "upload coarse inverse"));
        if (h->mixed) {
            if ((e = launch_cast(h->ainv64, h->ainv32, cells * cells, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return bail(hip_fail(h, e, "cast coarse inverse"));
        }
    }
    *out = h;
    return TPMG_OK;
}

int32_t tpmg_level_n(const tpmg_hierarchy *h, int32_t level)
{
    if (!h || level < 0 || level >= h->L) return -1;
    return h->l64[level].n;
}

tpmg_status tpmg_apply_operator(const tpmg_hierarchy *h, int32_t level, int32_t fp32, const void *x_dev,
                                void *y_dev, int32_t layout, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (level < 0 || level >= h->L) return fail(hm, TPMG_ERR_INVALID_ARG, "level out of range");
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_layout(h, layout)) != TPMG_OK ||
        (st = check_ptrs(h, {x_dev, y_dev})) != TPMG_OK)
        return st;
    hipStream_t s = as_stream(stream);
    const int elem = fp32 ? 4 : 8;
    const int plane = h->l64[level].plane;
    void *x = h->stage0, *y = h->stage1;
    HIP_TRY(hm, launch_cells_in(x_dev, layout, x, nullptr, plane, h->nz, elem, s));
    if (fp32)
        HIP_TRY(hm, launch_apply<float>(level_view<float>(h, level), (const float *)x, (float *)y, s));
    else
        HIP_TRY(hm, launch_apply<double>(level_view<double>(h, level), (const double *)x, (double *)y, s));
    HIP_TRY(hm, launch_cells_out(y, y_dev, layout, plane, h->nz, elem, s));
    return TPMG_OK;
}

tpmg_status tpmg_apply_operator_static(const tpmg_hierarchy *h, int32_t level, int32_t fp32, const void *x_dev,
                                       void *y_dev, int32_t layout, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (level < 0 || level >= h->L) return fail(hm, TPMG_ERR_INVALID_ARG, "level out of range");
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_layout(h, layout)) != TPMG_OK ||
        (st = check_ptrs(h, {x_dev, y_dev})) != TPMG_OK)
        return st;
    const int elem = fp32 ? 4 : 8;
    const int plane = h->l64[level].plane;
    const size_t half = kStaticScratchBytes / 2;
    if ((size_t)plane * h->nz * elem > half)
        return fail(hm, TPMG_ERR_WORKSPACE,
                    "level has " + std::to_string((size_t)plane * h->nz) + " cells; the static scratch stages at most " +
                        std::to_string(half / elem) + " per vector");
    void *base = nullptr;
    if ((st = static_scratch(hm, &base)) != TPMG_OK) return st;
    // both halves are written in full before they are read: nothing to clear
    void *x = base, *y = (char *)base + half;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hm, launch_cells_in(x_dev, layout, x, nullptr, plane, h->nz, elem, s));
    if (fp32)
        HIP_TRY(hm, launch_apply<float>(level_view<float>(h, level), (const float *)x, (float *)y, s));
    else
        HIP_TRY(hm, launch_apply<double>(level_view<double>(h, level), (const double *)x, (double *)y, s));
    HIP_TRY(hm, launch_cells_out(y, y_dev, layout, plane, h->nz, elem, s));
    return TPMG_OK;
}

tpmg_status tpmg_vcycle(const tpmg_hierarchy *h, int32_t fp32, const void *b_dev, void *z_dev, int32_t layout,
                        void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_layout(h, layout)) != TPMG_OK ||
        (st = check_ptrs(h, {b_dev, z_dev})) != TPMG_OK)
        return st;
    if (b_dev == z_dev) return fail(hm, TPMG_ERR_INVALID_ARG, "b and z must not alias");
    hipStream_t s = as_stream(stream);
    const int elem = fp32 ? 4 : 8;
    const int plane = h->l64[0].plane;
    void *b = h->stage0, *z = h->stage1;
    HIP_TRY(hm, launch_cells_in(b_dev, layout, b, nullptr, plane, h->nz, elem, s));
    st = fp32 ? vcycle<float>(h, (const float *)b, (float *)z, s) : vcycle<double>(h, (const double *)b, (double *)z, s);
    if (st != TPMG_OK) return st;
    HIP_TRY(hm, launch_cells_out(z, z_dev, layout, plane, h->nz, elem, s));
    return TPMG_OK;
}

tpmg_status tpmg_solve(const tpmg_hierarchy *hc, const double *b_dev, double *x_dev, int32_t layout,
                       const tpmg_solve_opts *opts, tpmg_solve_info *info, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(hc)) != TPMG_OK) return st;
    tpmg_hierarchy *h = const_cast<tpmg_hierarchy *>(hc);
    if ((st = check_layout(h, layout)) != TPMG_OK || (st = check_ptrs(h, {b_dev, x_dev})) != TPMG_OK) return st;
    if (!opts) return fail(h, TPMG_ERR_INVALID_ARG, "opts is NULL");
    if (!(opts->rtol >= 0.0) || opts->maxit < 0 || (opts->flexible != 0 && opts->flexible != 1) ||
        (opts->x0_nonzero != 0 && opts->x0_nonzero != 1) ||
        !(opts->omega_alt == 0.0 || (opts->omega_alt > 0.0 && opts->omega_alt <= 1.0)))
        return fail(h, TPMG_ERR_INVALID_ARG, "bad solve options");
    if ((const void *)b_dev == (const void *)x_dev) return fail(h, TPMG_ERR_INVALID_ARG, "b and x must not alias");
    hipStream_t s = as_stream(stream);
    const size_t n = h->ncell;
    const int plane = h->l64[0].plane;
    const Level<double> L0 = level_view<double>(h, 0);
    const int flex = opts->flexible;
    // V-cycle number i (the first is 0) uses omega_alt when i is odd and
    // omega_alt > 0, else the hierarchy's omega
    int napply = 0;
    auto next_omega = [&]() {
        h->omega_run = (opts->omega_alt > 0.0 && (napply++ % 2) == 1) ? opts->omega_alt : h->d.omega;
    };
    struct OmegaReset {
        tpmg_hierarchy *h;
        ~OmegaReset() { h->omega_run = h->d.omega; }
    } omega_reset{h};

    // b and x in the level's storage order (stage0, stage1)
    double *b = h->stage0, *x = h->stage1;
    HIP_TRY(h, launch_fill((double *)h->sc, 0.0, sizeof(Scalars) / sizeof(double), s));
    int G = 0;
    bool r32_ready = false;  // fl32(r) already written
    // Level-major start from x = 0: the tiled copy of b is not formed (the
    // final residual reads the caller's b) and x is not zeroed: the first
    // update writes x = alpha p, and x is zeroed only if no update runs.
    bool b_level = false, x_unset = false;
    if (opts->x0_nonzero) {
        HIP_TRY(h, launch_cells_in(b_dev, layout, b, nullptr, plane, h->nz, 8, s));
        HIP_TRY(h, launch_cells_in(x_dev, layout, x, nullptr, plane, h->nz, 8, s));
        HIP_TRY(h, launch_residual(L0, x, b, 0, h->r, nullptr, h->partials, &G, s));
        if ((st = finalize(h, G, 1, ST_RR, 0, s)) != TPMG_OK) return st;
        HIP_TRY(h, launch_dot(n, b, b, nullptr, h->partials, &G, s));
        if ((st = finalize(h, G, 1, ST_BB, 0, s)) != TPMG_OK) return st;
    } else {
        // r = b: one reduction gives both (b, b) and (r, r)
        if (layout == TPMG_LAYOUT_LEVEL_MAJOR) {
            // one pass: r, fl32(r) in storage order, (b, b)
            HIP_TRY(h, launch_solve_start(b_dev, nullptr, h->r, h->mixed ? h->r32 : nullptr, nullptr, plane, h->nz,
                                          h->partials, &G, s));
            r32_ready = h->mixed;
            b_level = x_unset = true;
        } else {
            HIP_TRY(h, launch_cells_in(b_dev, layout, b, h->r, plane, h->nz, 8, s));
            HIP_TRY(h, launch_fill(x, 0.0, n, s));
            HIP_TRY(h, launch_dot(n, b, b, nullptr, h->partials, &G, s));
        }
        if ((st = finalize(h, G, 1, ST_BB, 0, s)) != TPMG_OK) return st;
        if ((st = finalize(h, G, 1, ST_RR, 0, s)) != TPMG_OK) return st;
    }
    if ((st = read_scalars(h, s)) != TPMG_OK) return st;
    const double bnorm = std::sqrt(h->sc_host->bb);
    double rnorm = std::sqrt(h->sc_host->rr);
    double rel = bnorm > 0 ? rnorm / bnorm : 0.0;
    if (opts->history) opts->history[0] = rel;
    int it = 0;
    bool converged = false;
    tpmg_status result = TPMG_NOT_CONVERGED;
    if (!std::isfinite(bnorm) || !std::isfinite(rnorm)) {
        result = TPMG_ERR_BREAKDOWN;
        fail(h, result, "non-finite right-hand side or initial residual");
    } else if (bnorm == 0.0 || rnorm <= opts->rtol * bnorm) {
        if (bnorm == 0.0 && !x_unset) HIP_TRY(h, launch_fill(x, 0.0, n, s));
        converged = true;
        result = TPMG_OK;
    } else {
        if (h->mixed && !r32_ready) HIP_TRY(h, launch_cast(h->r, h->r32, n, s));
        next_omega();
        if ((st = precondition(h, s)) != TPMG_OK) return st;
        HIP_TRY(h, launch_dot(n, h->r, h->z, h->mixed ? h->z32 : nullptr, h->partials, &G, s));
        if ((st = finalize(h, G, 1, ST_RZ_FIRST, flex, s)) != TPMG_OK) return st;
        double *pold = h->p1, *pnew = h->p0;
        for (it = 1; it <= opts->maxit; ++it) {
            {
                Timed t(h, TPMG_K_PCG_APPLY, s);
                HIP_TRY(h, launch_pcg_apply(L0, h->z, h->mixed ? h->z32 : nullptr, pold, pnew, h->q, h->sc,
                                            it == 1, h->partials, &G, s));
            }
            if ((st = finalize(h, G, 1, ST_PQ, flex, s)) != TPMG_OK) return st;  // (p, q), alpha
            {
                Timed t(h, TPMG_K_PCG_UPDATE, s);
                HIP_TRY(h, launch_pcg_update(n, x, pnew, h->r, h->q, h->mixed ? h->r32 : nullptr, h->sc,
                                             h->partials, x_unset ? 1 : 0, &G, s));
                x_unset = false;
            }
            if ((st = finalize(h, G, 1, ST_RR, flex, s)) != TPMG_OK) return st;
            if ((st = read_scalars(h, s)) != TPMG_OK) return st;
            if (h->sc_host->breakdown) {
                result = TPMG_ERR_BREAKDOWN;
                fail(h, result, "CG breakdown: (p, Hp) not positive or non-finite scalars");
                break;
            }
            rnorm = std::sqrt(h->sc_host->rr);
            rel = rnorm / bnorm;
            if (opts->history) opts->history[it] = rel;
            if (!std::isfinite(rnorm)) {
                result = TPMG_ERR_BREAKDOWN;
                fail(h, result, "non-finite residual");
                break;
            }
            if (rnorm <= opts->rtol * bnorm) {
                converged = true;
                result = TPMG_OK;
                break;
            }
            if (it == opts->maxit) break;
            next_omega();
            if ((st = precondition(h, s)) != TPMG_OK) return st;
            // (r, z) and, flexible, (q, z) with q = H p of this iteration
            HIP_TRY(h, launch_dot(n, h->r, h->z, h->mixed ? h->z32 : nullptr, h->partials, &G, s,
                                  flex ? h->q : nullptr));
            if ((st = finalize(h, G, flex ? 2 : 1, ST_RZ, flex, s)) != TPMG_OK) return st;
            std::swap(pold, pnew);
        }
        if (it > opts->maxit) it = opts->maxit;
    }
    if (x_unset) HIP_TRY(h, launch_fill(x, 0.0, n, s));  // no update ran
    bool x_out = false;  // x already copied to x_dev
    if (info) {
        // true residual norm; a level-major x_dev is written by the same pass
        double *xo = layout == TPMG_LAYOUT_LEVEL_MAJOR ? x_dev : nullptr;
        HIP_TRY(h, launch_residual(L0, x, b_level ? b_dev : b, b_level ? 1 : 0, nullptr, xo, h->partials, &G, s));
        x_out = xo != nullptr;
        if ((st = finalize(h, G, 1, ST_TT, 0, s)) != TPMG_OK) return st;
        if ((st = read_scalars(h, s)) != TPMG_OK) return st;
        info->iterations = it;
        info->converged = converged ? 1 : 0;
        info->rel_residual = rel;
        info->true_rel_residual = bnorm > 0 ? std::sqrt(h->sc_host->tt) / bnorm : 0.0;
    }
    if (!x_out) HIP_TRY(h, launch_cells_out(x, x_dev, layout, plane, h->nz, 8, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    return result;
}

tpmg_status tpmg_face_gradient(const tpmg_hierarchy *h, const double *lambda_dev, const double *x_dev,
                               double *grad_dev, int32_t layout, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if ((st = check_layout(h, layout)) != TPMG_OK || (st = check_ptrs(h, {lambda_dev, x_dev, grad_dev})) != TPMG_OK)
        return st;
    hipStream_t s = as_stream(stream);
    const int plane = h->l64[0].plane;
    const Level<double> L0 = level_view<double>(h, 0);
    if (layout == TPMG_LAYOUT_LEVEL_MAJOR) {
        HIP_TRY(hm, launch_face_gradient(L0, lambda_dev, x_dev, grad_dev, s));
        return TPMG_OK;
    }
    // column-major: lambda and x staged level-major in r and z (free outside
    // tpmg_solve), the gradient written level-major to the staging block and
    // transposed into grad.
    HIP_TRY(hm, launch_cells_to_level(lambda_dev, h->r, plane, h->nz, 8, s));
    HIP_TRY(hm, launch_cells_to_level(x_dev, h->z, plane, h->nz, 8, s));
    HIP_TRY(hm, launch_face_gradient(L0, h->r, h->z, h->stage0, s));
    HIP_TRY(hm, launch_faces_to_column(h->stage0, grad_dev, plane, h->nz, s));
    return TPMG_OK;
}

tpmg_status tpmg_smooth(const tpmg_hierarchy *h, int32_t level, int32_t fp32, const void *u_dev, const void *b_dev,
                        void *u_out_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (level < 0 || level >= h->L) return fail(hm, TPMG_ERR_INVALID_ARG, "level out of range");
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_ptrs(h, {b_dev, u_out_dev})) != TPMG_OK) return st;
    if (u_dev && (st = check_ptrs(h, {u_dev})) != TPMG_OK) return st;
    if (u_dev == u_out_dev || b_dev == u_out_dev) return fail(hm, TPMG_ERR_INVALID_ARG, "output must not alias inputs");
    hipStream_t s = as_stream(stream);
    return fp32 ? smooth_impl<float>(h, level, u_dev, b_dev, u_out_dev, s)
                : smooth_impl<double>(h, level, u_dev, b_dev, u_out_dev, s);
}

tpmg_status tpmg_residual_restrict(const tpmg_hierarchy *h, int32_t level, int32_t fp32, const void *u_dev,
                                   const void *b_dev, void *b_coarse_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (level < 0 || level + 1 >= h->L) return fail(hm, TPMG_ERR_INVALID_ARG, "level out of range");
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_ptrs(h, {u_dev, b_dev, b_coarse_dev})) != TPMG_OK)
        return st;
    hipStream_t s = as_stream(stream);
    return fp32 ? resid_restrict_impl<float>(h, level, u_dev, b_dev, b_coarse_dev, s)
                : resid_restrict_impl<double>(h, level, u_dev, b_dev, b_coarse_dev, s);
}

tpmg_status tpmg_prolong_smooth(const tpmg_hierarchy *h, int32_t level, int32_t fp32, const void *u_dev,
                                const void *e_coarse_dev, const void *b_dev, void *u_out_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (level < 0 || level + 1 >= h->L) return fail(hm, TPMG_ERR_INVALID_ARG, "level out of range");
    if ((st = check_fp32(h, fp32)) != TPMG_OK ||
        (st = check_ptrs(h, {u_dev, e_coarse_dev, b_dev, u_out_dev})) != TPMG_OK)
        return st;
    if (u_dev == u_out_dev || b_dev == u_out_dev) return fail(hm, TPMG_ERR_INVALID_ARG, "output must not alias inputs");
    hipStream_t s = as_stream(stream);
    return fp32 ? prolong_smooth_impl<float>(h, level, u_dev, e_coarse_dev, b_dev, u_out_dev, s)
                : prolong_smooth_impl<double>(h, level, u_dev, e_coarse_dev, b_dev, u_out_dev, s);
}

tpmg_status tpmg_coarse_solve(const tpmg_hierarchy *h, int32_t fp32, const void *b_dev, void *u_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_ptrs(h, {b_dev, u_dev})) != TPMG_OK) return st;
    if (b_dev == u_dev) return fail(hm, TPMG_ERR_INVALID_ARG, "b and u must not alias");
    hipStream_t s = as_stream(stream);
    return fp32 ? coarse_solve_impl<float>(h, b_dev, u_dev, s) : coarse_solve_impl<double>(h, b_dev, u_dev, s);
}

tpmg_status tpmg_level_coefficients(const tpmg_hierarchy *h, int32_t level, int32_t fp32, void *c_out_dev,
                                    void *stream)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (level < 0 || level >= h->L) return fail(hm, TPMG_ERR_INVALID_ARG, "level out of range");
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_ptrs(h, {c_out_dev})) != TPMG_OK) return st;
    const LevelBufs &B = fp32 ? h->l32[level] : h->l64[level];
    const int elem = fp32 ? 4 : 8;
    const size_t bytes = (size_t)B.plane * h->nz * elem;
    for (int f = 0; f < 3; ++f)
        HIP_TRY(hm, launch_cells_out((const char *)B.c + f * bytes, (char *)c_out_dev + f * bytes,
                                     TPMG_LAYOUT_LEVEL_MAJOR, B.plane, h->nz, elem, as_stream(stream)));
    return TPMG_OK;
}

tpmg_status tpmg_profile_enable(tpmg_hierarchy *h, int32_t enable)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    if (enable < 0 || enable > 2) return fail(h, TPMG_ERR_INVALID_ARG, "enable must be 0, 1 or 2");
    for (int c = 0; c < kPools; ++c) {
        EventPool &P = h->pools[c];
        if (enable && P.start.empty()) {
            P.start.resize(512);
            P.stop.resize(512);
            for (int i = 0; i < 512; ++i) {
                if (hipEventCreate(&P.start[i]) != hipSuccess || hipEventCreate(&P.stop[i]) != hipSuccess)
                    return fail(h, TPMG_ERR_DEVICE, "hipEventCreate failed");
            }
        }
        P.used = 0;
        P.acc_ms = 0.0;
        P.launches = 0;
    }
    h->prof = enable != 0;
    h->prof_levels = enable == 2;
    return TPMG_OK;
}

tpmg_status tpmg_profile_read(tpmg_hierarchy *h, int32_t kernel_class, double *total_ms, int64_t *launches)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    if (kernel_class < 0 || kernel_class >= TPMG_K_COUNT || !total_ms || !launches)
        return fail(h, TPMG_ERR_INVALID_ARG, "bad profile query");
    return read_pool(h, kernel_class, total_ms, launches);
}

tpmg_status tpmg_profile_read_level(tpmg_hierarchy *h, int32_t level, double *total_ms, int64_t *launches)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    if (level < 0 || level >= h->L || !total_ms || !launches)
        return fail(h, TPMG_ERR_INVALID_ARG, "bad profile query");
    return read_pool(h, kLevelPool + level, total_ms, launches);
}

tpmg_status tpmg_bandwidth_probe(void *dst_dev, const void *src_dev, size_t bytes, void *stream)
{
    if (!dst_dev || !src_dev || bytes % 16 || !aligned16(dst_dev) || !aligned16(src_dev))
        return fail(nullptr, TPMG_ERR_INVALID_ARG, "probe needs 16-byte aligned buffers and a multiple of 16 bytes");
    hipError_t e = launch_probe_copy(dst_dev, src_dev, bytes, as_stream(stream));
    if (e != hipSuccess) return hip_fail(nullptr, e, "probe copy");
    return TPMG_OK;
}

// ---- velocity-pressure system (Sec. 4.2, Eq. PressureVelocitySystem; Sec. 5) ----

namespace {

struct MixedWs {
    double *V = nullptr, *Z = nullptr, *partials = nullptr, *stage = nullptr, *out = nullptr;
    size_t M = 0;
};

// Carve the GMRES workspace: V (restart + 1 vectors), Z (restart), partial
// sums, reduction stage and results.  With base == nullptr only the size.
size_t plan_mixed(const tpmg_hierarchy *h, int restart, char *base, MixedWs *W)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> double * {
        off = (off + kAlign - 1) / kAlign * kAlign;
        double *p = base ? reinterpret_cast<double *>(base + off) : nullptr;
        off += bytes;
        return p;
    };
    const size_t M = 4 * h->ncell;
    W->M = M;
    W->V = take((size_t)(restart + 1) * M * sizeof(double));
    W->Z = take((size_t)restart * M * sizeof(double));
    W->partials = take((size_t)(kMultiMax + 2) * kMaxPartials * sizeof(double));
    W->stage = take((size_t)(kMultiMax + 2) * kReduceSegs * sizeof(double));
    W->out = take((size_t)(kMultiMax + 2) * sizeof(double));
    return (off + kAlign - 1) / kAlign * kAlign;
}

// z = P^{-1} (a r): t = a (r_p - D W r_u), z_p = V t (hierarchy precision),
// z_u = W (a r_u + D^T z_p).
tpmg_status mixed_precondition(tpmg_hierarchy *h, const double *r, double a, double *z, bool fp32, hipStream_t s)
{
    const Level<double> L0 = level_view<double>(h, 0);
    HIP_TRY(h, launch_mixed_pre1(L0, r, a, h->r, fp32 ? h->r32 : nullptr, s));
    tpmg_status st = fp32 ? vcycle<float>(h, h->r32, h->z32, s) : vcycle<double>(h, h->r, h->z, s);
    if (st != TPMG_OK) return st;
    HIP_TRY(h, launch_mixed_pre2(L0, r, a, fp32 ? nullptr : h->z, fp32 ? h->z32 : nullptr, z, s));
    return TPMG_OK;
}

// res[i] = (w, v_i), i < nv, in groups of kMultiMax; synchronises.
tpmg_status mixed_dots(tpmg_hierarchy *h, const MixedWs &W, const double *w, const double *const *v, int nv,
                       double *res, hipStream_t s)
{
    for (int i0 = 0; i0 < nv; i0 += kMultiMax) {
        const int g = std::min(kMultiMax, nv - i0);
        HIP_TRY(h, launch_multidot(W.M, w, v + i0, g, W.partials, W.stage, W.out, s));
        HIP_TRY(h, hipMemcpyAsync(h->dots_host, W.out, g * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        for (int i = 0; i < g; ++i) res[i0 + i] = h->dots_host[i];
    }
    return TPMG_OK;
}

// y += sum a_i v_i in groups; with norm2 != nullptr also returns (y, y).
tpmg_status mixed_axpys(tpmg_hierarchy *h, const MixedWs &W, double *y, const double *const *v, const double *a,
                        int nv, double *norm2, hipStream_t s)
{
    int G = 0;
    for (int i0 = 0; i0 < nv; i0 += kMultiMax) {
        const int g = std::min(kMultiMax, nv - i0);
        const bool last = i0 + g >= nv;
        HIP_TRY(h, launch_multiaxpy(W.M, y, v + i0, a + i0, g, (last && norm2) ? W.partials : nullptr, &G, s));
    }
    if (norm2) {
        HIP_TRY(h, launch_sum_partials(W.partials, G, 1, W.stage, W.out, s));
        HIP_TRY(h, hipMemcpyAsync(h->dots_host, W.out, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        *norm2 = h->dots_host[0];
    }
    return TPMG_OK;
}

tpmg_status check_mixed_level(tpmg_hierarchy *h)
{
    if (h->l64[0].n < 2) return fail(h, TPMG_ERR_SHAPE, "the velocity-pressure system needs n >= 2");
    return TPMG_OK;
}

}  // namespace

tpmg_status tpmg_mixed_workspace_bytes(const tpmg_hierarchy *h, int32_t restart, size_t *bytes)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    if (!bytes) return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG, "bytes is NULL");
    if (restart < 1 || restart > TPMG_MAX_RESTART)
        return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG, "restart out of range");
    MixedWs W;
    *bytes = plan_mixed(h, restart, nullptr, &W);
    return TPMG_OK;
}

tpmg_status tpmg_mixed_apply(const tpmg_hierarchy *hc, const double *x_dev, double *y_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(hc)) != TPMG_OK) return st;
    tpmg_hierarchy *h = const_cast<tpmg_hierarchy *>(hc);
    if ((st = check_ptrs(h, {x_dev, y_dev})) != TPMG_OK || (st = check_mixed_level(h)) != TPMG_OK) return st;
    if ((const void *)x_dev == (const void *)y_dev) return fail(h, TPMG_ERR_INVALID_ARG, "x and y must not alias");
    HIP_TRY(h, launch_mixed_apply(level_view<double>(h, 0), x_dev, y_dev, as_stream(stream)));
    return TPMG_OK;
}

tpmg_status tpmg_mixed_precondition(const tpmg_hierarchy *hc, int32_t fp32, const double *r_dev, double *z_dev,
                                    void *stream)
{
    tpmg_status st;
    if ((st = check_handle(hc)) != TPMG_OK) return st;
    tpmg_hierarchy *h = const_cast<tpmg_hierarchy *>(hc);
    if ((st = check_fp32(h, fp32)) != TPMG_OK || (st = check_ptrs(h, {r_dev, z_dev})) != TPMG_OK ||
        (st = check_mixed_level(h)) != TPMG_OK)
        return st;
    if ((const void *)r_dev == (const void *)z_dev) return fail(h, TPMG_ERR_INVALID_ARG, "r and z must not alias");
    return mixed_precondition(h, r_dev, 1.0, z_dev, fp32 == 1, as_stream(stream));
}

tpmg_status tpmg_mixed_solve(const tpmg_hierarchy *hc, const double *b_dev, double *x_dev, void *workspace_dev,
                             size_t workspace_bytes, const tpmg_mixed_opts *opts, tpmg_solve_info *info, void *stream)
{
    tpmg_status st;
    if ((st = check_handle(hc)) != TPMG_OK) return st;
    tpmg_hierarchy *h = const_cast<tpmg_hierarchy *>(hc);
    if ((st = check_ptrs(h, {b_dev, x_dev})) != TPMG_OK || (st = check_mixed_level(h)) != TPMG_OK) return st;
    if (!opts) return fail(h, TPMG_ERR_INVALID_ARG, "opts is NULL");
    if (!(opts->rtol >= 0.0) || opts->maxit < 0 || opts->restart < 1 || opts->restart > TPMG_MAX_RESTART)
        return fail(h, TPMG_ERR_INVALID_ARG, "bad mixed-solve options");
    if ((const void *)b_dev == (const void *)x_dev) return fail(h, TPMG_ERR_INVALID_ARG, "b and x must not alias");
    const int R = opts->restart;
    MixedWs W;
    const size_t need = plan_mixed(h, R, nullptr, &W);
    if (!workspace_dev || workspace_bytes < need || ((uintptr_t)workspace_dev % kAlign) != 0)
        return fail(h, TPMG_ERR_WORKSPACE, "mixed workspace missing, misaligned or smaller than tpmg_mixed_workspace_bytes");
    plan_mixed(h, R, static_cast<char *>(workspace_dev), &W);
    hipStream_t s = as_stream(stream);
    const size_t M = W.M;
    const Level<double> L0 = level_view<double>(h, 0);
    const bool fp32 = h->mixed;
    double *x = x_dev;
    const double *b = b_dev;

    {
        // the U slots of the top cells hold no face: b must be 0 there
        const size_t plane = (size_t)h->l64[0].plane;
        const double *top = b + 3 * h->ncell - plane;
        double tt = 0.0;
        HIP_TRY(h, launch_multidot(plane, top, &top, 1, W.partials, W.stage, W.out, s));
        HIP_TRY(h, hipMemcpyAsync(h->dots_host, W.out, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        tt = h->dots_host[0];
        if (tt != 0.0)
            return fail(h, TPMG_ERR_INVALID_ARG, "b is not 0 in the U slots of the top cells (no face there)");
    }
    HIP_TRY(h, launch_fill(x, 0.0, M, s));
    double bb = 0.0;
    if ((st = mixed_dots(h, W, b, &b, 1, &bb, s)) != TPMG_OK) return st;
    const double bnorm = std::sqrt(bb);
    if (opts->history) opts->history[0] = bnorm > 0.0 ? 1.0 : 0.0;
    std::vector<double> H((size_t)(R + 1) * R, 0.0), cs(R), sn(R), g(R + 1), y(R), hcol(R + 1), c(R + 2);
    // Krylov basis stored unnormalised: the j-th basis vector is sc[j] * vptr[j]
    // (the scales are applied in the dots, the updates and the
    // preconditioner, which saves a scaling pass over every new vector).
    std::vector<const double *> vptr(R + 1), zptr(R);
    std::vector<double> coef(R + 1), sc(R + 1);
    for (int i = 0; i <= R; ++i) vptr[i] = W.V + (size_t)i * M;
    for (int i = 0; i < R; ++i) zptr[i] = W.Z + (size_t)i * M;
    int it = 0;
    bool converged = false;
    double est = bnorm > 0.0 ? 1.0 : 0.0;
    tpmg_status result = TPMG_NOT_CONVERGED;
    if (!std::isfinite(bnorm)) {
        result = fail(h, TPMG_ERR_BREAKDOWN, "non-finite right-hand side");
    } else if (bnorm == 0.0) {
        converged = true;
        est = 0.0;
    }
    double beta = bnorm;
    vptr[0] = b;  // first cycle: the residual is b itself
    while (!converged && result == TPMG_NOT_CONVERGED && it < opts->maxit) {
        if (beta <= opts->rtol * bnorm) {
            converged = true;
            est = beta / bnorm;
            break;
        }
        sc[0] = 1.0 / beta;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jj = 0;
        bool conv = false;
        // Orthogonalisation: classical Gram-Schmidt, twice, with the second
        // pass delayed.  The update of step j leaves the new vector u_{j+1}
        // orthogonalised once and yields, in the same pass, its projections
        // a_i onto the basis; a_i and rho_{j+1}^2 = |u|^2 - |a|^2 complete
        // Hessenberg column j at once, and the correction
        // q_{j+1} = (u_{j+1} - sum a_i q_i) / rho_{j+1} is applied in step
        // j + 1's update pass (one pass over the basis per step).  Step j + 1
        // preconditions u_{j+1} / rho_{j+1}: flexible GMRES only needs
        // A z_j in the span of the basis.  When the projections are not small
        // (|a|^2 > |u|^2 / 100) or the step has more than kMultiMax basis
        // vectors, the second pass runs at once instead.
        bool pend = false;  // slot j holds u_j, not yet corrected
        double rho = 0.0;   // norm of the corrected u_j when pend
        // aj: projections of u_{j+1} (then u_j) onto q_0 .. q_j; hv: of w
        std::vector<double> aj(R + 1, 0.0), hv(R + 1, 0.0), ca(R + 1), cw(R + 1), sd(R + 1);
        for (int j = 0; j < R && it < opts->maxit; ++j) {
            double *zj = W.Z + (size_t)j * M;
            double *wj = W.V + (size_t)(j + 1) * M;  // becomes basis vector j + 1
            double *uj = W.V + (size_t)j * M;        // (j >= 1) u_j, corrected in this step when pend
            if (pend && j > kMultiMax) {
                // too many basis vectors for the fused pass: correct u_j now
                for (int i = 0; i < j; ++i) coef[i] = -aj[i] * sc[i];
                if ((st = mixed_axpys(h, W, uj, vptr.data(), coef.data(), j, nullptr, s)) != TPMG_OK) return st;
                sc[j] = 1.0 / rho;
                pend = false;
            }
            if ((st = mixed_precondition(h, vptr[j], sc[j], zj, fp32, s)) != TPMG_OK) return st;
            HIP_TRY(h, launch_mixed_apply(L0, zj, wj, s));
            vptr[j + 1] = wj;  // (w, w) rides along with the first-pass dots
            if ((st = mixed_dots(h, W, wj, vptr.data(), j + 2, c.data(), s)) != TPMG_OK) return st;
            const double ww = c[j + 1];
            // projections of w onto q_0 .. q_j
            for (int i = 0; i < j; ++i) hv[i] = c[i] * sc[i];
            if (pend) {
                double t = c[j];  // (u_j, w)
                for (int i = 0; i < j; ++i) t -= aj[i] * hv[i];
                hv[j] = t / rho;
            } else {
                hv[j] = c[j] * sc[j];
            }
            double hn2 = 0.0;
            bool done = false;  // u_{j+1} projections in aj[0..j], |u_{j+1}|^2 in hn2
            if (pend) {
                for (int i = 0; i < j; ++i) {
                    ca[i] = aj[i] * sc[i] / rho;
                    cw[i] = hv[i] * sc[i];
                    sd[i] = sc[i];
                }
                HIP_TRY(h, launch_corr_axpy_dot(M, uj, wj, vptr.data(), ca.data(), cw.data(), sd.data(), j, 1.0 / rho,
                                                hv[j], W.partials, W.stage, W.out, s));
                HIP_TRY(h, hipMemcpyAsync(h->dots_host, W.out, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_TRY(h, hipStreamSynchronize(s));
                for (int i = 0; i <= j; ++i) aj[i] = h->dots_host[i];
                hn2 = h->dots_host[j + 1];
                sc[j] = 1.0;  // slot j now holds q_j
                pend = false;
                done = true;
            } else if (j + 1 <= kMultiMax) {
                for (int i = 0; i <= j; ++i) coef[i] = -hv[i] * sc[i];
                HIP_TRY(h, launch_multiaxpy_dot(M, wj, vptr.data(), coef.data(), j + 1, W.partials, W.stage, W.out,
                                                s));
                HIP_TRY(h, hipMemcpyAsync(h->dots_host, W.out, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_TRY(h, hipStreamSynchronize(s));
                for (int i = 0; i <= j; ++i) aj[i] = h->dots_host[i] * sc[i];
                hn2 = h->dots_host[j + 1];
                done = true;
            } else {
                for (int i = 0; i <= j; ++i) coef[i] = -hv[i] * sc[i];
                if ((st = mixed_axpys(h, W, wj, vptr.data(), coef.data(), j + 1, &hn2, s)) != TPMG_OK) return st;
            }
            for (int i = 0; i <= j; ++i) hcol[i] = hv[i];
            double aa = 0.0;
            if (done)
                for (int i = 0; i <= j; ++i) aa += aj[i] * aj[i];
            if (done && aa <= 0.01 * hn2) {
                // delay the correction of u_{j+1} to the next step
                for (int i = 0; i <= j; ++i) hcol[i] += aj[i];
                hn2 = hn2 - aa;
                pend = hn2 > 0.0;
            } else if (!(hn2 > 0.5 * ww) || done) {
                // second pass now: large projections after the fused pass,
                // or (more than kMultiMax basis vectors) the selective
                // criterion, a second pass only when the first one cancels
                // more than a factor 1/sqrt(2) of the norm of w
                if (!done && (st = mixed_dots(h, W, wj, vptr.data(), j + 1, aj.data(), s)) != TPMG_OK) return st;
                if (!done)
                    for (int i = 0; i <= j; ++i) aj[i] *= sc[i];
                for (int i = 0; i <= j; ++i) {
                    hcol[i] += aj[i];
                    coef[i] = -aj[i] * sc[i];
                }
                if ((st = mixed_axpys(h, W, wj, vptr.data(), coef.data(), j + 1, &hn2, s)) != TPMG_OK) return st;
            }
            const double hn = std::sqrt(hn2);
            if (!std::isfinite(hn)) {
                result = fail(h, TPMG_ERR_BREAKDOWN, "non-finite Arnoldi vector");
                break;
            }
            sc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
            rho = hn;
            for (int i = 0; i <= j; ++i) H[(size_t)i * R + j] = hcol[i];
            H[(size_t)(j + 1) * R + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * R + j], cc = H[(size_t)(i + 1) * R + j];
                H[(size_t)i * R + j] = cs[i] * a + sn[i] * cc;
                H[(size_t)(i + 1) * R + j] = -sn[i] * a + cs[i] * cc;
            }
            const double a = H[(size_t)j * R + j], cc = H[(size_t)(j + 1) * R + j];
            const double den = std::hypot(a, cc);
            cs[j] = a / den;
            sn[j] = cc / den;
            H[(size_t)j * R + j] = den;
            H[(size_t)(j + 1) * R + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            est = std::fabs(g[j + 1]) / bnorm;
            if (opts->history) opts->history[it] = est;
            jj = j + 1;
            if (std::fabs(g[j + 1]) <= opts->rtol * bnorm || hn == 0.0) {
                conv = true;
                break;
            }
        }
        if (result != TPMG_NOT_CONVERGED) break;
        for (int i = jj - 1; i >= 0; --i) {
            double t = g[i];
            for (int l = i + 1; l < jj; ++l) t -= H[(size_t)i * R + l] * y[l];
            y[i] = t / H[(size_t)i * R + i];
        }
        if (jj > 0 && (st = mixed_axpys(h, W, x, zptr.data(), y.data(), jj, nullptr, s)) != TPMG_OK) return st;
        if (conv) {
            converged = true;
            break;
        }
        // restart from the true residual, computed into basis slot 0
        double *r0 = W.V;
        HIP_TRY(h, launch_mixed_apply(L0, x, r0, s));
        HIP_TRY(h, launch_axpby(M, 1.0, b, -1.0, r0, r0, s));
        vptr[0] = r0;
        double rr = 0.0;
        if ((st = mixed_dots(h, W, r0, vptr.data(), 1, &rr, s)) != TPMG_OK) return st;
        beta = std::sqrt(rr);
    }
    if (converged) result = TPMG_OK;
    if (info) {
        double *r = W.V;  // the basis is no longer needed
        HIP_TRY(h, launch_mixed_apply(L0, x, r, s));
        HIP_TRY(h, launch_axpby(M, 1.0, b, -1.0, r, r, s));
        double tt = 0.0;
        const double *rp = r;
        if ((st = mixed_dots(h, W, r, &rp, 1, &tt, s)) != TPMG_OK) return st;
        info->iterations = it;
        info->converged = converged ? 1 : 0;
        info->rel_residual = est;
        info->true_rel_residual = bnorm > 0.0 ? std::sqrt(tt) / bnorm : 0.0;
    }
    HIP_TRY(h, hipStreamSynchronize(s));
    return result;
}

tpmg_status tpmg_destroy(tpmg_hierarchy *h)
{
    if (!h) return TPMG_OK;
    for (int c = 0; c < kPools; ++c) {
        for (hipEvent_t e : h->pools[c].start) (void)hipEventDestroy(e);
        for (hipEvent_t e : h->pools[c].stop) (void)hipEventDestroy(e);
    }
    pinned_give(h->sc_host);
    delete h;
    return TPMG_OK;
}

const char *tpmg_status_string(tpmg_status s)
{
    switch (s) {
    case TPMG_OK: return "ok";
    case TPMG_NOT_CONVERGED: return "not converged";
    case TPMG_ERR_INVALID_ARG: return "invalid argument";
    case TPMG_ERR_SHAPE: return "invalid shape";
    case TPMG_ERR_NOT_SPD: return "operator not SPD (non-positive coefficient or spacing)";
    case TPMG_ERR_WORKSPACE: return "workspace missing or too small";
    case TPMG_ERR_DEVICE: return "HIP device error";
    case TPMG_ERR_BREAKDOWN: return "CG breakdown";
    default: return "unknown status";
    }
}

const char *tpmg_last_error(const tpmg_hierarchy *h)
{
    if (h) return h->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"

// =============================================================================
// Next-to-lowest-order (DG1) pressure level on the finest grid: banded column
// factors, operator, sweeps, p-transfers, the NLO V-cycle and its CG.
// =============================================================================

struct tpmg_dg1 {
    tpmg_hierarchy *h = nullptr;
    Dg1Level G{};
    size_t nv = 0;                     // 6 n^2 nz unknowns
    void *fac = nullptr;   // band factors: FP32 for a mixed hierarchy, else FP64
    double *tab = nullptr;
    double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    double *A = nullptr, *B = nullptr;  // sweep vectors of the V-cycle and the component calls
    double *b0 = nullptr, *e0 = nullptr;  // lowest-order level-0 vectors (FP64 correction)
};

namespace {

constexpr int kDg1Nf = 11;  // band entries per factor row

// Carve a DG1 workspace; with g == nullptr only the size is computed.
size_t plan_dg1(const tpmg_hierarchy *h, tpmg_dg1 *g, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> double * {
        off = (off + kAlign - 1) / kAlign * kAlign;
        double *p = g ? (double *)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    const size_t plane = (size_t)h->l64[0].plane, nz = (size_t)h->nz;
    const size_t nv = plane * 6 * nz, ncell = plane * nz;
    // a mixed hierarchy keeps the band factors in FP32 (the NLO smoother of
    // the FP32 V-cycle path; arithmetic stays FP64), half the bytes
    void *fac = take(nv * kDg1Nf * (h->mixed ? 4 : 8));
    double *tab = take(5 * nz * 8);
    double *v[9];
    for (int i = 0; i < 9; ++i) v[i] = take(nv * 8);
    double *b0 = take(ncell * 8), *e0 = take(ncell * 8);
    if (g) {
        g->nv = nv;
        g->fac = fac;
        g->tab = tab;
        g->b = v[0];
        g->x = v[1];
        g->r = v[2];
        g->z = v[3];
        g->p0 = v[4];
        g->p1 = v[5];
        g->q = v[6];
        g->A = v[7];
        g->B = v[8];
        g->b0 = b0;
        g->e0 = e0;
    }
    return (off + kAlign - 1) / kAlign * kAlign;
}

tpmg_status check_dg1_shape(const tpmg_hierarchy *h)
{
    tpmg_hierarchy *hm = const_cast<tpmg_hierarchy *>(h);
    if (h->nz < 2) return fail(hm, TPMG_ERR_SHAPE, "the DG1 level needs nz >= 2");
    const size_t plane = (size_t)h->l64[0].plane, rows = 6 * (size_t)h->nz;
    if (plane * rows * 8 >= ((size_t)1 << 32))
        return fail(hm, TPMG_ERR_SHAPE, "DG1 vectors would reach 4 GiB (kernels use 32-bit byte offsets)");
    if ((plane & 63) != 0 && plane * rows * kDg1Nf * 8 >= ((size_t)1 << 32))
        return fail(hm, TPMG_ERR_SHAPE, "band factors of a plane that is not a multiple of 64 would reach 4 GiB");
    return TPMG_OK;
}

tpmg_status check_dg1(const tpmg_dg1 *g)
{
    if (!g || !g->h) return fail(nullptr, TPMG_ERR_INVALID_ARG, "DG1 handle is NULL");
    return TPMG_OK;
}

// caller's (6, nz, n, n) level-major DG1 array <-> the tiled storage
tpmg_status dg1_in(const tpmg_dg1 *g, const double *src, double *dst, double *dst2, hipStream_t s)
{
    HIP_TRY(g->h, launch_cells_in(src, TPMG_LAYOUT_LEVEL_MAJOR, dst, dst2, g->G.plane, 6 * g->G.nz, 8, s));
    return TPMG_OK;
}

tpmg_status dg1_out(const tpmg_dg1 *g, const double *src, double *dst, hipStream_t s)
{
    HIP_TRY(g->h, launch_cells_out(src, dst, TPMG_LAYOUT_LEVEL_MAJOR, g->G.plane, 6 * g->G.nz, 8, s));
    return TPMG_OK;
}

tpmg_status dg1_sweep(const tpmg_dg1 *g, int mode, const double *u, const double *b, double *out, hipStream_t s)
{
    Timed t(g->h, mode == DG1_SWEEP_GENERAL ? TPMG_K_DG1_SWEEP : -1, s);
    HIP_TRY(g->h, launch_dg1_sweep(g->G, g->fac, mode, u, b, out, g->h->d.omega, s));
    return TPMG_OK;
}

// out = V1 b (zero initial guess): nu_pre DG1 sweeps, p-restriction of the
// residual to the lowest-order level 0, one lowest-order V-cycle there (in the
// hierarchy's precision), the correction added by the embedding, nu_post DG1
// sweeps (Sec. 4.2.1: the first coarsening step is DG1 -> DG0).  b and out
// must not be A or B.
tpmg_status dg1_vcycle(const tpmg_dg1 *g, const double *b, double *out, hipStream_t s)
{
    tpmg_hierarchy *h = g->h;
    Timed t(h, TPMG_K_DG1_VCYCLE, s);
    double *cur = g->A, *other = g->B;
    tpmg_status st;
    if ((st = dg1_sweep(g, DG1_SWEEP_ZERO, nullptr, b, cur, s)) != TPMG_OK) return st;
    for (int i = 1; i < h->d.nu_pre; ++i) {
        if ((st = dg1_sweep(g, DG1_SWEEP_GENERAL, cur, b, other, s)) != TPMG_OK) return st;
        std::swap(cur, other);
    }
    if (h->mixed) {
        HIP_TRY(h, launch_dg1_resid_restrict(g->G, cur, b, h->r32, 1, s));
        if ((st = vcycle<float>(h, h->r32, h->z32, s)) != TPMG_OK) return st;
        HIP_TRY(h, launch_dg1_prolong(g->G, h->z32, 1, cur, s));
    } else {
        HIP_TRY(h, launch_dg1_resid_restrict(g->G, cur, b, g->b0, 0, s));
        if ((st = vcycle<double>(h, g->b0, g->e0, s)) != TPMG_OK) return st;
        HIP_TRY(h, launch_dg1_prolong(g->G, g->e0, 0, cur, s));
    }
    const double *src = cur;
    for (int i = 0; i < h->d.nu_post; ++i) {
        double *dst = (i == h->d.nu_post - 1) ? out : ((i % 2 == 0) ? other : cur);
        if ((st = dg1_sweep(g, DG1_SWEEP_GENERAL, src, b, dst, s)) != TPMG_OK) return st;
        src = dst;
    }
    return TPMG_OK;
}

}  // namespace

extern "C" {

tpmg_status tpmg_dg1_workspace_bytes(const tpmg_hierarchy *h, size_t *bytes)
{
    tpmg_status st;
    if ((st = check_handle(h)) != TPMG_OK) return st;
    if (!bytes) return fail(const_cast<tpmg_hierarchy *>(h), TPMG_ERR_INVALID_ARG, "bytes is NULL");
    if ((st = check_dg1_shape(h)) != TPMG_OK) return st;
    *bytes = plan_dg1(h, nullptr, nullptr);
    return TPMG_OK;
}

tpmg_status tpmg_dg1_setup(const tpmg_hierarchy *hc, void *workspace_dev, size_t workspace_bytes, void *stream,
                           tpmg_dg1 **out)
{
    tpmg_status st;
    if ((st = check_handle(hc)) != TPMG_OK) return st;
    tpmg_hierarchy *h = const_cast<tpmg_hierarchy *>(hc);
    if (!out) return fail(h, TPMG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if ((st = check_dg1_shape(h)) != TPMG_OK) return st;
    const size_t need = plan_dg1(h, nullptr, nullptr);
    if (!workspace_dev || workspace_bytes < need || ((uintptr_t)workspace_dev % kAlign) != 0)
        return fail(h, TPMG_ERR_WORKSPACE, "DG1 workspace missing, too small or not 256-byte aligned");
    hipStream_t s = as_stream(stream);
    tpmg_dg1 *g = new tpmg_dg1();
    g->h = h;
    plan_dg1(h, g, (char *)workspace_dev);
    const int nz = h->nz;
    g->G.n = h->l64[0].n;
    g->G.nz = nz;
    g->G.plane = h->l64[0].plane;
    g->G.c = (const double *)h->l64[0].c;
    g->G.tab = g->tab;
    g->G.fac32 = h->mixed ? 1 : 0;
    // per-k scalars of the finest level: s_k, a_h s_k, 4 a_h s_k, 4 a_z / s_k, a_z / t_{k+1/2}
    std::vector<double> sk(nz, 1.0), tk(nz, 1.0), tab(5 * (size_t)nz, 0.0);
    {
        double mean = 0.0;
        for (int k = 0; k < nz; ++k) mean += h->dz.empty() ? 1.0 : h->dz[k];
        mean /= nz;
        for (int k = 0; k < nz; ++k) sk[k] = (h->dz.empty() ? 1.0 : h->dz[k]) / mean;
        for (int k = 0; k + 1 < nz; ++k) tk[k] = 0.5 * (sk[k] + sk[k + 1]);
    }
    for (int k = 0; k < nz; ++k) {
        tab[k] = sk[k];
        tab[nz + k] = h->d.a_h * sk[k];
        tab[2 * nz + k] = 4.0 * h->d.a_h * sk[k];
        tab[3 * nz + k] = 4.0 * h->d.a_z / sk[k];
        tab[4 * nz + k] = (k + 1 < nz) ? h->d.a_z / tk[k] : 0.0;
    }
    hipError_t e;
    int bad = 0;
    if ((e = hipMemcpyAsync(g->tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_fill((double *)h->bad, 0.0, 1, s)) != hipSuccess ||
        (e = launch_dg1_factor(g->G, g->fac, h->bad, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&bad, h->bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        delete g;
        return hip_fail(h, e, "DG1 setup");
    }
    if (bad) {
        delete g;
        return fail(h, TPMG_ERR_NOT_SPD, std::to_string(bad) + " non-positive pivot(s) in the DG1 column factors");
    }
    *out = g;
    return TPMG_OK;
}

tpmg_status tpmg_dg1_apply(const tpmg_dg1 *g, const double *x_dev, double *y_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(g)) != TPMG_OK || (st = check_ptrs(g->h, {x_dev, y_dev})) != TPMG_OK) return st;
    hipStream_t s = as_stream(stream);
    if ((st = dg1_in(g, x_dev, g->A, nullptr, s)) != TPMG_OK) return st;
    HIP_TRY(g->h, launch_dg1_apply(g->G, g->A, g->B, s));
    return dg1_out(g, g->B, y_dev, s);
}

tpmg_status tpmg_dg1_line_solve(const tpmg_dg1 *g, const double *r_dev, double *x_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(g)) != TPMG_OK || (st = check_ptrs(g->h, {r_dev, x_dev})) != TPMG_OK) return st;
    hipStream_t s = as_stream(stream);
    if ((st = dg1_in(g, r_dev, g->A, nullptr, s)) != TPMG_OK) return st;
    if ((st = dg1_sweep(g, DG1_SWEEP_SOLVE, nullptr, g->A, g->B, s)) != TPMG_OK) return st;
    return dg1_out(g, g->B, x_dev, s);
}

tpmg_status tpmg_dg1_smooth(const tpmg_dg1 *g, const double *u_dev, const double *b_dev, double *u_out_dev,
                            void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(g)) != TPMG_OK || (st = check_ptrs(g->h, {b_dev, u_out_dev})) != TPMG_OK) return st;
    if (u_dev && (st = check_ptrs(g->h, {u_dev})) != TPMG_OK) return st;
    hipStream_t s = as_stream(stream);
    if (u_dev && (st = dg1_in(g, u_dev, g->A, nullptr, s)) != TPMG_OK) return st;
    if ((st = dg1_in(g, b_dev, g->b, nullptr, s)) != TPMG_OK) return st;
    if ((st = dg1_sweep(g, u_dev ? DG1_SWEEP_GENERAL : DG1_SWEEP_ZERO, u_dev ? g->A : nullptr, g->b, g->B, s)) !=
        TPMG_OK)
        return st;
    return dg1_out(g, g->B, u_out_dev, s);
}

tpmg_status tpmg_dg1_residual_restrict(const tpmg_dg1 *g, const double *u_dev, const double *b_dev, double *b0_dev,
                                       void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(g)) != TPMG_OK || (st = check_ptrs(g->h, {u_dev, b_dev, b0_dev})) != TPMG_OK) return st;
    hipStream_t s = as_stream(stream);
    if ((st = dg1_in(g, u_dev, g->A, nullptr, s)) != TPMG_OK || (st = dg1_in(g, b_dev, g->b, nullptr, s)) != TPMG_OK)
        return st;
    HIP_TRY(g->h, launch_dg1_resid_restrict(g->G, g->A, g->b, g->b0, 0, s));
    HIP_TRY(g->h, launch_cells_out(g->b0, b0_dev, TPMG_LAYOUT_LEVEL_MAJOR, g->G.plane, g->G.nz, 8, s));
    return TPMG_OK;
}

tpmg_status tpmg_dg1_prolong_add(const tpmg_dg1 *g, const double *e0_dev, double *u_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(g)) != TPMG_OK || (st = check_ptrs(g->h, {e0_dev, u_dev})) != TPMG_OK) return st;
    hipStream_t s = as_stream(stream);
    HIP_TRY(g->h, launch_cells_in(e0_dev, TPMG_LAYOUT_LEVEL_MAJOR, g->e0, nullptr, g->G.plane, g->G.nz, 8, s));
    if ((st = dg1_in(g, u_dev, g->A, nullptr, s)) != TPMG_OK) return st;
    HIP_TRY(g->h, launch_dg1_prolong(g->G, g->e0, 0, g->A, s));
    return dg1_out(g, g->A, u_dev, s);
}

tpmg_status tpmg_dg1_vcycle(const tpmg_dg1 *g, const double *b_dev, double *z_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(g)) != TPMG_OK || (st = check_ptrs(g->h, {b_dev, z_dev})) != TPMG_OK) return st;
    if ((const void *)b_dev == (const void *)z_dev) return fail(g->h, TPMG_ERR_INVALID_ARG, "b and z must not alias");
    hipStream_t s = as_stream(stream);
    if ((st = dg1_in(g, b_dev, g->b, nullptr, s)) != TPMG_OK) return st;
    if ((st = dg1_vcycle(g, g->b, g->z, s)) != TPMG_OK) return st;
    return dg1_out(g, g->z, z_dev, s);
}

tpmg_status tpmg_dg1_solve(const tpmg_dg1 *gc, const double *b_dev, double *x_dev, const tpmg_solve_opts *opts,
                           tpmg_solve_info *info, void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(gc)) != TPMG_OK) return st;
    tpmg_dg1 *g = const_cast<tpmg_dg1 *>(gc);
    tpmg_hierarchy *h = g->h;
    if ((st = check_ptrs(h, {b_dev, x_dev})) != TPMG_OK) return st;
    if (!opts) return fail(h, TPMG_ERR_INVALID_ARG, "opts is NULL");
    if (!(opts->rtol >= 0.0) || opts->maxit < 0 || (opts->flexible != 0 && opts->flexible != 1) ||
        opts->x0_nonzero != 0 || opts->omega_alt != 0.0)
        return fail(h, TPMG_ERR_INVALID_ARG, "bad DG1 solve options (x0_nonzero and omega_alt must be 0)");
    if ((const void *)b_dev == (const void *)x_dev) return fail(h, TPMG_ERR_INVALID_ARG, "b and x must not alias");
    hipStream_t s = as_stream(stream);
    const size_t n = g->nv;
    const int flex = opts->flexible;
    double *b = g->b, *x = g->x;
    int G = 0;
    // b in storage order, r = b, x = 0 (written by the first update)
    if ((st = dg1_in(g, b_dev, b, g->r, s)) != TPMG_OK) return st;
    HIP_TRY(h, launch_fill((double *)h->sc, 0.0, sizeof(Scalars) / sizeof(double), s));
    HIP_TRY(h, launch_dot(n, b, b, nullptr, h->partials, &G, s));
    if ((st = finalize(h, G, 1, ST_BB, 0, s)) != TPMG_OK) return st;
    if ((st = finalize(h, G, 1, ST_RR, 0, s)) != TPMG_OK) return st;
    if ((st = read_scalars(h, s)) != TPMG_OK) return st;
    const double bnorm = std::sqrt(h->sc_host->bb);
    double rnorm = std::sqrt(h->sc_host->rr);
    double rel = bnorm > 0 ? rnorm / bnorm : 0.0;
    if (opts->history) opts->history[0] = rel;
    int it = 0;
    bool converged = false, x_unset = true;
    tpmg_status result = TPMG_NOT_CONVERGED;
    if (!std::isfinite(bnorm)) {
        result = TPMG_ERR_BREAKDOWN;
        fail(h, result, "non-finite right-hand side");
    } else if (bnorm == 0.0) {
        converged = true;
        result = TPMG_OK;
    } else {
        if ((st = dg1_vcycle(g, g->r, g->z, s)) != TPMG_OK) return st;
        HIP_TRY(h, launch_dot(n, g->r, g->z, nullptr, h->partials, &G, s));
        if ((st = finalize(h, G, 1, ST_RZ_FIRST, flex, s)) != TPMG_OK) return st;
        double *pold = g->p1, *pnew = g->p0;
        for (it = 1; it <= opts->maxit; ++it) {
            {
                Timed t(h, TPMG_K_DG1_PCG_APPLY, s);
                HIP_TRY(h, launch_dg1_pcg_apply(g->G, g->z, pold, pnew, g->q, h->sc, it == 1, h->partials, &G, s));
            }
            if ((st = finalize(h, G, 1, ST_PQ, flex, s)) != TPMG_OK) return st;
            HIP_TRY(h, launch_pcg_update(n, x, pnew, g->r, g->q, nullptr, h->sc, h->partials, x_unset ? 1 : 0, &G, s));
            x_unset = false;
            if ((st = finalize(h, G, 1, ST_RR, flex, s)) != TPMG_OK) return st;
            if ((st = read_scalars(h, s)) != TPMG_OK) return st;
            if (h->sc_host->breakdown) {
                result = TPMG_ERR_BREAKDOWN;
                fail(h, result, "CG breakdown: (p, Hp) not positive or non-finite scalars");
                break;
            }
            rnorm = std::sqrt(h->sc_host->rr);
            rel = rnorm / bnorm;
            if (opts->history) opts->history[it] = rel;
            if (!std::isfinite(rnorm)) {
                result = TPMG_ERR_BREAKDOWN;
                fail(h, result, "non-finite residual");
                break;
            }
            if (rnorm <= opts->rtol * bnorm) {
                converged = true;
                result = TPMG_OK;
                break;
            }
            if (it == opts->maxit) break;
            if ((st = dg1_vcycle(g, g->r, g->z, s)) != TPMG_OK) return st;
            HIP_TRY(h, launch_dot(n, g->r, g->z, nullptr, h->partials, &G, s, flex ? g->q : nullptr));
            if ((st = finalize(h, G, flex ? 2 : 1, ST_RZ, flex, s)) != TPMG_OK) return st;
            std::swap(pold, pnew);
        }
        if (it > opts->maxit) it = opts->maxit;
    }
    if (x_unset) HIP_TRY(h, launch_fill(x, 0.0, n, s));
    if (info) {
        HIP_TRY(h, launch_dg1_residual(g->G, x, b, nullptr, h->partials, &G, s));
        if ((st = finalize(h, G, 1, ST_TT, 0, s)) != TPMG_OK) return st;
        if ((st = read_scalars(h, s)) != TPMG_OK) return st;
        info->iterations = it;
        info->converged = converged ? 1 : 0;
        info->rel_residual = rel;
        info->true_rel_residual = bnorm > 0 ? std::sqrt(h->sc_host->tt) / bnorm : 0.0;
    }
    if ((st = dg1_out(g, x, x_dev, s)) != TPMG_OK) return st;
    HIP_TRY(h, hipStreamSynchronize(s));
    return result;
}

tpmg_status tpmg_dg1_factors(const tpmg_dg1 *g, double *f_dev, void *stream)
{
    tpmg_status st;
    if ((st = check_dg1(g)) != TPMG_OK || (st = check_ptrs(g->h, {f_dev})) != TPMG_OK) return st;
    HIP_TRY(g->h, launch_dg1_factors_out(g->G, g->fac, f_dev, as_stream(stream)));
    return TPMG_OK;
}

tpmg_status tpmg_dg1_destroy(tpmg_dg1 *g)
{
    delete g;
    return TPMG_OK;
}

}  // extern "C"
