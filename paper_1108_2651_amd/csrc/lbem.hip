// lbem.hip -- host side of liblbem: handle, device memory, kernel dispatch and
// the C ABI declared in include/lbem.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <shared_mutex>
#include <vector>

#include "../../include/lbem.h"
#include "kernels.h"

using namespace lbem;

namespace {

enum Layout { LAYOUT_NATURAL = 0, LAYOUT_PULL_PENDING = 1, LAYOUT_AA_SWAPPED = 2 };

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Graph capture of the batched kernels (lbem_batch_create) holds this lock
// exclusively; the entry points that allocate or free device memory, or
// create and destroy HIP objects, hold it shared.  No allocation or free of
// this library then runs while a graph is captured and instantiated.
std::shared_mutex g_api_mu;
#define API_SHARED std::shared_lock<std::shared_mutex> api_lock_(g_api_mu)

int env_int(const char* name, int dflt)
{
    const char* v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

struct Sizes {
    size_t pop_one;   // bytes of one copy of the population state
    size_t copies;
    size_t medium;    // c_L^2
    size_t mu;        // mu_r (double) + grad ln mu (medium type) if mu_varies
    size_t scratch;   // 3*n doubles
    size_t total;
};

// the formats with FP32 moments + 16-bit deviations or ghost coordinates
bool is_dev(int prec) { return prec >= LBEM_F16DEV && prec <= LBEM_BF16GHOST; }

bool valid_cfg(const lbem_config* c)
{
    if (!c) return false;
    if (c->dim != 2 && c->dim != 3) return false;
    if (c->prec < LBEM_F64 || c->prec > LBEM_F16) return false;
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return false;
    if (c->dim == 2 && c->nz != 1) return false;
    if (c->nx > (1 << 30) || c->ny > (1 << 30) || c->nz > (1 << 30)) return false;
    const double n = (double)c->nx * (double)c->ny * (double)c->nz;
    if (n >= 2147483648.0) return false;
    if (!(c->tau > 0.0) || !std::isfinite(c->tau)) return false;
    if (!(c->w0_vac >= 0.0 && c->w0_vac < 1.0)) return false;
    if (c->streaming < LBEM_STREAM_AUTO || c->streaming > LBEM_STREAM_AA) return false;
    if (c->streaming == LBEM_STREAM_AA && is_dev(c->prec)) return false;
    return true;
}

// 3D FP32 runs two fused steps per launch from this many cells on (about
// 100^3), single AA steps below, where the state is Infinity-Cache resident
// and the pair's tiles cannot fill the chip.  Measured, us per step, fused
// pair (64 x 8 tiles) against single AA steps: 64^3 20.6 / 7.2, 80^3 23.6 /
// 15.1, 96^3 23.8 / 24.3, 112^3 29.7 / 37.5, 128^3 47.4 / 58.5, 144^3 76.1 /
// 82.5, 160^3 96.0 / 133.1.
constexpr double FUSE3D_MIN = 1.0e6;
// The column-tile z-march of the 16-bit formats (rows longer than the row
// tiles take) from this many cells on: the cache-residency threshold every 3D
// z-marching kernel shared before the row tiles and the 64 x 8 FP32 pair got
// their own, kept for these rare shapes (not re-measured).
constexpr double SMALL3D = 3.5e6;
// The 3D 16-bit formats take the whole-row tiles once the state one step
// touches (stored values read and written, c_L^2 read: 112 B per cell with
// ghost coordinates, 136 B with all deviations) exceeds the 256 MB Infinity
// Cache; per-cell tiles below.  Measured, us per step, per-cell against row
// tiles: FP16 ghost 128^3 (224 MiB) 48.4 / 67.1, 144^3 122.1 / 88.2; FP16-dev
// 128^3 (272 MiB) 76.3 / 74.5, 144^3 130.7 / 109.3.
constexpr double ROWTILE_BYTES = 256.0 * (1 << 20);
// plain FP16 storage on whole-row blocks: measured from 6e6 cells on
constexpr double XROW3D = 6.0e6;

int resolve_streaming(const lbem_config* c)
{
    // Pull by default: the fused multi-step kernels need the second copy.
    // 3D FP64 never fuses and small 3D FP32 boxes run single steps: there the
    // in-place AA pattern (half the memory) is as fast or faster.
    if (c->streaming != LBEM_STREAM_AUTO) return c->streaming;
    const double n = (double)c->nx * (double)c->ny * (double)c->nz;
    if (c->dim == 3 && (c->prec == LBEM_F64 || (c->prec == LBEM_F32 && n < FUSE3D_MIN))) return LBEM_STREAM_AA;
    return LBEM_STREAM_PULL;
}

Sizes sizes_of(const lbem_config* c)
{
    Sizes s{};
    const int D = c->dim, Q = 2 * D + 1, P = D * (D - 1) / 2;
    const size_t n = (size_t)(c->nx * c->ny * c->nz);
    const size_t tm = c->prec == LBEM_F64 ? 8 : 4;
    if (!is_dev(c->prec))
        s.pop_one = align256((size_t)Q * P * n * (c->prec == LBEM_F16 ? 2 : tm));
    else
        s.pop_one = align256((size_t)(P + D) * n * 4) +
                    align256((size_t)(c->prec >= LBEM_F16GHOST ? 2 * D * P - D : Q * P) * n * 2);
    s.copies = resolve_streaming(c) == LBEM_STREAM_AA ? 1 : 2;
    s.medium = align256(n * tm);
    s.mu = c->mu_varies ? align256(n * 8) + align256((size_t)D * n * tm) : 0;
    s.scratch = align256(3 * n * 8);
    s.total = s.pop_one * s.copies + s.medium + s.mu + s.scratch;
    return s;
}

}  // namespace

struct Impl;

struct lbem_s {
    lbem_config cfg;
    int D, Q, P, prec, streaming;
    int64_t n;
    hipStream_t stream;
    int device;
    bool own_mem;
    char* arena;
    size_t arena_bytes;
    // population state
    char* pop[2];
    int cur;
    int layout;
    // medium
    void* cl2;
    double* mu_r;
    void* dlnmu;
    bool mu_set;
    // scratch / reductions
    double* scratch;
    double* partials;   // nb_diag*4 + 4
    int nb_diag;
    // source (device tables, handle-owned)
    int* src_off;
    int2* src_ent;
    void* src_val;
    int64_t nsrc;
    // tiling of the step kernels
    Geo geo;
    int vec;
    // temporal blocking (fuse_ns steps per launch; 1 = off): 2D tiles 64 x fuse_ty,
    // 3D column tiles f3_tx x f3_ty marching over chunks of f3_lz planes
    int fuse_ns, fuse_ty, fuse_nt;
    int f3_tx, f3_ty, f3_lz;
    Geo fgeo;
    int* fsrc_off;
    int2* fsrc_ent;
    void* fsrc_val;
    int64_t nfsrc;
    // single steps with the streaming cache policy on the stored state
    // (lattices whose state a launch touches exceeds the last-level cache)
    int nts;
    // 3D deviation kernel marching along z (column tiles x z-chunks)
    int zmarch, zlz;
    Geo zgeo;
    int* zsrc_off;
    int2* zsrc_ent;
    void* zsrc_val;
    int64_t nzsrc;
    // 3D plain single steps on whole-row blocks (k_step_xrow)
    int xrow;
    XRowGeo xgeo;
    int* xsrc_off;
    int2* xsrc_ent;
    void* xsrc_val;
    int64_t nxsrc;
    // 3D deviation kernel on whole-row tiles (k_step_dev3r), marching along z
    int rowk;
    RowGeo rgeo;
    int rntb;            // threads per block of the row tiles
    int* rsrc_off;
    int2* rsrc_ent;
    float* rsrc_val;
    int64_t nrsrc;
    // the whole-row tiling of this handle inside a batch (3D deviation formats,
    // rows of up to 2 BROW_NT cells, BROW_NT-thread blocks) and its source table
    int brow;
    RowGeo bgeo;
    int* bsrc_off;
    int2* bsrc_ent;
    float* bsrc_val;
    int64_t nbsrc;
    // state
    // non-periodic faces and absorbing layer
    int bc_kind[3];
    void* keep;              // handle-owned, medium precision, or nullptr
    // frequency-dispersive permittivity (one Lorentz pole per cell)
    void* ade;               // [3][n] coefficients, handle-owned, or nullptr
    void* pol;               // [2P][n] auxiliary P and J per pair
    // anisotropy (plain formats): [D][n] ratios r_a, handle-owned; valid while ra_set
    void* ra;
    bool ra_set;
    int64_t t;
    bool have_medium, have_fields;
    Impl* impl;
    hipEvent_t sync_ev;      // set-up work on this handle's stream before a batch tick
    hipEvent_t tick_ev;      // end of the last batch tick that advanced this handle
    bool tick_pending;       // this handle's stream has not yet waited on tick_ev
};

// Work on the handle's own stream that touches its state follows the batch
// ticks that advanced it.  The wait is added here, at the handle's next use,
// not when the tick is enqueued: the stream may be shared with other
// handles' set-up, which need not wait for the tick.
static hipError_t follow_ticks(lbem_s* h)
{
    if (!h->tick_pending) return hipSuccess;
    h->tick_pending = false;
    return hipStreamWaitEvent(h->stream, h->tick_ev, 0);
}

// Set-up staging buffers: stream-ordered allocations, whose release does not
// wait for other streams' work (batch ticks in flight).  Buffers above 1 GiB
// (lattices of 4e7 cells and more, never served in batches) and any request
// the pool refuses use hipMalloc, whose hipFree synchronises the device: the
// pool keeps freed memory until the next synchronisation, which must not hold
// tens of GB beside a 2^30-cell lattice.
struct Staging {
    void* p = nullptr;
    bool pooled = false;
};
static bool stage_alloc(Staging& st, size_t bytes, hipStream_t s)
{
    if (bytes <= (size_t(1) << 30) && hipMallocAsync(&st.p, bytes, s) == hipSuccess) {
        st.pooled = true;
        return true;
    }
    (void)hipGetLastError();
    st.p = nullptr;
    st.pooled = false;
    return hipMalloc(&st.p, bytes) == hipSuccess;
}
static void stage_free(Staging& st, hipStream_t s)
{
    if (!st.p) return;
    if (st.pooled) (void)hipFreeAsync(st.p, s);
    else (void)hipFree(st.p);
    st.p = nullptr;
}

#define HIP_OK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return LBEM_EDEVICE; \
    } while (0)

// ---------------------------------------------------------------------------
// per (dimension, format) kernel dispatch
// ---------------------------------------------------------------------------
struct Impl {
    virtual ~Impl() {}
    virtual hipError_t step(lbem_s* h, double amp) = 0;
    // advance h->fuse_ns steps in one launch (only when fused_ok and pull-pending)
    virtual hipError_t step_fused(lbem_s* h, const double* amp) { return hipErrorInvalidValue; }
    virtual hipError_t fields(lbem_s* h, double* E, double* B, double* partials) = 0;
    virtual hipError_t init(lbem_s* h, const double* dE, const double* dB) = 0;
    virtual hipError_t medium(lbem_s* h, const double* deps, const double* dmu, int* dflag) = 0;
};

static Geo1 geo1(const lbem_s* h)
{
    Geo1 g;
    g.nx = (int)h->cfg.nx; g.ny = (int)h->cfg.ny; g.nz = (int)h->cfg.nz; g.n = h->n;
    return g;
}

static int blocks1(int64_t n) { return (int)((n + NT - 1) / NT); }

static CellExt ext_of(const lbem_s* h)
{
    CellExt b;
    for (int a = 0; a < 3; ++a) b.kind[a] = h->bc_kind[a];
    b.keep = h->keep;
    b.ade = h->ade;
    b.pol = h->pol;
    b.ra = h->ra_set ? h->ra : nullptr;
    return b;
}
// walls, an absorber or dispersion: the single-step kernels with cell extras
static bool has_bx(const lbem_s* h)
{
    return h->keep != nullptr || h->ade != nullptr || h->ra_set || ext_of(h).walls();
}
static size_t medium_size(const lbem_s* h) { return h->prec == LBEM_F64 ? 8 : 4; }
static size_t pol_bytes(const lbem_s* h) { return h->ade ? (size_t)2 * h->P * h->n * medium_size(h) : 0; }

template <int D, typename TM>
static hipError_t launch_medium(lbem_s* h, const double* deps, const double* dmu, int* dflag)
{
    hipLaunchKernelGGL((k_medium<TM>), dim3(blocks1(h->n)), dim3(NT), 0, h->stream, deps, dmu, D,
                       h->cfg.w0_vac, geo1(h), (TM*)h->cl2, h->cfg.mu_varies ? h->mu_r : nullptr,
                       (TM*)h->dlnmu, dflag, ext_of(h));
    return hipGetLastError();
}

template <typename TM>
static hipError_t launch_aniso(lbem_s* h, const double* dfac, int* dflag, int write)
{
    hipLaunchKernelGGL((k_aniso<TM>), dim3(blocks1(h->n)), dim3(NT), 0, h->stream, dfac, h->D, h->n,
                       (TM*)h->cl2, (TM*)h->ra, dflag, write);
    return hipGetLastError();
}

template <int D, typename TM, class R>
static hipError_t launch_fields(lbem_s* h, const R& rd, double* E, double* B, double* partials)
{
    hipLaunchKernelGGL((k_fields<D, TM, R>), dim3(blocks1(h->n)), dim3(NT), 0, h->stream, rd,
                       (const TM*)h->cl2, h->mu_set ? h->mu_r : nullptr, geo1(h), E, B, partials,
                       (const TM*)(h->ra_set ? h->ra : nullptr));
    return hipGetLastError();
}

// fused 2D launches: (steps per launch, tile rows) pairs that are instantiated
// The paper's tau = 1/2 gets its own instantiation: the reflection collision
// folds at compile time (measured 2 % faster at 2048^2, 12 % at 8192^2 with
// four steps per launch); other tau take the general one.
template <typename T, int NS, int TY, bool MU, bool O32, bool NTS, int NTB>
static void launch_fused2d(lbem_s* h, const T* src, T* dst, const FusedSrc<T>& fs, const AmpPack<T, NS>& a)
{
    const T om = (T)(1.0 / h->cfg.tau);
    if (h->cfg.tau == 0.5)
        hipLaunchKernelGGL((k_step_fused2d<T, NS, TY, MU, O32, NTS, true, NTB>), dim3(h->fgeo.nblocks), dim3(NTB), 0,
                           h->stream, src, dst, (const T*)h->cl2, (const T*)h->dlnmu, h->fgeo, fs, a, om, 1);
    else
        hipLaunchKernelGGL((k_step_fused2d<T, NS, TY, MU, O32, NTS, false, NTB>), dim3(h->fgeo.nblocks), dim3(NTB), 0,
                           h->stream, src, dst, (const T*)h->cl2, (const T*)h->dlnmu, h->fgeo, fs, a, om, 0);
}

template <typename T, int NS, int TY, bool MU, int NTB>
static hipError_t go_fused_ntm(lbem_s* h, const T* src, T* dst, const double* amp)
{
    FusedSrc<T> fs;
    fs.off = h->nfsrc ? h->fsrc_off : nullptr;
    fs.ent = h->fsrc_ent;
    fs.val = (const T*)h->fsrc_val;
    AmpPack<T, NS> a;
    for (int j = 0; j < NS; ++j) a.a[j] = (T)(amp ? amp[j] : 0.0);
    // 32-bit element offsets while one population plane fits 2^32 bytes;
    // streaming stores beyond the last-level cache (2-3 % there)
    if ((uint64_t)h->n * sizeof(T) <= (1ull << 32) && h->nts)
        launch_fused2d<T, NS, TY, MU, true, true, NTB>(h, src, dst, fs, a);
    else if ((uint64_t)h->n * sizeof(T) <= (1ull << 32))
        launch_fused2d<T, NS, TY, MU, true, false, NTB>(h, src, dst, fs, a);
    else
        launch_fused2d<T, NS, TY, MU, false, false, NTB>(h, src, dst, fs, a);
    return hipGetLastError();
}

template <typename T, int NS, int TY, int NTB = NT>
static hipError_t go_fused_nt(lbem_s* h, const T* src, T* dst, const double* amp)
{
    if (h->mu_set) return go_fused_ntm<T, NS, TY, true, NTB>(h, src, dst, amp);
    return go_fused_ntm<T, NS, TY, false, NTB>(h, src, dst, amp);
}

template <typename T>
static hipError_t go_fused(lbem_s* h, const T* src, T* dst, const double* amp)
{
    const int ns = h->fuse_ns, ty = h->fuse_ty;
    if constexpr (sizeof(T) == 4) {
        if (h->fuse_nt == 512) {
            if (ns == 2 && ty == 16) return go_fused_nt<T, 2, 16, 512>(h, src, dst, amp);
            if (ns == 2 && ty == 32) return go_fused_nt<T, 2, 32, 512>(h, src, dst, amp);
            if (ns == 4 && ty == 16) return go_fused_nt<T, 4, 16, 512>(h, src, dst, amp);
        }
        if (ns == 2 && ty == 16) return go_fused_nt<T, 2, 16>(h, src, dst, amp);
        if (ns == 2 && ty == 8) return go_fused_nt<T, 2, 8>(h, src, dst, amp);
        if (ns == 2 && ty == 4) return go_fused_nt<T, 2, 4>(h, src, dst, amp);
        if (ns == 3 && ty == 16) return go_fused_nt<T, 3, 16>(h, src, dst, amp);
        if (ns == 4 && ty == 16) return go_fused_nt<T, 4, 16>(h, src, dst, amp);
        if (ns == 4 && ty == 8) return go_fused_nt<T, 4, 8>(h, src, dst, amp);
    } else {
        if (ns == 2 && ty == 8) return go_fused_nt<T, 2, 8>(h, src, dst, amp);
        if (ns == 2 && ty == 4) return go_fused_nt<T, 2, 4>(h, src, dst, amp);
        if (ns == 3 && ty == 8) return go_fused_nt<T, 3, 8>(h, src, dst, amp);
    }
    return hipErrorInvalidValue;
}

template <typename T, int TX, int TY, bool MU, bool NTS>
static hipError_t go_fused3_t(lbem_s* h, const T* src, T* dst, const double* amp)
{
    FusedSrc<T> fs;
    fs.off = h->nfsrc ? h->fsrc_off : nullptr;
    fs.ent = h->fsrc_ent;
    fs.val = (const T*)h->fsrc_val;
    AmpPack<T, 2> a;
    for (int j = 0; j < 2; ++j) a.a[j] = (T)(amp ? amp[j] : 0.0);
    // tau = 1/2 folded at compile time (4.5 % at 256^3), other tau general
    if (h->cfg.tau == 0.5)
        hipLaunchKernelGGL((k_step_fused3d<T, TX, TY, MU, NTS, true>), dim3(h->fgeo.nblocks), dim3(TX * TY), 0,
                           h->stream, src, dst, (const T*)h->cl2, (const T*)h->dlnmu, h->fgeo, h->f3_lz, fs, a,
                           (T)(1.0 / h->cfg.tau), 1);
    else
        hipLaunchKernelGGL((k_step_fused3d<T, TX, TY, MU, NTS, false>), dim3(h->fgeo.nblocks), dim3(TX * TY), 0,
                           h->stream, src, dst, (const T*)h->cl2, (const T*)h->dlnmu, h->fgeo, h->f3_lz, fs, a,
                           (T)(1.0 / h->cfg.tau), 0);
    return hipGetLastError();
}

template <typename T, bool NTS>
static hipError_t go_fused3_n(lbem_s* h, const T* src, T* dst, const double* amp)
{
    if constexpr (std::is_same<T, float>::value) {
        if (h->f3_tx == 64 && h->f3_ty == 8) {
            if (h->mu_set) return go_fused3_t<T, 64, 8, true, NTS>(h, src, dst, amp);
            return go_fused3_t<T, 64, 8, false, NTS>(h, src, dst, amp);
        }
    }
    if (h->mu_set) {
        if (h->f3_tx == 64) return go_fused3_t<T, 64, 4, true, NTS>(h, src, dst, amp);
        return go_fused3_t<T, 32, 8, true, NTS>(h, src, dst, amp);
    }
    if (h->f3_tx == 64) return go_fused3_t<T, 64, 4, false, NTS>(h, src, dst, amp);
    return go_fused3_t<T, 32, 8, false, NTS>(h, src, dst, amp);
}

template <typename T>
static hipError_t go_fused3(lbem_s* h, const T* src, T* dst, const double* amp)
{
    return h->nts ? go_fused3_n<T, true>(h, src, dst, amp) : go_fused3_n<T, false>(h, src, dst, amp);
}

// formats with a multi-step kernel: the plain FP32/FP64 ones, and the 3D
// deviation formats (two steps)
static bool fused_format(const lbem_s* h) { return h->prec <= LBEM_F32 || (is_dev(h->prec) && h->D == 3); }

static bool fused_ok(const lbem_s* h)
{
    return fused_format(h) && h->streaming == LBEM_STREAM_PULL && h->fuse_ns > 1 && !has_bx(h);
}

// plain formats: populations stored as S, arithmetic in T
template <int D, typename T, typename S = T>
struct PlainImpl : Impl {
    template <int RM, int WM, bool MU, bool NTS>
    static hipError_t go_xrow(lbem_s* h, const S* src, S* dst, T amp)
    {
        hipLaunchKernelGGL((k_step_xrow<T, RM, WM, MU, S, NTS, 2>), dim3(h->xgeo.nblocks), dim3(NT), 0, h->stream,
                           src, dst, (const T*)h->cl2, (const T*)h->dlnmu, h->xgeo,
                           h->nxsrc ? h->xsrc_off : nullptr, h->xsrc_ent, (const T*)h->xsrc_val, amp,
                           (T)(1.0 / h->cfg.tau), (int)(h->cfg.tau == 0.5));
        return hipGetLastError();
    }
    template <int RM, int WM, int V, bool MU, bool BX = false>
    static hipError_t go(lbem_s* h, const S* src, S* dst, T amp)
    {
        if constexpr (D == 3 && !BX && V == 1) {
            if (h->xrow) return h->nts ? go_xrow<RM, WM, MU, true>(h, src, dst, amp)
                                       : go_xrow<RM, WM, MU, false>(h, src, dst, amp);
        }
        SrcArgs<T> s;
        s.off = h->nsrc ? h->src_off : nullptr;
        s.ent = h->src_ent;
        s.val = (const T*)h->src_val;
        s.amp = amp;
        const double om = 1.0 / h->cfg.tau;
        if (h->nts) {
            hipLaunchKernelGGL((k_step_plain<D, T, RM, WM, V, MU, BX, S, true>), dim3(h->geo.nblocks), dim3(NT), 0,
                               h->stream, src, dst, (const T*)h->cl2, (const T*)h->dlnmu, h->geo, s, (T)om,
                               (int)(h->cfg.tau == 0.5), ext_of(h));
            return hipGetLastError();
        }
        hipLaunchKernelGGL((k_step_plain<D, T, RM, WM, V, MU, BX, S>), dim3(h->geo.nblocks), dim3(NT), 0,
                           h->stream, src, dst, (const T*)h->cl2, (const T*)h->dlnmu, h->geo, s, (T)om,
                           (int)(h->cfg.tau == 0.5), ext_of(h));
        return hipGetLastError();
    }
    template <int RM, int WM>
    static hipError_t go_v(lbem_s* h, const S* src, S* dst, T amp)
    {
        if constexpr (WM == W_LOCAL && RM != R_PULL_SWAP) {
            if (has_bx(h)) {   // pull streaming only (AA is refused with walls or an absorber)
                if (h->mu_set) return go<RM, WM, 1, true, true>(h, src, dst, amp);
                return go<RM, WM, 1, false, true>(h, src, dst, amp);
            }
        }
        if (h->mu_set) return go<RM, WM, 1, true>(h, src, dst, amp);
        switch (h->vec) {
            case 2: return go<RM, WM, 2, false>(h, src, dst, amp);
            case 4:
                if constexpr (D == 2) return go<RM, WM, 4, false>(h, src, dst, amp);
                return hipErrorInvalidValue;
            default: return go<RM, WM, 1, false>(h, src, dst, amp);
        }
    }
    hipError_t step(lbem_s* h, double amp) override
    {
        S* a = (S*)h->pop[h->cur];
        if (h->streaming == LBEM_STREAM_AA) {
            hipError_t e;
            if (h->layout == LAYOUT_NATURAL) {
                e = go_v<R_LOCAL, W_SWAP>(h, a, a, (T)amp);
                h->layout = LAYOUT_AA_SWAPPED;
            } else {
                e = go_v<R_PULL_SWAP, W_PUSH>(h, a, a, (T)amp);
                h->layout = LAYOUT_NATURAL;
            }
            return e;
        }
        S* b = (S*)h->pop[1 - h->cur];
        hipError_t e = h->layout == LAYOUT_NATURAL ? go_v<R_LOCAL, W_LOCAL>(h, a, b, (T)amp)
                                                   : go_v<R_PULL, W_LOCAL>(h, a, b, (T)amp);
        h->cur = 1 - h->cur;
        h->layout = LAYOUT_PULL_PENDING;
        return e;
    }
    hipError_t step_fused(lbem_s* h, const double* amp) override
    {
        if constexpr (!std::is_same<S, T>::value) {
            return hipErrorInvalidValue;   // the multi-step kernels keep FP64/FP32 storage
        } else {
            const T* a = (const T*)h->pop[h->cur];
            T* b = (T*)h->pop[1 - h->cur];
            hipError_t e;
            if constexpr (D == 2) e = go_fused<T>(h, a, b, amp);
            else e = go_fused3<T>(h, a, b, amp);
            h->cur = 1 - h->cur;
            return e;
        }
    }
    hipError_t fields(lbem_s* h, double* E, double* B, double* partials) override
    {
        const S* a = (const S*)h->pop[h->cur];
        const CellExt bc = ext_of(h);
        if (h->layout == LAYOUT_NATURAL)
            return launch_fields<D, T>(h, PlainReader<D, S, R_LOCAL>{a, h->n, bc}, E, B, partials);
        if (h->layout == LAYOUT_PULL_PENDING)
            return launch_fields<D, T>(h, PlainReader<D, S, R_PULL>{a, h->n, bc}, E, B, partials);
        return launch_fields<D, T>(h, PlainReader<D, S, R_PULL_SWAP>{a, h->n, bc}, E, B, partials);
    }
    hipError_t init(lbem_s* h, const double* dE, const double* dB) override
    {
        h->cur = 0;
        h->layout = LAYOUT_NATURAL;
        hipLaunchKernelGGL((k_init_plain<D, T, S>), dim3(blocks1(h->n)), dim3(NT), 0, h->stream, dE, dB,
                           (const T*)h->cl2, h->n, (S*)h->pop[0], (const T*)(h->ra_set ? h->ra : nullptr));
        return hipGetLastError();
    }
    hipError_t medium(lbem_s* h, const double* deps, const double* dmu, int* dflag) override
    {
        return launch_medium<D, T>(h, deps, dmu, dflag);
    }
};

template <int D, typename H, bool GH>
struct DevImpl : Impl {
    static float* M(lbem_s* h, int k) { return (float*)h->pop[k]; }
    static H* Dv(lbem_s* h, int k)
    {
        const int P = Lat<D>::P;
        return (H*)(h->pop[k] + align256((size_t)(P + D) * h->n * 4));
    }
    template <bool MU, bool NTS, int NTB, int EXT = 0>
    static void go_row_n(lbem_s* h, int from, int to, const int* so, float amp, float om, int th)
    {
        hipLaunchKernelGGL((k_step_dev3r<H, GH, MU, NTS, 2, NTB, EXT>), dim3(h->rgeo.nblocks), dim3(NTB), 0,
                           h->stream, M(h, from), Dv(h, from), M(h, to), Dv(h, to), (const float*)h->cl2,
                           (const float*)h->dlnmu, h->rgeo, so, h->rsrc_ent, h->rsrc_val, amp, om, th, ext_of(h));
    }
    // the row-tile step with cell extras (walls, dispersion, absorbing
    // layer): 512-thread tiles, no anisotropy
    static bool row_ext_ok(const lbem_s* h)
    {
        return h->rowk && !h->ra_set && h->rntb == 512;
    }
    template <bool MU>
    static hipError_t go_row(lbem_s* h, int from, int to, const int* so, float amp, float om, int th)
    {
        if constexpr (D == 3) {
            const int nb = h->rntb;
            if (h->nts) {
                if (nb == 1024) go_row_n<MU, true, 1024>(h, from, to, so, amp, om, th);
                else if (nb == 512) go_row_n<MU, true, 512>(h, from, to, so, amp, om, th);
                else go_row_n<MU, true, 256>(h, from, to, so, amp, om, th);
            } else {
                if (nb == 1024) go_row_n<MU, false, 1024>(h, from, to, so, amp, om, th);
                else if (nb == 512) go_row_n<MU, false, 512>(h, from, to, so, amp, om, th);
                else go_row_n<MU, false, 256>(h, from, to, so, amp, om, th);
            }
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    // BX: 0 no cell extras, 1 walls only, 2 walls, dispersion and absorber
    template <int RM, int V, bool MU, int BX = 0>
    static hipError_t go(lbem_s* h, int from, int to, float amp)
    {
        SrcArgs<float> s;
        if constexpr (D == 3 && BX != 0 && RM == R_PULL) {
            if (row_ext_ok(h)) {
                const int* so = h->nrsrc ? h->rsrc_off : nullptr;
                const float om = (float)(1.0 / h->cfg.tau);
                const int th = h->cfg.tau == 0.5;
                // row extras mask: 1 walls, 2 dispersion / absorber
                if constexpr (BX == 1) {
                    if (h->nts) go_row_n<MU, true, 512, 1>(h, from, to, so, amp, om, th);
                    else go_row_n<MU, false, 512, 1>(h, from, to, so, amp, om, th);
                } else if (ext_of(h).walls()) {
                    if (h->nts) go_row_n<MU, true, 512, 3>(h, from, to, so, amp, om, th);
                    else go_row_n<MU, false, 512, 3>(h, from, to, so, amp, om, th);
                } else {
                    if (h->nts) go_row_n<MU, true, 512, 2>(h, from, to, so, amp, om, th);
                    else go_row_n<MU, false, 512, 2>(h, from, to, so, amp, om, th);
                }
                return hipGetLastError();
            }
        }
        if constexpr (D == 3 && !BX && RM == R_PULL) {
            if (h->rowk) {
                const int* so = h->nrsrc ? h->rsrc_off : nullptr;
                const float om = (float)(1.0 / h->cfg.tau);
                const int th = h->cfg.tau == 0.5;
                return go_row<MU>(h, from, to, so, amp, om, th);
            }
        }
        if constexpr (D == 3 && !BX) {
            if (h->zmarch) {
                s.off = h->nzsrc ? h->zsrc_off : nullptr;
                s.ent = h->zsrc_ent;
                s.val = (const float*)h->zsrc_val;
                s.amp = amp;
                if (h->nts)
                    hipLaunchKernelGGL((k_step_dev3z<H, GH, RM, MU, true>), dim3(h->zgeo.nblocks), dim3(NT), 0,
                                       h->stream, M(h, from), Dv(h, from), M(h, to), Dv(h, to),
                                       (const float*)h->cl2, (const float*)h->dlnmu, h->zgeo, h->zlz, s,
                                       (float)(1.0 / h->cfg.tau), (int)(h->cfg.tau == 0.5));
                else
                    hipLaunchKernelGGL((k_step_dev3z<H, GH, RM, MU>), dim3(h->zgeo.nblocks), dim3(NT), 0,
                                       h->stream, M(h, from), Dv(h, from), M(h, to), Dv(h, to),
                                       (const float*)h->cl2, (const float*)h->dlnmu, h->zgeo, h->zlz, s,
                                       (float)(1.0 / h->cfg.tau), (int)(h->cfg.tau == 0.5));
                return hipGetLastError();
            }
        }
        s.off = h->nsrc ? h->src_off : nullptr;
        s.ent = h->src_ent;
        s.val = (const float*)h->src_val;
        s.amp = amp;
        if (h->nts) {
            hipLaunchKernelGGL((k_step_dev<D, H, GH, RM, V, MU, BX, true>), dim3(h->geo.nblocks), dim3(NT), 0,
                               h->stream, M(h, from), Dv(h, from), M(h, to), Dv(h, to), (const float*)h->cl2,
                               (const float*)h->dlnmu, h->geo, s, (float)(1.0 / h->cfg.tau),
                               (int)(h->cfg.tau == 0.5), ext_of(h));
            return hipGetLastError();
        }
        hipLaunchKernelGGL((k_step_dev<D, H, GH, RM, V, MU, BX>), dim3(h->geo.nblocks), dim3(NT), 0,
                           h->stream, M(h, from), Dv(h, from), M(h, to), Dv(h, to), (const float*)h->cl2,
                           (const float*)h->dlnmu, h->geo, s, (float)(1.0 / h->cfg.tau),
                           (int)(h->cfg.tau == 0.5), ext_of(h));
        return hipGetLastError();
    }
    template <int RM>
    static hipError_t go_v(lbem_s* h, int from, int to, float amp)
    {
        if (has_bx(h)) {
            // walls only: the closed-form collision (no anisotropy in 16 bits)
            const bool walls_only = h->ade == nullptr && h->keep == nullptr;
            if (h->mu_set)
                return walls_only ? go<RM, 1, true, 1>(h, from, to, amp) : go<RM, 1, true, 2>(h, from, to, amp);
            return walls_only ? go<RM, 1, false, 1>(h, from, to, amp) : go<RM, 1, false, 2>(h, from, to, amp);
        }
        if (h->mu_set) return go<RM, 1, true>(h, from, to, amp);
        switch (h->vec) {
            case 2: return go<RM, 2, false>(h, from, to, amp);
            case 4:
                if constexpr (D == 2) return go<RM, 4, false>(h, from, to, amp);
                return hipErrorInvalidValue;
            default: return go<RM, 1, false>(h, from, to, amp);
        }
    }
    hipError_t step(lbem_s* h, double amp) override
    {
        hipError_t e = h->layout == LAYOUT_NATURAL ? go_v<R_LOCAL>(h, h->cur, 1 - h->cur, (float)amp)
                                                   : go_v<R_PULL>(h, h->cur, 1 - h->cur, (float)amp);
        h->cur = 1 - h->cur;
        h->layout = LAYOUT_PULL_PENDING;
        return e;
    }
    hipError_t step_fused(lbem_s* h, const double* amp) override
    {
        if constexpr (D == 3) {
            FusedSrc<float> fs;
            fs.off = h->nfsrc ? h->fsrc_off : nullptr;
            fs.ent = h->fsrc_ent;
            fs.val = (const float*)h->fsrc_val;
            AmpPack<float, 2> a;
            for (int j = 0; j < 2; ++j) a.a[j] = (float)(amp ? amp[j] : 0.0);
            const int from = h->cur, to = 1 - h->cur;
            if (h->mu_set)
                hipLaunchKernelGGL((k_step_dev3f<H, GH, true>), dim3(h->fgeo.nblocks), dim3(NT), 0, h->stream,
                                   M(h, from), Dv(h, from), M(h, to), Dv(h, to), (const float*)h->cl2,
                                   (const float*)h->dlnmu, h->fgeo, h->f3_lz, fs, a, (float)(1.0 / h->cfg.tau),
                                   (int)(h->cfg.tau == 0.5));
            else
                hipLaunchKernelGGL((k_step_dev3f<H, GH, false>), dim3(h->fgeo.nblocks), dim3(NT), 0, h->stream,
                                   M(h, from), Dv(h, from), M(h, to), Dv(h, to), (const float*)h->cl2,
                                   (const float*)h->dlnmu, h->fgeo, h->f3_lz, fs, a, (float)(1.0 / h->cfg.tau),
                                   (int)(h->cfg.tau == 0.5));
            h->cur = to;
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    hipError_t fields(lbem_s* h, double* E, double* B, double* partials) override
    {
        if (h->layout == LAYOUT_NATURAL)
            return launch_fields<D, float>(h, DevReader<D, H, GH, R_LOCAL>{M(h, h->cur), Dv(h, h->cur), h->n,
                                                                            ext_of(h)},
                                           E, B, partials);
        return launch_fields<D, float>(h, DevReader<D, H, GH, R_PULL>{M(h, h->cur), Dv(h, h->cur), h->n,
                                                                       ext_of(h)}, E,
                                       B, partials);
    }
    hipError_t init(lbem_s* h, const double* dE, const double* dB) override
    {
        h->cur = 0;
        h->layout = LAYOUT_NATURAL;
        hipLaunchKernelGGL((k_init_dev<D, H, GH>), dim3(blocks1(h->n)), dim3(NT), 0, h->stream, dE, dB,
                           (const float*)h->cl2, h->n, M(h, 0), Dv(h, 0));
        return hipGetLastError();
    }
    hipError_t medium(lbem_s* h, const double* deps, const double* dmu, int* dflag) override
    {
        return launch_medium<D, float>(h, deps, dmu, dflag);
    }
};

static Impl* make_impl(int D, int prec)
{
    if (D == 2) {
        switch (prec) {
            case LBEM_F64: return new (std::nothrow) PlainImpl<2, double>();
            case LBEM_F32: return new (std::nothrow) PlainImpl<2, float>();
            case LBEM_F16: return new (std::nothrow) PlainImpl<2, float, __half>();
            case LBEM_F16DEV: return new (std::nothrow) DevImpl<2, __half, false>();
            case LBEM_BF16DEV: return new (std::nothrow) DevImpl<2, __hip_bfloat16, false>();
            case LBEM_F16GHOST: return new (std::nothrow) DevImpl<2, __half, true>();
            default: return new (std::nothrow) DevImpl<2, __hip_bfloat16, true>();
        }
    }
    switch (prec) {
        case LBEM_F64: return new (std::nothrow) PlainImpl<3, double>();
        case LBEM_F32: return new (std::nothrow) PlainImpl<3, float>();
        case LBEM_F16: return new (std::nothrow) PlainImpl<3, float, __half>();
        case LBEM_F16DEV: return new (std::nothrow) DevImpl<3, __half, false>();
        case LBEM_BF16DEV: return new (std::nothrow) DevImpl<3, __hip_bfloat16, false>();
        case LBEM_F16GHOST: return new (std::nothrow) DevImpl<3, __half, true>();
        default: return new (std::nothrow) DevImpl<3, __hip_bfloat16, true>();
    }
}

static void make_geo(lbem_s* h)
{
    const int nx = (int)h->cfg.nx, ny = (int)h->cfg.ny, nz = (int)h->cfg.nz;
    int bx = 64;
    while (bx < nx && bx < NT) bx <<= 1;
    int sh = 0;
    while ((1 << sh) < bx) ++sh;
    const int rb = NT / bx;
    Geo& g = h->geo;
    g.nx = nx; g.ny = ny; g.nz = nz; g.n = h->n;
    g.bx_shift = sh;
    g.tiles_x = (nx + bx - 1) / bx;
    g.tiles_y = (ny + rb * h->vec - 1) / (rb * h->vec);
    g.nblocks = g.tiles_x * g.tiles_y * nz;
    // measured defaults: XCD-contiguous tile ranges help 2D; in 3D, runs of
    // 16 neighbouring tiles per XCD beyond the last-level cache (512^3 FP32
    // AA 4.39 -> 4.35 ms; at 256^3 1.5 % slower than tiles dealt one by one)
    const bool big3 = h->D == 3 && !is_dev(h->prec) && (double)h->n >= 4.0e7;
    g.xcd = env_int("LBEM_XCD", h->D == 2 ? 1 : (big3 ? 16 : 0));
    const int sdef = (h->D == 3 && is_dev(h->prec)) ? 32 : 0;
    g.strip = env_int("LBEM_STRIP", sdef);
    if (g.strip <= 0 || nz == 1 || g.strip >= g.tiles_y || g.tiles_y % g.strip != 0) g.strip = 0;
}

static void make_fused3_geo(lbem_s* h)
{
    const bool f64 = h->prec == LBEM_F64;
    // FP64 frames do not fit enough blocks per CU for the pair to pay off
    // (measured slower than single steps at 256^3), so FP64 runs single steps
    // unless asked for.
    const bool small = (double)h->n < FUSE3D_MIN;
    h->fuse_ns = env_int("LBEM_FUSE3", (f64 || small) ? 1 : 2) == 2 ? 2 : 1;
    h->f3_tx = env_int("LBEM_FUSE3_TX", f64 ? 32 : 64) == 64 && !f64 ? 64 : 32;
    if (is_dev(h->prec)) {
        // the two-step deviation kernel (64 x 4 column tiles)
        h->fuse_ns = env_int("LBEM_DEV3F", 0) ? 2 : 1;
        h->f3_tx = 64;
    }
    h->f3_ty = NT / h->f3_tx;
    // FP32 64-wide tiles take 8 rows: 512 threads, two blocks per CU (80 KB of
    // LDS, <= 128 VGPRs), and step 1 runs on a frame of 1.29x the tile instead
    // of 1.55x.  Measured, us per step, 64x4 / 64x8 / 32x16: 512^3 2801 / 2508
    // / 2663, 384^3 1219 / 1103 / 1233, 256^3 348 / 307 / 332, 192^3 167 / 150
    // / 161.  LBEM_FUSE3_TY=4 keeps the 256-thread tiles.
    if (h->prec == LBEM_F32 && h->f3_tx == 64 && env_int("LBEM_FUSE3_TY", 8) == 8) h->f3_ty = 8;
    Geo& g = h->fgeo;
    g = h->geo;
    g.tiles_x = (g.nx + h->f3_tx - 1) / h->f3_tx;
    g.tiles_y = (g.ny + h->f3_ty - 1) / h->f3_ty;
    // longest z chunk (fewest recomputed boundary planes) that still gives
    // enough blocks to fill 256 CUs
    int lz = 32;
    while (lz > 8 && (int64_t)g.tiles_x * g.tiles_y * ((g.nz + lz - 1) / lz) < 768) lz /= 2;
    h->f3_lz = std::max(1, env_int("LBEM_FUSE3_LZ", lz));
    g.nblocks = g.tiles_x * g.tiles_y * ((g.nz + h->f3_lz - 1) / h->f3_lz);
    g.strip = 0;
    // runs of 32 neighbouring tiles per XCD (measured, FP32: 512^3 2.82 ->
    // 2.79 ms against tiles dealt one by one; 384^3 1.27 -> 1.22, 256^3 0.365
    // -> 0.347, 192^3 0.170 -> 0.167 against contiguous ranges per XCD)
    g.xcd = env_int("LBEM_FUSE3_XCD", 32);
}

static void make_fused_geo(lbem_s* h)
{
    h->fuse_nt = 256;
    if (h->D == 3) {
        make_fused3_geo(h);
        return;
    }
    const bool f64 = h->prec == LBEM_F64;
    // FP32: four steps per pass on 64 x 16 tiles of 512 threads, at every size.
    // Measured, us per step, (steps, rows, threads): 2048^2 (2, 8, 256) 13.49,
    // (4, 8, 256) 13.23, (4, 16, 256) 13.29, (4, 16, 512) 10.49; 1024^2 5.13 /
    // 4.61 / 4.44 / 3.72; 512^2 2.45 / 1.85 / 2.29 / 1.65; 128^2 2.06 / 1.59 /
    // 2.12 / 1.48; 4096^2 80.4 / 59.6 / 56.4 / 50.3; 8192^2 296 / 223 / 210 /
    // 185.  The 512-thread block halves the frame per tile cell of the
    // 256-thread 64 x 16 tile at the same two cells per thread.  With a varying
    // mu the frame also stages grad ln mu, and the four-step 512-thread tile
    // (86 KB of LDS) leaves one block per CU: two steps on 64 x 8 tiles there
    // (2048^2, us per step: (2, 8, 256) 16.02, (2, 16, 512) 15.95, (4, 8, 256)
    // 19.36, (4, 16, 512) 18.73).  FP64: two steps on 64 x 4 tiles.
    const bool muv = h->cfg.mu_varies != 0;
    h->fuse_ns = env_int("LBEM_FUSE", (f64 || muv) ? 2 : 4);
    h->fuse_ty = env_int("LBEM_FUSE_TY", f64 ? 4 : (muv ? 8 : 16));
    // only the instantiated (steps, rows, threads) triples; anything else runs
    // single steps.  The thread count follows the (steps, rows) pair unless set.
    const int ns = h->fuse_ns, ty = h->fuse_ty;
    const bool pair512 = !f64 && ((ns == 2 && (ty == 16 || ty == 32)) || (ns == 4 && ty == 16));
    h->fuse_nt = (!f64 && env_int("LBEM_FUSE_NT", pair512 ? 512 : 256) == 512) ? 512 : 256;
    const bool ok = f64 ? ((ns == 2 && (ty == 8 || ty == 4)) || (ns == 3 && ty == 8))
                  : h->fuse_nt == 512 ? ((ns == 2 && (ty == 16 || ty == 32)) || (ns == 4 && ty == 16))
                        : ((ns == 2 && (ty == 16 || ty == 8 || ty == 4)) || (ns == 3 && ty == 16) ||
                           (ns == 4 && (ty == 16 || ty == 8)));
    if (!ok) h->fuse_ns = 1;
    Geo& g = h->fgeo;
    g = h->geo;
    g.tiles_x = (g.nx + TXF - 1) / TXF;
    g.tiles_y = (g.ny + h->fuse_ty - 1) / h->fuse_ty;
    g.nblocks = g.tiles_x * g.tiles_y;
    g.strip = 0;
}

static void make_zmarch_geo(lbem_s* h)
{
    // rows the row tiles take (with the default 512-thread block) go by the
    // state size, longer ones by the cell count
    const bool ghost = h->prec == LBEM_F16GHOST || h->prec == LBEM_BF16GHOST;
    const bool big = h->cfg.nx <= ROWX_MAX ? (double)h->n * (ghost ? 112.0 : 136.0) > ROWTILE_BYTES
                                           : (double)h->n >= SMALL3D;
    h->zmarch = (h->D == 3 && is_dev(h->prec)) ? env_int("LBEM_DEV3Z", big) : 0;
    h->zlz = std::max(1, env_int("LBEM_DEV3Z_LZ", 16));
    Geo& g = h->zgeo;
    g = h->geo;
    g.tiles_x = (g.nx + TXD - 1) / TXD;
    g.tiles_y = (g.ny + TYD - 1) / TYD;
    const int nzc = (g.nz + h->zlz - 1) / h->zlz;
    g.nblocks = g.tiles_x * g.tiles_y * nzc;
    g.strip = 0;
    g.xcd = env_int("LBEM_DEV3Z_XCD", 0);
}

// Whole-row blocks of k_step_xrow (3D plain formats, single steps without
// cell extras): CX = 2 cells per thread, tpr threads per row, NT/tpr rows per
// block, one plane.  Measured (same box, per step): plain FP16 AA 2.33 -> 2.15
// ms at 512^3 and 0.261 -> 0.244 ms at 256^3, where a 64-wide row of 16-bit
// values is one cache line and a shifted one touches two; FP32 AA and pull
// within +-3 % at 256^3 and 512^3; every format slower while the state is
// Infinity-Cache resident (128^3).  So the default takes it for FP16 storage
// beyond 6e6 cells; LBEM_XROW=1 selects it for the others.
static void make_xrow_geo(lbem_s* h)
{
    const int nx = (int)h->cfg.nx, ny = (int)h->cfg.ny, nz = (int)h->cfg.nz;
    const bool plain = h->prec <= LBEM_F32 || h->prec == LBEM_F16;
    const int dflt = h->prec == LBEM_F16 && (double)h->n >= XROW3D;
    h->xrow = (h->D == 3 && plain && nx <= 2 * NT && h->vec == 1) ? env_int("LBEM_XROW", dflt) : 0;
    if (!h->xrow) return;     // rows longer than 2*NT have no whole-row tiling (no rows per block)
    XRowGeo& g = h->xgeo;
    g.nx = nx; g.ny = ny; g.nz = nz; g.n = h->n;
    int tpr = 64;
    while (2 * tpr < nx) tpr <<= 1;
    g.tpr = tpr;
    g.rows = NT / tpr;
    g.tiles_y = (ny + g.rows - 1) / g.rows;
    g.nblocks = g.tiles_y * nz;
}

// Whole-row tiles of k_step_dev3r: CX = 2 cells per thread numbered through
// the tile's rows (short rows leave no thread idle and keep every wave on
// consecutive cells), 2 block / nx rows per tile; the planes per chunk are
// chosen below.  Rows longer than twice the block (or ROWX_MAX) keep the
// column-tile z-march.
static void make_row_geo(lbem_s* h)
{
    const int nx = (int)h->cfg.nx, ny = (int)h->cfg.ny, nz = (int)h->cfg.nz;
    // 512 threads: two blocks per CU (73 KB of LDS each) hide the memory
    // latency that one 1024-thread block with taller tiles leaves exposed
    // (measured at 512^3: 3.20 ms per step against 5.31, 256 threads 3.61)
    int ntb = env_int("LBEM_DEV3R_NT", 512);
    if (ntb != 256 && ntb != 1024) ntb = 512;
    h->rowk = (h->zmarch && nx <= std::min(ROWX_MAX, 2 * ntb)) ? env_int("LBEM_DEV3R", 1) : 0;
    RowGeo& g = h->rgeo;
    g.nx = nx; g.ny = ny; g.nz = nz; g.n = h->n;
    h->rntb = ntb;
    // Measured (512^3 and 256^3, FP16 ghost and Dev-Q): blocks dealt to the
    // XCDs in turn, so that the blocks resident at a time are neighbouring
    // tiles of one z band, run 5-7 % faster than contiguous tile ranges per XCD
    // (512^3 ghost 2.95 against 3.20 ms); runs of 8 neighbouring tiles per XCD
    // (their y-halo rows shared in one L2) another 0.8-1.2 % (2.92 ms; runs
    // of 2, 4 or 16 within 0.5 % of it).
    // As many rows per tile as the block holds: rows of a power-of-two thread
    // count with idle threads ran slower (FP16 ghost, us per step: 160^3 123
    // against 106, 320^3 796 against 732, 384^3 1326 against 1276), and so did
    // fewer rows with more blocks (192^3: 4 rows 171-183 against 5 rows 166).
    // Planes per chunk: the longest of 1..7 whose last round of resident
    // blocks (1024 / block threads per CU) is within 0.08 of the fullest,
    // among the lengths that give at least two rounds of blocks (all of them if
    // none does).  A thin last round costs more than the chunk ends decoded
    // twice: FP16 ghost, planes -> us per step, 192^3 (5 rows) 3 166, 5 166,
    // 6 176, 7 190; 160^3 (6 rows) 3 106, 4 120, 5 109; 144^3 (7 rows) 2 88,
    // 3 107; 512^3 (2 rows) 7 2909-2913, 8 2917-2925, 16 2945.
    int cus = 256, dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        cus = v;
    const int64_t slots = (int64_t)cus * (1024 / ntb);
    const int tymax = std::max(1, 2 * ntb / nx);
    g.ty = std::max(1, std::min(tymax, env_int("LBEM_DEV3R_TY", tymax)));
    g.tiles_y = (ny + g.ty - 1) / g.ty;
    auto nblk = [&](int c) { return (int64_t)g.tiles_y * ((nz + c - 1) / c); };
    auto fill = [&](int c) {
        const int64_t nb = nblk(c);
        return (double)nb / (double)(((nb + slots - 1) / slots) * slots);
    };
    const bool two = nblk(1) >= 2 * slots;
    double best = 0.0;
    for (int c = 1; c <= 7; ++c)
        if (!two || nblk(c) >= 2 * slots) best = std::max(best, fill(c));
    int lz = 1;
    for (int c = 7; c >= 1; --c)
        if ((!two || nblk(c) >= 2 * slots) && fill(c) >= best - 0.08) { lz = c; break; }
    g.lz = std::max(1, env_int("LBEM_DEV3R_LZ", lz));
    g.nblocks = g.tiles_y * ((nz + g.lz - 1) / g.lz);
    g.xcd = env_int("LBEM_DEV3R_XCD", 8);
}

// The whole-row tiling of a 3D deviation handle inside a batch: blocks of
// BROW_NT threads, two cells per thread numbered through the tile's rows,
// 2 BROW_NT / nx rows per tile (nx = 64: 16 rows); chunks of 8 planes.
// Rows longer than 2 BROW_NT cells keep the per-cell tiles.
static void make_batch_row_geo(lbem_s* h)
{
    const int nx = (int)h->cfg.nx, ny = (int)h->cfg.ny, nz = (int)h->cfg.nz;
    h->brow = (h->D == 3 && is_dev(h->prec) && nx <= std::min(ROWX_MAX, 2 * BROW_NT)) ? env_int("LBEM_BATCH_ROW", 1) : 0;
    if (!h->brow) return;
    RowGeo& g = h->bgeo;
    g.nx = nx; g.ny = ny; g.nz = nz; g.n = h->n;
    g.ty = 2 * BROW_NT / nx;
    g.tiles_y = (ny + g.ty - 1) / g.ty;
    g.lz = std::max(1, env_int("LBEM_BATCH_ROW_LZ", 8));
    g.nblocks = g.tiles_y * ((nz + g.lz - 1) / g.lz);
    g.xcd = 0;
}

// inverse of tile_coords()
static int tile_id(const Geo& g, int tx, int ty, int z)
{
    int r;
    if (g.strip > 0) r = ((ty / g.strip) * g.nz + z) * g.strip + ty % g.strip;
    else r = z * g.tiles_y + ty;
    return r * g.tiles_x + tx;
}

// ---------------------------------------------------------------------------
// static device scratch of lbem_energy_noalloc
// ---------------------------------------------------------------------------
// The FP64 B field (3n doubles) read by the divergence stencil and the
// per-block partial sums (4 per block + 4 results) live in this array instead
// of the handle's scratch.  Every GPU the library runs on holds its own copy
// until the process ends; every call on that GPU shares it and leaves the
// last call's contents.  The kernels write every element they later read, so
// nothing needs clearing between calls.
constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_BYTES / sizeof(double);
static __device__ __align__(256) double noalloc_scratch[NOALLOC_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES];   // device address of the array, per device

constexpr size_t noalloc_doubles(int64_t n) { return (size_t)3 * n + (size_t)((n + NT - 1) / NT) * 4 + 4; }
static_assert(noalloc_doubles(LBEM_NOALLOC_MAX_CELLS) <= NOALLOC_DOUBLES &&
                  noalloc_doubles(LBEM_NOALLOC_MAX_CELLS + 1) > NOALLOC_DOUBLES,
              "LBEM_NOALLOC_MAX_CELLS is the largest lattice the static scratch holds");

// Device address of noalloc_scratch on `device`, looked up once per device
// with that device current (host code never passes the symbol itself).
hipError_t noalloc_address(int device, double** out)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_noalloc_ptr[device] = (double*)p;
    }
    *out = g_noalloc_ptr[device];
    return hipSuccess;
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t lbem_required_bytes(const lbem_config* cfg)
{
    if (!valid_cfg(cfg)) return 0;
    return sizes_of(cfg).total;
}

const char* lbem_strerror(int code)
{
    switch (code) {
        case LBEM_OK: return "success";
        case LBEM_EINVAL: return "invalid argument";
        case LBEM_ENOMEM: return "out of device memory or arena too small";
        case LBEM_EUNSTABLE: return "medium gives a rest weight outside [0,1)";
        case LBEM_ENONFINITE: return "non-finite diagnostic (NaN or Inf)";
        case LBEM_EDEVICE: return "HIP device or launch error";
        case LBEM_ESTATE: return "call out of order";
        case LBEM_ETOOBIG:
            return "lattice too large for the static scratch of lbem_energy_noalloc (see LBEM_NOALLOC_MAX_CELLS)";
        default: return "unknown status";
    }
}

int lbem_create(const lbem_config* cfg, lbem_t* out)
{
    API_SHARED;
    if (!out) return LBEM_EINVAL;
    *out = nullptr;
    if (!valid_cfg(cfg)) return LBEM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LBEM_EDEVICE;
    lbem_s* h = new (std::nothrow) lbem_s();
    if (!h) return LBEM_ENOMEM;
    std::memset((void*)h, 0, sizeof(*h));
    h->cfg = *cfg;
    h->D = cfg->dim;
    h->Q = 2 * h->D + 1;
    h->P = h->D * (h->D - 1) / 2;
    h->prec = cfg->prec;
    h->streaming = resolve_streaming(cfg);
    h->n = cfg->nx * cfg->ny * cfg->nz;
    h->stream = (hipStream_t)cfg->stream;
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return LBEM_EDEVICE; }
    const Sizes s = sizes_of(cfg);
    if (cfg->dev_mem) {
        if (cfg->dev_bytes < s.total || ((uintptr_t)cfg->dev_mem & 255)) { delete h; return LBEM_ENOMEM; }
        h->arena = (char*)cfg->dev_mem;
        h->own_mem = false;
    } else {
        if (hipMalloc((void**)&h->arena, s.total) != hipSuccess) { delete h; return LBEM_ENOMEM; }
        h->own_mem = true;
    }
    h->arena_bytes = s.total;
    // the population copies start zeroed, so the alignment padding inside them
    // (which no kernel writes) reads back as zeros in an exported state
    if (hipMemsetAsync(h->arena, 0, s.pop_one * s.copies, h->stream) != hipSuccess) {
        if (h->own_mem) (void)hipFree(h->arena);
        delete h;
        return LBEM_EDEVICE;
    }
    char* p = h->arena;
    h->pop[0] = p; p += s.pop_one;
    h->pop[1] = s.copies == 2 ? p : nullptr; p += s.pop_one * (s.copies - 1);
    h->cl2 = p; p += s.medium;
    if (cfg->mu_varies) {
        h->mu_r = (double*)p; p += align256((size_t)h->n * 8);
        h->dlnmu = p; p += s.mu - align256((size_t)h->n * 8);
    }
    h->scratch = (double*)p;
    h->nb_diag = blocks1(h->n);
    if (hipMallocAsync((void**)&h->partials, ((size_t)h->nb_diag * 4 + 4) * sizeof(double), h->stream) !=
        hipSuccess) {
        if (h->own_mem) (void)hipFree(h->arena);
        delete h;
        return LBEM_ENOMEM;
    }
    int vdef = 1;
    h->vec = env_int("LBEM_VEC", vdef);
    if (h->vec != 1 && h->vec != 2 && h->vec != 4) h->vec = vdef;
    if (h->D == 3 && h->vec == 4) h->vec = 2;
    if (cfg->mu_varies) h->vec = 1;
    make_geo(h);
    make_fused_geo(h);
    make_zmarch_geo(h);
    make_row_geo(h);
    make_xrow_geo(h);
    make_batch_row_geo(h);
    // Measured: streaming loads/stores slow a launch whose state fits the
    // 256 MB Infinity Cache (by up to 1.8x) and speed it up beyond that: in 3D
    // from about 1.5 times the cache on (2-10 %; at 344 MB still 9 % slower),
    // in 2D as soon as the state leaves it (FP32 AA 16 % at 335 MB, 17 % at
    // 1.3 GB).  The copies a step touches count (one with AA streaming, two
    // with pull).
    {
        const double touched = (double)s.pop_one * (h->streaming == LBEM_STREAM_AA ? 1 : 2);
        const double lim = (double)env_int("LBEM_NT_MIB", h->D == 2 ? 256 : 384) * (1 << 20);
        h->nts = env_int("LBEM_NT", touched > lim ? 1 : 0) != 0;
    }
    h->impl = make_impl(h->D, h->prec);
    if (h->impl && (hipEventCreateWithFlags(&h->sync_ev, hipEventDisableTiming) != hipSuccess ||
                    hipEventCreateWithFlags(&h->tick_ev, hipEventDisableTiming) != hipSuccess)) {
        if (h->sync_ev) (void)hipEventDestroy(h->sync_ev);
        delete h->impl;
        h->impl = nullptr;
    }
    if (!h->impl) {
        (void)hipFreeAsync(h->partials, h->stream);
        if (h->own_mem) (void)hipFree(h->arena);
        delete h;
        return LBEM_ENOMEM;
    }
    *out = h;
    return LBEM_OK;
}

static void free_source(lbem_s* h)
{
    if (h->src_off) (void)hipFree(h->src_off);
    if (h->src_ent) (void)hipFree(h->src_ent);
    if (h->src_val) (void)hipFree(h->src_val);
    if (h->fsrc_off) (void)hipFree(h->fsrc_off);
    if (h->fsrc_ent) (void)hipFree(h->fsrc_ent);
    if (h->fsrc_val) (void)hipFree(h->fsrc_val);
    h->src_off = nullptr; h->src_ent = nullptr; h->src_val = nullptr;
    if (h->zsrc_off) (void)hipFree(h->zsrc_off);
    if (h->zsrc_ent) (void)hipFree(h->zsrc_ent);
    if (h->zsrc_val) (void)hipFree(h->zsrc_val);
    if (h->xsrc_off) (void)hipFree(h->xsrc_off);
    if (h->xsrc_ent) (void)hipFree(h->xsrc_ent);
    if (h->xsrc_val) (void)hipFree(h->xsrc_val);
    h->xsrc_off = nullptr; h->xsrc_ent = nullptr; h->xsrc_val = nullptr;
    h->nxsrc = 0;
    if (h->rsrc_off) (void)hipFree(h->rsrc_off);
    if (h->rsrc_ent) (void)hipFree(h->rsrc_ent);
    if (h->rsrc_val) (void)hipFree(h->rsrc_val);
    h->fsrc_off = nullptr; h->fsrc_ent = nullptr; h->fsrc_val = nullptr;
    h->zsrc_off = nullptr; h->zsrc_ent = nullptr; h->zsrc_val = nullptr;
    h->rsrc_off = nullptr; h->rsrc_ent = nullptr; h->rsrc_val = nullptr;
    h->nrsrc = 0;
    if (h->bsrc_off) (void)hipFree(h->bsrc_off);
    if (h->bsrc_ent) (void)hipFree(h->bsrc_ent);
    if (h->bsrc_val) (void)hipFree(h->bsrc_val);
    h->bsrc_off = nullptr; h->bsrc_ent = nullptr; h->bsrc_val = nullptr;
    h->nbsrc = 0;
    h->nsrc = 0;
    h->nfsrc = 0;
    h->nzsrc = 0;
}

// Per-block source entries of the fused 3D tiling: every (plane offset,
// frame cell) of the block's z range z0-1 .. z0+lz (periodic images included)
// that carries a current; entry.x = plane offset * frame cells + frame cell.
static int build_fused3_source(lbem_s* h, const std::vector<double>& dense, int pp)
{
    const Geo& g = h->fgeo;
    const int TX = h->f3_tx, TY = h->f3_ty, LZ = h->f3_lz;
    const int W = TX + 2, HH = TY + 2, FC = W * HH;
    std::vector<int> off(g.nblocks + 1, 0);
    std::vector<int2> ent;
    std::vector<double> val;
    for (int b = 0; b < g.nblocks; ++b) {
        const int tx = b % g.tiles_x, r = b / g.tiles_x;
        const int ty = r % g.tiles_y, zc = r / g.tiles_y;
        const int x0 = tx * TX, y0 = ty * TY, z0 = zc * LZ;
        for (int po = 0; po < LZ + 2; ++po) {
            int gz = (z0 - 1 + po) % g.nz;
            if (gz < 0) gz += g.nz;
            for (int hy = 0; hy < HH; ++hy) {
                int gy = (y0 - 1 + hy) % g.ny;
                if (gy < 0) gy += g.ny;
                for (int hx = 0; hx < W; ++hx) {
                    int gx = (x0 - 1 + hx) % g.nx;
                    if (gx < 0) gx += g.nx;
                    const double v = dense[(size_t)gx + (size_t)g.nx * ((size_t)gy + (size_t)g.ny * gz)];
                    if (v != 0.0) {
                        ent.push_back(make_int2(po * FC + hy * W + hx, pp));
                        val.push_back(v);
                    }
                }
            }
        }
        off[b + 1] = (int)ent.size();
    }
    const size_t ms = ent.size(), tv = h->prec == LBEM_F64 ? 8 : 4;
    if (hipMalloc((void**)&h->fsrc_off, off.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&h->fsrc_ent, std::max<size_t>(ms, 1) * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&h->fsrc_val, std::max<size_t>(ms, 1) * tv) != hipSuccess)
        return LBEM_ENOMEM;
    hipError_t e = hipMemcpy(h->fsrc_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) e = hipMemcpy(h->fsrc_ent, ent.data(), ms * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) {
        if (tv == 8) {
            e = hipMemcpy(h->fsrc_val, val.data(), ms * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> f(val.begin(), val.end());
            e = hipMemcpy(h->fsrc_val, f.data(), ms * 4, hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) return LBEM_EDEVICE;
    h->nfsrc = (int64_t)ms;
    return LBEM_OK;
}

// Per-block source entries of the z-marching 3D tiling: local index
// (plane within the chunk) * NT + thread, pair, value.
static int build_zmarch_source(lbem_s* h, const std::vector<std::pair<int64_t, double>>& cells, int pp)
{
    const Geo& g = h->zgeo;
    struct Item { int b, local; float v; };
    std::vector<Item> items;
    items.reserve(cells.size());
    for (auto& e : cells) {
        const int c = (int)e.first;
        const int x = c % g.nx, y = (c / g.nx) % g.ny, z = c / (g.nx * g.ny);
        const int tx = x / TXD, ty = y / TYD, zc = z / h->zlz;
        const int b = (zc * g.tiles_y + ty) * g.tiles_x + tx;
        const int local = (z - zc * h->zlz) * NT + (y - ty * TYD) * TXD + (x - tx * TXD);
        items.push_back({b, local, (float)e.second});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b2) {
        return a.b != b2.b ? a.b < b2.b : a.local < b2.local;
    });
    std::vector<int> off(g.nblocks + 1, 0);
    for (auto& it : items) off[it.b + 1]++;
    for (int b = 0; b < g.nblocks; ++b) off[b + 1] += off[b];
    std::vector<int2> ent(items.size());
    std::vector<float> val(items.size());
    for (size_t k = 0; k < items.size(); ++k) {
        ent[k] = make_int2(items[k].local, pp);
        val[k] = items[k].v;
    }
    const size_t ms = items.size();
    if (hipMalloc((void**)&h->zsrc_off, off.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&h->zsrc_ent, std::max<size_t>(ms, 1) * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&h->zsrc_val, std::max<size_t>(ms, 1) * sizeof(float)) != hipSuccess)
        return LBEM_ENOMEM;
    hipError_t e = hipMemcpy(h->zsrc_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) e = hipMemcpy(h->zsrc_ent, ent.data(), ms * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) e = hipMemcpy(h->zsrc_val, val.data(), ms * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return LBEM_EDEVICE;
    h->nzsrc = (int64_t)ms;
    return LBEM_OK;
}

// Source entries of a whole-row tiling g: per (block, plane of its chunk) the
// cells (row * nx + x) that carry a current, with S per unit amplitude.
static int build_row_source(const RowGeo& g, const std::vector<std::pair<int64_t, double>>& cells, int pp,
                            int** off_out, int2** ent_out, float** val_out, int64_t* count)
{
    struct Item { int64_t key; int local; float v; };
    std::vector<Item> items;
    items.reserve(cells.size());
    for (auto& e : cells) {
        const int64_t c = e.first;
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((int64_t)g.nx * g.ny));
        const int tyi = y / g.ty, zc = z / g.lz;
        const int64_t b = (int64_t)zc * g.tiles_y + tyi;
        items.push_back({b * g.lz + (z - zc * g.lz), (y - tyi * g.ty) * g.nx + x, (float)e.second});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b2) { return a.key < b2.key; });
    const size_t nkeys = (size_t)g.nblocks * g.lz;
    std::vector<int> off(nkeys + 1, 0);
    for (auto& it : items) off[it.key + 1]++;
    for (size_t k = 0; k < nkeys; ++k) off[k + 1] += off[k];
    std::vector<int2> ent(items.size());
    std::vector<float> val(items.size());
    for (size_t k = 0; k < items.size(); ++k) {
        ent[k] = make_int2(items[k].local, pp);
        val[k] = items[k].v;
    }
    const size_t ms = items.size();
    if (hipMalloc((void**)off_out, off.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)ent_out, std::max<size_t>(ms, 1) * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)val_out, std::max<size_t>(ms, 1) * sizeof(float)) != hipSuccess)
        return LBEM_ENOMEM;
    hipError_t e = hipMemcpy(*off_out, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) e = hipMemcpy(*ent_out, ent.data(), ms * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) e = hipMemcpy(*val_out, val.data(), ms * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return LBEM_EDEVICE;
    *count = (int64_t)ms;
    return LBEM_OK;
}

// Source entries of the whole-row plain tiling: per block (tiles_y * z + row
// tile) the cells (row * nx + x) that carry a current, with S per unit amplitude.
static int build_xrow_source(lbem_s* h, const std::vector<std::pair<int64_t, double>>& cells, int pp)
{
    const XRowGeo& g = h->xgeo;
    struct Item { int b; int local; double v; };
    std::vector<Item> items;
    items.reserve(cells.size());
    for (auto& e : cells) {
        const int64_t c = e.first;
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((int64_t)g.nx * g.ny));
        const int yt = y / g.rows;
        items.push_back({z * g.tiles_y + yt, (y - yt * g.rows) * g.nx + x, e.second});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b2) { return a.b < b2.b; });
    std::vector<int> off((size_t)g.nblocks + 1, 0);
    for (auto& it : items) off[it.b + 1]++;
    for (int b = 0; b < g.nblocks; ++b) off[b + 1] += off[b];
    std::vector<int2> ent(items.size());
    for (size_t k = 0; k < items.size(); ++k) ent[k] = make_int2(items[k].local, pp);
    const size_t ms = items.size(), tv = h->prec == LBEM_F64 ? 8 : 4;
    if (hipMalloc((void**)&h->xsrc_off, off.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&h->xsrc_ent, std::max<size_t>(ms, 1) * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&h->xsrc_val, std::max<size_t>(ms, 1) * tv) != hipSuccess)
        return LBEM_ENOMEM;
    hipError_t e = hipMemcpy(h->xsrc_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) e = hipMemcpy(h->xsrc_ent, ent.data(), ms * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) {
        if (tv == 8) {
            std::vector<double> v(ms);
            for (size_t k = 0; k < ms; ++k) v[k] = items[k].v;
            e = hipMemcpy(h->xsrc_val, v.data(), ms * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> v(ms);
            for (size_t k = 0; k < ms; ++k) v[k] = (float)items[k].v;
            e = hipMemcpy(h->xsrc_val, v.data(), ms * 4, hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) return LBEM_EDEVICE;
    h->nxsrc = (int64_t)ms;
    return LBEM_OK;
}

// Per-tile source entries of the fused 2D tiling: every frame cell (tile plus
// halo, periodic images included) that carries a current.
static int build_fused_source(lbem_s* h, const std::vector<double>& dense)
{
    const Geo& g = h->fgeo;
    const int H = h->fuse_ns - 1, TY = h->fuse_ty;
    const int W = TXF + 2 * H, FH = TY + 2 * H;
    std::vector<int> off(g.nblocks + 1, 0);
    std::vector<int2> ent;
    std::vector<double> val;
    for (int b = 0; b < g.nblocks; ++b) {
        const int tx = b % g.tiles_x, ty = b / g.tiles_x;
        const int x0 = tx * TXF - H, y0 = ty * TY - H;
        for (int fy = 0; fy < FH; ++fy) {
            int gy = (y0 + fy) % g.ny;
            if (gy < 0) gy += g.ny;
            for (int fx = 0; fx < W; ++fx) {
                int gx = (x0 + fx) % g.nx;
                if (gx < 0) gx += g.nx;
                const double v = dense[(size_t)gx + (size_t)g.nx * gy];
                if (v != 0.0) {
                    ent.push_back(make_int2(fy * W + fx, 0));
                    val.push_back(v);
                }
            }
        }
        off[b + 1] = (int)ent.size();
    }
    const size_t ms = ent.size(), tv = h->prec == LBEM_F64 ? 8 : 4;
    if (hipMalloc((void**)&h->fsrc_off, off.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&h->fsrc_ent, std::max<size_t>(ms, 1) * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&h->fsrc_val, std::max<size_t>(ms, 1) * tv) != hipSuccess)
        return LBEM_ENOMEM;
    hipError_t e = hipMemcpy(h->fsrc_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) e = hipMemcpy(h->fsrc_ent, ent.data(), ms * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess && ms) {
        if (tv == 8) {
            e = hipMemcpy(h->fsrc_val, val.data(), ms * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> f(val.begin(), val.end());
            e = hipMemcpy(h->fsrc_val, f.data(), ms * 4, hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) return LBEM_EDEVICE;
    h->nfsrc = (int64_t)ms;
    return LBEM_OK;
}

int lbem_destroy(lbem_t h)
{
    if (!h) return LBEM_OK;
    API_SHARED;
    (void)follow_ticks(h);
    (void)hipStreamSynchronize(h->stream);
    free_source(h);
    if (h->keep) (void)hipFree(h->keep);
    if (h->ade) (void)hipFree(h->ade);
    if (h->pol) (void)hipFree(h->pol);
    if (h->ra) (void)hipFree(h->ra);
    // stream-ordered: returns the memory without waiting for the whole device
    if (h->partials) (void)hipFreeAsync(h->partials, h->stream);
    if (h->own_mem && h->arena) (void)hipFree(h->arena);
    if (h->sync_ev) (void)hipEventDestroy(h->sync_ev);
    if (h->tick_ev) (void)hipEventDestroy(h->tick_ev);
    delete h->impl;
    delete h;
    return LBEM_OK;
}

int lbem_set_medium(lbem_t h, const double* eps_r, const double* mu_r)
{
    if (!h || !eps_r) return LBEM_EINVAL;
    const int64_t n = h->n;
    bool nonunit_mu = false;
    if (mu_r)
        for (int64_t c = 0; c < n; ++c)
            if (mu_r[c] != 1.0) { nonunit_mu = true; break; }
    if (nonunit_mu && !h->cfg.mu_varies) return LBEM_EINVAL;
    API_SHARED;
    HIP_OK(follow_ticks(h));
    Staging s_eps, s_mu, s_flag;      // see stage_alloc
    int flag = 0, rc = LBEM_OK;
    if (!stage_alloc(s_eps, n * 8, h->stream) || (mu_r && !stage_alloc(s_mu, n * 8, h->stream)) ||
        !stage_alloc(s_flag, sizeof(int), h->stream)) {
        stage_free(s_eps, h->stream);
        stage_free(s_mu, h->stream);
        stage_free(s_flag, h->stream);
        return LBEM_ENOMEM;
    }
    double* deps = (double*)s_eps.p;
    double* dmu = (double*)s_mu.p;
    int* dflag = (int*)s_flag.p;
    hipError_t e = hipMemcpyAsync(deps, eps_r, n * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && mu_r) e = hipMemcpyAsync(dmu, mu_r, n * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(dflag, 0, sizeof(int), h->stream);
    h->mu_set = h->cfg.mu_varies != 0;
    h->ra_set = false;                 // a new medium is isotropic until lbem_set_anisotropy
    if (e == hipSuccess) e = h->impl->medium(h, deps, dmu, dflag);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = LBEM_EDEVICE;
    else if (flag) rc = LBEM_EUNSTABLE;
    stage_free(s_eps, h->stream);
    stage_free(s_mu, h->stream);
    stage_free(s_flag, h->stream);
    h->have_medium = rc == LBEM_OK;
    h->have_fields = false;
    return rc;
}

int lbem_init_fields(lbem_t h, const double* E, const double* B)
{
    if (!h || !E || !B) return LBEM_EINVAL;
    if (!h->have_medium) return LBEM_ESTATE;
    const int64_t n = h->n;
    for (int64_t k = 0; k < 3 * n; ++k)
        if (!std::isfinite(E[k]) || !std::isfinite(B[k])) return LBEM_EINVAL;
    if (h->D == 2) {
        for (int64_t c = 0; c < n; ++c)
            if (E[c] != 0.0 || E[n + c] != 0.0 || B[2 * n + c] != 0.0) return LBEM_EINVAL;
    }
    API_SHARED;
    HIP_OK(follow_ticks(h));
    Staging s_E, s_B;                 // see stage_alloc
    if (!stage_alloc(s_E, 3 * n * 8, h->stream) || !stage_alloc(s_B, 3 * n * 8, h->stream)) {
        stage_free(s_E, h->stream);
        stage_free(s_B, h->stream);
        return LBEM_ENOMEM;
    }
    double* dE = (double*)s_E.p;
    double* dB = (double*)s_B.p;
    hipError_t e = hipMemcpyAsync(dE, E, 3 * n * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dB, B, 3 * n * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = h->impl->init(h, dE, dB);
    if (e == hipSuccess && h->pol) e = hipMemsetAsync(h->pol, 0, pol_bytes(h), h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    stage_free(s_E, h->stream);
    stage_free(s_B, h->stream);
    if (e != hipSuccess) return LBEM_EDEVICE;
    h->t = 0;
    h->have_fields = true;
    return LBEM_OK;
}

int lbem_set_boundary(lbem_t h, int axis, int kind)
{
    if (!h || axis < 0 || axis >= h->D || kind < LBEM_BC_PERIODIC || kind > LBEM_BC_PMC) return LBEM_EINVAL;
    if (kind != LBEM_BC_PERIODIC && h->streaming != LBEM_STREAM_PULL) return LBEM_EINVAL;
    if (h->have_medium) return LBEM_ESTATE;
    h->bc_kind[axis] = kind;
    return LBEM_OK;
}

int lbem_set_anisotropy(lbem_t h, const double* fac)
{
    if (!h || !fac) return LBEM_EINVAL;
    if (h->prec > LBEM_F32 || h->streaming != LBEM_STREAM_PULL) return LBEM_EINVAL;
    if (!h->have_medium) return LBEM_ESTATE;
    API_SHARED;
    HIP_OK(follow_ticks(h));
    const int64_t n = h->n;
    const size_t tm = h->prec == LBEM_F64 ? 8 : 4;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBEM_EDEVICE;
    if (!h->ra && hipMalloc(&h->ra, (size_t)h->D * n * tm) != hipSuccess) {
        h->ra = nullptr;
        return LBEM_ENOMEM;
    }
    double* dfac = nullptr;
    int* dflag = nullptr;
    if (hipMalloc((void**)&dfac, (size_t)h->D * n * 8) != hipSuccess) return LBEM_ENOMEM;
    if (hipMalloc((void**)&dflag, sizeof(int)) != hipSuccess) { (void)hipFree(dfac); return LBEM_ENOMEM; }
    int flag = 0, rc = LBEM_OK;
    hipError_t e = hipMemcpyAsync(dfac, fac, (size_t)h->D * n * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(dflag, 0, sizeof(int), h->stream);
    if (e == hipSuccess) e = tm == 8 ? launch_aniso<double>(h, dfac, dflag, 0) : launch_aniso<float>(h, dfac, dflag, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess && !flag) {
        e = tm == 8 ? launch_aniso<double>(h, dfac, dflag, 1) : launch_aniso<float>(h, dfac, dflag, 1);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (e != hipSuccess) rc = LBEM_EDEVICE;
    else if (flag) rc = LBEM_EUNSTABLE;
    (void)hipFree(dfac);
    (void)hipFree(dflag);
    if (rc == LBEM_OK) {
        h->ra_set = true;
        h->have_fields = false;        // the populations must be re-initialised for the new weights
    }
    return rc;
}

int lbem_set_dispersion(lbem_t h, const double* wp2, const double* w02, const double* gamma)
{
    if (!h) return LBEM_EINVAL;
    API_SHARED;
    HIP_OK(follow_ticks(h));
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBEM_EDEVICE;
    if (!wp2) {
        if (h->ade) (void)hipFree(h->ade);
        if (h->pol) (void)hipFree(h->pol);
        h->ade = h->pol = nullptr;
        return LBEM_OK;
    }
    if (h->streaming != LBEM_STREAM_PULL) return LBEM_EINVAL;
    const int64_t n = h->n;
    for (int64_t c = 0; c < n; ++c) {
        const double a = wp2[c], b = w02 ? w02[c] : 0.0, g = gamma ? gamma[c] : 0.0;
        if (!(a >= 0.0) || !(b >= 0.0) || !(g >= 0.0) || !std::isfinite(a) || !std::isfinite(b) ||
            !std::isfinite(g))
            return LBEM_EINVAL;
    }
    const bool f64 = h->prec == LBEM_F64;
    const size_t tm = f64 ? 8 : 4;
    std::vector<char> host((size_t)3 * n * tm);
    for (int64_t c = 0; c < n; ++c) {
        const double g = gamma ? gamma[c] : 0.0, den = 1.0 + 0.5 * g;
        const double co[3] = {(1.0 - 0.5 * g) / den, wp2[c] / den, (w02 ? w02[c] : 0.0) / den};
        for (int k = 0; k < 3; ++k) {
            if (f64) ((double*)host.data())[k * n + c] = co[k];
            else ((float*)host.data())[k * n + c] = (float)co[k];
        }
    }
    const size_t pb = (size_t)2 * h->P * n * tm;
    if (!h->ade) {
        if (hipMalloc(&h->ade, (size_t)3 * n * tm) != hipSuccess) { h->ade = nullptr; return LBEM_ENOMEM; }
        if (hipMalloc(&h->pol, pb) != hipSuccess) {
            (void)hipFree(h->ade);
            h->ade = h->pol = nullptr;
            return LBEM_ENOMEM;
        }
    }
    if (hipMemcpyAsync(h->ade, host.data(), (size_t)3 * n * tm, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemsetAsync(h->pol, 0, pb, h->stream) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
        return LBEM_EDEVICE;
    return LBEM_OK;
}

int lbem_set_absorber(lbem_t h, const double* sigma)
{
    if (!h) return LBEM_EINVAL;
    API_SHARED;
    HIP_OK(follow_ticks(h));
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBEM_EDEVICE;
    if (!sigma) {
        if (h->keep) (void)hipFree(h->keep);
        h->keep = nullptr;
        return LBEM_OK;
    }
    if (h->streaming != LBEM_STREAM_PULL) return LBEM_EINVAL;
    const int64_t n = h->n;
    for (int64_t c = 0; c < n; ++c)
        if (!(sigma[c] >= 0.0 && sigma[c] < 1.0)) return LBEM_EINVAL;
    const bool f64 = h->prec == LBEM_F64;
    const size_t tm = f64 ? 8 : 4;
    std::vector<char> host((size_t)n * tm);
    for (int64_t c = 0; c < n; ++c) {
        const double k = 1.0 - sigma[c];
        if (f64) ((double*)host.data())[c] = k;
        else ((float*)host.data())[c] = (float)k;
    }
    if (!h->keep && hipMalloc(&h->keep, (size_t)n * tm) != hipSuccess) {
        h->keep = nullptr;
        return LBEM_ENOMEM;
    }
    if (hipMemcpyAsync(h->keep, host.data(), (size_t)n * tm, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return LBEM_EDEVICE;
    return LBEM_OK;
}

int lbem_set_source(lbem_t h, int comp, const int64_t* cells, const double* weight, int64_t m)
{
    if (!h || m < 0 || comp < 0 || comp > 2) return LBEM_EINVAL;
    if (h->D == 2 && comp != 2) return LBEM_EINVAL;
    if (m > 0 && (!cells || !weight)) return LBEM_EINVAL;
    if (!h->have_medium) return LBEM_ESTATE;
    API_SHARED;
    HIP_OK(follow_ticks(h));
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBEM_EDEVICE;
    free_source(h);
    if (m == 0) return LBEM_OK;
    const int64_t n = h->n;
    const int D = h->D;
    // pair carrying component comp and its Levi-Civita sign
    int pp = -1, sg = 0;
    for (int p = 0; p < h->P; ++p)
        if (pair_g(D, p) == comp) { pp = p; sg = pair_s(D, p); }
    // eps_abs = eps_r/c_vac^2 = (D-1)/(mu_r c_L^2): read back c_L^2 and mu_r
    std::vector<double> cl2(n), mu(n, 1.0);
    if (h->prec == LBEM_F64) {
        if (hipMemcpy(cl2.data(), h->cl2, n * 8, hipMemcpyDeviceToHost) != hipSuccess) return LBEM_EDEVICE;
    } else {
        std::vector<float> f(n);
        if (hipMemcpy(f.data(), h->cl2, n * 4, hipMemcpyDeviceToHost) != hipSuccess) return LBEM_EDEVICE;
        for (int64_t c = 0; c < n; ++c) cl2[c] = f[c];
    }
    if (h->mu_set && hipMemcpy(mu.data(), h->mu_r, n * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return LBEM_EDEVICE;
    // merge repeated cells, then bucket by tile
    std::vector<std::pair<int64_t, double>> ent;
    ent.reserve(m);
    for (int64_t k = 0; k < m; ++k) {
        if (cells[k] < 0 || cells[k] >= n || !std::isfinite(weight[k])) return LBEM_EINVAL;
        ent.push_back({cells[k], weight[k]});
    }
    std::sort(ent.begin(), ent.end(), [](auto& a, auto& b) { return a.first < b.first; });
    std::vector<std::pair<int64_t, double>> merged;
    for (auto& e : ent) {
        if (!merged.empty() && merged.back().first == e.first) merged.back().second += e.second;
        else merged.push_back(e);
    }
    const Geo& g = h->geo;
    const int bx = 1 << g.bx_shift, rb = NT / bx;
    struct Item { int b; int local; double v; };
    std::vector<Item> items;
    std::vector<double> src_value;
    items.reserve(merged.size());
    src_value.reserve(merged.size());
    for (auto& e : merged) {
        const int c = (int)e.first;
        const int x = c % g.nx, y = (c / g.nx) % g.ny, z = c / (g.nx * g.ny);
        const int tx = x / bx, ty = y / (rb * h->vec);
        const int b = tile_id(g, tx, ty, z);
        const int yr = y - ty * rb * h->vec;
        const int v = yr / rb, tyi = yr % rb;
        const int local = v * NT + tyi * bx + (x - tx * bx);
        // S per unit amplitude on pair pp: sgn * (-weight/eps_abs)
        const double eps_abs = (double)(D - 1) / (mu[c] * cl2[c]);
        items.push_back({b, local, -(double)sg * e.second / eps_abs});
        src_value.push_back(items.back().v);
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.b < b.b; });
    std::vector<int> off(g.nblocks + 1, 0);
    for (auto& it : items) off[it.b + 1]++;
    for (int b = 0; b < g.nblocks; ++b) off[b + 1] += off[b];
    std::vector<int2> ents(items.size());
    for (size_t k = 0; k < items.size(); ++k) ents[k] = make_int2(items[k].local, pp);
    const size_t ms = items.size();
    const size_t tv = h->prec == LBEM_F64 ? 8 : 4;
    if (hipMalloc((void**)&h->src_off, off.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&h->src_ent, ms * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&h->src_val, ms * tv) != hipSuccess) {
        free_source(h);
        return LBEM_ENOMEM;
    }
    hipError_t e = hipMemcpy(h->src_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->src_ent, ents.data(), ms * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        if (tv == 8) {
            std::vector<double> v(ms);
            for (size_t k = 0; k < ms; ++k) v[k] = items[k].v;
            e = hipMemcpy(h->src_val, v.data(), ms * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> v(ms);
            for (size_t k = 0; k < ms; ++k) v[k] = (float)items[k].v;
            e = hipMemcpy(h->src_val, v.data(), ms * 4, hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) { free_source(h); return LBEM_EDEVICE; }
    h->nsrc = (int64_t)ms;
    if (h->zmarch || h->brow) {
        std::vector<std::pair<int64_t, double>> cv(merged.size());
        for (size_t k = 0; k < merged.size(); ++k) cv[k] = {merged[k].first, src_value[k]};
        int rc = h->zmarch ? build_zmarch_source(h, cv, pp) : LBEM_OK;
        if (rc == LBEM_OK && h->zmarch && h->rowk)
            rc = build_row_source(h->rgeo, cv, pp, &h->rsrc_off, &h->rsrc_ent, &h->rsrc_val, &h->nrsrc);
        if (rc == LBEM_OK && h->brow)
            rc = build_row_source(h->bgeo, cv, pp, &h->bsrc_off, &h->bsrc_ent, &h->bsrc_val, &h->nbsrc);
        if (rc != LBEM_OK) { free_source(h); return rc; }
    }
    if (h->xrow) {
        std::vector<std::pair<int64_t, double>> cv(merged.size());
        for (size_t k = 0; k < merged.size(); ++k) cv[k] = {merged[k].first, src_value[k]};
        const int rc = build_xrow_source(h, cv, pp);
        if (rc != LBEM_OK) { free_source(h); return rc; }
    }
    if (fused_format(h) && h->fuse_ns > 1) {
        std::vector<double> dense((size_t)n, 0.0);
        for (size_t k = 0; k < merged.size(); ++k) dense[(size_t)merged[k].first] = src_value[k];
        const int rc = D == 2 ? build_fused_source(h, dense) : build_fused3_source(h, dense, pp);
        if (rc != LBEM_OK) { free_source(h); return rc; }
    }
    return LBEM_OK;
}

int lbem_step(lbem_t h, int64_t nsteps, const double* amp)
{
    if (!h || nsteps < 0) return LBEM_EINVAL;
    if (!h->have_fields) return LBEM_ESTATE;
    HIP_OK(follow_ticks(h));
    const bool fuse = fused_ok(h);
    int64_t k = 0;
    while (k < nsteps) {
        if (fuse && h->layout == LAYOUT_PULL_PENDING && nsteps - k >= h->fuse_ns) {
            if (h->impl->step_fused(h, (amp && h->nsrc) ? amp + k : nullptr) != hipSuccess) return LBEM_EDEVICE;
            k += h->fuse_ns;
            h->t += h->fuse_ns;
            continue;
        }
        const double a = (amp && h->nsrc) ? amp[k] : 0.0;
        if (h->impl->step(h, a) != hipSuccess) return LBEM_EDEVICE;
        h->t += 1;
        ++k;
    }
    return LBEM_OK;
}

int lbem_moments(lbem_t h, double* E, double* B, int on_device)
{
    if (!h) return LBEM_EINVAL;
    if (!h->have_fields) return LBEM_ESTATE;
    HIP_OK(follow_ticks(h));
    const size_t bytes = (size_t)3 * h->n * 8;
    if (on_device) {
        if (h->impl->fields(h, E, B, nullptr) != hipSuccess) return LBEM_EDEVICE;
        return hipStreamSynchronize(h->stream) == hipSuccess ? LBEM_OK : LBEM_EDEVICE;
    }
    if (E) {
        HIP_OK(h->impl->fields(h, h->scratch, nullptr, nullptr));
        HIP_OK(hipMemcpyAsync(E, h->scratch, bytes, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));
    }
    if (B) {
        HIP_OK(h->impl->fields(h, nullptr, h->scratch, nullptr));
        HIP_OK(hipMemcpyAsync(B, h->scratch, bytes, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));
    }
    return LBEM_OK;
}

int lbem_energy(lbem_t h, double out[4])
{
    if (!h || !out) return LBEM_EINVAL;
    if (!h->have_fields) return LBEM_ESTATE;
    HIP_OK(follow_ticks(h));
    double* res = h->partials + (size_t)h->nb_diag * 4;
    HIP_OK(h->impl->fields(h, nullptr, h->scratch, h->partials));
    Geo1 g = geo1(h);
    if (h->D == 2)
        hipLaunchKernelGGL((k_divb<2>), dim3(h->nb_diag), dim3(NT), 0, h->stream, h->scratch, g, h->partials);
    else
        hipLaunchKernelGGL((k_divb<3>), dim3(h->nb_diag), dim3(NT), 0, h->stream, h->scratch, g, h->partials);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(NT), 0, h->stream, h->partials, h->nb_diag, res);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(out[k])) return LBEM_ENONFINITE;
    return LBEM_OK;
}

// lbem_energy with its scratch in the static device array: no allocation.
int lbem_energy_noalloc(lbem_t h, double out[4])
{
    if (!h || !out) return LBEM_EINVAL;
    if (!h->have_fields) return LBEM_ESTATE;
    if (h->n > LBEM_NOALLOC_MAX_CELLS) return LBEM_ETOOBIG;
    double* base = nullptr;
    HIP_OK(noalloc_address(h->device, &base));
    HIP_OK(follow_ticks(h));
    double* bfield = base;                          // [3][n]
    double* partials = base + (size_t)3 * h->n;     // [nb_diag][4], then the 4 results
    double* res = partials + (size_t)h->nb_diag * 4;
    HIP_OK(h->impl->fields(h, nullptr, bfield, partials));
    Geo1 g = geo1(h);
    if (h->D == 2)
        hipLaunchKernelGGL((k_divb<2>), dim3(h->nb_diag), dim3(NT), 0, h->stream, bfield, g, partials);
    else
        hipLaunchKernelGGL((k_divb<3>), dim3(h->nb_diag), dim3(NT), 0, h->stream, bfield, g, partials);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(NT), 0, h->stream, partials, h->nb_diag, res);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(out[k])) return LBEM_ENONFINITE;
    return LBEM_OK;
}

int64_t lbem_time(lbem_t h) { return h ? h->t : -1; }

int lbem_steps_per_launch(lbem_t h)
{
    if (!h) return LBEM_EINVAL;
    return fused_ok(h) ? h->fuse_ns : 1;
}

namespace {
constexpr size_t STATE_HDR = 128;
struct StateHeader {
    char magic[8];
    int32_t dim, prec, streaming, layout;
    int64_t nx, ny, nz, t;
    uint64_t payload;
    uint64_t aux;      // auxiliary dispersion fields after the populations (0 if none)
};
static_assert(sizeof(StateHeader) <= STATE_HDR, "state header");
const char STATE_MAGIC[8] = {'L', 'B', 'E', 'M', 'S', 'T', '0', '1'};
}  // namespace

size_t lbem_state_bytes(lbem_t h)
{
    if (!h) return 0;
    return STATE_HDR + sizes_of(&h->cfg).pop_one + pol_bytes(h);
}

int lbem_get_state(lbem_t h, void* buf, size_t bytes, int on_device)
{
    if (!h || !buf || bytes < lbem_state_bytes(h)) return LBEM_EINVAL;
    if (!h->have_fields) return LBEM_ESTATE;
    HIP_OK(follow_ticks(h));
    char hdr[STATE_HDR] = {0};
    StateHeader sh{};
    std::memcpy(sh.magic, STATE_MAGIC, 8);
    sh.dim = h->D;
    sh.prec = h->prec;
    sh.streaming = h->streaming;
    sh.layout = h->layout;
    sh.nx = h->cfg.nx;
    sh.ny = h->cfg.ny;
    sh.nz = h->cfg.nz;
    sh.t = h->t;
    sh.payload = sizes_of(&h->cfg).pop_one;
    sh.aux = pol_bytes(h);
    std::memcpy(hdr, &sh, sizeof(sh));
    char* out = (char*)buf;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (on_device) {
        HIP_OK(hipMemcpyAsync(out, hdr, STATE_HDR, hipMemcpyHostToDevice, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));  // hdr is on this stack frame
    } else {
        std::memcpy(out, hdr, STATE_HDR);
    }
    HIP_OK(hipMemcpyAsync(out + STATE_HDR, h->pop[h->cur], sh.payload, k, h->stream));
    if (sh.aux) HIP_OK(hipMemcpyAsync(out + STATE_HDR + sh.payload, h->pol, sh.aux, k, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return LBEM_OK;
}

int lbem_set_state(lbem_t h, const void* buf, size_t bytes, int on_device)
{
    if (!h || !buf || bytes < lbem_state_bytes(h)) return LBEM_EINVAL;
    if (!h->have_medium) return LBEM_ESTATE;
    HIP_OK(follow_ticks(h));
    const char* in = (const char*)buf;
    StateHeader sh{};
    if (on_device) {
        HIP_OK(hipMemcpyAsync(&sh, in, sizeof(sh), hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));
    } else {
        std::memcpy(&sh, in, sizeof(sh));
    }
    const size_t pay = sizes_of(&h->cfg).pop_one;
    if (std::memcmp(sh.magic, STATE_MAGIC, 8) != 0 || sh.dim != h->D || sh.prec != h->prec ||
        sh.streaming != h->streaming || sh.nx != h->cfg.nx || sh.ny != h->cfg.ny || sh.nz != h->cfg.nz ||
        sh.payload != pay || sh.aux != pol_bytes(h) || sh.t < 0 || sh.layout < LAYOUT_NATURAL ||
        sh.layout > LAYOUT_AA_SWAPPED)
        return LBEM_EINVAL;
    // pull steps never leave the AA layout, AA steps never the pull one
    if ((h->streaming == LBEM_STREAM_PULL && sh.layout == LAYOUT_AA_SWAPPED) ||
        (h->streaming == LBEM_STREAM_AA && sh.layout == LAYOUT_PULL_PENDING))
        return LBEM_EINVAL;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_OK(hipMemcpyAsync(h->pop[0], in + STATE_HDR, pay, k, h->stream));
    if (sh.aux) HIP_OK(hipMemcpyAsync(h->pol, in + STATE_HDR + pay, sh.aux, k, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    h->cur = 0;
    h->layout = sh.layout;
    h->t = sh.t;
    h->have_fields = true;
    return LBEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched stepping of many resident lattices (serving)
// ---------------------------------------------------------------------------
namespace {
constexpr int NPREC = 7;   // LBEM_F64 .. LBEM_F16
constexpr int NCLASS = 2 * NPREC;  // (dim - 2) * NPREC + prec
constexpr int BATCH_BLOCKS = 8192;  // persistent grid (more blocks than fit: the rest start as others finish)
// How a class's steps after the first of a tick run: the per-cell kernel, or
// (3D deviation classes whose members all have the whole-row tiling) the
// row-tile kernel with mu == 1 or with varying mu
constexpr int NMODE = 3;
enum { MODE_CELL = 0, MODE_ROWS = 1, MODE_ROWS_MU = 2 };

int class_of(const lbem_s* h) { return (h->D - 2) * NPREC + h->prec; }

size_t class_bytes(int max_grids) { return align256(sizeof(BatchHdr)) + align256(sizeof(BatchGrid) * (size_t)max_grids); }
}  // namespace

constexpr int NRING = 8;      // pinned staging slots of the table uploads

struct lbem_batch_s {
    hipStream_t stream;
    int max_grids, ksteps;
    char* dev;                 // NCLASS x (header, table), then the amplitudes [max_grids][ksteps] (8 B each)
    size_t amp_off;            // offset of the amplitudes
    char* pinned[NRING];
    hipEvent_t ev[NRING];      // each slot is free again once its upload has executed
    int ring;
    size_t group_bytes;        // members of one call run in groups touching at most this much state per step
    // per class and mode one graph of ksteps launches, captured and
    // instantiated once, in lbem_batch_create (the row modes of the 3D
    // deviation classes only)
    hipGraph_t graph[NCLASS][NMODE];
    hipGraphExec_t exec[NCLASS][NMODE];
    int use_graph;
    int blocks;                // persistent grid of each class launch
    int rows_min;              // fewest whole-row work items for the row modes
    // the classes of a tick run concurrently, one stream each (default
    // priority), forked from the batch stream after the table upload and
    // joined back before anything later on it
    hipStream_t cstream[NCLASS];
    hipEvent_t fork_ev, join_ev[NCLASS];
    int concurrent;
};

// the first step of a tick always takes the per-cell kernel: it reads
// members that start from the natural layout
template <int D, typename H, bool GH>
static void launch_batch_dev(dim3 g, dim3 t, hipStream_t st, const BatchHdr* hdr, const BatchGrid* tab, int k,
                             int mode)
{
    if constexpr (D == 3) {
        if (k > 0 && mode == MODE_ROWS) {
            hipLaunchKernelGGL((k_step_batch_dev3_rows<H, GH, false>), g, dim3(BROW_NT), 0, st, hdr, tab, k);
            return;
        }
        if (k > 0 && mode == MODE_ROWS_MU) {
            hipLaunchKernelGGL((k_step_batch_dev3_rows<H, GH, true>), g, dim3(BROW_NT), 0, st, hdr, tab, k);
            return;
        }
    }
    hipLaunchKernelGGL((k_step_batch_dev<D, H, GH>), g, t, 0, st, hdr, tab, k);
}

template <int D>
static void launch_class_d(lbem_batch_s* b, int prec, const BatchHdr* hdr, const BatchGrid* tab, int k,
                           hipStream_t st, int mode)
{
    dim3 g(b->blocks), t(NT);
    switch (prec) {
        case LBEM_F64: hipLaunchKernelGGL((k_step_batch_plain<D, double>), g, t, 0, st, hdr, tab, k); break;
        case LBEM_F32: hipLaunchKernelGGL((k_step_batch_plain<D, float>), g, t, 0, st, hdr, tab, k); break;
        case LBEM_F16DEV: launch_batch_dev<D, __half, false>(g, t, st, hdr, tab, k, mode); break;
        case LBEM_BF16DEV: launch_batch_dev<D, __hip_bfloat16, false>(g, t, st, hdr, tab, k, mode); break;
        case LBEM_F16GHOST: launch_batch_dev<D, __half, true>(g, t, st, hdr, tab, k, mode); break;
        case LBEM_BF16GHOST: launch_batch_dev<D, __hip_bfloat16, true>(g, t, st, hdr, tab, k, mode); break;
        default:
            hipLaunchKernelGGL((k_step_batch_plain<D, float, __half>), g, t, 0, st, hdr, tab, k);
            break;
    }
}

static void launch_class(lbem_batch_s* b, int c, int k, hipStream_t st, int mode)
{
    const size_t cb = class_bytes(b->max_grids);
    const BatchHdr* hdr = (const BatchHdr*)(b->dev + c * cb);
    const BatchGrid* tab = (const BatchGrid*)(b->dev + c * cb + align256(sizeof(BatchHdr)));
    if (c < NPREC) launch_class_d<2>(b, c, hdr, tab, k, st, mode);
    else launch_class_d<3>(b, c - NPREC, hdr, tab, k, st, mode);
}

// classes that have the row modes: 3D deviation formats
static bool has_row_modes(int c) { return c >= NPREC && is_dev(c - NPREC); }

// Capture the per-class graphs.  Done once, at creation, with the library
// lock held exclusively: no graph is ever captured or instantiated while
// other threads allocate, free or launch through this library.
static bool capture_classes(lbem_batch_s* b)
{
    std::unique_lock<std::shared_mutex> lk(g_api_mu);
    for (int c = 0; c < NCLASS; ++c) {
        for (int mode = 0; mode < (has_row_modes(c) ? NMODE : 1); ++mode) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (int k = 0; k < b->ksteps; ++k) launch_class(b, c, k, b->stream, mode);
                e = hipStreamEndCapture(b->stream, &graph);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                return false;
            }
            b->graph[c][mode] = graph;
            b->exec[c][mode] = exec;
        }
    }
    return true;
}

static hipError_t enqueue_tick(lbem_batch_s* b, unsigned mask, const int* mode)
{
    const bool conc = b->concurrent && (mask & (mask - 1)) != 0;   // two classes or more
    hipError_t e = hipSuccess;
    if (conc && (e = hipEventRecord(b->fork_ev, b->stream)) != hipSuccess) return e;
    for (int c = 0; c < NCLASS; ++c) {
        if (!(mask & (1u << c))) continue;
        hipStream_t st = b->stream;
        if (conc) {
            st = b->cstream[c];
            if ((e = hipStreamWaitEvent(st, b->fork_ev, 0)) != hipSuccess) return e;
        }
        if (b->use_graph) {
            if ((e = hipGraphLaunch(b->exec[c][mode[c]], st)) != hipSuccess) return e;
        } else {
            for (int k = 0; k < b->ksteps; ++k) launch_class(b, c, k, st, mode[c]);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (conc) {
            if ((e = hipEventRecord(b->join_ev[c], st)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(b->stream, b->join_ev[c], 0)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

static void release_graphs(lbem_batch_s* b)
{
    for (int c = 0; c < NCLASS; ++c)
        for (int mode = 0; mode < NMODE; ++mode) {
            if (b->exec[c][mode]) (void)hipGraphExecDestroy(b->exec[c][mode]);
            if (b->graph[c][mode]) (void)hipGraphDestroy(b->graph[c][mode]);
            b->exec[c][mode] = nullptr;
            b->graph[c][mode] = nullptr;
        }
}

// State bytes one step of a member reads or writes: its population copies
// (one in place, two with pull), c_L^2 and the mu gradient.
static size_t touched_bytes(const lbem_s* h)
{
    const Sizes z = sizes_of(&h->cfg);
    return z.pop_one * (h->streaming == LBEM_STREAM_AA ? 1 : 2) + z.medium + (h->mu_set ? z.mu : 0);
}

// One group of a tick: its descriptor table through the next staging slot,
// the ordering against the members' own streams, and the classes' graphs.
static int enqueue_group(lbem_batch_s* b, const lbem_t* handles, const int64_t* nsteps, const double* amp,
                         const int* idx, int m)
{
    // the staging slot is free once its previous upload has executed
    if (hipEventSynchronize(b->ev[b->ring]) != hipSuccess) return LBEM_EDEVICE;
    char* host = b->pinned[b->ring];
    const size_t cb = class_bytes(b->max_grids);
    int cnt[NCLASS] = {0}, tiles[NCLASS] = {0}, rows[NCLASS] = {0};
    int nrow[NCLASS] = {0}, nmu[NCLASS] = {0};
    unsigned mask = 0;
    size_t amp_used = 0;      // end of the amplitudes written for this group
    for (int q = 0; q < m; ++q) {
        const int i = idx[q];
        lbem_s* h = handles[i];
        const int c = class_of(h);
        BatchGrid* tab = (BatchGrid*)(host + c * cb + align256(sizeof(BatchHdr)));
        BatchGrid& G = tab[cnt[c]++];
        std::memset(&G, 0, sizeof(G));
        if (h->prec <= LBEM_F32 || h->prec == LBEM_F16) {     // plain populations (FP16 storage included)
            const bool aa = h->streaming == LBEM_STREAM_AA;
            G.buf[0] = h->pop[0];
            G.buf[1] = aa ? h->pop[0] : h->pop[1];
            G.aa = aa;
        } else {
            const size_t moff = align256((size_t)(h->P + h->D) * h->n * 4);
            G.buf[0] = h->pop[0];
            G.buf[1] = h->pop[1];
            G.dev[0] = h->pop[0] + moff;
            G.dev[1] = h->pop[1] + moff;
            if (h->brow) {
                G.row = 1;
                G.row_base = rows[c];
                rows[c] += h->bgeo.nblocks;
                nrow[c]++;
                G.rgeo = h->bgeo;
                if (h->nbsrc) {
                    G.rsrc_off = h->bsrc_off;
                    G.rsrc_ent = h->bsrc_ent;
                    G.rsrc_val = h->bsrc_val;
                }
            }
        }
        G.cl2 = h->cl2;
        G.dlnmu = h->mu_set ? h->dlnmu : nullptr;
        nmu[c] += h->mu_set ? 1 : 0;
        // the member's own tiling, so that its per-tile source table applies
        Geo& g = G.geo;
        g = h->geo;
        g.xcd = 0;
        if (h->nsrc) {
            G.src_off = h->src_off;
            G.src_ent = h->src_ent;
            G.src_val = h->src_val;
            if (amp) {
                // this member's amplitudes, in the class's arithmetic type
                char* slot = host + b->amp_off + (size_t)i * b->ksteps * 8;
                const size_t dslot = b->amp_off + (size_t)i * b->ksteps * 8;
                for (int64_t j = 0; j < nsteps[i]; ++j) {
                    const double a = amp[(size_t)i * b->ksteps + j];
                    if (h->prec == LBEM_F64) ((double*)slot)[j] = a;
                    else ((float*)slot)[j] = (float)a;
                }
                G.amp = b->dev + dslot;
                amp_used = std::max(amp_used, dslot + (size_t)b->ksteps * 8);
            }
        }
        G.omega = 1.0 / h->cfg.tau;
        G.tau_half = h->cfg.tau == 0.5;
        G.cur0 = h->cur;
        G.fresh = h->layout == LAYOUT_NATURAL;
        G.nsteps = (int)nsteps[i];
        G.tile_base = tiles[c];
        tiles[c] += g.nblocks;
        mask |= 1u << c;
    }
    int mode[NCLASS];
    for (int c = 0; c < NCLASS; ++c) {
        BatchHdr* hd = (BatchHdr*)(host + c * cb);
        hd->count = cnt[c];
        hd->total_tiles = tiles[c];
        hd->total_rows = rows[c];
        mode[c] = MODE_CELL;
        if (has_row_modes(c) && cnt[c] > 0 && nrow[c] == cnt[c] && rows[c] >= b->rows_min) {
            if (nmu[c] == 0) mode[c] = MODE_ROWS;
            else if (nmu[c] == cnt[c]) mode[c] = MODE_ROWS_MU;
        }
    }
    // members set up on other streams: their work so far precedes the group
    for (int q = 0; q < m; ++q) {
        lbem_s* h = handles[idx[q]];
        if (h->stream == b->stream) continue;
        if (hipEventRecord(h->sync_ev, h->stream) != hipSuccess ||
            hipStreamWaitEvent(b->stream, h->sync_ev, 0) != hipSuccess)
            return LBEM_EDEVICE;
    }
    if (hipMemcpyAsync(b->dev, host, amp_used ? amp_used : cb * NCLASS, hipMemcpyHostToDevice, b->stream) !=
        hipSuccess)
        return LBEM_EDEVICE;
    if (hipEventRecord(b->ev[b->ring], b->stream) != hipSuccess) return LBEM_EDEVICE;
    b->ring = (b->ring + 1) % NRING;
    if (mask && enqueue_tick(b, mask, mode) != hipSuccess) return LBEM_EDEVICE;
    // ... and later work on a member's own stream (moments, destroy) follows
    // it: the member's stream waits on this event at its next use (follow_ticks)
    for (int q = 0; q < m; ++q) {
        lbem_s* h = handles[idx[q]];
        if (h->stream == b->stream) continue;
        if (hipEventRecord(h->tick_ev, b->stream) != hipSuccess) return LBEM_EDEVICE;
        h->tick_pending = true;
    }
    return LBEM_OK;
}

extern "C" {

int lbem_batch_create(int max_lattices, int steps_per_tick, void* stream, lbem_batch_t* out)
{
    if (!out || max_lattices < 1 || max_lattices > 65536 || steps_per_tick < 1 || steps_per_tick > 4096)
        return LBEM_EINVAL;
    *out = nullptr;
    if (!stream) return LBEM_EINVAL;  // a capturable stream is required
    lbem_batch_s* b = new (std::nothrow) lbem_batch_s();
    if (!b) return LBEM_ENOMEM;
    b->stream = (hipStream_t)stream;
    b->max_grids = max_lattices;
    b->ksteps = steps_per_tick;
    b->ring = 0;
    b->use_graph = env_int("LBEM_BATCH_GRAPH", 1);
    b->blocks = std::max(1, env_int("LBEM_BATCH_BLOCKS", BATCH_BLOCKS));
    // A row work item is a chunk of planes of a whole-row tile: 8-16 times a
    // per-cell tile.  Measured (FP16-dev): 20 lattices of 128^3 (10240 items)
    // 35.2k MLUPS with row tiles against 29.9k per-cell; 20 of 64^3 (1280
    // items) 27.0k against 33.0k; the serving mix at 200 req/s, whose 3D
    // classes hold a few small lattices, 37.2 against 38.6 GLUPS with the row
    // tiles always on (100 req/s: p50 141 against 62 ms).  So a class takes
    // them only with enough items to fill the GPU several times over.
    b->rows_min = std::max(0, env_int("LBEM_BATCH_ROWS_MIN", 1536));
    b->amp_off = class_bytes(max_lattices) * NCLASS;
    const size_t bytes = b->amp_off + align256((size_t)max_lattices * steps_per_tick * 8);
    b->dev = nullptr;
    for (int r = 0; r < NRING; ++r) {
        b->pinned[r] = nullptr;
        b->ev[r] = nullptr;
    }
    // Lattices small enough for the 256 MB Infinity Cache are served from it
    // when several steps run on them back to back: with a budget, a tick runs
    // the members of each 3D class in groups whose state a step touches fits
    // it, each group for all of its steps, instead of every member once per
    // step.  Measured on the serving mix at 200 req/s: 38.7 GLUPS without
    // groups; 41.8, 43.4, 44.3-44.4, 44.0, 41.6 and 38.8 with 96, 160, 224,
    // 256, 320 and 640 MiB (100 req/s at 224 MiB: p50 68 ms, p99 0.37 s).
    // Groups that mixed classes (each group replaying every class's graph)
    // had measured 37.9.  LBEM_BATCH_GROUP_MIB=0 turns grouping off.
    b->group_bytes = (size_t)std::max(0, env_int("LBEM_BATCH_GROUP_MIB", 224)) << 20;
    for (int c = 0; c < NCLASS; ++c) {
        for (int mode = 0; mode < NMODE; ++mode) {
            b->graph[c][mode] = nullptr;
            b->exec[c][mode] = nullptr;
        }
        b->cstream[c] = nullptr;
        b->join_ev[c] = nullptr;
    }
    b->fork_ev = nullptr;
    // measured on the serving mix at 200 req/s: 36.0 GLUPS with the classes
    // concurrent against 38.6 one after another (the GPU is busy 99 % of the
    // time either way), so the default runs them in order on the batch stream
    b->concurrent = env_int("LBEM_BATCH_CONCURRENT", 0);
    bool ok;
    {
        API_SHARED;
        ok = hipMalloc((void**)&b->dev, bytes) == hipSuccess;
        for (int r = 0; ok && r < NRING; ++r) {
            ok = hipHostMalloc((void**)&b->pinned[r], bytes, hipHostMallocDefault) == hipSuccess &&
                 hipEventCreateWithFlags(&b->ev[r], hipEventDisableTiming) == hipSuccess;
            if (ok) std::memset(b->pinned[r], 0, bytes);
        }
        ok = ok && hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) == hipSuccess;
        for (int c = 0; ok && c < NCLASS; ++c) {
            ok = hipStreamCreateWithFlags(&b->cstream[c], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&b->join_ev[c], hipEventDisableTiming) == hipSuccess;
        }
    }
    if (ok && b->use_graph && !capture_classes(b)) {
        release_graphs(b);
        b->use_graph = 0;  // direct launches of the same kernels
    }
    if (ok) {
        ok = hipMemcpyAsync(b->dev, b->pinned[0], bytes, hipMemcpyHostToDevice, b->stream) == hipSuccess &&
             hipEventRecord(b->ev[0], b->stream) == hipSuccess;
    }
    if (!ok) {
        (void)lbem_batch_destroy(b);
        return LBEM_ENOMEM;
    }
    *out = b;
    return LBEM_OK;
}

int lbem_batch_destroy(lbem_batch_t b)
{
    if (!b) return LBEM_OK;
    API_SHARED;
    (void)hipStreamSynchronize(b->stream);
    for (int c = 0; c < NCLASS; ++c)
        if (b->cstream[c]) (void)hipStreamSynchronize(b->cstream[c]);
    release_graphs(b);
    for (int c = 0; c < NCLASS; ++c) {
        if (b->join_ev[c]) (void)hipEventDestroy(b->join_ev[c]);
        if (b->cstream[c]) (void)hipStreamDestroy(b->cstream[c]);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    for (int i = 0; i < NRING; ++i) {
        if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
        if (b->pinned[i]) (void)hipHostFree(b->pinned[i]);
    }
    if (b->dev) (void)hipFree(b->dev);
    delete b;
    return LBEM_OK;
}

int lbem_batch_run(lbem_batch_t b, const lbem_t* handles, const int64_t* nsteps, int count)
{
    return lbem_batch_run_amp(b, handles, nsteps, nullptr, count);
}

int lbem_batch_run_amp(lbem_batch_t b, const lbem_t* handles, const int64_t* nsteps, const double* amp, int count)
{
    if (!b || count < 0 || count > b->max_grids || (count > 0 && (!handles || !nsteps))) return LBEM_EINVAL;
    for (int i = 0; i < count; ++i) {
        const lbem_s* h = handles[i];
        if (!h || nsteps[i] < 0 || nsteps[i] > b->ksteps) return LBEM_EINVAL;
        const bool plain = h->prec <= LBEM_F32 || h->prec == LBEM_F16;
        if (h->streaming != LBEM_STREAM_PULL && !(h->streaming == LBEM_STREAM_AA && plain)) return LBEM_EINVAL;
        if (has_bx(h)) return LBEM_EINVAL;                // periodic, no cell extras
        if (h->vec != 1) return LBEM_EINVAL;              // the batch tiles one row of cells per thread
        if (!h->have_fields) return LBEM_ESTATE;
        for (int j = 0; j < i; ++j)
            if (handles[j] == h) return LBEM_EINVAL;
    }
    // With a budget, members run in groups, each for all its steps: the
    // members of one class in call order, a 3D class split into runs of
    // members whose state touched per step fits the budget (a member larger
    // than it runs alone), a 2D class in one group.  Without one, all members
    // form one group.
    std::vector<int> order;
    order.reserve(count);
    for (int i = 0; i < count; ++i)
        if (nsteps[i] > 0) order.push_back(i);
    if (b->group_bytes)
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return class_of(handles[x]) < class_of(handles[y]); });
    size_t g0 = 0;
    while (g0 < order.size()) {
        size_t g1 = g0, used = 0;
        const int c0 = class_of(handles[order[g0]]);
        while (g1 < order.size()) {
            const lbem_s* h = handles[order[g1]];
            if (b->group_bytes) {
                if (class_of(h) != c0) break;
                const size_t t = touched_bytes(h);
                if (g1 > g0 && h->D == 3 && used + t > b->group_bytes) break;
                used += t;
            }
            ++g1;
        }
        const int rc = enqueue_group(b, handles, nsteps, amp, order.data() + g0, (int)(g1 - g0));
        if (rc != LBEM_OK) return rc;
        g0 = g1;
    }
    for (int i = 0; i < count; ++i) {
        lbem_s* h = handles[i];
        if (nsteps[i] == 0) continue;
        if (h->streaming == LBEM_STREAM_AA) {
            if (nsteps[i] & 1) h->layout = h->layout == LAYOUT_NATURAL ? LAYOUT_AA_SWAPPED : LAYOUT_NATURAL;
        } else {
            if (nsteps[i] & 1) h->cur = 1 - h->cur;
            h->layout = LAYOUT_PULL_PENDING;
        }
        h->t += nsteps[i];
    }
    return LBEM_OK;
}

}  // extern "C"
