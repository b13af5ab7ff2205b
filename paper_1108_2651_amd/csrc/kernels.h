// kernels.h -- gfx950 kernels of the pseudo-vector lattice-BGK Maxwell scheme
// (Hanasoge, Succi & Orszag, arXiv:1108.2651).
//
// One launch = one time step: gather the pre-collision populations (eq.
// STREAM, applied as a pull or as the in-place AA pattern), form the moments
// (eqs. relate.1-2 with Bbar = K/(D-1)), the equilibrium (eq. distrib.func),
// the tensor source T_i = -(w_i/c^2) eps S (eq. LBE), the BGK update
// (eq. COLLI) and store.  The work is a bandwidth-bound stencil: populations
// are structure-of-arrays (slot k = i*P + p, then cell), every value is read
// once and written once per step, no MFMA.
//
// Storage formats
//   plain  : T = double or float per population.
//   dev    : per cell the post-collision moments (Lambda_p, Bbar_b) in FP32
//            and, per population, its deviation from the equilibrium of those
//            moments in FP16/BF16, divided by a per-cell power-of-two scale
//            times the velocity's equilibrium prefactor.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lattice.h"

namespace lbem {

constexpr int NT = 256;  // threads per block (4 wave64)

// read / write patterns of the population slots
enum { R_LOCAL = 0, R_PULL = 1, R_PULL_SWAP = 2 };
enum { W_LOCAL = 0, W_SWAP = 1, W_PUSH = 2 };

struct Geo {
    int nx, ny, nz;
    int bx_shift;          // block covers BX = 1<<bx_shift cells along x ...
    int tiles_x, tiles_y;  // ... and RB*VEC rows along y (RB = NT/BX)
    int nblocks;
    int xcd;               // remap block ids so each XCD owns a contiguous range
    int strip;             // >0: tiles ordered as strips of `strip` tile-rows
                           // marching through z (keeps z-neighbours in L2)
    int64_t n;
};

// logical tile id -> (tile_x, tile_y, z); the host mirrors this in tile_id()
__host__ __device__ __forceinline__ void tile_coords(const Geo& g, int b, int& tx, int& ty, int& z)
{
    tx = b % g.tiles_x;
    const int r = b / g.tiles_x;
    if (g.strip > 0) {
        const int rs = r % g.strip, r2 = r / g.strip;
        z = r2 % g.nz;
        ty = (r2 / g.nz) * g.strip + rs;
    } else {
        ty = r % g.tiles_y;
        z = r / g.tiles_y;
    }
}

struct Cell {
    int c;
    int xm, xp, ym, yp, zm, zp;
    unsigned wall;         // bit i: the upstream cell x - c_i lies beyond a wall
};

__device__ __forceinline__ Cell make_cell(const Geo& g, int x, int y, int z)
{
    Cell C;
    C.wall = 0;
    const int row = g.nx * (y + g.ny * z);
    C.c = row + x;
    C.xm = row + (x == 0 ? g.nx - 1 : x - 1);
    C.xp = row + (x == g.nx - 1 ? 0 : x + 1);
    const int sy = g.nx;
    C.ym = C.c + (y == 0 ? (g.ny - 1) * sy : -sy);
    C.yp = C.c + (y == g.ny - 1 ? -(g.ny - 1) * sy : sy);
    const int sz = g.nx * g.ny;
    C.zm = C.c + (z == 0 ? (g.nz - 1) * sz : -sz);
    C.zp = C.c + (z == g.nz - 1 ? -(g.nz - 1) * sz : sz);
    return C;
}

// index of the cell at x + sgn*c_i
template <int D>
__device__ __forceinline__ int shifted(const Cell& C, int i, int sgn)
{
    if (i == 0) return C.c;
    const int a = vaxis(D, i), s = vsign(D, i) * sgn;
    if (a == 0) return s > 0 ? C.xp : C.xm;
    if (a == 1) return s > 0 ? C.yp : C.ym;
    return s > 0 ? C.zp : C.zm;
}

// Cell-local extras of the single-step pull kernels.
// Walls: a wall sits half a cell outside the first and last cell of an axis.
// A population that would stream in from beyond it is the cell's own outgoing
// population along the opposite velocity, reflected as a tensor under the
// mirror of that axis: negated for the pairs that contain the axis at a PEC
// wall (tangential E odd about the wall), for the other pairs at a PMC wall.
// Absorbing layer: a cell's post-collision populations times keep = 1 - sigma.
// Dispersion: one Lorentz pole per cell (the convolution term of the Maxwell
// source by an auxiliary differential equation).  Per pair p, with E_p =
// sgn(p) E_gamma(p) = -Lambda_p: J(t+1/2) = c1 J(t-1/2) + c2 E_p(t) - c3 P(t),
// P(t+1) = P(t) + J(t+1/2) (c1 = (1-g/2)/(1+g/2), c2 = wp2/(1+g/2),
// c3 = w02/(1+g/2)); the source -J(t+1/2) enters the rest particle only,
// T_0p = J(t+1/2)/c^2, which keeps the coupled update a centred leapfrog.
struct CellExt {
    int kind[3];           // per axis: 0 periodic, 1 PEC wall, 2 PMC wall
    const void* keep;      // per-cell 1 - sigma (medium precision), or nullptr
    const void* ade;       // [3][n] c1, c2, c3 (medium precision), or nullptr
    void* pol;             // [2P][n] P_p then J_p, updated in place by the cell's thread
    const void* ra;        // [D][n] anisotropy ratios r_a = s_a / c^2 (plain formats), or nullptr
    __host__ __device__ bool walls() const { return (kind[0] | kind[1] | kind[2]) != 0; }
};

// the dispersion update of one cell: new J per pair (the caller adds J/c^2 to
// the rest particle after collision)
template <int D, typename T>
__device__ __forceinline__ void ade_update(const CellExt& bc, int64_t n, int c, T cl2, const T (&rho)[Lat<D>::P],
                                           T (&Jn)[Lat<D>::P])
{
    constexpr int P = Lat<D>::P;
    const T* co = (const T*)bc.ade;
    T* st = (T*)bc.pol;
    const T c1 = co[c], c2 = co[n + c], c3 = co[2 * n + c];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const T Po = st[(int64_t)p * n + c], Jo = st[(int64_t)(P + p) * n + c];
        const T J = c1 * Jo - c2 * (cl2 * rho[p]) - c3 * Po;
        Jn[p] = J;
        st[(int64_t)p * n + c] = Po + J;
        st[(int64_t)(P + p) * n + c] = J;
    }
}

template <int D>
__device__ __forceinline__ void mark_walls(Cell& C, const CellExt& bc, const Geo& g, int x, int y, int z)
{
    unsigned w = 0;
#pragma unroll
    for (int i = 1; i < Lat<D>::Q; ++i) {
        const int a = vaxis(D, i);
        const int v = a == 0 ? x : (a == 1 ? y : z);
        const int nv = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
        if (bc.kind[a] != 0 && (vsign(D, i) > 0 ? v == 0 : v == nv - 1)) w |= 1u << i;
    }
    C.wall = w;
}

// sign of the reflection of pair p for a population entering along i
template <int D>
__device__ __forceinline__ bool wall_negates(const CellExt& bc, int i, int p)
{
    const int a = vaxis(D, i);
    const bool in_pair = pair_a(D, p) == a || pair_b(D, p) == a;
    return (bc.kind[a] == 1) == in_pair;
}

template <int D, int RM>
__device__ __forceinline__ int read_cell(const Cell& C, int i)
{
    return RM == R_LOCAL ? C.c : shifted<D>(C, i, -1);
}
template <int D, int RM>
__device__ __forceinline__ int read_slot(int i)
{
    return RM == R_PULL_SWAP ? opp(D, i) : i;
}
template <int D, int WM>
__device__ __forceinline__ int write_cell(const Cell& C, int i)
{
    return WM == W_PUSH ? shifted<D>(C, i, +1) : C.c;
}
template <int D, int WM>
__device__ __forceinline__ int write_slot(int i)
{
    return WM == W_SWAP ? opp(D, i) : i;
}

__device__ __forceinline__ int remap_block(int bid, int nb, int on)
{
    // Workgroups are dealt round-robin to the 8 XCDs.  on == 1: give each XCD
    // one contiguous range of tiles, so that neighbouring tiles share its L2.
    // on = G >= 2: deal runs of G consecutive tiles to each XCD in turn (the
    // blocks resident at a time stay one band of neighbouring tiles, and the
    // G tiles of a run share one L2); the last nb mod 8G tiles keep their ids.
    if (on == 1) return (nb & 7) == 0 ? (bid & 7) * (nb >> 3) + (bid >> 3) : bid;
    if (on >= 2) {
        const int full = nb - nb % (8 * on);
        if (bid < full) {
            const int x = bid & 7, j = bid >> 3;
            return ((j / on) * 8 + x) * on + j % on;
        }
    }
    return bid;
}

// ---------------------------------------------------------------------------
// moments and equilibrium pieces shared by all formats
// ---------------------------------------------------------------------------

// rho_p = sum_i h_ip and K_b = sum_a sum_i c_ia g_iab (pair form)
template <int D, typename T>
__device__ __forceinline__ void moments(const T (&f)[Lat<D>::Q][Lat<D>::P], T (&rho)[Lat<D>::P],
                                        T (&K)[D])
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        T s = f[0][p];
#pragma unroll
        for (int i = 1; i < Q; ++i) s += f[i][p];
        rho[p] = s;
    }
#pragma unroll
    for (int b = 0; b < D; ++b) K[b] = T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int a = pair_a(D, p), b = pair_b(D, p);
        // first moments of h_p along a and b
        const T Ja = f[1 + a][p] - f[1 + D + a][p];
        const T Jb = f[1 + b][p] - f[1 + D + b][p];
        K[b] += Ja;
        K[a] -= Jb;
    }
}

// 2*g0 of a moving population: Lambda_p + c_ia Bbar_b - c_ib Bbar_a
template <int D, typename T>
__device__ __forceinline__ T twice_eq_moving(int i, int p, T Lam, const T (&Bb)[D])
{
    const int a = pair_a(D, p), b = pair_b(D, p);
    const int ca = cvel(D, i, a), cb = cvel(D, i, b);
    T A = Lam;
    if (ca > 0) A += Bb[b];
    if (ca < 0) A -= Bb[b];
    if (cb > 0) A -= Bb[a];
    if (cb < 0) A += Bb[a];
    return A;
}

// Source S_gamma = c_M^2 (B x grad ln mu)_gamma (+ sparse current part already
// in Sp), mapped to pairs: Sp[p] = sgn(p) S_gamma(p).
template <int D, typename T>
__device__ __forceinline__ void add_mu_source(const T (&K)[D], T cl2, const T* dl, T (&Sp)[Lat<D>::P])
{
    const T cM2 = D == 2 ? cl2 : T(0.5) * cl2;
    T B[3] = {K[0], K[1], D == 3 ? K[D - 1] : T(0)};
    T G[3] = {dl[0], dl[1], D == 3 ? dl[2] : T(0)};
    T S[3];
    S[0] = cM2 * (B[1] * G[2] - B[2] * G[1]);
    S[1] = cM2 * (B[2] * G[0] - B[0] * G[2]);
    S[2] = cM2 * (B[0] * G[1] - B[1] * G[0]);
#pragma unroll
    for (int p = 0; p < Lat<D>::P; ++p) Sp[p] += pair_s(D, p) > 0 ? S[pair_g(D, p)] : -S[pair_g(D, p)];
}

// BGK collision with tensor source, all in precision T.
// f: pre-collision populations; Sp: source per pair (sgn(p) S_gamma(p));
// out: post-collision populations.
template <int D, typename T>
__device__ __forceinline__ void collide(const T (&f)[Lat<D>::Q][Lat<D>::P], T cl2, const T (&Sp)[Lat<D>::P],
                                        bool any_src, T omega, bool tau_half,
                                        const T (&rho)[Lat<D>::P], const T (&K)[D],
                                        T (&out)[Lat<D>::Q][Lat<D>::P])
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    T Lam[P], Bb[D];
#pragma unroll
    for (int p = 0; p < P; ++p) Lam[p] = cl2 * rho[p];
#pragma unroll
    for (int b = 0; b < D; ++b) Bb[b] = D == 2 ? K[b] : T(0.5) * K[b];
    const T wc0 = any_src ? (T(1) / cl2 - T(D)) : T(0);  // w0/c^2 of the rest particle
#pragma unroll
    for (int p = 0; p < P; ++p) {
        // rest equilibrium w0 rho written as the remainder rho - D Lambda (the
        // moving ones carry D Lambda): equal in exact arithmetic (relate.1), but
        // w0 rounded once per cell would bias the mass of every collision by
        // the same factor and make the error grow linearly in time
        const T geq = rho[p] - T(D) * Lam[p];
        T o = tau_half ? (geq + geq) - f[0][p] : f[0][p] + omega * (geq - f[0][p]);
        if (any_src) o -= wc0 * Sp[p];
        out[0][p] = o;
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const T A = twice_eq_moving<D, T>(i, p, Lam[p], Bb);
            T o = tau_half ? A - f[i][p] : f[i][p] + omega * (T(0.5) * A - f[i][p]);
            if (any_src) o -= T(0.5) * Sp[p];
            out[i][p] = o;
        }
    }
}

// Anisotropic collision: per-axis weights w_a = r_a c^2 / 2 (r_a = s_a/c^2,
// s_a the per-axis second moment, c^2 their mean).  The equilibrium keeps the
// form (w_i/c^2)[Lambda + c_ia Bbar_b - c_ib Bbar_a] with Bbar_b = K_b /
// sum_{a != b} r_a, the orthogonal projection onto the conserved moments in
// the 1/w_i inner product (all r_a = 1 is the isotropic collide()).
template <int D, typename T>
__device__ __forceinline__ void collide_an(const T (&f)[Lat<D>::Q][Lat<D>::P], T cl2, const T (&r)[D],
                                           const T (&Sp)[Lat<D>::P], bool any_src, T omega, bool tau_half,
                                           const T (&rho)[Lat<D>::P], const T (&K)[D],
                                           T (&out)[Lat<D>::Q][Lat<D>::P])
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    T Lam[P], Bb[D];
#pragma unroll
    for (int p = 0; p < P; ++p) Lam[p] = cl2 * rho[p];
    T rsum = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) rsum += r[a];
#pragma unroll
    for (int b = 0; b < D; ++b) Bb[b] = K[b] / (rsum - r[b]);
    const T wc0 = any_src ? (T(1) / cl2 - rsum) : T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const T geq = rho[p] - rsum * Lam[p];       // w0 rho as the remainder (see collide())
        T o = tau_half ? (geq + geq) - f[0][p] : f[0][p] + omega * (geq - f[0][p]);
        if (any_src) o -= wc0 * Sp[p];
        out[0][p] = o;
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const T ri = r[vaxis(D, i)];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const T A = ri * twice_eq_moving<D, T>(i, p, Lam[p], Bb);
            T o = tau_half ? A - f[i][p] : f[i][p] + omega * (T(0.5) * A - f[i][p]);
            if (any_src) o -= T(0.5) * ri * Sp[p];
            out[i][p] = o;
        }
    }
}

// ---------------------------------------------------------------------------
// block decomposition shared by the step kernels
// ---------------------------------------------------------------------------
struct Tile {
    int b;       // logical tile id
    int x, y0, z;
    int rb;      // rows per sub-block
};

__device__ __forceinline__ Tile tile_of(const Geo& g, int vec)
{
    Tile t;
    t.b = remap_block(blockIdx.x, g.nblocks, g.xcd);
    int tx, ty;
    tile_coords(g, t.b, tx, ty, t.z);
    const int bx = 1 << g.bx_shift;
    t.rb = NT >> g.bx_shift;
    t.x = tx * bx + (threadIdx.x & (bx - 1));
    t.y0 = ty * t.rb * vec + (threadIdx.x >> g.bx_shift);
    return t;
}

// Sparse current source: per tile a range [off[b], off[b+1]) of entries
// (local cell slot v*NT + tid, pair p) with value sval (S per unit amplitude
// for that pair).  Staged into LDS by the tiles that own source cells.
template <typename T>
struct SrcArgs {
    const int* off;      // nblocks+1 or nullptr
    const int2* ent;
    const T* val;
    T amp;
};

template <int P, int VEC, typename T>
__device__ __forceinline__ bool stage_source(const SrcArgs<T>& s, int b, T* lds)
{
    if (s.off == nullptr) return false;
    const int s0 = s.off[b], s1 = s.off[b + 1];
    if (s1 <= s0) return false;
    for (int k = threadIdx.x; k < P * NT * VEC; k += NT) lds[k] = T(0);
    __syncthreads();
    for (int k = s0 + threadIdx.x; k < s1; k += NT) {
        const int2 e = s.ent[k];
        lds[e.y * NT * VEC + e.x] = s.val[k] * s.amp;
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------------------
// plain FP64/FP32 stream-collide
// ---------------------------------------------------------------------------
// Storage <-> arithmetic of the plain formats: populations are stored as S
// and computed in T (S = T except plain FP16 storage with FP32 arithmetic,
// rounded to nearest even on the store).
template <typename T, typename S>
__device__ __forceinline__ T ld_pop(S v) { return (T)v; }
template <>
__device__ __forceinline__ float ld_pop<float, __half>(__half v) { return __half2float(v); }
template <typename S, typename T>
__device__ __forceinline__ S st_pop(T v) { return (S)v; }
template <>
__device__ __forceinline__ __half st_pop<__half, float>(float v) { return __float2half_rn(v); }

// Global access with the streaming (non-temporal) cache policy when NTS is
// set, plain access otherwise; the values are the same either way.  A step on
// a lattice larger than the last-level cache touches each stored value once
// per launch, and marking those lines for early eviction keeps the caches for
// the halo lines that neighbouring tiles share.  Loads that neighbouring tiles
// share are never marked: those lose their reuse.
template <bool NTS, typename S>
__device__ __forceinline__ S ld_stream(const S* p)
{
    if constexpr (!NTS) {
        return *p;
    } else if constexpr (sizeof(S) == 2) {
        const unsigned short u = __builtin_nontemporal_load((const unsigned short*)p);
        S r;
        __builtin_memcpy(&r, &u, 2);
        return r;
    } else {
        return __builtin_nontemporal_load(p);
    }
}
template <bool NTS, typename S>
__device__ __forceinline__ void st_stream(S* p, S v)
{
    if constexpr (!NTS) {
        *p = v;
    } else if constexpr (sizeof(S) == 2) {
        unsigned short u;
        __builtin_memcpy(&u, &v, 2);
        __builtin_nontemporal_store(u, (unsigned short*)p);
    } else {
        __builtin_nontemporal_store(v, p);
    }
}

// NTS: streaming loads and stores of the populations (each is read and written
// once per launch; lattices beyond the last-level cache)
template <int D, typename T, int RM, int WM, int VEC, bool MU, bool BX, typename S = T, bool NTS = false>
__global__ __launch_bounds__(NT) void k_step_plain(const S* src, S* dst, const T* __restrict__ cl2a,
                                                  const T* __restrict__ dlnmu, const Geo g,
                                                  const SrcArgs<T> s, const T omega, const int tau_half,
                                                  const CellExt bc)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    __shared__ T lds[P * NT * VEC];
    const Tile t = tile_of(g, VEC);
    const bool has_src = stage_source<P, VEC, T>(s, t.b, lds);
    const bool any_src = has_src || MU;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const int y = t.y0 + v * t.rb;
        if (t.x >= g.nx || y >= g.ny) continue;
        Cell C = make_cell(g, t.x, y, t.z);
        if (BX && RM == R_PULL) mark_walls<D>(C, bc, g, t.x, y, t.z);
        T f[Q][P];
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (BX && RM == R_PULL && ((C.wall >> i) & 1u)) {
                    const T v = ld_pop<T>(ld_stream<NTS>(&src[(int64_t)(opp(D, i) * P + p) * g.n + C.c]));
                    f[i][p] = wall_negates<D>(bc, i, p) ? -v : v;
                } else {
                    f[i][p] = ld_pop<T>(ld_stream<NTS>(&src[(int64_t)(read_slot<D, RM>(i) * P + p) * g.n + read_cell<D, RM>(C, i)]));
                }
            }
        const T cl2 = cl2a[C.c];
        T rho[P], K[D], Sp[P];
        moments<D, T>(f, rho, K);
#pragma unroll
        for (int p = 0; p < P; ++p) Sp[p] = has_src ? lds[p * NT * VEC + v * NT + threadIdx.x] : T(0);
        if (MU) {
            T dl[D];
#pragma unroll
            for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * g.n + C.c];
            add_mu_source<D, T>(K, cl2, dl, Sp);
        }
        T Jn[P];
        const bool ade = BX && bc.ade != nullptr;
        if (ade) ade_update<D, T>(bc, g.n, C.c, cl2, rho, Jn);
        T out[Q][P];
        if (BX && bc.ra) {
            T r[D];
#pragma unroll
            for (int a = 0; a < D; ++a) r[a] = ((const T*)bc.ra)[(int64_t)a * g.n + C.c];
            collide_an<D, T>(f, cl2, r, Sp, any_src, omega, tau_half != 0, rho, K, out);
        } else {
            collide<D, T>(f, cl2, Sp, any_src, omega, tau_half != 0, rho, K, out);
        }
        if (ade) {
#pragma unroll
            for (int p = 0; p < P; ++p) out[0][p] += Jn[p] / cl2;
        }
        if (BX && bc.keep) {
            const T k = ((const T*)bc.keep)[C.c];
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int p = 0; p < P; ++p) out[i][p] *= k;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int p = 0; p < P; ++p)
                st_stream<NTS>(&dst[(int64_t)(write_slot<D, WM>(i) * P + p) * g.n + write_cell<D, WM>(C, i)], st_pop<S>(out[i][p]));
    }
}

// ---------------------------------------------------------------------------
// 3D plain formats, single step on whole-row blocks
// ---------------------------------------------------------------------------
// A block of NT threads owns `rows` whole x-rows of one plane; a thread owns
// CX cells of one row (x = q + k*tpr).  The populations that move along y or
// z are read from (and, pushed, written to) the neighbouring rows directly:
// those rows are aligned to the same x, so every access is a whole, aligned
// row segment.  The ones that move along x go through LDS: a thread loads
// (and stores) the slot at its own cell and the row shifts by one in LDS, so
// no load or store straddles cache lines.  With the in-place AA pattern each
// stored location is still read and written by one thread only.  The
// arithmetic is k_step_plain's, so the two agree bit for bit.
struct XRowGeo {
    int nx, ny, nz;
    int tpr, rows;       // threads per row (multiple of 64, CX*tpr >= nx), rows per block (NT / tpr)
    int tiles_y, nblocks;
    int64_t n;
};

template <typename T, int RM, int WM, bool MU, typename S, bool NTS, int CX>
__global__ __launch_bounds__(NT) void k_step_xrow(const S* src, S* dst, const T* __restrict__ cl2a,
                                                 const T* __restrict__ dlnmu, const XRowGeo g,
                                                 const int* __restrict__ soff, const int2* __restrict__ sent,
                                                 const T* __restrict__ sval, const T amp, const T omega,
                                                 const int tau_half)
{
    constexpr int D = 3, Q = 7, P = 3;
    constexpr int RC = CX * NT;               // cells of the block
    __shared__ T lx[2 * P * RC];              // [side*P + p][row*nx + x]
    const int b = blockIdx.x;
    const int yt = b % g.tiles_y, z = b / g.tiles_y;
    const int y0 = yt * g.rows;
    const int nx = g.nx;
    const int r = threadIdx.x / g.tpr, q = threadIdx.x % g.tpr;
    const int y = y0 + r;
    const bool row_ok = r < g.rows && y < g.ny;
    const int64_t n = g.n;
    int xs[CX];
    bool ok[CX];
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        xs[k] = q + k * g.tpr;
        ok[k] = row_ok && xs[k] < nx;
    }
    // the slot that arrives along +x (side 0) and -x (side 1), read at the own cell
    constexpr int in_p = RM == R_PULL_SWAP ? 4 : 1;   // arrives along +x: slot 1 (pull) / 4 (AA odd)
    constexpr int in_m = RM == R_PULL_SWAP ? 1 : 4;
    constexpr bool XIN = RM != R_LOCAL;
    constexpr bool XOUT = WM == W_PUSH;

    T f[CX][Q][P];
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        if (!ok[k]) continue;
        Cell C = make_cell(Geo{nx, g.ny, g.nz, 0, 0, 0, 0, 0, 0, n}, xs[k], y, z);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const bool along_x = i == 1 || i == 4;
            if (XIN && along_x) continue;
#pragma unroll
            for (int p = 0; p < P; ++p)
                f[k][i][p] = ld_pop<T>(ld_stream<NTS>(&src[(int64_t)(read_slot<D, RM>(i) * P + p) * n + read_cell<D, RM>(C, i)]));
        }
        if constexpr (XIN) {
            const int loc = r * nx + xs[k];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                lx[(0 * P + p) * RC + loc] = ld_pop<T>(ld_stream<NTS>(&src[(int64_t)(in_p * P + p) * n + C.c]));
                lx[(1 * P + p) * RC + loc] = ld_pop<T>(ld_stream<NTS>(&src[(int64_t)(in_m * P + p) * n + C.c]));
            }
        }
    }
    if constexpr (XIN) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            if (!ok[k]) continue;
            const int x = xs[k];
            const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                f[k][1][p] = lx[(0 * P + p) * RC + r * nx + xm];    // from x-1
                f[k][4][p] = lx[(1 * P + p) * RC + r * nx + xp];    // from x+1
            }
        }
        __syncthreads();
    }
    // source entries of this block: (row*nx + x, pair)
    int s0 = 0, s1 = 0;
    if (soff) {
        s0 = soff[b];
        s1 = soff[b + 1];
    }
    const bool has_src = s1 > s0;
    T out[CX][Q][P];
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        if (!ok[k]) continue;
        const int64_t c = (int64_t)z * ((int64_t)nx * g.ny) + (int64_t)y * nx + xs[k];
        const T cl2 = cl2a[c];
        T rho[P], K[D], Sp[P];
        moments<D, T>(f[k], rho, K);
#pragma unroll
        for (int p = 0; p < P; ++p) Sp[p] = T(0);
        const int loc = r * nx + xs[k];
        for (int e = s0; e < s1; ++e) {
            const int2 en = sent[e];
            if (en.x == loc) {
                const T v = sval[e] * amp;
#pragma unroll
                for (int p = 0; p < P; ++p)
                    if (en.y == p) Sp[p] = v;
            }
        }
        if (MU) {
            T dl[D];
#pragma unroll
            for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * n + c];
            add_mu_source<D, T>(K, cl2, dl, Sp);
        }
        collide<D, T>(f[k], cl2, Sp, has_src || MU, omega, tau_half != 0, rho, K, out[k]);
    }
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        if (!ok[k]) continue;
        Cell C = make_cell(Geo{nx, g.ny, g.nz, 0, 0, 0, 0, 0, 0, n}, xs[k], y, z);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const bool along_x = i == 1 || i == 4;
            if (XOUT && along_x) continue;
#pragma unroll
            for (int p = 0; p < P; ++p)
                st_stream<NTS>(&dst[(int64_t)(write_slot<D, WM>(i) * P + p) * n + write_cell<D, WM>(C, i)],
                               st_pop<S>(out[k][i][p]));
        }
        if constexpr (XOUT) {
            const int x = xs[k];
            const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                lx[(0 * P + p) * RC + r * nx + xp] = out[k][1][p];   // pushed to x+1
                lx[(1 * P + p) * RC + r * nx + xm] = out[k][4][p];   // pushed to x-1
            }
        }
    }
    if constexpr (XOUT) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            if (!ok[k]) continue;
            const int64_t c = (int64_t)z * ((int64_t)nx * g.ny) + (int64_t)y * nx + xs[k];
            const int loc = r * nx + xs[k];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                st_stream<NTS>(&dst[(int64_t)(1 * P + p) * n + c], st_pop<S>(lx[(0 * P + p) * RC + loc]));
                st_stream<NTS>(&dst[(int64_t)(4 * P + p) * n + c], st_pop<S>(lx[(1 * P + p) * RC + loc]));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 2D temporal blocking: NS time steps per launch (plain formats, pull)
// ---------------------------------------------------------------------------
// A block owns an output tile of TXF x TY cells.  All work happens in one LDS
// frame: the tile grown by H = NS-1 cells on every side.  Step 1 pulls the
// stored populations from HBM for the whole frame and collides; steps 2..NS
// pull from the previous LDS layer, each on a region one cell smaller, the
// last one on the tile itself, which is written back.  State bytes therefore
// cross HBM once per NS steps; every cell update runs the same collide() code
// as the single-step kernel, so NS fused steps equal NS single steps bit for
// bit.  Periodic wrap is applied to the frame's global coordinates.
constexpr int TXF = 64;

// Element idx of an array whose byte size fits 32 bits: the offset is formed
// in 32-bit arithmetic, so the load or store takes the scalar-base plus
// 32-bit vector-offset form and needs no 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T& at32(T* base, unsigned idx)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T& at32(const T* base, unsigned idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}

template <typename T>
struct FusedSrc {
    const int* off;      // per tile range into ent/val (nullptr: no source)
    const int2* ent;     // (frame cell index, pair)
    const T* val;        // S per unit amplitude
};

template <typename T, int NS>
struct AmpPack {
    T a[NS];             // source amplitude of each fused step
};

// O32: every population plane fits 2^32 bytes (32-bit element offsets)
// NTS: streaming stores of the state (lattices beyond the last-level cache).
// TH: tau = 1/2 known when compiling (the reflection collision, whatever
// tau_half says), else tau_half chooses at run time.
template <typename T, int NS, int TY, bool MU, bool O32, bool NTS, bool TH, int NTB = NT>
__global__ __launch_bounds__(NTB) void k_step_fused2d(const T* src, T* dst, const T* __restrict__ cl2a,
                                                    const T* __restrict__ dlnmu, const Geo g,
                                                    const FusedSrc<T> fs, const AmpPack<T, NS> amps,
                                                    const T omega, const int tau_half)
{
    constexpr int H = NS - 1;
    constexpr int W = TXF + 2 * H;          // frame width
    constexpr int FH = TY + 2 * H;          // frame height
    constexpr int FC = W * FH;
    constexpr int NB = NS > 2 ? 2 : 1;      // LDS population layers
    constexpr int Q = 5;
    __shared__ T lp[NB][Q][FC];
    __shared__ T lc[FC];
    __shared__ T ls[FC];
    __shared__ T ldl[MU ? 2 : 1][MU ? FC : 1];   // grad ln mu of the frame

    const int b = remap_block(blockIdx.x, g.nblocks, g.xcd);
    const int tx = b % g.tiles_x, ty = b / g.tiles_x;
    const int x0 = tx * TXF - H, y0 = ty * TY - H;     // global coords of frame (0,0)

    // source coefficients of the frame (tiles that own none skip this)
    bool has_src = false;
    if (fs.off) {
        const int s0 = fs.off[b], s1 = fs.off[b + 1];
        if (s1 > s0) {
            has_src = true;
            for (int k = threadIdx.x; k < FC; k += NTB) ls[k] = T(0);
            __syncthreads();
            for (int k = s0 + threadIdx.x; k < s1; k += NTB) {
                const int2 e = fs.ent[k];
                ls[e.x] = fs.val[k];
            }
            __syncthreads();
        }
    }

    // step 1 over the whole frame: every thread first issues the HBM loads of
    // all its frame cells, then collides them into LDS layer 0
    {
        constexpr int C0 = (FC + NTB - 1) / NTB;
        T fv0[C0][Q][1];
        T cl0[C0];
        T dl0[C0][2];
        // frame coordinates wrap at most once when the box is at least a
        // frame wide (no division); smaller boxes take the remainder
        const bool wide = g.nx >= W && g.ny >= FH;
#pragma unroll
        for (int j = 0; j < C0; ++j) {
            const int k = threadIdx.x + j * NTB;
            if (k < FC) {
                const int fx = k % W, fy = k / W;
                int gx = x0 + fx, gy = y0 + fy;
                if (wide) {
                    gx = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
                    gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
                } else {
                    gx %= g.nx;
                    gy %= g.ny;
                    if (gx < 0) gx += g.nx;
                    if (gy < 0) gy += g.ny;
                }
                const Cell C = make_cell(g, gx, gy, 0);
                if constexpr (O32) {
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        fv0[j][i][0] = at32(src + (int64_t)i * g.n, (unsigned)read_cell<2, R_PULL>(C, i));
                    cl0[j] = at32(cl2a, (unsigned)C.c);
                    if (MU) {
                        dl0[j][0] = at32(dlnmu, (unsigned)C.c);
                        dl0[j][1] = at32(dlnmu + g.n, (unsigned)C.c);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < Q; ++i) fv0[j][i][0] = src[(int64_t)i * g.n + read_cell<2, R_PULL>(C, i)];
                    cl0[j] = cl2a[C.c];
                    if (MU) {
                        dl0[j][0] = dlnmu[C.c];
                        dl0[j][1] = dlnmu[(int64_t)g.n + C.c];
                    }
                }
            }
        }
        const T amp = has_src ? amps.a[0] : T(0);
#pragma unroll
        for (int j = 0; j < C0; ++j) {
            const int k = threadIdx.x + j * NTB;
            if (k < FC) {
                T rho[1], K[2], Sp[1], o[Q][1];
                moments<2, T>(fv0[j], rho, K);
                Sp[0] = has_src ? ls[k] * amp : T(0);
                if (MU) {
                    add_mu_source<2, T>(K, cl0[j], dl0[j], Sp);
                    ldl[0][k] = dl0[j][0];
                    ldl[MU ? 1 : 0][k] = dl0[j][1];
                }
                collide<2, T>(fv0[j], cl0[j], Sp, has_src || MU, omega, TH || tau_half != 0, rho, K, o);
                lc[k] = cl0[j];
#pragma unroll
                for (int i = 0; i < Q; ++i) lp[0][i][k] = o[i][0];
            }
        }
        __syncthreads();
    }

    // steps 2..NS from LDS on shrinking regions; the last one writes the tile
#pragma unroll
    for (int st = 1; st < NS; ++st) {
        const int r = H - st;               // region = tile grown by r
        const int wr = TXF + 2 * r, hr = TY + 2 * r, off = H - r;
        const T amp = has_src ? amps.a[st] : T(0);
        const int in = (st - 1) % NB, out = st % NB;
        for (int k = threadIdx.x; k < wr * hr; k += NTB) {
            const int fx = off + k % wr, fy = off + k / wr;
            const int f = fy * W + fx;
            T fv[Q][1];
            // pull from the previous layer: x - c_i in frame coordinates
            fv[0][0] = lp[in][0][f];
            fv[1][0] = lp[in][1][f - 1];
            fv[2][0] = lp[in][2][f - W];
            fv[3][0] = lp[in][3][f + 1];
            fv[4][0] = lp[in][4][f + W];
            const T cl2 = lc[f];
            T rho[1], K[2], Sp[1];
            moments<2, T>(fv, rho, K);
            Sp[0] = has_src ? ls[f] * amp : T(0);
            if (MU) {
                const T dl[2] = {ldl[0][f], ldl[MU ? 1 : 0][f]};
                add_mu_source<2, T>(K, cl2, dl, Sp);
            }
            T o[Q][1];
            collide<2, T>(fv, cl2, Sp, has_src || MU, omega, TH || tau_half != 0, rho, K, o);
            if (st == NS - 1) {
                const int gx = x0 + fx, gy = y0 + fy;    // inside the tile: no wrap needed
                if (gx < g.nx && gy < g.ny) {
                    const int gcell = gx + g.nx * gy;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        if constexpr (O32) st_stream<NTS>(&at32(dst + (int64_t)i * g.n, (unsigned)gcell), o[i][0]);
                        else st_stream<NTS>(&dst[(int64_t)i * g.n + gcell], o[i][0]);
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) lp[out][i][f] = o[i][0];
            }
        }
        if (st < NS - 1) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3D temporal blocking: two time steps per launch, marching along z
// ---------------------------------------------------------------------------
// A block of TX x TY threads owns a TX x TY column tile and a chunk of lz
// planes.  For every
// plane zz from z0-1 to z0+lz it runs step 1 on the tile grown by one cell in
// x and y (pulling the stored state from HBM), keeping for tile cells the +z
// components (LDS ring of 3 planes) and -z components (one plane) and holding
// the in-plane components (rest, +-x, +-y, halo included) in registers; then
// it runs step 2 on plane zz-1 of the tile, pulling from LDS, writes it, and
// only then stores plane zz's in-plane components into the single LDS frame
// (one frame instead of two: three 64 x 4 blocks or two 64 x 8 blocks per CU).
// Every update is the same collide() as the single-step kernel: bit-identical.
// NTS: streaming stores (the frame loads stay plain: neighbouring tiles share
// them).  TH: tau = 1/2 known when compiling, as for the 2D kernel.  Tiles
// of 512 threads ask for four waves per SIMD (<= 128 VGPRs), so that two
// blocks share a CU; 256-thread tiles keep the compiler's choice.
template <typename T, int TX, int TY, bool MU, bool NTS, bool TH>
__global__ __launch_bounds__(TX * TY, TX * TY >= 512 ? 4 : 1) void k_step_fused3d(const T* src, T* dst, const T* __restrict__ cl2a,
                                                    const T* __restrict__ dlnmu, const Geo g, const int lz,
                                                    const FusedSrc<T> fs, const AmpPack<T, 2> amps,
                                                    const T omega, const int tau_half)
{
    constexpr int D = 3, Q = 7, P = 3;
    constexpr int W = TX + 2, HH = TY + 2, FC = W * HH, TC = TX * TY;   // one tile cell per thread
    constexpr int NIP = 5;                       // in-plane velocities 0, +x, +y, -x, -y
    constexpr int CF = (FC + TC - 1) / TC;       // frame cells per thread
    __shared__ T lin[NIP * P][FC];               // in-plane outputs of plane zz-1 (frame)
    __shared__ T lpz[3][P][TC];
    __shared__ T lmz[P][TC];
    __shared__ T lsrc[2][P][FC];

    const int b = remap_block(blockIdx.x, g.nblocks, g.xcd);
    const int tx = b % g.tiles_x, r = b / g.tiles_x;
    const int ty = r % g.tiles_y, zc = r / g.tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = zc * lz;
    const int z1 = min(z0 + lz, g.nz);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int hc = (ly + 1) * W + (lx + 1);

    int s0 = 0, s1 = 0;
    if (fs.off) {
        s0 = fs.off[b];
        s1 = fs.off[b + 1];
    }
    const bool has_src = s1 > s0;

    // in-plane slot of velocity i (0, +x, +y, -x, -y), -1 for +-z
    auto ipl = [](int i) { return i == 0 ? 0 : (i == 1 ? 1 : (i == 2 ? 2 : (i == 4 ? 3 : (i == 5 ? 4 : -1)))); };

    for (int zz = z0 - 1; zz <= z1; ++zz) {
        const int rel = zz - (z0 - 1);          // 0 .. lz+1
        const int bi = rel & 1;
        int gz = zz % g.nz;
        if (gz < 0) gz += g.nz;
        if (has_src) {
            for (int k = threadIdx.x; k < P * FC; k += TC) (&lsrc[bi][0][0])[k] = T(0);
            __syncthreads();
            for (int k = s0 + threadIdx.x; k < s1; k += TC) {
                const int2 e = fs.ent[k];          // x = plane offset * FC + frame cell, y = pair
                if (e.x / FC == rel) lsrc[bi][e.y][e.x % FC] = fs.val[k];
            }
            __syncthreads();
        }
        // ---- step 1 on plane zz, frame cells; the in-plane outputs stay in
        // registers until step 2 has read plane zz-1 from the frame buffer
        T held[CF][NIP * P];
#pragma unroll
        for (int j = 0; j < CF; ++j) {
            const int k = threadIdx.x + j * TC;
            if (k >= FC) continue;
            const int hx = k % W, hy = k / W;
            int gx = (x0 - 1 + hx) % g.nx, gy = (y0 - 1 + hy) % g.ny;
            if (gx < 0) gx += g.nx;
            if (gy < 0) gy += g.ny;
            const Cell C = make_cell(g, gx, gy, gz);
            T f[Q][P];
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int p = 0; p < P; ++p) f[i][p] = src[(int64_t)(i * P + p) * g.n + read_cell<D, R_PULL>(C, i)];
            const T cl2 = cl2a[C.c];
            T rho[P], K[D], Sp[P], out[Q][P];
            moments<D, T>(f, rho, K);
#pragma unroll
            for (int p = 0; p < P; ++p) Sp[p] = has_src ? lsrc[bi][p][k] * amps.a[0] : T(0);
            if (MU) {
                T dl[D];
#pragma unroll
                for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * g.n + C.c];
                add_mu_source<D, T>(K, cl2, dl, Sp);
            }
            collide<D, T>(f, cl2, Sp, has_src || MU, omega, TH || tau_half != 0, rho, K, out);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int sl = ipl(i);
                if (sl >= 0) {
#pragma unroll
                    for (int p = 0; p < P; ++p) held[j][sl * P + p] = out[i][p];
                }
            }
            const bool tile = hx >= 1 && hx <= TX && hy >= 1 && hy <= TY;
            if (tile) {
                const int tcell = (hy - 1) * TX + (hx - 1);
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    lpz[rel % 3][p][tcell] = out[3][p];
                    lmz[p][tcell] = out[6][p];
                }
            }
        }
        __syncthreads();
        // ---- step 2 on plane zz-1 of the tile
        const int zc2 = zz - 1;
        if (zc2 >= z0 && zc2 < z1) {
            const int x = x0 + lx, y = y0 + ly;
            if (x < g.nx && y < g.ny) {
                const int pb = (rel - 1) & 1;       // plane zz-1's source buffer
                T f[Q][P];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    f[0][p] = lin[0 * P + p][hc];
                    f[1][p] = lin[1 * P + p][hc - 1];
                    f[2][p] = lin[2 * P + p][hc - W];
                    f[4][p] = lin[3 * P + p][hc + 1];
                    f[5][p] = lin[4 * P + p][hc + W];
                    f[3][p] = lpz[(rel + 1) % 3][p][threadIdx.x];   // plane zz-2, moving +z
                    f[6][p] = lmz[p][threadIdx.x];                   // plane zz, moving -z
                }
                const int c = x + g.nx * (y + g.ny * zc2);
                const T cl2 = cl2a[c];
                T rho[P], K[D], Sp[P], out[Q][P];
                moments<D, T>(f, rho, K);
#pragma unroll
                for (int p = 0; p < P; ++p) Sp[p] = has_src ? lsrc[pb][p][hc] * amps.a[1] : T(0);
                if (MU) {
                    T dl[D];
#pragma unroll
                    for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * g.n + c];
                    add_mu_source<D, T>(K, cl2, dl, Sp);
                }
                collide<D, T>(f, cl2, Sp, has_src || MU, omega, TH || tau_half != 0, rho, K, out);
#pragma unroll
                for (int i = 0; i < Q; ++i)
#pragma unroll
                    for (int p = 0; p < P; ++p) st_stream<NTS>(&dst[(int64_t)(i * P + p) * g.n + c], out[i][p]);
            }
        }
        __syncthreads();
        // ---- plane zz's in-plane outputs into the frame buffer (read by the
        // next iteration's step 2, after its step-1 barrier)
#pragma unroll
        for (int j = 0; j < CF; ++j) {
            const int k = threadIdx.x + j * TC;
            if (k >= FC) continue;
#pragma unroll
            for (int q = 0; q < NIP * P; ++q) lin[q][k] = held[j][q];
        }
    }
}

// ---------------------------------------------------------------------------
// deviation storage: FP32 moments + 16-bit scaled deviations, FP32 arithmetic
// ---------------------------------------------------------------------------
template <typename H>
__device__ __forceinline__ float h2f(H v);
template <>
__device__ __forceinline__ float h2f<__half>(__half v) { return __half2float(v); }
template <>
__device__ __forceinline__ float h2f<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }
template <typename H>
__device__ __forceinline__ H f2h(float v);
template <>
__device__ __forceinline__ __half f2h<__half>(float v) { return __float2half_rn(v); }
template <>
__device__ __forceinline__ __hip_bfloat16 f2h<__hip_bfloat16>(float v) { return __float2bfloat16(v); }

// Scale of the stored deviations.  Per cell, s(x) is the smallest power of two
// >= max |stored moment| of that cell (its FP32 Lambda_p and Bbar_b, which the
// writer and every reader see identically), so 16-bit precision is relative
// to the local field whatever its absolute size.  Per velocity the scale is
// s(x) times the equilibrium prefactor of that velocity: 1/2 for the moving
// ones, w0/c^2(x) for the rest particle.
__device__ __forceinline__ void pow2_scale(float m, float& s, float& inv)
{
    unsigned u = __float_as_uint(fabsf(m));
    int e = (int)((u >> 23) & 0xffu);
    if (e == 0) {               // zero or subnormal moments: unit scale
        s = 1.f;
        inv = 1.f;
        return;
    }
    if (u & 0x7fffffu) ++e;     // round up to the next power of two
    if (e > 253) e = 253;
    s = __uint_as_float((unsigned)e << 23);
    inv = __uint_as_float((unsigned)(254 - e) << 23);
}

template <int D>
__device__ __forceinline__ float cell_magnitude(const float* M, int64_t n, int cs)
{
    constexpr int P = Lat<D>::P;
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < P + D; ++q) m = fmaxf(m, fabsf(M[(int64_t)q * n + cs]));
    return m;
}

// 16-bit codes saturate at the largest finite value instead of overflowing
template <typename H>
__device__ __forceinline__ float sat16(float v)
{
    const float lim = sizeof(H) == 2 && std::is_same<H, __half>::value ? 65504.f : 3.0e38f;
    return fminf(fmaxf(v, -lim), lim);
}

// equilibrium of the stored moments, as used by both the writer and readers
template <int D>
__device__ __forceinline__ float dev_eq(int i, int p, const float (&Lam)[Lat<D>::P], const float (&Bb)[D], float wc0)
{
    if (i == 0) return wc0 * Lam[p];
    return 0.5f * twice_eq_moving<D, float>(i, p, Lam[p], Bb);
}

// Ghost-coordinate encoding.  The deviation n = g' - g0(m(g')) of a cell has
// vanishing moments: sum_i n_{i,p} = 0 for every pair p, and each component e
// of the contracted first moment, sum_{i,p} k(i,p,e) n_{i,p} with k below, is
// zero.  So P + D of the Q P entries follow from the others and only the
// remaining (Q-1) P - D moving entries are stored.  Dropped: every rest entry
// (recovered at its own cell from the cell's moving entries) and, for each e,
// the entry moving along -o in the lowest pair {e, o}; that entry appears in no
// other constraint, and its own constraint involves no other dropped entry.
__host__ __device__ constexpr int kcoef(int D, int i, int p, int e)
{
    return (e == pair_b(D, p) ? cvel(D, i, pair_a(D, p)) : 0) -
           (e == pair_a(D, p) ? cvel(D, i, pair_b(D, p)) : 0);
}
__host__ __device__ constexpr int ghost_pair(int D, int e) { return D == 2 ? 0 : (e == 2 ? 1 : 0); }
__host__ __device__ constexpr int ghost_dir(int D, int e)
{
    return 1 + D + (pair_a(D, ghost_pair(D, e)) == e ? pair_b(D, ghost_pair(D, e)) : pair_a(D, ghost_pair(D, e)));
}
// the first-moment component whose constraint recovers entry (i,p), or -1
__host__ __device__ constexpr int ghost_dropped_by(int D, int i, int p)
{
    for (int e = 0; e < D; ++e)
        if (ghost_dir(D, e) == i && ghost_pair(D, e) == p) return e;
    return -1;
}
// slot of entry (i,p) in the deviation arrays, -1 if it is not stored
template <int D, bool GH>
__host__ __device__ constexpr int dev_slot(int i, int p)
{
    constexpr int P = Lat<D>::P;
    if (!GH) return i * P + p;
    if (i == 0 || ghost_dropped_by(D, i, p) >= 0) return -1;
    int s = 0;
    for (int j = 1; j <= 2 * D; ++j)
        for (int q = 0; q < P; ++q) {
            if (j == i && q == p) return s;
            if (ghost_dropped_by(D, j, q) < 0) ++s;
        }
    return -1;
}
template <int D, bool GH>
struct DevSlots {
    static constexpr int N = GH ? 2 * D * Lat<D>::P - D : Lat<D>::Q * Lat<D>::P;
};

// scaled code of moving entry (i,p) of one cell: stored, or recovered from its
// first-moment constraint; get(slot) returns the cell's stored code of a slot
// (read from HBM or held in registers: the arithmetic is the same)
template <int D, bool GH, class Get>
__device__ __forceinline__ float dev_code_of(const Get& get, int i, int p)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    const int e = GH ? ghost_dropped_by(D, i, p) : -1;
    if (e < 0) return get(dev_slot<D, GH>(i, p));
    float sum = 0.f;
#pragma unroll
    for (int j = 1; j < Q; ++j)
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = kcoef(D, j, q, e);
            if (k == 0 || (j == i && q == p)) continue;
            const float v = get(dev_slot<D, GH>(j, q));
            sum = k > 0 ? sum + v : sum - v;
        }
    return kcoef(D, i, p, e) > 0 ? -sum : sum;
}

// deviation of population (i,p) of one cell with cell scale s
template <int D, bool GH, class Get>
__device__ __forceinline__ float dev_value_of(const Get& get, int i, int p, float s, float wc0)
{
    constexpr int Q = Lat<D>::Q;
    if (!GH) return (i == 0 ? s * wc0 : 0.5f * s) * dev_code_of<D, false>(get, i, p);
    if (i != 0) return 0.5f * s * dev_code_of<D, true>(get, i, p);
    float sum = 0.f;
#pragma unroll
    for (int j = 1; j < Q; ++j) sum += dev_code_of<D, true>(get, j, p);
    return -0.5f * s * sum;
}

// the same, reading the codes of cell cs from the deviation arrays
template <int D, typename H, bool GH>
__device__ __forceinline__ float dev_value(const H* Dv, int64_t n, int i, int p, int cs, float s, float wc0)
{
    auto get = [&](int sl) { return h2f<H>(Dv[(int64_t)sl * n + cs]); };
    return dev_value_of<D, GH>(get, i, p, s, wc0);
}

// Reconstruct population (i,p) stored at cell cs (moments M, deviations Dv).
template <int D, typename H, bool GH>
__device__ __forceinline__ float dev_load(const float* M, const H* Dv, int64_t n, int i, int p, int cs,
                                          float wc0_here)
{
    constexpr int P = Lat<D>::P;
    float Lam[P], Bb[D];
    // only the moments this population needs are read (the rest fold away)
#pragma unroll
    for (int q = 0; q < P; ++q) Lam[q] = (q == p) ? M[(int64_t)q * n + cs] : 0.f;
    const int a = pair_a(D, p), b = pair_b(D, p);
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const bool need = i != 0 && ((e == b && cvel(D, i, a) != 0) || (e == a && cvel(D, i, b) != 0));
        Bb[e] = need ? M[(int64_t)(P + e) * n + cs] : 0.f;
    }
    const float g0 = dev_eq<D>(i, p, Lam, Bb, wc0_here);
    float s, inv;
    pow2_scale(cell_magnitude<D>(M, n, cs), s, inv);
    return g0 + dev_value<D, H, GH>(Dv, n, i, p, cs, s, wc0_here);
}

// Encode a post-collision state: its moments (FP32) and the scaled 16-bit
// deviations from the equilibrium of those moments.
template <int D, typename H, bool GH, bool NTS = false>
__device__ __forceinline__ void dev_store(const float (&out)[Lat<D>::Q][Lat<D>::P], float cl2, float wc0,
                                          int64_t n, int c, float* Mout, H* Dout)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    float rho2[P], K2[D], Lam2[P], Bb2[D];
    moments<D, float>(out, rho2, K2);
#pragma unroll
    for (int p = 0; p < P; ++p) Lam2[p] = cl2 * rho2[p];
#pragma unroll
    for (int b = 0; b < D; ++b) Bb2[b] = D == 2 ? K2[b] : 0.5f * K2[b];
#pragma unroll
    for (int p = 0; p < P; ++p) st_stream<NTS>(&Mout[(int64_t)p * n + c], Lam2[p]);
#pragma unroll
    for (int b = 0; b < D; ++b) st_stream<NTS>(&Mout[(int64_t)(P + b) * n + c], Bb2[b]);
    float m = 0.f;
#pragma unroll
    for (int p = 0; p < P; ++p) m = fmaxf(m, fabsf(Lam2[p]));
#pragma unroll
    for (int b = 0; b < D; ++b) m = fmaxf(m, fabsf(Bb2[b]));
    float s, inv;
    pow2_scale(m, s, inv);
    const float inv0 = inv / wc0, invm = 2.f * inv;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int sl = dev_slot<D, GH>(i, p);
            if (sl < 0) continue;
            const float d = out[i][p] - dev_eq<D>(i, p, Lam2, Bb2, wc0);
            st_stream<NTS>(&Dout[(int64_t)sl * n + c], f2h<H>(sat16<H>(d * (i == 0 ? inv0 : invm))));
        }
}

// Collide and encode in one pass (deviation formats, no cell extras).  The
// collision takes a state g with moments m = (Lambda, Bbar) to
// (1 - omega) g + omega g0(m) + T, and the source term T has the shape of an
// equilibrium: it moves each pair moment Lambda_p by -Sp_p and leaves K as it
// is.  The new moments are therefore (Lambda - Sp, Bbar), and the deviation of
// the new state from their equilibrium is (1 - omega)(g - g0(m)) exactly.
// Only that product is rounded; the post-collision populations are never
// formed and their moments never summed again.  M receives the stored FP32
// moments, code the stored 16-bit codes (slot order).
template <int D, typename H, bool GH>
__device__ __forceinline__ void dev_encode(const float (&f)[Lat<D>::Q][Lat<D>::P], float cl2, float wc0,
                                           const float (&Sp)[Lat<D>::P], bool any_src, float omega, bool tau_half,
                                           const float (&rho)[Lat<D>::P], const float (&K)[D],
                                           float (&M)[Lat<D>::P + D], H (&code)[DevSlots<D, GH>::N])
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    float Lam[P], Bb[D];
#pragma unroll
    for (int p = 0; p < P; ++p) Lam[p] = cl2 * rho[p];
#pragma unroll
    for (int b = 0; b < D; ++b) Bb[b] = D == 2 ? K[b] : 0.5f * K[b];
    float m = 0.f;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const float l2 = any_src ? Lam[p] - Sp[p] : Lam[p];
        M[p] = l2;
        m = fmaxf(m, fabsf(l2));
    }
#pragma unroll
    for (int b = 0; b < D; ++b) {
        M[P + b] = Bb[b];
        m = fmaxf(m, fabsf(Bb[b]));
    }
    float s, inv;
    pow2_scale(m, s, inv);
    const float f1 = tau_half ? -1.f : 1.f - omega;
    const float km = f1 * (2.f * inv);
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int sl = dev_slot<D, GH>(i, p);
            if (sl < 0) continue;
            float c;
            if (i == 0) c = (f[0][p] - (rho[p] - float(D) * Lam[p])) * (f1 * (inv / wc0));
            else c = (f[i][p] - 0.5f * twice_eq_moving<D, float>(i, p, Lam[p], Bb)) * km;
            code[sl] = f2h<H>(sat16<H>(c));
        }
}

template <int D, typename H, bool GH, bool NTS = false>
__device__ __forceinline__ void dev_collide_store(const float (&f)[Lat<D>::Q][Lat<D>::P], float cl2, float wc0,
                                                  const float (&Sp)[Lat<D>::P], bool any_src, float omega,
                                                  bool tau_half, const float (&rho)[Lat<D>::P],
                                                  const float (&K)[D], int64_t n, int c, float* Mout, H* Dout)
{
    constexpr int P = Lat<D>::P;
    float M[P + D];
    H code[DevSlots<D, GH>::N];
    dev_encode<D, H, GH>(f, cl2, wc0, Sp, any_src, omega, tau_half, rho, K, M, code);
#pragma unroll
    for (int q = 0; q < P + D; ++q) st_stream<NTS>(&Mout[(int64_t)q * n + c], M[q]);
#pragma unroll
    for (int sl = 0; sl < DevSlots<D, GH>::N; ++sl) st_stream<NTS>(&Dout[(int64_t)sl * n + c], code[sl]);
}

// NTS: streaming stores of the state (the gathered loads stay plain).  BX:
// 0 no cell extras; 1 walls only (they change the arrivals, not the
// collision, which keeps its closed form); 2 walls, dispersion and absorber.
template <int D, typename H, bool GH, int RM, int VEC, bool MU, int BX, bool NTS = false>
__global__ __launch_bounds__(NT) void k_step_dev(const float* Min, const H* Din, float* Mout, H* Dout,
                                                const float* __restrict__ cl2a, const float* __restrict__ dlnmu,
                                                const Geo g, const SrcArgs<float> s, const float omega,
                                                const int tau_half, const CellExt bc)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    __shared__ float lds[P * NT * VEC];
    const Tile t = tile_of(g, VEC);
    const bool has_src = stage_source<P, VEC, float>(s, t.b, lds);
    const bool any_src = has_src || MU;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const int y = t.y0 + v * t.rb;
        if (t.x >= g.nx || y >= g.ny) continue;
        Cell C = make_cell(g, t.x, y, t.z);
        if (BX && RM == R_PULL) mark_walls<D>(C, bc, g, t.x, y, t.z);
        const float cl2 = cl2a[C.c];
        const float wc0 = 1.f / cl2 - float(D);
        float f[Q][P];
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (BX && RM == R_PULL && ((C.wall >> i) & 1u)) {
                    const float v = dev_load<D, H, GH>(Min, Din, g.n, opp(D, i), p, C.c, wc0);
                    f[i][p] = wall_negates<D>(bc, i, p) ? -v : v;
                } else {
                    f[i][p] = dev_load<D, H, GH>(Min, Din, g.n, i, p, read_cell<D, RM>(C, i), wc0);
                }
            }
        float rho[P], K[D], Sp[P];
        moments<D, float>(f, rho, K);
#pragma unroll
        for (int p = 0; p < P; ++p) Sp[p] = has_src ? lds[p * NT * VEC + v * NT + threadIdx.x] : 0.f;
        if (MU) {
            float dl[D];
#pragma unroll
            for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * g.n + C.c];
            add_mu_source<D, float>(K, cl2, dl, Sp);
        }
        if constexpr (BX <= 1) {
            dev_collide_store<D, H, GH, NTS>(f, cl2, wc0, Sp, any_src, omega, tau_half != 0, rho, K, g.n, C.c,
                                             Mout, Dout);
        } else {
            float Jn[P];
            const bool ade = bc.ade != nullptr;
            if (ade) ade_update<D, float>(bc, g.n, C.c, cl2, rho, Jn);
            float out[Q][P];
            collide<D, float>(f, cl2, Sp, any_src, omega, tau_half != 0, rho, K, out);
            if (ade) {
#pragma unroll
                for (int p = 0; p < P; ++p) out[0][p] += Jn[p] / cl2;
            }
            if (bc.keep) {
                const float k = ((const float*)bc.keep)[C.c];
#pragma unroll
                for (int i = 0; i < Q; ++i)
#pragma unroll
                    for (int p = 0; p < P; ++p) out[i][p] *= k;
            }
            dev_store<D, H, GH, NTS>(out, cl2, wc0, g.n, C.c, Mout, Dout);
        }
    }
}

// ---------------------------------------------------------------------------
// 3D deviation storage, z-marching: neighbour moments staged in LDS
// ---------------------------------------------------------------------------
// A block owns a TXD x TYD column tile and a chunk of `lz` planes.  The FP32
// moments of planes z-1, z, z+1 (tile plus a one-cell halo, periodic) and the
// per-cell deviation scale sit in a rolling three-plane LDS window; the
// 16-bit deviations are read once from HBM.  The reconstruction uses the same
// formulas as dev_load, so the result equals k_step_dev bit for bit.
constexpr int TXD = 64, TYD = 4;

// NTS: streaming stores (the window, code and medium loads stay plain)
template <typename H, bool GH, int RM, bool MU, bool NTS = false>
__global__ __launch_bounds__(NT) void k_step_dev3z(const float* Min, const H* Din, float* Mout, H* Dout,
                                                  const float* __restrict__ cl2a, const float* __restrict__ dlnmu,
                                                  const Geo g, const int lz, const SrcArgs<float> s,
                                                  const float omega, const int tau_half)
{
    constexpr int D = 3, Q = 7, P = 3, NM = P + D;
    constexpr int W = TXD + 2, HH = TYD + 2, PC = W * HH;
    __shared__ float lm[3][NM][PC];
    __shared__ float lsc[3][PC];
    __shared__ float lsrc[P * NT];

    const int b = remap_block(blockIdx.x, g.nblocks, g.xcd);
    const int tx = b % g.tiles_x, r = b / g.tiles_x;
    const int ty = r % g.tiles_y, zc = r / g.tiles_y;
    const int x0 = tx * TXD, y0 = ty * TYD, z0 = zc * lz;
    const int z1 = min(z0 + lz, g.nz);
    const int lx = threadIdx.x % TXD, ly = threadIdx.x / TXD;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = x < g.nx && y < g.ny;
    const int hc = (ly + 1) * W + (lx + 1);

    // source entries of this block, sorted by local index (plane * NT + thread)
    int s0 = 0, s1 = 0;
    if (s.off) {
        s0 = s.off[b];
        s1 = s.off[b + 1];
    }
    const bool has_src = s1 > s0;
    const bool any_src = has_src || MU;

    // in-plane cells of the window entries this thread loads (the same in
    // every plane; periodic images wrapped once here)
    constexpr int KW = (PC + NT - 1) / NT;
    int off2d[KW];
#pragma unroll
    for (int j = 0; j < KW; ++j) {
        const int k = threadIdx.x + j * NT;
        const int hx = k % W, hy = k / W;
        int gx = (x0 - 1 + hx) % g.nx, gy = (y0 - 1 + hy) % g.ny;
        if (gx < 0) gx += g.nx;
        if (gy < 0) gy += g.ny;
        off2d[j] = gx + g.nx * gy;
    }
    const int nxy = g.nx * g.ny;
    // Window planes are fetched one iteration ahead into registers, so their
    // loads are in flight while the previous plane is updated.
    float pre[KW][NM];
    auto fetch_plane = [&](int zz) {
        zz %= g.nz;
        if (zz < 0) zz += g.nz;
        const int64_t zoff = (int64_t)zz * nxy;
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            if (threadIdx.x + j * NT >= PC) break;
            const int64_t c = zoff + off2d[j];
#pragma unroll
            for (int t = 0; t < NM; ++t) pre[j][t] = Min[(int64_t)t * g.n + c];
        }
    };
    auto stash_plane = [&](int q) {
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            const int k = threadIdx.x + j * NT;
            if (k >= PC) break;
            float m = 0.f;
#pragma unroll
            for (int t = 0; t < NM; ++t) {
                lm[q][t][k] = pre[j][t];
                m = fmaxf(m, fabsf(pre[j][t]));
            }
            float sv, iv;
            pow2_scale(m, sv, iv);
            lsc[q][k] = sv;
        }
    };

    fetch_plane(z0 - 1);
    stash_plane(0);
    fetch_plane(z0);
    stash_plane(1);
    fetch_plane(z0 + 1);
    for (int z = z0; z < z1; ++z) {
        const int rel = z - z0;
        const int qm = rel % 3, qc = (rel + 1) % 3, qp = (rel + 2) % 3;
        stash_plane(qp);                       // plane z + 1
        if (z + 1 < z1) fetch_plane(z + 2);    // lands during this plane's update
        if (has_src) {
            for (int k = threadIdx.x; k < P * NT; k += NT) lsrc[k] = 0.f;
            __syncthreads();
            for (int k = s0 + threadIdx.x; k < s1; k += NT) {
                const int2 e = s.ent[k];
                if (e.x / NT == rel) lsrc[e.y * NT + e.x % NT] = s.val[k] * s.amp;
            }
        }
        __syncthreads();
        if (active) {
            const Cell C = make_cell(g, x, y, z);
            const float cl2 = cl2a[C.c];
            const float wc0 = 1.f / cl2 - float(D);
            float f[Q][P];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                // source cell of population i in the LDS window
                const int ci_x = RM == R_LOCAL ? 0 : cvel(D, i, 0);
                const int ci_y = RM == R_LOCAL ? 0 : cvel(D, i, 1);
                const int ci_z = RM == R_LOCAL ? 0 : cvel(D, i, 2);
                const int q = ci_z > 0 ? qm : (ci_z < 0 ? qp : qc);
                const int hi = hc - ci_x - ci_y * W;
                const int cs = read_cell<D, RM>(C, i);
                const float sc = lsc[q][hi];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    float Lam[P], Bb[D];
#pragma unroll
                    for (int t = 0; t < P; ++t) Lam[t] = (t == p) ? lm[q][t][hi] : 0.f;
                    const int a = pair_a(D, p), bq = pair_b(D, p);
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        const bool need = i != 0 && ((e == bq && cvel(D, i, a) != 0) || (e == a && cvel(D, i, bq) != 0));
                        Bb[e] = need ? lm[q][P + e][hi] : 0.f;
                    }
                    const float g0 = dev_eq<D>(i, p, Lam, Bb, wc0);
                    f[i][p] = g0 + dev_value<D, H, GH>(Din, g.n, i, p, cs, sc, wc0);
                }
            }
            float rho[P], K[D], Sp[P];
            moments<D, float>(f, rho, K);
#pragma unroll
            for (int p = 0; p < P; ++p) Sp[p] = has_src ? lsrc[p * NT + threadIdx.x] : 0.f;
            if (MU) {
                float dl[D];
#pragma unroll
                for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * g.n + C.c];
                add_mu_source<D, float>(K, cl2, dl, Sp);
            }
            dev_collide_store<D, H, GH, NTS>(f, cl2, wc0, Sp, any_src, omega, tau_half != 0, rho, K, g.n, C.c,
                                             Mout, Dout);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3D deviation storage, row tiles: every stored cell decoded once
// ---------------------------------------------------------------------------
// A block of NTB threads owns `ty` whole x-rows (y0 .. y0+rows-1) of a chunk
// of `lz` planes and marches along z.  The tile's rows are contiguous in a
// plane; a thread owns up to CX of its cells, the ones at tile-flat indices
// threadIdx.x + k*NTB, so that every wave loads consecutive cells whatever
// the row length.  Per plane it reads its cells' stored moments and 16-bit
// codes once, with aligned loads, and decodes every outgoing population (rest
// and dropped ghost entries included) in FP32; the +-x and +-y ones go to LDS
// for the in-plane neighbours, the +-z and rest ones stay in registers for
// the planes the march visits next.  The rows y0-1 and y0+rows are decoded
// only for the +y / -y populations that enter the tile.  The update of plane
// z then pulls every population from LDS or registers.  The decoding and the
// collision are those of k_step_dev, so the two agree bit for bit.
constexpr int NTR = 1024;        // largest block
constexpr int ROWX_MAX = 1024;   // longest row

struct RowGeo {
    int nx, ny, nz;
    int ty;               // rows per tile (CX * NTB / nx)
    int tiles_y, lz, nblocks, xcd;
    int64_t n;
};

// in-plane velocities of the LDS exchange: j = 0 +x, 1 +y, 2 -x, 3 -y
__host__ __device__ constexpr int inplane_vel(int j) { return j == 0 ? 1 : (j == 1 ? 2 : (j == 2 ? 4 : 5)); }

// population (i,p) of a cell from its stored moments Mv, scale sc and codes
// (get), exactly as dev_load forms it
template <bool GH, class Get>
__device__ __forceinline__ float row_pop(const float (&Mv)[6], const Get& get, float sc, float wc0, int i, int p)
{
    constexpr int D = 3, P = 3;
    float Lam[P], Bb[D];
#pragma unroll
    for (int t = 0; t < P; ++t) Lam[t] = (t == p) ? Mv[t] : 0.f;
    const int a = pair_a(D, p), bq = pair_b(D, p);
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const bool need = i != 0 && ((e == bq && cvel(D, i, a) != 0) || (e == a && cvel(D, i, bq) != 0));
        Bb[e] = need ? Mv[P + e] : 0.f;
    }
    const float g0 = dev_eq<D>(i, p, Lam, Bb, wc0);
    return g0 + dev_value_of<D, GH>(get, i, p, sc, wc0);
}

__device__ __forceinline__ float row_scale(const float (&Mv)[6])
{
    float m = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) m = fmaxf(m, fabsf(Mv[t]));
    float s, inv;
    pow2_scale(m, s, inv);
    return s;
}

// populations (i, p = 0..2) of velocity i of cell c, reading only the
// moments and codes they need (halo rows, first and last plane of a chunk)
template <typename H, bool GH>
__device__ __forceinline__ void row_pops_of(const float* Min, const H* Din, int64_t n, int64_t c, int i,
                                            float (&out)[3])
{
    float Mv[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) Mv[t] = Min[(int64_t)t * n + c];
    const float sc = row_scale(Mv);
    auto get = [&](int sl) { return h2f<H>(Din[(int64_t)sl * n + c]); };
#pragma unroll
    for (int p = 0; p < 3; ++p) out[p] = row_pop<GH>(Mv, get, sc, 0.f, i, p);
}

// NTS: streaming stores of the state.  src_*: per (block, plane of the chunk)
// a range [off[b*lz + rel], off[b*lz + rel + 1]) of (row*nx + x, pair) entries
// with their value per unit amplitude.
// At least four waves per SIMD (<= 128 VGPRs): two 512-thread blocks per CU.
// With fewer, one block holds a CU and the latency of its loads between the
// barriers of a plane has nothing to hide it (measured 3.19 -> 4.38 ms at
// 512^3 when a change took the kernel to 141 VGPRs).  The Dev-Q
// instantiations with cell extras ask for three: at the four-wave target the
// scheduler issued their 21 code loads one at a time (load, wait, convert);
// at three it keeps them in flight and still allocates <= 128 VGPRs.
// One tile (block b of the tiling g) of the row-tile step; every thread of the
// block calls it (it holds barriers).  lp: 12 * CX * NTB floats, lh: 6 * RX
// floats of LDS.
template <int CX, int NTB>
struct RowLds {
    static constexpr int ROWC_MAX = CX * NTB;       // cells of one plane of the tile (ty * nx <= CX * NTB)
    static constexpr int RX = CX * NTB < ROWX_MAX ? CX * NTB : ROWX_MAX;   // longest row of this block size
    static constexpr int FLOATS = 12 * ROWC_MAX + 6 * RX;
};

// EXT: the cell extras as the per-cell kernel applies them, a bit mask (each
// combination compiles only its own code: wall branches in the same kernel
// as the general collision cost 45 % at 256^3).  Bit 1: walls -- a
// population that would enter through a wall face is the cell's own outgoing
// one in the opposite direction, with the reflection sign; the collision is
// unchanged, so walls alone keep the closed-form store.  Bit 2: the
// dispersion pole (ade_update before the collision, J/c^2 added to the rest
// particle after it) and the absorbing layer (the outgoing state scaled by
// 1 - sigma).  No anisotropy.
template <typename H, bool GH, bool MU, bool NTS, int CX, int NTB, int EXT = 0, bool HALO2 = false>
__device__ __forceinline__ void dev3r_tile(const float* Min, const H* Din, float* Mout, H* Dout,
                                           const float* __restrict__ cl2a, const float* __restrict__ dlnmu,
                                           const RowGeo& g, const int b, const int* __restrict__ soff,
                                           const int2* __restrict__ sent, const float* __restrict__ sval,
                                           const float amp, const float omega, const int tau_half, float* lp,
                                           float* lh, const CellExt& bc = CellExt{})
{
    constexpr int D = 3, Q = 7, P = 3, NM = P + D, NC = DevSlots<D, GH>::N;
    constexpr int ROWC_MAX = RowLds<CX, NTB>::ROWC_MAX;
    constexpr int RX = RowLds<CX, NTB>::RX;
    // lp: [j*3 + p][row*nx + x], the in-plane outgoing populations; lh:
    // [side*3 + p][x], +y of row y0-1 (side 0) and -y of row y0+rows (side 1)

    const int tyi = b % g.tiles_y, zc = b / g.tiles_y;
    const int y0 = tyi * g.ty, z0 = zc * g.lz;
    const int z1 = min(z0 + g.lz, g.nz);
    const int rows = min(g.ty, g.ny - y0);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int64_t n = g.n, nxy = (int64_t)nx * ny;
    const int64_t ty0 = (int64_t)y0 * nx;          // first cell of the tile within a plane
    const int yh0 = (y0 - 1 + ny) % ny, yh1 = (y0 + rows) % ny;
    const bool has_src = soff != nullptr;

    // cell k of the thread: tile-flat index fl (also its LDS slot and its
    // source key), row rr, column xs
    int fl[CX], rr[CX], xs[CX];
    bool ok[CX];
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        fl[k] = (int)threadIdx.x + k * NTB;
        rr[k] = fl[k] / nx;
        xs[k] = fl[k] - rr[k] * nx;
        ok[k] = rr[k] < rows;
    }
    auto wrapz = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };

    float pz_prev[CX][P], pz_cur[CX][P], rest_cur[CX][P], cl2_cur[CX];
    float mz_new[CX][P], pz_next[CX][P], rest_next[CX][P], cl2_next[CX];

    // decode plane zz of the own cells: in-plane populations to LDS (if
    // to_lds), -z to mz, +z to pz, rest to rs
    auto decode_plane = [&](int zz, bool to_lds, float (&mz)[CX][P], float (&pz)[CX][P], float (&rs)[CX][P],
                            float (&cl)[CX]) {
        const int64_t zo = (int64_t)zz * nxy + ty0;
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            if (!ok[k]) continue;
            const int64_t c = zo + fl[k];
            float Mv[NM], cd[NC];
#pragma unroll
            for (int t = 0; t < NM; ++t) Mv[t] = Min[(int64_t)t * n + c];
#pragma unroll
            for (int sl = 0; sl < NC; ++sl) cd[sl] = h2f<H>(Din[(int64_t)sl * n + c]);
            const float cl2 = cl2a[c];
            const float wc0 = 1.f / cl2 - float(D);
            cl[k] = cl2;
            const float sc = row_scale(Mv);
            auto get = [&](int sl) { return cd[sl]; };
#pragma unroll
            for (int p = 0; p < P; ++p) {
                rs[k][p] = row_pop<GH>(Mv, get, sc, wc0, 0, p);
                pz[k][p] = row_pop<GH>(Mv, get, sc, wc0, 3, p);
                mz[k][p] = row_pop<GH>(Mv, get, sc, wc0, 6, p);
            }
            if (to_lds) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        lp[(j * 3 + p) * ROWC_MAX + fl[k]] =
                            row_pop<GH>(Mv, get, sc, wc0, inplane_vel(j), p);
            }
        }
    };
    // the +y populations of row y0-1 and the -y ones of row y0+rows, plane zz.
    // HALO2: one pass per row, its velocity fixed at compile time; otherwise
    // one pass over both rows with the velocity chosen per item.  Which one
    // the compiler schedules better depends on the instantiation: for the
    // single-lattice ghost kernel the run-time velocity made the decode pick
    // its codes in branches and load them one at a time, while the two passes
    // make the Dev-Q and batched kernels issue their code loads one at a time.
    auto decode_halo = [&](int zz) {
        if constexpr (HALO2) {
            const int64_t r0 = (int64_t)zz * nxy + (int64_t)yh0 * nx;
            const int64_t r1 = (int64_t)zz * nxy + (int64_t)yh1 * nx;
            for (int x = threadIdx.x; x < nx; x += NTB) {
                float o[3];
                row_pops_of<H, GH>(Min, Din, n, r0 + x, 2, o);
#pragma unroll
                for (int p = 0; p < P; ++p) lh[(0 * 3 + p) * RX + x] = o[p];
            }
            for (int x = threadIdx.x; x < nx; x += NTB) {
                float o[3];
                row_pops_of<H, GH>(Min, Din, n, r1 + x, 5, o);
#pragma unroll
                for (int p = 0; p < P; ++p) lh[(1 * 3 + p) * RX + x] = o[p];
            }
        } else {
            for (int t = threadIdx.x; t < 2 * nx; t += NTB) {
                const int side = t >= nx, x = t - side * nx;
                const int64_t c = (int64_t)zz * nxy + (int64_t)(side ? yh1 : yh0) * nx + x;
                float o[3];
                row_pops_of<H, GH>(Min, Din, n, c, side ? 5 : 2, o);
#pragma unroll
                for (int p = 0; p < P; ++p) lh[(side * 3 + p) * RX + x] = o[p];
            }
        }
    };

    // prologue: +z populations of plane z0-1, all of plane z0 (with a wall
    // on z, plane 0 receives its own -z populations reflected instead)
    {
        const int zm = wrapz(z0 - 1);
        const bool zwall0 = (EXT & 1) && bc.kind[2] != 0 && z0 == 0;
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            if (!ok[k]) continue;
            float o[3];
            if (zwall0) {
                row_pops_of<H, GH>(Min, Din, n, ty0 + fl[k], 6, o);
#pragma unroll
                for (int p = 0; p < P; ++p) pz_prev[k][p] = wall_negates<D>(bc, 3, p) ? -o[p] : o[p];
                continue;
            }
            row_pops_of<H, GH>(Min, Din, n, (int64_t)zm * nxy + ty0 + fl[k], 3, o);
#pragma unroll
            for (int p = 0; p < P; ++p) pz_prev[k][p] = o[p];
        }
        decode_plane(z0, true, mz_new, pz_cur, rest_cur, cl2_cur);
        decode_halo(z0);
    }
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        // in-plane arrivals of plane z
        float arr[CX][4][P];
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            if (!ok[k]) continue;
            const int x = xs[k], i = fl[k];
            const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
            const int rc = i - x;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                arr[k][0][p] = lp[(0 * 3 + p) * ROWC_MAX + rc + xm];                       // +x from x-1
                arr[k][2][p] = lp[(2 * 3 + p) * ROWC_MAX + rc + xp];                       // -x from x+1
                arr[k][1][p] = rr[k] > 0 ? lp[(1 * 3 + p) * ROWC_MAX + i - nx]             // +y from y-1
                                         : lh[(0 * 3 + p) * RX + x];
                arr[k][3][p] = rr[k] < rows - 1 ? lp[(3 * 3 + p) * ROWC_MAX + i + nx]      // -y from y+1
                                                : lh[(1 * 3 + p) * RX + x];
            }
            if constexpr ((EXT & 1) != 0) {
                // wall faces: the own outgoing population in the opposite direction
                const bool wx = bc.kind[0] != 0, wy = bc.kind[1] != 0;
                const int y = y0 + rr[k];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (wx && x == 0) {                                                   // +x: own -x
                        const float v = lp[(2 * 3 + p) * ROWC_MAX + i];
                        arr[k][0][p] = wall_negates<D>(bc, 1, p) ? -v : v;
                    }
                    if (wx && x == nx - 1) {                                              // -x: own +x
                        const float v = lp[(0 * 3 + p) * ROWC_MAX + i];
                        arr[k][2][p] = wall_negates<D>(bc, 4, p) ? -v : v;
                    }
                    if (wy && y == 0) {                                                   // +y: own -y
                        const float v = lp[(3 * 3 + p) * ROWC_MAX + i];
                        arr[k][1][p] = wall_negates<D>(bc, 2, p) ? -v : v;
                    }
                    if (wy && y == ny - 1) {                                              // -y: own +y
                        const float v = lp[(1 * 3 + p) * ROWC_MAX + i];
                        arr[k][3][p] = wall_negates<D>(bc, 5, p) ? -v : v;
                    }
                }
            }
        }
        __syncthreads();
        // plane z+1: all of it while the march continues, else only its -z populations
        const int zn = wrapz(z + 1);
        if (z + 1 < z1) {
            decode_plane(zn, true, mz_new, pz_next, rest_next, cl2_next);
            decode_halo(zn);
        } else if ((EXT & 1) && bc.kind[2] != 0 && z == nz - 1) {
            // wall on z: the last plane receives its own +z populations reflected
#pragma unroll
            for (int k = 0; k < CX; ++k)
#pragma unroll
                for (int p = 0; p < P; ++p) mz_new[k][p] = wall_negates<D>(bc, 6, p) ? -pz_cur[k][p] : pz_cur[k][p];
        } else {
#pragma unroll
            for (int k = 0; k < CX; ++k) {
                if (!ok[k]) continue;
                float o[3];
                row_pops_of<H, GH>(Min, Din, n, (int64_t)zn * nxy + ty0 + fl[k], 6, o);
#pragma unroll
                for (int p = 0; p < P; ++p) mz_new[k][p] = o[p];
            }
        }
        // update plane z
        int s0 = 0, s1 = 0;
        if (has_src) {
            s0 = soff[b * g.lz + (z - z0)];
            s1 = soff[b * g.lz + (z - z0) + 1];
        }
        const bool any_src = s1 > s0 || MU;
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            if (!ok[k]) continue;
            const int64_t c = (int64_t)z * nxy + ty0 + fl[k];
            float f[Q][P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                f[0][p] = rest_cur[k][p];
                f[1][p] = arr[k][0][p];
                f[2][p] = arr[k][1][p];
                f[3][p] = pz_prev[k][p];
                f[4][p] = arr[k][2][p];
                f[5][p] = arr[k][3][p];
                f[6][p] = mz_new[k][p];
            }
            const float cl2 = cl2_cur[k];
            const float wc0 = 1.f / cl2 - float(D);
            float rho[P], K[D], Sp[P];
            moments<D, float>(f, rho, K);
#pragma unroll
            for (int p = 0; p < P; ++p) Sp[p] = 0.f;
            const int loc = fl[k];
            for (int e = s0; e < s1; ++e) {
                const int2 en = sent[e];
                if (en.x == loc) {
                    const float v = sval[e] * amp;
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        if (en.y == p) Sp[p] = v;
                }
            }
            if (MU) {
                float dl[D];
#pragma unroll
                for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * n + c];
                add_mu_source<D, float>(K, cl2, dl, Sp);
            }
            if constexpr ((EXT & 2) == 0) {
                dev_collide_store<D, H, GH, NTS>(f, cl2, wc0, Sp, any_src, omega, tau_half != 0, rho, K, n,
                                                 (int)c, Mout, Dout);
            } else {
                float Jn[P];
                const bool ade = bc.ade != nullptr;
                if (ade) ade_update<D, float>(bc, n, (int)c, cl2, rho, Jn);
                float out[Q][P];
                collide<D, float>(f, cl2, Sp, any_src, omega, tau_half != 0, rho, K, out);
                if (ade) {
#pragma unroll
                    for (int p = 0; p < P; ++p) out[0][p] += Jn[p] / cl2;
                }
                if (bc.keep) {
                    const float kp = ((const float*)bc.keep)[c];
#pragma unroll
                    for (int i = 0; i < Q; ++i)
#pragma unroll
                        for (int p = 0; p < P; ++p) out[i][p] *= kp;
                }
                dev_store<D, H, GH, NTS>(out, cl2, wc0, n, (int)c, Mout, Dout);
            }
        }
        // the march moves on one plane
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            cl2_cur[k] = cl2_next[k];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                pz_prev[k][p] = pz_cur[k][p];
                pz_cur[k][p] = pz_next[k][p];
                rest_cur[k][p] = rest_next[k][p];
            }
        }
        __syncthreads();
    }
}

template <typename H, bool GH, bool MU, bool NTS, int CX, int NTB, int EXT = 0>
__global__ __launch_bounds__(NTB, (EXT != 0 && !GH) ? 3 : 4) void k_step_dev3r(const float* Min, const H* Din, float* Mout, H* Dout,
                                                   const float* __restrict__ cl2a, const float* __restrict__ dlnmu,
                                                   const RowGeo g, const int* __restrict__ soff,
                                                   const int2* __restrict__ sent, const float* __restrict__ sval,
                                                   const float amp, const float omega, const int tau_half,
                                                   const CellExt bc)
{
    __shared__ float lds[RowLds<CX, NTB>::FLOATS];
    dev3r_tile<H, GH, MU, NTS, CX, NTB, EXT, GH && EXT == 0>(Min, Din, Mout, Dout, cl2a, dlnmu, g,
                                             remap_block(blockIdx.x, g.nblocks, g.xcd), soff, sent, sval, amp,
                                             omega, tau_half, lds, lds + 12 * RowLds<CX, NTB>::ROWC_MAX, bc);
}

// ---------------------------------------------------------------------------
// 3D deviation storage, two steps per launch (temporal blocking)
// ---------------------------------------------------------------------------
// The column tiling, z-march and LDS buffers of k_step_fused3d, on the 16-bit
// formats.  Step 1 runs on the tile grown by one cell (the frame) of plane zz:
// it decodes the pulled populations from the stored state exactly as a single
// step does (the pair moments and scale of the source cells come from an LDS
// window of plane zz and from registers for planes zz -+ 1), collides, and
// encodes the result as a single step would store it (dev_encode).  Instead of
// writing that encoding it decodes it at once, as every reader of it would,
// and hands the decoded populations to step 2 through LDS; step 2 on plane
// zz-1 of the tile collides and stores.  Two launches of the single-step
// kernel and one of this one therefore give the same bits.
template <typename H, bool GH, bool MU>
__global__ __launch_bounds__(NT) void k_step_dev3f(const float* Min, const H* Din, float* Mout, H* Dout,
                                                  const float* __restrict__ cl2a, const float* __restrict__ dlnmu,
                                                  const Geo g, const int lz, const FusedSrc<float> fs,
                                                  const AmpPack<float, 2> amps, const float omega,
                                                  const int tau_half)
{
    constexpr int D = 3, Q = 7, P = 3, NM = P + D, NSL = DevSlots<D, GH>::N;
    constexpr int TX = 64, TY = 4;
    constexpr int W = TX + 2, HH = TY + 2, FC = W * HH, TC = TX * TY;  // frame = tile + 1
    constexpr int WW = TX + 4, WH = TY + 4, WC = WW * WH;              // window = frame + 1
    constexpr int NRING = 2 * (WW - 2) + 2 * (WH - 2);                 // window minus frame and corners
    static_assert(TC == NT && NRING <= NT, "tile and window ring");
    constexpr int NIP = 5;                       // in-plane velocities 0, +x, +y, -x, -y
    constexpr int CF = (FC + NT - 1) / NT;       // frame cells per thread
    __shared__ float lin[NIP * P][FC];           // decoded in-plane outputs of plane zz-1 (frame)
    __shared__ float lpz[3][P][TC];
    __shared__ float lmz[P][TC];
    __shared__ float lsrc[2][P][FC];
    __shared__ float lw[NM][WC];                 // stored moments of plane zz over the window
    __shared__ float lws[WC];                    // and their per-cell scale

    const int b = remap_block(blockIdx.x, g.nblocks, g.xcd);
    const int tx = b % g.tiles_x, r = b / g.tiles_x;
    const int ty = r % g.tiles_y, zc = r / g.tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = zc * lz;
    const int z1 = min(z0 + lz, g.nz);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int hc = (ly + 1) * W + (lx + 1);
    const int nxy = g.nx * g.ny;

    int s0 = 0, s1 = 0;
    if (fs.off) {
        s0 = fs.off[b];
        s1 = fs.off[b + 1];
    }
    const bool has_src = s1 > s0;

    auto wrapx = [&](int v) { v %= g.nx; return v < 0 ? v + g.nx : v; };
    auto wrapy = [&](int v) { v %= g.ny; return v < 0 ? v + g.ny : v; };

    // this thread's frame cells (in-plane offset, window index) and ring cell
    int f2d[CF], fwin[CF];
    bool fact[CF];
#pragma unroll
    for (int j = 0; j < CF; ++j) {
        const int k = threadIdx.x + j * NT;
        const int hx = k % W, hy = k / W;
        fact[j] = k < FC;
        f2d[j] = wrapx(x0 - 1 + hx) + g.nx * wrapy(y0 - 1 + hy);
        fwin[j] = (hy + 1) * WW + (hx + 1);
    }
    int r2d = 0, rwin = 0;
    const bool ract = threadIdx.x < NRING;
    {
        const int k = threadIdx.x;
        int wx, wy;
        if (k < WW - 2) { wx = 1 + k; wy = 0; }
        else if (k < 2 * (WW - 2)) { wx = 1 + k - (WW - 2); wy = WH - 1; }
        else if (k < 2 * (WW - 2) + (WH - 2)) { wx = 0; wy = 1 + k - 2 * (WW - 2); }
        else { wx = WW - 1; wy = 1 + k - 2 * (WW - 2) - (WH - 2); }
        r2d = wrapx(x0 - 2 + wx) + g.nx * wrapy(y0 - 2 + wy);
        rwin = wy * WW + wx;
    }

    // stored moments of the frame cells for planes zz-1, zz, zz+1
    float mp[CF][NM], mc[CF][NM], mn[CF][NM];
    auto load_m = [&](int zz, float (&dst)[CF][NM]) {
        int gz = zz % g.nz;
        if (gz < 0) gz += g.nz;
        const int64_t zoff = (int64_t)gz * nxy;
#pragma unroll
        for (int j = 0; j < CF; ++j) {
            if (!fact[j]) continue;
#pragma unroll
            for (int t = 0; t < NM; ++t) dst[j][t] = Min[(int64_t)t * g.n + zoff + f2d[j]];
        }
    };
    auto scale_of = [](const float (&m)[NM]) {
        float mx = 0.f;
#pragma unroll
        for (int t = 0; t < NM; ++t) mx = fmaxf(mx, fabsf(m[t]));
        float sv, iv;
        pow2_scale(mx, sv, iv);
        return sv;
    };
    // decoded population (i,p) from stored moments mm and scale sc of its
    // source cell cs, for a reader with rest weight wc0 (as k_step_dev3z)
    auto pulled = [&](const float (&mm)[NM], float sc, int i, int p, int64_t cs, float wc0) {
        float Lam[P], Bb[D];
#pragma unroll
        for (int t = 0; t < P; ++t) Lam[t] = (t == p) ? mm[t] : 0.f;
        const int a = pair_a(D, p), bq = pair_b(D, p);
#pragma unroll
        for (int e = 0; e < D; ++e) {
            const bool need = i != 0 && ((e == bq && cvel(D, i, a) != 0) || (e == a && cvel(D, i, bq) != 0));
            Bb[e] = need ? mm[P + e] : 0.f;
        }
        const float g0 = dev_eq<D>(i, p, Lam, Bb, wc0);
        return g0 + dev_value<D, H, GH>(Din, g.n, i, p, (int)cs, sc, wc0);
    };

    load_m(z0 - 2, mp);
    load_m(z0 - 1, mc);
    load_m(z0, mn);
    for (int zz = z0 - 1; zz <= z1; ++zz) {
        const int rel = zz - (z0 - 1);
        const int bi = rel & 1;
        int gz = zz % g.nz;
        if (gz < 0) gz += g.nz;
        const int64_t zoff = (int64_t)gz * nxy;
        if (has_src) {
            for (int k = threadIdx.x; k < P * FC; k += NT) (&lsrc[bi][0][0])[k] = 0.f;
            __syncthreads();
            for (int k = s0 + threadIdx.x; k < s1; k += NT) {
                const int2 e = fs.ent[k];
                if (e.x / FC == rel) lsrc[bi][e.y][e.x % FC] = fs.val[k];
            }
        }
        // moments window of plane zz: the frame from registers, the ring from HBM
#pragma unroll
        for (int j = 0; j < CF; ++j) {
            if (!fact[j]) continue;
#pragma unroll
            for (int t = 0; t < NM; ++t) lw[t][fwin[j]] = mc[j][t];
            lws[fwin[j]] = scale_of(mc[j]);
        }
        if (ract) {
            float rm[NM];
#pragma unroll
            for (int t = 0; t < NM; ++t) {
                rm[t] = Min[(int64_t)t * g.n + zoff + r2d];
                lw[t][rwin] = rm[t];
            }
            lws[rwin] = scale_of(rm);
        }
        __syncthreads();
        // ---- step 1 on the frame cells of plane zz
        float held[CF][NIP * P];
#pragma unroll
        for (int j = 0; j < CF; ++j) {
            if (!fact[j]) continue;
            const int k = threadIdx.x + j * NT;
            const int hx = k % W, hy = k / W;
            const int64_t c = zoff + f2d[j];
            const int gx = f2d[j] % g.nx, gy = f2d[j] / g.nx;
            const float cl2 = cl2a[c];
            const float wc0 = 1.f / cl2 - float(D);
            float f[Q][P];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int cx = cvel(D, i, 0), cy = cvel(D, i, 1), cz = cvel(D, i, 2);
                int64_t cs;
                float sc;
                float mm[NM];
                if (cz == 0) {
                    const int wi = fwin[j] - cx - cy * WW;
#pragma unroll
                    for (int t = 0; t < NM; ++t) mm[t] = lw[t][wi];
                    sc = lws[wi];
                    cs = zoff + wrapx(gx - cx) + (int64_t)g.nx * wrapy(gy - cy);
                } else {
#pragma unroll
                    for (int t = 0; t < NM; ++t) mm[t] = cz > 0 ? mp[j][t] : mn[j][t];
                    sc = scale_of(mm);
                    int sz = (gz - cz) % g.nz;
                    if (sz < 0) sz += g.nz;
                    cs = (int64_t)sz * nxy + f2d[j];
                }
#pragma unroll
                for (int p = 0; p < P; ++p) f[i][p] = pulled(mm, sc, i, p, cs, wc0);
            }
            float rho[P], K[D], Sp[P];
            moments<D, float>(f, rho, K);
#pragma unroll
            for (int p = 0; p < P; ++p) Sp[p] = has_src ? lsrc[bi][p][k] * amps.a[0] : 0.f;
            if (MU) {
                float dl[D];
#pragma unroll
                for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * g.n + c];
                add_mu_source<D, float>(K, cl2, dl, Sp);
            }
            float M1[NM];
            H cd[NSL];
            dev_encode<D, H, GH>(f, cl2, wc0, Sp, has_src || MU, omega, tau_half != 0, rho, K, M1, cd);
            // decode the encoding as its readers will
            const float s1c = scale_of(M1);
            auto get = [&](int sl) { return h2f<H>(cd[sl]); };
            float out[Q][P];
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    float Lam[P], Bb[D];
#pragma unroll
                    for (int t = 0; t < P; ++t) Lam[t] = (t == p) ? M1[t] : 0.f;
                    const int a = pair_a(D, p), bq = pair_b(D, p);
#pragma unroll
                    for (int e = 0; e < D; ++e) {
                        const bool need = i != 0 && ((e == bq && cvel(D, i, a) != 0) || (e == a && cvel(D, i, bq) != 0));
                        Bb[e] = need ? M1[P + e] : 0.f;
                    }
                    out[i][p] = dev_eq<D>(i, p, Lam, Bb, wc0) + dev_value_of<D, GH>(get, i, p, s1c, wc0);
                }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int sl = i == 0 ? 0 : (i == 1 ? 1 : (i == 2 ? 2 : (i == 4 ? 3 : (i == 5 ? 4 : -1))));
                if (sl >= 0) {
#pragma unroll
                    for (int p = 0; p < P; ++p) held[j][sl * P + p] = out[i][p];
                }
            }
            const bool tile = hx >= 1 && hx <= TX && hy >= 1 && hy <= TY;
            if (tile) {
                const int tcell = (hy - 1) * TX + (hx - 1);
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    lpz[rel % 3][p][tcell] = out[3][p];
                    lmz[p][tcell] = out[6][p];
                }
            }
        }
        __syncthreads();
        // ---- step 2 on plane zz-1 of the tile
        const int zc2 = zz - 1;
        if (zc2 >= z0 && zc2 < z1) {
            const int x = x0 + lx, y = y0 + ly;
            if (x < g.nx && y < g.ny) {
                const int pb = (rel - 1) & 1;
                float f[Q][P];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    f[0][p] = lin[0 * P + p][hc];
                    f[1][p] = lin[1 * P + p][hc - 1];
                    f[2][p] = lin[2 * P + p][hc - W];
                    f[4][p] = lin[3 * P + p][hc + 1];
                    f[5][p] = lin[4 * P + p][hc + W];
                    f[3][p] = lpz[(rel + 1) % 3][p][threadIdx.x];
                    f[6][p] = lmz[p][threadIdx.x];
                }
                const int c = x + g.nx * (y + g.ny * zc2);
                const float cl2 = cl2a[c];
                const float wc0 = 1.f / cl2 - float(D);
                float rho[P], K[D], Sp[P];
                moments<D, float>(f, rho, K);
#pragma unroll
                for (int p = 0; p < P; ++p) Sp[p] = has_src ? lsrc[pb][p][hc] * amps.a[1] : 0.f;
                if (MU) {
                    float dl[D];
#pragma unroll
                    for (int a = 0; a < D; ++a) dl[a] = dlnmu[(int64_t)a * g.n + c];
                    add_mu_source<D, float>(K, cl2, dl, Sp);
                }
                dev_collide_store<D, H, GH>(f, cl2, wc0, Sp, has_src || MU, omega, tau_half != 0, rho, K, g.n, c,
                                            Mout, Dout);
            }
        }
        __syncthreads();
        // plane zz's decoded in-plane outputs into the frame buffer; roll the
        // moment registers one plane on
#pragma unroll
        for (int j = 0; j < CF; ++j) {
            if (!fact[j]) continue;
            const int k = threadIdx.x + j * NT;
#pragma unroll
            for (int q = 0; q < NIP * P; ++q) lin[q][k] = held[j][q];
#pragma unroll
            for (int t = 0; t < NM; ++t) {
                mp[j][t] = mc[j][t];
                mc[j][t] = mn[j][t];
            }
        }
        if (zz < z1) load_m(zz + 2, mn);
    }
}

// ---------------------------------------------------------------------------
// batched persistent stream-collide: many independent lattices per launch
// ---------------------------------------------------------------------------
// One descriptor per resident lattice.  Work items are (lattice, tile) pairs
// numbered by the prefix tile_base; a persistent grid strides over them.  The
// per-cell code is the same inline code as the single-lattice kernels, so a
// lattice advanced here is bit-identical to the same lattice stepped alone.
// Members may carry a current source (amplitudes per step of the tick) and a
// varying mu; cell extras (walls, absorber, dispersion, anisotropy) are not
// batched.
struct BatchGrid {
    void* buf[2];        // plain: population copies; dev: moment arrays
    void* dev[2];        // dev: deviation arrays (unused for plain)
    const void* cl2;
    const void* dlnmu;   // grad ln mu [D][n] (medium precision) when mu varies, else nullptr
    const int* src_off;  // the member's sparse current source, per tile of its own tiling, or nullptr
    const int2* src_ent;
    const void* src_val;
    const void* amp;     // [nsteps] source amplitudes of this tick (arithmetic type), or nullptr (zero)
    Geo geo;             // the member's own tiling (VEC = 1); tile ids match its source table
    double omega;
    int tau_half;
    int cur0;            // copy holding the state when the tick starts
    int fresh;           // state in the natural layout (first step)
    int nsteps;          // steps of this lattice in this tick
    int tile_base;       // first work item of this lattice
    int aa;              // plain formats stored in place (AA pattern); fresh then
                         // means the natural (even-step) layout at the tick start
    int row;             // 3D deviation member that also has the whole-row tiling
                         // rgeo (work items row_base.., source table rsrc_*)
    int row_base;
    RowGeo rgeo;
    const int* rsrc_off;
    const int2* rsrc_ent;
    const float* rsrc_val;
};

// A pointer read from the descriptor table, as a global-memory pointer.  The
// table holds generic pointers; read as such, every access through them
// compiles to a flat instruction, which also counts against the LDS counter,
// so an LDS wait can also wait for outstanding HBM loads.  Typed this way the
// batched kernels use global instructions, as the single-lattice kernels do
// with their kernel-argument pointers (alone, this measured no change in the
// time of the batched row tile).
template <typename T>
__device__ __forceinline__ T* gmem(const void* p)
{
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

struct BatchHdr {
    int count;           // lattices in the table
    int total_tiles;     // work items of the per-cell tiles
    int total_rows;      // work items of the whole-row tiles (all members row)
};

// the member that owns work item w (ROWS: of the whole-row numbering)
template <bool ROWS = false>
__device__ __forceinline__ int batch_find(const BatchGrid* __restrict__ tab, int count, int w)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((ROWS ? tab[mid].row_base : tab[mid].tile_base) <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Source of one tile of a member (the staging of the single-step kernels):
// every thread of the block takes part, before any of them leaves the tile.
template <int P, typename T>
__device__ __forceinline__ bool batch_source(const BatchGrid& G, int tile, int k, T* lds)
{
    SrcArgs<T> s;
    s.off = G.src_off ? gmem<const int>(G.src_off) : nullptr;
    s.ent = gmem<const int2>(G.src_ent);
    s.val = gmem<const T>(G.src_val);
    s.amp = G.amp ? gmem<const T>(G.amp)[k] : T(0);
    return stage_source<P, 1, T>(s, tile, lds);
}

// S: storage type of the populations (T itself, or FP16 under FP32 arithmetic)
template <int D, typename T, int RM, int WM, typename S>
__device__ __forceinline__ void batch_tile_plain(const BatchGrid& G, int tile, int k, T* lds)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    const Geo& g = G.geo;
    int tx, ty, z;
    tile_coords(g, tile, tx, ty, z);
    const int bx = 1 << g.bx_shift;
    const int x = tx * bx + (threadIdx.x & (bx - 1));
    const int y = ty * (NT >> g.bx_shift) + (threadIdx.x >> g.bx_shift);
    const bool has_src = batch_source<P, T>(G, tile, k, lds);
    const bool mu = G.dlnmu != nullptr;
    if (x >= g.nx || y >= g.ny) return;
    const int s = G.aa ? 0 : (G.cur0 + k) & 1;
    const S* src = gmem<const S>(G.buf[s]);
    S* dst = gmem<S>(G.buf[G.aa ? 0 : s ^ 1]);     // AA: in place, each location read and written by one thread
    const Cell C = make_cell(g, x, y, z);
    T f[Q][P];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p)
            f[i][p] = ld_pop<T>(src[(int64_t)(read_slot<D, RM>(i) * P + p) * g.n + read_cell<D, RM>(C, i)]);
    const T cl2 = gmem<const T>(G.cl2)[C.c];
    T rho[P], K[D], Sp[P];
    moments<D, T>(f, rho, K);
#pragma unroll
    for (int p = 0; p < P; ++p) Sp[p] = has_src ? lds[p * NT + threadIdx.x] : T(0);
    if (mu) {
        T dl[D];
#pragma unroll
        for (int a = 0; a < D; ++a) dl[a] = gmem<const T>(G.dlnmu)[(int64_t)a * g.n + C.c];
        add_mu_source<D, T>(K, cl2, dl, Sp);
    }
    T out[Q][P];
    collide<D, T>(f, cl2, Sp, has_src || mu, (T)G.omega, G.tau_half != 0, rho, K, out);
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p)
            dst[(int64_t)(write_slot<D, WM>(i) * P + p) * g.n + write_cell<D, WM>(C, i)] = st_pop<S>(out[i][p]);
}

template <int D, typename H, bool GH, int RM>
__device__ __forceinline__ void batch_tile_dev(const BatchGrid& G, int tile, int k, float* lds)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    const Geo& g = G.geo;
    int tx, ty, z;
    tile_coords(g, tile, tx, ty, z);
    const int bx = 1 << g.bx_shift;
    const int x = tx * bx + (threadIdx.x & (bx - 1));
    const int y = ty * (NT >> g.bx_shift) + (threadIdx.x >> g.bx_shift);
    const bool has_src = batch_source<P, float>(G, tile, k, lds);
    const bool mu = G.dlnmu != nullptr;
    if (x >= g.nx || y >= g.ny) return;
    const int s = (G.cur0 + k) & 1;
    const float* Min = gmem<const float>(G.buf[s]);
    const H* Din = gmem<const H>(G.dev[s]);
    float* Mout = gmem<float>(G.buf[s ^ 1]);
    H* Dout = gmem<H>(G.dev[s ^ 1]);
    const Cell C = make_cell(g, x, y, z);
    const float cl2 = gmem<const float>(G.cl2)[C.c];
    const float wc0 = 1.f / cl2 - float(D);
    float f[Q][P];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p)
            f[i][p] = dev_load<D, H, GH>(Min, Din, g.n, i, p, read_cell<D, RM>(C, i), wc0);
    float rho[P], K[D], Sp[P];
    moments<D, float>(f, rho, K);
#pragma unroll
    for (int p = 0; p < P; ++p) Sp[p] = has_src ? lds[p * NT + threadIdx.x] : 0.f;
    if (mu) {
        float dl[D];
#pragma unroll
        for (int a = 0; a < D; ++a) dl[a] = gmem<const float>(G.dlnmu)[(int64_t)a * g.n + C.c];
        add_mu_source<D, float>(K, cl2, dl, Sp);
    }
    dev_collide_store<D, H, GH>(f, cl2, wc0, Sp, has_src || mu, (float)G.omega, G.tau_half != 0, rho, K, g.n,
                                C.c, Mout, Dout);
}

// Launch k of a tick: every lattice with k < nsteps advances one step.
template <int D, typename T, typename S = T>
__global__ __launch_bounds__(NT) void k_step_batch_plain(const BatchHdr* __restrict__ hdr,
                                                        const BatchGrid* __restrict__ tab, int k)
{
    __shared__ T lds[Lat<D>::P * NT];
    const int count = hdr->count, total = hdr->total_tiles;
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int gi = batch_find(tab, count, w);
        const BatchGrid& G = tab[gi];
        if (k >= G.nsteps) continue;
        if (G.aa) {
            // even steps from the natural layout, odd ones from the swapped one
            if ((G.fresh != 0) == ((k & 1) == 0)) batch_tile_plain<D, T, R_LOCAL, W_SWAP, S>(G, w - G.tile_base, k, lds);
            else batch_tile_plain<D, T, R_PULL_SWAP, W_PUSH, S>(G, w - G.tile_base, k, lds);
        } else if (G.fresh && k == 0) {
            batch_tile_plain<D, T, R_LOCAL, W_LOCAL, S>(G, w - G.tile_base, k, lds);
        } else {
            batch_tile_plain<D, T, R_PULL, W_LOCAL, S>(G, w - G.tile_base, k, lds);
        }
        __syncthreads();   // the next work item may stage its source into lds
    }
}

template <int D, typename H, bool GH>
__global__ __launch_bounds__(NT) void k_step_batch_dev(const BatchHdr* __restrict__ hdr,
                                                      const BatchGrid* __restrict__ tab, int k)
{
    __shared__ float lds[Lat<D>::P * NT];
    const int count = hdr->count, total = hdr->total_tiles;
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int gi = batch_find(tab, count, w);
        const BatchGrid& G = tab[gi];
        if (k >= G.nsteps) continue;
        if (G.fresh && k == 0) batch_tile_dev<D, H, GH, R_LOCAL>(G, w - G.tile_base, k, lds);
        else batch_tile_dev<D, H, GH, R_PULL>(G, w - G.tile_base, k, lds);
        __syncthreads();   // the next work item may stage its source into lds
    }
}

// 3D deviation members on the whole-row tiling (rows of up to 2 BROW_NT
// cells): the row-tile step, work items numbered by row_base (the member's
// RowGeo blocks), BROW_NT threads per block.  A tick launches it for steps after its first when every member of
// the class is on that tiling and all or none of them have a varying mu (MU);
// otherwise, and for the first step (which may start from the natural layout),
// the per-cell kernel above.  This kernel holds nothing but the row tile: with
// the per-cell paths or a run-time mu branch in the same kernel the compiler
// issues the code loads of a plane one at a time (measured 1.8x slower).
constexpr int BROW_NT = 512;
template <typename H, bool GH, bool MU>
__global__ __launch_bounds__(BROW_NT, 4) void k_step_batch_dev3_rows(const BatchHdr* __restrict__ hdr,
                                                                  const BatchGrid* __restrict__ tab, int k)
{
    constexpr int CX = 2;
    using L = RowLds<CX, BROW_NT>;
    __shared__ float lds[L::FLOATS];
    const int count = hdr->count, total = hdr->total_rows;
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int gi = batch_find<true>(tab, count, w);
        const BatchGrid& G = tab[gi];
        if (k >= G.nsteps) continue;
        const int s = (G.cur0 + k) & 1;
        const RowGeo rg = G.rgeo;       // held in registers: the tile's stores cannot alias it
        dev3r_tile<H, GH, MU, false, CX, BROW_NT>(
            gmem<const float>(G.buf[s]), gmem<const H>(G.dev[s]), gmem<float>(G.buf[s ^ 1]), gmem<H>(G.dev[s ^ 1]),
            gmem<const float>(G.cl2), MU ? gmem<const float>(G.dlnmu) : nullptr, rg, w - G.row_base,
            G.rsrc_off ? gmem<const int>(G.rsrc_off) : nullptr, gmem<const int2>(G.rsrc_ent),
            gmem<const float>(G.rsrc_val), G.amp ? gmem<const float>(G.amp)[k] : 0.f, (float)G.omega, G.tau_half,
            lds, lds + 12 * L::ROWC_MAX);
    }
}

// ---------------------------------------------------------------------------
// readers for the field / diagnostic kernels
// ---------------------------------------------------------------------------
template <int D, typename S, int RM>
struct PlainReader {
    const S* pop;
    int64_t n;
    CellExt bc;
    static constexpr bool PULL = RM == R_PULL;
    using Wide = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
    __device__ __forceinline__ double get(const Cell& C, int i, int p, double) const
    {
        if (PULL && ((C.wall >> i) & 1u)) {
            const double v = (double)ld_pop<Wide>(pop[(int64_t)(opp(D, i) * Lat<D>::P + p) * n + C.c]);
            return wall_negates<D>(bc, i, p) ? -v : v;
        }
        return (double)ld_pop<Wide>(pop[(int64_t)(read_slot<D, RM>(i) * Lat<D>::P + p) * n + read_cell<D, RM>(C, i)]);
    }
};

template <int D, typename H, bool GH, int RM>
struct DevReader {
    const float* M;
    const H* Dv;
    int64_t n;
    CellExt bc;
    static constexpr bool PULL = RM == R_PULL;
    __device__ __forceinline__ double get(const Cell& C, int i, int p, double cl2) const
    {
        const float wc0 = 1.f / (float)cl2 - float(D);
        if (PULL && ((C.wall >> i) & 1u)) {
            const float v = dev_load<D, H, GH>(M, Dv, n, opp(D, i), p, C.c, wc0);
            return (double)(wall_negates<D>(bc, i, p) ? -v : v);
        }
        return (double)dev_load<D, H, GH>(M, Dv, n, i, p, read_cell<D, RM>(C, i), wc0);
    }
};

// ---------------------------------------------------------------------------
// E, B and FP64 diagnostics.  Deterministic two-pass reductions: per-block
// partials in a fixed tree order, then one block sums the partials.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

struct Geo1 {
    int nx, ny, nz;
    int64_t n;
};

// partials layout: [block][4] = {energy, Q_c, (div B)^2, |B|^2}
template <int D, typename TM, class R>
__global__ __launch_bounds__(NT) void k_fields(const R rd, const TM* __restrict__ cl2a,
                                               const double* __restrict__ mu_r, const Geo1 g1,
                                               double* E, double* B, double* partials,
                                               const TM* __restrict__ ra)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    __shared__ double sh[4];
    const int64_t c64 = (int64_t)blockIdx.x * NT + threadIdx.x;
    double en = 0.0, qc = 0.0, b2 = 0.0;
    if (c64 < g1.n) {
        const int c = (int)c64;
        const int x = c % g1.nx, y = (c / g1.nx) % g1.ny, z = c / (g1.nx * g1.ny);
        Geo g;
        g.nx = g1.nx; g.ny = g1.ny; g.nz = g1.nz;
        Cell C = make_cell(g, x, y, z);
        if (R::PULL && rd.bc.walls()) mark_walls<D>(C, rd.bc, g, x, y, z);
        const double cl2 = (double)cl2a[c];
        double f[Q][P];
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int p = 0; p < P; ++p) f[i][p] = rd.get(C, i, p, cl2);
        double rho[P], K[D];
        moments<D, double>(f, rho, K);
        double Ev[3] = {0.0, 0.0, 0.0}, Bv[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < P; ++p) Ev[pair_g(D, p)] = -(double)pair_s(D, p) * (cl2 * rho[p]);
#pragma unroll
        for (int b = 0; b < D; ++b) Bv[b] = K[b];
        if (E) {
#pragma unroll
            for (int k = 0; k < 3; ++k) E[(int64_t)k * g1.n + c] = Ev[k];
        }
        if (B) {
#pragma unroll
            for (int k = 0; k < 3; ++k) B[(int64_t)k * g1.n + c] = Bv[k];
        }
        if (partials) {
            const double mu = mu_r ? mu_r[c] : 1.0;
            const double eps_abs = (double)(D - 1) / (mu * cl2);
            const double e2 = Ev[0] * Ev[0] + Ev[1] * Ev[1] + Ev[2] * Ev[2];
            b2 = Bv[0] * Bv[0] + Bv[1] * Bv[1] + Bv[2] * Bv[2];
            en = eps_abs * e2 + b2 / mu;
            double rr[D], rs = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                rr[a] = ra ? (double)ra[(int64_t)a * g1.n + c] : 1.0;
                rs += rr[a];
            }
            const double w0 = 1.0 - rs * cl2;
            double sm = 0.0, s0 = 0.0;
#pragma unroll
            for (int p = 0; p < P; ++p) s0 += f[0][p] * f[0][p];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                double si = 0.0;
#pragma unroll
                for (int p = 0; p < P; ++p) si += f[i][p] * f[i][p];
                sm += ra ? si / rr[vaxis(D, i)] : si;
            }
            // c_L^2 / w_i = 2 / r_a for moving particles; rest skipped when w0 = 0
            qc = 2.0 * sm + (w0 > 0.0 ? cl2 / w0 * s0 : 0.0);
        }
    }
    if (partials) {
        const double a = block_sum(en, sh);
        const double q = block_sum(qc, sh);
        const double bb = block_sum(b2, sh);
        if (threadIdx.x == 0) {
            partials[blockIdx.x * 4 + 0] = a;
            partials[blockIdx.x * 4 + 1] = q;
            partials[blockIdx.x * 4 + 3] = bb;
        }
    }
}

template <int D>
__global__ __launch_bounds__(NT) void k_divb(const double* __restrict__ B, const Geo1 g1, double* partials)
{
    __shared__ double sh[4];
    const int64_t c64 = (int64_t)blockIdx.x * NT + threadIdx.x;
    double dv2 = 0.0;
    if (c64 < g1.n) {
        const int c = (int)c64;
        const int x = c % g1.nx, y = (c / g1.nx) % g1.ny, z = c / (g1.nx * g1.ny);
        Geo g;
        g.nx = g1.nx; g.ny = g1.ny; g.nz = g1.nz;
        const Cell C = make_cell(g, x, y, z);
        double d = 0.5 * (B[C.xp] - B[C.xm]);
        d += 0.5 * (B[g1.n + C.yp] - B[g1.n + C.ym]);
        if (D == 3) d += 0.5 * (B[2 * g1.n + C.zp] - B[2 * g1.n + C.zm]);
        dv2 = d * d;
    }
    const double r = block_sum(dv2, sh);
    if (threadIdx.x == 0) partials[blockIdx.x * 4 + 2] = r;
}

__global__ __launch_bounds__(NT) void k_reduce_partials(const double* __restrict__ partials, int nb, double* out)
{
    __shared__ double sh[4];
    for (int k = 0; k < 4; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += NT) s += partials[b * 4 + k];
        const double r = block_sum(s, sh);
        if (threadIdx.x == 0) out[k] = r;
    }
}

// ---------------------------------------------------------------------------
// set-up kernels: medium preparation and equilibrium initialisation
// ---------------------------------------------------------------------------

// c_L^2 = (1 - w0_vac)/(D eps_r mu_r); flag |= 1 when w0 = 1 - D c_L^2 is not
// in [0,1) or an input is not a positive finite number.
template <typename TM>
__global__ __launch_bounds__(NT) void k_medium(const double* __restrict__ eps, const double* __restrict__ mu,
                                               int D, double w0_vac, const Geo1 g1, TM* cl2, double* mu_out,
                                               TM* dlnmu, int* flag, const CellExt bc)
{
    const int64_t c64 = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (c64 >= g1.n) return;
    const int c = (int)c64;
    const double e = eps[c], m = mu ? mu[c] : 1.0;
    bool bad = !(e > 0.0) || !(m > 0.0) || !isfinite(e) || !isfinite(m);
    const double cl = (1.0 - w0_vac) / ((double)D * e * m);
    const double w0 = 1.0 - (double)D * cl;
    bad = bad || !(w0 >= 0.0 && w0 < 1.0);
    if (bad) atomicOr(flag, 1);
    cl2[c] = (TM)cl;
    if (mu_out) {
        mu_out[c] = m;
        const int x = c % g1.nx, y = (c / g1.nx) % g1.ny, z = c / (g1.nx * g1.ny);
        Geo g;
        g.nx = g1.nx; g.ny = g1.ny; g.nz = g1.nz;
        Cell C = make_cell(g, x, y, z);
        // beside a wall the medium is mirrored: the missing neighbour is the cell itself
        if (bc.kind[0] && x == 0) C.xm = c;
        if (bc.kind[0] && x == g1.nx - 1) C.xp = c;
        if (bc.kind[1] && y == 0) C.ym = c;
        if (bc.kind[1] && y == g1.ny - 1) C.yp = c;
        if (bc.kind[2] && z == 0) C.zm = c;
        if (bc.kind[2] && z == g1.nz - 1) C.zp = c;
        const double mxp = mu ? mu[C.xp] : 1.0, mxm = mu ? mu[C.xm] : 1.0;
        const double myp = mu ? mu[C.yp] : 1.0, mym = mu ? mu[C.ym] : 1.0;
        dlnmu[c] = (TM)(0.5 * (log(mxp) - log(mxm)));
        dlnmu[g1.n + c] = (TM)(0.5 * (log(myp) - log(mym)));
        if (D == 3) {
            const double mzp = mu ? mu[C.zp] : 1.0, mzm = mu ? mu[C.zm] : 1.0;
            dlnmu[2 * g1.n + c] = (TM)(0.5 * (log(mzp) - log(mzm)));
        }
    }
}

// Equilibrium of E0, B0 with Lambda_p = -sgn(p) E_gamma(p), Bbar = B/(D-1),
// written in the natural (pre-collision, local) layout.
template <int D>
__device__ __forceinline__ void init_eq(const double* E, const double* B, int64_t n, int c, double cl2,
                                        double (&g0)[Lat<D>::Q][Lat<D>::P], double (&Lam)[Lat<D>::P],
                                        double (&Bb)[D], const double (&r)[D])
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    double rs = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) rs += r[a];
#pragma unroll
    for (int p = 0; p < P; ++p) Lam[p] = -(double)pair_s(D, p) * E[(int64_t)pair_g(D, p) * n + c];
#pragma unroll
    for (int b = 0; b < D; ++b) Bb[b] = B[(int64_t)b * n + c] / (rs - r[b]);
    const double w0 = 1.0 - rs * cl2;
    const double wc = w0 / cl2;
#pragma unroll
    for (int p = 0; p < P; ++p) g0[0][p] = wc * Lam[p];
#pragma unroll
    for (int i = 1; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) g0[i][p] = 0.5 * r[vaxis(D, i)] * twice_eq_moving<D, double>(i, p, Lam[p], Bb);
}

// per-axis ratios of one cell (1 when isotropic)
template <int D, typename TM>
__device__ __forceinline__ void ratios(const TM* ra, int64_t n, int c, double (&r)[D])
{
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = ra ? (double)ra[(int64_t)a * n + c] : 1.0;
}

// Anisotropy: factors f_a on the isotropic c_L^2 give the per-axis second
// moments s_a = f_a c_L^2; c_L^2 becomes their mean and ra the ratios
// s_a / c^2.  flag is set where the rest weight 1 - sum s_a leaves [0,1).
template <typename TM>
__global__ __launch_bounds__(NT) void k_aniso(const double* __restrict__ fac, int D, int64_t n, TM* cl2, TM* ra,
                                              int* flag, int write)
{
    const int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (c >= n) return;
    const double cb = (double)cl2[c];
    double s[3], sum = 0.0;
    bool bad = false;
    for (int a = 0; a < D; ++a) {
        const double f = fac[a * n + c];
        bad = bad || !(f > 0.0) || !isfinite(f);
        s[a] = f * cb;
        sum += s[a];
    }
    const double w0 = 1.0 - sum;
    bad = bad || !(w0 >= 0.0 && w0 < 1.0);
    if (bad) atomicOr(flag, 1);
    if (bad || !write) return;   // the first pass only validates, so a rejected call changes nothing
    const double cbar = sum / (double)D;
    for (int a = 0; a < D; ++a) ra[a * n + c] = (TM)(s[a] / cbar);
    cl2[c] = (TM)cbar;
}

template <int D, typename T, typename S = T>
__global__ __launch_bounds__(NT) void k_init_plain(const double* __restrict__ E, const double* __restrict__ B,
                                                   const T* __restrict__ cl2a, int64_t n, S* pop,
                                                   const T* __restrict__ ra)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    const int64_t c64 = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (c64 >= n) return;
    const int c = (int)c64;
    double g0[Q][P], Lam[P], Bb[D], r[D];
    ratios<D, T>(ra, n, c, r);
    init_eq<D>(E, B, n, c, (double)cl2a[c], g0, Lam, Bb, r);
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) pop[(int64_t)(i * P + p) * n + c] = st_pop<S>((T)g0[i][p]);
}

template <int D, typename H, bool GH>
__global__ __launch_bounds__(NT) void k_init_dev(const double* __restrict__ E, const double* __restrict__ B,
                                                 const float* __restrict__ cl2a, int64_t n, float* M, H* Dv)
{
    constexpr int Q = Lat<D>::Q, P = Lat<D>::P;
    const int64_t c64 = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (c64 >= n) return;
    const int c = (int)c64;
    const float cl2 = cl2a[c];
    double g0[Q][P], Lam[P], Bb[D];
    double r1[D];
#pragma unroll
    for (int a = 0; a < D; ++a) r1[a] = 1.0;   // the 16-bit formats are isotropic
    init_eq<D>(E, B, n, c, (double)cl2, g0, Lam, Bb, r1);
    float Lf[P], Bf[D];
#pragma unroll
    for (int p = 0; p < P; ++p) Lf[p] = (float)Lam[p];
#pragma unroll
    for (int b = 0; b < D; ++b) Bf[b] = (float)Bb[b];
#pragma unroll
    for (int p = 0; p < P; ++p) M[(int64_t)p * n + c] = Lf[p];
#pragma unroll
    for (int b = 0; b < D; ++b) M[(int64_t)(P + b) * n + c] = Bf[b];
    const float wc0 = 1.f / cl2 - float(D);
    float m = 0.f;
#pragma unroll
    for (int p = 0; p < P; ++p) m = fmaxf(m, fabsf(Lf[p]));
#pragma unroll
    for (int b = 0; b < D; ++b) m = fmaxf(m, fabsf(Bf[b]));
    float s, inv;
    pow2_scale(m, s, inv);
    const float inv0 = inv / wc0, invm = 2.f * inv;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int sl = dev_slot<D, GH>(i, p);
            if (sl < 0) continue;
            const float d = (float)(g0[i][p] - (double)dev_eq<D>(i, p, Lf, Bf, wc0));
            Dv[(int64_t)sl * n + c] = f2h<H>(sat16<H>(d * (i == 0 ? inv0 : invm)));
        }
}

}  // namespace lbem
