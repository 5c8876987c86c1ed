// Device code of the FWI-gradient library (gfx950).
//
// Work item = (medium, group of G transmits).  Its wavefields are stored
// transmit-interleaved, [nz][nx][G], so one lane loads the G values of a
// cell with one vector load and the per-cell medium coefficients are read
// once for G transmits.
//
// Per cell the medium is reduced to two numbers, (Q, bt):
//   bt = rho_ref / rho                       (normalised buoyancy),
//   Q  = gamma kappa / (h^2 rho_ref),        gamma = dt^2 / (1 + D dt),
// so that gamma kappa (L_b v)_x = Q_x * sum_f bt_f (v_x' - v_x) with the
// face value bt_f = (bt_x + bt_x')/2 (bt_x on a border face, where the
// ghost field is 0) -- the flux form of eq. 1's density term.  The
// damping enters through a = (2 - e^2)/(1 + e) and beta = (e - 1)/(1 + e),
// e = D dt (eq. 2), rebuilt per cell from two 1-D profiles; inside the
// absorbing layer only, since a = 2 and beta = -1 elsewhere.
//
// One launch advances every active item by one step of its own schedule:
//   FWD     u^{n+1} = a u^n + beta u^{n-1} + Q L u^n, + w[n] at the source,
//           traces d[n] = u^{n+1}[rcv]                        (eq. 2-3),
//           evaluated in increment form (v = u^n - u^{n-1} carried, below)
//   RECOMP  the same update without sampling, re-running a checkpointed
//           segment into the segment buffer
//   ADJ     lam^{t-1} = a lam^t + L(Q lam^t) + beta lam^{t+1} + s[t-2] at rcv,
//           and the zero-lag imaging of lam^t with u^{t-1}   (eq. 6)
// with the schedule: T forward steps; then the last segment's adjoint steps;
// then, per earlier segment, K recompute steps followed by K adjoint steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fwi {

constexpr double kRhoRef = 1000.0;   // reference density (water, the paper's rho_0)
constexpr int kTileX = 64;           // cells per tile row = one wavefront
constexpr int kWavesZ = 4;           // wavefronts per workgroup, stacked in z
constexpr int kBlock = kTileX * kWavesZ;

enum Phase : int { kIdle = 0, kFwd = 1, kRecomp = 2, kAdj = 3 };
enum RunMode : int { kRunAll = 0, kRunFwdOnly = 1, kRunAdjOnly = 2 };

// Status bits raised on the device.
enum : unsigned { kFlagCfl = 1u, kFlagMedium = 2u, kFlagNonfinite = 4u, kFlagBarrier = 8u };

// One receiver entry of a tile: field slot cell*G + g, and the offset of
// trace (transmit, receiver) sample 0 in the medium's trace array.
// Entries of a tile are sorted by slot; ``run`` > 0 marks the first entry of
// a run of equal slots and gives its length (0 on the others).
struct Entry {
    int32_t slot;
    int32_t trace_off;
    int32_t run;
    int32_t pad;
};

// Quotient of a non-negative 31-bit value by a divisor d >= 1 fixed at plan
// creation, as a multiply-high and a shift (Granlund and Montgomery,
// "Division by invariant integers using multiplication", 1994, Thm. 4.2 with
// N = 32): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1 (below
// 2^32), floor(n / d) = (mulhi(m, n) + n) >> l for 0 <= n < 2^31, where the
// sum stays below 2^32.  Wave-uniform operands keep it on the scalar unit;
// the hardware has no integer divide, so n / d with d known only at run time
// costs a dozen vector instructions and a long dependent chain.
struct Div {
    uint32_t m, l;
};

inline Div make_div(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    return Div{(uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1), l};
}

__host__ __device__ __forceinline__ int quo(int n, Div v)
{
    const uint32_t t = (uint32_t)(((uint64_t)(uint32_t)n * v.m) >> 32);
    return (int)((t + (uint32_t)n) >> v.l);
}

// Schedule constants of an item (T steps, interval K, J segments, S
// forward-type and Sa adjoint steps per launch): the launch counts of its
// runs and the dividers that decoding a launch index needs.
struct Sched {
    int32_t T, K, J, S, Sa;
    int32_t nf, last, nl, nkf, nb;   // forward launches, last segment's levels and adjoint launches, per-segment counts
    Div dK, dnb;
};

template <typename T, typename Acc>
struct Item {
    int32_t nx, nz, nt, g_used;      // g_used <= G real transmits
    int32_t K, J, tiles_x, n_tiles;
    int32_t n_rcv, tx0, inject_adj, sample;   // inject_adj: 1 if d_adj drives the adjoint
    int32_t S, nlam;                 // forward-type steps fused per launch; lambda planes (lam^tau in tau mod nlam)
    int32_t keep_from, Sa;           // first level the adjoint reads from the first forward pass; adjoint steps per launch
    int64_t plane;                   // elements per field plane = nx*nz*G
    int64_t wavelet_stride;
    const T* coef;                   // [nz*nx] x (Q, bt)
    const T* ex;                     // [nx]  Dx(ix) dt
    const T* ez;                     // [nz]  Dz(iz) dt
    T* seg;                          // K planes
    T* ck;                           // 2 (J-1) planes: pair of segment j >= 1 at 2(j-1): v^{jK}, u^{jK}
    T* lam;                          // nlam planes
    T* vel;                          // 2 planes: v^tau = u^tau - u^{tau-1} in slot (tau / 2) mod 2
    Acc* acc;                        // [2][nz*nx]: S_kappa, S_b
    const T* zero;                   // zero plane
    const T* wavelet;                // transmit tx row at wavelet + tx * wavelet_stride
    const int32_t* src;              // [G] source cells, -1 for padding slots
    T* traces;                       // medium's [n_tx][nt][n_rcv]
    const T* d_obs;
    const T* d_adj;
    const int32_t* tile_off;         // [n_tiles + 1]: receivers inside each tile
    const Entry* entries;
    const int32_t* tile_off_x;       // [n_tiles + 1]: receivers inside each tile grown by one cell
    const Entry* entries_x;
    const T* eatt;                   // [nz*nx] attenuation eta dt added to the damping e, or NULL
    Sched sc;                        // schedule constants (nt, K, J, S, Sa)
    Div dtx, dnx;                    // dividers by tiles_x and nx
};

template <typename T, int G>
struct alignas(sizeof(T) * G) Vec {
    T v[G];
};

// ---------------------------------------------------------------- dual numbers
//
// A value and its derivative along one direction of the medium, (x, x').
// Instantiating the one-step kernels on Dual<S> differentiates the whole
// gradient computation forward along that direction: the forward fields
// carry their tangent-linear perturbation, the adjoint fields the
// second-order adjoint (its source 2 d' comes from the traces' tangents),
// and the imaging sums their derivatives -- so the gradient's tangent is
// the Hessian-vector product of the misfit, exact up to rounding.  Every
// operation below is the product or quotient rule written with explicit
// fused multiply-adds and contraction off, so a kernel rounds the same way
// on every pass (checkpointed replay stays bitwise).
template <typename S>
struct Dual {
    S v, d;
    __host__ __device__ constexpr Dual() : v(S(0)), d(S(0)) {}
    __host__ __device__ constexpr Dual(double x) : v(S(x)), d(S(0)) {}
    __host__ __device__ constexpr Dual(S x, S dx) : v(x), d(dx) {}
    template <typename R>
    __host__ __device__ explicit constexpr Dual(const Dual<R>& o) : v(S(o.v)), d(S(o.d)) {}
    __host__ __device__ explicit operator double() const { return (double)v; }
};

template <typename T>
struct DualOf { static constexpr bool is = false; using scalar = T; };
template <typename S>
struct DualOf<Dual<S>> { static constexpr bool is = true; using scalar = S; };

template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator+(Dual<S> a, Dual<S> b)
{
#pragma clang fp contract(off)
    return Dual<S>(a.v + b.v, a.d + b.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator-(Dual<S> a, Dual<S> b)
{
#pragma clang fp contract(off)
    return Dual<S>(a.v - b.v, a.d - b.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator-(Dual<S> a)
{
    return Dual<S>(-a.v, -a.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator*(Dual<S> a, Dual<S> b)
{
#pragma clang fp contract(off)
    return Dual<S>(a.v * b.v, fma(a.d, b.v, a.v * b.d));
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator/(Dual<S> a, Dual<S> b)
{
#pragma clang fp contract(off)
    const S q = a.v / b.v;
    return Dual<S>(q, (a.d - q * b.d) / b.v);
}
// the scalar overloads stay visible next to the dual one
using ::fma;

template <typename S>
__host__ __device__ __forceinline__ Dual<S> fma(Dual<S> a, Dual<S> b, Dual<S> c)
{
#pragma clang fp contract(off)
    return Dual<S>(fma(a.v, b.v, c.v), fma(a.d, b.v, fma(a.v, b.d, c.d)));
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S>& operator+=(Dual<S>& a, Dual<S> b)
{
    a = a + b;
    return a;
}
template <typename S>
__host__ __device__ __forceinline__ bool operator==(Dual<S> a, Dual<S> b)
{
    return a.v == b.v;
}

// Every buffer the kernels touch outside LDS is device global memory.  The
// pointers reach the kernels inside work-item descriptors, where the compiler
// cannot see their address space; without the cast it emits flat loads, which
// also count against the LDS wait counter, so that every LDS wait in the
// compute phase would wait for outstanding global loads as well.
template <typename T>
__device__ __forceinline__ T ldg(const T* p, int64_t i)
{
    if constexpr (DualOf<T>::is) {
        // one access for the (value, derivative) pair
        using S = typename DualOf<T>::scalar;
        typedef S P2 __attribute__((ext_vector_type(2)));
        const P2 v = ((const P2 __attribute__((address_space(1)))*)p)[i];
        return T(v[0], v[1]);
    } else {
        return ((const T __attribute__((address_space(1)))*)p)[i];
    }
}

template <typename T>
__device__ __forceinline__ void stg(T* p, int64_t i, T v)
{
    if constexpr (DualOf<T>::is) {
        using S = typename DualOf<T>::scalar;
        typedef S P2 __attribute__((ext_vector_type(2)));
        P2 w;
        w[0] = v.v;
        w[1] = v.d;
        ((P2 __attribute__((address_space(1)))*)p)[i] = w;
    } else {
        ((T __attribute__((address_space(1)))*)p)[i] = v;
    }
}

// The G values of a cell move as one native vector (one 16-byte access for
// four floats).
template <typename T, int G>
struct Native {
    typedef T type __attribute__((ext_vector_type(G)));
};
template <typename T>
struct Native<T, 1> {
    typedef T type;
};

template <typename T, int G>
__device__ __forceinline__ Vec<T, G> vload(const T* p, int64_t cell)
{
    if constexpr (DualOf<T>::is) {
        // dual fields: G consecutive (value, tangent) pairs
        Vec<T, G> r;
#pragma unroll
        for (int g = 0; g < G; ++g) r.v[g] = ldg(p, cell * G + g);
        return r;
    } else {
    using N = typename Native<T, G>::type;
    const N n = *(const N __attribute__((address_space(1)))*)(p + cell * G);
    Vec<T, G> r;
    if constexpr (G == 1) {
        r.v[0] = n;
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g) r.v[g] = n[g];
    }
    return r;
    }
}

template <typename T, int G>
__device__ __forceinline__ void vstore(T* p, int64_t cell, const Vec<T, G>& v)
{
    if constexpr (DualOf<T>::is) {
#pragma unroll
        for (int g = 0; g < G; ++g) stg(p, cell * G + g, v.v[g]);
    } else {
    using N = typename Native<T, G>::type;
    N n;
    if constexpr (G == 1) {
        n = v.v[0];
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g) n[g] = v.v[g];
    }
    *(N __attribute__((address_space(1)))*)(p + cell * G) = n;
    }
}

// The same accesses with a 32-bit element index into a plane whose base is
// uniform across the workgroup: the byte offset is formed in 32 bits, so the
// access takes the scalar-base form (64-bit base in SGPRs, 32-bit offset per
// lane) instead of 64-bit address arithmetic in every lane.  Plans keep every
// plane and coefficient array below 4 GiB, so the offsets cannot wrap.
// (Dual fields take the pairwise accesses above.)
template <typename T>
__device__ __forceinline__ T ldg32(const T* p, uint32_t i)
{
    if constexpr (DualOf<T>::is) {
        return ldg(p, (int64_t)i);
    } else {
    using B = const char __attribute__((address_space(1)))*;
    return *(const T __attribute__((address_space(1)))*)((B)p + i * (uint32_t)sizeof(T));
    }
}

template <typename T>
__device__ __forceinline__ void stg32(T* p, uint32_t i, T v)
{
    if constexpr (DualOf<T>::is) {
        stg(p, (int64_t)i, v);
    } else {
    using B = char __attribute__((address_space(1)))*;
    *(T __attribute__((address_space(1)))*)((B)p + i * (uint32_t)sizeof(T)) = v;
    }
}

template <typename T, int G>
__device__ __forceinline__ Vec<T, G> vload32(const T* p, uint32_t cell)
{
    if constexpr (DualOf<T>::is) return vload<T, G>(p, (int64_t)cell);
    else {
    using N = typename Native<T, G>::type;
    using B = const char __attribute__((address_space(1)))*;
    const N n = *(const N __attribute__((address_space(1)))*)((B)p + cell * (uint32_t)(sizeof(T) * G));
    Vec<T, G> r;
    if constexpr (G == 1) {
        r.v[0] = n;
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g) r.v[g] = n[g];
    }
    return r;
    }
}

template <typename T, int G>
__device__ __forceinline__ void vstore32(T* p, uint32_t cell, const Vec<T, G>& v)
{
    if constexpr (DualOf<T>::is) {
        vstore<T, G>(p, (int64_t)cell, v);
        return;
    } else {
    using N = typename Native<T, G>::type;
    using B = char __attribute__((address_space(1)))*;
    N n;
    if constexpr (G == 1) {
        n = v.v[0];
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g) n[g] = v.v[g];
    }
    *(N __attribute__((address_space(1)))*)((B)p + cell * (uint32_t)(sizeof(T) * G)) = n;
    }
}

template <typename T, int G>
__device__ __forceinline__ Vec<T, G> vzero()
{
    Vec<T, G> r;
#pragma unroll
    for (int g = 0; g < G; ++g) r.v[g] = T(0);
    return r;
}

template <typename T, int G>
__device__ __forceinline__ Vec<T, G> vkeep(bool keep, const Vec<T, G>& v)
{
    Vec<T, G> r;
#pragma unroll
    for (int g = 0; g < G; ++g) r.v[g] = keep ? v.v[g] : T(0);
    return r;
}

struct Step {
    int phase;
    int n;      // FWD/RECOMP: first step index (produces u^{n+1}); ADJ: first time t
    int j;      // segment
    int count;  // steps of this launch (1 or 2)
};

// Position of an item with (T, K, J) at launch s of its schedule, with up to
// S forward-type steps (first pass, recompute) or Sa adjoint steps fused per
// launch: forward steps in runs of S, then the last segment's adjoint steps,
// then per earlier segment its recompute and its adjoint steps, each run cut
// into launches of S (forward-type) or Sa (adjoint) steps, the last launch of
// a run possibly shorter.
__host__ __device__ inline int imin(int x, int y) { return x < y ? x : y; }

__host__ __device__ inline Step decode(int T, int K, int J, int s, int S, int Sa)
{
    Step r{kIdle, 0, 0, 0};
    if (s < 0) return r;
    const int nf = (T + S - 1) / S;
    if (s < nf) {
        r.phase = kFwd; r.n = s * S; r.j = r.n / K; r.count = imin(S, T - r.n);
        return r;
    }
    s -= nf;
    const int last = T - (J - 1) * K;
    const int nl = (last + Sa - 1) / Sa;
    if (s < nl) {
        r.phase = kAdj; r.n = T + 1 - s * Sa; r.j = J - 1; r.count = imin(Sa, last - s * Sa);
        return r;
    }
    s -= nl;
    const int nkf = (K + S - 1) / S, nka = (K + Sa - 1) / Sa, nb = nkf + nka;
    if (s < nb * (J - 1)) {
        const int blk = s / nb, rem = s - blk * nb;
        r.j = J - 2 - blk;
        if (rem < nkf) {
            r.phase = kRecomp; r.n = r.j * K + rem * S; r.count = imin(S, K - rem * S);
        } else {
            const int m = rem - nkf;
            r.phase = kAdj; r.n = r.j * K + K + 1 - m * Sa; r.count = imin(Sa, K - m * Sa);
        }
    }
    return r;
}

inline Sched make_sched(int T, int K, int J, int S, int Sa)
{
    Sched c{};
    c.T = T; c.K = K; c.J = J; c.S = S; c.Sa = Sa;
    c.nf = (T + S - 1) / S;
    c.last = T - (J - 1) * K;
    c.nl = (c.last + Sa - 1) / Sa;
    c.nkf = (K + S - 1) / S;
    c.nb = c.nkf + (K + Sa - 1) / Sa;
    c.dK = make_div((uint32_t)K);
    c.dnb = make_div((uint32_t)c.nb);
    return c;
}

// decode() from the precomputed constants: the same step for every s, with
// no division left to the lanes.
__host__ __device__ inline Step decode_s(const Sched& c, int s)
{
    Step r{kIdle, 0, 0, 0};
    if (s < 0) return r;
    if (s < c.nf) {
        r.phase = kFwd; r.n = s * c.S; r.j = quo(r.n, c.dK); r.count = imin(c.S, c.T - r.n);
        return r;
    }
    s -= c.nf;
    if (s < c.nl) {
        r.phase = kAdj; r.n = c.T + 1 - s * c.Sa; r.j = c.J - 1; r.count = imin(c.Sa, c.last - s * c.Sa);
        return r;
    }
    s -= c.nl;
    if (s < c.nb * (c.J - 1)) {
        const int blk = quo(s, c.dnb), rem = s - blk * c.nb;
        r.j = c.J - 2 - blk;
        if (rem < c.nkf) {
            r.phase = kRecomp; r.n = r.j * c.K + rem * c.S; r.count = imin(c.S, c.K - rem * c.S);
        } else {
            const int m = rem - c.nkf;
            r.phase = kAdj; r.n = r.j * c.K + c.K + 1 - m * c.Sa; r.count = imin(c.Sa, c.K - m * c.Sa);
        }
    }
    return r;
}

// x mod K of an item for x >= 0.
template <typename I>
__device__ __forceinline__ int kmod(const I& it, int x)
{
    return x - quo(x, it.sc.dK) * it.K;
}

// The per-cell arithmetic below spells out every fused multiply-add and
// disables contraction, so that every kernel (one step per launch, either
// half of a two-step launch, first pass or recompute) rounds a cell exactly
// the same way: checkpointed replay then reproduces the first pass bitwise.
template <typename T>
__device__ __forceinline__ void damp_coeffs(T e, T& a, T& b)
{
#pragma clang fp contract(off)
    if (e == T(0)) {
        a = T(2);
        b = T(-1);
    } else {
        const T inv = T(1) / (T(1) + e);
        a = (T(2) - e * e) * inv;
        b = (e - T(1)) * inv;
    }
}

// Forward update in increment form.  With v^n = u^n - u^{n-1} the update of
// eq. 2, u^{n+1} = a u^n + beta u^{n-1} + q L u^n, is the same map written as
//     v^{n+1} = -beta v^n + c2 u^n + q L u^n,   u^{n+1} = u^n + v^{n+1},
// with c2 = a + beta - 1 = -e^2/(1+e) (e = D dt); inside the absorbing layer's
// inner edge -beta = 1 and c2 = 0.  In floating point the two forms differ:
// the rounding error of each step enters u^{n+1} and, through the two-level
// recurrence, is summed twice over time in the first form but once in the
// second, which matters for the slowly varying late part of the field.
template <typename T>
__device__ __forceinline__ void damp_inc(T e, T& nb, T& c2)
{
#pragma clang fp contract(off)
    if (e == T(0)) {
        nb = T(1);
        c2 = T(0);
    } else {
        const T inv = T(1) / (T(1) + e);
        nb = (T(1) - e) * inv;
        c2 = -(e * e) * inv;
    }
}

// v^{n+1} of one cell (before the source): -beta v0 + c2 u0 + q sum_f b_f (u_f - u0).
template <typename T>
__device__ __forceinline__ T fwd_cell(T nb, T c2, T q, T fw, T fe, T fn, T fs, T u0, T uw, T ue, T un, T us, T v0)
{
#pragma clang fp contract(off)
    T L = fw * (uw - u0);
    L = fma(fe, ue - u0, L);
    L = fma(fn, un - u0, L);
    L = fma(fs, us - u0, L);
    return fma(q, L, fma(nb, v0, c2 * u0));
}

// The same update where no damping acts (-beta = 1, c2 = 0): v0 + q L.  It
// equals fwd_cell's value there (the two vanishing terms add a signed zero
// at most).
template <typename T>
__device__ __forceinline__ T fwd_cell_free(T q, T fw, T fe, T fn, T fs, T u0, T uw, T ue, T un, T us, T v0)
{
#pragma clang fp contract(off)
    T L = fw * (uw - u0);
    L = fma(fe, ue - u0, L);
    L = fma(fn, un - u0, L);
    L = fma(fs, us - u0, L);
    return fma(q, L, v0);
}

// One cell of the adjoint update: a l0 + b lp + sum_f b_f (w_f - w0), w = q l.
template <typename T>
__device__ __forceinline__ T adj_cell(T a, T b, T fw, T fe, T fn, T fs, T w0, T ww, T we, T wn, T ws, T l0, T lp)
{
#pragma clang fp contract(off)
    T L = fw * (ww - w0);
    L = fma(fe, we - w0, L);
    L = fma(fn, wn - w0, L);
    L = fma(fs, ws - w0, L);
    return fma(a, l0, fma(b, lp, L));
}

// The same update in terms of w = q lam (the second-order kernels carry w):
// w^{t-1} = a w^t + b w^{t+1} + q sum_f b_f (w_f - w0), the lam update
// multiplied by the cell's q, so no neighbour's q enters.
template <typename T>
__device__ __forceinline__ T adjw_cell(T a, T b, T q, T fw, T fe, T fn, T fs, T w0, T ww, T we, T wn, T ws, T wp)
{
#pragma clang fp contract(off)
    T L = fw * (ww - w0);
    L = fma(fe, we - w0, L);
    L = fma(fn, wn - w0, L);
    L = fma(fs, ws - w0, L);
    return fma(a, w0, fma(b, wp, q * L));
}

// Zero-lag imaging terms of one cell: S_kappa += l0 sum_f b_f du_f,
// S_b += sum_f c_f du_f dw_f (c_f = 1/2 on interior faces, 1 on border faces).
template <typename T>
__device__ __forceinline__ void image_cell(T fw, T fe, T fn, T fs, T cw, T ce, T cn, T cs, T l0, T w0, T ww, T we,
                                           T wn, T ws, T u0, T uw, T ue, T un, T us, T& sk, T& sb)
{
#pragma clang fp contract(off)
    const T duw = uw - u0, due = ue - u0, dun = un - u0, dus = us - u0;
    T Lu = fw * duw;
    Lu = fma(fe, due, Lu);
    Lu = fma(fn, dun, Lu);
    Lu = fma(fs, dus, Lu);
    T gb = (cw * duw) * (ww - w0);
    gb = fma(ce * due, we - w0, gb);
    gb = fma(cn * dun, wn - w0, gb);
    gb = fma(cs * dus, ws - w0, gb);
    sk = l0 * Lu;
    sb = gb;
}

// Face buoyancies of a cell from its own and its neighbours' bt (border rule
// bt_f = bt_x where the neighbour is outside the grid).
template <typename T>
__device__ __forceinline__ void faces(bool hw, bool he, bool hn, bool hs, T bc, T bw, T be, T bn, T bs,
                                      T& fw, T& fe, T& fn, T& fs)
{
    const T hf = T(0.5);
    fw = hw ? hf * (bc + bw) : bc;
    fe = he ? hf * (bc + be) : bc;
    fn = hn ? hf * (bc + bn) : bc;
    fs = hs ? hf * (bc + bs) : bc;
}

// The same face buoyancies from staged values hb = bt/2 that repeat the
// nearest grid cell's beyond the grid edge: one addition per face, equal to
// faces() bit for bit (halving is exact and commutes with the rounding of the
// sum; a border face gives bt/2 + bt/2 = bt).
template <typename T>
__device__ __forceinline__ void faces_h(T bc, T bw, T be, T bn, T bs, T& fw, T& fe, T& fn, T& fs)
{
    fw = bc + bw;
    fe = bc + be;
    fn = bc + bn;
    fs = bc + bs;
}

// (q, bt/2) of one staged cell (gx, gz): q in the grid (zero outside, where
// no update reads it), bt/2 of the nearest grid cell, for faces_h.
template <typename T>
__device__ __forceinline__ void stage_coef(const T* cf, bool in, int gx, int gz, int nx, int nz, T& q, T& hb)
{
    const int cx = min(max(gx, 0), nx - 1), cz = min(max(gz, 0), nz - 1);
    const uint32_t x = (uint32_t)(cz * nx + cx);
    const T qv = ldg32(cf, 2 * x), bv = ldg32(cf, 2 * x + 1);
    q = in ? qv : T(0);
    hb = T(0.5) * bv;
}

// Plane of u^tau read by a forward-type step: zero for tau = 0; on
// recompute, the checkpoint of segment j for tau = jK; else segment slot
// (tau-1) mod K.
template <typename T, typename Acc>
__device__ __forceinline__ const T* fwd_plane(const Item<T, Acc>& it, const Step& st, int tau)
{
    if (tau <= 0) return it.zero;
    if (st.phase == kRecomp && tau == st.j * it.K) return it.ck + (int64_t)(2 * (st.j - 1) + 1) * it.plane;
    return it.seg + (int64_t)kmod(it, tau - 1) * it.plane;
}

// v slot of level tau in a run of forward-type launches.  A launch of two or
// more steps reads v^n at other tiles' cells, so it must write v^{n+c} to
// the other slot.  With at most two steps per launch, slot floor(tau/2) mod
// 2: a run's launches start two levels apart, so every two-step launch flips
// it.  With three, slot ceil((tau - base)/3) mod 2 with base the run's first
// level (0 for the first pass, jK for the recompute of segment j): launches
// start at base + 3m, and one of 2 or 3 steps (a run's last launch may be
// shorter) ends in the other slot.  A one-step launch reads and writes each
// cell's own value, in place or across slots.
template <typename T, typename Acc>
__device__ __forceinline__ int vel_slot(const Item<T, Acc>& it, const Step& st, int tau)
{
    if (it.S != 3) return (tau >> 1) & 1;
    const int base = st.phase == kRecomp ? st.j * it.K : 0;
    return ((tau - base + 2) / 3) & 1;
}

// Plane of v^tau read by a forward-type step: zero for tau = 0; on
// recompute, the checkpoint of segment j for tau = jK; else its v slot.
template <typename T, typename Acc>
__device__ __forceinline__ const T* vel_in(const Item<T, Acc>& it, const Step& st, int tau)
{
    if (tau <= 0) return it.zero;
    if (st.phase == kRecomp && tau == st.j * it.K) return it.ck + (int64_t)(2 * (st.j - 1)) * it.plane;
    return it.vel + (int64_t)vel_slot(it, st, tau) * it.plane;
}

template <typename T, typename Acc>
__device__ __forceinline__ T* vel_out(const Item<T, Acc>& it, const Step& st, int tau)
{
    return it.vel + (int64_t)vel_slot(it, st, tau) * it.plane;
}

// Checkpoint pair that level t1 = jK (1 <= j <= J-1, the start of segment j)
// is also written to during the first forward pass: v^{t1} at the pair's
// first plane, u^{t1} at its second; null for every other level.
template <typename T, typename Acc>
__device__ __forceinline__ T* ckpt_pair(const Item<T, Acc>& it, const Step& st, int t1)
{
    if (st.phase != kFwd) return nullptr;
    const int j = quo(t1, it.sc.dK);
    if (t1 != j * it.K) return nullptr;
    if (j < 1 || j > it.J - 1) return nullptr;
    return it.ck + (int64_t)(2 * (j - 1)) * it.plane;
}

template <typename T, int G>
struct Src {
    int cell[G];
    T w[G];
};

template <typename T, int G, typename Acc>
__device__ __forceinline__ Src<T, G> sources(const Item<T, Acc>& it, int n)
{
    Src<T, G> s;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        s.cell[g] = ldg(it.src, g);
        s.w[g] = s.cell[g] >= 0 ? ldg(it.wavelet, (int64_t)(it.tx0 + g) * it.wavelet_stride + n) : T(0);
    }
    return s;
}

// Whether a source cell of s lies in the tile-relative columns [xa, xb) and
// rows [za, zb) of the tile at (x0, z0): where none does, the launch skips the
// per-cell source test (a wave-uniform branch).
template <typename T, int G, typename Acc>
__device__ __forceinline__ bool src_near(const Src<T, G>& s, const Item<T, Acc>& it, int x0, int z0, int xa, int xb,
                                         int za, int zb)
{
    bool any = false;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int c = s.cell[g];
        if (c >= 0) {
            const int cz = quo(c, it.dnx), cx = c - cz * it.nx;
            any = any || (cx >= x0 + xa && cx < x0 + xb && cz >= z0 + za && cz < z0 + zb);
        }
    }
    return any;
}

// v += w at this cell for the transmits whose source it is.
template <typename T, int G>
__device__ __forceinline__ void add_src(Vec<T, G>& v, int cell, const Src<T, G>& s)
{
#pragma unroll
    for (int g = 0; g < G; ++g)
        if (cell == s.cell[g]) v.v[g] += s.w[g];
}

__device__ __forceinline__ Entry ld_entry(const Entry* p, int i)
{
    typedef int32_t I4 __attribute__((ext_vector_type(4)));
    const I4 v = ((const I4 __attribute__((address_space(1)))*)p)[i];
    return Entry{v[0], v[1], v[2], v[3]};
}

// Receiver entries [e0, e1) of one tile.
struct Span {
    int e0, e1;
};

__device__ __forceinline__ Span span_of(const int32_t* off, int tile)
{
    return Span{ldg(off, tile), ldg(off, tile + 1)};
}

// Traces d[n] (and d[n+1] from out2) at the receivers of one tile, read back
// after the whole workgroup has stored its cells.
template <typename T, typename Acc>
__device__ __forceinline__ void sample_tile(const Item<T, Acc>& it, Span sp, int n, const T* out, const T* out2)
{
    if (sp.e1 <= sp.e0) return;
    __syncthreads();
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    for (int e = sp.e0 + tid; e < sp.e1; e += kBlock) {
        const Entry en = ld_entry(it.entries, e);
        stg(it.traces, en.trace_off + (int64_t)n * it.n_rcv, ldg(out, en.slot));
        if (out2) stg(it.traces, en.trace_off + (int64_t)(n + 1) * it.n_rcv, ldg(out2, en.slot));
    }
}

// Traces d[n] from the LDS copy of u^{n+1} (tile grown by one, row width W1)
// and d[n+1] from the stored u^{n+2}, at the receivers of one tile.
template <typename T, int G, typename Acc>
__device__ __forceinline__ void sample_tile2(const Item<T, Acc>& it, Span sp, int n, const Vec<T, G>* U1, int W1,
                                             int x0, int z0, const T* out2)
{
    if (sp.e1 <= sp.e0) return;
    __syncthreads();
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    for (int e = sp.e0 + tid; e < sp.e1; e += kBlock) {
        const Entry en = ld_entry(it.entries, e);
        const int cell = en.slot / G, g = en.slot - cell * G;
        const int k = (quo(cell, it.dnx) - z0 + 1) * W1 + (cell - quo(cell, it.dnx) * it.nx - x0 + 1);
        stg(it.traces, en.trace_off + (int64_t)n * it.n_rcv, U1[k].v[g]);
        stg(it.traces, en.trace_off + (int64_t)(n + 1) * it.n_rcv, ldg(out2, en.slot));
    }
}

// Adjoint source of sample m (transmit, receiver) at one entry.
template <typename T, typename Acc>
__device__ __forceinline__ T adj_source(const Item<T, Acc>& it, const Entry& en, int m)
{
    const int64_t o = en.trace_off + (int64_t)m * it.n_rcv;
    return it.inject_adj ? ldg(it.d_adj, o) : T(2) * (ldg(it.traces, o) - ldg(it.d_obs, o));
}

template <typename T, typename Acc>
__device__ __forceinline__ bool has_adj_source(const Item<T, Acc>& it)
{
    return it.inject_adj ? it.d_adj != nullptr : it.d_obs != nullptr;
}

// Add the adjoint source of sample m to field plane ``f`` at the receivers of
// one tile (one thread per run of equal slots, entries of a run in order);
// W: the plane holds w = q lam, so the source is scaled by the cell's q.
template <bool W, int G, typename T, typename Acc>
__device__ __forceinline__ void inject_tile(const Item<T, Acc>& it, Span sp, int m, T* f)
{
    if (sp.e1 <= sp.e0 || m < 0 || !has_adj_source(it)) return;
    __syncthreads();
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    for (int e = sp.e0 + tid; e < sp.e1; e += kBlock) {
        const Entry en = ld_entry(it.entries, e);
        if (en.run == 0) continue;
        T s = T(0);
        for (int k = 0; k < en.run; ++k) s += adj_source(it, ld_entry(it.entries, e + k), m);
        if (W) s = ldg(it.coef, 2 * (int64_t)(en.slot / G)) * s;
        stg(f, en.slot, ldg(f, en.slot) + s);
    }
}

// ============================================================== one step per launch

// Forward-type step (FWD or RECOMP) on one tile, straight from global memory:
// each lane marches ``rows`` rows keeping the vertical neighbours in registers.
// V distinguishes the persistent kernel's copy of a tile routine from the
// per-step kernels' copy: each instantiation keeps one caller and is inlined
// there by the ordinary inliner, so the per-step kernels' code is unaffected
// by the persistent form.
template <typename T, int G, typename Acc, int V = 0>
__device__ void tile_forward(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, int rows, bool sample)
{
    const int nx = it.nx, nz = it.nz, n = st.n;
    const T* cur = fwd_plane(it, st, n);
    const T* vin = vel_in(it, st, n);
    T* out = it.seg + (int64_t)kmod(it, n) * it.plane;
    T* vout = vel_out(it, st, n + 1);
    T* ckv = ckpt_pair(it, st, n + 1);
    T* cku = ckv ? ckv + it.plane : nullptr;
    const Src<T, G> src = sources<T, G>(it, n);
    const bool near = src_near<T, G, Acc>(src, it, tile_x * kTileX, tile_z * kWavesZ * rows, 0, kTileX, 0,
                                          kWavesZ * rows);

    const int ix = tile_x * kTileX + (int)threadIdx.x;
    const int z0 = tile_z * kWavesZ * rows + (int)threadIdx.y * rows;
    if (ix < nx && z0 < nz) {
        const T ex = ldg(it.ex, ix);
        const T* cf = it.coef;
        int iz = z0;
        int64_t x = (int64_t)iz * nx + ix;
        Vec<T, G> un = iz > 0 ? vload<T, G>(cur, x - nx) : vzero<T, G>();
        Vec<T, G> uc = vload<T, G>(cur, x);
        T bn = iz > 0 ? ldg(cf, 2 * (x - nx) + 1) : T(0);
        T q = ldg(cf, 2 * x), bc = ldg(cf, 2 * x + 1);
        const int zend = min(z0 + rows, nz);
        for (; iz < zend; ++iz, x += nx) {
            const bool hs = iz < nz - 1, hw = ix > 0, he = ix < nx - 1;
            const Vec<T, G> us = hs ? vload<T, G>(cur, x + nx) : vzero<T, G>();
            const T qs = hs ? ldg(cf, 2 * (x + nx)) : T(0);
            const T bs = hs ? ldg(cf, 2 * (x + nx) + 1) : T(0);
            const Vec<T, G> uw = hw ? vload<T, G>(cur, x - 1) : vzero<T, G>();
            const Vec<T, G> ue = he ? vload<T, G>(cur, x + 1) : vzero<T, G>();
            const T bw = hw ? ldg(cf, 2 * (x - 1) + 1) : T(0);
            const T be = he ? ldg(cf, 2 * (x + 1) + 1) : T(0);
            T fw, fe, fn, fs;
            faces<T>(hw, he, iz > 0, hs, bc, bw, be, bn, bs, fw, fe, fn, fs);
            T nb, c2;
            T e = ex + ldg(it.ez, iz);
            if (it.eatt) e = e + ldg(it.eatt, x);
            damp_inc<T>(e, nb, c2);
            const Vec<T, G> vp = vload<T, G>(vin, x);
            Vec<T, G> r, rv;
#pragma unroll
            for (int g = 0; g < G; ++g)
                rv.v[g] = fwd_cell<T>(nb, c2, q, fw, fe, fn, fs, uc.v[g], uw.v[g], ue.v[g], un.v[g], us.v[g], vp.v[g]);
            if (near) add_src<T, G>(rv, (int)x, src);
#pragma unroll
            for (int g = 0; g < G; ++g) r.v[g] = uc.v[g] + rv.v[g];
            vstore<T, G>(out, x, r);
            vstore<T, G>(vout, x, rv);
            if (ckv) {
                vstore<T, G>(cku, x, r);
                vstore<T, G>(ckv, x, rv);
            }
            un = uc; uc = us;
            bn = bc; bc = bs; q = qs;
        }
    }
    if (sample) sample_tile(it, span_of(it.tile_off, tile_z * it.tiles_x + tile_x), n, out, (const T*)nullptr);
}

// Adjoint step at time t on one tile, with the imaging of lam^t and u^{t-1}.
template <typename T, int G, typename Acc, int V = 0>
__device__ void tile_adjoint(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, int rows)
{
    const int nx = it.nx, nz = it.nz, t = st.n;
    const int64_t P = it.plane, ncell = (int64_t)nx * nz;
    const T* cur = it.lam + (int64_t)(t & (it.nlam - 1)) * P;          // w^t = q lam^t
    const T* p1 = it.lam + (int64_t)((t + 1) & (it.nlam - 1)) * P;     // w^{t+1}
    T* out = it.lam + (int64_t)((t - 1) & (it.nlam - 1)) * P;          // w^{t-1} (in place when nlam = 2)
    const T* um = it.seg + (int64_t)kmod(it, t - 2) * P;        // u^{t-1}
    Acc* accK = it.acc;
    Acc* accB = it.acc + ncell;
    // attenuation: the eta term of the imaging also reads u^{t-2} at the cell
    // (zero before u^1, the segment's checkpoint at its first level)
    Acc* accE = it.acc + 2 * ncell;
    const T* um2 = nullptr;
    if (it.eatt) {
        const int l2 = t - 2;
        um2 = l2 <= 0 ? it.zero
            : (l2 == st.j * it.K && st.j >= 1) ? it.ck + (int64_t)(2 * (st.j - 1) + 1) * P
            : it.seg + (int64_t)kmod(it, t - 3) * P;
    }

    const int ix = tile_x * kTileX + (int)threadIdx.x;
    const int z0 = tile_z * kWavesZ * rows + (int)threadIdx.y * rows;
    if (ix < nx && z0 < nz) {
        const T ex = ldg(it.ex, ix);
        const T* cf = it.coef;
        const bool hw = ix > 0, he = ix < nx - 1;
        const T hf = T(0.5);
        const T cw = hw ? hf : T(1), ce = he ? hf : T(1);
        int iz = z0;
        int64_t x = (int64_t)iz * nx + ix;
        Vec<T, G> ln = iz > 0 ? vload<T, G>(cur, x - nx) : vzero<T, G>();
        Vec<T, G> lc = vload<T, G>(cur, x);
        Vec<T, G> uN = iz > 0 ? vload<T, G>(um, x - nx) : vzero<T, G>();
        Vec<T, G> uC = vload<T, G>(um, x);
        T bn = iz > 0 ? ldg(cf, 2 * (x - nx) + 1) : T(0);
        T qc = ldg(cf, 2 * x), bc = ldg(cf, 2 * x + 1);
        const int zend = min(z0 + rows, nz);
        for (; iz < zend; ++iz, x += nx) {
            const bool hs = iz < nz - 1, hn = iz > 0;
            const Vec<T, G> ls = hs ? vload<T, G>(cur, x + nx) : vzero<T, G>();
            const Vec<T, G> uS = hs ? vload<T, G>(um, x + nx) : vzero<T, G>();
            const T qs = hs ? ldg(cf, 2 * (x + nx)) : T(0);
            const T bs = hs ? ldg(cf, 2 * (x + nx) + 1) : T(0);
            const Vec<T, G> lw = hw ? vload<T, G>(cur, x - 1) : vzero<T, G>();
            const Vec<T, G> le = he ? vload<T, G>(cur, x + 1) : vzero<T, G>();
            const Vec<T, G> uW = hw ? vload<T, G>(um, x - 1) : vzero<T, G>();
            const Vec<T, G> uE = he ? vload<T, G>(um, x + 1) : vzero<T, G>();
            const T bw = hw ? ldg(cf, 2 * (x - 1) + 1) : T(0);
            const T be = he ? ldg(cf, 2 * (x + 1) + 1) : T(0);
            T fw, fe, fn, fs;
            faces<T>(hw, he, hn, hs, bc, bw, be, bn, bs, fw, fe, fn, fs);
            const T cn = hn ? hf : T(1), cs = hs ? hf : T(1);
            T a, b;
            T e = ex + ldg(it.ez, iz);
            if (it.eatt) e = e + ldg(it.eatt, x);
            damp_coeffs<T>(e, a, b);
            const Vec<T, G> lp = vload<T, G>(p1, x);
            Vec<T, G> r;
            Acc sk = Acc(0), sb = Acc(0), se = Acc(0);
            // derivatives of a, beta and gamma/gamma in e for the attenuation term
            T da = T(0), dbeta = T(0), dgr = T(0), iq = T(0);
            Vec<T, G> u2 = vzero<T, G>();
            if (um2) {
                const T inv = T(1) / (T(1) + e);
                da = -((e * e + T(2) * e) + T(2)) * (inv * inv);
                dbeta = T(2) * (inv * inv);
                dgr = -inv;
                iq = T(1) / qc;
                u2 = vload<T, G>(um2, x);
            }
            // the planes hold w = q lam: the kappa imaging term w0 sum_f b_f du_f
            // is q times the lam one (undone per cell when the gradient is formed)
#pragma unroll
            for (int g = 0; g < G; ++g) {
                r.v[g] = adjw_cell<T>(a, b, qc, fw, fe, fn, fs, lc.v[g], lw.v[g], le.v[g], ln.v[g], ls.v[g], lp.v[g]);
                T k1, b1;
                image_cell<T>(fw, fe, fn, fs, cw, ce, cn, cs, lc.v[g], lc.v[g], lw.v[g], le.v[g], ln.v[g], ls.v[g],
                              uC.v[g], uW.v[g], uE.v[g], uN.v[g], uS.v[g], k1, b1);
                sk += Acc(k1);
                sb += Acc(b1);
                // lam (a' u^{t-1} + beta' u^{t-2}) + lam gamma' kappa L u^{t-1}, lam = w / q
                if (um2) se += Acc((lc.v[g] * iq) * (da * uC.v[g] + dbeta * u2.v[g]) + dgr * k1);
            }
            vstore<T, G>(out, x, r);
            stg(accK, x, ldg(accK, x) + sk);
            stg(accB, x, ldg(accB, x) + sb);
            if (um2) stg(accE, x, ldg(accE, x) + se);
            ln = lc; lc = ls; uN = uC; uC = uS;
            qc = qs; bn = bc; bc = bs;
        }
    }
    // adjoint source of w^{t-1}: q times sample t-2
    inject_tile<true, G>(it, span_of(it.tile_off, tile_z * it.tiles_x + tile_x), t - 2, out);
}

// ============================================================== two steps per launch
//
// The workgroup stages its tile grown by two cells (field and coefficients)
// in LDS, computes the first step on the tile grown by one cell into LDS
// and the second step on the tile itself; both time levels are stored (the
// replay needs every plane).  The tile height is a compile-time constant so
// that every global load of the launch is issued in one burst into
// registers before the first barrier: a workgroup then waits for memory
// once, not once per loop trip.

template <typename T, int G, int R, bool ADJ>
struct Lds2 {
    static constexpr int TZ = kWavesZ * R;
    static constexpr int W0 = kTileX + 4, H0 = TZ + 4, N0 = W0 * H0;   // tile grown by 2
    static constexpr int W1 = kTileX + 2, H1 = TZ + 2, N1 = W1 * H1;   // tile grown by 1
    static constexpr int P0 = (N0 + kBlock - 1) / kBlock;               // per-thread shares
    static constexpr int P1 = (N1 + kBlock - 1) / kBlock;
    static constexpr int ND = W0 + H0;                                  // damping: columns, then rows
    static constexpr int NR1 = 2 * W1 + 2 * TZ;                         // ring of the tile grown by 1
    static_assert(ND <= kBlock && NR1 <= kBlock, "one damping value and ring cell per thread");
    // F0[N0] fields, Q0[N0] and B0[N0] coefficients (separate arrays: unit-stride
    // neighbour reads), then (adjoint only) two tile + 1 field planes without
    // their first and last cells, the top-left and bottom-right corners that
    // no tile cell reads; then D[ND] damping values of the grown tile.  The
    // forward writes its tile + 1 plane over F0.  For FP32 and four transmits
    // the adjoint takes exactly 40 KiB, so four workgroups share a CU's
    // 160 KiB, and the forward 19.4 KiB (eight).
    static constexpr size_t bytes =
        ((size_t)N0 * (G + 2) + (ADJ ? (size_t)(N1 - 2) * G * 2 : 0) + (size_t)ND) * sizeof(T);
};

template <typename T, int G, int R, bool ADJ>
__device__ __forceinline__ void cell_of(int c, int grow, int x0, int z0, int& ix, int& iz)
{
    const int W = kTileX + 2 * grow;
    ix = x0 - grow + c % W;
    iz = z0 - grow + c / W;
}

// Damping value e = D dt of column x0 - GROW + tid (tid < W0) or of row
// z0 - GROW + (tid - W0) (W0 <= tid < ND) of the tile grown by GROW cells;
// zero outside the grid.  Loaded with the burst so that the compute phase reads it from LDS.
// (nx, nz and the profile pointers come in as values already held in scalar
// registers: selecting them per lane through the descriptor would turn the
// selection into a dependent vector load.)
template <typename T, int W0, int ND, int GROW = 2>
__device__ __forceinline__ T damping_of(const T* exd, const T* ezd, int nx, int nz, int tid, int x0, int z0)
{
    const bool col = tid < W0;
    const int i = col ? x0 - GROW + tid : z0 - GROW + (tid - W0);
    const bool in = tid < ND && i >= 0 && i < (col ? nx : nz);
    const T v = ldg(col ? exd : ezd, in ? i : 0);
    return in ? v : T(0);
}

// Cell (ex, ez) of the ring of the tile grown by one (ring index r < NR):
// top row, bottom row, left column, right column.
template <int W1, int TZ>
__device__ __forceinline__ void ring_cell(int r, int& ex, int& ez)
{
    if (r < W1) { ex = r; ez = 0; }
    else if (r < 2 * W1) { ex = r - W1; ez = TZ + 1; }
    else if (r < 2 * W1 + TZ) { ex = 0; ez = 1 + r - 2 * W1; }
    else { ex = W1 - 1; ez = 1 + r - 2 * W1 - TZ; }
}

template <typename T, int G, typename Acc, int R, int V = 0>
__device__ void tile_forward2(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, bool sample,
                              unsigned char* smem)
{
    using L = Lds2<T, G, R, false>;
    constexpr int NR = 2 * L::W1 + 2 * L::TZ;                            // ring cells of the tile grown by 1
    static_assert(NR <= kBlock, "one ring cell per thread");
    const int nx = it.nx, nz = it.nz, n = st.n;
    Vec<T, G>* U0 = reinterpret_cast<Vec<T, G>*>(smem);                  // u^n, tile + 2
    T* Q0 = reinterpret_cast<T*>(U0 + L::N0);                            // q, tile + 2
    T* B0 = Q0 + L::N0;                                                  // bt/2, tile + 2 (edge-replicated)
    Vec<T, G>* U1 = U0;                                                  // u^{n+1}, tile + 1, over u^n
    T* D = B0 + L::N0;                                                   // damping
    const T* cur = fwd_plane(it, st, n);
    const T* vin = vel_in(it, st, n);
    T* out1 = it.seg + (int64_t)kmod(it, n) * it.plane;
    T* out2 = it.seg + (int64_t)kmod(it, n + 1) * it.plane;
    T* vout = vel_out(it, st, n + 2);
    T* ck1 = ckpt_pair(it, st, n + 1);
    T* ck2 = ckpt_pair(it, st, n + 2);
    // u^{n+1} is the next launch's input only when this launch stops there;
    // in a two-step launch it is stored only where the adjoint will read it
    // (every recomputed level, and the first pass's levels from the last
    // segment on)
    const bool keep1 = st.phase != kFwd || n + 1 >= it.keep_from;
    const Src<T, G> s1 = sources<T, G>(it, n);
    const Src<T, G> s2 = sources<T, G>(it, n + 1);
    const Span rcv = sample ? span_of(it.tile_off, tile_z * it.tiles_x + tile_x) : Span{0, 0};
    const int x0 = tile_x * kTileX, z0 = tile_z * L::TZ;
    // a source within the cells this launch updates (step n on the tile grown by one)
    const bool near = src_near<T, G, Acc>(s1, it, x0, z0, -1, kTileX + 1, -1, L::TZ + 1);
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    const int ix = x0 + (int)threadIdx.x;
    const T* cf = it.coef;
    const T* exd_p = it.ex;
    const T* ezd_p = it.ez;

    // one burst: u^n and (q, bt/2) on the tile grown by 2; v^n at this lane's
    // tile cells and ring cell; the damping profile.  Cells outside the grid
    // (or beyond the grown tile) load cell 0 and are replaced by zeros.
    Vec<T, G> f0[L::P0], vt[R], vr;
    T q0[L::P0], b0[L::P0];
#pragma unroll
    for (int i = 0; i < L::P0; ++i) {
        const int c = tid + i * kBlock;
        int gx, gz;
        cell_of<T, G, R, false>(c, 2, x0, z0, gx, gz);
        const bool in = c < L::N0 && gx >= 0 && gx < nx && gz >= 0 && gz < nz;
        const uint32_t x = in ? (uint32_t)(gz * nx + gx) : 0u;
        f0[i] = vkeep<T, G>(in, vload32<T, G>(cur, x));
        stage_coef<T>(cf, in, gx, gz, nx, nz, q0[i], b0[i]);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int iz = z0 + (int)threadIdx.y * R + k;
        const bool in = ix < nx && iz < nz;
        vt[k] = vkeep<T, G>(in, vload32<T, G>(vin, in ? (uint32_t)(iz * nx + ix) : 0u));
    }
    int rex = 0, rez = 0;
    ring_cell<L::W1, L::TZ>(tid, rex, rez);
    const int rix = x0 - 1 + rex, riz = z0 - 1 + rez;
    const bool rin = tid < NR && rix >= 0 && rix < nx && riz >= 0 && riz < nz;
    vr = vkeep<T, G>(rin, vload32<T, G>(vin, rin ? (uint32_t)(riz * nx + rix) : 0u));
    const T dmp = damping_of<T, L::W0, L::ND>(exd_p, ezd_p, nx, nz, tid, x0, z0);
#pragma unroll
    for (int i = 0; i < L::P0; ++i) {
        const int c = tid + i * kBlock;
        if (c < L::N0) {
            U0[c] = f0[i];
            Q0[c] = q0[i];
            B0[c] = b0[i];
        }
    }
    if (tid < L::ND) D[tid] = dmp;
    __syncthreads();

    // step n at cell (ex, ez) of the tile grown by one: v^{n+1} into vv (v^n
    // given there), u^{n+1} returned; the caller knows the cell is in the grid
    auto step1 = [&](int ex, int ez, int gx, int gz, Vec<T, G>& vv) {
        const int k = (ez + 1) * L::W0 + ex + 1;
        const uint32_t x = (uint32_t)(gz * nx + gx);
        T fw, fe, fn, fs, nb, c2;
        faces_h<T>(B0[k], B0[k - 1], B0[k + 1], B0[k - L::W0], B0[k + L::W0], fw, fe, fn, fs);
        damp_inc<T>(D[ex + 1] + D[L::W0 + ez + 1], nb, c2);
        const T q = Q0[k];
        const Vec<T, G> u0 = U0[k], uw = U0[k - 1], ue = U0[k + 1], un = U0[k - L::W0], us = U0[k + L::W0];
        Vec<T, G> r;
#pragma unroll
        for (int g = 0; g < G; ++g)
            vv.v[g] = fwd_cell<T>(nb, c2, q, fw, fe, fn, fs, u0.v[g], uw.v[g], ue.v[g], un.v[g], us.v[g], vv.v[g]);
        if (near) add_src<T, G>(vv, (int)x, s1);
#pragma unroll
        for (int g = 0; g < G; ++g) r.v[g] = u0.v[g] + vv.v[g];
        return r;
    };
    // step n: the ring (u^{n+1} for LDS only), then the tile cells of this
    // lane, with the map of step n+1, so that v^{n+1} stays in registers;
    // u^{n+1} is held in registers until every lane has read u^n, then
    // written over it
    Vec<T, G> ur = vzero<T, G>(), ut[R];
    if (rin) ur = step1(rex, rez, rix, riz, vr);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int ez = (int)threadIdx.y * R + k, iz = z0 + ez;
        ut[k] = vzero<T, G>();
        if (ix < nx && iz < nz) {
            ut[k] = step1((int)threadIdx.x + 1, ez + 1, ix, iz, vt[k]);
            const uint32_t x = (uint32_t)(iz * nx + ix);
            if (keep1) vstore32<T, G>(out1, x, ut[k]);
            if (ck1) {
                vstore32<T, G>(ck1, x, vt[k]);
                vstore32<T, G>(ck1 + it.plane, x, ut[k]);
            }
        }
    }
    __syncthreads();
    if (tid < NR) U1[rez * L::W1 + rex] = ur;
#pragma unroll
    for (int k = 0; k < R; ++k) U1[((int)threadIdx.y * R + k + 1) * L::W1 + threadIdx.x + 1] = ut[k];
    __syncthreads();
    // step n+1 on the tile
    if (ix < nx) {
        const T exd = D[threadIdx.x + 2];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int ez = (int)threadIdx.y * R + k, iz = z0 + ez;
            if (iz < nz) {
                const int k1 = (ez + 1) * L::W1 + threadIdx.x + 1;
                const int k0 = (ez + 2) * L::W0 + threadIdx.x + 2;
                const uint32_t x = (uint32_t)(iz * nx + ix);
                T fw, fe, fn, fs, nb, c2;
                faces_h<T>(B0[k0], B0[k0 - 1], B0[k0 + 1], B0[k0 - L::W0], B0[k0 + L::W0], fw, fe, fn, fs);
                damp_inc<T>(exd + D[L::W0 + ez + 2], nb, c2);
                const T q = Q0[k0];
                const Vec<T, G> u0 = U1[k1], uw = U1[k1 - 1], ue = U1[k1 + 1], un = U1[k1 - L::W1],
                                us = U1[k1 + L::W1];
                Vec<T, G> r, rv;
#pragma unroll
                for (int g = 0; g < G; ++g)
                    rv.v[g] = fwd_cell<T>(nb, c2, q, fw, fe, fn, fs, u0.v[g], uw.v[g], ue.v[g], un.v[g], us.v[g],
                                          vt[k].v[g]);
                if (near) add_src<T, G>(rv, (int)x, s2);
#pragma unroll
                for (int g = 0; g < G; ++g) r.v[g] = u0.v[g] + rv.v[g];
                vstore32<T, G>(out2, x, r);
                vstore32<T, G>(vout, x, rv);
                if (ck2) {
                    vstore32<T, G>(ck2, x, rv);
                    vstore32<T, G>(ck2 + it.plane, x, r);
                }
            }
        }
    }
    sample_tile2<T, G>(it, rcv, n, U1, L::W1, x0, z0, out2);
}

// ============================================================== three forward steps per launch
//
// The workgroup stages its tile grown by three cells (field, coefficients,
// damping) in LDS and runs step n on the tile grown by two, step n+1 on the
// tile grown by one and step n+2 on the tile.  Every level lives in the one
// LDS plane laid out on the tile grown by three: a step's results are held in
// registers until every lane has read the level before, then written over
// it.  A lane keeps v of its cells in registers through the steps that need
// them: its R tile cells (all three steps), one cell of the ring of the tile
// grown by one (steps n and n+1) and one of the ring of the tile grown by two
// (step n).  Only forward-type steps (first pass, recompute) take this form;
// adjoint launches fuse at most two steps.

template <typename T, int G, int R>
struct Lds3 {
    static constexpr int TZ = kWavesZ * R;
    static constexpr int W3 = kTileX + 6, H3 = TZ + 6, N3 = W3 * H3;   // tile grown by 3
    static constexpr int P3 = (N3 + kBlock - 1) / kBlock;               // per-thread shares
    static constexpr int ND = W3 + H3;                                  // damping: columns, then rows
    static constexpr int NR1 = 2 * (kTileX + 2) + 2 * TZ;               // ring of the tile grown by 1
    static constexpr int NR2 = 2 * (kTileX + 4) + 2 * (TZ + 2);         // ring of the tile grown by 2
    static_assert(ND <= kBlock && NR1 <= kBlock && NR2 <= kBlock, "one ring cell and damping value per thread");
    // F[N3] fields, Q[N3] and B[N3] coefficients, D[ND] damping values
    static constexpr size_t bytes = ((size_t)N3 * (G + 2) + (size_t)ND) * sizeof(T);
    // workgroups of 4 waves that the 160 KiB of LDS of a CU hold = waves per
    // SIMD (at most 6); the register allocation is held to what that
    // occupancy allows, so registers do not lower it further
    static constexpr int kWaves = (int)(160 * 1024 / bytes) < 6 ? (int)(160 * 1024 / bytes) : 6;
};

// Traces d[m] from an LDS level laid out on the tile grown by GROW (row
// width W), at the receivers of one tile.  The caller has made the level
// visible to the workgroup and does not overwrite it before a barrier.
template <typename T, int G, int GROW, typename Acc>
__device__ __forceinline__ void sample_lds(const Item<T, Acc>& it, Span sp, int m, const Vec<T, G>* U, int W,
                                           int x0, int z0)
{
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    for (int e = sp.e0 + tid; e < sp.e1; e += kBlock) {
        const Entry en = ld_entry(it.entries, e);
        const int cell = en.slot / G, g = en.slot - cell * G;
        const int k = (quo(cell, it.dnx) - z0 + GROW) * W + (cell - quo(cell, it.dnx) * it.nx - x0 + GROW);
        stg(it.traces, en.trace_off + (int64_t)m * it.n_rcv, U[k].v[g]);
    }
}

template <typename T, int G, typename Acc, int R, int V = 0>
__device__ void tile_forward3(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, bool sample,
                              unsigned char* smem)
{
    using L = Lds3<T, G, R>;
    constexpr int W = L::W3;
    const int nx = it.nx, nz = it.nz, n = st.n;
    Vec<T, G>* U = reinterpret_cast<Vec<T, G>*>(smem);                   // u^n, then u^{n+1}, u^{n+2}
    T* Q = reinterpret_cast<T*>(U + L::N3);                              // q, tile + 3
    T* B = Q + L::N3;                                                    // bt/2, tile + 3 (edge-replicated)
    T* D = B + L::N3;                                                    // damping
    const T* cur = fwd_plane(it, st, n);
    const T* vin = vel_in(it, st, n);
    T* out1 = it.seg + (int64_t)kmod(it, n) * it.plane;
    T* out2 = it.seg + (int64_t)kmod(it, n + 1) * it.plane;
    T* out3 = it.seg + (int64_t)kmod(it, n + 2) * it.plane;
    T* vout = vel_out(it, st, n + 3);
    T* ck1 = ckpt_pair(it, st, n + 1);
    T* ck2 = ckpt_pair(it, st, n + 2);
    T* ck3 = ckpt_pair(it, st, n + 3);
    // u^{n+1} and u^{n+2} are stored only where the adjoint will read them
    const bool keep1 = st.phase != kFwd || n + 1 >= it.keep_from;
    const bool keep2 = st.phase != kFwd || n + 2 >= it.keep_from;
    const Src<T, G> s1 = sources<T, G>(it, n);
    const Src<T, G> s2 = sources<T, G>(it, n + 1);
    const Src<T, G> s3 = sources<T, G>(it, n + 2);
    const Span rcv = sample ? span_of(it.tile_off, tile_z * it.tiles_x + tile_x) : Span{0, 0};
    const int x0 = tile_x * kTileX, z0 = tile_z * L::TZ;
    // a source within the cells this launch updates (step n on the tile grown by two)
    const bool near = src_near<T, G, Acc>(s1, it, x0, z0, -2, kTileX + 2, -2, L::TZ + 2);
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    const int tx = (int)threadIdx.x, ix = x0 + tx;
    const T* cf = it.coef;

    // this lane's ring cells, relative to the tile origin
    int r1x = 0, r1z = 0, r2x = 0, r2z = 0;
    ring_cell<kTileX + 2, L::TZ>(tid, r1x, r1z);
    ring_cell<kTileX + 4, L::TZ + 2>(tid, r2x, r2z);
    r1x -= 1; r1z -= 1; r2x -= 2; r2z -= 2;
    const bool in1 = tid < L::NR1 && x0 + r1x >= 0 && x0 + r1x < nx && z0 + r1z >= 0 && z0 + r1z < nz;
    const bool in2 = tid < L::NR2 && x0 + r2x >= 0 && x0 + r2x < nx && z0 + r2z >= 0 && z0 + r2z < nz;

    // one burst: u^n and (q, bt/2) on the tile grown by 3; v^n at this lane's
    // cells; the damping profile
    Vec<T, G> f[L::P3], vt[R], v1, v2;
    T q[L::P3], b[L::P3];
#pragma unroll
    for (int i = 0; i < L::P3; ++i) {
        const int c = tid + i * kBlock;
        int gx, gz;
        cell_of<T, G, R, false>(c, 3, x0, z0, gx, gz);
        const bool in = c < L::N3 && gx >= 0 && gx < nx && gz >= 0 && gz < nz;
        const uint32_t x = in ? (uint32_t)(gz * nx + gx) : 0u;
        f[i] = vkeep<T, G>(in, vload32<T, G>(cur, x));
        stage_coef<T>(cf, in, gx, gz, nx, nz, q[i], b[i]);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int iz = z0 + (int)threadIdx.y * R + k;
        const bool in = ix < nx && iz < nz;
        vt[k] = vkeep<T, G>(in, vload32<T, G>(vin, in ? (uint32_t)(iz * nx + ix) : 0u));
    }
    v1 = vkeep<T, G>(in1, vload32<T, G>(vin, in1 ? (uint32_t)((z0 + r1z) * nx + x0 + r1x) : 0u));
    v2 = vkeep<T, G>(in2, vload32<T, G>(vin, in2 ? (uint32_t)((z0 + r2z) * nx + x0 + r2x) : 0u));
    const T dmp = damping_of<T, W, L::ND, 3>(it.ex, it.ez, nx, nz, tid, x0, z0);
#pragma unroll
    for (int i = 0; i < L::P3; ++i) {
        const int c = tid + i * kBlock;
        if (c < L::N3) {
            U[c] = f[i];
            Q[c] = q[i];
            B[c] = b[i];
        }
    }
    if (tid < L::ND) D[tid] = dmp;
    // no absorbing layer within the tile grown by three: -beta = 1 and c2 = 0
    // at every cell this launch updates (a wave-uniform branch below)
    const bool damp = __syncthreads_or(tid < L::ND && !(dmp == T(0))) != 0;

    // one step at cell (x, z) of the grid (tile-relative) from the level in
    // U: v of the next level into vv (v of this level given there), u of the
    // next level returned
    auto step = [&](int x, int z, Vec<T, G>& vv, const Src<T, G>& sc) {
        const int gx = x0 + x, gz = z0 + z;
        const int k = (z + 3) * W + x + 3;
        const int cell = gz * nx + gx;
        T fw, fe, fn, fs;
        faces_h<T>(B[k], B[k - 1], B[k + 1], B[k - W], B[k + W], fw, fe, fn, fs);
        Vec<T, G> r;
        const T qc = Q[k];
        const Vec<T, G> u0 = U[k], uw = U[k - 1], ue = U[k + 1], un = U[k - W], us = U[k + W];
        if (damp) {
            T nb, c2;
            damp_inc<T>(D[x + 3] + D[W + z + 3], nb, c2);
#pragma unroll
            for (int g = 0; g < G; ++g)
                vv.v[g] = fwd_cell<T>(nb, c2, qc, fw, fe, fn, fs, u0.v[g], uw.v[g], ue.v[g], un.v[g], us.v[g],
                                      vv.v[g]);
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g)
                vv.v[g] = fwd_cell_free<T>(qc, fw, fe, fn, fs, u0.v[g], uw.v[g], ue.v[g], un.v[g], us.v[g],
                                           vv.v[g]);
        }
        if (near) add_src<T, G>(vv, cell, sc);
#pragma unroll
        for (int g = 0; g < G; ++g) r.v[g] = u0.v[g] + vv.v[g];
        return r;
    };
    auto lds_at = [&](int x, int z) { return (z + 3) * W + x + 3; };

    // step n on the tile grown by two
    Vec<T, G> a1 = vzero<T, G>(), a2 = vzero<T, G>(), at[R];
    if (in2) a2 = step(r2x, r2z, v2, s1);
    if (in1) a1 = step(r1x, r1z, v1, s1);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int z = (int)threadIdx.y * R + k, iz = z0 + z;
        at[k] = vzero<T, G>();
        if (ix < nx && iz < nz) {
            at[k] = step(tx, z, vt[k], s1);
            const uint32_t x = (uint32_t)(iz * nx + ix);
            if (keep1) vstore32<T, G>(out1, x, at[k]);
            if (ck1) {
                vstore32<T, G>(ck1, x, vt[k]);
                vstore32<T, G>(ck1 + it.plane, x, at[k]);
            }
        }
    }
    __syncthreads();
    if (tid < L::NR2) U[lds_at(r2x, r2z)] = a2;
    if (tid < L::NR1) U[lds_at(r1x, r1z)] = a1;
#pragma unroll
    for (int k = 0; k < R; ++k) U[lds_at(tx, (int)threadIdx.y * R + k)] = at[k];
    __syncthreads();
    if (rcv.e1 > rcv.e0) sample_lds<T, G, 3>(it, rcv, n, U, W, x0, z0);

    // step n+1 on the tile grown by one
    if (in1) a1 = step(r1x, r1z, v1, s2);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int z = (int)threadIdx.y * R + k, iz = z0 + z;
        if (ix < nx && iz < nz) {
            at[k] = step(tx, z, vt[k], s2);
            const uint32_t x = (uint32_t)(iz * nx + ix);
            if (keep2) vstore32<T, G>(out2, x, at[k]);
            if (ck2) {
                vstore32<T, G>(ck2, x, vt[k]);
                vstore32<T, G>(ck2 + it.plane, x, at[k]);
            }
        }
    }
    __syncthreads();
    if (tid < L::NR1) U[lds_at(r1x, r1z)] = a1;
#pragma unroll
    for (int k = 0; k < R; ++k) U[lds_at(tx, (int)threadIdx.y * R + k)] = at[k];
    __syncthreads();
    if (rcv.e1 > rcv.e0) sample_lds<T, G, 3>(it, rcv, n + 1, U, W, x0, z0);

    // step n+2 on the tile
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int z = (int)threadIdx.y * R + k, iz = z0 + z;
        if (ix < nx && iz < nz) {
            const Vec<T, G> r = step(tx, z, vt[k], s3);
            const uint32_t x = (uint32_t)(iz * nx + ix);
            vstore32<T, G>(out3, x, r);
            vstore32<T, G>(vout, x, vt[k]);
            if (ck3) {
                vstore32<T, G>(ck3, x, vt[k]);
                vstore32<T, G>(ck3 + it.plane, x, r);
            }
        }
    }
    // trace d[n+2] from the stored u^{n+3}
    if (rcv.e1 > rcv.e0) {
        __syncthreads();
        for (int e = rcv.e0 + tid; e < rcv.e1; e += kBlock) {
            const Entry en = ld_entry(it.entries, e);
            stg(it.traces, en.trace_off + (int64_t)(n + 2) * it.n_rcv, ldg(out3, en.slot));
        }
    }
}

template <typename T, int G, typename Acc, int R, int V = 0>
__device__ void tile_adjoint2(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, unsigned char* smem)
{
    using L = Lds2<T, G, R, true>;
    const int nx = it.nx, nz = it.nz, t = st.n, nl = it.nlam;
    const int64_t P = it.plane, ncell = (int64_t)nx * nz;
    // The adjoint planes hold w = q lam (adjw_cell); "lam" below names the
    // level, the values are w.
    Vec<T, G>* L0 = reinterpret_cast<Vec<T, G>*>(smem);                  // w^t, tile + 2
    T* Q0 = reinterpret_cast<T*>(L0 + L::N0);                            // q, tile + 2
    T* B0 = Q0 + L::N0;                                                  // bt/2, tile + 2 (edge-replicated)
    // two tile + 1 planes without their first and last (corner) cells: X holds
    // u^{t-1} for the imaging of (lam^t, u^{t-1}), then w^{t-1}; Y holds u^{t-2}
    Vec<T, G>* X = reinterpret_cast<Vec<T, G>*>(B0 + L::N0) - 1;
    Vec<T, G>* Y = X + (L::N1 - 2);
    T* D = reinterpret_cast<T*>(Y + (L::N1 - 1));                        // damping
    const T* cur = it.lam + (int64_t)(t & (nl - 1)) * P;
    const T* p1 = it.lam + (int64_t)((t + 1) & (nl - 1)) * P;
    T* out1 = it.lam + (int64_t)((t - 1) & (nl - 1)) * P;
    T* out2 = it.lam + (int64_t)((t - 2) & (nl - 1)) * P;
    const T* um1 = it.seg + (int64_t)kmod(it, t - 2) * P;
    const T* um2 = it.seg + (int64_t)kmod(it, t - 3) * P;
    const int x0 = tile_x * kTileX, z0 = tile_z * L::TZ;
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    const int tile = tile_z * it.tiles_x + tile_x;
    const Span rcv = span_of(it.tile_off, tile), rcv_x = span_of(it.tile_off_x, tile);
    const T* cf = it.coef;
    const T* exd_p = it.ex;
    const T* ezd_p = it.ez;
    Acc* accK = it.acc;
    Acc* accB = it.acc + ncell;
    const int ix = x0 + (int)threadIdx.x;

    // one burst: lam^t and (q, bt/2) on the tile grown by 2; lam^{t+1}, u^{t-1},
    // u^{t-2} on the tile grown by 1; the damping profile; this thread's
    // imaging accumulators
    Vec<T, G> f0[L::P0], ua[L::P1], ub[L::P1], pvt[R], pvr;
    T q0[L::P0], b0[L::P0];
    Acc sK[R], sB[R];
    // this lane's cell of the ring between the tile and the tile grown by
    // one (grown-tile coordinates), for the lam^{t-1} it computes there
    int rex = 0, rez = 0;
    ring_cell<L::W1, L::TZ>(tid, rex, rez);
    const int rx1 = x0 - 1 + rex, rz1 = z0 - 1 + rez;
    const bool rin = tid < L::NR1 && rx1 >= 0 && rx1 < nx && rz1 >= 0 && rz1 < nz;
#pragma unroll
    for (int i = 0; i < L::P0; ++i) {
        const int c = tid + i * kBlock;
        int ix0, iz0;
        cell_of<T, G, R, true>(c, 2, x0, z0, ix0, iz0);
        const bool in = c < L::N0 && ix0 >= 0 && ix0 < nx && iz0 >= 0 && iz0 < nz;
        const uint32_t x = in ? (uint32_t)(iz0 * nx + ix0) : 0u;
        f0[i] = vkeep<T, G>(in, vload32<T, G>(cur, x));
        stage_coef<T>(cf, in, ix0, iz0, nx, nz, q0[i], b0[i]);
    }
#pragma unroll
    for (int i = 0; i < L::P1; ++i) {
        const int c = tid + i * kBlock;
        int ix1, iz1;
        cell_of<T, G, R, true>(c, 1, x0, z0, ix1, iz1);
        const bool in = c < L::N1 && ix1 >= 0 && ix1 < nx && iz1 >= 0 && iz1 < nz;
        const uint32_t x = in ? (uint32_t)(iz1 * nx + ix1) : 0u;
        ua[i] = vkeep<T, G>(in, vload32<T, G>(um1, x));
        ub[i] = vkeep<T, G>(in, vload32<T, G>(um2, x));
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int iz = z0 + (int)threadIdx.y * R + k;
        const uint32_t x = ix < nx && iz < nz ? (uint32_t)(iz * nx + ix) : 0u;
        sK[k] = ldg32(accK, x);
        sB[k] = ldg32(accB, x);
        pvt[k] = vload32<T, G>(p1, x);
    }
    pvr = vload32<T, G>(p1, rin ? (uint32_t)(rz1 * nx + rx1) : 0u);
    const T dmp = damping_of<T, L::W0, L::ND>(exd_p, ezd_p, nx, nz, tid, x0, z0);
#pragma unroll
    for (int i = 0; i < L::P0; ++i) {
        const int c = tid + i * kBlock;
        if (c < L::N0) {
            L0[c] = f0[i];
            Q0[c] = q0[i];
            B0[c] = b0[i];
        }
    }
#pragma unroll
    for (int i = 0; i < L::P1; ++i) {
        const int c = tid + i * kBlock;
        if (c > 0 && c < L::N1 - 1) {
            X[c] = ua[i];
            Y[c] = ub[i];
        }
    }
    if (tid < L::ND) D[tid] = dmp;
    __syncthreads();
    // lam^{t-1} on the tile grown by one cell, into registers until X is
    // free: at this lane's ring cell, then at its R tile cells together with
    // the imaging of (lam^t, u^{t-1}) there (summed over the transmits), which
    // shares the cell's face buoyancies and differences of lam^t
    Vec<T, G> m1r = vzero<T, G>(), m1t[R];
    if (rin) {
        const int k = (rez + 1) * L::W0 + rex + 1;
        T fw, fe, fn, fs, a, b;
        faces_h<T>(B0[k], B0[k - 1], B0[k + 1], B0[k - L::W0], B0[k + L::W0], fw, fe, fn, fs);
        damp_coeffs<T>(D[rex + 1] + D[L::W0 + rez + 1], a, b);
        const T qc = Q0[k];
        const Vec<T, G> l0 = L0[k], lw = L0[k - 1], le = L0[k + 1], ln = L0[k - L::W0], ls = L0[k + L::W0];
#pragma unroll
        for (int g = 0; g < G; ++g)
            m1r.v[g] = adjw_cell<T>(a, b, qc, fw, fe, fn, fs, l0.v[g], lw.v[g], le.v[g], ln.v[g], ls.v[g], pvr.v[g]);
    }
    const bool hw = ix > 0, he = ix < nx - 1;
    const T hf = T(0.5);
    const T cw = hw ? hf : T(1), ce = he ? hf : T(1);
    Acc ska[R], sba[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int ez = (int)threadIdx.y * R + k, iz = z0 + ez;
        m1t[k] = vzero<T, G>();
        ska[k] = Acc(0);
        sba[k] = Acc(0);
        if (ix < nx && iz < nz) {
            const int k1 = (ez + 1) * L::W1 + threadIdx.x + 1;
            const int k0 = (ez + 2) * L::W0 + threadIdx.x + 2;
            const bool hn = iz > 0, hs = iz < nz - 1;
            T fw, fe, fn, fs, a, b;
            faces_h<T>(B0[k0], B0[k0 - 1], B0[k0 + 1], B0[k0 - L::W0], B0[k0 + L::W0], fw, fe, fn, fs);
            damp_coeffs<T>(D[threadIdx.x + 2] + D[L::W0 + ez + 2], a, b);
            const T cn = hn ? hf : T(1), cs = hs ? hf : T(1);
            const T qc = Q0[k0];
            const Vec<T, G> l0 = L0[k0], lw = L0[k0 - 1], le = L0[k0 + 1], ln = L0[k0 - L::W0],
                            ls = L0[k0 + L::W0];
            const Vec<T, G> a0 = X[k1], aw = X[k1 - 1], ae = X[k1 + 1], an = X[k1 - L::W1], as = X[k1 + L::W1];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                m1t[k].v[g] = adjw_cell<T>(a, b, qc, fw, fe, fn, fs, l0.v[g], lw.v[g], le.v[g], ln.v[g], ls.v[g],
                                           pvt[k].v[g]);
                T k1a, b1a;
                image_cell<T>(fw, fe, fn, fs, cw, ce, cn, cs, l0.v[g], l0.v[g], lw.v[g], le.v[g], ln.v[g], ls.v[g],
                              a0.v[g], aw.v[g], ae.v[g], an.v[g], as.v[g], k1a, b1a);
                ska[k] += Acc(k1a);
                sba[k] += Acc(b1a);
            }
        }
    }
    __syncthreads();
    // the two corner cells of the grown tile, which no tile cell reads, are
    // not stored (X leaves them out)
    if (tid < L::NR1) {
        const int c = rez * L::W1 + rex;
        if (c > 0 && c < L::N1 - 1) X[c] = m1r;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) X[((int)threadIdx.y * R + k + 1) * L::W1 + threadIdx.x + 1] = m1t[k];
    __syncthreads();
    // adjoint source of lam^{t-1} (sample t-2, times q) at the receivers of
    // the grown tile (the two corner cells that X does not hold are read by
    // no tile cell)
    if (rcv_x.e1 > rcv_x.e0 && has_adj_source(it)) {
        for (int e = rcv_x.e0 + tid; e < rcv_x.e1; e += kBlock) {
            const Entry en = ld_entry(it.entries_x, e);
            if (en.run == 0) continue;
            T sum = T(0);
            for (int k = 0; k < en.run; ++k) sum += adj_source(it, ld_entry(it.entries_x, e + k), t - 2);
            const int cell = en.slot / G, g = en.slot - cell * G;
            const int cz = quo(cell, it.dnx), ex = cell - cz * nx - (x0 - 1), ez = cz - (z0 - 1);
            const int c = ez * L::W1 + ex;
            if (c > 0 && c < L::N1 - 1) X[c].v[g] += Q0[(ez + 1) * L::W0 + ex + 1] * sum;
        }
        __syncthreads();
    }
    // on the tile: lam^{t-2}, the imaging of (lam^{t-1}, u^{t-2})
    if (ix < nx) {
        const T exd = D[threadIdx.x + 2];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int ez = (int)threadIdx.y * R + k, iz = z0 + ez;
            if (iz < nz) {
                const int k1 = (ez + 1) * L::W1 + threadIdx.x + 1;
                const int k0 = (ez + 2) * L::W0 + threadIdx.x + 2;
                const uint32_t x = (uint32_t)(iz * nx + ix);
                const bool hn = iz > 0, hs = iz < nz - 1;
                T fw, fe, fn, fs, a, b;
                faces_h<T>(B0[k0], B0[k0 - 1], B0[k0 + 1], B0[k0 - L::W0], B0[k0 + L::W0], fw, fe, fn, fs);
                const T cn = hn ? hf : T(1), cs = hs ? hf : T(1);
                damp_coeffs<T>(exd + D[L::W0 + ez + 2], a, b);
                const T qc = Q0[k0];
                const Vec<T, G> l0 = L0[k0];
                const Vec<T, G> m0 = X[k1], mw = X[k1 - 1], me = X[k1 + 1], mn = X[k1 - L::W1],
                                ms = X[k1 + L::W1];
                const Vec<T, G> c0 = Y[k1], cw2 = Y[k1 - 1], ce2 = Y[k1 + 1], cn2 = Y[k1 - L::W1],
                                cs2 = Y[k1 + L::W1];
                Vec<T, G> r;
                Acc skb = Acc(0), sbb = Acc(0);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    r.v[g] = adjw_cell<T>(a, b, qc, fw, fe, fn, fs, m0.v[g], mw.v[g], me.v[g], mn.v[g], ms.v[g],
                                          l0.v[g]);
                    T k1b, b1b;
                    image_cell<T>(fw, fe, fn, fs, cw, ce, cn, cs, m0.v[g], m0.v[g], mw.v[g], me.v[g], mn.v[g],
                                  ms.v[g], c0.v[g], cw2.v[g], ce2.v[g], cn2.v[g], cs2.v[g], k1b, b1b);
                    skb += Acc(k1b);
                    sbb += Acc(b1b);
                }
                vstore32<T, G>(out1, x, m0);
                vstore32<T, G>(out2, x, r);
                // the two time levels' imaging sums are added to the accumulators one
                // after the other, exactly as two one-step launches would
                Acc vk = sK[k], vb = sB[k];
                vk += ska[k];
                vb += sba[k];
                vk += skb;
                vb += sbb;
                stg32(accK, x, vk);
                stg32(accB, x, vb);
            }
        }
    }
    // adjoint source of lam^{t-2}: sample t-3, times q
    inject_tile<true, G>(it, rcv, t - 3, out2);
}

// Item position at launch s of a call (mode shifts / limits the schedule).
template <typename T, typename Acc>
__device__ __forceinline__ Step item_step(const Item<T, Acc>& it, int s, int mode)
{
    Step st = decode_s(it.sc, mode == kRunAdjOnly ? s + it.sc.nf : s);
    if (mode == kRunFwdOnly && st.phase != kFwd) st.phase = kIdle;
    return st;
}

// Forward-type launches of one step at launch s; blocks[b] = (item, tile).
template <typename T, int G, typename Acc>
__global__ __launch_bounds__(kBlock) void fwd1_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s, int mode, int rows)
{
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if ((st.phase != kFwd && st.phase != kRecomp) || st.count != 1) return;
    tile_forward<T, G, Acc>(it, st, bt.y - quo(bt.y, it.dtx) * it.tiles_x, quo(bt.y, it.dtx), rows, st.phase == kFwd && it.sample);
}

// Forward-type launches of two steps, tiles of 64 x 4R cells.
template <typename T, int G, typename Acc, int R>
__global__ __launch_bounds__(kBlock) void fwd2_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s, int mode)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if ((st.phase != kFwd && st.phase != kRecomp) || st.count != 2) return;
    tile_forward2<T, G, Acc, R>(it, st, bt.y - quo(bt.y, it.dtx) * it.tiles_x, quo(bt.y, it.dtx), st.phase == kFwd && it.sample, smem);
}

// Forward-type launches of three steps, tiles of 64 x 4R cells.
template <typename T, int G, typename Acc, int R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Lds3<T, G, R>::kWaves))) void fwd3_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s, int mode)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if ((st.phase != kFwd && st.phase != kRecomp) || st.count != 3) return;
    tile_forward3<T, G, Acc, R>(it, st, bt.y - quo(bt.y, it.dtx) * it.tiles_x, quo(bt.y, it.dtx), st.phase == kFwd && it.sample, smem);
}

// Adjoint + imaging launches of one step.
template <typename T, int G, typename Acc>
__global__ __launch_bounds__(kBlock) void adj1_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s, int mode, int rows)
{
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if (st.phase != kAdj || st.count != 1) return;
    tile_adjoint<T, G, Acc>(it, st, bt.y - quo(bt.y, it.dtx) * it.tiles_x, quo(bt.y, it.dtx), rows);
}

// Adjoint + imaging launches of two steps, tiles of 64 x 4R cells.
template <typename T, int G, typename Acc, int R>
__global__ __launch_bounds__(kBlock) void adj2_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s, int mode)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if (st.phase != kAdj || st.count != 2) return;
    tile_adjoint2<T, G, Acc, R>(it, st, bt.y - quo(bt.y, it.dtx) * it.tiles_x, quo(bt.y, it.dtx), smem);
}

// ============================================================== fourth-order variant
//
// Staggered fourth-order differences: the flux through the face between
// cells j and j+1 of a row or column is bt_f (9/8 (u_{j+1} - u_j) - 1/24
// (u_{j+2} - u_{j-1})) with bt_f the mean of the two cells' bt, and the
// operator is 9/8 (F_{+1/2} - F_{-1/2}) - 1/24 (F_{+3/2} - F_{-3/2}) summed
// over both axes, so it reaches three cells out.  Outside the grid the
// fields are zero and bt repeats the nearest in-grid cell of the row or
// column (the staged value at the clamped position), the border rule of the
// second-order operator carried to the wider stencil.
//
// A face's flux enters the operator of the four cells around it, so each
// launch evaluates every face it needs once: the field(s) and (q, bt) are
// staged in LDS on the tile grown by three; each thread evaluates its share
// of the faces (the x-faces of the tile's rows, kTileX + 3 per row, then the
// z-faces of its columns, TZ + 3 per column) into registers; once every
// thread has read the staged values the faces are written over them; each
// cell then combines its eight faces.

template <typename T, int G, int R, bool ADJ>
struct Lds4 {
    static constexpr int TZ = kWavesZ * R;
    static constexpr int W = kTileX + 6, H = TZ + 6, N = W * H;        // tile grown by 3
    static constexpr int P = (N + kBlock - 1) / kBlock;                // staging shares per thread
    static constexpr int FXW = kTileX + 3;                             // x-faces per tile row
    static constexpr int NFX = TZ * FXW, NF = NFX + (TZ + 3) * kTileX; // x-faces, then z-faces
    static constexpr int PF = (NF + kBlock - 1) / kBlock;              // face shares per thread
    // staging: field [N] (adjoint: w^t, then u^{t-1}) and (q, bt) [N][2];
    // then, over it, the fluxes [NF] (adjoint: of w, then of u) and the
    // adjoint's imaging products [NF]
    static constexpr size_t stage = (size_t)N * (G * (ADJ ? 2 : 1) + 2) * sizeof(T);
    static constexpr size_t face = (size_t)NF * (G * (ADJ ? 2 : 1) + (ADJ ? 1 : 0)) * sizeof(T);
    static constexpr size_t bytes = stage > face ? stage : face;
};

// D v at a face from the four values around it (v_{j-1}, v_j, v_{j+1}, v_{j+2}).
template <typename T>
__device__ __forceinline__ T d4(T vm, T v0, T v1, T v2)
{
#pragma clang fp contract(off)
    return fma(T(9) / T(8), v1 - v0, (T(-1) / T(24)) * (v2 - vm));
}

// Combination of the four face fluxes around a cell.
template <typename T>
__device__ __forceinline__ T div4(T fm3, T fm1, T fp1, T fp3)
{
#pragma clang fp contract(off)
    return fma(T(9) / T(8), fp1 - fm1, (T(-1) / T(24)) * (fp3 - fm3));
}

// First of the four LDS cells that face f of a step's list differences, and
// the stride along its axis.  The step updates a region of CW x RH cells
// whose first cell sits at (OFF + 3, OFF + 3) of the staged layout (row width
// W); its list holds the x-faces, CW + 3 per row and row by row (face i of a
// row lies between the region's columns i - 3 and i - 2), then the z-faces,
// RH + 3 per column and stored by face row (face row j lies between the
// region's rows j - 3 and j - 2).
template <int W, int CW, int RH, int OFF>
__device__ __forceinline__ void face_cells(int f, int& k0, int& s)
{
    constexpr int FXW = CW + 3, NFX = RH * FXW;
    if (f < NFX) {
        const int r = f / FXW;
        k0 = (r + 3 + OFF) * W + (f - r * FXW) + OFF;
        s = 1;
    } else {
        const int h = f - NFX, j = h / CW;
        k0 = (j + OFF) * W + (h - j * CW) + 3 + OFF;
        s = W;
    }
}

// Flux bt_f D u through a face (k0, s) for every transmit.
template <typename T, int G>
__device__ __forceinline__ Vec<T, G> flux4(const Vec<T, G>* V, const T* C, int k0, int s)
{
    const Vec<T, G> a = V[k0], b = V[k0 + s], c = V[k0 + 2 * s], d = V[k0 + 3 * s];
    const T bf = T(0.5) * (C[2 * (k0 + s) + 1] + C[2 * (k0 + 2 * s) + 1]);
    Vec<T, G> r;
#pragma unroll
    for (int g = 0; g < G; ++g) r.v[g] = bf * d4<T>(a.v[g], b.v[g], c.v[g], d.v[g]);
    return r;
}

// The adjoint's face values: the fluxes bt_f D w and bt_f D u (w = q lam^t,
// u = u^{t-1}) for every transmit, and the imaging product sum_g D u D w.
template <typename T, int G>
__device__ __forceinline__ void flux4_adj(const Vec<T, G>* Wl, const Vec<T, G>* U, const T* C, int k0, int s,
                                          Vec<T, G>& fw, Vec<T, G>& fu, T& pr)
{
#pragma clang fp contract(off)
    const Vec<T, G> w0 = Wl[k0], w1 = Wl[k0 + s], w2 = Wl[k0 + 2 * s], w3 = Wl[k0 + 3 * s];
    const Vec<T, G> u0 = U[k0], u1 = U[k0 + s], u2 = U[k0 + 2 * s], u3 = U[k0 + 3 * s];
    const T bf = T(0.5) * (C[2 * (k0 + s) + 1] + C[2 * (k0 + 2 * s) + 1]);
    pr = T(0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const T dw = d4<T>(w0.v[g], w1.v[g], w2.v[g], w3.v[g]);
        const T du = d4<T>(u0.v[g], u1.v[g], u2.v[g], u3.v[g]);
        fw.v[g] = bf * dw;
        fu.v[g] = bf * du;
        pr = fma(du, dw, pr);
    }
}

// Imaging share of a cell's bt along one axis (position i of n) from the
// products at its four faces, p0 .. p3 at j - 3/2 .. j + 3/2: half of each
// neighbouring face, the whole face where the neighbour is a ghost repeating
// this cell, and the face between the two ghosts beyond a border cell.
template <typename T>
__device__ __forceinline__ T img4(T p0, T p1, T p2, T p3, int i, int n)
{
#pragma clang fp contract(off)
    const T hf = T(0.5);
    T s = (i == 0 ? p1 : hf * p1) + (i == n - 1 ? p2 : hf * p2);
    if (i == 0) s = s + p0;
    if (i == n - 1) s = s + p3;
    return s;
}

// Forward update (increment form) of the cell at (cx, cz) of a CW x RH
// region from its eight fluxes in F (the region's face list): v^{n+1} into vv
// (v^n given there), u^{n+1} returned.  Every fourth-order forward kernel
// updates a cell through this function, so launches of one and of two steps
// round a cell identically.
template <typename T, int G, int CW, int RH>
__device__ __forceinline__ Vec<T, G> cell4(const Vec<T, G>* F, int cx, int cz, T q, T e, const Vec<T, G>& u0,
                                          Vec<T, G>& vv, int cell, const Src<T, G>& sc, bool near)
{
    constexpr int FXW = CW + 3, NFX = RH * FXW;
    const int ax = cz * FXW + cx, az = NFX + cz * CW + cx;
    const Vec<T, G> x0f = F[ax], x1f = F[ax + 1], x2f = F[ax + 2], x3f = F[ax + 3];
    const Vec<T, G> z0f = F[az], z1f = F[az + CW], z2f = F[az + 2 * CW], z3f = F[az + 3 * CW];
    T nb, c2;
    damp_inc<T>(e, nb, c2);
    Vec<T, G> r;
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma clang fp contract(off)
        T Lu = div4<T>(x0f.v[g], x1f.v[g], x2f.v[g], x3f.v[g]);
        Lu += div4<T>(z0f.v[g], z1f.v[g], z2f.v[g], z3f.v[g]);
        vv.v[g] = fma(q, Lu, fma(nb, vv.v[g], c2 * u0.v[g]));
    }
    if (near) add_src<T, G>(vv, cell, sc);
#pragma unroll
    for (int g = 0; g < G; ++g) r.v[g] = u0.v[g] + vv.v[g];
    return r;
}

// Global loads of one tile of a one-step fourth-order launch, issued
// together and held in registers until the LDS is free: the field(s) (zero
// outside the grid) and (q, bt) at clamped positions on the tile grown by
// three, and at the lane's R cells v^n (forward) or w^{t+1} and the two
// imaging sums (adjoint), with the damping profile.
template <typename T, int G, typename Acc, int R, bool ADJ>
struct Load4 {
    using L = Lds4<T, G, R, ADJ>;
    Vec<T, G> a[L::P], b[ADJ ? L::P : 1];
    T q[L::P], bt[L::P];
    Vec<T, G> v[R];
    Acc sK[R], sB[R];
    T ez[R];
    T ex;
};

template <typename T, int G, typename Acc, int R, bool ADJ>
__device__ __forceinline__ void load4(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z,
                                      Load4<T, G, Acc, R, ADJ>& ld)
{
    using L = Lds4<T, G, R, ADJ>;
    const int nx = it.nx, nz = it.nz;
    const int x0 = tile_x * kTileX, z0 = tile_z * L::TZ;
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    const int ix = x0 + (int)threadIdx.x;
    const T* f1;
    const T* f2 = nullptr;
    const T* pv;
    if (ADJ) {
        const int t = st.n;
        f1 = it.lam + (int64_t)(t & (it.nlam - 1)) * it.plane;          // w^t
        f2 = it.seg + (int64_t)kmod(it, t - 2) * it.plane;              // u^{t-1}
        pv = it.lam + (int64_t)((t + 1) & (it.nlam - 1)) * it.plane;    // w^{t+1}
    } else {
        f1 = fwd_plane(it, st, st.n);                                   // u^n
        pv = vel_in(it, st, st.n);                                      // v^n
    }
#pragma unroll
    for (int i = 0; i < L::P; ++i) {
        const int c = tid + i * kBlock;
        const int gx = x0 - 3 + c % L::W, gz = z0 - 3 + c / L::W;
        const bool in = c < L::N && gx >= 0 && gx < nx && gz >= 0 && gz < nz;
        const int cx = min(max(gx, 0), nx - 1), cz = min(max(gz, 0), nz - 1);
        const uint32_t xc = c < L::N ? (uint32_t)(cz * nx + cx) : 0u;
        const uint32_t xi = in ? (uint32_t)(gz * nx + gx) : 0u;
        ld.a[i] = vkeep<T, G>(in, vload32<T, G>(f1, xi));
        if (ADJ) ld.b[i] = vkeep<T, G>(in, vload32<T, G>(f2, xi));
        ld.q[i] = ldg32(it.coef, 2 * xc);
        ld.bt[i] = ldg32(it.coef, 2 * xc + 1);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int iz = z0 + (int)threadIdx.y * R + k;
        const bool in = ix < nx && iz < nz;
        const uint32_t x = in ? (uint32_t)(iz * nx + ix) : 0u;
        ld.v[k] = vload32<T, G>(pv, x);
        if (ADJ) {
            ld.sK[k] = ldg32(it.acc, x);
            ld.sB[k] = ldg32(it.acc + (int64_t)nx * nz, x);
        }
        ld.ez[k] = ldg(it.ez, iz < nz ? iz : 0);
    }
    ld.ex = ldg(it.ex, ix < nx ? ix : 0);
}

// The staged values into LDS: field(s) F1 (F2) and (q, bt) C.
template <typename T, int G, typename Acc, int R, bool ADJ>
__device__ __forceinline__ void commit4(const Load4<T, G, Acc, R, ADJ>& ld, Vec<T, G>* F1, Vec<T, G>* F2, T* C)
{
    using L = Lds4<T, G, R, ADJ>;
    const int tid = threadIdx.y * kTileX + threadIdx.x;
#pragma unroll
    for (int i = 0; i < L::P; ++i) {
        const int c = tid + i * kBlock;
        if (c < L::N) {
            F1[c] = ld.a[i];
            if (ADJ) F2[c] = ld.b[i];
            C[2 * c] = ld.q[i];
            C[2 * c + 1] = ld.bt[i];
        }
    }
}

// Forward step n of one tile from the staged values (committed to LDS and
// made visible by the caller's barrier).
template <typename T, int G, typename Acc, int R>
__device__ void tile_forward4(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, bool sample,
                              unsigned char* smem, const Load4<T, G, Acc, R, false>& ld)
{
    using L = Lds4<T, G, R, false>;
    const int nx = it.nx, nz = it.nz, n = st.n;
    const Vec<T, G>* U = reinterpret_cast<const Vec<T, G>*>(smem);
    const T* C = reinterpret_cast<const T*>(U + L::N);
    Vec<T, G>* F = reinterpret_cast<Vec<T, G>*>(smem);                  // fluxes, over the staging
    T* out = it.seg + (int64_t)kmod(it, n) * it.plane;
    T* vout = vel_out(it, st, n + 1);
    T* ckv = ckpt_pair(it, st, n + 1);
    const Src<T, G> src = sources<T, G>(it, n);
    const Span rcv = sample ? span_of(it.tile_off, tile_z * it.tiles_x + tile_x) : Span{0, 0};
    const int x0 = tile_x * kTileX, z0 = tile_z * L::TZ;
    // a source within the cells this launch updates (the tile)
    const bool near = src_near<T, G, Acc>(src, it, x0, z0, 0, kTileX, 0, L::TZ);
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    const int tx = (int)threadIdx.x, ix = x0 + tx;
    // the lane's own u^n and q, then its faces, before the fluxes overwrite them
    Vec<T, G> u0[R], vt[R];
    T qc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int kk = ((int)threadIdx.y * R + k + 3) * L::W + tx + 3;
        u0[k] = U[kk];
        qc[k] = C[2 * kk];
        vt[k] = ld.v[k];
    }
    Vec<T, G> fl[L::PF];
#pragma unroll
    for (int i = 0; i < L::PF; ++i) {
        const int f = tid + i * kBlock;
        if (f < L::NF) {
            int k0, s;
            face_cells<L::W, kTileX, L::TZ, 0>(f, k0, s);
            fl[i] = flux4<T, G>(U, C, k0, s);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < L::PF; ++i) {
        const int f = tid + i * kBlock;
        if (f < L::NF) F[f] = fl[i];
    }
    __syncthreads();
    if (ix < nx) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int z = (int)threadIdx.y * R + k, iz = z0 + z;
            if (iz < nz) {
                const uint32_t x = (uint32_t)(iz * nx + ix);
                const Vec<T, G> r =
                    cell4<T, G, kTileX, L::TZ>(F, tx, z, qc[k], ld.ex + ld.ez[k], u0[k], vt[k], (int)x, src, near);
                vstore32<T, G>(out, x, r);
                vstore32<T, G>(vout, x, vt[k]);
                if (ckv) {
                    vstore32<T, G>(ckv, x, vt[k]);
                    vstore32<T, G>(ckv + it.plane, x, r);
                }
            }
        }
    }
    sample_tile(it, rcv, n, out, (const T*)nullptr);
}

// Adjoint step t of one tile, with the imaging of (w^t, u^{t-1}), from the
// staged values (committed and made visible by the caller).
template <typename T, int G, typename Acc, int R>
__device__ void tile_adjoint4(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, unsigned char* smem,
                              const Load4<T, G, Acc, R, true>& ld)
{
    using L = Lds4<T, G, R, true>;
    const int nx = it.nx, nz = it.nz, t = st.n;
    const int64_t P = it.plane, ncell = (int64_t)nx * nz;
    // the planes hold w = q lam, as for the second-order operator: w^{t-1} =
    // a w^t + b w^{t+1} + q (flux terms of w), and the kappa term w^t L u is q
    // times the lambda one (undone when the gradient is formed)
    const Vec<T, G>* Lm = reinterpret_cast<const Vec<T, G>*>(smem);     // w^t
    const Vec<T, G>* U = Lm + L::N;                                     // u^{t-1}
    const T* C = reinterpret_cast<const T*>(U + L::N);
    Vec<T, G>* FW = reinterpret_cast<Vec<T, G>*>(smem);                 // faces, over the staging
    Vec<T, G>* FU = FW + L::NF;
    T* FP = reinterpret_cast<T*>(FU + L::NF);
    T* out = it.lam + (int64_t)((t - 1) & (it.nlam - 1)) * P;           // w^{t-1}
    Acc* accK = it.acc;
    Acc* accB = it.acc + ncell;
    const Span rcv = span_of(it.tile_off, tile_z * it.tiles_x + tile_x);
    const int x0 = tile_x * kTileX, z0 = tile_z * L::TZ;
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    const int tx = (int)threadIdx.x, ix = x0 + tx;
    Vec<T, G> w0[R];
    T qc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int kk = ((int)threadIdx.y * R + k + 3) * L::W + tx + 3;
        w0[k] = Lm[kk];
        qc[k] = C[2 * kk];
    }
    Vec<T, G> fw[L::PF], fu[L::PF];
    T pr[L::PF];
#pragma unroll
    for (int i = 0; i < L::PF; ++i) {
        const int f = tid + i * kBlock;
        if (f < L::NF) {
            int k0, s;
            face_cells<L::W, kTileX, L::TZ, 0>(f, k0, s);
            flux4_adj<T, G>(Lm, U, C, k0, s, fw[i], fu[i], pr[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < L::PF; ++i) {
        const int f = tid + i * kBlock;
        if (f < L::NF) {
            FW[f] = fw[i];
            FU[f] = fu[i];
            FP[f] = pr[i];
        }
    }
    __syncthreads();
    if (ix < nx) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int z = (int)threadIdx.y * R + k, iz = z0 + z;
            if (iz < nz) {
                const int ax = z * L::FXW + tx, az = L::NFX + z * kTileX + tx;
                T a, b;
                damp_coeffs<T>(ld.ex + ld.ez[k], a, b);
                const uint32_t x = (uint32_t)(iz * nx + ix);
                Vec<T, G> r;
                Acc sk = Acc(0);
                {
                    const Vec<T, G> f0 = FW[ax], f1 = FW[ax + 1], f2 = FW[ax + 2], f3 = FW[ax + 3];
                    const Vec<T, G> h0 = FW[az], h1 = FW[az + kTileX], h2 = FW[az + 2 * kTileX],
                                    h3 = FW[az + 3 * kTileX];
#pragma unroll
                    for (int g = 0; g < G; ++g) {
#pragma clang fp contract(off)
                        T Lw = div4<T>(f0.v[g], f1.v[g], f2.v[g], f3.v[g]);
                        Lw += div4<T>(h0.v[g], h1.v[g], h2.v[g], h3.v[g]);
                        r.v[g] = fma(a, w0[k].v[g], fma(b, ld.v[k].v[g], qc[k] * Lw));
                    }
                }
                {
                    const Vec<T, G> f0 = FU[ax], f1 = FU[ax + 1], f2 = FU[ax + 2], f3 = FU[ax + 3];
                    const Vec<T, G> h0 = FU[az], h1 = FU[az + kTileX], h2 = FU[az + 2 * kTileX],
                                    h3 = FU[az + 3 * kTileX];
#pragma unroll
                    for (int g = 0; g < G; ++g) {
#pragma clang fp contract(off)
                        T Lu = div4<T>(f0.v[g], f1.v[g], f2.v[g], f3.v[g]);
                        Lu += div4<T>(h0.v[g], h1.v[g], h2.v[g], h3.v[g]);
                        sk += Acc(w0[k].v[g] * Lu);
                    }
                }
                const Acc sb = Acc(img4<T>(FP[ax], FP[ax + 1], FP[ax + 2], FP[ax + 3], ix, nx)) +
                               Acc(img4<T>(FP[az], FP[az + kTileX], FP[az + 2 * kTileX], FP[az + 3 * kTileX], iz, nz));
                vstore32<T, G>(out, x, r);
                stg32(accK, x, ld.sK[k] + sk);
                stg32(accB, x, ld.sB[k] + sb);
            }
        }
    }
    // adjoint source of w^{t-1}: q times sample t-2
    inject_tile<true, G>(it, rcv, t - 2, out);
}

// Two fourth-order forward steps per launch.  u^n and (q, bt) are staged on
// the tile grown by six; step n runs on the tile grown by three (whose faces
// read three cells further out), step n+1 on the tile.  Each lane keeps v in
// registers for its R tile cells and for its share of the ring between the
// tile and the tile grown by three, so v is read once per launch; u^{n+1}
// goes back into the staged layout (zero outside the grid) for step n+1.
template <typename T, int G, int R>
struct Lds4x2 {
    static constexpr int TZ = kWavesZ * R;
    static constexpr int W = kTileX + 12, H = TZ + 12, N = W * H;        // tile grown by 6
    static constexpr int P = (N + kBlock - 1) / kBlock;                 // staging shares per thread
    static constexpr int CW1 = kTileX + 6, RH1 = TZ + 6;                 // step n: tile grown by 3
    static constexpr int NR = CW1 * RH1 - kTileX * TZ;                   // its ring around the tile
    static constexpr int PR = (NR + kBlock - 1) / kBlock;               // ring cells per thread
    static constexpr int NF1 = RH1 * (CW1 + 3) + (RH1 + 3) * CW1;        // faces of step n
    static constexpr int NF2 = TZ * (kTileX + 3) + (TZ + 3) * kTileX;    // faces of step n+1
    static constexpr int PF1 = (NF1 + kBlock - 1) / kBlock, PF2 = (NF2 + kBlock - 1) / kBlock;
    // one region holding in turn u^n [N], the fluxes of step n [NF1], u^{n+1}
    // [N] and the fluxes of step n+1 [NF2]; then (q, bt) [N][2]
    static constexpr size_t field = (size_t)(N > NF1 ? N : NF1) * G * sizeof(T);
    static constexpr size_t bytes = field + (size_t)N * 2 * sizeof(T);
};

// Cell c of the ring between the tile (kTileX x TZ) and the tile grown by
// three, tile-relative: the three rows above, the three below (full width),
// then the three columns left and right of the tile's rows.
template <int TZ>
__device__ __forceinline__ void ring4_cell(int c, int& x, int& z)
{
    constexpr int WR = kTileX + 6, TB = 3 * WR;
    if (c < TB) {
        z = c / WR - 3;
        x = c % WR - 3;
    } else if (c < 2 * TB) {
        c -= TB;
        z = TZ + c / WR;
        x = c % WR - 3;
    } else if (c < 2 * TB + 3 * TZ) {
        c -= 2 * TB;
        z = c / 3;
        x = c % 3 - 3;
    } else {
        c -= 2 * TB + 3 * TZ;
        z = c / 3;
        x = kTileX + c % 3;
    }
}

template <typename T, int G, typename Acc, int R>
__device__ void tile_forward4x2(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, bool sample,
                                unsigned char* smem)
{
    using L = Lds4x2<T, G, R>;
    constexpr int W = L::W;
    const int nx = it.nx, nz = it.nz, n = st.n;
    Vec<T, G>* U = reinterpret_cast<Vec<T, G>*>(smem);       // u^n, fluxes, u^{n+1}, fluxes
    T* C = reinterpret_cast<T*>(smem + L::field);             // (q, bt) on the tile grown by 6
    const T* cur = fwd_plane(it, st, n);
    const T* vin = vel_in(it, st, n);
    T* out1 = it.seg + (int64_t)kmod(it, n) * it.plane;
    T* out2 = it.seg + (int64_t)kmod(it, n + 1) * it.plane;
    T* vout = vel_out(it, st, n + 2);
    T* ck1 = ckpt_pair(it, st, n + 1);
    T* ck2 = ckpt_pair(it, st, n + 2);
    // u^{n+1} is stored only where the adjoint will read it
    const bool keep1 = st.phase != kFwd || n + 1 >= it.keep_from;
    const Src<T, G> s1 = sources<T, G>(it, n);
    const Src<T, G> s2 = sources<T, G>(it, n + 1);
    const Span rcv = sample ? span_of(it.tile_off, tile_z * it.tiles_x + tile_x) : Span{0, 0};
    const int x0 = tile_x * kTileX, z0 = tile_z * L::TZ;
    // a source within the cells this launch updates (step n on the tile grown by three)
    const bool near = src_near<T, G, Acc>(s1, it, x0, z0, -3, kTileX + 3, -3, L::TZ + 3);
    const int tid = threadIdx.y * kTileX + threadIdx.x;
    const int tx = (int)threadIdx.x, ix = x0 + tx;

    // this lane's ring cells (tile-relative), each in the grid or not
    int rx[L::PR], rz[L::PR];
    bool rin[L::PR];
#pragma unroll
    for (int i = 0; i < L::PR; ++i) {
        const int c = tid + i * kBlock;
        ring4_cell<L::TZ>(c, rx[i], rz[i]);
        const int gx = x0 + rx[i], gz = z0 + rz[i];
        rin[i] = c < L::NR && gx >= 0 && gx < nx && gz >= 0 && gz < nz;
    }

    // one burst: u^n (zero outside the grid) and (q, bt) at clamped
    // positions on the tile grown by 6; v^n and e = (D_x + D_z) dt at the
    // lane's tile and ring cells
    Vec<T, G> fv[L::P];
    T qv[L::P], bv[L::P];
#pragma unroll
    for (int i = 0; i < L::P; ++i) {
        const int c = tid + i * kBlock;
        const int gx = x0 - 6 + c % W, gz = z0 - 6 + c / W;
        const bool in = c < L::N && gx >= 0 && gx < nx && gz >= 0 && gz < nz;
        const int cx = min(max(gx, 0), nx - 1), cz = min(max(gz, 0), nz - 1);
        const uint32_t xc = c < L::N ? (uint32_t)(cz * nx + cx) : 0u;
        fv[i] = vkeep<T, G>(in, vload32<T, G>(cur, in ? (uint32_t)(gz * nx + gx) : 0u));
        qv[i] = ldg32(it.coef, 2 * xc);
        bv[i] = ldg32(it.coef, 2 * xc + 1);
    }
    Vec<T, G> vt[R], vr[L::PR];
    T et[R], er[L::PR];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int iz = z0 + (int)threadIdx.y * R + k;
        const bool in = ix < nx && iz < nz;
        vt[k] = vload32<T, G>(vin, in ? (uint32_t)(iz * nx + ix) : 0u);
        et[k] = ldg(it.ex, ix < nx ? ix : 0) + ldg(it.ez, iz < nz ? iz : 0);
    }
#pragma unroll
    for (int i = 0; i < L::PR; ++i) {
        const int gx = x0 + rx[i], gz = z0 + rz[i];
        vr[i] = vload32<T, G>(vin, rin[i] ? (uint32_t)(gz * nx + gx) : 0u);
        er[i] = ldg(it.ex, rin[i] ? gx : 0) + ldg(it.ez, rin[i] ? gz : 0);
    }
#pragma unroll
    for (int i = 0; i < L::P; ++i) {
        const int c = tid + i * kBlock;
        if (c < L::N) {
            U[c] = fv[i];
            C[2 * c] = qv[i];
            C[2 * c + 1] = bv[i];
        }
    }
    __syncthreads();

    // the lane's own u^n and q, then the fluxes of step n, before they
    // overwrite u^n
    Vec<T, G> ut[R], ur[L::PR];
    T qt[R], qr[L::PR];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int kk = ((int)threadIdx.y * R + k + 6) * W + tx + 6;
        ut[k] = U[kk];
        qt[k] = C[2 * kk];
    }
#pragma unroll
    for (int i = 0; i < L::PR; ++i) {
        const int kk = tid + i * kBlock < L::NR ? (rz[i] + 6) * W + rx[i] + 6 : 0;
        ur[i] = U[kk];
        qr[i] = C[2 * kk];
    }
    {
        Vec<T, G> fl[L::PF1];
#pragma unroll
        for (int i = 0; i < L::PF1; ++i) {
            const int f = tid + i * kBlock;
            if (f < L::NF1) {
                int k0, s;
                face_cells<W, L::CW1, L::RH1, 0>(f, k0, s);
                fl[i] = flux4<T, G>(U, C, k0, s);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < L::PF1; ++i) {
            const int f = tid + i * kBlock;
            if (f < L::NF1) U[f] = fl[i];
        }
    }
    __syncthreads();

    // step n on the tile grown by three; outside the grid u stays zero
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int z = (int)threadIdx.y * R + k, iz = z0 + z;
        if (ix < nx && iz < nz) {
            const uint32_t x = (uint32_t)(iz * nx + ix);
            ut[k] = cell4<T, G, L::CW1, L::RH1>(U, tx + 3, z + 3, qt[k], et[k], ut[k], vt[k], (int)x, s1, near);
            if (keep1) vstore32<T, G>(out1, x, ut[k]);
            if (ck1) {
                vstore32<T, G>(ck1, x, vt[k]);
                vstore32<T, G>(ck1 + it.plane, x, ut[k]);
            }
        } else {
            ut[k] = vzero<T, G>();
        }
    }
#pragma unroll
    for (int i = 0; i < L::PR; ++i) {
        if (rin[i]) {
            const int cell = (z0 + rz[i]) * nx + x0 + rx[i];
            ur[i] = cell4<T, G, L::CW1, L::RH1>(U, rx[i] + 3, rz[i] + 3, qr[i], er[i], ur[i], vr[i], cell, s1, near);
        } else {
            ur[i] = vzero<T, G>();
        }
    }
    __syncthreads();
    // u^{n+1} over the fluxes, in the staged layout
#pragma unroll
    for (int k = 0; k < R; ++k) U[((int)threadIdx.y * R + k + 6) * W + tx + 6] = ut[k];
#pragma unroll
    for (int i = 0; i < L::PR; ++i)
        if (tid + i * kBlock < L::NR) U[(rz[i] + 6) * W + rx[i] + 6] = ur[i];
    __syncthreads();
    if (rcv.e1 > rcv.e0) sample_lds<T, G, 6>(it, rcv, n, U, W, x0, z0);

    // the fluxes of step n+1, then step n+1 on the tile
    {
        Vec<T, G> fl[L::PF2];
#pragma unroll
        for (int i = 0; i < L::PF2; ++i) {
            const int f = tid + i * kBlock;
            if (f < L::NF2) {
                int k0, s;
                face_cells<W, kTileX, L::TZ, 3>(f, k0, s);
                fl[i] = flux4<T, G>(U, C, k0, s);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < L::PF2; ++i) {
            const int f = tid + i * kBlock;
            if (f < L::NF2) U[f] = fl[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int z = (int)threadIdx.y * R + k, iz = z0 + z;
        if (ix < nx && iz < nz) {
            const uint32_t x = (uint32_t)(iz * nx + ix);
            const Vec<T, G> r = cell4<T, G, kTileX, L::TZ>(U, tx, z, qt[k], et[k], ut[k], vt[k], (int)x, s2, near);
            vstore32<T, G>(out2, x, r);
            vstore32<T, G>(vout, x, vt[k]);
            if (ck2) {
                vstore32<T, G>(ck2, x, vt[k]);
                vstore32<T, G>(ck2 + it.plane, x, r);
            }
        }
    }
    // trace d[n+1] from the stored u^{n+2}
    if (rcv.e1 > rcv.e0) {
        __syncthreads();
        for (int e = rcv.e0 + tid; e < rcv.e1; e += kBlock) {
            const Entry en = ld_entry(it.entries, e);
            stg(it.traces, en.trace_off + (int64_t)(n + 1) * it.n_rcv, ldg(out2, en.slot));
        }
    }
}

// One-step fourth-order launches: one tile per workgroup; its global loads
// are issued together (load4), then written to LDS (commit4).
template <typename T, int G, typename Acc, int R, bool ADJ>
__device__ __forceinline__ void one_tile4(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z,
                                          unsigned char* smem)
{
    using L = Lds4<T, G, R, ADJ>;
    Vec<T, G>* F1 = reinterpret_cast<Vec<T, G>*>(smem);
    Vec<T, G>* F2 = F1 + L::N;
    T* C = reinterpret_cast<T*>(F1 + (ADJ ? 2 : 1) * L::N);
    Load4<T, G, Acc, R, ADJ> ld;
    load4<T, G, Acc, R, ADJ>(it, st, tile_x, tile_z, ld);
    commit4<T, G, Acc, R, ADJ>(ld, F1, F2, C);
    __syncthreads();
    if constexpr (ADJ)
        tile_adjoint4<T, G, Acc, R>(it, st, tile_x, tile_z, smem, ld);
    else
        tile_forward4<T, G, Acc, R>(it, st, tile_x, tile_z, st.phase == kFwd && it.sample, smem, ld);
}

template <typename T, int G, typename Acc, int R>
__global__ __launch_bounds__(kBlock) void fwd4_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s, int mode)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if ((st.phase != kFwd && st.phase != kRecomp) || st.count != 1) return;
    const int tz = quo(bt.y, it.dtx);
    one_tile4<T, G, Acc, R, false>(it, st, bt.y - tz * it.tiles_x, tz, smem);
}

template <typename T, int G, typename Acc, int R>
__global__ __launch_bounds__(kBlock) void fwd4x2_kernel(const Item<T, Acc>* __restrict__ items,
                                                         const int2* __restrict__ blocks, int s, int mode)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if ((st.phase != kFwd && st.phase != kRecomp) || st.count != 2) return;
    tile_forward4x2<T, G, Acc, R>(it, st, bt.y - quo(bt.y, it.dtx) * it.tiles_x, quo(bt.y, it.dtx), st.phase == kFwd && it.sample, smem);
}

template <typename T, int G, typename Acc, int R>
__global__ __launch_bounds__(kBlock) void adj4_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s, int mode)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blocks[blockIdx.x];
    if (bt.x < 0) return;
    const Item<T, Acc>& it = items[bt.x];
    const Step st = item_step(it, s, mode);
    if (st.phase != kAdj) return;
    const int tz = quo(bt.y, it.dtx);
    one_tile4<T, G, Acc, R, true>(it, st, bt.y - tz * it.tiles_x, tz, smem);
}

// ---------------------------------------------------------------- persistent form
//
// One launch runs every step of a wave: each workgroup walks its share of
// the launch's blocks (block b on workgroup b mod grid, so the XCD dealing
// of the block table is kept when the grid is a multiple of 8), then all
// workgroups meet at a grid barrier before the next step.  The grid never
// exceeds what is co-resident.  The barrier is bounded: a workgroup that
// polls spin_limit times without the barrier opening raises the abort
// word, every workgroup then leaves, and the host reports the failure.

// bar[0]: arrivals, bar[1]: generation, bar[2]: abort.
// One agent-scope release fence per workgroup before it arrives (its stores,
// and those of the workgroup's other waves ordered by the workgroup barrier,
// written back from this XCD's L2) and one agent-scope acquire fence after
// the generation moved (stale lines of this XCD's caches invalidated); the
// counter and the flag are relaxed atomics, except the last arrival's
// release of the new generation.  Each fence costs a pass over the XCD's L2,
// so there is one of each per workgroup.
__device__ __forceinline__ bool grid_sync(unsigned* bar, unsigned nblocks, unsigned spin_limit)
{
    __shared__ unsigned ok;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        bool good = true;
        // the generation cannot move before this workgroup arrives
        const unsigned g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned a = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a + 1 == nblocks) {
            // the reset of the counter is released with the new generation
            // (acquired by the waiting workgroups' fence below)
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned polls = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    ++polls > spin_limit) {
                    good = false;
                    __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = good ? 1u : 0u;
    }
    __syncthreads();
    return ok != 0u;
}

template <typename T, int G, typename Acc, int R>
__global__ __launch_bounds__(kBlock) void persistent_kernel(const Item<T, Acc>* __restrict__ items,
                                                             const int2* __restrict__ blocks,
                                                             const int* __restrict__ nblk, int n_launch, int mode,
                                                             int rows, unsigned* bar, unsigned spin_limit,
                                                             unsigned* status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    for (int s = 0; s < n_launch; ++s) {
        const int nb = nblk[s];
        for (int b = blockIdx.x; b < nb; b += gridDim.x) {
            const int2 bt = blocks[b];
            if (bt.x >= 0) {
                const Item<T, Acc>& it = items[bt.x];
                const Step st = item_step(it, s, mode);
                const int tz = quo(bt.y, it.dtx), tx = bt.y - tz * it.tiles_x;
                if (st.phase == kFwd || st.phase == kRecomp) {
                    const bool smp = st.phase == kFwd && it.sample;
                    if (st.count == 2) tile_forward2<T, G, Acc, R, 1>(it, st, tx, tz, smp, smem);
                    else tile_forward<T, G, Acc, 1>(it, st, tx, tz, rows, smp);
                } else if (st.phase == kAdj) {
                    if (st.count == 2) tile_adjoint2<T, G, Acc, R, 1>(it, st, tx, tz, smem);
                    else tile_adjoint<T, G, Acc, 1>(it, st, tx, tz, rows);
                }
            }
            __syncthreads();   // LDS is reused by this workgroup's next block
        }
        if (s + 1 < n_launch && !grid_sync(bar, gridDim.x, spin_limit)) {
            if (threadIdx.x == 0 && threadIdx.y == 0) atomicOr(status, kFlagBarrier);
            return;
        }
    }
}

// ---------------------------------------------------------------- medium prep

template <typename T>
struct MediumDev {
    int32_t nx, nz, item0, item1;     // items [item0, item1) own accumulators of this medium
    int32_t n_tx, nt, n_rcv, pad;
    double h, dt, dmax, c_max;
    int32_t npml, pad2;
    int64_t acc_stride;               // elements between two accumulator slots
    const T* c;
    const T* rho;
    T* coef;
    const T* traces;
    const T* d_obs;
    T* grad_c;
    T* grad_rho;
    double* misfit;
    const void* acc0;                 // first accumulator slot of the medium
    int32_t acc_slots;
    int32_t pad3;
    const T* eta;                     // attenuation rate (1/s), or NULL
    T* eatt;                          // workspace: eta dt per cell, or NULL
    T* grad_eta;                      // out dJ/deta, or NULL
};

__device__ __forceinline__ double dprof(int i, int n, int N, double dmax)
{
    if (i < N) {
        const double r = (double)(N - i) / N;
        return dmax * r * r;
    }
    if (i > n - 1 - N) {
        const double r = (double)(i - (n - 1 - N)) / N;
        return dmax * r * r;
    }
    return 0.0;
}

// (Q, bt) per cell in double, rounded once to T; flags unusable media.
template <typename T>
__global__ void prep_kernel(const MediumDev<T>* __restrict__ media, unsigned* status)
{
    const MediumDev<T>& m = media[blockIdx.y];
    const int64_t n = (int64_t)m.nx * m.nz;
    const double ih2 = 1.0 / (m.h * m.h);
    unsigned flag = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(x % m.nx), iz = (int)(x / m.nx);
        const double c = (double)m.c[x], rho = (double)m.rho[x];
        if (!(c > 0.0) || !(rho > 0.0) || !isfinite(c) || !isfinite(rho)) flag |= kFlagMedium;
        if (c > m.c_max) flag |= kFlagCfl;
        double e = (dprof(ix, m.nx, m.npml, m.dmax) + dprof(iz, m.nz, m.npml, m.dmax)) * m.dt;
        if (m.eatt) {
            // attenuation joins the damping: gamma below takes it too
            const double eta = m.eta ? (double)m.eta[x] : 0.0;
            if (!(eta >= 0.0) || !isfinite(eta)) flag |= kFlagMedium;
            const T ea = (T)(eta * m.dt);
            m.eatt[x] = ea;
            e += (double)ea;
        }
        const double gam = m.dt * m.dt / (1.0 + e);
        const double q = gam * rho * c * c * ih2 / kRhoRef;
        m.coef[2 * x] = (T)q;
        m.coef[2 * x + 1] = (T)(kRhoRef / rho);
    }
    if (flag) atomicOr(status, flag);
}

// Fill n elements of type T with zero (graph-safe replacement of memset).
template <typename T>
__global__ void zero_kernel(T* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

// Fill n elements with v (synthetic probe inputs of the autotuner).
template <typename T>
__global__ void fill_kernel(T* __restrict__ p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Misfit partial sums: block b of medium m sums (d - d_obs)^2 over a strided
// share.  Without observed traces it sums (0 d)^2, which is zero unless a
// trace sample is not finite, so that every forward solve checks its traces.
constexpr int kMisfitBlocks = 64;

template <typename T>
__global__ __launch_bounds__(256) void misfit_partial_kernel(const MediumDev<T>* __restrict__ media,
                                                              double* __restrict__ partial)
{
    const MediumDev<T>& m = media[blockIdx.y];
    __shared__ double red[4];
    double s = 0.0;
    const int64_t n = (int64_t)m.n_tx * m.nt * m.n_rcv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)m.traces[i];
        const double r = m.d_obs ? d - (double)m.d_obs[i] : 0.0 * d;
        s += r * r;
    }
    // wavefront reduction by lane shuffles, then the four wave sums in a fixed order
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.y * kMisfitBlocks + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
__global__ void misfit_final_kernel(const MediumDev<T>* __restrict__ media, int n_media,
                                    const double* __restrict__ partial, unsigned* status)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_media) return;
    const MediumDev<T>& md = media[m];
    double s = 0.0;
    for (int b = 0; b < kMisfitBlocks; ++b) s += partial[m * kMisfitBlocks + b];
    if (!isfinite(s)) atomicOr(status, kFlagNonfinite);
    if (md.misfit) *md.misfit = md.d_obs ? s : 0.0;
}

// g_kappa = gamma/(h^2 rho_ref) S_kappa, g_b = -rho_ref S_b, summed over the
// medium's accumulator slots in order; g_c = 2 rho c g_kappa,
// g_rho = c^2 g_kappa - g_b / rho^2.
template <typename T, typename Acc>
__global__ void finalize_kernel(const MediumDev<T>* __restrict__ media, unsigned* status)
{
    const MediumDev<T>& m = media[blockIdx.y];
    const int64_t n = (int64_t)m.nx * m.nz;
    const Acc* acc = reinterpret_cast<const Acc*>(m.acc0);
    unsigned flag = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        double sk = 0.0, sb = 0.0;
        for (int k = 0; k < m.acc_slots; ++k) {
            sk += (double)acc[k * m.acc_stride + x];
            sb += (double)acc[k * m.acc_stride + n + x];
        }
        const int ix = (int)(x % m.nx), iz = (int)(x / m.nx);
        double e = (dprof(ix, m.nx, m.npml, m.dmax) + dprof(iz, m.nz, m.npml, m.dmax)) * m.dt;
        if (m.eatt) e += (double)m.eatt[x];
        const double gam = m.dt * m.dt / (1.0 + e);
        // the adjoint kernels carry w = q lam, so the kappa sum is q times
        // the lam one, q the stored coefficient they multiplied by
        sk /= (double)m.coef[2 * x];
        const double gk = gam / (m.h * m.h * kRhoRef) * sk;
        const double gb = -kRhoRef * sb;
        const double c = (double)m.c[x], rho = (double)m.rho[x];
        const double gc = 2.0 * rho * c * gk;
        const double gr = c * c * gk - gb / (rho * rho);
        if (!isfinite(gc) || !isfinite(gr)) flag |= kFlagNonfinite;
        if (m.grad_c) m.grad_c[x] = (T)gc;
        if (m.grad_rho) m.grad_rho[x] = (T)gr;
        if (m.eatt) {
            // dJ/deta = dt dJ/de, the third accumulator of each slot
            double se = 0.0;
            for (int k = 0; k < m.acc_slots; ++k) se += (double)acc[k * m.acc_stride + 2 * n + x];
            const double ge = m.dt * se;
            if (!isfinite(ge)) flag |= kFlagNonfinite;
            if (m.grad_eta) m.grad_eta[x] = (T)ge;
        }
    }
    if (flag) atomicOr(status, flag);
}

// ---------------------------------------------------------------- Hessian-vector product
//
// Host-facing arrays stay plain; the dual copies live in the workspace.  One
// descriptor per medium.
template <typename S>
struct MediumHvp {
    int32_t nx, nz, n_tx, nt;
    int32_t n_rcv, npml, acc_slots, wavelet_shared;
    double h, dt, dmax, c_max;
    int64_t acc_stride;               // elements between two accumulator slots
    const S* c;
    const S* rho;
    const S* dc;                      // direction (c component)
    const S* drho;                    // direction (rho component), or NULL = 0
    const S* wavelet;
    const S* d_obs;
    S* traces;                        // out: primal traces
    S* dtraces;                       // out: tangent-linear traces, or NULL
    S* grad_c;
    S* grad_rho;
    S* hv_c;
    S* hv_rho;
    Dual<S>* coef;                    // [nz*nx] x (Q, bt) with their derivatives
    Dual<S>* wav;                     // dual wavelet rows
    Dual<S>* obs;                     // dual observed traces (zero derivative)
    Dual<S>* tr;                      // dual traces written by the forward kernels
    const void* acc0;                 // dual accumulators of the medium's first slot
};

// (Q, bt) and their derivatives along (dc, drho), in double and rounded once:
// Q = gamma rho c^2 / (h^2 rho_ref), dQ = gamma (drho c^2 + 2 rho c dc) / (h^2 rho_ref),
// bt = rho_ref / rho, dbt = -rho_ref drho / rho^2.
template <typename S>
__global__ void prep_hvp_kernel(const MediumHvp<S>* __restrict__ media, unsigned* status)
{
    const MediumHvp<S>& m = media[blockIdx.y];
    const int64_t n = (int64_t)m.nx * m.nz;
    const double ih2 = 1.0 / (m.h * m.h);
    unsigned flag = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(x % m.nx), iz = (int)(x / m.nx);
        const double c = (double)m.c[x], rho = (double)m.rho[x];
        const double dc = (double)m.dc[x], drho = m.drho ? (double)m.drho[x] : 0.0;
        if (!(c > 0.0) || !(rho > 0.0) || !isfinite(c) || !isfinite(rho)) flag |= kFlagMedium;
        if (!isfinite(dc) || !isfinite(drho)) flag |= kFlagMedium;
        if (c > m.c_max) flag |= kFlagCfl;
        const double e = (dprof(ix, m.nx, m.npml, m.dmax) + dprof(iz, m.nz, m.npml, m.dmax)) * m.dt;
        const double k = m.dt * m.dt / (1.0 + e) * ih2 / kRhoRef;
        m.coef[2 * x] = Dual<S>((S)(k * rho * c * c), (S)(k * (drho * c * c + 2.0 * rho * c * dc)));
        m.coef[2 * x + 1] = Dual<S>((S)(kRhoRef / rho), (S)(-kRhoRef * drho / (rho * rho)));
    }
    if (flag) atomicOr(status, flag);
}

// Dual copies of the wavelet and the observed traces (both independent of the medium).
template <typename S>
__global__ void pack_hvp_kernel(const MediumHvp<S>* __restrict__ media)
{
    const MediumHvp<S>& m = media[blockIdx.y];
    const int64_t nw = (int64_t)(m.wavelet_shared ? 1 : m.n_tx) * m.nt;
    const int64_t no = (int64_t)m.n_tx * m.nt * m.n_rcv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw + no;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nw) m.wav[i] = Dual<S>(m.wavelet[i], S(0));
        else m.obs[i - nw] = Dual<S>(m.d_obs[i - nw], S(0));
    }
}

// Primal traces and their tangent-linear part out of the dual traces.
template <typename S>
__global__ void unpack_hvp_kernel(const MediumHvp<S>* __restrict__ media)
{
    const MediumHvp<S>& m = media[blockIdx.y];
    const int64_t n = (int64_t)m.n_tx * m.nt * m.n_rcv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Dual<S> d = m.tr[i];
        m.traces[i] = d.v;
        if (m.dtraces) m.dtraces[i] = d.d;
    }
}

// The gradient of finalize_kernel evaluated in dual double arithmetic with
// c and rho carrying the direction: values = g_c, g_rho; derivatives = the
// c and rho components of H v.
template <typename S, typename A>
__global__ void finalize_hvp_kernel(const MediumHvp<S>* __restrict__ media, unsigned* status)
{
    using D = Dual<double>;
    const MediumHvp<S>& m = media[blockIdx.y];
    const int64_t n = (int64_t)m.nx * m.nz;
    const Dual<A>* acc = reinterpret_cast<const Dual<A>*>(m.acc0);
    unsigned flag = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        D sk(0.0), sb(0.0);
        for (int k = 0; k < m.acc_slots; ++k) {
            sk += D(acc[k * m.acc_stride + x]);
            sb += D(acc[k * m.acc_stride + n + x]);
        }
        const int ix = (int)(x % m.nx), iz = (int)(x / m.nx);
        const double e = (dprof(ix, m.nx, m.npml, m.dmax) + dprof(iz, m.nz, m.npml, m.dmax)) * m.dt;
        const double gam = m.dt * m.dt / (1.0 + e);
        // the accumulated kappa sum is q times the lambda one (the kernels carry w = q lam)
        const D s = sk / D(m.coef[2 * x]);
        const D gk = D(gam / (m.h * m.h * kRhoRef)) * s;
        const D gb = D(-kRhoRef) * sb;
        const D c((double)m.c[x], (double)m.dc[x]);
        const D rho((double)m.rho[x], m.drho ? (double)m.drho[x] : 0.0);
        const D gc = D(2.0) * rho * c * gk;
        const D gr = c * c * gk - gb / (rho * rho);
        if (!isfinite(gc.v) || !isfinite(gr.v) || !isfinite(gc.d) || !isfinite(gr.d)) flag |= kFlagNonfinite;
        if (m.grad_c) m.grad_c[x] = (S)gc.v;
        if (m.grad_rho) m.grad_rho[x] = (S)gr.v;
        m.hv_c[x] = (S)gc.d;
        if (m.hv_rho) m.hv_rho[x] = (S)gr.d;
    }
    if (flag) atomicOr(status, flag);
}

}  // namespace fwi
