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
//           traces d[n] = u^{n+1}[rcv]                        (eq. 2-3)
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
enum : unsigned { kFlagCfl = 1u, kFlagMedium = 2u, kFlagNonfinite = 4u };

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

template <typename T, typename Acc>
struct Item {
    int32_t nx, nz, nt, g_used;      // g_used <= G real transmits
    int32_t K, J, tiles_x, n_tiles;
    int32_t n_rcv, tx0, inject_adj, sample;   // inject_adj: 1 if d_adj drives the adjoint
    int64_t plane;                   // elements per field plane = nx*nz*G
    int64_t wavelet_stride;
    const T* coef;                   // [nz*nx] x (Q, bt)
    const T* ex;                     // [nx]  Dx(ix) dt
    const T* ez;                     // [nz]  Dz(iz) dt
    T* seg;                          // K planes
    T* ck;                           // 2 (J-1) planes: pair j >= 1 at 2(j-1): prev, cur
    T* lam;                          // 2 planes
    Acc* acc;                        // [2][nz*nx]: S_kappa, S_b
    const T* zero;                   // zero plane
    const T* wavelet;                // transmit tx row at wavelet + tx * wavelet_stride
    const int32_t* src;              // [G] source cells, -1 for padding slots
    T* traces;                       // medium's [n_tx][nt][n_rcv]
    const T* d_obs;
    const T* d_adj;
    const int32_t* tile_off;         // [n_tiles + 1]
    const Entry* entries;
};

template <typename T, int G>
struct alignas(sizeof(T) * G) Vec {
    T v[G];
};

template <typename T, int G>
__device__ __forceinline__ Vec<T, G> vload(const T* p, int64_t cell)
{
    return *reinterpret_cast<const Vec<T, G>*>(p + cell * G);
}

template <typename T, int G>
__device__ __forceinline__ void vstore(T* p, int64_t cell, const Vec<T, G>& v)
{
    *reinterpret_cast<Vec<T, G>*>(p + cell * G) = v;
}

template <typename T, int G>
__device__ __forceinline__ Vec<T, G> vzero()
{
    Vec<T, G> r;
#pragma unroll
    for (int g = 0; g < G; ++g) r.v[g] = T(0);
    return r;
}

struct Step {
    int phase;
    int n;      // FWD/RECOMP: step index (produces u^{n+1}); ADJ: time t
    int j;      // segment
};

// Position of an item with (T, K, J) at its local step s.
__device__ __forceinline__ Step decode(int T, int K, int J, int s)
{
    Step r{kIdle, 0, 0};
    if (s < 0) return r;
    if (s < T) {
        r.phase = kFwd; r.n = s; r.j = s / K;
        return r;
    }
    s -= T;
    const int last = T - (J - 1) * K;
    if (s < last) {
        r.phase = kAdj; r.n = T + 1 - s; r.j = J - 1;
        return r;
    }
    s -= last;
    if (s < 2 * K * (J - 1)) {
        const int blk = s / (2 * K), rem = s - blk * 2 * K;
        r.j = J - 2 - blk;
        if (rem < K) { r.phase = kRecomp; r.n = r.j * K + rem; }
        else { r.phase = kAdj; r.n = r.j * K + K + 1 - (rem - K); }
    }
    return r;
}

template <typename T>
__device__ __forceinline__ void damp_coeffs(T e, T& a, T& b)
{
    if (e == T(0)) {
        a = T(2);
        b = T(-1);
    } else {
        const T inv = T(1) / (T(1) + e);
        a = (T(2) - e * e) * inv;
        b = (e - T(1)) * inv;
    }
}

// Forward-type step (FWD or RECOMP) on one tile.
template <typename T, int G, typename Acc>
__device__ void tile_forward(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z,
                             int rows, bool sample)
{
    const int nx = it.nx, nz = it.nz, K = it.K, n = st.n, j = st.j;
    const int64_t P = it.plane;
    // u^tau: zero for tau <= 0; on recompute the segment's first two planes come
    // from checkpoint pair j; otherwise the segment buffer slot (tau - 1) mod K.
    auto plane = [&](int tau) -> const T* {
        if (tau <= 0) return it.zero;
        if (st.phase == kRecomp && tau <= j * K)
            return it.ck + (int64_t)(2 * (j - 1) + (tau == j * K ? 1 : 0)) * P;
        return it.seg + (int64_t)((tau - 1) % K) * P;
    };
    const T* cur = plane(n);
    const T* prev = plane(n - 1);
    T* out = it.seg + (int64_t)(n % K) * P;
    T* ck_out = nullptr;
    if (st.phase == kFwd && j + 1 <= it.J - 1) {
        const int t1 = n + 1, jn = j + 1;
        if (t1 == jn * K - 1) ck_out = it.ck + (int64_t)(2 * (jn - 1)) * P;
        else if (t1 == jn * K) ck_out = it.ck + (int64_t)(2 * (jn - 1) + 1) * P;
    }
    // source samples of this step
    T wv[G];
    int sc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        sc[g] = it.src[g];
        wv[g] = sc[g] >= 0 ? it.wavelet[(int64_t)(it.tx0 + g) * it.wavelet_stride + n] : T(0);
    }

    const int ix = tile_x * kTileX + (int)threadIdx.x;
    const int z0 = tile_z * kWavesZ * rows + (int)threadIdx.y * rows;
    const bool colok = ix < nx;
    if (colok && z0 < nz) {
        T ex = it.ex[ix];
        const T* cf = it.coef;
        // rolling values of the row above and the current row
        int iz = z0;
        int64_t x = (int64_t)iz * nx + ix;
        Vec<T, G> un = iz > 0 ? vload<T, G>(cur, x - nx) : vzero<T, G>();
        Vec<T, G> uc = vload<T, G>(cur, x);
        T bn = iz > 0 ? cf[2 * (x - nx) + 1] : T(0);
        T q = cf[2 * x], bc = cf[2 * x + 1];
        const int zend = min(z0 + rows, nz);
        for (; iz < zend; ++iz, x += nx) {
            const bool has_s = iz < nz - 1;
            Vec<T, G> us = has_s ? vload<T, G>(cur, x + nx) : vzero<T, G>();
            T qs = has_s ? cf[2 * (x + nx)] : T(0);
            T bs = has_s ? cf[2 * (x + nx) + 1] : T(0);
            Vec<T, G> uw = ix > 0 ? vload<T, G>(cur, x - 1) : vzero<T, G>();
            Vec<T, G> ue = ix < nx - 1 ? vload<T, G>(cur, x + 1) : vzero<T, G>();
            const T bw = ix > 0 ? cf[2 * (x - 1) + 1] : T(0);
            const T be = ix < nx - 1 ? cf[2 * (x + 1) + 1] : T(0);
            const T hf = T(0.5);
            const T fw = ix > 0 ? hf * (bc + bw) : bc;
            const T fe = ix < nx - 1 ? hf * (bc + be) : bc;
            const T fn = iz > 0 ? hf * (bc + bn) : bc;
            const T fs = has_s ? hf * (bc + bs) : bc;
            T a, b;
            damp_coeffs<T>(ex + it.ez[iz], a, b);
            const Vec<T, G> up = vload<T, G>(prev, x);
            Vec<T, G> r;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const T u0 = uc.v[g];
                T L = fw * (uw.v[g] - u0);
                L += fe * (ue.v[g] - u0);
                L += fn * (un.v[g] - u0);
                L += fs * (us.v[g] - u0);
                T v = a * u0 + b * up.v[g] + q * L;
                if ((int)x == sc[g]) v += wv[g];
                r.v[g] = v;
            }
            vstore<T, G>(out, x, r);
            if (ck_out) vstore<T, G>(ck_out, x, r);
            un = uc; uc = us;
            bn = bc; bc = bs; q = qs;
        }
    }
    if (sample) {
        const int tile = tile_z * it.tiles_x + tile_x;
        const int e0 = it.tile_off[tile], e1 = it.tile_off[tile + 1];
        if (e1 > e0) {
            __syncthreads();
            const int tid = threadIdx.y * kTileX + threadIdx.x;
            for (int e = e0 + tid; e < e1; e += kBlock) {
                const Entry en = it.entries[e];
                it.traces[en.trace_off + (int64_t)n * it.n_rcv] = out[en.slot];
            }
        }
    }
}

// Adjoint step at time t on one tile, with the imaging of lam^t and u^{t-1}.
template <typename T, int G, typename Acc>
__device__ void tile_adjoint(const Item<T, Acc>& it, const Step& st, int tile_x, int tile_z, int rows)
{
    const int nx = it.nx, nz = it.nz, K = it.K, t = st.n;
    const int64_t P = it.plane;
    const int64_t ncell = (int64_t)nx * nz;
    const T* cur = it.lam + (int64_t)(t & 1) * P;          // lam^t
    T* io = it.lam + (int64_t)((t + 1) & 1) * P;           // lam^{t+1} in, lam^{t-1} out
    const T* um = it.seg + (int64_t)((t - 2) % K) * P;     // u^{t-1}
    Acc* accK = it.acc;
    Acc* accB = it.acc + ncell;

    const int ix = tile_x * kTileX + (int)threadIdx.x;
    const int z0 = tile_z * kWavesZ * rows + (int)threadIdx.y * rows;
    if (ix < nx && z0 < nz) {
        const T ex = it.ex[ix];
        const T* cf = it.coef;
        const T hf = T(0.5);
        const T cw = ix > 0 ? hf : T(1), ce = ix < nx - 1 ? hf : T(1);
        int iz = z0;
        int64_t x = (int64_t)iz * nx + ix;
        // rolling (above, centre): lam, Q*lam, u, bt
        Vec<T, G> ln = iz > 0 ? vload<T, G>(cur, x - nx) : vzero<T, G>();
        Vec<T, G> lc = vload<T, G>(cur, x);
        Vec<T, G> uN = iz > 0 ? vload<T, G>(um, x - nx) : vzero<T, G>();
        Vec<T, G> uC = vload<T, G>(um, x);
        T qn = iz > 0 ? cf[2 * (x - nx)] : T(0);
        T bn = iz > 0 ? cf[2 * (x - nx) + 1] : T(0);
        T qc = cf[2 * x], bc = cf[2 * x + 1];
        const int zend = min(z0 + rows, nz);
        for (; iz < zend; ++iz, x += nx) {
            const bool has_s = iz < nz - 1;
            const Vec<T, G> ls = has_s ? vload<T, G>(cur, x + nx) : vzero<T, G>();
            const Vec<T, G> uS = has_s ? vload<T, G>(um, x + nx) : vzero<T, G>();
            const T qs = has_s ? cf[2 * (x + nx)] : T(0);
            const T bs = has_s ? cf[2 * (x + nx) + 1] : T(0);
            const Vec<T, G> lw = ix > 0 ? vload<T, G>(cur, x - 1) : vzero<T, G>();
            const Vec<T, G> le = ix < nx - 1 ? vload<T, G>(cur, x + 1) : vzero<T, G>();
            const Vec<T, G> uW = ix > 0 ? vload<T, G>(um, x - 1) : vzero<T, G>();
            const Vec<T, G> uE = ix < nx - 1 ? vload<T, G>(um, x + 1) : vzero<T, G>();
            const T qw = ix > 0 ? cf[2 * (x - 1)] : T(0);
            const T bw = ix > 0 ? cf[2 * (x - 1) + 1] : T(0);
            const T qe = ix < nx - 1 ? cf[2 * (x + 1)] : T(0);
            const T be = ix < nx - 1 ? cf[2 * (x + 1) + 1] : T(0);
            const T fw = ix > 0 ? hf * (bc + bw) : bc;
            const T fe = ix < nx - 1 ? hf * (bc + be) : bc;
            const T fn = iz > 0 ? hf * (bc + bn) : bc;
            const T fs = has_s ? hf * (bc + bs) : bc;
            const T cn = iz > 0 ? hf : T(1), cs = has_s ? hf : T(1);
            T a, b;
            damp_coeffs<T>(ex + it.ez[iz], a, b);
            const Vec<T, G> lp = vload<T, G>(io, x);
            Vec<T, G> r;
            Acc sk = Acc(0), sb = Acc(0);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const T l0 = lc.v[g];
                const T w0 = qc * l0;
                const T dww = qw * lw.v[g] - w0, dwe = qe * le.v[g] - w0;
                const T dwn = qn * ln.v[g] - w0, dws = qs * ls.v[g] - w0;
                T L = fw * dww;
                L += fe * dwe;
                L += fn * dwn;
                L += fs * dws;
                r.v[g] = a * l0 + b * lp.v[g] + L;
                const T u0 = uC.v[g];
                const T duw = uW.v[g] - u0, due = uE.v[g] - u0;
                const T dun = uN.v[g] - u0, dus = uS.v[g] - u0;
                T Lu = fw * duw;
                Lu += fe * due;
                Lu += fn * dun;
                Lu += fs * dus;
                T gb = cw * duw * dww;
                gb += ce * due * dwe;
                gb += cn * dun * dwn;
                gb += cs * dus * dws;
                sk += Acc(l0 * Lu);
                sb += Acc(gb);
            }
            vstore<T, G>(io, x, r);
            accK[x] += sk;
            accB[x] += sb;
            ln = lc; lc = ls; uN = uC; uC = uS;
            qn = qc; qc = qs; bn = bc; bc = bs;
        }
    }
    // adjoint source of lam^{t-1}: sample t-2 at the receivers of this tile
    const int tile = tile_z * it.tiles_x + tile_x;
    const int e0 = it.tile_off[tile], e1 = it.tile_off[tile + 1];
    const bool has_src = it.inject_adj ? it.d_adj != nullptr : it.d_obs != nullptr;
    if (e1 > e0 && t >= 2 && has_src) {
        __syncthreads();
        const int tid = threadIdx.y * kTileX + threadIdx.x;
        const int64_t so = (int64_t)(t - 2) * it.n_rcv;
        for (int e = e0 + tid; e < e1; e += kBlock) {
            const Entry en = it.entries[e];
            if (en.run == 0) continue;
            T s = T(0);
            for (int k = 0; k < en.run; ++k) {
                const Entry ek = it.entries[e + k];
                const int64_t o = ek.trace_off + so;
                s += it.inject_adj ? it.d_adj[o] : T(2) * (it.traces[o] - it.d_obs[o]);
            }
            io[en.slot] += s;
        }
    }
}

// One step of every item whose schedule has work at this step.
// blocks[b] = (item, tile); mode shifts/limits each item's local step.
template <typename T, int G, typename Acc>
__global__ __launch_bounds__(kBlock) void step_kernel(const Item<T, Acc>* __restrict__ items,
                                                       const int2* __restrict__ blocks, int s,
                                                       int mode, int rows)
{
    const int2 bt = blocks[blockIdx.x];
    const Item<T, Acc>& it = items[bt.x];
    int sl = s;
    if (mode == kRunAdjOnly) sl = s + it.nt;
    Step st = decode(it.nt, it.K, it.J, sl);
    if (mode == kRunFwdOnly && st.phase != kFwd) st.phase = kIdle;
    if (st.phase == kIdle) return;
    const int tile_x = bt.y % it.tiles_x, tile_z = bt.y / it.tiles_x;
    if (st.phase == kAdj)
        tile_adjoint<T, G, Acc>(it, st, tile_x, tile_z, rows);
    else
        tile_forward<T, G, Acc>(it, st, tile_x, tile_z, rows, st.phase == kFwd && it.sample);
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
        const double e = (dprof(ix, m.nx, m.npml, m.dmax) + dprof(iz, m.nz, m.npml, m.dmax)) * m.dt;
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

// Misfit partial sums: block b of medium m sums (d - d_obs)^2 over a strided share.
constexpr int kMisfitBlocks = 64;

template <typename T>
__global__ __launch_bounds__(256) void misfit_partial_kernel(const MediumDev<T>* __restrict__ media,
                                                              double* __restrict__ partial)
{
    const MediumDev<T>& m = media[blockIdx.y];
    __shared__ double red[256];
    double s = 0.0;
    if (m.d_obs) {
        const int64_t n = (int64_t)m.n_tx * m.nt * m.n_rcv;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x) {
            const double r = (double)m.traces[i] - (double)m.d_obs[i];
            s += r * r;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.y * kMisfitBlocks + blockIdx.x] = red[0];
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
        const double e = (dprof(ix, m.nx, m.npml, m.dmax) + dprof(iz, m.nz, m.npml, m.dmax)) * m.dt;
        const double gam = m.dt * m.dt / (1.0 + e);
        const double gk = gam / (m.h * m.h * kRhoRef) * sk;
        const double gb = -kRhoRef * sb;
        const double c = (double)m.c[x], rho = (double)m.rho[x];
        const double gc = 2.0 * rho * c * gk;
        const double gr = c * c * gk - gb / (rho * rho);
        if (!isfinite(gc) || !isfinite(gr)) flag |= kFlagNonfinite;
        if (m.grad_c) m.grad_c[x] = (T)gc;
        if (m.grad_rho) m.grad_rho[x] = (T)gr;
    }
    if (flag) atomicOr(status, flag);
}

}  // namespace fwi
