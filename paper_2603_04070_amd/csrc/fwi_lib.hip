// Host side of the FWI-gradient library: C ABI declared in include/fwi.h.
//
// A plan turns media + geometry into work items (medium, group of G
// transmits), lays out one caller-provided workspace, builds the per-tile
// receiver tables, and enqueues the step kernels of fwi_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fwi.h"
#include "fwi_kernels.hpp"

using namespace fwi;

namespace {

thread_local std::string g_create_error;

constexpr size_t kAlign = 256;
constexpr int kXcd = 8;        // MI355X: 8 accelerator complex dies, each with its own L2
constexpr size_t kLdsBytes = 160 * 1024;   // LDS per compute unit on gfx950
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct ItemPlan {
    int medium;
    int tx0, g_used;
    int K, J;
    int tiles_x, tiles_z, n_tiles;
    int blk0;                  // first block of this item in the block table
    int steps;                 // schedule length 2T + K(J-1)
    size_t seg_off, ck_off, lam_off, vel_off, acc_off;   // workspace byte offsets
    size_t src_off, tile_off_off, entry_off;    // plan-table byte offsets
    size_t tile_off_x_off, entry_x_off;         // receivers of each tile grown by one cell
};

struct Wave {
    std::vector<int> items;    // items resident together, longest schedule first
    int blk0 = 0, nblk = 0;    // their blocks, contiguous in the block table
    std::vector<int> prefix;   // prefix[m]: blocks covering the first m items
    size_t nblk_off[3] = {0, 0, 0};   // per call mode: active blocks of each launch (persistent form)
    int n_launch[3] = {0, 0, 0};
    int steps = 0, fwd = 0, adj = 0;
    size_t lam_off = 0, lam_bytes = 0;
};

struct MediumPlan {
    fwi_grid g;
    std::vector<int32_t> src, rcv;
    double dmax;
    int item0, item1;
    int acc_slots;
    size_t coef_off, acc_off;  // workspace
    size_t wav_off, obs_off, trd_off;   // workspace, hvp plans: dual wavelet, observed and traces
    size_t eatt_off;           // workspace, attenuation plans: eta dt per cell
    size_t ex_off, ez_off;     // plan tables
};

}  // namespace

struct fwi_plan {
    fwi_dtype dtype = FWI_F32;
    fwi_options opt{};
    int G = 1, rows = 4, S = 1, nlam = 2, order = 2;
    int Sa = 1;                     // adjoint steps per launch (S: forward-type steps)
    bool acc_double = false;
    bool hvp = false;               // dual-number plan of fwi_plan_hvp
    bool att = false;               // attenuation rate in the damping (one-step kernels)
    int nacc = 2;                   // imaging accumulators per cell and slot (S_kappa, S_b[, S_e])
    size_t tsize = 4, asize = 4;
    std::vector<MediumPlan> media;
    std::vector<ItemPlan> items;
    std::vector<int2> blocks;
    std::vector<Wave> waves;
    int64_t cell_updates = 0, recompute_updates = 0;
    int64_t kernel_launches = 0;    // step-kernel launches of one gradient

    // workspace layout
    size_t ws_bytes = 0;
    size_t zero_off = 0, zero_bytes = 0;
    size_t clear_off = 0, clear_bytes = 0;       // zero plane + accumulators
    size_t acc_region_off = 0, acc_region_bytes = 0;
    size_t partial_off = 0;

    // plan-owned device tables
    void* d_tables = nullptr;
    size_t tables_bytes = 0;
    int2* d_blocks = nullptr;
    void* d_items = nullptr;        // Item<T, Acc>[n_items]
    void* d_media = nullptr;        // MediumDev<T>[n_media]
    void* d_hvp = nullptr;          // MediumHvp<T>[n_media] (hvp plans)
    size_t hvp_bytes = 0;
    unsigned* d_status = nullptr;
    unsigned* d_bar = nullptr;      // grid barrier words of the persistent form
    int pgrid = 0;                  // co-resident workgroups of the persistent kernel
    unsigned spin_limit = 0;
    void* h_stage = nullptr;        // pinned staging for items + media descriptors
    size_t item_bytes = 0, media_bytes = 0;
    hipEvent_t stage_ev = nullptr;
    bool stage_pending = false;
    hipStream_t last_stream = nullptr;
    bool have_call = false;

    // workspaces holding a forward's replay state for a later adjoint
    std::vector<const void*> fwd_ws;

    // hipGraph replay of the batched gradient
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void* graph_ws = nullptr;
    unsigned graph_flags = 0;

    std::string last_error;
};

namespace {

fwi_status fail(fwi_plan* p, fwi_status st, const std::string& msg)
{
    if (p) p->last_error = msg;
    return st;
}

#define HIPCHK(plan, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(plan, FWI_ERR_HIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

double dmax_of(const fwi_grid& g)
{
    if (g.npml <= 0) return 0.0;
    return 3.0 * g.pml_cref * std::log(1.0 / g.pml_r) / (2.0 * g.npml * g.h);
}

double prof(int i, int n, int N, double dmax)
{
    if (i < N) { double r = (double)(N - i) / N; return dmax * r * r; }
    if (i > n - 1 - N) { double r = (double)(i - (n - 1 - N)) / N; return dmax * r * r; }
    return 0.0;
}

// Launch recorder of fwi_plan_launches: while ``out`` is set, the enqueue
// functions append what they would launch instead of launching it.
struct LaunchRec {
    std::vector<fwi_launch>* out = nullptr;
    int wave = -1, step = -1;
};
thread_local LaunchRec g_rec;

bool recording() { return g_rec.out != nullptr; }

void record(int kernel, dim3 grid, dim3 block, size_t lds)
{
    g_rec.out->push_back(fwi_launch{kernel, g_rec.wave, g_rec.step, (int32_t)grid.x, (int32_t)grid.y,
                                    (int32_t)(block.x * block.y * block.z), (int32_t)lds, 0});
}

// Host-side validation of one grid (no HIP call).
fwi_status validate_grid(const fwi_grid& g, int idx, std::string& msg, int order)
{
    char buf[256];
    auto bad = [&](fwi_status st, const char* what) {
        std::snprintf(buf, sizeof buf, "medium %d: %s", idx, what);
        msg = buf;
        return st;
    };
    if (g.npml < 0) return bad(FWI_ERR_INVALID, "npml < 0");
    if (g.nx < 2 * g.npml + 3 || g.nz < 2 * g.npml + 3) return bad(FWI_ERR_INVALID, "nx, nz must be >= 2*npml+3");
    if (g.nt < 1) return bad(FWI_ERR_INVALID, "nt < 1");
    if (!(g.h > 0) || !(g.dt > 0) || !std::isfinite(g.h) || !std::isfinite(g.dt))
        return bad(FWI_ERR_INVALID, "h and dt must be positive");
    if (g.npml > 0 && (!(g.pml_r > 0) || !(g.pml_r < 1) || !(g.pml_cref > 0)))
        return bad(FWI_ERR_INVALID, "pml_r must be in (0,1) and pml_cref > 0");
    if (!(g.c_max > 0) || !std::isfinite(g.c_max)) return bad(FWI_ERR_INVALID, "c_max must be positive");
    if (g.n_tx < 1 || g.n_rcv < 1) return bad(FWI_ERR_INVALID, "n_tx and n_rcv must be >= 1");
    if (!g.src || !g.rcv) return bad(FWI_ERR_INVALID, "src and rcv must be host arrays");
    const int64_t ncell = (int64_t)g.nx * g.nz;
    if (ncell * 4 > INT32_MAX) return bad(FWI_ERR_INVALID, "grid too large (nx*nz*4 must fit int32)");
    if ((int64_t)g.n_tx * g.nt * g.n_rcv > INT32_MAX) return bad(FWI_ERR_INVALID, "n_tx*nt*n_rcv too large");
    for (int p = 0; p < g.n_tx; ++p) {
        if (g.src[p] < 0 || g.src[p] >= ncell) return bad(FWI_ERR_GEOMETRY, "source cell outside the grid");
        for (int r = 0; r < g.n_rcv; ++r) {
            const int32_t c = g.rcv[(int64_t)p * g.n_rcv + r];
            if (c < 0 || c >= ncell) return bad(FWI_ERR_GEOMETRY, "receiver cell outside the grid");
        }
    }
    // frozen-coefficient stability of the damped leapfrog update:
    // (D dt)^2 + c^2 dt^2 k/h^2 < 4 with D = 2 D_max in the corners and k the
    // operator's largest eigenvalue times h^2/b: 2 x 4 for the 5-point form,
    // 2 x (9/8 * 2 + 1/24 * 2)^2 = 98/9 for the fourth-order form
    const double e = 2.0 * dmax_of(g) * g.dt, cr = g.c_max * g.dt / g.h;
    const double k = order == 4 ? 98.0 / 9.0 : 8.0;
    if (e * e + k * cr * cr >= 4.0)
        return bad(FWI_ERR_CFL, order == 4 ? "unstable: 4 (Dmax dt)^2 + 98/9 (c_max dt/h)^2 >= 4"
                                           : "unstable: 4 (Dmax dt)^2 + 8 (c_max dt/h)^2 >= 4");
    return FWI_OK;
}

// Step launches per (dtype, accumulator, G).  kind: 0 forward one step,
// 1 forward two steps, 2 adjoint one step, 3 adjoint two steps, 4 forward
// three steps.  Multi-step kernels exist for tile heights of 4, 8 and 16 rows
// (R = 1, 2, 4).
template <typename T, typename Acc, int G, int R>
void launch2(int kind, dim3 grid, hipStream_t st, const Item<T, Acc>* it, const int2* blocks, int s, int mode)
{
    const dim3 blk(kTileX, kWavesZ);
    constexpr size_t lds_f = Lds2<T, G, R, false>::bytes;
    constexpr size_t lds_a = Lds2<T, G, R, true>::bytes;
    constexpr size_t lds_3 = Lds3<T, G, R>::bytes;
    if (kind == 1)
        hipLaunchKernelGGL((fwd2_kernel<T, G, Acc, R>), grid, blk, lds_f, st, it, blocks, s, mode);
    else if (kind == 4)
        hipLaunchKernelGGL((fwd3_kernel<T, G, Acc, R>), grid, blk, lds_3, st, it, blocks, s, mode);
    else
        hipLaunchKernelGGL((adj2_kernel<T, G, Acc, R>), grid, blk, lds_a, st, it, blocks, s, mode);
}

// Fourth-order launches (kind 0 one forward step, 1 two forward steps, 2
// one adjoint step), R = 1, 2, 4.
template <typename T, typename Acc, int G, int R>
void launch4(int kind, dim3 grid, hipStream_t st, const Item<T, Acc>* it, const int2* blocks, int s, int mode)
{
    const dim3 blk(kTileX, kWavesZ);
    constexpr size_t lds_f = Lds4<T, G, R, false>::bytes;
    constexpr size_t lds_2 = Lds4x2<T, G, R>::bytes;
    constexpr size_t lds_a = Lds4<T, G, R, true>::bytes;
    if (kind == 0)
        hipLaunchKernelGGL((fwd4_kernel<T, G, Acc, R>), grid, blk, lds_f, st, it, blocks, s, mode);
    else if (kind == 1)
        hipLaunchKernelGGL((fwd4x2_kernel<T, G, Acc, R>), grid, blk, lds_2, st, it, blocks, s, mode);
    else if constexpr (lds_a <= kLdsBytes)     // plans whose adjoint tile exceeds the LDS are refused
        hipLaunchKernelGGL((adj4_kernel<T, G, Acc, R>), grid, blk, lds_a, st, it, blocks, s, mode);
}

template <typename T, typename Acc, int G>
void launch_step(int kind, dim3 grid, hipStream_t st, const void* items, const int2* blocks, int s, int mode,
                 int rows, int order)
{
    const auto* it = reinterpret_cast<const Item<T, Acc>*>(items);
    const dim3 blk(kTileX, kWavesZ);
    if (order == 4) {
        if (rows == 1) launch4<T, Acc, G, 1>(kind, grid, st, it, blocks, s, mode);
        else if (rows == 2) launch4<T, Acc, G, 2>(kind, grid, st, it, blocks, s, mode);
        else launch4<T, Acc, G, 4>(kind, grid, st, it, blocks, s, mode);
        return;
    }
    if (kind == 0) {
        hipLaunchKernelGGL((fwd1_kernel<T, G, Acc>), grid, blk, 0, st, it, blocks, s, mode, rows);
    } else if (kind == 2) {
        hipLaunchKernelGGL((adj1_kernel<T, G, Acc>), grid, blk, 0, st, it, blocks, s, mode, rows);
    } else if (rows == 1) {
        launch2<T, Acc, G, 1>(kind, grid, st, it, blocks, s, mode);
    } else if (rows == 2) {
        launch2<T, Acc, G, 2>(kind, grid, st, it, blocks, s, mode);
    } else {
        launch2<T, Acc, G, 4>(kind, grid, st, it, blocks, s, mode);
    }
}

// Allow the two-step kernels more than the default 64 KiB of dynamic LDS.
template <typename T, typename Acc, int G, int R>
hipError_t allow_lds()
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fwd2_kernel<T, G, Acc, R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds2<T, G, R, false>::bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fwd3_kernel<T, G, Acc, R>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds3<T, G, R>::bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&adj2_kernel<T, G, Acc, R>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds2<T, G, R, true>::bytes);
}

template <typename T, typename Acc, int G, int R>
hipError_t allow_lds4()
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fwd4_kernel<T, G, Acc, R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds4<T, G, R, false>::bytes);
    if (e != hipSuccess) return e;
    if (Lds4x2<T, G, R>::bytes <= kLdsBytes) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fwd4x2_kernel<T, G, Acc, R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds4x2<T, G, R>::bytes);
        if (e != hipSuccess) return e;
    }
    if constexpr (Lds4<T, G, R, true>::bytes <= kLdsBytes)
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&adj4_kernel<T, G, Acc, R>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds4<T, G, R, true>::bytes);
    return hipSuccess;
}

template <typename T, typename Acc, int G>
hipError_t allow_lds_r(int rows, int order)
{
    if (order == 4) {
        if (rows == 1) return allow_lds4<T, Acc, G, 1>();
        if (rows == 2) return allow_lds4<T, Acc, G, 2>();
        return allow_lds4<T, Acc, G, 4>();
    }
    if (rows == 1) return allow_lds<T, Acc, G, 1>();
    if (rows == 2) return allow_lds<T, Acc, G, 2>();
    return allow_lds<T, Acc, G, 4>();
}

template <typename T, typename Acc>
void launch_step_g(int G, int kind, dim3 grid, hipStream_t st, const void* items, const int2* blocks, int s,
                   int mode, int rows, int order)
{
    if (G == 1) launch_step<T, Acc, 1>(kind, grid, st, items, blocks, s, mode, rows, order);
    else if (G == 2) launch_step<T, Acc, 2>(kind, grid, st, items, blocks, s, mode, rows, order);
    else launch_step<T, Acc, 4>(kind, grid, st, items, blocks, s, mode, rows, order);
}

// Dynamic LDS of a step launch of this plan (compile-time tile layouts).
template <typename T, int G>
size_t lds_of(int kind, int rows, int order)
{
    auto byR = [&](auto r) -> size_t {
        constexpr int R = decltype(r)::value;
        if (order == 4)
            return kind == 0 ? Lds4<T, G, R, false>::bytes : kind == 1 ? Lds4x2<T, G, R>::bytes : Lds4<T, G, R, true>::bytes;
        if (kind == 1) return Lds2<T, G, R, false>::bytes;
        if (kind == 3) return Lds2<T, G, R, true>::bytes;
        return Lds3<T, G, R>::bytes;
    };
    if (order != 4 && (kind == 0 || kind == 2)) return 0;
    if (rows == 1) return byR(std::integral_constant<int, 1>());
    if (rows == 2) return byR(std::integral_constant<int, 2>());
    return byR(std::integral_constant<int, 4>());
}

// LDS of the fourth-order launches of a plan with this dtype, G, rows and
// forward steps per launch (the largest layout the plan launches).
size_t lds4_need(fwi_dtype dtype, int G, int rows, int S)
{
    auto byR = [&](auto t, auto g) -> size_t {
        using T = decltype(t);
        constexpr int GG = decltype(g)::value;
        auto one = [&](auto r) -> size_t {
            constexpr int R = decltype(r)::value;
            const size_t one = std::max(Lds4<T, GG, R, false>::bytes, Lds4<T, GG, R, true>::bytes);
            return S >= 2 ? std::max(one, Lds4x2<T, GG, R>::bytes) : one;
        };
        if (rows == 1) return one(std::integral_constant<int, 1>());
        if (rows == 2) return one(std::integral_constant<int, 2>());
        return one(std::integral_constant<int, 4>());
    };
    auto byG = [&](auto t) -> size_t {
        if (G == 1) return byR(t, std::integral_constant<int, 1>());
        if (G == 2) return byR(t, std::integral_constant<int, 2>());
        return byR(t, std::integral_constant<int, 4>());
    };
    return dtype == FWI_F64 ? byG(double()) : byG(float());
}

// Adjoint steps fused per launch: up to two for the second-order operator,
// one for the fourth-order operator.
int adjoint_steps(int order, int S) { return order == 4 ? 1 : std::min(S, 2); }

size_t step_lds(const fwi_plan* p, int kind)
{
    auto byG = [&](auto t) -> size_t {
        using T = decltype(t);
        if (p->G == 1) return lds_of<T, 1>(kind, p->rows, p->order);
        if (p->G == 2) return lds_of<T, 2>(kind, p->rows, p->order);
        return lds_of<T, 4>(kind, p->rows, p->order);
    };
    if (p->hvp) return p->dtype == FWI_F64 ? byG(Dual<double>()) : byG(Dual<float>());
    return p->dtype == FWI_F64 ? byG(double()) : byG(float());
}

void step(fwi_plan* p, int kind, dim3 grid, hipStream_t st, const int2* blocks, int s, int mode)
{
    if (recording()) {
        const int id = p->order == 4 ? (kind == 0 ? FWI_K_FWD4 : kind == 1 ? FWI_K_FWD4X2 : FWI_K_ADJ4) : kind;
        record(id, grid, dim3(kTileX, kWavesZ), step_lds(p, kind));
        return;
    }
    if (p->dtype == FWI_F64)
        launch_step_g<double, double>(p->G, kind, grid, st, p->d_items, blocks, s, mode, p->rows, p->order);
    else if (p->acc_double)
        launch_step_g<float, double>(p->G, kind, grid, st, p->d_items, blocks, s, mode, p->rows, p->order);
    else
        launch_step_g<float, float>(p->G, kind, grid, st, p->d_items, blocks, s, mode, p->rows, p->order);
}

hipError_t allow_lds_plan(const fwi_plan* p)
{
    if (p->S < 2 && p->order != 4) return hipSuccess;
    auto pick = [&](auto t, auto a) -> hipError_t {
        using T = decltype(t);
        using A = decltype(a);
        if (p->G == 1) return allow_lds_r<T, A, 1>(p->rows, p->order);
        if (p->G == 2) return allow_lds_r<T, A, 2>(p->rows, p->order);
        return allow_lds_r<T, A, 4>(p->rows, p->order);
    };
    if (p->hvp) {
        // dual instantiations run multi-step launches with groups of 1 or 2 only
        auto pick_h = [&](auto t, auto a) -> hipError_t {
            using T = decltype(t);
            using A = decltype(a);
            auto byR = [&](auto g) -> hipError_t {
                constexpr int GG = decltype(g)::value;
                if (p->rows == 1) return allow_lds<T, A, GG, 1>();
                if (p->rows == 2) return allow_lds<T, A, GG, 2>();
                return allow_lds<T, A, GG, 4>();
            };
            if (p->G == 1) return byR(std::integral_constant<int, 1>());
            if (p->G == 2) return byR(std::integral_constant<int, 2>());
            return hipSuccess;
        };
        if (p->dtype == FWI_F64) return pick_h(Dual<double>(), Dual<double>());
        if (p->acc_double) return pick_h(Dual<float>(), Dual<double>());
        return pick_h(Dual<float>(), Dual<float>());
    }
    if (p->dtype == FWI_F64) return pick(double(), double());
    if (p->acc_double) return pick(float(), double());
    return pick(float(), float());
}

// ---------------------------------------------------------------- persistent form

template <typename T, typename Acc, int G, int R>
void* persistent_fn()
{
    return reinterpret_cast<void*>(&persistent_kernel<T, G, Acc, R>);
}

// The persistent kernel of a plan, and its dynamic LDS (none without two-step tiles).
void* persistent_kernel_of(const fwi_plan* p, size_t* lds)
{
    auto pick = [&](auto t, auto a) -> void* {
        using T = decltype(t);
        using A = decltype(a);
        const int R = p->S == 2 ? p->rows : 1;
        *lds = 0;
        auto byG = [&](auto g) -> void* {
            constexpr int G = decltype(g)::value;
            if (R == 2) { if (p->S == 2) *lds = Lds2<T, G, 2, true>::bytes; return persistent_fn<T, A, G, 2>(); }
            if (R == 4) { if (p->S == 2) *lds = Lds2<T, G, 4, true>::bytes; return persistent_fn<T, A, G, 4>(); }
            if (p->S == 2) *lds = Lds2<T, G, 1, true>::bytes;
            return persistent_fn<T, A, G, 1>();
        };
        if (p->G == 1) return byG(std::integral_constant<int, 1>());
        if (p->G == 2) return byG(std::integral_constant<int, 2>());
        return byG(std::integral_constant<int, 4>());
    };
    if (p->dtype == FWI_F64) return pick(double(), double());
    if (p->acc_double) return pick(float(), double());
    return pick(float(), float());
}

// Workgroups of the persistent kernel that are co-resident, a multiple of the XCD count.
hipError_t persistent_grid(fwi_plan* p, int* grid)
{
    size_t lds = 0;
    const void* fn = persistent_kernel_of(p, &lds);
    if (lds > 0) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int cap = per_cu * cus / kXcd * kXcd;
    *grid = std::max(kXcd, cap);
    return hipSuccess;
}

void launch_persistent(fwi_plan* p, hipStream_t st, const Wave& w, int mode_idx, int mode)
{
    size_t lds = 0;
    void* fn = persistent_kernel_of(p, &lds);
    int max_nb = 0;
    for (int nb : w.prefix) max_nb = std::max(max_nb, nb);
    const int grid = std::max(kXcd, std::min(p->pgrid, (max_nb + kXcd - 1) / kXcd * kXcd));
    auto* tabs = reinterpret_cast<unsigned char*>(p->d_tables);
    const void* items = p->d_items;
    const int2* blocks = p->d_blocks + w.blk0;
    const int* nblk = reinterpret_cast<const int*>(tabs + w.nblk_off[mode_idx]);
    int n_launch = w.n_launch[mode_idx];
    int rows = p->rows;
    unsigned* bar = p->d_bar;
    unsigned spin = p->spin_limit;
    unsigned* status = p->d_status;
    if (recording()) { record(FWI_K_PERSISTENT, dim3(p->pgrid > 0 ? grid : 0), dim3(kTileX, kWavesZ), lds); return; }
    void* args[] = {&items, &blocks, &nblk, &n_launch, &mode, &rows, &bar, &spin, &status};
    (void)hipLaunchKernel(fn, dim3(grid), dim3(kTileX, kWavesZ), args, lds, st);
}

// Launch kinds present in a wave at launch s of a call: bit k set when some
// item needs kind k (the schedule the kernels decode, evaluated on the host).
unsigned wave_kinds(const fwi_plan* p, const Wave& w, int s, int mode, int* n_active)
{
    unsigned bits = 0;
    *n_active = 0;
    for (int pos = 0; pos < (int)w.items.size(); ++pos) {
        const ItemPlan& it = p->items[w.items[pos]];
        const int T = p->media[it.medium].g.nt;
        const int nf = (T + p->S - 1) / p->S;
        const Step st = decode(T, it.K, it.J, mode == kRunAdjOnly ? s + nf : s, p->S, p->Sa);
        if (st.phase == kIdle || (mode == kRunFwdOnly && st.phase != kFwd)) continue;
        if (st.phase == kAdj) bits |= st.count == 2 ? 8u : 4u;
        else bits |= st.count == 3 ? 16u : st.count == 2 ? 2u : 1u;
        *n_active = pos + 1;
    }
    return bits;
}

int grid_for(int64_t n, int per_block, int cap)
{
    int64_t b = (n + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// Zero a byte range of the workspace (multiple of 4 bytes, 4-byte aligned).
void zero_bytes(hipStream_t st, void* base, size_t bytes)
{
    if (!bytes) return;
    const int64_t n = (int64_t)(bytes / 4);
    if (recording()) { record(FWI_K_FILL, dim3(grid_for(n, 256, 8192)), dim3(256), 0); return; }
    hipLaunchKernelGGL(zero_kernel<uint32_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st,
                       reinterpret_cast<uint32_t*>(base), n);
}

// Clear n status or barrier words.
void zero_words(hipStream_t st, unsigned* w, int64_t n)
{
    if (recording()) { record(FWI_K_FILL, dim3(1), dim3(64), 0); return; }
    hipLaunchKernelGGL(zero_kernel<unsigned>, dim3(1), dim3(64), 0, st, w, n);
}

}  // namespace

// ----------------------------------------------------------------------------- plan creation

extern "C" const char* fwi_last_create_error(void) { return g_create_error.c_str(); }

extern "C" const char* fwi_status_string(fwi_status s)
{
    switch (s) {
    case FWI_OK: return "ok";
    case FWI_ERR_INVALID: return "invalid argument";
    case FWI_ERR_CFL: return "time step violates the stability bound";
    case FWI_ERR_GEOMETRY: return "source or receiver outside the grid";
    case FWI_ERR_NOMEM: return "out of device memory";
    case FWI_ERR_WORKSPACE: return "workspace missing or too small";
    case FWI_ERR_HIP: return "HIP runtime error";
    case FWI_ERR_NONFINITE: return "non-finite result";
    case FWI_ERR_MEDIUM: return "invalid medium values (c or rho not positive and finite)";
    case FWI_ERR_STATE: return "adjoint called without a preceding forward";
    }
    return "unknown status";
}

extern "C" const char* fwi_plan_last_error(const fwi_plan* p) { return p ? p->last_error.c_str() : ""; }

static fwi_status create_impl(fwi_plan* p, fwi_dtype dtype, const fwi_grid* grids, int32_t n_media,
                              const fwi_options* opt)
{
    // ---------------- host validation (no HIP calls before this passes)
    if (!grids || n_media < 1) return fail(p, FWI_ERR_INVALID, "grids must be non-NULL and n_media >= 1");
    if (dtype != FWI_F32 && dtype != FWI_F64) return fail(p, FWI_ERR_INVALID, "unknown dtype");
    fwi_options o{};
    o.mode = FWI_BATCHED;
    if (opt) o = *opt;
    if (o.mode != FWI_PLAIN && o.mode != FWI_BATCHED) return fail(p, FWI_ERR_INVALID, "unknown mode");
    if (o.group != 0 && o.group != 1 && o.group != 2 && o.group != 4)
        return fail(p, FWI_ERR_INVALID, "group must be 0, 1, 2 or 4");
    if (o.mode == FWI_PLAIN && o.group > 1) return fail(p, FWI_ERR_INVALID, "plain mode runs one transmit per item");
    if (o.rows < 0 || o.rows > 64) return fail(p, FWI_ERR_INVALID, "rows must be in [0, 64]");
    if (o.steps_per_launch < 0 || o.steps_per_launch > 3)
        return fail(p, FWI_ERR_INVALID, "steps_per_launch must be 0, 1, 2 or 3");
    if (o.persistent && o.steps_per_launch == 3)
        return fail(p, FWI_ERR_INVALID, "the persistent form fuses at most two steps per launch");
    if (o.ckpt_interval < 0) return fail(p, FWI_ERR_INVALID, "ckpt_interval must be >= 0");
    if (o.mem_budget < 0) return fail(p, FWI_ERR_INVALID, "mem_budget must be >= 0");
    if (o.use_graph && o.mode != FWI_BATCHED) return fail(p, FWI_ERR_INVALID, "use_graph requires FWI_BATCHED");
    if (o.forward_only != 0 && o.forward_only != 1) return fail(p, FWI_ERR_INVALID, "forward_only must be 0 or 1");
    if (o.persistent != 0 && o.persistent != 1) return fail(p, FWI_ERR_INVALID, "persistent must be 0 or 1");
    if (o.persistent && o.mode != FWI_BATCHED) return fail(p, FWI_ERR_INVALID, "persistent requires FWI_BATCHED");
    if (o.barrier_spin < 0) return fail(p, FWI_ERR_INVALID, "barrier_spin must be >= 0");
    if (o.order != 0 && o.order != 2 && o.order != 4) return fail(p, FWI_ERR_INVALID, "order must be 0, 2 or 4");
    if (o.hvp != 0 && o.hvp != 1) return fail(p, FWI_ERR_INVALID, "hvp must be 0 or 1");
    if (o.host_only != 0 && o.host_only != 1) return fail(p, FWI_ERR_INVALID, "host_only must be 0 or 1");
    if (o.single_wave != 0 && o.single_wave != 1) return fail(p, FWI_ERR_INVALID, "single_wave must be 0 or 1");
    if (o.attenuation != 0 && o.attenuation != 1) return fail(p, FWI_ERR_INVALID, "attenuation must be 0 or 1");
    if (o.attenuation && (o.order == 4 || o.persistent || o.hvp || o.steps_per_launch > 1))
        return fail(p, FWI_ERR_INVALID, "attenuation runs the second-order operator one step per launch, "
                                        "not persistent, not hvp");
    if (o.hvp && (o.order == 4 || o.persistent || o.use_graph || o.forward_only || (o.group == 4 && o.steps_per_launch > 1)))
        return fail(p, FWI_ERR_INVALID, "hvp plans run the second-order operator, not persistent, without graph, "
                                        "not forward-only, several steps per launch with groups of 1 or 2 only");
    if (o.order == 4) {
        if (o.persistent) return fail(p, FWI_ERR_INVALID, "the fourth-order operator has no persistent form");
        if (o.steps_per_launch >= 3)
            return fail(p, FWI_ERR_INVALID, "the fourth-order operator runs one or two forward steps per launch");
        if (o.rows != 0 && o.rows != 1 && o.rows != 2 && o.rows != 4)
            return fail(p, FWI_ERR_INVALID, "the fourth-order operator needs rows of 1, 2 or 4");
    }
    for (int i = 0; i < n_media; ++i) {
        std::string msg;
        fwi_status st = validate_grid(grids[i], i, msg, o.order);
        if (st != FWI_OK) return fail(p, st, msg);
    }

    p->dtype = dtype;
    p->opt = o;
    // hvp plans: groups of 2 by default, so that the dual fields of the
    // multi-step kernels take the LDS of four FP32 transmits
    p->G = o.group ? o.group : (o.mode == FWI_PLAIN ? 1 : o.hvp ? 2 : 4);
    // default: three forward-type and two adjoint steps per launch on 64 x 8
    // tiles (one step on 64 x 16 for the plain form); with an explicit rows
    // value that multi-step tiles do not support, one step
    auto two_step_ok = [&](int rows) {
        if (rows != 1 && rows != 2 && rows != 4) return false;
        // LDS of the two-step adjoint: tile + 2 (fields, q, bt) and two tile + 1
        // field planes less their two corner cells
        const size_t n0 = (size_t)(kTileX + 4) * (kWavesZ * rows + 4), n1 = (size_t)(kTileX + 2) * (kWavesZ * rows + 2);
        const size_t ts = (dtype == FWI_F64 ? 8 : 4) * (o.hvp ? 2 : 1);
        return (n0 * (p->G + 2) + 2 * (n1 - 2) * p->G) * ts <= kLdsBytes;
    };
    p->order = o.order == 4 ? 4 : 2;
    if (p->order == 4) {
        // one forward step per launch unless two are asked for (plain mode:
        // one); the adjoint runs one step per launch
        p->S = (o.steps_per_launch == 2 && o.mode != FWI_PLAIN) ? 2 : 1;
        p->rows = o.rows ? o.rows : 1;
        if (lds4_need(dtype, p->G, p->rows, p->S) > kLdsBytes)
            return fail(p, FWI_ERR_INVALID, "the fourth-order tile of these rows does not fit the LDS");
    } else if (o.steps_per_launch == 3) {
        // three forward-type steps and two adjoint steps per launch
        p->S = 3;
        p->rows = o.rows ? o.rows : 2;
        if (!two_step_ok(p->rows))
            return fail(p, FWI_ERR_INVALID, "multi-step launches need rows of 1, 2 or 4 whose tile fits the LDS");
    } else if (o.steps_per_launch == 2) {
        p->S = 2;
        p->rows = o.rows ? o.rows : 2;
        if (!two_step_ok(p->rows))
            return fail(p, FWI_ERR_INVALID, "two steps per launch need rows of 1, 2 or 4 whose tile fits the LDS");
    } else if (o.steps_per_launch == 1 || o.mode == FWI_PLAIN || (o.hvp && p->G == 4) || o.attenuation) {
        p->S = 1;
        p->rows = o.rows ? o.rows : 4;
    } else {
        // default: three forward steps and two adjoint steps per launch (two
        // and two for the persistent form)
        p->rows = o.rows ? o.rows : 2;
        p->S = two_step_ok(p->rows) ? (o.persistent ? 2 : 3) : 1;
    }
    p->acc_double = dtype == FWI_F64 || o.acc_double;
    p->hvp = o.hvp != 0;
    p->att = o.attenuation != 0;
    p->nacc = p->att ? 3 : 2;
    // an hvp plan stores (value, derivative) pairs in every field, coefficient and accumulator
    p->tsize = (dtype == FWI_F64 ? 8 : 4) * (p->hvp ? 2 : 1);
    p->asize = (p->acc_double ? 8 : 4) * (p->hvp ? 2 : 1);
    const int G = p->G, rows = p->rows;
    const int tile_rows = kWavesZ * rows;

    // ---------------- media and items
    p->media.resize(n_media);
    for (int i = 0; i < n_media; ++i) {
        MediumPlan& m = p->media[i];
        m.g = grids[i];
        m.src.assign(grids[i].src, grids[i].src + grids[i].n_tx);
        m.rcv.assign(grids[i].rcv, grids[i].rcv + (size_t)grids[i].n_tx * grids[i].n_rcv);
        m.g.src = nullptr;
        m.g.rcv = nullptr;
        // the step kernels address a field plane ([nz][nx][G]) and the
        // coefficient array ([nz][nx][2]) with 32-bit byte offsets
        const uint64_t span = (uint64_t)m.g.nx * m.g.nz * (uint64_t)std::max(G, 2) * p->tsize;
        if (span >= (1ULL << 32))
            return fail(p, FWI_ERR_INVALID, "grid too large: nx*nz*max(group,2)*sizeof(dtype) must be below 4 GiB");
        m.dmax = dmax_of(m.g);
        m.item0 = (int)p->items.size();
        for (int tx = 0; tx < m.g.n_tx; tx += G) {
            ItemPlan it{};
            it.medium = i;
            it.tx0 = tx;
            it.g_used = std::min(G, m.g.n_tx - tx);
            it.tiles_x = (m.g.nx + kTileX - 1) / kTileX;
            it.tiles_z = (m.g.nz + tile_rows - 1) / tile_rows;
            it.n_tiles = it.tiles_x * it.tiles_z;
            p->items.push_back(it);
        }
        m.item1 = (int)p->items.size();
        m.acc_slots = o.mode == FWI_PLAIN ? 1 : (m.item1 - m.item0);
        p->cell_updates += 2LL * m.g.nx * m.g.nz * m.g.nt * m.g.n_tx;
    }

    // ---------------- checkpoint intervals and waves under the memory budget
    double budget = o.mem_budget;
    if (o.host_only && !(budget > 0))
        return fail(p, FWI_ERR_INVALID, "a host-only plan needs mem_budget > 0 (there is no device to ask)");
    if (budget <= 0) {
        size_t fr = 0, tot = 0;
        HIPCHK(p, hipMemGetInfo(&fr, &tot));
        budget = 0.6 * (double)fr;
    }
    auto plane_bytes = [&](const ItemPlan& it) {
        const MediumPlan& m = p->media[it.medium];
        return align_up((size_t)m.g.nx * m.g.nz * G * p->tsize);
    };
    auto state_bytes = [&](const ItemPlan& it, int K) {
        const int T = p->media[it.medium].g.nt;
        const int J = o.forward_only ? 1 : (T + K - 1) / K;
        // segment K + checkpoints 2 (J-1) + up to 4 lambda planes + 2 v planes
        return plane_bytes(it) * (size_t)(K + 2 * (J - 1) + 6);
    };
    auto auto_k = [&](int T) {
        if (T <= 2) return T;
        int K = (int)std::lround(std::sqrt(2.0 * T));
        // an even K lets two-step launches tile every segment exactly; with
        // three forward steps per launch a multiple of 6 lets both kinds do so
        if (p->S == 2 && K % 2) ++K;
        if (p->S == 3 && K % 6) K += 6 - K % 6;
        return std::max(2, std::min(K, T));
    };
    for (auto& it : p->items) {
        const int T = p->media[it.medium].g.nt;
        int K;
        if (o.forward_only) K = 4;       // rolling buffer of four planes, no replay
        else if (o.ckpt_interval == 0) K = auto_k(T);
        else if (o.ckpt_interval >= T) K = T;
        else K = std::max(2, o.ckpt_interval);
        if (T == 1) K = 1;
        it.K = std::min(K, T);
    }
    size_t fixed = 0;
    {
        size_t zmax = 0;
        for (auto& it : p->items) zmax = std::max(zmax, plane_bytes(it));
        fixed += zmax + align_up((size_t)n_media * kMisfitBlocks * sizeof(double));
        for (auto& m : p->media) {
            fixed += align_up((size_t)m.acc_slots * p->nacc * m.g.nx * m.g.nz * p->asize) +
                     align_up((size_t)2 * m.g.nx * m.g.nz * p->tsize);
            if (p->att) fixed += align_up((size_t)m.g.nx * m.g.nz * p->tsize);
            if (p->hvp)
                fixed += align_up((size_t)m.g.n_tx * m.g.nt * p->tsize) +
                         2 * align_up((size_t)m.g.n_tx * m.g.nt * m.g.n_rcv * p->tsize);
        }
    }
    const double state_budget = budget - (double)fixed;
    if (o.forward_only)
        for (auto& it : p->items) it.J = 1;
    const int n_items = (int)p->items.size();
    if (o.mode == FWI_PLAIN) {
        // items run one after another and share one state slot
        if (o.ckpt_interval == 0) {
            size_t mx_all = 0;
            for (auto& it : p->items) mx_all = std::max(mx_all, state_bytes(it, p->media[it.medium].g.nt));
            if ((double)mx_all <= state_budget)
                for (auto& it : p->items) it.K = p->media[it.medium].g.nt;
        }
        for (int i = 0; i < n_items; ++i) p->waves.push_back(Wave{{i}});
    } else {
        // Replay strategies: (a) K ~ sqrt(2T) for every item, all items resident
        // together when they fit (one wave), items upgraded to store-all
        // smallest first while the budget allows, else waves; (b) every plane
        // kept (no recompute), items packed into as many waves as the budget
        // needs; (c) two segments per item (half the planes, half a forward
        // recomputed), in waves.  With an automatic interval the planner keeps
        // the one its cost model prices lowest (executed cell-updates plus a
        // fixed cost per launch); a given interval takes (a)'s packing.
        auto pack = [&]() {
            // waves of items with similar schedule length, each within the budget
            std::vector<Wave> waves;
            std::vector<int> order(n_items);
            for (int i = 0; i < n_items; ++i) order[i] = i;
            auto steps_of = [&](int i) {
                const ItemPlan& it = p->items[i];
                const int T = p->media[it.medium].g.nt, J = (T + it.K - 1) / it.K;
                return 2 * T + it.K * (J - 1);
            };
            std::stable_sort(order.begin(), order.end(), [&](int a2, int b2) { return steps_of(a2) > steps_of(b2); });
            Wave w;
            double used = 0;
            for (int i : order) {
                const double sb = (double)state_bytes(p->items[i], p->items[i].K);
                if (!w.items.empty() && used + sb > state_budget) {
                    waves.push_back(w);
                    w = Wave{};
                    used = 0;
                }
                w.items.push_back(i);
                used += sb;
            }
            if (!w.items.empty()) waves.push_back(w);
            return waves;
        };
        auto strategy_a = [&]() {
            double total = 0;
            for (auto& it : p->items) total += (double)state_bytes(it, it.K);
            if (total > state_budget) return pack();
            if (o.ckpt_interval == 0) {
                // one wave: keep every plane for as many items as the budget allows
                std::vector<int> order(n_items);
                for (int i = 0; i < n_items; ++i) order[i] = i;
                std::stable_sort(order.begin(), order.end(), [&](int a2, int b2) {
                    return state_bytes(p->items[a2], p->media[p->items[a2].medium].g.nt) <
                           state_bytes(p->items[b2], p->media[p->items[b2].medium].g.nt);
                });
                for (int i : order) {
                    ItemPlan& it = p->items[i];
                    const int T = p->media[it.medium].g.nt;
                    const double extra = (double)state_bytes(it, T) - (double)state_bytes(it, it.K);
                    if (total + extra <= state_budget) { total += extra; it.K = T; }
                }
            }
            Wave w;
            for (int i = 0; i < n_items; ++i) w.items.push_back(i);
            return std::vector<Wave>{w};
        };
        // modelled seconds of one gradient: executed cell-updates (recompute
        // included) at the step kernels' rate plus a fixed cost per launch
        // (MI355X, FP32, groups of 4, three forward steps per launch: 2.26 ps
        // per executed update and 10 us per launch reproduce both the
        // one-wave checkpointed and the 22-wave store-all timing of the
        // 64-media benchmark workload; FP64 updates cost twice as much, and
        // so does a Hessian-vector product's dual-number update against one
        // of its real type: 5.76 s per product on the 16-media 512^2
        // unfolded workload, every plane kept in 37 waves, is 4.2 ps per
        // FP32 dual update once 10 us per launch is taken off)
        auto model_seconds = [&](const std::vector<Wave>& waves) {
            const double t_update = 2.26e-12 * (dtype == FWI_F64 ? 2.0 : 1.0) * (p->hvp ? 2.0 : 1.0),
                         t_launch = 10e-6;
            int S = p->S;
            for (auto& it : p->items)
                if (S >= 2 && it.K < 4 && it.K < p->media[it.medium].g.nt) S = 1;
            const int Sa = adjoint_steps(p->order, S);
            double exec = 0, launches = 0;
            for (auto& it : p->items) {
                const MediumPlan& m = p->media[it.medium];
                const int T = m.g.nt, J = (T + it.K - 1) / it.K;
                exec += (double)m.g.nx * m.g.nz * it.g_used * (2.0 * T + (double)it.K * (J - 1));
            }
            for (const Wave& w : waves) {
                int steps = 0;
                for (int i : w.items) {
                    const ItemPlan& it = p->items[i];
                    const int T = p->media[it.medium].g.nt, J = (T + it.K - 1) / it.K, last = T - (J - 1) * it.K;
                    steps = std::max(steps, (T + S - 1) / S + (last + Sa - 1) / Sa +
                                                ((it.K + S - 1) / S + (it.K + Sa - 1) / Sa) * (J - 1));
                }
                for (int s2 = 0; s2 < steps; ++s2) {
                    unsigned bits = 0;
                    for (int i : w.items) {
                        const ItemPlan& it = p->items[i];
                        const int T = p->media[it.medium].g.nt;
                        const Step st = decode(T, it.K, (T + it.K - 1) / it.K, s2, S, Sa);
                        if (st.phase == kIdle) continue;
                        bits |= st.phase == kAdj ? (st.count == 2 ? 8u : 4u)
                                                 : (st.count == 3 ? 16u : st.count == 2 ? 2u : 1u);
                    }
                    launches += __builtin_popcount(bits);
                }
            }
            return exec * t_update + launches * t_launch;
        };
        std::vector<Wave> best = strategy_a();
        if (o.ckpt_interval == 0 && !o.forward_only && !o.single_wave) {
            std::vector<int> best_k(n_items);
            for (int i = 0; i < n_items; ++i) best_k[i] = p->items[i].K;
            double best_t = model_seconds(best);
            for (int variant = 0; variant < 2; ++variant) {
                for (auto& it : p->items) {
                    const int T = p->media[it.medium].g.nt;
                    int K = variant == 0 ? T : (T + 1) / 2;
                    if (variant == 1 && p->S == 3 && K % 6 && K < T) K += 6 - K % 6;
                    if (variant == 1 && p->S == 2 && K % 2 && K < T) ++K;
                    it.K = std::max(1, std::min(K, T));
                }
                std::vector<Wave> cand = pack();
                const double t = model_seconds(cand);
                if (t < best_t) {
                    best_t = t;
                    best = cand;
                    for (int i = 0; i < n_items; ++i) best_k[i] = p->items[i].K;
                }
            }
            for (int i = 0; i < n_items; ++i) p->items[i].K = best_k[i];
        }
        p->waves = best;
    }
    // a launch of two or three steps reads and writes up to four field planes
    // of the segment buffer at once: that needs K >= 4 wherever the buffer wraps
    if (p->S >= 2)
        for (auto& it : p->items)
            if (it.K < 4 && it.K < p->media[it.medium].g.nt) p->S = 1;
    p->Sa = adjoint_steps(p->order, p->S);
    p->nlam = p->Sa == 2 ? 4 : 2;
    for (auto& it : p->items) {
        const int T = p->media[it.medium].g.nt;
        it.J = o.forward_only ? 1 : (T + it.K - 1) / it.K;
        const int S = p->S, Sa = p->Sa, last = T - (it.J - 1) * it.K;
        it.steps = (T + S - 1) / S + (last + Sa - 1) / Sa + ((it.K + S - 1) / S + (it.K + Sa - 1) / Sa) * (it.J - 1);
        const MediumPlan& m = p->media[it.medium];
        p->recompute_updates += (int64_t)it.K * (it.J - 1) * m.g.nx * m.g.nz * it.g_used;
    }

    // ---------------- workspace layout:
    // [zero plane][accumulators][misfit partials][coefficients][state of one wave]
    // with a wave's state laid out as [lambda planes of its items][checkpoints][segments][v planes]
    size_t off = 0;
    size_t zmax = 0;
    for (auto& it : p->items) zmax = std::max(zmax, plane_bytes(it));
    p->zero_off = off; p->zero_bytes = zmax; off += zmax;
    p->acc_region_off = off;
    for (auto& m : p->media) {
        m.acc_off = off;
        off += align_up((size_t)m.acc_slots * p->nacc * m.g.nx * m.g.nz * p->asize);
    }
    p->acc_region_bytes = off - p->acc_region_off;
    p->clear_off = p->zero_off;
    p->clear_bytes = off - p->zero_off;
    p->partial_off = off;
    off += align_up((size_t)n_media * kMisfitBlocks * sizeof(double));
    for (auto& m : p->media) { m.coef_off = off; off += align_up((size_t)2 * m.g.nx * m.g.nz * p->tsize); }
    if (p->att)
        for (auto& m : p->media) { m.eatt_off = off; off += align_up((size_t)m.g.nx * m.g.nz * p->tsize); }
    if (p->hvp)
        for (auto& m : p->media) {
            const size_t ntr = (size_t)m.g.n_tx * m.g.nt * m.g.n_rcv * p->tsize;
            m.wav_off = off; off += align_up((size_t)m.g.n_tx * m.g.nt * p->tsize);
            m.obs_off = off; off += align_up(ntr);
            m.trd_off = off; off += align_up(ntr);
        }
    const size_t state_off = off;
    size_t state_max = 0;
    for (auto& w : p->waves) {
        size_t o2 = state_off;
        w.lam_off = o2;
        for (int i : w.items) { p->items[i].lam_off = o2; o2 += (size_t)p->nlam * plane_bytes(p->items[i]); }
        w.lam_bytes = o2 - w.lam_off;
        for (int i : w.items) { p->items[i].ck_off = o2; o2 += plane_bytes(p->items[i]) * 2 * (size_t)(p->items[i].J - 1); }
        for (int i : w.items) { p->items[i].seg_off = o2; o2 += plane_bytes(p->items[i]) * (size_t)p->items[i].K; }
        for (int i : w.items) { p->items[i].vel_off = o2; o2 += plane_bytes(p->items[i]) * 2; }
        state_max = std::max(state_max, o2 - state_off);
        w.steps = w.fwd = w.adj = 0;
        for (int i : w.items) {
            const ItemPlan& it = p->items[i];
            const int nf = (p->media[it.medium].g.nt + p->S - 1) / p->S;
            w.steps = std::max(w.steps, it.steps);
            w.fwd = std::max(w.fwd, nf);
            w.adj = std::max(w.adj, it.steps - nf);
        }
    }
    off += state_max;
    p->ws_bytes = off;
    for (auto& it : p->items) {
        const MediumPlan& m = p->media[it.medium];
        it.acc_off = m.acc_off + (o.mode == FWI_PLAIN ? 0
                                  : (size_t)(&it - &p->items[m.item0]) * p->nacc * m.g.nx * m.g.nz * p->asize);
    }

    // ---------------- plan tables: profiles, sources, per-tile receiver entries, blocks
    std::vector<unsigned char> tab;
    auto tab_put = [&](const void* src, size_t bytes) {
        size_t o2 = align_up(tab.size());
        tab.resize(o2 + align_up(bytes));
        if (bytes) std::memcpy(tab.data() + o2, src, bytes);
        return o2;
    };
    for (auto& m : p->media) {
        std::vector<double> ex(m.g.nx), ez(m.g.nz);
        for (int i = 0; i < m.g.nx; ++i) ex[i] = prof(i, m.g.nx, m.g.npml, m.dmax) * m.g.dt;
        for (int i = 0; i < m.g.nz; ++i) ez[i] = prof(i, m.g.nz, m.g.npml, m.dmax) * m.g.dt;
        if (p->hvp) {
            // (value, derivative) pairs: the profiles do not depend on the medium
            if (dtype == FWI_F64) {
                std::vector<double> dx(2 * ex.size(), 0.0), dz(2 * ez.size(), 0.0);
                for (size_t i = 0; i < ex.size(); ++i) dx[2 * i] = ex[i];
                for (size_t i = 0; i < ez.size(); ++i) dz[2 * i] = ez[i];
                m.ex_off = tab_put(dx.data(), dx.size() * 8);
                m.ez_off = tab_put(dz.data(), dz.size() * 8);
            } else {
                std::vector<float> dx(2 * ex.size(), 0.0f), dz(2 * ez.size(), 0.0f);
                for (size_t i = 0; i < ex.size(); ++i) dx[2 * i] = (float)ex[i];
                for (size_t i = 0; i < ez.size(); ++i) dz[2 * i] = (float)ez[i];
                m.ex_off = tab_put(dx.data(), dx.size() * 4);
                m.ez_off = tab_put(dz.data(), dz.size() * 4);
            }
        } else if (dtype == FWI_F64) {
            m.ex_off = tab_put(ex.data(), ex.size() * 8);
            m.ez_off = tab_put(ez.data(), ez.size() * 8);
        } else {
            std::vector<float> fx(ex.begin(), ex.end()), fz(ez.begin(), ez.end());
            m.ex_off = tab_put(fx.data(), fx.size() * 4);
            m.ez_off = tab_put(fz.data(), fz.size() * 4);
        }
    }
    for (auto& it : p->items) {
        const MediumPlan& m = p->media[it.medium];
        std::vector<int32_t> src(G, -1);
        for (int g = 0; g < it.g_used; ++g) src[g] = m.src[it.tx0 + g];
        it.src_off = tab_put(src.data(), src.size() * 4);
        // receiver entries grouped by tile, sorted by slot within a tile
        struct Raw { int tile; int32_t slot; int32_t trace_off; int order; };
        std::vector<Raw> raw;
        for (int g = 0; g < it.g_used; ++g) {
            const int tx = it.tx0 + g;
            for (int r = 0; r < m.g.n_rcv; ++r) {
                const int32_t cell = m.rcv[(size_t)tx * m.g.n_rcv + r];
                const int ix = cell % m.g.nx, iz = cell / m.g.nx;
                const int tile = (iz / tile_rows) * it.tiles_x + ix / kTileX;
                raw.push_back({tile, cell * G + g, (int32_t)((int64_t)tx * m.g.nt * m.g.n_rcv + r), (int)raw.size()});
            }
        }
        std::stable_sort(raw.begin(), raw.end(), [](const Raw& a, const Raw& b) {
            return a.tile != b.tile ? a.tile < b.tile : (a.slot != b.slot ? a.slot < b.slot : a.order < b.order);
        });
        std::vector<int32_t> toff(it.n_tiles + 1, 0);
        std::vector<Entry> ent(raw.size());
        for (size_t k = 0; k < raw.size(); ++k) {
            toff[raw[k].tile + 1]++;
            ent[k] = {raw[k].slot, raw[k].trace_off, 0, 0};
        }
        for (int t = 0; t < it.n_tiles; ++t) toff[t + 1] += toff[t];
        for (size_t k = 0; k < ent.size();) {
            size_t e = k;
            while (e < ent.size() && raw[e].tile == raw[k].tile && ent[e].slot == ent[k].slot) ++e;
            ent[k].run = (int32_t)(e - k);
            k = e;
        }
        it.tile_off_off = tab_put(toff.data(), toff.size() * 4);
        it.entry_off = tab_put(ent.data(), ent.size() * sizeof(Entry));
        // the same receivers listed for every tile whose region grown by one cell holds them
        std::vector<Raw> rx;
        for (const Raw& r0 : raw) {
            const int cell = r0.slot / G, ix = cell % m.g.nx, iz = cell / m.g.nx;
            for (int tz = std::max(0, (iz - 1) / tile_rows); tz <= std::min(it.tiles_z - 1, (iz + 1) / tile_rows); ++tz)
                for (int tx = std::max(0, (ix - 1) / kTileX); tx <= std::min(it.tiles_x - 1, (ix + 1) / kTileX); ++tx) {
                    const int xa = tx * kTileX - 1, xb = tx * kTileX + kTileX;
                    const int za = tz * tile_rows - 1, zb = tz * tile_rows + tile_rows;
                    if (ix >= xa && ix <= xb && iz >= za && iz <= zb)
                        rx.push_back({tz * it.tiles_x + tx, r0.slot, r0.trace_off, r0.order});
                }
        }
        std::stable_sort(rx.begin(), rx.end(), [](const Raw& a, const Raw& b) {
            return a.tile != b.tile ? a.tile < b.tile : (a.slot != b.slot ? a.slot < b.slot : a.order < b.order);
        });
        std::vector<int32_t> toffx(it.n_tiles + 1, 0);
        std::vector<Entry> entx(rx.size());
        for (size_t k = 0; k < rx.size(); ++k) {
            toffx[rx[k].tile + 1]++;
            entx[k] = {rx[k].slot, rx[k].trace_off, 0, 0};
        }
        for (int t = 0; t < it.n_tiles; ++t) toffx[t + 1] += toffx[t];
        for (size_t k = 0; k < entx.size();) {
            size_t e = k;
            while (e < entx.size() && rx[e].tile == rx[k].tile && entx[e].slot == entx[k].slot) ++e;
            entx[k].run = (int32_t)(e - k);
            k = e;
        }
        it.tile_off_x_off = tab_put(toffx.data(), toffx.size() * 4);
        it.entry_x_off = tab_put(entx.data(), entx.size() * sizeof(Entry));
    }
    // XCD-aware block table: workgroups are dealt to the XCDs round-robin by
    // block index, so block 8j + k runs on XCD k.  Each item's tiles are cut
    // into kXcd contiguous runs (row-major tile order) and run k is dealt to
    // XCD k, so the halo rows and columns shared by neighbouring tiles are
    // fetched into one L2 instead of several.  Unused slots hold item -1.
    // Items of a wave are ordered longest schedule first, so that the items
    // still active at a late launch own a prefix of the wave's blocks and the
    // launch grid can stop there.
    for (auto& w : p->waves) {
        std::stable_sort(w.items.begin(), w.items.end(),
                         [&](int a2, int b2) { return p->items[a2].steps > p->items[b2].steps; });
        w.blk0 = (int)p->blocks.size();
        std::vector<std::vector<int2>> per(kXcd);
        w.prefix.assign(1, 0);
        for (int i : w.items) {
            const ItemPlan& it = p->items[i];
            size_t rows_needed = 0;
            for (int k = 0; k < kXcd; ++k) {
                const int t0 = (int)((int64_t)it.n_tiles * k / kXcd), t1 = (int)((int64_t)it.n_tiles * (k + 1) / kXcd);
                for (int t = t0; t < t1; ++t) per[k].push_back(make_int2(i, t));
                rows_needed = std::max(rows_needed, per[k].size());
            }
            w.prefix.push_back((int)(rows_needed * kXcd));
        }
        size_t len = 0;
        for (auto& v : per) len = std::max(len, v.size());
        for (size_t j = 0; j < len; ++j)
            for (int k = 0; k < kXcd; ++k)
                p->blocks.push_back(j < per[k].size() ? per[k][j] : make_int2(-1, 0));
        w.nblk = (int)p->blocks.size() - w.blk0;
    }
    const size_t blocks_off = tab_put(p->blocks.data(), p->blocks.size() * sizeof(int2));
    // step-kernel launches of one gradient (per-step form), or one per wave (persistent)
    for (auto& w : p->waves) {
        if (o.persistent) { ++p->kernel_launches; continue; }
        for (int s2 = 0; s2 < w.steps; ++s2) {
            int n_active = 0;
            p->kernel_launches += __builtin_popcount(wave_kinds(p, w, s2, kRunAll, &n_active));
        }
    }
    // persistent form: active-block count of every launch of every wave and call mode
    for (auto& w : p->waves) {
        const int counts[3] = {w.steps, w.fwd, w.adj};
        const int modes[3] = {kRunAll, kRunFwdOnly, kRunAdjOnly};
        for (int m = 0; m < 3; ++m) {
            std::vector<int32_t> nb(std::max(1, counts[m]), 0);
            for (int s2 = 0; s2 < counts[m]; ++s2) {
                int n_active = 0;
                (void)wave_kinds(p, w, s2, modes[m], &n_active);
                nb[s2] = w.prefix[n_active];
            }
            w.nblk_off[m] = tab_put(nb.data(), nb.size() * 4);
            w.n_launch[m] = counts[m];
        }
    }
    p->item_bytes = (p->dtype == FWI_F64 ? sizeof(Item<double, double>)
                     : p->acc_double ? sizeof(Item<float, double>) : sizeof(Item<float, float>)) * p->items.size();
    p->media_bytes = (p->dtype == FWI_F64 ? sizeof(MediumDev<double>) : sizeof(MediumDev<float>)) * p->media.size();
    p->hvp_bytes = p->hvp ? (dtype == FWI_F64 ? sizeof(MediumHvp<double>) : sizeof(MediumHvp<float>)) * p->media.size()
                          : 0;
    const size_t items_off = align_up(tab.size());
    const size_t media_off = align_up(items_off + p->item_bytes);
    const size_t hvp_off = align_up(media_off + p->media_bytes);
    const size_t status_off = align_up(hvp_off + p->hvp_bytes);
    const size_t bar_off = status_off + kAlign;
    p->tables_bytes = bar_off + kAlign;
    tab.resize(p->tables_bytes, 0);
    p->spin_limit = o.barrier_spin > 0 ? (unsigned)o.barrier_spin : (1u << 21);
    if (o.host_only) return FWI_OK;      // no device tables: sizes and launch lists only

    HIPCHK(p, hipMalloc(&p->d_tables, p->tables_bytes));
    HIPCHK(p, hipMemcpy(p->d_tables, tab.data(), p->tables_bytes, hipMemcpyHostToDevice));
    auto* base = reinterpret_cast<unsigned char*>(p->d_tables);
    p->d_blocks = reinterpret_cast<int2*>(base + blocks_off);
    p->d_items = base + items_off;
    p->d_media = base + media_off;
    p->d_hvp = p->hvp ? base + hvp_off : nullptr;
    p->d_status = reinterpret_cast<unsigned*>(base + status_off);
    p->d_bar = reinterpret_cast<unsigned*>(base + bar_off);
    if (o.persistent) HIPCHK(p, persistent_grid(p, &p->pgrid));
    HIPCHK(p, hipHostMalloc(&p->h_stage, align_up(p->item_bytes) + align_up(p->media_bytes) + align_up(p->hvp_bytes),
                            hipHostMallocDefault));
    HIPCHK(p, allow_lds_plan(p));
    HIPCHK(p, hipEventCreateWithFlags(&p->stage_ev, hipEventDisableTiming));
    return FWI_OK;
}

extern "C" fwi_status fwi_plan_create(fwi_plan** out, fwi_dtype dtype, const fwi_grid* grids, int32_t n_media,
                                      const fwi_options* opt)
{
    g_create_error.clear();
    if (!out) { g_create_error = "out must be non-NULL"; return FWI_ERR_INVALID; }
    *out = nullptr;
    fwi_plan* p = new (std::nothrow) fwi_plan();
    if (!p) { g_create_error = "host allocation failed"; return FWI_ERR_NOMEM; }
    fwi_status st = create_impl(p, dtype, grids, n_media, opt);
    if (st != FWI_OK) {
        g_create_error = p->last_error;
        fwi_plan_destroy(p);
        return st;
    }
    *out = p;
    return FWI_OK;
}

extern "C" void fwi_plan_destroy(fwi_plan* p)
{
    if (!p) return;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->stage_ev) (void)hipEventDestroy(p->stage_ev);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->d_tables) (void)hipFree(p->d_tables);
    delete p;
}

extern "C" fwi_status fwi_plan_workspace_size(const fwi_plan* p, size_t* bytes)
{
    if (!p || !bytes) return FWI_ERR_INVALID;
    *bytes = p->ws_bytes;
    return FWI_OK;
}

extern "C" fwi_status fwi_plan_get_info(const fwi_plan* p, fwi_plan_info* info)
{
    if (!p || !info) return FWI_ERR_INVALID;
    std::memset(info, 0, sizeof *info);
    info->cell_updates = p->cell_updates;
    info->recompute_updates = p->recompute_updates;
    info->workspace_bytes = (int64_t)p->ws_bytes;
    info->n_items = (int32_t)p->items.size();
    info->group = p->G;
    info->rows = p->rows;
    info->launches = (int32_t)std::min<int64_t>(p->kernel_launches, INT32_MAX);
    info->waves = (int32_t)p->waves.size();
    info->steps_per_launch = p->S;
    info->max_ckpt = 0;
    info->min_ckpt = INT32_MAX;
    for (auto& it : p->items) {
        info->max_ckpt = std::max(info->max_ckpt, it.K);
        info->min_ckpt = std::min(info->min_ckpt, it.K);
    }
    return FWI_OK;
}

// ----------------------------------------------------------------------------- calls

namespace {

enum Call { kExecute = 0, kForward = 1, kAdjoint = 2, kHvp = 3 };

template <typename T, typename Acc>
void fill_items(fwi_plan* p, const fwi_io* io, unsigned char* ws, bool adj_from_dadj)
{
    auto* items = reinterpret_cast<Item<T, Acc>*>(p->h_stage);
    auto* tabs = reinterpret_cast<unsigned char*>(p->d_tables);
    for (size_t i = 0; i < p->items.size(); ++i) {
        const ItemPlan& ip = p->items[i];
        const MediumPlan& m = p->media[ip.medium];
        const fwi_io& mio = io[ip.medium];
        Item<T, Acc> d{};
        d.nx = m.g.nx; d.nz = m.g.nz; d.nt = m.g.nt; d.g_used = ip.g_used;
        d.K = ip.K; d.J = ip.J; d.tiles_x = ip.tiles_x; d.n_tiles = ip.n_tiles;
        d.n_rcv = m.g.n_rcv; d.tx0 = ip.tx0;
        d.inject_adj = adj_from_dadj ? 1 : 0;
        d.sample = 1;
        d.plane = (int64_t)m.g.nx * m.g.nz * p->G;
        d.wavelet_stride = mio.wavelet_shared ? 0 : m.g.nt;
        d.coef = reinterpret_cast<const T*>(ws + m.coef_off);
        d.ex = reinterpret_cast<const T*>(tabs + m.ex_off);
        d.ez = reinterpret_cast<const T*>(tabs + m.ez_off);
        d.seg = reinterpret_cast<T*>(ws + ip.seg_off);
        d.ck = reinterpret_cast<T*>(ws + ip.ck_off);
        d.lam = reinterpret_cast<T*>(ws + ip.lam_off);
        d.vel = reinterpret_cast<T*>(ws + ip.vel_off);
        d.acc = reinterpret_cast<Acc*>(ws + ip.acc_off);
        d.zero = reinterpret_cast<const T*>(ws + p->zero_off);
        d.wavelet = reinterpret_cast<const T*>(mio.wavelet);
        d.src = reinterpret_cast<const int32_t*>(tabs + ip.src_off);
        d.traces = reinterpret_cast<T*>(mio.traces);
        d.d_obs = reinterpret_cast<const T*>(mio.d_obs);
        d.d_adj = reinterpret_cast<const T*>(mio.d_adj);
        d.tile_off = reinterpret_cast<const int32_t*>(tabs + ip.tile_off_off);
        d.entries = reinterpret_cast<const Entry*>(tabs + ip.entry_off);
        d.tile_off_x = reinterpret_cast<const int32_t*>(tabs + ip.tile_off_x_off);
        d.entries_x = reinterpret_cast<const Entry*>(tabs + ip.entry_x_off);
        d.S = p->S;
        d.Sa = p->Sa;
        d.nlam = p->nlam;                         // 2 or 4: levels are taken modulo it by a mask
        d.sc = make_sched(m.g.nt, ip.K, ip.J, p->S, p->Sa);
        d.dtx = make_div((uint32_t)ip.tiles_x);
        d.dnx = make_div((uint32_t)m.g.nx);
        // the adjoint of the last segment reads levels (J-1)K + 1 .. T of the first pass
        d.keep_from = p->opt.forward_only ? INT_MAX : (ip.J - 1) * ip.K + 1;
        d.eatt = p->att ? reinterpret_cast<const T*>(ws + m.eatt_off) : nullptr;
        if (p->hvp) {
            // the dual kernels read and write the dual copies in the workspace
            d.wavelet = reinterpret_cast<const T*>(ws + m.wav_off);
            d.traces = reinterpret_cast<T*>(ws + m.trd_off);
            d.d_obs = reinterpret_cast<const T*>(ws + m.obs_off);
            d.d_adj = nullptr;
            d.inject_adj = 0;
        }
        items[i] = d;
    }
}

template <typename T>
void fill_media(fwi_plan* p, const fwi_io* io, unsigned char* ws)
{
    auto* media = reinterpret_cast<MediumDev<T>*>(reinterpret_cast<unsigned char*>(p->h_stage) + align_up(p->item_bytes));
    for (size_t i = 0; i < p->media.size(); ++i) {
        const MediumPlan& m = p->media[i];
        const fwi_io& mio = io[i];
        MediumDev<T> d{};
        d.nx = m.g.nx; d.nz = m.g.nz; d.item0 = m.item0; d.item1 = m.item1;
        d.n_tx = m.g.n_tx; d.nt = m.g.nt; d.n_rcv = m.g.n_rcv;
        d.h = m.g.h; d.dt = m.g.dt; d.dmax = m.dmax; d.c_max = m.g.c_max;
        d.npml = m.g.npml;
        d.acc_stride = (int64_t)p->nacc * m.g.nx * m.g.nz;
        d.c = reinterpret_cast<const T*>(mio.c);
        d.rho = reinterpret_cast<const T*>(mio.rho);
        d.coef = reinterpret_cast<T*>(ws + m.coef_off);
        d.eta = p->att ? reinterpret_cast<const T*>(mio.eta) : nullptr;
        d.eatt = p->att ? reinterpret_cast<T*>(ws + m.eatt_off) : nullptr;
        d.grad_eta = p->att ? reinterpret_cast<T*>(mio.grad_eta) : nullptr;
        d.traces = reinterpret_cast<const T*>(mio.traces);
        d.d_obs = reinterpret_cast<const T*>(mio.d_obs);
        d.grad_c = reinterpret_cast<T*>(mio.grad_c);
        d.grad_rho = reinterpret_cast<T*>(mio.grad_rho);
        d.misfit = mio.misfit;
        d.acc0 = ws + m.acc_off;
        d.acc_slots = m.acc_slots;
        media[i] = d;
    }
}

template <typename T>
void fill_hvp(fwi_plan* p, const fwi_io* io, const fwi_hvp_io* dir, unsigned char* ws)
{
    auto* hv = reinterpret_cast<MediumHvp<T>*>(reinterpret_cast<unsigned char*>(p->h_stage) + align_up(p->item_bytes) +
                                               align_up(p->media_bytes));
    for (size_t i = 0; i < p->media.size(); ++i) {
        const MediumPlan& m = p->media[i];
        const fwi_io& mio = io[i];
        MediumHvp<T> d{};
        d.nx = m.g.nx; d.nz = m.g.nz; d.n_tx = m.g.n_tx; d.nt = m.g.nt;
        d.n_rcv = m.g.n_rcv; d.npml = m.g.npml; d.acc_slots = m.acc_slots; d.wavelet_shared = mio.wavelet_shared ? 1 : 0;
        d.h = m.g.h; d.dt = m.g.dt; d.dmax = m.dmax; d.c_max = m.g.c_max;
        d.acc_stride = 2LL * m.g.nx * m.g.nz;
        d.c = reinterpret_cast<const T*>(mio.c);
        d.rho = reinterpret_cast<const T*>(mio.rho);
        d.dc = reinterpret_cast<const T*>(dir[i].dc);
        d.drho = reinterpret_cast<const T*>(dir[i].drho);
        d.wavelet = reinterpret_cast<const T*>(mio.wavelet);
        d.d_obs = reinterpret_cast<const T*>(mio.d_obs);
        d.traces = reinterpret_cast<T*>(mio.traces);
        d.dtraces = reinterpret_cast<T*>(dir[i].dtraces);
        d.grad_c = reinterpret_cast<T*>(mio.grad_c);
        d.grad_rho = reinterpret_cast<T*>(mio.grad_rho);
        d.hv_c = reinterpret_cast<T*>(dir[i].hv_c);
        d.hv_rho = reinterpret_cast<T*>(dir[i].hv_rho);
        d.coef = reinterpret_cast<Dual<T>*>(ws + m.coef_off);
        d.wav = reinterpret_cast<Dual<T>*>(ws + m.wav_off);
        d.obs = reinterpret_cast<Dual<T>*>(ws + m.obs_off);
        d.tr = reinterpret_cast<Dual<T>*>(ws + m.trd_off);
        d.acc0 = ws + m.acc_off;
        hv[i] = d;
    }
}

void fill_descriptors(fwi_plan* p, const fwi_io* io, const fwi_hvp_io* dir, unsigned char* ws, bool adj_from_dadj)
{
    if (p->hvp) {
        if (p->dtype == FWI_F64) {
            fill_items<Dual<double>, Dual<double>>(p, io, ws, false);
            fill_media<double>(p, io, ws);
            fill_hvp<double>(p, io, dir, ws);
        } else {
            if (p->acc_double) fill_items<Dual<float>, Dual<double>>(p, io, ws, false);
            else fill_items<Dual<float>, Dual<float>>(p, io, ws, false);
            fill_media<float>(p, io, ws);
            fill_hvp<float>(p, io, dir, ws);
        }
        return;
    }
    if (p->dtype == FWI_F64) fill_items<double, double>(p, io, ws, adj_from_dadj);
    else if (p->acc_double) fill_items<float, double>(p, io, ws, adj_from_dadj);
    else fill_items<float, float>(p, io, ws, adj_from_dadj);
    if (p->dtype == FWI_F64) fill_media<double>(p, io, ws);
    else fill_media<float>(p, io, ws);
}

template <typename T, typename Acc>
void enqueue_medium(fwi_plan* p, hipStream_t st, int which, unsigned char* ws)
{
    const int nm = (int)p->media.size();
    int64_t nmax = 0;
    for (auto& m : p->media) nmax = std::max<int64_t>(nmax, (int64_t)m.g.nx * m.g.nz);
    const auto* md = reinterpret_cast<const MediumDev<T>*>(p->d_media);
    const dim3 g2(grid_for(nmax, 256, 2048), nm);
    if (recording()) {
        if (which == 0) record(FWI_K_PREP, g2, dim3(256), 0);
        else if (which == 1) {
            record(FWI_K_MISFIT_PARTIAL, dim3(kMisfitBlocks, nm), dim3(256), 0);
            record(FWI_K_MISFIT_FINAL, dim3((nm + 63) / 64), dim3(64), 0);
        } else record(FWI_K_FINALIZE, g2, dim3(256), 0);
        return;
    }
    if (which == 0) {
        hipLaunchKernelGGL(prep_kernel<T>, g2, dim3(256), 0, st, md, p->d_status);
    } else if (which == 1) {
        double* partial = reinterpret_cast<double*>(ws + p->partial_off);
        hipLaunchKernelGGL(misfit_partial_kernel<T>, dim3(kMisfitBlocks, nm), dim3(256), 0, st, md, partial);
        hipLaunchKernelGGL(misfit_final_kernel<T>, dim3((nm + 63) / 64), dim3(64), 0, st, md, nm,
                           (const double*)partial, p->d_status);
    } else {
        hipLaunchKernelGGL((finalize_kernel<T, Acc>), g2, dim3(256), 0, st, md, p->d_status);
    }
}

void medium_kernels(fwi_plan* p, hipStream_t st, int which, unsigned char* ws)
{
    if (p->dtype == FWI_F64) enqueue_medium<double, double>(p, st, which, ws);
    else if (p->acc_double) enqueue_medium<float, double>(p, st, which, ws);
    else enqueue_medium<float, float>(p, st, which, ws);
}

// The whole launch sequence of one call on stream st (no host synchronisation).
void enqueue_sequence(fwi_plan* p, hipStream_t st, unsigned char* ws, int call, bool want_grad)
{
    zero_words(st, p->d_status, 1);
    // an execute without gradient outputs is a forward solve (+ misfit)
    if (call == kExecute && !want_grad) call = kForward;
    if (call != kAdjoint) {
        zero_bytes(st, ws + p->clear_off, p->clear_bytes);
        medium_kernels(p, st, 0, ws);
    } else {
        zero_bytes(st, ws + p->acc_region_off, p->acc_region_bytes);
    }
    const int mode = call == kExecute ? kRunAll : call == kForward ? kRunFwdOnly : kRunAdjOnly;
    for (const Wave& w : p->waves) {
        const int S = call == kExecute ? w.steps : call == kForward ? w.fwd : w.adj;
        g_rec.wave = (int)(&w - p->waves.data());
        if (call != kForward) zero_bytes(st, ws + w.lam_off, w.lam_bytes);
        if (p->opt.persistent) {
            zero_words(st, p->d_bar, 4);
            launch_persistent(p, st, w, call == kExecute ? 0 : call == kForward ? 1 : 2, mode);
            continue;
        }
        for (int s = 0; s < S; ++s) {
            int n_active = 0;
            const unsigned kinds = wave_kinds(p, w, s, mode, &n_active);
            const dim3 grid((unsigned)w.prefix[n_active]);
            g_rec.step = s;
            for (int k = 0; k < 5; ++k)
                if (kinds & (1u << k)) step(p, k, grid, st, p->d_blocks + w.blk0, s, mode);
        }
        g_rec.step = -1;
    }
    g_rec.wave = -1;
    if (call != kAdjoint) medium_kernels(p, st, 1, ws);
    if (call != kForward) medium_kernels(p, st, 2, ws);
}

// One-step dual kernels of an hvp plan (kind 0 forward-type, 2 adjoint).
template <typename T, typename Acc>
void step_hvp_t(int G, int kind, dim3 grid, hipStream_t st, const void* items, const int2* blocks, int s, int rows)
{
    const dim3 blk(kTileX, kWavesZ);
    auto go = [&](auto g) {
        constexpr int GG = decltype(g)::value;
        const auto* it = reinterpret_cast<const Item<T, Acc>*>(items);
        if (kind == 0) {
            hipLaunchKernelGGL((fwd1_kernel<T, GG, Acc>), grid, blk, 0, st, it, blocks, s, (int)kRunAll, rows);
        } else if (kind == 2) {
            hipLaunchKernelGGL((adj1_kernel<T, GG, Acc>), grid, blk, 0, st, it, blocks, s, (int)kRunAll, rows);
        } else if constexpr (GG <= 2) {
            // two- and three-step launches (plans with groups of 4 run one step)
            if (rows == 1) launch2<T, Acc, GG, 1>(kind, grid, st, it, blocks, s, (int)kRunAll);
            else if (rows == 2) launch2<T, Acc, GG, 2>(kind, grid, st, it, blocks, s, (int)kRunAll);
            else launch2<T, Acc, GG, 4>(kind, grid, st, it, blocks, s, (int)kRunAll);
        }
    };
    if (G == 1) go(std::integral_constant<int, 1>());
    else if (G == 2) go(std::integral_constant<int, 2>());
    else go(std::integral_constant<int, 4>());
}

void step_hvp(fwi_plan* p, int kind, dim3 grid, hipStream_t st, const int2* blocks, int s)
{
    if (recording()) { record(kind, grid, dim3(kTileX, kWavesZ), step_lds(p, kind)); return; }
    if (p->dtype == FWI_F64) step_hvp_t<Dual<double>, Dual<double>>(p->G, kind, grid, st, p->d_items, blocks, s, p->rows);
    else if (p->acc_double) step_hvp_t<Dual<float>, Dual<double>>(p->G, kind, grid, st, p->d_items, blocks, s, p->rows);
    else step_hvp_t<Dual<float>, Dual<float>>(p->G, kind, grid, st, p->d_items, blocks, s, p->rows);
}

template <typename T, typename A>
void hvp_medium(fwi_plan* p, hipStream_t st, int which)
{
    const int nm = (int)p->media.size();
    int64_t nmax = 0, tmax = 0;
    for (auto& m : p->media) {
        nmax = std::max<int64_t>(nmax, (int64_t)m.g.nx * m.g.nz);
        tmax = std::max<int64_t>(tmax, (int64_t)m.g.n_tx * m.g.nt * (m.g.n_rcv + 1));
    }
    const auto* md = reinterpret_cast<const MediumHvp<T>*>(p->d_hvp);
    if (recording()) {
        if (which == 0) {
            record(FWI_K_PREP_HVP, dim3(grid_for(nmax, 256, 2048), nm), dim3(256), 0);
            record(FWI_K_PACK_HVP, dim3(grid_for(tmax, 256, 2048), nm), dim3(256), 0);
        } else if (which == 1) {
            record(FWI_K_UNPACK_HVP, dim3(grid_for(tmax, 256, 2048), nm), dim3(256), 0);
        } else {
            record(FWI_K_FINALIZE_HVP, dim3(grid_for(nmax, 256, 2048), nm), dim3(256), 0);
        }
        return;
    }
    if (which == 0) {
        hipLaunchKernelGGL(prep_hvp_kernel<T>, dim3(grid_for(nmax, 256, 2048), nm), dim3(256), 0, st, md, p->d_status);
        hipLaunchKernelGGL(pack_hvp_kernel<T>, dim3(grid_for(tmax, 256, 2048), nm), dim3(256), 0, st, md);
    } else if (which == 1) {
        hipLaunchKernelGGL(unpack_hvp_kernel<T>, dim3(grid_for(tmax, 256, 2048), nm), dim3(256), 0, st, md);
    } else {
        hipLaunchKernelGGL((finalize_hvp_kernel<T, A>), dim3(grid_for(nmax, 256, 2048), nm), dim3(256), 0, st, md,
                           p->d_status);
    }
}

void hvp_medium_kernels(fwi_plan* p, hipStream_t st, int which)
{
    if (p->dtype == FWI_F64) hvp_medium<double, double>(p, st, which);
    else if (p->acc_double) hvp_medium<float, double>(p, st, which);
    else hvp_medium<float, float>(p, st, which);
}

// The launch sequence of fwi_plan_hvp: dual coefficients and inputs, the
// dual gradient schedule of every wave, then traces, misfit and the gradient
// with its derivative.
void enqueue_hvp(fwi_plan* p, hipStream_t st, unsigned char* ws)
{
    zero_words(st, p->d_status, 1);
    zero_bytes(st, ws + p->clear_off, p->clear_bytes);
    hvp_medium_kernels(p, st, 0);
    for (const Wave& w : p->waves) {
        g_rec.wave = (int)(&w - p->waves.data());
        zero_bytes(st, ws + w.lam_off, w.lam_bytes);
        for (int s = 0; s < w.steps; ++s) {
            int n_active = 0;
            const unsigned kinds = wave_kinds(p, w, s, kRunAll, &n_active);
            const dim3 grid((unsigned)w.prefix[n_active]);
            g_rec.step = s;
            for (int k = 0; k < 5; ++k)
                if (kinds & (1u << k)) step_hvp(p, k, grid, st, p->d_blocks + w.blk0, s);
        }
        g_rec.step = -1;
    }
    g_rec.wave = -1;
    hvp_medium_kernels(p, st, 1);
    medium_kernels(p, st, 1, ws);       // misfit of the primal traces
    hvp_medium_kernels(p, st, 2);
}

// allow_graph = false: eager launches only and no replay state recorded for
// the workspace (the no-allocation variant, whose workspace callers never see).
fwi_status run_call(fwi_plan* p, const fwi_io* io, void* workspace, size_t bytes, void* stream, int call,
                    bool allow_graph = true, const fwi_hvp_io* dir = nullptr)
{
    if (!p) return FWI_ERR_INVALID;
    p->last_error.clear();
    if (p->opt.host_only) return fail(p, FWI_ERR_INVALID, "host-only plan: no device calls");
    if (!io) return fail(p, FWI_ERR_INVALID, "io must be non-NULL");
    if (p->hvp != (call == kHvp))
        return fail(p, FWI_ERR_INVALID, p->hvp ? "this plan was created for fwi_plan_hvp (options.hvp = 1)"
                                               : "fwi_plan_hvp needs a plan created with options.hvp = 1");
    if (call == kHvp) {
        if (!dir) return fail(p, FWI_ERR_INVALID, "dir must be non-NULL");
        for (size_t i = 0; i < p->media.size(); ++i) {
            if (!dir[i].dc || !dir[i].hv_c) return fail(p, FWI_ERR_INVALID, "dc and hv_c are required");
            if (!io[i].d_obs) return fail(p, FWI_ERR_INVALID, "a Hessian-vector product needs d_obs");
        }
    }
    if (!workspace || bytes < p->ws_bytes) return fail(p, FWI_ERR_WORKSPACE, "workspace missing or too small");
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0)
        return fail(p, FWI_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    bool want_grad = false, dadj = false;
    for (size_t i = 0; i < p->media.size(); ++i) {
        const fwi_io& m = io[i];
        if (!m.c || !m.rho || !m.wavelet || !m.traces) return fail(p, FWI_ERR_INVALID, "c, rho, wavelet and traces are required");
        const bool g = m.grad_c || m.grad_rho || (p->att && m.grad_eta);
        want_grad |= g;
        if (call == kExecute && g && !m.d_obs) return fail(p, FWI_ERR_INVALID, "a gradient needs d_obs");
        if (call == kAdjoint) {
            if (!m.d_adj && !m.d_obs) return fail(p, FWI_ERR_INVALID, "adjoint needs d_adj or d_obs");
            if (i == 0) dadj = m.d_adj != nullptr;
            else if (dadj != (m.d_adj != nullptr)) return fail(p, FWI_ERR_INVALID, "d_adj must be given for all media or none");
        }
    }
    if (p->opt.forward_only && (want_grad || call == kAdjoint))
        return fail(p, FWI_ERR_INVALID, "forward-only plan: no adjoint or gradient");
    if (call == kAdjoint && std::find(p->fwd_ws.begin(), p->fwd_ws.end(), workspace) == p->fwd_ws.end())
        return fail(p, FWI_ERR_STATE, "no forward state in this workspace");
    if (call != kExecute && call != kHvp && p->waves.size() > 1)
        return fail(p, FWI_ERR_INVALID, "forward/adjoint need every item resident at once: create the plan "
                                        "with single_wave = 1 and a memory budget that holds all items");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);

    // descriptors: reuse the pinned staging buffer once the previous upload has been consumed
    if (p->stage_pending) HIPCHK(p, hipEventSynchronize(p->stage_ev));
    fill_descriptors(p, io, dir, ws, dadj);
    HIPCHK(p, hipMemcpyAsync(p->d_items, p->h_stage,
                             p->hvp ? align_up(p->item_bytes) + align_up(p->media_bytes) + p->hvp_bytes
                                    : align_up(p->item_bytes) + p->media_bytes,
                             hipMemcpyHostToDevice, st));
    HIPCHK(p, hipEventRecord(p->stage_ev, st));
    p->stage_pending = true;

    const bool graph = allow_graph && p->opt.use_graph && call == kExecute;
    if (call == kHvp) {
        enqueue_hvp(p, st, ws);
        HIPCHK(p, hipGetLastError());
        p->last_stream = st;
        p->have_call = true;
        p->fwd_ws.erase(std::remove(p->fwd_ws.begin(), p->fwd_ws.end(), workspace), p->fwd_ws.end());
        return FWI_OK;
    }
    if (graph) {
        const unsigned flags = want_grad ? 1u : 0u;
        if (!p->gexec || p->graph_ws != workspace || p->graph_flags != flags) {
            if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
            if (!p->cap_stream) HIPCHK(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
            hipGraph_t gr = nullptr;
            HIPCHK(p, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
            enqueue_sequence(p, p->cap_stream, ws, call, want_grad);
            HIPCHK(p, hipStreamEndCapture(p->cap_stream, &gr));
            hipError_t e = hipGraphInstantiate(&p->gexec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) return fail(p, FWI_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            p->graph_ws = workspace;
            p->graph_flags = flags;
        }
        HIPCHK(p, hipGraphLaunch(p->gexec, st));
    } else {
        enqueue_sequence(p, st, ws, call, want_grad);
    }
    HIPCHK(p, hipGetLastError());
    p->last_stream = st;
    p->have_call = true;
    // a forward leaves replay state in its workspace; any other call consumes or overwrites it
    p->fwd_ws.erase(std::remove(p->fwd_ws.begin(), p->fwd_ws.end(), workspace), p->fwd_ws.end());
    if (allow_graph && (call == kForward || (call == kExecute && !want_grad))) p->fwd_ws.push_back(workspace);
    return FWI_OK;
}

}  // namespace

extern "C" fwi_status fwi_plan_execute(fwi_plan* p, const fwi_io* io, void* ws, size_t bytes, void* stream)
{
    return run_call(p, io, ws, bytes, stream, kExecute);
}

extern "C" fwi_status fwi_plan_forward(fwi_plan* p, const fwi_io* io, void* ws, size_t bytes, void* stream)
{
    return run_call(p, io, ws, bytes, stream, kForward);
}

extern "C" fwi_status fwi_plan_adjoint(fwi_plan* p, const fwi_io* io, void* ws, size_t bytes, void* stream)
{
    return run_call(p, io, ws, bytes, stream, kAdjoint);
}

extern "C" fwi_status fwi_plan_hvp(fwi_plan* p, const fwi_io* io, const fwi_hvp_io* dir, void* ws, size_t bytes,
                                   void* stream)
{
    return run_call(p, io, ws, bytes, stream, kHvp, true, dir);
}

// ----------------------------------------------------------------------------- no-allocation variant
//
// The workspace of fwi_plan_execute_scratch lives in a file-scope device
// array.  In host code its name stands for a host-side shadow, not a device
// address: the device address is looked up once per device with
// hipGetSymbolAddress (each GPU holds its own copy) and only that pointer is
// handed to kernels.  Every call on a device shares the array; the launch
// sequence clears what must start at zero (zero plane, accumulators, adjoint
// planes) and writes everything else before reading it.

static __device__ __align__(256) unsigned char scratch[FWI_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up once).
fwi_status scratch_of_current_device(fwi_plan* p, void** out)
{
    int dev = -1;
    HIPCHK(p, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(p, FWI_ERR_INVALID, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(p, FWI_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FWI_OK;
}

}  // namespace

extern "C" fwi_status fwi_plan_execute_scratch(fwi_plan* p, const fwi_io* io, void* stream)
{
    if (!p) return FWI_ERR_INVALID;
    p->last_error.clear();
    if (p->ws_bytes > FWI_SCRATCH_BYTES) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "plan needs %zu bytes of workspace, the static scratch holds %zu: create the plan with a "
                      "smaller mem_budget or fewer media",
                      p->ws_bytes, (size_t)FWI_SCRATCH_BYTES);
        return fail(p, FWI_ERR_WORKSPACE, buf);
    }
    void* ws = nullptr;
    const fwi_status st = scratch_of_current_device(p, &ws);
    if (st != FWI_OK) return st;
    // the eager launch sequence only: recording a graph would allocate
    return run_call(p, io, ws, FWI_SCRATCH_BYTES, stream, kExecute, /*allow_graph=*/false);
}

extern "C" fwi_status fwi_plan_launches(const fwi_plan* cp, int32_t call, fwi_launch* out, int64_t capacity,
                                        int64_t* count)
{
    if (!cp || !count || capacity < 0 || (capacity > 0 && !out) || call < 0 || call > 3) return FWI_ERR_INVALID;
    fwi_plan* p = const_cast<fwi_plan*>(cp);
    if (p->hvp != (call == 3)) return fail(p, FWI_ERR_INVALID, "call does not match the plan (hvp)");
    if (p->opt.forward_only && call != 1) return fail(p, FWI_ERR_INVALID, "forward-only plan: forward calls only");
    if ((call == 1 || call == 2) && p->waves.size() > 1)
        return fail(p, FWI_ERR_INVALID, "forward/adjoint need every item resident at once");
    std::vector<fwi_launch> v;
    g_rec = LaunchRec{&v, -1, -1};
    // addresses are never formed into device pointers while recording
    unsigned char* ws = reinterpret_cast<unsigned char*>(kAlign);
    if (call == 3) enqueue_hvp(p, nullptr, ws);
    else enqueue_sequence(p, nullptr, ws, call == 0 ? kExecute : call == 1 ? kForward : kAdjoint, call == 0);
    g_rec = LaunchRec{};
    *count = (int64_t)v.size();
    const int64_t nw = std::min<int64_t>(capacity, (int64_t)v.size());
    for (int64_t i = 0; i < nw; ++i) out[i] = v[(size_t)i];
    return FWI_OK;
}

extern "C" fwi_status fwi_plan_check(fwi_plan* p)
{
    if (!p) return FWI_ERR_INVALID;
    if (!p->have_call) return FWI_OK;
    HIPCHK(p, hipStreamSynchronize(p->last_stream));
    unsigned flags = 0;
    HIPCHK(p, hipMemcpy(&flags, p->d_status, sizeof flags, hipMemcpyDeviceToHost));
    // the first cause wins: a bad medium or an abandoned launch also leaves non-finite outputs
    if (flags & kFlagMedium) return fail(p, FWI_ERR_MEDIUM, "c or rho not positive and finite");
    if (flags & kFlagCfl) return fail(p, FWI_ERR_CFL, "a cell's c exceeds the declared c_max");
    if (flags & kFlagBarrier) return fail(p, FWI_ERR_HIP, "persistent grid barrier abandoned after its spin limit");
    if (flags & kFlagNonfinite) return fail(p, FWI_ERR_NONFINITE, "non-finite traces, misfit or gradient");
    return FWI_OK;
}

// ----------------------------------------------------------------------------- autotuner
//
// Tile shape and steps per launch are picked by timing short probes of the
// real kernels on the device: the caller's grids (a spread of up to 12 of
// them) with their schedules cut to 24 steps, every plane kept, a
// homogeneous medium at 80% of c_max, zero wavelets and observed traces
// (the kernels' cost does not depend on the values).  Each feasible
// candidate runs one warm-up gradient and two timed ones; the fastest per
// cell-update wins.  Unless the caller fixes it, the group (transmits per
// work item) is searched too.  Results are cached in a small JSON file keyed
// by the GPU architecture, dtype, mode, group and the grids' size class.

namespace {

struct TuneChoice {
    int S = 0, rows = 0, group = 0;
    double ns = 0;
};

// G = 0: the group is part of the search (the size class counts transmits).
std::string tune_key(const char* arch, fwi_dtype dtype, const fwi_options& o, int G, const fwi_grid* grids, int n)
{
    double cells = 0;
    int items = 0;
    for (int i = 0; i < n; ++i) {
        cells += (double)grids[i].nx * grids[i].nz;
        items += G ? (grids[i].n_tx + G - 1) / G : grids[i].n_tx;
    }
    char buf[256];
    std::string a(arch);
    a = a.substr(0, a.find(':'));
    char gs[16];
    if (G) std::snprintf(gs, sizeof gs, "G%d", G);
    else std::snprintf(gs, sizeof gs, "Gauto");
    std::snprintf(buf, sizeof buf, "%s|%s|%s|o%d|%s|c%ld|i%ld", a.c_str(), dtype == FWI_F64 ? "f64" : "f32",
                  o.mode == FWI_PLAIN ? "plain" : "batched", o.order == 4 ? 4 : 2, gs,
                  std::lround(std::log2(cells / n)), std::lround(std::log2((double)items)));
    return buf;
}

// Entries are lines  "key": {"steps_per_launch": S, "rows": R, "group": G, "ns_per_update": X}
bool cache_read(const char* path, std::vector<std::pair<std::string, TuneChoice>>& ent)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        const char* q0 = std::strchr(line, '"');
        if (!q0) continue;
        const char* q1 = std::strchr(q0 + 1, '"');
        if (!q1) continue;
        TuneChoice c;
        const char* sp = std::strstr(q1, "\"steps_per_launch\":");
        const char* rw = std::strstr(q1, "\"rows\":");
        const char* gp = std::strstr(q1, "\"group\":");
        const char* ns = std::strstr(q1, "\"ns_per_update\":");
        if (!sp || !rw || !gp || !ns) continue;
        c.S = std::atoi(sp + 19);
        c.rows = std::atoi(rw + 7);
        c.group = std::atoi(gp + 8);
        c.ns = std::atof(ns + 16);
        ent.emplace_back(std::string(q0 + 1, q1), c);
    }
    std::fclose(f);
    return true;
}

void cache_write(const char* path, const std::vector<std::pair<std::string, TuneChoice>>& ent)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < ent.size(); ++i)
        std::fprintf(f, "\"%s\": {\"steps_per_launch\": %d, \"rows\": %d, \"group\": %d, \"ns_per_update\": %.6g}%s\n",
                     ent[i].first.c_str(), ent[i].second.S, ent[i].second.rows, ent[i].second.group,
                     ent[i].second.ns, i + 1 < ent.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

template <typename T>
void fill(hipStream_t st, void* p, int64_t n, double v)
{
    hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, reinterpret_cast<T*>(p), n, (T)v);
}

struct ProbeBuffers {
    std::vector<void*> ptr;
    ~ProbeBuffers()
    {
        for (void* q : ptr) (void)hipFree(q);
    }
    void* get(size_t bytes)
    {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
        ptr.push_back(q);
        return q;
    }
};

}  // namespace

extern "C" fwi_status fwi_autotune(fwi_dtype dtype, const fwi_grid* grids, int32_t n_media, const fwi_options* base,
                                   fwi_options* out, double* ns_per_update)
{
    g_create_error.clear();
    if (!grids || n_media < 1 || !out) { g_create_error = "grids and out must be non-NULL"; return FWI_ERR_INVALID; }
    if (dtype != FWI_F32 && dtype != FWI_F64) { g_create_error = "unknown dtype"; return FWI_ERR_INVALID; }
    fwi_options o{};
    o.mode = FWI_BATCHED;
    if (base) o = *base;
    for (int i = 0; i < n_media; ++i) {
        std::string msg;
        fwi_status st = validate_grid(grids[i], i, msg, o.order);
        if (st != FWI_OK) { g_create_error = msg; return st; }
    }
    // transmits per work item: the caller's, else searched over 4, 2, 1 (plain: 1)
    const int G = o.group ? o.group : (o.mode == FWI_PLAIN ? 1 : 0);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        g_create_error = "no HIP device";
        return FWI_ERR_HIP;
    }
    const std::string key = tune_key(prop.gcnArchName, dtype, o, G, grids, n_media);
    std::vector<std::pair<std::string, TuneChoice>> cache;
    if (o.tune_cache && cache_read(o.tune_cache, cache))
        for (auto& e : cache)
            if (e.first == key && e.second.S > 0 && e.second.group > 0) {
                *out = o;
                out->steps_per_launch = e.second.S;
                out->rows = e.second.rows;
                out->group = e.second.group;
                if (ns_per_update) *ns_per_update = e.second.ns;
                return FWI_OK;
            }

    // probe grids: a spread of up to 12 media with their schedules cut to 24
    // steps, or lengthened (up to their own step counts) until one timed call
    // covers about 1e9 cell-updates, so that small grids are not timed in
    // the noise of a few launches
    const int n_probe = std::min(n_media, 12);
    std::vector<fwi_grid> pg(n_probe);
    double work = 0.0;
    for (int i = 0; i < n_probe; ++i) {
        pg[i] = grids[(int64_t)i * n_media / n_probe];
        pg[i].nt = std::min(pg[i].nt, 24);
        work += 2.0 * pg[i].nx * pg[i].nz * (double)pg[i].n_tx * pg[i].nt;
    }
    constexpr double kProbeWork = 1e9;
    if (work > 0.0 && work < kProbeWork)
        for (int i = 0; i < n_probe; ++i) {
            const int full = grids[(int64_t)i * n_media / n_probe].nt;
            pg[i].nt = (int)std::min<double>(full, std::ceil(pg[i].nt * kProbeWork / work));
        }
    const size_t ts = dtype == FWI_F64 ? 8 : 4;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        g_create_error = "hipStreamCreate failed";
        return FWI_ERR_HIP;
    }
    ProbeBuffers buf;
    std::vector<fwi_io> io(n_probe);
    bool ok = true;
    for (int i = 0; i < n_probe && ok; ++i) {
        const fwi_grid& g = pg[i];
        const int64_t nc = (int64_t)g.nx * g.nz, ntr = (int64_t)g.n_tx * g.nt * g.n_rcv;
        fwi_io& d = io[i];
        std::memset(&d, 0, sizeof d);
        void *c = buf.get(nc * ts), *rho = buf.get(nc * ts), *w = buf.get((int64_t)g.n_tx * g.nt * ts);
        void *obs = buf.get(ntr * ts), *tr = buf.get(ntr * ts), *gc = buf.get(nc * ts), *gr = buf.get(nc * ts);
        void* mf = buf.get(sizeof(double));
        if (!c || !rho || !w || !obs || !tr || !gc || !gr || !mf) { ok = false; break; }
        if (dtype == FWI_F64) {
            fill<double>(st, c, nc, 0.8 * g.c_max); fill<double>(st, rho, nc, 1000.0);
            fill<double>(st, w, (int64_t)g.n_tx * g.nt, 0.0); fill<double>(st, obs, ntr, 0.0);
        } else {
            fill<float>(st, c, nc, 0.8 * g.c_max); fill<float>(st, rho, nc, 1000.0);
            fill<float>(st, w, (int64_t)g.n_tx * g.nt, 0.0); fill<float>(st, obs, ntr, 0.0);
        }
        d.c = c; d.rho = rho; d.wavelet = w; d.d_obs = obs; d.traces = tr; d.grad_c = gc; d.grad_rho = gr;
        d.misfit = reinterpret_cast<double*>(mf);
    }
    TuneChoice best;
    if (ok) {
        const int cands[][2] = {{3, 1}, {3, 2}, {3, 4}, {2, 1}, {2, 2}, {2, 4}, {1, 1}, {1, 2}, {1, 4}, {1, 8}};
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        const int groups_auto[] = {4, 2, 1};
        const int n_groups = G ? 1 : 3;
        for (int gi = 0; gi < n_groups; ++gi)
        for (auto& cd : cands) {
            const int grp = G ? G : groups_auto[gi];
            if (o.mode == FWI_PLAIN && cd[0] >= 2) continue;
            fwi_options po = o;
            po.group = grp;
            po.steps_per_launch = cd[0];
            po.rows = cd[1];
            po.ckpt_interval = 1 << 30;
            po.use_graph = 0;
            po.persistent = 0;
            po.forward_only = 0;
            po.tune_cache = nullptr;
            fwi_plan* plan = nullptr;
            if (fwi_plan_create(&plan, dtype, pg.data(), n_probe, &po) != FWI_OK) continue;
            if (plan->S != cd[0]) { fwi_plan_destroy(plan); continue; }
            void* ws = nullptr;
            if (hipMalloc(&ws, plan->ws_bytes) != hipSuccess) { fwi_plan_destroy(plan); continue; }
            bool good = fwi_plan_execute(plan, io.data(), ws, plan->ws_bytes, st) == FWI_OK;
            good = good && hipEventRecord(e0, st) == hipSuccess;
            for (int r = 0; r < 2 && good; ++r)
                good = fwi_plan_execute(plan, io.data(), ws, plan->ws_bytes, st) == FWI_OK;
            good = good && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            good = good && fwi_plan_check(plan) == FWI_OK;
            float ms = 0;
            if (good && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
                const double ns = ms * 1e6 / (2.0 * (double)plan->cell_updates);
                if (best.S == 0 || ns < best.ns) best = TuneChoice{cd[0], cd[1], grp, ns};
            }
            (void)hipStreamSynchronize(st);
            (void)hipFree(ws);
            fwi_plan_destroy(plan);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (best.S == 0) {
        g_create_error = ok ? "no candidate could be timed" : "probe allocation failed";
        return ok ? FWI_ERR_HIP : FWI_ERR_NOMEM;
    }
    if (o.tune_cache) {
        bool found = false;
        for (auto& e : cache)
            if (e.first == key) { e.second = best; found = true; }
        if (!found) cache.emplace_back(key, best);
        cache_write(o.tune_cache, cache);
    }
    *out = o;
    out->steps_per_launch = best.S;
    out->rows = best.rows;
    out->group = best.group;
    if (ns_per_update) *ns_per_update = best.ns;
    return FWI_OK;
}
