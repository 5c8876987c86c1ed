// Standalone client of the C ABI (no PyTorch): device memory from hipMalloc,
// one non-blocking HIP stream, one batched gradient of one medium.
//
//   capi_gradient <input.bin> <output.bin>
//
// input.bin (little endian): int32 nx, nz, nt, npml, n_tx, n_rcv, ckpt;
// float64 h, dt, pml_r, pml_cref, c_max; int32 src[n_tx], rcv[n_tx*n_rcv];
// float32 c[nz*nx], rho[nz*nx], wavelet[n_tx*nt], d_obs[n_tx*nt*n_rcv].
// output.bin: float32 traces[n_tx*nt*n_rcv], grad_c[nz*nx], grad_rho[nz*nx];
// float64 misfit.  Exit status 0, or 1 with the library's message.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fwi.h"

namespace {

template <typename T>
bool rd(FILE* f, T* p, size_t n)
{
    return std::fread(p, sizeof(T), n, f) == n;
}

int die(const char* what)
{
    std::fprintf(stderr, "capi_gradient: %s\n", what);
    return 1;
}

void* dev_copy(const void* h, size_t bytes)
{
    void* d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return nullptr;
    if (h && hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return d;
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 3) return die("usage: capi_gradient <input.bin> <output.bin>");
    FILE* in = std::fopen(argv[1], "rb");
    if (!in) return die("cannot open input");
    int32_t hdr[7];
    double par[5];
    if (!rd(in, hdr, 7) || !rd(in, par, 5)) return die("short header");
    const int nx = hdr[0], nz = hdr[1], nt = hdr[2], npml = hdr[3], ntx = hdr[4], nrcv = hdr[5], ckpt = hdr[6];
    const size_t nc = (size_t)nx * nz, ntr = (size_t)ntx * nt * nrcv;
    std::vector<int32_t> src(ntx), rcv((size_t)ntx * nrcv);
    std::vector<float> c(nc), rho(nc), w((size_t)ntx * nt), obs(ntr);
    if (!rd(in, src.data(), src.size()) || !rd(in, rcv.data(), rcv.size()) || !rd(in, c.data(), nc) ||
        !rd(in, rho.data(), nc) || !rd(in, w.data(), w.size()) || !rd(in, obs.data(), ntr))
        return die("short input");
    std::fclose(in);

    fwi_grid g{};
    g.nx = nx; g.nz = nz; g.nt = nt; g.npml = npml;
    g.h = par[0]; g.dt = par[1]; g.pml_r = par[2]; g.pml_cref = par[3]; g.c_max = par[4];
    g.n_tx = ntx; g.n_rcv = nrcv; g.src = src.data(); g.rcv = rcv.data();
    fwi_options o{};
    o.mode = FWI_BATCHED;
    o.ckpt_interval = ckpt;
    fwi_plan* plan = nullptr;
    fwi_status st = fwi_plan_create(&plan, FWI_F32, &g, 1, &o);
    if (st != FWI_OK) {
        std::fprintf(stderr, "capi_gradient: fwi_plan_create: %s: %s\n", fwi_status_string(st), fwi_last_create_error());
        return 1;
    }
    size_t wsb = 0;
    fwi_plan_workspace_size(plan, &wsb);
    void* ws = dev_copy(nullptr, wsb);
    fwi_io io{};
    io.c = dev_copy(c.data(), nc * 4);
    io.rho = dev_copy(rho.data(), nc * 4);
    io.wavelet = dev_copy(w.data(), w.size() * 4);
    io.d_obs = dev_copy(obs.data(), ntr * 4);
    io.traces = dev_copy(nullptr, ntr * 4);
    io.grad_c = dev_copy(nullptr, nc * 4);
    io.grad_rho = dev_copy(nullptr, nc * 4);
    io.misfit = static_cast<double*>(dev_copy(nullptr, sizeof(double)));
    if (!ws || !io.c || !io.rho || !io.wavelet || !io.d_obs || !io.traces || !io.grad_c || !io.grad_rho || !io.misfit)
        return die("device allocation failed");
    hipStream_t stream;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return die("stream");
    st = fwi_plan_execute(plan, &io, ws, wsb, stream);
    if (st == FWI_OK) st = fwi_plan_check(plan);
    if (st != FWI_OK) {
        std::fprintf(stderr, "capi_gradient: %s: %s\n", fwi_status_string(st), fwi_plan_last_error(plan));
        return 1;
    }
    std::vector<float> tr(ntr), gc(nc), gr(nc);
    double J = 0;
    if (hipMemcpy(tr.data(), io.traces, ntr * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(gc.data(), io.grad_c, nc * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(gr.data(), io.grad_rho, nc * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&J, io.misfit, sizeof J, hipMemcpyDeviceToHost) != hipSuccess)
        return die("copy back failed");
    FILE* out = std::fopen(argv[2], "wb");
    if (!out) return die("cannot open output");
    std::fwrite(tr.data(), 4, ntr, out);
    std::fwrite(gc.data(), 4, nc, out);
    std::fwrite(gr.data(), 4, nc, out);
    std::fwrite(&J, 8, 1, out);
    std::fclose(out);
    fwi_plan_destroy(plan);
    (void)hipStreamDestroy(stream);
    for (const void* p : {io.c, io.rho, io.wavelet, io.d_obs, (const void*)io.traces, (const void*)io.grad_c,
                          (const void*)io.grad_rho, (const void*)io.misfit, (const void*)ws})
        (void)hipFree(const_cast<void*>(p));
    return 0;
}
