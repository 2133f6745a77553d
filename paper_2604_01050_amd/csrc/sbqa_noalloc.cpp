// sbqa_energy_noalloc: energies of given spins with no device allocation.
//
// Its float64 scratch (the dense path's spin matrix and GEMM partials, or the
// relabelled rows of a CSR instance) is one library-owned device array per
// GPU, `scratch` below. Host code never passes the array's name to a kernel
// (in host code it names a host-side stand-in): the device address is looked
// up once per device with hipGetSymbolAddress, with that device current, and
// only that address is used.
#include "sbqa_ctx.h"

#include <mutex>
#include <vector>

namespace {

static __device__ __align__(256) uint8_t scratch[SBQA_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::vector<uint8_t *> g_scratch;   // per device; nullptr until looked up

// Device address of `scratch` on device dev (looked up once, dev made current
// for the lookup and the previous device restored).
sbqa_status scratch_on(int dev, uint8_t **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize((size_t)dev + 1, nullptr);
    if (!g_scratch[(size_t)dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess || !p)
            return sbqa::fail(SBQA_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[(size_t)dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch[(size_t)dev];
    return SBQA_OK;
}

bool is_device_memory(const void *p, int dev) {
    hipPointerAttribute_t a;
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // an unknown host pointer: clear the error it leaves
        return false;
    }
    return a.type == hipMemoryTypeDevice && a.device == dev;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

using namespace sbqa;

extern "C" sbqa_status sbqa_energy_noalloc(sbqa_ctx *c, const int8_t *spins, int32_t count, double *out) {
    clear_error();
    if (!c || (count && (!spins || !out))) return fail(SBQA_EINVAL, "NULL argument");
    if (count < 0) return fail(SBQA_EINVAL, "count must be >= 0");
    if (count == 0) return SBQA_OK;
    const int N = c->N;
    // scratch plan: relabelled rows (CSR), or S [cp][Np] and P [es][cp][Np] (dense)
    size_t off_rows = 0, off_S = 0, off_P = 0, need = 0;
    const bool relabel = c->facts.path == PATH_CSR && !c->pnew.empty();
    EnergyGemm g;
    if (c->facts.path != PATH_CSR) {
        g = energy_gemm(c, count);
        off_S = 0;
        off_P = align256(sizeof(double) * (size_t)g.cp * c->L.Np);
        need = off_P + sizeof(double) * (size_t)g.es * g.cp * c->L.Np;
    } else if (relabel) {
        off_rows = 0;
        need = (size_t)count * N;
    }
    if (need > SBQA_NOALLOC_SCRATCH_BYTES)
        return fail(SBQA_EINVAL, "%d configurations of %d spins need %zu bytes of scratch, above the %zu-byte limit",
                    count, N, need, (size_t)SBQA_NOALLOC_SCRATCH_BYTES);
    if (!is_device_memory(spins, c->device) || !is_device_memory(out, c->device))
        return fail(SBQA_EINVAL, "spins and out must be device memory on the context's device %d", c->device);
    uint8_t *base = nullptr;
    sbqa_status st = scratch_on(c->device, &base);
    if (st != SBQA_OK) return st;
    const int8_t *ds = spins;
    if (relabel) {
        int8_t *rows = reinterpret_cast<int8_t *>(base + off_rows);
        const hipError_t e = launch_spins_to_rows(N, count, c->porig, spins, rows, c->stream);
        if (e != hipSuccess) return fail(SBQA_EDEVICE, "spins to rows: %s", hipGetErrorString(e));
        ds = rows;
    }
    double *S = c->facts.path != PATH_CSR ? reinterpret_cast<double *>(base + off_S) : nullptr;
    double *P = c->facts.path != PATH_CSR ? reinterpret_cast<double *>(base + off_P) : nullptr;
    return ctx_energies_dev(c, ds, count, out, S, P);
}
