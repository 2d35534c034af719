// sht_synth_noalloc: the float64 synthesis map = Y alm (Sec. 2.1, eq.
// sh-synthesis) for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The transform's workspaces -- the packed input U (T layout) and the
// ring-major Fourier coefficients F -- live in one file-scope device array,
// `scratch`, of kScratchBytes.  Its device address is taken once per device
// with hipGetSymbolAddress (the array's name is only a host-side stand-in)
// and used for every kernel argument.  Each GPU keeps one copy for the life
// of the process; every call on a GPU shares it, so calls that overlap on
// one GPU race.  The kernels write every entry they later read (U including
// its padded RHS columns, F for every ring and order), so nothing needs
// clearing between calls.
#include <hip/hip_runtime.h>

#include <atomic>

#include "mlcr_internal.h"

namespace mlcr {

constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::atomic<void *> g_scratch[kMaxDevices];

// Device address of this device's scratch array (taken on first use, with
// the device current).
static int scratch_address(void **out) {
    int dev = -1;
    MLCR_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MLCR_EUNSUPPORTED, "device index out of range");
    void *p = g_scratch[dev].load();
    if (!p) {
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MLCR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev].store(p);
    }
    *out = p;
    return MLCR_OK;
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace mlcr

using namespace mlcr;

extern "C" int sht_synth_noalloc(mlcr_geom *g, int lmax, int nrhs, const double *alm, double *map,
                                 void *stream) {
    if (!g || !alm || !map) return fail(MLCR_EINVAL, "NULL argument");
    if (((uintptr_t)map & 15u) != 0) return fail(MLCR_EINVAL, "map must be 16-byte aligned");
    if (lmax < 0 || lmax > g->lmax) return fail(MLCR_EINVAL, "lmax exceeds the geometry's lmax");
    if (nrhs < 1) return fail(MLCR_EINVAL, "nrhs must be >= 1");
    const int rc8 = synth_rc(nrhs);
    const size_t ub = round256((size_t)tlayout_doubles(lmax, nrhs, rc8) * sizeof(double));
    const size_t fb = (size_t)nrhs * g->nrings * (lmax + 1) * sizeof(double2);
    if (ub + fb > kScratchBytes)
        return fail(MLCR_EINVAL, "sht_synth_noalloc needs " + std::to_string(ub + fb) +
                                     " bytes of scratch; the limit is " +
                                     std::to_string(kScratchBytes) + " (use sht_synth)");
    void *base = nullptr;
    int rc;
    if ((rc = scratch_address(&base))) return rc;
    double *U = static_cast<double *>(base);
    double2 *F = reinterpret_cast<double2 *>(static_cast<unsigned char *>(base) + ub);
    hipStream_t s = (hipStream_t)stream;
    LegendreArgs a{g, lmax, nrhs, s};
    if ((rc = launch_pack_t(lmax, nrhs, rc8, alm, nullptr, U, s))) return rc;
    if ((rc = launch_legendre_synth(a, U, F))) return rc;
    return launch_ring_synth(g, lmax, nrhs, F, map, MLCR_FP64, s);
}
