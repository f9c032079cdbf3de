// Gram products C = X^+ Y without any allocation, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The workspace (the contraction's chunk partials and the ka x kb result) is a file-scope
// device array of LQT_STATIC_SCRATCH_BYTES bytes; each device the library runs on holds its
// own copy until the process ends.  Host code never uses the array's name as an address: its
// device address is looked up once per device (hipGetSymbolAddress, with that device
// current) when a context is created there, and kept per device.
#include <mutex>

#include "gemm.h"
#include "lqt_internal.h"

static __device__ __align__(256) unsigned char scratch[LQT_STATIC_SCRATCH_BYTES];

namespace lqt {

namespace {
constexpr int MAXDEV = 64;
std::mutex g_mu;
void* g_ptr[MAXDEV] = {};
}  // namespace

// Look up the device address of the workspace on the current device (once per device).
void static_scratch_init(int device) {
    LQT_CHECK(device >= 0 && device < MAXDEV, LQT_EINVAL, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return;
    void* p = nullptr;
    LQT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    LQT_CHECK(p != nullptr, LQT_EHIP, "hipGetSymbolAddress returned no address for the static workspace");
    g_ptr[device] = p;
}

static void* static_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (device >= 0 && device < MAXDEV) ? g_ptr[device] : nullptr;
}

// Chunks of the contraction for a ka x kb product of length-n vectors: as many as the
// workspace holds (partials plus the result), at most one per 8192 entries; 0 if even one
// chunk does not fit.
long long static_gram_chunks(long long n, int ka, int kb) {
    const long long ne = (long long)ka * kb;
    const long long cap = (long long)LQT_STATIC_SCRATCH_BYTES / (long long)sizeof(double2);
    if (ne <= 0 || ne > cap / 2) return 0;
    long long nc = cap / ne - 1;
    const long long want = (n + 8191) / 8192;
    if (nc > want) nc = want;
    if (nc > n / 4) nc = n / 4 > 0 ? n / 4 : 1;
    return nc < 1 ? 0 : nc;
}

}  // namespace lqt

extern "C" int lqt_gram_noalloc(lqt_ctx* c, const double* d_x, int ka, const double* d_y, int kb, double* h_c) {
    if (!c) return LQT_EINVAL;
    try {
        LQT_CHECK(ka >= 1 && kb >= 1 && d_x && d_y && h_c, LQT_EINVAL, "bad gram arguments");
        const long long n = 12LL * c->g.canon_sites;
        const long long nc = lqt::static_gram_chunks(n, ka, kb);
        LQT_CHECK(nc >= 1, LQT_EINVAL,
                  "ka * kb too large for the static workspace (" + std::to_string(LQT_STATIC_SCRATCH_BYTES) +
                      " bytes hold at most " +
                      std::to_string(LQT_STATIC_SCRATCH_BYTES / sizeof(double2) / 2) + " result entries)");
        double2* part = (double2*)lqt::static_scratch(c->device);
        LQT_CHECK(part != nullptr, LQT_ESTATE, "static workspace not set up on this device");
        double2* C = part + nc * (long long)ka * kb;
        // every partial entry that k_sum_chunks reads is written by k_gram_part first, so the
        // workspace needs no clearing between calls
        lqt::gemm_gram_into(c->stream, (const double2*)d_x, ka, (const double2*)d_y, kb, n, (int)nc, part, C);
        LQT_HIP(hipMemcpyAsync(h_c, C, sizeof(double2) * (size_t)ka * kb, hipMemcpyDeviceToHost, c->stream));
        LQT_HIP(hipStreamSynchronize(c->stream));
        return LQT_OK;
    } catch (const lqt::Error& e) {
        c->err = e.msg;
        return e.code;
    } catch (...) {
        c->err = "unexpected exception";
        return LQT_EINVAL;
    }
}
