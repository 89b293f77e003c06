// The count-only listing that allocates nothing, for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid it).  It runs the same plan and probe kernels as
// tl_list without an output buffer, with every device block the call needs
// carved from one file-scope device array instead of the library's pool.
#include <map>
#include <mutex>
#include <string>

#include "tl_internal.h"

namespace {

// Each GPU the library runs on holds its own copy of this array until the
// process ends.  In host code its name stands for no device address: the
// address is looked up per device (hipGetSymbolAddress) and only that
// pointer is used.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)TL_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;  // device -> address of its copy of scratch

// Address of the current device's copy of scratch, looked up once per
// device with that device current.
char *scratch_on_current_device() {
    int dev = 0;
    TL_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *p = nullptr;
    TL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TL_REQUIRE(p, TL_EHIP, "hipGetSymbolAddress returned no address for the no-allocation scratch");
    g_scratch_ptr[dev] = static_cast<char *>(p);
    return static_cast<char *>(p);
}

}  // namespace

extern "C" int tl_list_count_noalloc(const tl_csr *g, tl_algo a, void *stream, tl_summary *out) {
    try {
        TL_REQUIRE(g && out, TL_EINVAL, "NULL argument");
        TL_REQUIRE(a == TL_APP || a == TL_APM || a == TL_AMM, TL_EINVAL, "unknown algorithm");
        const u64 need = list_count_scratch_bytes(g->n, g->m);
        TL_REQUIRE(need <= NOALLOC_SCRATCH_BYTES, TL_ECAPACITY,
                   "graph too large for the no-allocation listing: its plan needs " + std::to_string(need) +
                       " bytes of scratch, the limit is " + std::to_string(NOALLOC_SCRATCH_BYTES));
        ScratchArena arena{scratch_on_current_device(), NOALLOC_SCRATCH_BYTES, 0};
        const hipStream_t s = (hipStream_t)stream;
        try {
            ArenaScope scope(&arena);
            return list_impl(g, (int)a, 0u, g->n, nullptr, 0, nullptr, nullptr, s, out);
        } catch (...) {
            // nothing may still use the scratch when the error returns
            (void)hipStreamSynchronize(s);
            throw;
        }
    } catch (const TlError &e) {
        tl_set_error(e.msg);
        return e.code;
    } catch (...) {
        tl_set_error("unexpected exception");
        return TL_EHIP;
    }
}
