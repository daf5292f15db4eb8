// Whole-volume solve that allocates nothing, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid allocation).  It is rw_solve with its workspace taken
// from a static device array of fixed size instead of from the caller.
//
// The array lives in this library's code object, one copy per device the
// library is loaded on, for the life of the process.  Host code never uses
// its name as an address: rw_context_create looks its device address up once
// per device (hipGetSymbolAddress, with that device current) and the entry
// point passes that address to the solve, as rw_solve passes a caller's
// workspace.  Every call on one device shares the array, so calls that
// overlap on one device race; nothing in it needs clearing between calls
// (the solve initialises every vector it reads).
#include <map>
#include <mutex>
#include <string>

#include "rw_internal.h"
#include "rw_kernels.h"

namespace rw {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_noalloc_mu;
std::map<int, void*> g_noalloc_ptr;  // device -> device address of `scratch`
}  // namespace

// Called by rw_context_create with `device` current.
rw_status noalloc_register_device(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr.count(device)) return RW_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return RW_ERR_HIP;
    }
    g_noalloc_ptr[device] = ptr;
    return RW_OK;
}

static void* noalloc_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(device);
    return it == g_noalloc_ptr.end() ? nullptr : it->second;
}

}  // namespace rw

using namespace rw;

extern "C" {

size_t rw_solve_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

rw_status rw_solve_noalloc(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                           const rw_options* opts, void* prob_out, uint8_t* argmax_out,
                           rw_stats* stats, void* stream) {
    if (!ctx) return invalid("context is NULL");
    rw_status e = check_volume(vol);
    if (e) return e;
    if (!opts) return invalid("options is NULL");
    if (!seeds) return invalid("seeds are NULL");
    const size_t need =
        rw_solve_workspace_bytes(vol->dims, seeds->num_labels, opts->precision,
                                 opts->solve_all_labels);
    if (need == 0) return invalid("unsupported grid or label count");
    if (need > NOALLOC_SCRATCH_BYTES) {
        set_error("rw_solve_noalloc: this solve needs " + std::to_string(need) +
                  " bytes of scratch, more than the static " +
                  std::to_string(NOALLOC_SCRATCH_BYTES) + " (use rw_solve with a workspace)");
        return RW_ERR_WORKSPACE;
    }
    void* ptr = noalloc_ptr(ctx->device);
    if (!ptr) {
        set_error("rw_solve_noalloc: the static scratch of this context's device is not set up");
        return RW_ERR_HIP;
    }
    // plain launches: no graph objects are built, no timing events are added
    rw_options o = *opts;
    o.use_graph = 0;
    o.kernel_timing = 0;
    return rw_solve(ctx, vol, seeds, &o, prob_out, argmax_out, ptr, NOALLOC_SCRATCH_BYTES, stats,
                    stream);
}

}  // extern "C"
