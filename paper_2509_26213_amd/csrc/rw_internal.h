// Internal declarations shared by the HIP translation units of librw.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>
#include <string>
#include <vector>

#include "rw.h"

namespace rw {

// Grid geometry.  Voxel (x, y, z) lives at z * plane + y * nx + x.  A
// volume time series [nt][nz][ny][nx] (4-D random walker) is stored as the
// grid (nx, ny, nt * nz) with tz = nz planes per time step: plane Z is z =
// Z mod tz of time step Z / tz; tz = 0 for a 3-D grid.
struct Geom {
    int nx, ny, nz;
    int64_t plane, n;
    int tz = 0;
};

// Edge-weight coefficients.  With s = 1 / (hi - lo) (0 for a constant
// image) and dv the raw intensity difference of the two endpoints,
//   w = exp(c64 * dv^2) + eps              (float64 path)
//   w = max(2^(c2_32 * dv^2), FLT_MIN) + eps   (float32 path)
// where c64 = -beta s^2 and c2_32 = c64 log2(e) rounded once to float.
struct WCoef {
    double c64;
    double eps64;
    float c2_32;
    float eps32;
};

template <typename T>
struct Weight;

template <>
struct Weight<float> {
    static __device__ __forceinline__ float of(float dv, const WCoef& c) {
        return fmaxf(__builtin_amdgcn_exp2f(c.c2_32 * (dv * dv)), FLT_MIN) + c.eps32;
    }
};

template <>
struct Weight<double> {
    static __device__ __forceinline__ double of(double dv, const WCoef& c) {
        return exp(c.c64 * (dv * dv)) + c.eps64;
    }
};

// Per right-hand-side CG state, kept on the device between launches.
enum : int {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,
    ST_MAXITER = 2,
    ST_SINGULAR = -3,
    ST_BREAKDOWN = -4,
    ST_NONFINITE = -5,
};

struct RhsState {
    double rho;       // r.z of the current residual
    double rho_prev;  // r.z before the last update of rho
    double alpha;     // rho / p.q
    double beta;      // rho / rho_prev for the next p (0 before the first pass)
    double bb;        // ||b||^2
    double thresh2;   // stop iterating when r.r <= thresh2
    double rr;        // last r.r of the CG recurrence
    double rr64;      // last float64 true residual ||b - A x||^2
    double rr_ref;    // r.r right after the last float64 residual refresh
    int iter;          // CG iterations of the current inner run
    int iter_total;    // summed over inner runs
    int status;        // ST_*
    int active;        // iterating now
    int outer_active;  // not final yet (more refinement / refresh may follow)
    int max_iter;
    int pcur;          // which p buffer (0/1) holds the current search direction
    int refreshes;     // float64 residual refreshes (mixed precision)
};

// Workspace carving helper.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// Error reporting (thread-local message).
void set_error(const std::string& msg);
rw_status hip_fail(hipError_t e, const char* what, int line);

#define RW_HIP(call)                                                       \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return ::rw::hip_fail(e_, #call, __LINE__);  \
    } while (0)

}  // namespace rw

// Opaque context.
struct rw_context {
    int device = 0;
    hipStream_t s = nullptr;
    hipEvent_t ev_begin = nullptr, ev_end = nullptr, ev_join = nullptr;
    hipEvent_t ev_loop0 = nullptr, ev_loop1 = nullptr;
    std::vector<hipEvent_t> pool;   // per-launch timing events
    void* host_pinned = nullptr;    // polling buffer
    size_t host_pinned_bytes = 0;
    void* dev_small = nullptr;      // small device scratch for tiny reductions
    size_t dev_small_bytes = 0;
};
