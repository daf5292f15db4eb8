#include <algorithm>
// Context, status strings, options, small reductions (minmax, label counts)
// and the materialised-weights kernel of librw.so.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "rw_internal.h"
#include "rw_kernels.h"

namespace rw {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

rw_status hip_fail(hipError_t e, const char* what, int line) {
    char buf[512];
    snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at line %d", int(e),
             hipGetErrorString(e), what, line);
    g_last_error = buf;
    return RW_ERR_HIP;
}

rw_status invalid(const std::string& msg) {
    g_last_error = msg;
    return RW_ERR_INVALID_ARG;
}

// ------------------------------------------------------------------ kernels

// Per-block min / max / NaN count of a volume (grid-stride).
template <typename V>
__global__ __launch_bounds__(256) void k_minmax_partial(const V* __restrict__ v, int64_t n,
                                                        double* __restrict__ part) {
    double lo = INFINITY, hi = -INFINITY, nan = 0.0;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        const double a = (double)v[i];
        if (a != a) {
            nan += 1.0;
        } else {
            lo = fmin(lo, a);
            hi = fmax(hi, a);
        }
    }
    __shared__ double s_lo[256], s_hi[256], s_nan[256];
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    s_nan[threadIdx.x] = nan;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + o]);
            s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + o]);
            s_nan[threadIdx.x] += s_nan[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = s_lo[0];
        part[3 * blockIdx.x + 1] = s_hi[0];
        part[3 * blockIdx.x + 2] = s_nan[0];
    }
}

__global__ __launch_bounds__(256) void k_minmax_final(const double* __restrict__ part, int nb,
                                                      double* __restrict__ out) {
    __shared__ double s_lo[256], s_hi[256], s_nan[256];
    double lo = INFINITY, hi = -INFINITY, nan = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        lo = fmin(lo, part[3 * b]);
        hi = fmax(hi, part[3 * b + 1]);
        nan += part[3 * b + 2];
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    s_nan[threadIdx.x] = nan;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + o]);
            s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + o]);
            s_nan[threadIdx.x] += s_nan[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s_lo[0];
        out[1] = s_hi[0];
        out[2] = s_nan[0];
    }
}

// Histogram of label values (256 bins).
__global__ __launch_bounds__(256) void k_label_counts(const uint8_t* __restrict__ lab, int64_t n,
                                                      unsigned int* __restrict__ counts) {
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x)
        atomicAdd(&h[lab[i]], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

// Materialised weights w[3][n] and (optionally) dinv.
template <typename V, typename T>
__global__ __launch_bounds__(256) void k_build_weights(const V* __restrict__ vol, Geom G, WCoef wc,
                                                       const uint8_t* __restrict__ lab,
                                                       T* __restrict__ w, T* __restrict__ dinv) {
    const int64_t i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= G.n) return;
    const int z = int(i / G.plane);
    const int64_t rem = i - z * G.plane;
    const int y = int(rem / G.nx);
    const int x = int(rem - (int64_t)y * G.nx);
    const T vc = (T)vol[i];
    const T wxp = (x + 1 < G.nx) ? Weight<T>::of(vc - (T)vol[i + 1], wc) : T(0);
    const T wyp = (y + 1 < G.ny) ? Weight<T>::of(vc - (T)vol[i + G.nx], wc) : T(0);
    const T wzp = (z + 1 < G.nz) ? Weight<T>::of(vc - (T)vol[i + G.plane], wc) : T(0);
    w[i] = wxp;
    w[G.n + i] = wyp;
    w[2 * G.n + i] = wzp;
    if (dinv) {
        const T wxm = (x > 0) ? Weight<T>::of(vc - (T)vol[i - 1], wc) : T(0);
        const T wym = (y > 0) ? Weight<T>::of(vc - (T)vol[i - G.nx], wc) : T(0);
        const T wzm = (z > 0) ? Weight<T>::of(vc - (T)vol[i - G.plane], wc) : T(0);
        // same summation order as the CG kernels
        const T d = wxm + wxp + wym + wyp + wzm + wzp;
        dinv[i] = (lab && lab[i] != 0) ? T(0) : T(1) / d;
    }
}

// ------------------------------------------------------------------ helpers

rw_status check_volume(const rw_volume* vol, bool pool) {
    if (!vol) return invalid("volume is NULL");
    if (!vol->data) return invalid("volume data is NULL");
    if (vol->dims.nx <= 0 || vol->dims.ny <= 0 || vol->dims.nz <= 0)
        return invalid("volume dimensions must be positive");
    const int64_t lim = int64_t(1) << 40;
    const rw_dims& d = vol->dims;
    const bool pool_ok = d.nx <= lim && d.ny <= lim / d.nx && d.nz <= lim / (d.nx * d.ny);
    if (pool ? !pool_ok : !dims_supported(d))
        return invalid("volume too large (sides at most 2^30, nx * ny at most 2^29, "
                       "nx * ny * nz at most 2^40 voxels)");
    if (vol->dtype != RW_DT_U16 && vol->dtype != RW_DT_F32 && vol->dtype != RW_DT_F64)
        return invalid("unknown volume dtype");
    if (!std::isfinite(vol->norm_lo) || !std::isfinite(vol->norm_hi))
        return (set_error("normalisation range is not finite"), RW_ERR_NONFINITE);
    return RW_OK;
}

bool dims_supported(rw_dims d) {
    if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0) return false;
    if (d.nx > (1 << 30) || d.ny > (1 << 30) || d.nz > (1 << 30)) return false;
    const int64_t plane = d.nx * d.ny;
    return plane <= (int64_t(1) << 29) && plane * d.nz <= (int64_t(1) << 40);
}

Geom make_geom(rw_dims d) {
    Geom G;
    G.nx = int(d.nx);
    G.ny = int(d.ny);
    G.nz = int(d.nz);
    G.plane = (int64_t)d.nx * d.ny;
    G.n = G.plane * d.nz;
    return G;
}

WCoef make_wcoef(const rw_volume* vol, double beta, double w_eps) {
    WCoef c;
    const double span = vol->norm_hi - vol->norm_lo;
    const double s = span > 0 ? 1.0 / span : 0.0;
    c.c64 = -beta * s * s;
    c.eps64 = w_eps;
    c.c2_32 = float(c.c64 * 1.4426950408889634);  // log2(e)
    c.eps32 = float(w_eps);
    return c;
}

// Join: work on ctx->s starts after `user` work; `user` waits for ctx->s.
rw_status stream_enter(rw_context* ctx, void* user) {
    RW_HIP(hipEventRecord(ctx->ev_join, (hipStream_t)user));
    RW_HIP(hipStreamWaitEvent(ctx->s, ctx->ev_join, 0));
    return RW_OK;
}

rw_status stream_leave(rw_context* ctx, void* user) {
    RW_HIP(hipEventRecord(ctx->ev_join, ctx->s));
    RW_HIP(hipStreamWaitEvent((hipStream_t)user, ctx->ev_join, 0));
    return RW_OK;
}

// Seed counts per label value, read back to the host.
rw_status label_counts(rw_context* ctx, const uint8_t* lab, int64_t n, unsigned int* host256) {
    unsigned int* d = static_cast<unsigned int*>(ctx->dev_small);
    RW_HIP(hipMemsetAsync(d, 0, 256 * sizeof(unsigned int), ctx->s));
    int nb = int(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_label_counts, dim3(nb), dim3(256), 0, ctx->s, lab, n, d);
    RW_HIP(hipGetLastError());
    RW_HIP(hipMemcpyAsync(ctx->host_pinned, d, 256 * sizeof(unsigned int), hipMemcpyDeviceToHost,
                          ctx->s));
    RW_HIP(hipStreamSynchronize(ctx->s));
    memcpy(host256, ctx->host_pinned, 256 * sizeof(unsigned int));
    return RW_OK;
}

rw_status ensure_host_pinned(rw_context* ctx, size_t bytes) {
    if (ctx->host_pinned_bytes >= bytes) return RW_OK;
    RW_HIP(hipStreamSynchronize(ctx->s));
    if (ctx->host_pinned) RW_HIP(hipHostFree(ctx->host_pinned));
    ctx->host_pinned = nullptr;
    ctx->host_pinned_bytes = 0;
    RW_HIP(hipHostMalloc(&ctx->host_pinned, bytes, hipHostMallocDefault));
    ctx->host_pinned_bytes = bytes;
    return RW_OK;
}

rw_status ensure_dev_small(rw_context* ctx, size_t bytes) {
    if (ctx->dev_small_bytes >= bytes) return RW_OK;
    RW_HIP(hipStreamSynchronize(ctx->s));
    if (ctx->dev_small) RW_HIP(hipFree(ctx->dev_small));
    ctx->dev_small = nullptr;
    ctx->dev_small_bytes = 0;
    RW_HIP(hipMalloc(&ctx->dev_small, bytes));
    ctx->dev_small_bytes = bytes;
    return RW_OK;
}

rw_status ensure_events(rw_context* ctx, size_t n) {
    while (ctx->pool.size() < n) {
        hipEvent_t e;
        RW_HIP(hipEventCreate(&e));
        ctx->pool.push_back(e);
    }
    return RW_OK;
}


// Label of the highest probability per voxel, lowest label on ties, from K
// planar probability arrays.
template <typename P>
__global__ __launch_bounds__(256) void k_argmax(const P* __restrict__ prob, int K, int64_t n,
                                                uint8_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        P best = prob[i];
        int arg = 1;
        for (int L = 2; L <= K; ++L) {
            const P v = prob[(int64_t)(L - 1) * n + i];
            if (v > best) {
                best = v;
                arg = L;
            }
        }
        out[i] = uint8_t(arg);
    }
}

}  // namespace rw

using namespace rw;

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* rw_status_string(rw_status s) {
    switch (s) {
        case RW_OK: return "RW_OK";
        case RW_NOT_CONVERGED: return "RW_NOT_CONVERGED";
        case RW_ERR_INVALID_ARG: return "RW_ERR_INVALID_ARG";
        case RW_ERR_NO_SEEDS: return "RW_ERR_NO_SEEDS";
        case RW_ERR_SINGULAR: return "RW_ERR_SINGULAR";
        case RW_ERR_BREAKDOWN: return "RW_ERR_BREAKDOWN";
        case RW_ERR_NONFINITE: return "RW_ERR_NONFINITE";
        case RW_ERR_WORKSPACE: return "RW_ERR_WORKSPACE";
        case RW_ERR_HIP: return "RW_ERR_HIP";
        case RW_ERR_UNSUPPORTED: return "RW_ERR_UNSUPPORTED";
    }
    return "unknown rw_status";
}

const char* rw_last_error(void) { return g_last_error.c_str(); }

void rw_default_options(rw_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->beta = 100.0;
    o->w_eps = 0.0;
    o->tol = 1e-6;
    o->inner_tol = 1e-3;
    o->update_delta = 0.1;
    o->refine_mode = 0;
    o->max_iter = 20000;
    o->max_refine = 5;
    o->precision = RW_PREC_FP64;
    o->solve_all_labels = 0;
    o->check_interval = 16;
    o->use_graph = 1;
    o->kernel_timing = 0;
    o->x0 = nullptr;
    o->brick_voxels = 0;
}

rw_status rw_context_create(rw_context** out) {
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    rw_context* c = new rw_context();
    RW_HIP(hipGetDevice(&c->device));
    RW_HIP(hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking));
    RW_HIP(hipEventCreate(&c->ev_begin));
    RW_HIP(hipEventCreate(&c->ev_end));
    RW_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    RW_HIP(hipEventCreate(&c->ev_loop0));
    RW_HIP(hipEventCreate(&c->ev_loop1));
    c->host_pinned_bytes = 1 << 16;
    RW_HIP(hipHostMalloc(&c->host_pinned, c->host_pinned_bytes, hipHostMallocDefault));
    c->dev_small_bytes = 1 << 20;
    RW_HIP(hipMalloc(&c->dev_small, c->dev_small_bytes));
    load_tuning();
    rw_status e = noalloc_register_device(c->device);
    if (e) {
        rw_context_destroy(c);
        return e;
    }
    *out = c;
    return RW_OK;
}

void rw_context_destroy(rw_context* c) {
    if (!c) return;
    if (c->s) (void)hipStreamSynchronize(c->s);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    if (c->ev_begin) (void)hipEventDestroy(c->ev_begin);
    if (c->ev_end) (void)hipEventDestroy(c->ev_end);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_loop0) (void)hipEventDestroy(c->ev_loop0);
    if (c->ev_loop1) (void)hipEventDestroy(c->ev_loop1);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    if (c->dev_small) (void)hipFree(c->dev_small);
    if (c->s) (void)hipStreamDestroy(c->s);
    delete c;
}

rw_status rw_minmax(rw_context* ctx, const rw_volume* vol, double* lo_hi, void* stream) {
    if (!ctx || !lo_hi) return invalid("NULL argument");
    rw_volume v = *vol;
    v.norm_lo = 0;
    v.norm_hi = 1;
    rw_status st = check_volume(&v);
    if (st) return st;
    const Geom G = make_geom(vol->dims);
    if ((st = stream_enter(ctx, stream))) return st;
    double* part = static_cast<double*>(ctx->dev_small);
    const int nb = 1024;
    if (vol->dtype == RW_DT_U16)
        hipLaunchKernelGGL(k_minmax_partial<uint16_t>, dim3(nb), dim3(256), 0, ctx->s,
                           (const uint16_t*)vol->data, G.n, part);
    else if (vol->dtype == RW_DT_F32)
        hipLaunchKernelGGL(k_minmax_partial<float>, dim3(nb), dim3(256), 0, ctx->s,
                           (const float*)vol->data, G.n, part);
    else
        hipLaunchKernelGGL(k_minmax_partial<double>, dim3(nb), dim3(256), 0, ctx->s,
                           (const double*)vol->data, G.n, part);
    RW_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(256), 0, ctx->s, part, nb, part + 3 * nb);
    RW_HIP(hipGetLastError());
    RW_HIP(hipMemcpyAsync(ctx->host_pinned, part + 3 * nb, 3 * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->s));
    RW_HIP(hipStreamSynchronize(ctx->s));
    if ((st = stream_leave(ctx, stream))) return st;
    const double* h = static_cast<const double*>(ctx->host_pinned);
    if (h[2] > 0 || !std::isfinite(h[0]) || !std::isfinite(h[1])) {
        set_error("volume holds NaN or Inf");
        return RW_ERR_NONFINITE;
    }
    lo_hi[0] = h[0];
    lo_hi[1] = h[1];
    return RW_OK;
}

rw_status rw_argmax(rw_context* ctx, const void* prob, int32_t dtype, int32_t num_labels,
                    int64_t n, uint8_t* labels_out, void* stream) {
    if (!ctx || !prob || !labels_out) return invalid("NULL argument");
    if (num_labels < 1 || num_labels > 255) return invalid("num_labels must be in [1, 255]");
    if (n < 0) return invalid("n must be >= 0");
    if (dtype != RW_DT_F32 && dtype != RW_DT_F64) return invalid("probabilities must be f32 or f64");
    if (n == 0) return RW_OK;
    rw_status st = stream_enter(ctx, stream);
    if (st) return st;
    const dim3 grid(unsigned(std::min<int64_t>((n + 255) / 256, 8192)));
    if (dtype == RW_DT_F32)
        hipLaunchKernelGGL(k_argmax<float>, grid, dim3(256), 0, ctx->s, (const float*)prob,
                           num_labels, n, labels_out);
    else
        hipLaunchKernelGGL(k_argmax<double>, grid, dim3(256), 0, ctx->s, (const double*)prob,
                           num_labels, n, labels_out);
    RW_HIP(hipGetLastError());
    return stream_leave(ctx, stream);
}

rw_status rw_build_weights(rw_context* ctx, const rw_volume* vol, double beta, double w_eps,
                           int32_t precision, void* w_out, void* dinv_out,
                           const rw_seeds* seeds, void* stream) {
    if (!ctx || !w_out) return invalid("NULL argument");
    rw_status st = check_volume(vol);
    if (st) return st;
    if (!(beta >= 0) || !std::isfinite(beta)) return invalid("beta must be finite and >= 0");
    if (precision != RW_PREC_FP64 && precision != RW_PREC_MIXED) return invalid("bad precision");
    const uint8_t* lab = seeds ? seeds->labels : nullptr;
    if (dinv_out && !lab) return invalid("dinv needs the seed labels");
    const Geom G = make_geom(vol->dims);
    const WCoef wc = make_wcoef(vol, beta, w_eps);
    if ((st = stream_enter(ctx, stream))) return st;
    const dim3 grid(unsigned((G.n + 255) / 256));
#define RW_BW(V, T)                                                                         \
    hipLaunchKernelGGL((k_build_weights<V, T>), grid, dim3(256), 0, ctx->s, (const V*)vol->data, \
                       G, wc, lab, (T*)w_out, (T*)dinv_out)
    if (precision == RW_PREC_FP64) {
        if (vol->dtype == RW_DT_U16) RW_BW(uint16_t, double);
        else if (vol->dtype == RW_DT_F32) RW_BW(float, double);
        else RW_BW(double, double);
    } else {
        if (vol->dtype == RW_DT_U16) RW_BW(uint16_t, float);
        else if (vol->dtype == RW_DT_F32) RW_BW(float, float);
        else RW_BW(double, float);
    }
#undef RW_BW
    RW_HIP(hipGetLastError());
    return stream_leave(ctx, stream);
}

}  // extern "C"
