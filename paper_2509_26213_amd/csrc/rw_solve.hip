// Whole-volume Jacobi-PCG solve of the random-walker Dirichlet problem.
//
// Each label s solves, for every unseeded voxel i,
//     sum_j w_ij (x_i - x_j) = 0,   x_j = [label_j == s] on seeds,
// (random walker; the paper cites it in Sec. III-A and benchmarks the
// hierarchical form in Sec. IV-B), by Jacobi-preconditioned CG stopped at
// ||r|| <= tol ||b||.  The operator is never stored: every pass recomputes
// the six edge weights of each voxel from the raw intensities.
//
// Two passes per CG iteration (vectors x, z = D^-1 r, p; r is never stored,
// r = d * z is rebuilt where needed):
//   pass 1:  p <- z + beta p (formed on the fly at the voxel and its six
//            neighbours, written to the other p buffer); q = A p; sum p.q
//   pass 2:  q = A p again; x += alpha p; r = d z - alpha q; z = r / d;
//            sums r.z and r.r
// Between them one-block kernels turn the per-block float64 partials into
// alpha, beta and convergence flags, in a fixed order (deterministic).
// The host only polls the flags every `check_interval` iterations.
//
// Mixed precision: the CG runs in float32 (weights, vectors) with float64
// dot products, inside float64 iterative refinement: r64 = b - A64 x64 with
// float64 weights, inner float32 solve of A32 d = r64, x64 += d.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "rw_internal.h"
#include "rw_kernels.h"

namespace rw {

// ================================================================== kernels

// Residual of the current float64 iterate (or of x = 0) and CG start.
// Per block, per label r: [r.z, r.r, r64.r64, b.b]; then the number of
// unseeded voxels with a non-positive degree and with a non-finite degree.
template <typename V, typename T, int R>
__global__ __launch_bounds__(NT) void k_residual(
    const V* __restrict__ vol, const uint8_t* __restrict__ lab, Geom G, WCoef wc, int zc,
    int lab0, const double* __restrict__ x64, T* __restrict__ zv, T* __restrict__ p0,
    T* __restrict__ p1, T* __restrict__ xi, int write, double* __restrict__ part) {
    constexpr int NQ = 4 * R + 2;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z0 = blockIdx.z * zc;
    const int z1 = min(z0 + zc, G.nz);
    const int64_t n = G.n;
    if (x < G.nx && y < G.ny) {
        for (int z = z0; z < z1; ++z) {
            const int64_t c = (int64_t)z * G.plane + (int64_t)y * G.nx + x;
            const uint8_t lc = lab[c];
            if (lc != 0) {
                if (write) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        zv[r * n + c] = T(0);
                        p0[r * n + c] = T(0);
                        p1[r * n + c] = T(0);
                        if (xi) xi[r * n + c] = T(0);
                    }
                }
                continue;
            }
            const bool has[6] = {x > 0, x + 1 < G.nx, y > 0, y + 1 < G.ny, z > 0, z + 1 < G.nz};
            const int64_t nb[6] = {c - 1, c + 1, c - G.nx, c + G.nx, c - G.plane, c + G.plane};
            const double vc = (double)vol[c];
            double w[6];
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                w[k] = has[k] ? Weight<double>::of(vc - (double)vol[nb[k]], wc) : 0.0;
                d += w[k];
            }
            float d32 = 0.f;
            if constexpr (std::is_same<T, float>::value) {
                const float vc32 = (float)vol[c];
                float w32[6];
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    w32[k] = has[k] ? Weight<float>::of(vc32 - (float)vol[nb[k]], wc) : 0.f;
                d32 = w32[0] + w32[1] + w32[2] + w32[3] + w32[4] + w32[5];
            }
            uint8_t ln[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) ln[k] = has[k] ? lab[nb[k]] : 0;
            if (!(d > 0.0)) acc[4 * R] += 1.0;
            if (!isfinite(d)) acc[4 * R + 1] += 1.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int L = lab0 + r;
                const double xc = x64 ? x64[r * n + c] : 0.0;
                double res = 0.0, b = 0.0;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    if (!has[k]) continue;
                    double xj;
                    if (ln[k] != 0) {
                        xj = (ln[k] == L) ? 1.0 : 0.0;
                        b += w[k] * xj;
                    } else {
                        xj = x64 ? x64[r * n + nb[k]] : 0.0;
                    }
                    res += w[k] * (xj - xc);
                }
                T zval;
                if constexpr (std::is_same<T, double>::value) {
                    const double dinv = 1.0 / d;
                    zval = dinv * res;
                    acc[4 * r + 0] += res * zval;
                    acc[4 * r + 1] += res * res;
                } else {
                    const float r32 = (float)res;
                    const float dinv = 1.f / d32;
                    zval = dinv * r32;
                    acc[4 * r + 0] += (double)r32 * (double)zval;
                    acc[4 * r + 1] += (double)r32 * (double)r32;
                }
                acc[4 * r + 2] += res * res;
                acc[4 * r + 3] += b * b;
                if (write) {
                    zv[r * n + c] = zval;
                    p0[r * n + c] = T(0);
                    p1[r * n + c] = T(0);
                    if (xi) xi[r * n + c] = T(0);
                }
            }
        }
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_sum_store<NQ>(acc, part + (int64_t)bid * NQ);
}

// Pass 1: p_new = z + beta p_old (at the voxel and its neighbours),
// q = A p_new, write p_new (and q when asked), partial p.q per label.
template <typename V, typename T, int R>
__global__ __launch_bounds__(NT) void k_pass1(const V* __restrict__ vol, Geom G, WCoef wc, int zc,
                                              const T* __restrict__ zv, const T* __restrict__ pold,
                                              T* __restrict__ pnew, T* __restrict__ qout,
                                              const RhsState* __restrict__ st,
                                              double* __restrict__ part) {
    bool act[R];
    T bet[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        act[r] = st[r].active != 0;
        bet[r] = (T)st[r].beta;
        any |= act[r];
    }
    if (!any) return;  // uniform over the grid
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z0 = blockIdx.z * zc;
    const int z1 = min(z0 + zc, G.nz);
    const int64_t n = G.n;
    if (x < G.nx && y < G.ny && z0 < G.nz) {
        const bool hxm = x > 0, hxp = x + 1 < G.nx, hym = y > 0, hyp = y + 1 < G.ny;
        int64_t c = (int64_t)z0 * G.plane + (int64_t)y * G.nx + x;
        T vc = (T)vol[c];
        T vm = z0 > 0 ? (T)vol[c - G.plane] : vc;
        T pc[R], pm[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pc[r] = act[r] ? zv[r * n + c] + bet[r] * pold[r * n + c] : T(0);
            pm[r] = (act[r] && z0 > 0)
                        ? zv[r * n + c - G.plane] + bet[r] * pold[r * n + c - G.plane]
                        : T(0);
        }
        for (int z = z0; z < z1; ++z) {
            const bool hzm = z > 0, hzp = z + 1 < G.nz;
            const T vp = hzp ? (T)vol[c + G.plane] : vc;
            const T wxm = hxm ? Weight<T>::of(vc - (T)vol[c - 1], wc) : T(0);
            const T wxp = hxp ? Weight<T>::of(vc - (T)vol[c + 1], wc) : T(0);
            const T wym = hym ? Weight<T>::of(vc - (T)vol[c - G.nx], wc) : T(0);
            const T wyp = hyp ? Weight<T>::of(vc - (T)vol[c + G.nx], wc) : T(0);
            const T wzm = hzm ? Weight<T>::of(vc - vm, wc) : T(0);
            const T wzp = hzp ? Weight<T>::of(vc - vp, wc) : T(0);
            const T d = wxm + wxp + wym + wyp + wzm + wzp;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!act[r]) continue;
                const T* zr = zv + r * n;
                const T* por = pold + r * n;
                const T b = bet[r];
                const T pp = hzp ? zr[c + G.plane] + b * por[c + G.plane] : T(0);
                const T pxm = hxm ? zr[c - 1] + b * por[c - 1] : T(0);
                const T pxp = hxp ? zr[c + 1] + b * por[c + 1] : T(0);
                const T pym = hym ? zr[c - G.nx] + b * por[c - G.nx] : T(0);
                const T pyp = hyp ? zr[c + G.nx] + b * por[c + G.nx] : T(0);
                const T q = d * pc[r] - (wxm * pxm + wxp * pxp + wym * pym + wyp * pyp +
                                         wzm * pm[r] + wzp * pp);
                pnew[r * n + c] = pc[r];
                if (qout) qout[r * n + c] = q;
                acc[r] += (double)pc[r] * (double)q;
                pm[r] = pc[r];
                pc[r] = pp;
            }
            vm = vc;
            vc = vp;
            c += G.plane;
        }
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_sum_store<R>(acc, part + (int64_t)bid * R);
}

// Pass 2: q = A p; x += alpha p; r = d z - alpha q; z = r / d; partial r.z, r.r.
template <typename V, typename T, int R>
__global__ __launch_bounds__(NT) void k_pass2(const V* __restrict__ vol,
                                              const uint8_t* __restrict__ lab, Geom G, WCoef wc,
                                              int zc, T* __restrict__ xv, T* __restrict__ zv,
                                              const T* __restrict__ p,
                                              const RhsState* __restrict__ st,
                                              double* __restrict__ part) {
    bool act[R];
    T alp[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        act[r] = st[r].active != 0;
        alp[r] = (T)st[r].alpha;
        any |= act[r];
    }
    if (!any) return;
    double acc[2 * R];
#pragma unroll
    for (int q = 0; q < 2 * R; ++q) acc[q] = 0.0;
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z0 = blockIdx.z * zc;
    const int z1 = min(z0 + zc, G.nz);
    const int64_t n = G.n;
    if (x < G.nx && y < G.ny && z0 < G.nz) {
        const bool hxm = x > 0, hxp = x + 1 < G.nx, hym = y > 0, hyp = y + 1 < G.ny;
        int64_t c = (int64_t)z0 * G.plane + (int64_t)y * G.nx + x;
        T vc = (T)vol[c];
        T vm = z0 > 0 ? (T)vol[c - G.plane] : vc;
        T pc[R], pm[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pc[r] = act[r] ? p[r * n + c] : T(0);
            pm[r] = (act[r] && z0 > 0) ? p[r * n + c - G.plane] : T(0);
        }
        for (int z = z0; z < z1; ++z) {
            const bool hzm = z > 0, hzp = z + 1 < G.nz;
            const T vp = hzp ? (T)vol[c + G.plane] : vc;
            T pp[R];
#pragma unroll
            for (int r = 0; r < R; ++r) pp[r] = (act[r] && hzp) ? p[r * n + c + G.plane] : T(0);
            if (lab[c] == 0) {
                const T wxm = hxm ? Weight<T>::of(vc - (T)vol[c - 1], wc) : T(0);
                const T wxp = hxp ? Weight<T>::of(vc - (T)vol[c + 1], wc) : T(0);
                const T wym = hym ? Weight<T>::of(vc - (T)vol[c - G.nx], wc) : T(0);
                const T wyp = hyp ? Weight<T>::of(vc - (T)vol[c + G.nx], wc) : T(0);
                const T wzm = hzm ? Weight<T>::of(vc - vm, wc) : T(0);
                const T wzp = hzp ? Weight<T>::of(vc - vp, wc) : T(0);
                const T d = wxm + wxp + wym + wyp + wzm + wzp;
                const T dinv = T(1) / d;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!act[r]) continue;
                    const T* pr = p + r * n;
                    const T pxm = hxm ? pr[c - 1] : T(0);
                    const T pxp = hxp ? pr[c + 1] : T(0);
                    const T pym = hym ? pr[c - G.nx] : T(0);
                    const T pyp = hyp ? pr[c + G.nx] : T(0);
                    const T q = d * pc[r] - (wxm * pxm + wxp * pxp + wym * pym + wyp * pyp +
                                             wzm * pm[r] + wzp * pp[r]);
                    xv[r * n + c] += alp[r] * pc[r];
                    const T rres = d * zv[r * n + c] - alp[r] * q;
                    const T zn = dinv * rres;
                    zv[r * n + c] = zn;
                    acc[2 * r] += (double)rres * (double)zn;
                    acc[2 * r + 1] += (double)rres * (double)rres;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                pm[r] = pc[r];
                pc[r] = pp[r];
            }
            vm = vc;
            vc = vp;
            c += G.plane;
        }
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_sum_store<2 * R>(acc, part + (int64_t)bid * (2 * R));
}

__device__ __forceinline__ bool any_active(const RhsState* st, int R) {
    bool a = false;
    for (int r = 0; r < R; ++r) a |= st[r].active != 0;
    return a;
}

// After pass 1: alpha = rho / p.q, or breakdown.
template <int R>
__global__ __launch_bounds__(256) void k_fin1(const double* __restrict__ part, int nb,
                                              RhsState* __restrict__ st) {
    if (!any_active(st, R)) return;
    __shared__ double sums[R];
    sum_partials<R>(part, nb, sums);
    const int r = threadIdx.x;
    if (r < R && st[r].active) {
        const double sigma = sums[r];
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            st[r].status = ST_BREAKDOWN;
            st[r].active = 0;
            st[r].outer_active = 0;
        } else {
            st[r].alpha = st[r].rho / sigma;
        }
    }
}

// After pass 2: convergence test, iteration cap, beta.
template <int R>
__global__ __launch_bounds__(256) void k_fin2(const double* __restrict__ part, int nb,
                                              RhsState* __restrict__ st, int mixed) {
    if (!any_active(st, R)) return;
    __shared__ double sums[2 * R];
    sum_partials<2 * R>(part, nb, sums);
    const int r = threadIdx.x;
    if (r < R && st[r].active) {
        RhsState& s = st[r];
        const double rz = sums[2 * r], rr = sums[2 * r + 1];
        s.iter += 1;
        s.iter_total += 1;
        s.rr = rr;
        if (!isfinite(rr) || !isfinite(rz)) {
            s.status = ST_NONFINITE;
            s.active = 0;
            s.outer_active = 0;
        } else if (rr <= s.thresh2) {
            s.active = 0;
            if (!mixed) s.status = ST_CONVERGED;
        } else if (s.iter >= s.max_iter) {
            s.active = 0;
            s.status = ST_MAXITER;
            s.outer_active = 0;
        } else {
            s.beta = rz / s.rho;
            s.rho = rz;
        }
    }
}

// After a residual evaluation: record ||b||, test the float64 residual, set
// up the next (inner) CG run.
template <int R>
__global__ __launch_bounds__(256) void k_fin_init(const double* __restrict__ part, int nb,
                                                  RhsState* __restrict__ st, double tol,
                                                  double eta, int first, int mixed,
                                                  int max_iter) {
    constexpr int NQ = 4 * R + 2;
    __shared__ double sums[NQ];
    sum_partials<NQ>(part, nb, sums);
    const int r = threadIdx.x;
    if (r >= R) return;
    RhsState& s = st[r];
    if (first) {
        s.bb = sums[4 * r + 3];
        s.iter_total = 0;
        s.status = ST_RUNNING;
        s.outer_active = 1;
    }
    s.rr64 = sums[4 * r + 2];
    s.iter = 0;
    s.max_iter = max_iter;
    if (s.status != ST_RUNNING || !s.outer_active) {
        s.active = 0;
        return;
    }
    if (sums[4 * R + 1] > 0) {
        s.status = ST_NONFINITE;
    } else if (sums[4 * R] > 0) {
        s.status = ST_SINGULAR;
    } else if (s.bb == 0.0 || s.rr64 <= tol * tol * s.bb) {
        s.status = ST_CONVERGED;
    }
    if (s.status != ST_RUNNING) {
        s.active = 0;
        s.outer_active = 0;
        return;
    }
    s.active = 1;
    s.rho = sums[4 * r + 0];
    s.rr = sums[4 * r + 1];
    s.beta = 0.0;
    s.alpha = 0.0;
    s.thresh2 = mixed ? eta * eta * s.rr : tol * tol * s.bb;
}

// x64 += xi on the unseeded voxels of the labels in `mask`.
template <typename T, int R>
__global__ __launch_bounds__(256) void k_update64(const uint8_t* __restrict__ lab, int64_t n,
                                                  const T* __restrict__ xi,
                                                  double* __restrict__ x64, int mask) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        if (lab[i] != 0) continue;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (mask & (1 << r)) x64[r * n + i] += (double)xi[r * n + i];
    }
}

// Probabilities of the solved labels lab0..lab0+R-1, seeds exact.
template <typename TO, int R>
__global__ __launch_bounds__(256) void k_write_labels(const uint8_t* __restrict__ lab, int64_t n,
                                                      const double* __restrict__ x64, int lab0,
                                                      TO* __restrict__ prob) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        const uint8_t lc = lab[i];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int L = lab0 + r;
            prob[(int64_t)(L - 1) * n + i] = lc ? TO(lc == L ? 1 : 0) : TO(x64[r * n + i]);
        }
    }
}

// Background label as the complement, and the argmax (lowest label on ties).
template <typename TO>
__global__ __launch_bounds__(256) void k_finish(const uint8_t* __restrict__ lab, int64_t n, int K,
                                                int complement, TO* __restrict__ prob,
                                                uint8_t* __restrict__ amax) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
        const uint8_t lc = lab[i];
        if (complement) {
            double s = 0.0;
            for (int L = 2; L <= K; ++L) s += (double)prob[(int64_t)(L - 1) * n + i];
            prob[i] = lc ? TO(lc == 1 ? 1 : 0) : TO(1.0 - s);
        }
        if (amax) {
            TO best = prob[i];
            int arg = 1;
            for (int L = 2; L <= K; ++L) {
                const TO v = prob[(int64_t)(L - 1) * n + i];
                if (v > best) {
                    best = v;
                    arg = L;
                }
            }
            amax[i] = uint8_t(arg);
        }
    }
}

// ================================================================== host

struct Launch {
    int zc;
    dim3 grid;
    dim3 block;
    int nblocks;
};

static Launch make_launch(const Geom& G, int zc) {
    Launch L;
    L.zc = zc;
    L.block = dim3(BX, BY, 1);
    L.grid = dim3(unsigned((G.nx + BX - 1) / BX), unsigned((G.ny + BY - 1) / BY),
                  unsigned((G.nz + zc - 1) / zc));
    L.nblocks = int(L.grid.x * L.grid.y * L.grid.z);
    return L;
}

// z extent walked by one thread: long enough to amortise the z-queue warm-up,
// short enough to give >= ~4 blocks per compute unit.
static int choose_zc(const Geom& G) {
    const int64_t cols = (int64_t)((G.nx + BX - 1) / BX) * ((G.ny + BY - 1) / BY);
    int zc = 32;
    while (zc > 4 && cols * ((G.nz + zc - 1) / zc) < 2048) zc /= 2;
    return zc;
}

static int max_blocks(const Geom& G) {
    return make_launch(G, 4).nblocks;
}

static int grid1d(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 8192)); }

struct GroupBuffers {
    double* x64;   // [R][n] float64 iterate (the CG x itself for FP64)
    void* xi;      // [R][n] inner float32 x (mixed only)
    void* z;       // [R][n]
    void* p0;      // [R][n]
    void* p1;      // [R][n]
    double* part;  // per-block partials
    RhsState* st;  // [R]
};

static size_t carve_group(Carver& cv, const Geom& G, int R, bool mixed, GroupBuffers* b) {
    const size_t vs = mixed ? sizeof(float) : sizeof(double);
    GroupBuffers t;
    t.x64 = cv.take<double>(size_t(R) * G.n);
    t.xi = mixed ? (void*)cv.take<char>(vs * R * G.n) : nullptr;
    t.z = cv.take<char>(vs * R * G.n);
    t.p0 = cv.take<char>(vs * R * G.n);
    t.p1 = cv.take<char>(vs * R * G.n);
    t.part = cv.take<double>(size_t(max_blocks(G)) * (4 * 4 + 2));
    t.st = cv.take<RhsState>(4);
    if (b) *b = t;
    return cv.bytes();
}

struct PassTiming {
    std::vector<float> t1, t2;  // per iteration of the current inner solve
};

template <typename V, typename T, int R>
struct WholeSolve {
    rw_context* ctx;
    const V* vol;
    const uint8_t* lab;
    Geom G;
    WCoef wc;
    Launch L;
    int lab0;
    bool mixed;
    const rw_options* o;
    GroupBuffers B;
    T* xv;  // CG x
    T* zv;
    T* p[2];
    RhsState host_st[R];
    double loop_ms = 0.0;
    double pass_ms[2] = {0, 0};
    int64_t launches[2] = {0, 0};
    int64_t rhs_iters = 0;
    int refinements = 0;

    rw_status launch_iteration(int k, hipEvent_t* ev) {
        hipStream_t s = ctx->s;
        T* pold = p[k & 1];
        T* pnew = p[(k + 1) & 1];
        if (ev) RW_HIP(hipEventRecord(ev[0], s));
        hipLaunchKernelGGL((k_pass1<V, T, R>), L.grid, L.block, 0, s, vol, G, wc, L.zc, zv, pold,
                           pnew, (T*)nullptr, B.st, B.part);
        if (ev) RW_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL((k_fin1<R>), dim3(1), dim3(256), 0, s, B.part, L.nblocks, B.st);
        if (ev) RW_HIP(hipEventRecord(ev[2], s));
        hipLaunchKernelGGL((k_pass2<V, T, R>), L.grid, L.block, 0, s, vol, lab, G, wc, L.zc, xv,
                           zv, pnew, B.st, B.part);
        if (ev) RW_HIP(hipEventRecord(ev[3], s));
        hipLaunchKernelGGL((k_fin2<R>), dim3(1), dim3(256), 0, s, B.part, L.nblocks, B.st,
                           mixed ? 1 : 0);
        RW_HIP(hipGetLastError());
        return RW_OK;
    }

    rw_status read_state() {
        RW_HIP(hipMemcpyAsync(ctx->host_pinned, B.st, sizeof(RhsState) * R, hipMemcpyDeviceToHost,
                              ctx->s));
        RW_HIP(hipStreamSynchronize(ctx->s));
        memcpy(host_st, ctx->host_pinned, sizeof(RhsState) * R);
        return RW_OK;
    }

    // Float64 residual of x64 and CG start; returns after reading the state.
    rw_status residual(bool first, double eta, bool write) {
        hipStream_t s = ctx->s;
        hipLaunchKernelGGL((k_residual<V, T, R>), L.grid, L.block, 0, s, vol, lab, G, wc, L.zc,
                           lab0, B.x64, zv, p[0], p[1], mixed ? (T*)B.xi : (T*)nullptr,
                           write ? 1 : 0, B.part);
        hipLaunchKernelGGL((k_fin_init<R>), dim3(1), dim3(256), 0, s, B.part, L.nblocks, B.st,
                           o->tol, eta, first ? 1 : 0, mixed ? 1 : 0, o->max_iter);
        RW_HIP(hipGetLastError());
        return read_state();
    }

    bool any_active() const {
        for (int r = 0; r < R; ++r)
            if (host_st[r].active) return true;
        return false;
    }

    // CG iterations until every label of this group stops.
    rw_status inner() {
        hipStream_t s = ctx->s;
        int m = std::max(2, o->check_interval);
        m += m & 1;  // even: the p buffers are back in place after a block
        const bool timing = o->kernel_timing != 0;
        const bool graph = o->use_graph != 0 && !timing;
        int start_iter[R];
        bool was_active[R];
        for (int r = 0; r < R; ++r) {
            start_iter[r] = host_st[r].iter;
            was_active[r] = host_st[r].active != 0;
        }
        PassTiming pt;
        if (timing) {
            rw_status e = ensure_events(ctx, size_t(4 * m));
            if (e) return e;
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        RW_HIP(hipEventRecord(ctx->ev_loop0, s));
        int done = 0;
        rw_status err = RW_OK;
        while (true) {
            if (graph) {
                if (!ge) {
                    RW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                    for (int k = 0; k < m; ++k) {
                        err = launch_iteration(k, nullptr);
                        if (err) break;
                    }
                    hipError_t e1 = hipStreamEndCapture(s, &g);
                    if (err) return err;
                    RW_HIP(e1);
                    RW_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
                }
                RW_HIP(hipGraphLaunch(ge, s));
            } else {
                for (int k = 0; k < m; ++k) {
                    err = launch_iteration(k, timing ? &ctx->pool[4 * k] : nullptr);
                    if (err) return err;
                }
            }
            err = read_state();
            if (err) break;
            if (timing) {
                for (int k = 0; k < m; ++k) {
                    float a = 0.f, b = 0.f;
                    RW_HIP(hipEventElapsedTime(&a, ctx->pool[4 * k], ctx->pool[4 * k + 1]));
                    RW_HIP(hipEventElapsedTime(&b, ctx->pool[4 * k + 2], ctx->pool[4 * k + 3]));
                    pt.t1.push_back(a);
                    pt.t2.push_back(b);
                }
            }
            done += m;
            if (!any_active()) break;
            if (done > o->max_iter + 4 * m) {
                set_error("CG loop did not stop at max_iter");
                err = RW_ERR_HIP;
                break;
            }
        }
        RW_HIP(hipEventRecord(ctx->ev_loop1, s));
        RW_HIP(hipEventSynchronize(ctx->ev_loop1));
        float ms = 0.f;
        RW_HIP(hipEventElapsedTime(&ms, ctx->ev_loop0, ctx->ev_loop1));
        loop_ms += ms;
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (err) return err;
        // iterations in which label r was iterating: [0, iter_r - start_r)
        int it_r[R];
        int kmax = 0;
        for (int r = 0; r < R; ++r) {
            it_r[r] = was_active[r] ? host_st[r].iter - start_iter[r] : 0;
            kmax = std::max(kmax, it_r[r]);
        }
        if (timing) {
            for (int k = 0; k < kmax && k < (int)pt.t1.size(); ++k) {
                pass_ms[0] += pt.t1[k];
                pass_ms[1] += pt.t2[k];
                launches[0] += 1;
                launches[1] += 1;
            }
        }
        for (int k = 0; k < kmax; ++k)
            for (int r = 0; r < R; ++r) rhs_iters += (k < it_r[r]) ? 1 : 0;
        return RW_OK;
    }

    rw_status run(const double* x0) {
        hipStream_t s = ctx->s;
        const size_t vbytes = sizeof(double) * size_t(R) * G.n;
        if (x0)
            RW_HIP(hipMemcpyAsync(B.x64, x0, vbytes, hipMemcpyDeviceToDevice, s));
        else
            RW_HIP(hipMemsetAsync(B.x64, 0, vbytes, s));
        rw_status e;
        if (!mixed) {
            if ((e = residual(true, o->tol, true))) return e;
            if (any_active())
                if ((e = inner())) return e;
            // final float64 true residual (no vector writes)
            RhsState keep[R];
            memcpy(keep, host_st, sizeof(keep));
            if ((e = residual(false, o->tol, false))) return e;
            for (int r = 0; r < R; ++r) {
                const double rr64 = host_st[r].rr64;
                keep[r].rr64 = rr64;
            }
            memcpy(host_st, keep, sizeof(keep));
            return RW_OK;
        }
        // mixed: float64 iterative refinement around float32 CG
        for (int ref = 0;; ++ref) {
            if ((e = residual(ref == 0, ref == 0 ? o->tol : o->inner_tol, true))) return e;
            if (ref > 0) refinements += 1;
            if (!any_active()) break;
            if (ref > o->max_refine) {
                // refinement budget spent: stop with the residual just measured
                for (int r = 0; r < R; ++r)
                    if (host_st[r].outer_active && host_st[r].status == ST_RUNNING)
                        host_st[r].status = ST_MAXITER;
                break;
            }
            int mask = 0;
            for (int r = 0; r < R; ++r)
                if (host_st[r].active) mask |= 1 << r;
            if ((e = inner())) return e;
            hipLaunchKernelGGL((k_update64<T, R>), dim3(grid1d(G.n)), dim3(256), 0, s, lab, G.n,
                               (const T*)B.xi, B.x64, mask);
            RW_HIP(hipGetLastError());
        }
        return RW_OK;
    }
};

template <typename V, typename T, int R>
static rw_status run_group(rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                           const rw_options* o, int lab0, const double* x0, const GroupBuffers& B,
                           void* prob_out, rw_stats* stats, int r_base, int* worst) {
    WholeSolve<V, T, R> S;
    S.ctx = ctx;
    S.vol = static_cast<const V*>(vol->data);
    S.lab = lab;
    S.G = make_geom(vol->dims);
    S.wc = make_wcoef(vol, o->beta, o->w_eps);
    S.L = make_launch(S.G, choose_zc(S.G));
    S.lab0 = lab0;
    S.mixed = o->precision == RW_PREC_MIXED;
    S.o = o;
    S.B = B;
    S.zv = static_cast<T*>(B.z);
    S.p[0] = static_cast<T*>(B.p0);
    S.p[1] = static_cast<T*>(B.p1);
    S.xv = S.mixed ? static_cast<T*>(B.xi) : reinterpret_cast<T*>(B.x64);
    rw_status e = S.run(x0);
    if (e) return e;
    // per-label status
    for (int r = 0; r < R; ++r) {
        const RhsState& h = S.host_st[r];
        int code = RW_OK;
        switch (h.status) {
            case ST_CONVERGED: code = RW_OK; break;
            case ST_RUNNING: code = S.mixed ? RW_NOT_CONVERGED : RW_OK; break;
            case ST_MAXITER: code = RW_NOT_CONVERGED; break;
            case ST_SINGULAR: code = RW_ERR_SINGULAR; break;
            case ST_BREAKDOWN: code = RW_ERR_BREAKDOWN; break;
            default: code = RW_ERR_NONFINITE; break;
        }
        if (stats && r_base + r < RW_MAX_LABELS) {
            stats->iters[r_base + r] = h.iter_total;
            stats->label_status[r_base + r] = code;
            stats->rel_residual[r_base + r] = h.bb > 0 ? std::sqrt(h.rr64 / h.bb) : 0.0;
        }
        if (code < 0 && (*worst >= 0 || code < *worst)) *worst = code;
        if (code > 0 && *worst == RW_OK) *worst = code;
    }
    if (stats) {
        stats->loop_ms += S.loop_ms;
        stats->pass_ms[0] += S.pass_ms[0];
        stats->pass_ms[1] += S.pass_ms[1];
        stats->pass_launches[0] += S.launches[0];
        stats->pass_launches[1] += S.launches[1];
        stats->rhs_iterations += S.rhs_iters;
        stats->refinements += S.refinements;
    }
    if (*worst < 0) return RW_OK;  // caller reports, outputs untouched
    const int64_t n = S.G.n;
    if (S.mixed)
        hipLaunchKernelGGL((k_write_labels<float, R>), dim3(grid1d(n)), dim3(256), 0, ctx->s, lab,
                           n, B.x64, lab0, (float*)prob_out);
    else
        hipLaunchKernelGGL((k_write_labels<double, R>), dim3(grid1d(n)), dim3(256), 0, ctx->s,
                           lab, n, B.x64, lab0, (double*)prob_out);
    RW_HIP(hipGetLastError());
    return RW_OK;
}

template <typename V, typename T>
static rw_status dispatch_r(int R, rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                            const rw_options* o, int lab0, const double* x0,
                            const GroupBuffers& B, void* prob, rw_stats* st, int rb, int* worst) {
    switch (R) {
        case 1: return run_group<V, T, 1>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst);
        case 2: return run_group<V, T, 2>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst);
        case 3: return run_group<V, T, 3>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst);
        case 4: return run_group<V, T, 4>(ctx, vol, lab, o, lab0, x0, B, prob, st, rb, worst);
    }
    return invalid("bad group size");
}

static rw_status dispatch_group(int R, rw_context* ctx, const rw_volume* vol, const uint8_t* lab,
                                const rw_options* o, int lab0, const double* x0,
                                const GroupBuffers& B, void* prob, rw_stats* st, int rb,
                                int* worst) {
    const bool mixed = o->precision == RW_PREC_MIXED;
    switch (vol->dtype) {
        case RW_DT_U16:
            return mixed ? dispatch_r<uint16_t, float>(R, ctx, vol, lab, o, lab0, x0, B, prob, st,
                                                       rb, worst)
                         : dispatch_r<uint16_t, double>(R, ctx, vol, lab, o, lab0, x0, B, prob,
                                                        st, rb, worst);
        case RW_DT_F32:
            return mixed ? dispatch_r<float, float>(R, ctx, vol, lab, o, lab0, x0, B, prob, st, rb,
                                                    worst)
                         : dispatch_r<float, double>(R, ctx, vol, lab, o, lab0, x0, B, prob, st,
                                                     rb, worst);
        default:
            return mixed ? dispatch_r<double, float>(R, ctx, vol, lab, o, lab0, x0, B, prob, st,
                                                     rb, worst)
                         : dispatch_r<double, double>(R, ctx, vol, lab, o, lab0, x0, B, prob, st,
                                                      rb, worst);
    }
}

rw_status check_options(const rw_options* o) {
    if (!o) return invalid("options is NULL");
    if (!(o->beta >= 0) || !std::isfinite(o->beta)) return invalid("beta must be finite and >= 0");
    if (!std::isfinite(o->w_eps)) return invalid("w_eps must be finite");
    if (!(o->tol > 0) || !std::isfinite(o->tol)) return invalid("tol must be > 0");
    if (o->precision == RW_PREC_MIXED && !(o->inner_tol > 0 && o->inner_tol < 1))
        return invalid("inner_tol must be in (0, 1)");
    if (o->max_iter <= 0) return invalid("max_iter must be > 0");
    if (o->max_refine < 0) return invalid("max_refine must be >= 0");
    if (o->precision != RW_PREC_FP64 && o->precision != RW_PREC_MIXED)
        return invalid("unknown precision");
    if (o->check_interval <= 0 || o->check_interval > 1024)
        return invalid("check_interval must be in [1, 1024]");
    return RW_OK;
}

// Labels present (0..255) and their validity for a solve with K labels.
rw_status check_labels(rw_context* ctx, const uint8_t* lab, int64_t n, int K, int lab0,
                       int R_total, int64_t* unknowns) {
    unsigned int cnt[256];
    rw_status e = label_counts(ctx, lab, n, cnt);
    if (e) return e;
    for (int v = K + 1; v < 256; ++v)
        if (cnt[v]) return invalid("a seed label exceeds num_labels");
    uint64_t seeds = 0;
    for (int v = 1; v <= K; ++v) seeds += cnt[v];
    if (seeds == 0) {
        set_error("no seeds");
        return RW_ERR_NO_SEEDS;
    }
    for (int r = 0; r < R_total; ++r)
        if (cnt[lab0 + r] == 0) {
            set_error("label " + std::to_string(lab0 + r) + " has no seed");
            return RW_ERR_NO_SEEDS;
        }
    if (unknowns) *unknowns = cnt[0];
    return RW_OK;
}

template <typename V, typename T>
static rw_status apply_op(rw_context* ctx, const rw_volume* vol, const WCoef& wc, const void* p,
                          void* q, void* ws) {
    const Geom G = make_geom(vol->dims);
    const Launch L = make_launch(G, choose_zc(G));
    Carver cv(ws);
    T* pnew = cv.take<T>(size_t(G.n));
    double* part = cv.take<double>(size_t(max_blocks(G)));
    RhsState* st = cv.take<RhsState>(1);
    RhsState h;
    memset(&h, 0, sizeof(h));
    h.active = 1;
    h.beta = 0.0;
    RW_HIP(hipMemcpyAsync(st, &h, sizeof(h), hipMemcpyHostToDevice, ctx->s));
    // beta = 0: p_new = z = p; the old-p operand is p itself (multiplied by 0)
    hipLaunchKernelGGL((k_pass1<V, T, 1>), L.grid, L.block, 0, ctx->s, (const V*)vol->data, G, wc,
                       L.zc, (const T*)p, (const T*)p, pnew, (T*)q, st, part);
    RW_HIP(hipGetLastError());
    RW_HIP(hipStreamSynchronize(ctx->s));
    return RW_OK;
}

}  // namespace rw

using namespace rw;

extern "C" {

size_t rw_solve_workspace_bytes(rw_dims dims, int32_t num_labels, int32_t precision,
                                int32_t solve_all_labels) {
    if (dims.nx <= 0 || dims.ny <= 0 || dims.nz <= 0 || num_labels < 1) return 0;
    const int R_total = solve_all_labels ? num_labels : num_labels - 1;
    const int Rg = std::max(1, std::min(4, R_total));
    Carver cv(nullptr);
    return carve_group(cv, make_geom(dims), Rg, precision == RW_PREC_MIXED, nullptr);
}

rw_status rw_solve(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                   const rw_options* o, void* prob_out, uint8_t* argmax_out, void* ws,
                   size_t ws_bytes, rw_stats* stats, void* stream) {
    if (!ctx) return invalid("context is NULL");
    rw_status e = check_volume(vol);
    if (e) return e;
    if ((e = check_options(o))) return e;
    if (!seeds || !seeds->labels) return invalid("seeds are NULL");
    const int K = seeds->num_labels;
    if (K < 1 || K > RW_MAX_LABELS) return invalid("num_labels must be in [1, 16]");
    if (!prob_out) return invalid("prob_out is NULL");
    const size_t need = rw_solve_workspace_bytes(vol->dims, K, o->precision, o->solve_all_labels);
    if (!ws || ws_bytes < need) {
        set_error("workspace needs " + std::to_string(need) + " bytes");
        return RW_ERR_WORKSPACE;
    }
    if (stats) memset(stats, 0, sizeof(*stats));
    const Geom G = make_geom(vol->dims);
    const int R_total = o->solve_all_labels ? K : K - 1;
    const int lab0 = o->solve_all_labels ? 1 : 2;
    if ((e = stream_enter(ctx, stream))) return e;
    RW_HIP(hipEventRecord(ctx->ev_begin, ctx->s));
    int64_t unknowns = 0;
    if ((e = check_labels(ctx, seeds->labels, G.n, K, lab0, R_total, &unknowns))) {
        (void)stream_leave(ctx, stream);
        return e;
    }
    int worst = RW_OK;
    for (int g0 = 0; g0 < R_total; g0 += 4) {
        const int Rg = std::min(4, R_total - g0);
        Carver cv(ws);
        GroupBuffers B;
        carve_group(cv, G, Rg, o->precision == RW_PREC_MIXED, &B);
        const double* x0 = o->x0 ? static_cast<const double*>(o->x0) + (int64_t)g0 * G.n : nullptr;
        e = dispatch_group(Rg, ctx, vol, seeds->labels, o, lab0 + g0, x0, B, prob_out, stats, g0,
                           &worst);
        if (e) {
            (void)stream_leave(ctx, stream);
            return e;
        }
        if (worst < 0) break;
    }
    if (worst >= 0) {
        const int complement = o->solve_all_labels ? 0 : 1;
        if (o->precision == RW_PREC_MIXED)
            hipLaunchKernelGGL((k_finish<float>), dim3(grid1d(G.n)), dim3(256), 0, ctx->s,
                               seeds->labels, G.n, K, complement, (float*)prob_out, argmax_out);
        else
            hipLaunchKernelGGL((k_finish<double>), dim3(grid1d(G.n)), dim3(256), 0, ctx->s,
                               seeds->labels, G.n, K, complement, (double*)prob_out, argmax_out);
        RW_HIP(hipGetLastError());
    }
    RW_HIP(hipEventRecord(ctx->ev_end, ctx->s));
    RW_HIP(hipEventSynchronize(ctx->ev_end));
    if (stats) {
        float ms = 0.f;
        RW_HIP(hipEventElapsedTime(&ms, ctx->ev_begin, ctx->ev_end));
        stats->device_ms = ms;
        stats->num_solved = R_total;
        stats->unknowns = unknowns;
    }
    if ((e = stream_leave(ctx, stream))) return e;
    if (worst < 0) {
        set_error(std::string("solve failed: ") + rw_status_string((rw_status)worst));
    }
    return (rw_status)worst;
}

size_t rw_operator_workspace_bytes(rw_dims dims, int32_t precision) {
    if (dims.nx <= 0 || dims.ny <= 0 || dims.nz <= 0) return 0;
    const Geom G = make_geom(dims);
    Carver cv(nullptr);
    cv.take<char>((precision == RW_PREC_MIXED ? 4 : 8) * size_t(G.n));
    cv.take<double>(size_t(max_blocks(G)));
    cv.take<RhsState>(1);
    return cv.bytes();
}

rw_status rw_apply_operator(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                            double beta, double w_eps, int32_t precision, const void* p,
                            void* q_out, void* ws, size_t ws_bytes, void* stream) {
    (void)seeds;
    if (!ctx || !p || !q_out) return invalid("NULL argument");
    rw_status e = check_volume(vol);
    if (e) return e;
    if (!(beta >= 0) || !std::isfinite(beta)) return invalid("beta must be finite and >= 0");
    if (precision != RW_PREC_FP64 && precision != RW_PREC_MIXED) return invalid("bad precision");
    const size_t need = rw_operator_workspace_bytes(vol->dims, precision);
    if (!ws || ws_bytes < need) {
        set_error("workspace needs " + std::to_string(need) + " bytes");
        return RW_ERR_WORKSPACE;
    }
    const WCoef wc = make_wcoef(vol, beta, w_eps);
    if ((e = stream_enter(ctx, stream))) return e;
    const bool m = precision == RW_PREC_MIXED;
    switch (vol->dtype) {
        case RW_DT_U16:
            e = m ? apply_op<uint16_t, float>(ctx, vol, wc, p, q_out, ws)
                  : apply_op<uint16_t, double>(ctx, vol, wc, p, q_out, ws);
            break;
        case RW_DT_F32:
            e = m ? apply_op<float, float>(ctx, vol, wc, p, q_out, ws)
                  : apply_op<float, double>(ctx, vol, wc, p, q_out, ws);
            break;
        default:
            e = m ? apply_op<double, float>(ctx, vol, wc, p, q_out, ws)
                  : apply_op<double, double>(ctx, vol, wc, p, q_out, ws);
    }
    if (e) return e;
    return stream_leave(ctx, stream);
}

}  // extern "C"
