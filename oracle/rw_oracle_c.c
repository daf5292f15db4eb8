/* CPU oracle, C part — TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load
 * this library.  It shares no source with the GPU library.
 *
 * Random-walker combinatorial Dirichlet problem (the random-walker operator of
 * the paper's Sec. III-A; hierarchical use in Sec. IV-B) on a box of a 6-connected
 * voxel grid:
 *   w_ij = exp(-beta (g_i - g_j)^2) + w_eps           (Gaussian edge weight)
 *   for every unseeded voxel i of the box:
 *       sum_j w_ij (x_i - x_j) = 0
 *   where x_j is fixed for seeds ([label_j == s]) and for in-volume voxels
 *   outside the box (the "shell": seed value if seeded, else a given value).
 * Edges never leave the volume.  The whole volume is the box with no shell.
 *
 * Solver: Jacobi-preconditioned CG in float64, the textbook sequence
 *   r = b - A x0; z = D^-1 r; p = z; rho = r.z
 *   loop: q = A p; sigma = p.q; alpha = rho/sigma; x += alpha p; r -= alpha q;
 *         stop if ||r|| <= tol ||b||; z = D^-1 r; rho' = r.z; p = z + rho'/rho p
 * with all six weights of every box voxel precomputed (matrix-free, three
 * separate sweeps per iteration).  Sums are formed per z-plane and the planes
 * added in order, so results do not depend on the thread count.
 *
 * Status: 0 ok, 1 not converged (last iterate returned), -2 no seed reachable
 * (b == 0 is not an error: x = 0), -3 zero diagonal on an unknown, -4 CG
 * breakdown (p.q <= 0 or not finite), -1 bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t nx, ny, nz;          /* volume */
    int64_t ox, oy, oz;          /* box origin */
    int64_t sx, sy, sz;          /* box size */
} geom_t;

static inline int in_box(const geom_t* G, int64_t x, int64_t y, int64_t z) {
    return x >= G->ox && x < G->ox + G->sx && y >= G->oy && y < G->oy + G->sy &&
           z >= G->oz && z < G->oz + G->sz;
}

static inline int in_vol(const geom_t* G, int64_t x, int64_t y, int64_t z) {
    return x >= 0 && x < G->nx && y >= 0 && y < G->ny && z >= 0 && z < G->nz;
}

/* wall-clock split of the last orc_solve_box call (set-up, CG loop) */
static double g_setup_s = 0.0, g_loop_s = 0.0;

void orc_last_timing(double* setup_s, double* loop_s) {
    *setup_s = g_setup_s;
    *loop_s = g_loop_s;
}

static const int DX[6] = {+1, -1, 0, 0, 0, 0};
static const int DY[6] = {0, 0, +1, -1, 0, 0};
static const int DZ[6] = {0, 0, 0, 0, +1, -1};

/* Sum a per-plane array in plane order. */
static double ordered_sum(const double* part, int64_t n) {
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s += part[k];
    return s;
}

/* The six edge weights of every box voxel (0 where the neighbour is outside
 * the volume). */
int orc_box_weights(const double* g, const int64_t dims[3], const int64_t box[6], double beta,
                    double w_eps, int nthreads, double* w6 /* [6][sz][sy][sx] */) {
    geom_t G = {dims[0], dims[1], dims[2], box[0], box[1], box[2], box[3], box[4], box[5]};
    const int64_t nb = G.sx * G.sy * G.sz;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t lz = 0; lz < G.sz; ++lz)
        for (int64_t ly = 0; ly < G.sy; ++ly)
            for (int64_t lx = 0; lx < G.sx; ++lx) {
                const int64_t x = G.ox + lx, y = G.oy + ly, z = G.oz + lz;
                const int64_t li = (lz * G.sy + ly) * G.sx + lx;
                const double gi = g[(z * G.ny + y) * G.nx + x];
                for (int k = 0; k < 6; ++k) {
                    const int64_t xx = x + DX[k], yy = y + DY[k], zz = z + DZ[k];
                    double w = 0.0;
                    if (in_vol(&G, xx, yy, zz)) {
                        const double d = gi - g[(zz * G.ny + yy) * G.nx + xx];
                        w = exp(-beta * d * d) + w_eps;
                    }
                    w6[k * nb + li] = w;
                }
            }
    return 0;
}

/* One label on a box by Jacobi-PCG.  b is formed from the Dirichlet data
 * (seeds, shell) or, when rhs is given, taken from rhs on the unknowns (box
 * layout); arguments otherwise as for orc_solve_box below. */
static int solve_box_core(const double* g, const uint8_t* labels, const int64_t dims[3],
                          const int64_t box[6], const double* shell, const double* rhs,
                          double beta, double w_eps, int label, const double* x0, double tol,
                          int max_iter, int nthreads, double* x_out, int* iters_out,
                          double* rel_true_out) {
    geom_t G = {dims[0], dims[1], dims[2], box[0], box[1], box[2], box[3], box[4], box[5]};
    if (G.nx <= 0 || G.ny <= 0 || G.nz <= 0 || G.sx <= 0 || G.sy <= 0 || G.sz <= 0) return -1;
    if (G.ox < 0 || G.oy < 0 || G.oz < 0 || G.ox + G.sx > G.nx || G.oy + G.sy > G.ny ||
        G.oz + G.sz > G.nz)
        return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int64_t n = G.sx * G.sy * G.sz;
    const int64_t fx = G.sx + 2, fy = G.sy + 2;
    double* w6 = (double*)malloc(sizeof(double) * 6 * n);
    double* dinv = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    double* r = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    double* part = (double*)malloc(sizeof(double) * G.sz * 2);
    uint8_t* unk = (uint8_t*)malloc(n);
    int status = 0;
    const double t_start = omp_get_wtime();
    if (!w6 || !dinv || !b || !r || !z || !p || !q || !part || !unk) {
        status = -1;
        goto done;
    }
    orc_box_weights(g, dims, box, beta, w_eps, nthreads, w6);

    /* unknown mask, diagonal, right-hand side b (Dirichlet neighbours) */
    int zero_diag = 0;
#pragma omp parallel for schedule(static) reduction(| : zero_diag)
    for (int64_t lz = 0; lz < G.sz; ++lz)
        for (int64_t ly = 0; ly < G.sy; ++ly)
            for (int64_t lx = 0; lx < G.sx; ++lx) {
                const int64_t x = G.ox + lx, y = G.oy + ly, zz0 = G.oz + lz;
                const int64_t li = (lz * G.sy + ly) * G.sx + lx;
                const uint8_t lab = labels[(zz0 * G.ny + y) * G.nx + x];
                unk[li] = (lab == 0);
                double d = 0.0, bb = 0.0;
                for (int k = 0; k < 6; ++k) {
                    const double w = w6[k * n + li];
                    d += w;
                    const int64_t xx = x + DX[k], yy = y + DY[k], zz = zz0 + DZ[k];
                    if (!in_vol(&G, xx, yy, zz)) continue;
                    const uint8_t lj = labels[(zz * G.ny + yy) * G.nx + xx];
                    double m;
                    if (lj != 0) {
                        m = (lj == label) ? 1.0 : 0.0;
                    } else if (!in_box(&G, xx, yy, zz)) {
                        m = shell ? shell[((lz + 1 + DZ[k]) * fy + (ly + 1 + DY[k])) * fx +
                                          (lx + 1 + DX[k])]
                                  : 0.0;
                    } else {
                        continue; /* an unknown neighbour: part of A, not of b */
                    }
                    bb += w * m;
                }
                if (lab == 0) {
                    if (!(d > 0.0)) zero_diag = 1;
                    dinv[li] = d > 0.0 ? 1.0 / d : 0.0;
                    b[li] = rhs ? rhs[li] : bb;
                } else {
                    dinv[li] = 0.0;
                    b[li] = 0.0;
                }
            }
    if (zero_diag) {
        status = -3;
        goto done;
    }

/* q = A v over the unknowns (v is zero on seeds) */
#define APPLY_A(vin, vout)                                                                 \
    _Pragma("omp parallel for schedule(static)") for (int64_t lz = 0; lz < G.sz; ++lz) {    \
        for (int64_t ly = 0; ly < G.sy; ++ly)                                              \
            for (int64_t lx = 0; lx < G.sx; ++lx) {                                        \
                const int64_t li = (lz * G.sy + ly) * G.sx + lx;                           \
                if (!unk[li]) {                                                            \
                    (vout)[li] = 0.0;                                                      \
                    continue;                                                              \
                }                                                                          \
                double acc = 0.0, d = 0.0;                                                 \
                for (int k = 0; k < 6; ++k) {                                              \
                    const double w = w6[k * n + li];                                       \
                    d += w;                                                                \
                    const int64_t jx = lx + DX[k], jy = ly + DY[k], jz = lz + DZ[k];       \
                    if (jx < 0 || jx >= G.sx || jy < 0 || jy >= G.sy || jz < 0 ||          \
                        jz >= G.sz)                                                        \
                        continue;                                                          \
                    const int64_t lj = (jz * G.sy + jy) * G.sx + jx;                       \
                    if (unk[lj]) acc += w * (vin)[lj];                                     \
                }                                                                          \
                (vout)[li] = d * (vin)[li] - acc;                                          \
            }                                                                              \
    }

/* per-plane dot products, added in plane order */
#define DOT(a, bvec, res)                                                                  \
    do {                                                                                   \
        _Pragma("omp parallel for schedule(static)") for (int64_t lz = 0; lz < G.sz; ++lz) { \
            double s = 0.0;                                                                \
            const int64_t o = lz * G.sy * G.sx;                                            \
            for (int64_t t = 0; t < G.sy * G.sx; ++t) s += (a)[o + t] * (bvec)[o + t];     \
            part[lz] = s;                                                                  \
        }                                                                                  \
        (res) = ordered_sum(part, G.sz);                                                   \
    } while (0)

    double bnorm2;
    DOT(b, b, bnorm2);
    g_setup_s = omp_get_wtime() - t_start;
    const double t_loop = omp_get_wtime();
    const double nb = sqrt(bnorm2);
    /* x: start from x0 on the unknowns */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) x_out[i] = (unk[i] && x0) ? x0[i] : 0.0;
    int it = 0;
    if (nb == 0.0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) x_out[i] = 0.0;
    } else {
        APPLY_A(x_out, q);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        double rr;
        DOT(r, r, rr);
        if (sqrt(rr) > tol * nb) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                z[i] = dinv[i] * r[i];
                p[i] = z[i];
            }
            double rho;
            DOT(r, z, rho);
            status = 1;
            for (it = 0; it < max_iter;) {
                APPLY_A(p, q);
                double sigma;
                DOT(p, q, sigma);
                if (!(sigma > 0.0) || !isfinite(sigma)) {
                    status = -4;
                    break;
                }
                const double alpha = rho / sigma;
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) {
                    x_out[i] += alpha * p[i];
                    r[i] -= alpha * q[i];
                }
                ++it;
                DOT(r, r, rr);
                if (sqrt(rr) <= tol * nb) {
                    status = 0;
                    break;
                }
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
                double rho_new;
                DOT(r, z, rho_new);
                const double bet = rho_new / rho;
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) p[i] = z[i] + bet * p[i];
                rho = rho_new;
            }
        }
    }
    g_loop_s = omp_get_wtime() - t_loop;
    /* true relative residual */
    if (rel_true_out) {
        APPLY_A(x_out, q);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        double rr;
        DOT(r, r, rr);
        *rel_true_out = nb > 0.0 ? sqrt(rr) / nb : 0.0;
    }
    /* seeds exact */
#pragma omp parallel for schedule(static)
    for (int64_t lz = 0; lz < G.sz; ++lz)
        for (int64_t ly = 0; ly < G.sy; ++ly)
            for (int64_t lx = 0; lx < G.sx; ++lx) {
                const int64_t li = (lz * G.sy + ly) * G.sx + lx;
                if (!unk[li]) {
                    const uint8_t lab =
                        labels[((G.oz + lz) * G.ny + (G.oy + ly)) * G.nx + (G.ox + lx)];
                    x_out[li] = (lab == label) ? 1.0 : 0.0;
                }
            }
    if (iters_out) *iters_out = it;
done:
    free(w6);
    free(dinv);
    free(b);
    free(r);
    free(z);
    free(p);
    free(q);
    free(part);
    free(unk);
    return status;
}

/* Solve one label on a box.  shell: Dirichlet value of every non-seed voxel
 * of the one-voxel frame around the box, [(sz+2)][(sy+2)][(sx+2)] (frame
 * coordinates = box coordinates + 1), or NULL when the box is the volume.
 * x0: initial guess on the box (read on unknowns only) or NULL for 0.
 * x_out: box values, seeds set to [label == s]. */
int orc_solve_box(const double* g, const uint8_t* labels, const int64_t dims[3],
                  const int64_t box[6], const double* shell, double beta, double w_eps,
                  int label, const double* x0, double tol, int max_iter, int nthreads,
                  double* x_out, int* iters_out, double* rel_true_out) {
    return solve_box_core(g, labels, dims, box, shell, NULL, beta, w_eps, label, x0, tol,
                          max_iter, nthreads, x_out, iters_out, rel_true_out);
}

/* Adjoint gradient of a loss L(x) of one label's whole-volume solution
 * (the plain definition, by the chain rule through L_U x = b):
 *   adjoint system  L_U lam = dL/dx on the unknowns, lam = 0 on seeds
 *                   (L_U is symmetric, so the forward operator serves);
 *   per edge e = (i, j)  c_e = (lam_i - lam_j)(x_i - x_j) w_e, x with its
 *                   Dirichlet values on seeds;
 *   dL/dbeta = sum_e c_e (g_i - g_j)^2,
 *   dL/dg_i  = sum over the edges of i of 2 beta c_e (g_i - g_j).
 * The adjoint system is solved by the same Jacobi-PCG (x0 = 0) to `tol`.
 * x_full, dLdx: [nz][ny][nx]; lam_out, grad_g_out: [nz][ny][nx] or NULL.
 * Returns the PCG status. */
int orc_adjoint_grad(const double* g, const uint8_t* labels, const int64_t dims[3], double beta,
                     double w_eps, const double* x_full, const double* dLdx, double tol,
                     int max_iter, int nthreads, double* lam_out, double* grad_g_out,
                     double* grad_beta_out, int* iters_out) {
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    if (nx <= 0 || ny <= 0 || nz <= 0) return -1;
    const int64_t n = nx * ny * nz;
    const int64_t box[6] = {0, 0, 0, nx, ny, nz};
    double* lam = (double*)malloc(sizeof(double) * n);
    double* rhs = (double*)malloc(sizeof(double) * n);
    double* part = (double*)calloc((size_t)nz, sizeof(double));
    if (!lam || !rhs || !part) {
        free(lam);
        free(rhs);
        free(part);
        return -1;
    }
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) rhs[i] = labels[i] == 0 ? dLdx[i] : 0.0;
    /* label 0 matches no seed, so lam is 0 on every seed */
    int st = solve_box_core(g, labels, dims, box, NULL, rhs, beta, w_eps, 0, NULL, tol, max_iter,
                            nthreads, lam, iters_out, NULL);
    if (st >= 0) {
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z) {
            double sb = 0.0;
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t xx = 0; xx < nx; ++xx) {
                    const int64_t i = (z * ny + y) * nx + xx;
                    double gi_sum = 0.0;
                    for (int k = 0; k < 6; ++k) {
                        const int64_t X = xx + DX[k], Y = y + DY[k], Z = z + DZ[k];
                        if (X < 0 || X >= nx || Y < 0 || Y >= ny || Z < 0 || Z >= nz) continue;
                        const int64_t j = (Z * ny + Y) * nx + X;
                        const double dg = g[i] - g[j];
                        const double w = exp(-beta * dg * dg) + w_eps;
                        const double c = (lam[i] - lam[j]) * (x_full[i] - x_full[j]) * w;
                        gi_sum += 2.0 * beta * c * dg;
                        /* each edge once for beta: the +x, +y, +z direction */
                        if (k == 0 || k == 2 || k == 4) sb += c * dg * dg;
                    }
                    if (grad_g_out) grad_g_out[i] = gi_sum;
                }
            part[z] = sb;
        }
        if (grad_beta_out) *grad_beta_out = ordered_sum(part, nz);
        if (lam_out) memcpy(lam_out, lam, sizeof(double) * n);
    }
    free(lam);
    free(rhs);
    free(part);
    return st;
}

/* Time per PCG iteration without convergence: run exactly n_iter iterations
 * (or until breakdown) from x0 = 0.  Used for bounded CPU timing samples. */
int orc_pcg_fixed_iters(const double* g, const uint8_t* labels, const int64_t dims[3],
                        double beta, int label, int n_iter, int nthreads, double* x_out,
                        int* iters_out) {
    const int64_t box[6] = {0, 0, 0, dims[0], dims[1], dims[2]};
    double rel;
    /* tol = 0 never converges, so exactly n_iter iterations run */
    int st = orc_solve_box(g, labels, dims, box, NULL, beta, 0.0, label, NULL, 0.0, n_iter,
                           nthreads, x_out, iters_out, &rel);
    return st == 1 ? 0 : st;
}

int orc_max_threads(void) { return omp_get_max_threads(); }

/* Relative float64 residual ||b - A x|| / ||b|| of a given full-volume
 * solution x of label `label` (seeds' values in x are ignored, the Dirichlet
 * data [label_j == s] are used).  Returns -1 on a bad argument. */
double orc_residual(const double* g, const uint8_t* labels, const int64_t dims[3], double beta,
                    double w_eps, int label, const double* x, int nthreads) {
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    if (nx <= 0 || ny <= 0 || nz <= 0) return -1.0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    double* pr = (double*)calloc((size_t)nz, sizeof(double));
    double* pb = (double*)calloc((size_t)nz, sizeof(double));
    if (!pr || !pb) {
        free(pr);
        free(pb);
        return -1.0;
    }
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        double sr = 0.0, sb = 0.0;
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t xx = 0; xx < nx; ++xx) {
                const int64_t i = (z * ny + y) * nx + xx;
                if (labels[i] != 0) continue;
                double res = 0.0, bb = 0.0;
                for (int k = 0; k < 6; ++k) {
                    const int64_t X = xx + DX[k], Y = y + DY[k], Z = z + DZ[k];
                    if (X < 0 || X >= nx || Y < 0 || Y >= ny || Z < 0 || Z >= nz) continue;
                    const int64_t j = (Z * ny + Y) * nx + X;
                    const double d = g[i] - g[j];
                    const double w = exp(-beta * d * d) + w_eps;
                    double xj;
                    if (labels[j] != 0) {
                        xj = labels[j] == label ? 1.0 : 0.0;
                        bb += w * xj;
                    } else {
                        xj = x[j];
                    }
                    res += w * (xj - x[i]);
                }
                sr += res * res;
                sb += bb * bb;
            }
        pr[z] = sr;
        pb[z] = sb;
    }
    const double rr = ordered_sum(pr, nz), bbs = ordered_sum(pb, nz);
    free(pr);
    free(pb);
    return bbs > 0.0 ? sqrt(rr / bbs) : 0.0;
}
