/*
 * Reference oracle: plain, serial, FP64 CPU implementations of every result the
 * hx library computes.  TEST INFRASTRUCTURE ONLY: nothing in the product path
 * links, loads or calls this file; only tests/, the package smoke check and the
 * CPU-baseline leg of bench.py do.  It shares no code, header or constant with
 * the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so the
 * evaluation order written below is exactly what runs).
 *
 * What the paper fixes and what is a reading of it:
 *  - Sec. V-A.1 defines the benchmark stencil as the 3-point weighted sum
 *    s(x_i) = 0.5 x_{i-1} + x_i + 0.5 x_{i+1} on a vector.  The library builds
 *    the explicit heat-equation form of that 3-point stencil,
 *    u'_i = u_i + r (u_{i-1} - 2 u_i + u_{i+1}); s is exactly twice the heat
 *    step at r = 1/4, and orc_prk_stencil keeps the paper's own kernel so a
 *    test can tie the two together.
 *  - Sec. V-A.2 / Algorithm 1 partitions the vector and runs copy-in, kernel,
 *    copy-out per partition.  Partitioning, overlap, batching and temporal
 *    blocking only reorder independent work, so the oracle is the plain
 *    whole-array time-stepping loop (time outer, cells inner, ping-pong arrays).
 *  - Boundaries (the paper is silent): periodic or zero-Dirichlet in 1D,
 *    zero-Dirichlet in 2D.  The variable-coefficient form is the conservative
 *    five-point discretisation of u_t = div(kappa grad u) with h = 1, face
 *    conductivity = arithmetic mean of the two cells, and at the domain edge a
 *    face of conductivity kappa_c to a ghost value 0.
 *  - The adjoint is the plain reverse-mode derivation of that explicit scheme
 *    for the loss 0.5 ||u_T - y||^2.
 *
 * Every function returns 0 on success and -1 on a bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* 1D                                                                        */
/* ------------------------------------------------------------------------ */

/* One explicit heat step of the 3-point stencil (Sec. V-A.1 in heat form):
 * v_i = u_i + r*((u_{i-1} - 2 u_i) + u_{i+1}), evaluated left to right. */
static double heat1d_point(double ul, double uc, double ur, double r) {
    return uc + r * ((ul - 2.0 * uc) + ur);
}

/* `steps` heat steps on a periodic vector of n cells (index arithmetic mod n). */
ORC_API int orc_heat1d_periodic(const double* u0, int64_t n, double r, int64_t steps,
                                double* out) {
    if (n <= 0 || steps < 0 || !u0 || !out) return -1;
    double* a = (double*)malloc((size_t)n * sizeof(double));
    double* b = (double*)malloc((size_t)n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, u0, (size_t)n * sizeof(double));
    for (int64_t t = 0; t < steps; ++t) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t il = (i == 0) ? n - 1 : i - 1;
            int64_t ir = (i == n - 1) ? 0 : i + 1;
            b[i] = heat1d_point(a[il], a[i], a[ir], r);
        }
        double* tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, (size_t)n * sizeof(double));
    free(a); free(b);
    return 0;
}

/* `steps` heat steps on n cells whose outside neighbours are held at 0
 * (zero-Dirichlet ghost cells at i = -1 and i = n). */
ORC_API int orc_heat1d_dirichlet(const double* u0, int64_t n, double r, int64_t steps,
                                 double* out) {
    if (n <= 0 || steps < 0 || !u0 || !out) return -1;
    double* a = (double*)malloc((size_t)n * sizeof(double));
    double* b = (double*)malloc((size_t)n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, u0, (size_t)n * sizeof(double));
    for (int64_t t = 0; t < steps; ++t) {
        for (int64_t i = 0; i < n; ++i) {
            double ul = (i == 0) ? 0.0 : a[i - 1];
            double ur = (i == n - 1) ? 0.0 : a[i + 1];
            b[i] = heat1d_point(ul, a[i], ur, r);
        }
        double* tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, (size_t)n * sizeof(double));
    free(a); free(b);
    return 0;
}

/* Light-cone form used to check single outputs of very large runs: `len` cells
 * with no boundary at all.  After step t only cells [t, len-1-t] are defined, so
 * after `steps` steps out[0 .. len-2*steps) receives cells [steps, len-steps). */
ORC_API int orc_heat1d_open(const double* u, int64_t len, double r, int64_t steps,
                            double* out) {
    if (len <= 2 * steps || steps < 0 || !u || !out) return -1;
    double* a = (double*)malloc((size_t)len * sizeof(double));
    double* b = (double*)malloc((size_t)len * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, u, (size_t)len * sizeof(double));
    for (int64_t t = 1; t <= steps; ++t) {
        for (int64_t i = t; i < len - t; ++i) b[i] = heat1d_point(a[i - 1], a[i], a[i + 1], r);
        double* tmp = a; a = b; b = tmp;
    }
    for (int64_t i = steps; i < len - steps; ++i) out[i - steps] = a[i];
    free(a); free(b);
    return 0;
}

/* The paper's own benchmark kernel (Sec. V-A.1): s(x_i) = 0.5 x_{i-1} + x_i +
 * 0.5 x_{i+1}, one application on a periodic vector. */
ORC_API int orc_prk_stencil(const double* x, int64_t n, double* out) {
    if (n <= 0 || !x || !out) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t il = (i == 0) ? n - 1 : i - 1;
        int64_t ir = (i == n - 1) ? 0 : i + 1;
        out[i] = (0.5 * x[il] + x[i]) + 0.5 * x[ir];
    }
    return 0;
}

/* The partition benchmark's kernel (Sec. V-A.2): k(x_i) = sqrt(sin^2 i +
 * cos^2 i), read literally with the index i as the argument.  The input value
 * is not used by the formula. */
ORC_API int orc_partition_kernel(int64_t first_index, int64_t n, double* out) {
    if (n < 0 || !out) return -1;
    for (int64_t k = 0; k < n; ++k) {
        double i = (double)(first_index + k);
        double s = sin(i), c = cos(i);
        out[k] = sqrt(s * s + c * c);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2D constant coefficient, zero-Dirichlet                                  */
/* ------------------------------------------------------------------------ */

/* v = u + r*(((uN + uS) + (uW + uE)) - 4u) on a row-major ny x nx grid whose
 * outside ghosts are 0. */
ORC_API int orc_heat2d_dirichlet(const double* u0, int64_t ny, int64_t nx, double r,
                                 int64_t steps, double* out) {
    if (ny <= 0 || nx <= 0 || steps < 0 || !u0 || !out) return -1;
    size_t cells = (size_t)ny * (size_t)nx;
    double* a = (double*)malloc(cells * sizeof(double));
    double* b = (double*)malloc(cells * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, u0, cells * sizeof(double));
    for (int64_t t = 0; t < steps; ++t) {
        for (int64_t i = 0; i < ny; ++i) {
            for (int64_t j = 0; j < nx; ++j) {
                double c = a[i * nx + j];
                double n_ = (i > 0) ? a[(i - 1) * nx + j] : 0.0;
                double s_ = (i < ny - 1) ? a[(i + 1) * nx + j] : 0.0;
                double w_ = (j > 0) ? a[i * nx + j - 1] : 0.0;
                double e_ = (j < nx - 1) ? a[i * nx + j + 1] : 0.0;
                b[i * nx + j] = c + r * (((n_ + s_) + (w_ + e_)) - 4.0 * c);
            }
        }
        double* tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, cells * sizeof(double));
    free(a); free(b);
    return 0;
}

/* Light-cone form of orc_heat2d_dirichlet for checking one output of a large
 * grid: `w` is the m x m window (m = 2*steps + 1) of u0 whose top-left cell sits
 * at global (gi0, gj0) of a ny x nx domain; window cells outside the domain are
 * ignored and treated as the zero ghosts.  Returns the centre value after
 * `steps` steps in *centre. */
ORC_API int orc_heat2d_window(const double* w, int64_t gi0, int64_t gj0, int64_t ny,
                              int64_t nx, double r, int64_t steps, double* centre) {
    if (steps < 0 || !w || !centre) return -1;
    int64_t m = 2 * steps + 1;
    double* a = (double*)malloc((size_t)(m * m) * sizeof(double));
    double* b = (double*)malloc((size_t)(m * m) * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < m; ++j) {
            int64_t gi = gi0 + i, gj = gj0 + j;
            int inside = gi >= 0 && gi < ny && gj >= 0 && gj < nx;
            a[i * m + j] = inside ? w[i * m + j] : 0.0;
        }
    for (int64_t t = 1; t <= steps; ++t) {
        for (int64_t i = t; i < m - t; ++i)
            for (int64_t j = t; j < m - t; ++j) {
                int64_t gi = gi0 + i, gj = gj0 + j;
                int inside = gi >= 0 && gi < ny && gj >= 0 && gj < nx;
                if (!inside) { b[i * m + j] = 0.0; continue; }
                double c = a[i * m + j];
                double n_ = a[(i - 1) * m + j], s_ = a[(i + 1) * m + j];
                double w_ = a[i * m + j - 1], e_ = a[i * m + j + 1];
                b[i * m + j] = c + r * (((n_ + s_) + (w_ + e_)) - 4.0 * c);
            }
        double* tmp = a; a = b; b = tmp;
    }
    *centre = a[steps * m + steps];
    free(a); free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2D variable coefficient and its adjoint                                  */
/* ------------------------------------------------------------------------ */

/* Conductivity of the face between cell c and its neighbour in direction d of a
 * ny x nx grid (d: 0 = west, 1 = east, 2 = north, 3 = south).  Interior faces
 * take the arithmetic mean of the two cells; a face on the domain edge takes the
 * cell's own value and connects to a ghost held at 0.  Sets *nb to the
 * neighbour's flat index, or -1 for an edge face. */
static double face_kappa(const double* kappa, int64_t ny, int64_t nx, int64_t i, int64_t j,
                         int d, int64_t* nb) {
    int64_t ni = i, nj = j;
    if (d == 0) nj = j - 1;
    else if (d == 1) nj = j + 1;
    else if (d == 2) ni = i - 1;
    else ni = i + 1;
    double kc = kappa[i * nx + j];
    if (ni < 0 || ni >= ny || nj < 0 || nj >= nx) { *nb = -1; return kc; }
    *nb = ni * nx + nj;
    return 0.5 * (kc + kappa[*nb]);
}

/* One forward step v = A(kappa) u: v_c = u_c + dt * sum_f kappa_f (u_n(f) - u_c),
 * faces taken in the order west, east, north, south. */
ORC_API int orc_heatvc_step(const double* u, const double* kappa, int64_t ny, int64_t nx,
                            double dt, double* v) {
    if (ny <= 0 || nx <= 0 || !u || !kappa || !v) return -1;
    for (int64_t i = 0; i < ny; ++i)
        for (int64_t j = 0; j < nx; ++j) {
            int64_t c = i * nx + j;
            double acc = 0.0;
            for (int d = 0; d < 4; ++d) {
                int64_t nb;
                double kf = face_kappa(kappa, ny, nx, i, j, d, &nb);
                double un = (nb >= 0) ? u[nb] : 0.0;
                acc = acc + kf * (un - u[c]);
            }
            v[c] = u[c] + dt * acc;
        }
    return 0;
}

/* `steps` forward steps from u0. */
ORC_API int orc_heatvc_forward(const double* u0, const double* kappa, int64_t ny, int64_t nx,
                               double dt, int64_t steps, double* out) {
    if (ny <= 0 || nx <= 0 || steps < 0 || !u0 || !kappa || !out) return -1;
    size_t cells = (size_t)ny * (size_t)nx;
    double* a = (double*)malloc(cells * sizeof(double));
    double* b = (double*)malloc(cells * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, u0, cells * sizeof(double));
    for (int64_t t = 0; t < steps; ++t) {
        orc_heatvc_step(a, kappa, ny, nx, dt, b);
        double* tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, cells * sizeof(double));
    free(a); free(b);
    return 0;
}

/* One transposed step lam_out = A(kappa)^T lam_in, written as the scatter of
 * the forward matrix's columns (it does not assume A is symmetric): every cell
 * m adds A[m][m] lam_m to itself and A[m][n] lam_m = dt kappa_f lam_m to each
 * interior neighbour n. */
ORC_API int orc_heatvc_step_transpose(const double* lam_in, const double* kappa, int64_t ny,
                                      int64_t nx, double dt, double* lam_out) {
    if (ny <= 0 || nx <= 0 || !lam_in || !kappa || !lam_out) return -1;
    size_t cells = (size_t)ny * (size_t)nx;
    for (size_t c = 0; c < cells; ++c) lam_out[c] = 0.0;
    for (int64_t i = 0; i < ny; ++i)
        for (int64_t j = 0; j < nx; ++j) {
            int64_t m = i * nx + j;
            double diag = 1.0;
            for (int d = 0; d < 4; ++d) {
                int64_t nb;
                double kf = face_kappa(kappa, ny, nx, i, j, d, &nb);
                diag = diag - dt * kf;
                /* Row m of A holds dt*kf in column nb: its transpose sends
                 * lam_m to cell nb. */
                if (nb >= 0) lam_out[nb] = lam_out[nb] + (dt * kf) * lam_in[m];
            }
            lam_out[m] = lam_out[m] + diag * lam_in[m];
        }
    return 0;
}

/* Accumulate the conductivity gradient of one step into gk:
 * lam_next^T (dA/dkappa_c) u_t for every cell c.  An interior face f between
 * cells a and b with kappa_f = (kappa_a + kappa_b)/2 contributes
 * -dt/2 (u_b - u_a)(lam_b - lam_a) to both cells; an edge face of cell c
 * contributes -dt u_c lam_c. */
ORC_API int orc_heatvc_grad_kappa_step(const double* u_t, const double* lam_next, int64_t ny,
                                       int64_t nx, double dt, double* gk) {
    if (ny <= 0 || nx <= 0 || !u_t || !lam_next || !gk) return -1;
    for (int64_t i = 0; i < ny; ++i)
        for (int64_t j = 0; j < nx; ++j) {
            int64_t c = i * nx + j;
            double acc = 0.0;
            /* faces in the order west, east, north, south */
            int64_t nbs[4] = {
                (j > 0) ? c - 1 : -1,
                (j < nx - 1) ? c + 1 : -1,
                (i > 0) ? c - nx : -1,
                (i < ny - 1) ? c + nx : -1,
            };
            for (int d = 0; d < 4; ++d) {
                int64_t nb = nbs[d];
                if (nb >= 0)
                    acc = acc + 0.5 * ((u_t[nb] - u_t[c]) * (lam_next[nb] - lam_next[c]));
                else
                    acc = acc + u_t[c] * lam_next[c];
            }
            gk[c] = gk[c] - dt * acc;
        }
    return 0;
}

/* Loss 0.5 ||u - y||^2, summed sequentially in index order. */
ORC_API double orc_loss(const double* u, const double* y, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = u[i] - y[i];
        s = s + d * d;
    }
    return 0.5 * s;
}

/* Inner product, summed sequentially in index order. */
ORC_API double orc_dot(const double* a, const double* b, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

/* Loss and gradients of L = 0.5 ||u_T - y||^2 with u_T = A(kappa)^T u0:
 *   lam_T = u_T - y;  for t = T-1 .. 0:  gk += lam_{t+1}^T dA/dkappa u_t,
 *   lam_t = A^T lam_{t+1};  dL/du0 = lam_0.
 * ckpt = 0 keeps every state u_0..u_{T-1}.  ckpt = S > 0 keeps only u_{kS} and,
 * segment by segment from the last, recomputes the segment's states from its
 * checkpoint before sweeping it backwards; the arithmetic is the same, so both
 * modes give bit-identical results. */
ORC_API int orc_heatvc_grad(const double* u0, const double* kappa, const double* y, int64_t ny,
                            int64_t nx, double dt, int64_t steps, int64_t ckpt, double* loss,
                            double* lam0, double* gk) {
    if (ny <= 0 || nx <= 0 || steps < 0 || ckpt < 0 || !u0 || !kappa || !y || !loss || !lam0 ||
        !gk)
        return -1;
    size_t cells = (size_t)ny * (size_t)nx;
    int64_t S = (ckpt == 0) ? (steps > 0 ? steps : 1) : ckpt;
    int64_t nseg = (steps + S - 1) / S;
    if (nseg == 0) nseg = 1;
    /* checkpoints u_{kS}, k = 0..nseg-1, plus a store for one segment's states */
    double* ck = (double*)malloc((size_t)nseg * cells * sizeof(double));
    double* seg = (double*)malloc((size_t)S * cells * sizeof(double));
    double* cur = (double*)malloc(cells * sizeof(double));
    double* nxt = (double*)malloc(cells * sizeof(double));
    double* lam = (double*)malloc(cells * sizeof(double));
    double* lam2 = (double*)malloc(cells * sizeof(double));
    if (!ck || !seg || !cur || !nxt || !lam || !lam2) {
        free(ck); free(seg); free(cur); free(nxt); free(lam); free(lam2);
        return -1;
    }
    /* forward sweep, keeping u_{kS} */
    memcpy(cur, u0, cells * sizeof(double));
    for (int64_t t = 0; t < steps; ++t) {
        if (t % S == 0) memcpy(ck + (size_t)(t / S) * cells, cur, cells * sizeof(double));
        orc_heatvc_step(cur, kappa, ny, nx, dt, nxt);
        double* tmp = cur; cur = nxt; nxt = tmp;
    }
    if (steps == 0) memcpy(ck, cur, cells * sizeof(double));
    *loss = orc_loss(cur, y, (int64_t)cells);
    for (size_t c = 0; c < cells; ++c) lam[c] = cur[c] - y[c];
    for (size_t c = 0; c < cells; ++c) gk[c] = 0.0;
    /* backward sweep, one segment at a time from the last */
    for (int64_t k = nseg - 1; k >= 0 && steps > 0; --k) {
        int64_t t0 = k * S;
        int64_t t1 = (t0 + S < steps) ? t0 + S : steps;
        memcpy(seg, ck + (size_t)k * cells, cells * sizeof(double));
        for (int64_t t = t0 + 1; t < t1; ++t)
            orc_heatvc_step(seg + (size_t)(t - t0 - 1) * cells, kappa, ny, nx, dt,
                            seg + (size_t)(t - t0) * cells);
        for (int64_t t = t1 - 1; t >= t0; --t) {
            const double* ut = seg + (size_t)(t - t0) * cells;
            orc_heatvc_grad_kappa_step(ut, lam, ny, nx, dt, gk);
            orc_heatvc_step_transpose(lam, kappa, ny, nx, dt, lam2);
            double* tmp = lam; lam = lam2; lam2 = tmp;
        }
    }
    memcpy(lam0, lam, cells * sizeof(double));
    free(ck); free(seg); free(cur); free(nxt); free(lam); free(lam2);
    return 0;
}
