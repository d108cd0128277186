/*
 * CPU FP64 oracle: Lorenz-96 model, its RK4 integration, and the tangent-linear
 * (TL) and adjoint (AD) of that integration about a stored trajectory.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the HIP
 * library is checked against.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source with the library.
 *
 * Arithmetic: IEEE binary64, compiled with -ffp-contract=off so that every
 * product and sum is rounded as written.  The nonlinear model is written in a
 * fixed evaluation order (stated at each function) so that a second, independent
 * implementation that keeps the same order reproduces the trajectory bit for bit.
 *
 * Indexing: states are 0-based and cyclic (index taken mod n), which is the
 * paper's 1-based convention X^(0) = X^(n), X^(-1) = X^(n-1), X^(n+1) = X^(1)
 * of the Lorenz-96 equation in the numerical-experiments section.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;       /* state size */
    int32_t nsteps;  /* window length N (RK4 steps) */
    double F;        /* forcing */
    double dt;       /* RK4 time step */
    int32_t obs_dt;  /* observation times s = obs_dt, 2 obs_dt, ..., <= N (time 0 excluded) */
    int32_t obs_dx;  /* observed variables i = obs_x0, obs_x0 + obs_dx, ... < n */
    int32_t obs_x0;
    double sigma_o;  /* R = sigma_o^2 I */
} orc_model;

static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

static int n_obs_times(const orc_model *m) { return m->nsteps / m->obs_dt; }
static int n_obs_vars(const orc_model *m) {
    return m->obs_x0 >= m->n ? 0 : (m->n - 1 - m->obs_x0) / m->obs_dx + 1;
}

/* Lorenz-96 tendency (numerical-experiments section, the L96 ODE):
 *   f_i = -x_{i-2} x_{i-1} + x_{i-1} x_{i+1} - x_i + F
 * evaluated as  ((x_{i+1} - x_{i-2}) * x_{i-1} - x_i) + F. */
void orc_l96_tendency(int n, double F, const double *x, double *f) {
    for (int i = 0; i < n; i++) {
        double a = x[wrap(i + 1, n)] - x[wrap(i - 2, n)];
        double t = a * x[wrap(i - 1, n)];
        t = t - x[i];
        f[i] = t + F;
    }
}

/* One classical RK4 step of length dt (numerical-experiments section):
 *   k1 = f(x), k2 = f(x + (dt/2) k1), k3 = f(x + (dt/2) k2), k4 = f(x + dt k3)
 *   x' = x + (dt/6) (((k1 + 2 k2) + 2 k3) + k4)
 * with dt/2 and dt/6 rounded once.  xout may alias x. */
void orc_rk4_step(int n, double F, double dt, const double *x, double *xout) {
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *xs = malloc(sizeof(double) * n);
    const double h = 0.5 * dt, c6 = dt / 6.0;
    orc_l96_tendency(n, F, x, k1);
    for (int i = 0; i < n; i++) xs[i] = x[i] + h * k1[i];
    orc_l96_tendency(n, F, xs, k2);
    for (int i = 0; i < n; i++) xs[i] = x[i] + h * k2[i];
    orc_l96_tendency(n, F, xs, k3);
    for (int i = 0; i < n; i++) xs[i] = x[i] + dt * k3[i];
    orc_l96_tendency(n, F, xs, k4);
    for (int i = 0; i < n; i++) {
        double s = k1[i] + 2.0 * k2[i];
        s = s + 2.0 * k3[i];
        s = s + k4[i];
        xout[i] = x[i] + c6 * s;
    }
    free(k1); free(k2); free(k3); free(k4); free(xs);
}

/* nsteps RK4 steps in place (truth spin-up). */
void orc_rk4_run(int n, double F, double dt, int nsteps, double *x) {
    for (int s = 0; s < nsteps; s++) orc_rk4_step(n, F, dt, x, x);
}

/* Stored trajectory traj[s*n + i], s = 0..N, from x0 (the linearisation
 * trajectory of one member, ensemble-formulation section). */
void orc_nl_traj(const orc_model *m, const double *x0, double *traj) {
    const int n = m->n;
    memcpy(traj, x0, sizeof(double) * n);
    for (int s = 0; s < m->nsteps; s++)
        orc_rk4_step(n, m->F, m->dt, traj + (size_t)s * n, traj + (size_t)(s + 1) * n);
}

/* Jacobian of the tendency at y applied to v:
 *   (J(y) v)_i = y_{i-1} (v_{i+1} - v_{i-2}) + (y_{i+1} - y_{i-2}) v_{i-1} - v_i */
static void jac(int n, const double *y, const double *v, double *out) {
    for (int i = 0; i < n; i++) {
        int im2 = wrap(i - 2, n), im1 = wrap(i - 1, n), ip1 = wrap(i + 1, n);
        out[i] = y[im1] * (v[ip1] - v[im2]) + (y[ip1] - y[im2]) * v[im1] - v[i];
    }
}

/* Transpose of the above applied to w (each column of J(y) scattered back):
 *   (J(y)^T w)_k = y_{k-2} w_{k-1} - y_{k+1} w_{k+2} + (y_{k+2} - y_{k-1}) w_{k+1} - w_k */
static void jac_t(int n, const double *y, const double *w, double *out) {
    for (int k = 0; k < n; k++) {
        int km2 = wrap(k - 2, n), km1 = wrap(k - 1, n), kp1 = wrap(k + 1, n), kp2 = wrap(k + 2, n);
        out[k] = y[km2] * w[km1] - y[kp1] * w[kp2] + (y[kp2] - y[km1]) * w[kp1] - w[k];
    }
}

/* RK4 stage states about x: x1 = x, x2 = x + (dt/2) f(x1), x3 = x + (dt/2) f(x2),
 * x4 = x + dt f(x3).  st holds 4 consecutive vectors of length n. */
static void stage_states(int n, double F, double dt, const double *x, double *st, double *tmp) {
    const double h = 0.5 * dt;
    memcpy(st, x, sizeof(double) * n);
    orc_l96_tendency(n, F, st, tmp);
    for (int i = 0; i < n; i++) st[n + i] = x[i] + h * tmp[i];
    orc_l96_tendency(n, F, st + n, tmp);
    for (int i = 0; i < n; i++) st[2 * n + i] = x[i] + h * tmp[i];
    orc_l96_tendency(n, F, st + 2 * n, tmp);
    for (int i = 0; i < n; i++) st[3 * n + i] = x[i] + dt * tmp[i];
}

/* TL of one RK4 step about state x (the derivative of orc_rk4_step w.r.t. x):
 *   dk1 = J(x1) dx, dk2 = J(x2)(dx + h dk1), dk3 = J(x3)(dx + h dk2),
 *   dk4 = J(x4)(dx + dt dk3),  dx' = dx + (dt/6)(dk1 + 2 dk2 + 2 dk3 + dk4).
 * dxout may alias dx. */
void orc_tl_step(int n, double F, double dt, const double *x, const double *dx, double *dxout) {
    double *st = malloc(sizeof(double) * 4 * n), *tmp = malloc(sizeof(double) * n);
    double *dk = malloc(sizeof(double) * 4 * n), *v = malloc(sizeof(double) * n);
    const double h = 0.5 * dt;
    stage_states(n, F, dt, x, st, tmp);
    jac(n, st, dx, dk);
    for (int i = 0; i < n; i++) v[i] = dx[i] + h * dk[i];
    jac(n, st + n, v, dk + n);
    for (int i = 0; i < n; i++) v[i] = dx[i] + h * dk[n + i];
    jac(n, st + 2 * n, v, dk + 2 * n);
    for (int i = 0; i < n; i++) v[i] = dx[i] + dt * dk[2 * n + i];
    jac(n, st + 3 * n, v, dk + 3 * n);
    for (int i = 0; i < n; i++)
        dxout[i] = dx[i] + dt / 6.0 * (dk[i] + 2.0 * dk[n + i] + 2.0 * dk[2 * n + i] + dk[3 * n + i]);
    free(st); free(tmp); free(dk); free(v);
}

/* AD of one RK4 step about state x: lamout = M^T lam, the exact transpose of
 * orc_tl_step (reverse-mode differentiation of its statements).  lamout may
 * alias lam. */
void orc_ad_step(int n, double F, double dt, const double *x, const double *lam, double *lamout) {
    double *st = malloc(sizeof(double) * 4 * n), *tmp = malloc(sizeof(double) * n);
    double *mu1 = malloc(sizeof(double) * n), *mu2 = malloc(sizeof(double) * n);
    double *mu3 = malloc(sizeof(double) * n), *mu4 = malloc(sizeof(double) * n);
    double *nu = malloc(sizeof(double) * n), *acc = malloc(sizeof(double) * n);
    const double h = 0.5 * dt;
    stage_states(n, F, dt, x, st, tmp);
    for (int i = 0; i < n; i++) {
        acc[i] = lam[i];
        mu1[i] = dt / 6.0 * lam[i];
        mu2[i] = dt / 3.0 * lam[i];
        mu3[i] = dt / 3.0 * lam[i];
        mu4[i] = dt / 6.0 * lam[i];
    }
    jac_t(n, st + 3 * n, mu4, nu);           /* through dk4 = J(x4)(dx + dt dk3) */
    for (int i = 0; i < n; i++) { acc[i] += nu[i]; mu3[i] += dt * nu[i]; }
    jac_t(n, st + 2 * n, mu3, nu);           /* through dk3 = J(x3)(dx + h dk2) */
    for (int i = 0; i < n; i++) { acc[i] += nu[i]; mu2[i] += h * nu[i]; }
    jac_t(n, st + n, mu2, nu);               /* through dk2 = J(x2)(dx + h dk1) */
    for (int i = 0; i < n; i++) { acc[i] += nu[i]; mu1[i] += h * nu[i]; }
    jac_t(n, st, mu1, nu);                   /* through dk1 = J(x1) dx */
    for (int i = 0; i < n; i++) lamout[i] = acc[i] + nu[i];
    free(st); free(tmp); free(mu1); free(mu2); free(mu3); free(mu4); free(nu); free(acc);
}

/* Linearised generalized observation operator G about a stored trajectory
 * (incremental 4D-Var section): dx_0 = v, dx_{s+1} = M_s dx_s, and for each
 * observation time s the observed components H dx_s are written to
 * obs[t * nv + q] (t-th observation time, q-th observed variable). */
void orc_tl_window(const orc_model *m, const double *traj, const double *v, double *obs) {
    const int n = m->n, nv = n_obs_vars(m);
    double *dx = malloc(sizeof(double) * n);
    memcpy(dx, v, sizeof(double) * n);
    for (int s = 0; s < m->nsteps; s++) {
        orc_tl_step(n, m->F, m->dt, traj + (size_t)s * n, dx, dx);
        if ((s + 1) % m->obs_dt == 0) {
            int t = (s + 1) / m->obs_dt - 1;
            for (int q = 0; q < nv; q++) obs[(size_t)t * nv + q] = dx[m->obs_x0 + q * m->obs_dx];
        }
    }
    free(dx);
}

/* Transpose G^T w: lam = 0; for s = N..1 { if s is an observation time, add
 * H^T w_s; lam = M_{s-1}^T lam }.  Returns lam at time 0. */
void orc_ad_window(const orc_model *m, const double *traj, const double *w, double *lam) {
    const int n = m->n, nv = n_obs_vars(m);
    memset(lam, 0, sizeof(double) * n);
    for (int s = m->nsteps; s >= 1; s--) {
        if (s % m->obs_dt == 0) {
            int t = s / m->obs_dt - 1;
            for (int q = 0; q < nv; q++) lam[m->obs_x0 + q * m->obs_dx] += w[(size_t)t * nv + q];
        }
        orc_ad_step(n, m->F, m->dt, traj + (size_t)(s - 1) * n, lam, lam);
    }
}

/* Batched forms: column c uses the trajectory of member[c]; trajectories are
 * stored member-major with stride (N+1)*n.  Columns are independent, so the
 * loop over them is parallel; the arithmetic per column is unchanged. */
void orc_tl_window_batch(const orc_model *m, const double *traj, int nb, const int32_t *member,
                         const double *V, double *obs) {
    const size_t ts = (size_t)(m->nsteps + 1) * m->n;
    const size_t p = (size_t)n_obs_times(m) * n_obs_vars(m);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nb; c++)
        orc_tl_window(m, traj + ts * member[c], V + (size_t)c * m->n, obs + p * c);
}

void orc_ad_window_batch(const orc_model *m, const double *traj, int nb, const int32_t *member,
                         const double *W, double *Lam) {
    const size_t ts = (size_t)(m->nsteps + 1) * m->n;
    const size_t p = (size_t)n_obs_times(m) * n_obs_vars(m);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nb; c++)
        orc_ad_window(m, traj + ts * member[c], W + p * c, Lam + (size_t)c * m->n);
}

/* Trajectories of several initial states (one per member), parallel over members. */
void orc_nl_traj_batch(const orc_model *m, int nm, const double *X0, double *traj) {
    const size_t ts = (size_t)(m->nsteps + 1) * m->n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < nm; j++) orc_nl_traj(m, X0 + (size_t)j * m->n, traj + ts * j);
}
