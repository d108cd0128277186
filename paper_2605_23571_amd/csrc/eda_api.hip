// The C ABI (include/eda.h): workspace planning, problem set-up, Hessian
// products, randomized eigendecomposition, spectral LMP and batched PCG.
// Host code only sequences kernels on the context's stream; every arithmetic
// step of the path runs in this library's HIP kernels.
#include <cmath>
#include <cstring>
#include <new>

#include "eda_internal.h"

using namespace eda;

struct eda_ctx {
    Ctx c;
};

namespace {

#define HIP_TRY(expr)                              \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return EDA_ERR_HIP;  \
    } while (0)

#define EDA_TRY(expr)               \
    do {                            \
        int r_ = (expr);            \
        if (r_ < 0) return r_;      \
    } while (0)

constexpr int HIST_CAP = 2049;  // cost history rows: iterations 0..2048

bool valid_cfg(const eda_config *c) {
    if (!c) return false;
    if (c->n < 4 || c->n > 4096) return false;
    if (c->nsteps < 1 || c->obs_dt < 1 || c->obs_dx < 1 || c->obs_x0 < 0 || c->obs_x0 >= c->n) return false;
    if (c->nsteps / c->obs_dt < 1) return false;
    if (!(c->sigma_o > 0) || !(c->sigma_b > 0) || !(c->len_b >= 2.0) || !(c->dt > 0)) return false;
    if (c->members < 1 || c->spinup < 0) return false;
    if (c->max_ell < 1 || c->max_ell > 128) return false;
    if (c->max_cols < 0) return false;
    if (c->ub_mode != EDA_UB_DENSE && c->ub_mode != EDA_UB_BANDED) return false;
    return true;
}

struct Plan {
    int n, N, L, nt, nv, p, maxc, maxl;
    int pad_l, ext_len;
    size_t off_trajx, off_ub16;
    size_t off_ubrow, off_ub, off_truth, off_spin, off_xb, off_traj, off_y, off_d, off_force, off_b, off_costc;
    size_t off_hv_v, off_hv_obs, off_hv_lam, off_zero;
    size_t off_phi, off_sy, off_sq, off_sq1, off_ss, off_small, off_eig, off_coef, off_coefu, off_info, off_splitk,
        off_lmpt;
    size_t off_x, off_r, off_z, off_pp, off_q, off_scal, off_status, off_iters, off_members, off_hist;
    size_t splitk_elems;
    size_t total;
};

Plan make_plan(const eda_config *c) {
    Plan P{};
    P.n = c->n;
    P.N = c->nsteps;
    P.L = c->members;
    P.nt = c->nsteps / c->obs_dt;
    P.nv = (c->n - 1 - c->obs_x0) / c->obs_dx + 1;
    P.p = P.nt * P.nv;
    P.maxl = c->max_ell;
    P.maxc = c->max_cols > 0 ? c->max_cols : (P.L + 1 > 2 * P.maxl ? P.L + 1 : 2 * P.maxl);
    if (P.maxc < P.L + 1) P.maxc = P.L + 1;  // set-up runs all members in one batch
    const size_t d = sizeof(double);
    const size_t n = P.n, L1 = P.L + 1, p = P.p, mc = P.maxc, ml = P.maxl;
    Layout lay;
    P.off_ubrow = lay.take(n * d);
    P.off_ub = c->ub_mode == EDA_UB_DENSE ? lay.take(n * n * d) : (size_t)-1;
    P.off_ub16 = c->ub_mode == EDA_UB_DENSE ? lay.take(n * n * sizeof(uint16_t)) : (size_t)-1;
    P.off_truth = lay.take((P.N + 1) * n * d);
    P.off_spin = lay.take(n * d);
    P.off_xb = lay.take(n * L1 * d);
    P.off_traj = lay.take(L1 * (P.N + 1) * n * d);
    {
        int pl, pr;
        tlad_pads(P.n, &pl, &pr);
        P.pad_l = pl;
        P.ext_len = ((P.n + pl + pr + 31) / 32) * 32;
    }
    P.off_trajx = lay.take(L1 * (size_t)P.N * P.ext_len * d);
    P.off_y = lay.take(p * L1 * d);
    P.off_d = lay.take(p * L1 * d);
    P.off_force = lay.take(p * L1 * d);
    P.off_b = lay.take(n * L1 * d);
    P.off_costc = lay.take(L1 * d);
    P.off_hv_v = lay.take(n * mc * d);
    P.off_hv_obs = lay.take(p * mc * d);
    P.off_hv_lam = lay.take(n * mc * d);
    P.off_zero = lay.take(mc * sizeof(int32_t));
    P.off_phi = lay.take(n * ml * d);
    P.off_sy = lay.take(n * ml * d);
    P.off_sq = lay.take(n * ml * d);
    P.off_sq1 = lay.take(n * ml * d);
    P.off_ss = lay.take(n * ml * d);
    P.off_small = lay.take(10 * ml * ml * d);
    P.off_eig = lay.take(ml * d);
    P.off_coef = lay.take(ml * d);
    P.off_coefu = lay.take(ml * d);
    P.off_info = lay.take(16 * sizeof(int32_t) + 16 * d);
    size_t sk = gemm_splitk_elems(P.maxl, P.maxl, P.n);
    size_t sk2 = gemm_splitk_elems(P.maxl, P.maxc, P.n);
    P.splitk_elems = sk > sk2 ? sk : sk2;
    P.off_splitk = lay.take((P.splitk_elems ? P.splitk_elems : 1) * d);
    P.off_lmpt = lay.take(ml * mc * d);
    P.off_x = lay.take(n * mc * d);
    P.off_r = lay.take(n * mc * d);
    P.off_z = lay.take(n * mc * d);
    P.off_pp = lay.take(n * mc * d);
    P.off_q = lay.take(n * mc * d);
    P.off_scal = lay.take(4 * mc * d);
    P.off_status = lay.take(mc * sizeof(int32_t));
    P.off_iters = lay.take(mc * sizeof(int32_t));
    P.off_members = lay.take(mc * sizeof(int32_t));
    P.off_hist = lay.take(mc * (size_t)HIST_CAP * d);
    P.total = lay.total;
    return P;
}

template <typename T>
T *at(char *ws, size_t off) {
    return reinterpret_cast<T *>(ws + off);
}

// Banded U_B taps: offsets o with r(|o|) > 2^-60 r(0), i.e. o^2 < 60 ln 2 len^2,
// clipped to one full period of the ring.
void band_taps(int n, double len_b, int &lo, int &hi) {
    const double lim = 60.0 * std::log(2.0) * len_b * len_b;
    int w = 0;
    while (w + 1 <= n / 2 && (double)(w + 1) * (w + 1) < lim) w++;
    if (2 * w + 1 >= n) {
        lo = -((n - 1) / 2);
        hi = n / 2;
    } else {
        lo = -w;
        hi = w;
    }
}

// Y = U_B X (+ Add), columns optionally masked.  lowp: the dense product runs
// with BF16 operands and FP32 accumulation (reduced-precision sketch).
int ub_apply(Ctx &c, int nb, const double *X, long long ldx, double *Y, long long ldy, const double *Add,
             long long ldadd, const int32_t *active, bool lowp = false) {
    if (c.cfg.ub_mode == EDA_UB_DENSE && lowp) {
        HIP_TRY(gemm_bf16(c.stream, c.n, nb, c.n, c.ub16, c.n, X, ldx, Y, ldy, Add, ldadd));
    } else if (c.cfg.ub_mode == EDA_UB_DENSE) {
        HIP_TRY(gemm_f64(c.stream, false, c.n, nb, c.n, c.ub, c.n, X, ldx, Y, ldy, Add, ldadd, nullptr, nullptr, 0));
    } else {
        HIP_TRY(launch_band_conv(c.stream, c.n, nb, c.band_lo, c.band_hi, c.ubrow, X, ldx, Y, ldy, Add, ldadd,
                                 active));
    }
    return EDA_OK;
}

TladArgs tlad_args(Ctx &c, int nb, const int32_t *cols, const int32_t *active) {
    TladArgs a{};
    a.n = c.n;
    a.N = c.N;
    a.nb = nb;
    a.F = c.cfg.F;
    a.dt = c.cfg.dt;
    a.h = 0.5 * c.cfg.dt;
    a.dt6 = c.cfg.dt / 6.0;
    a.dt3 = c.cfg.dt / 3.0;
    a.obs_dt = c.cfg.obs_dt;
    a.obs_dx = c.cfg.obs_dx;
    a.obs_x0 = c.cfg.obs_x0;
    a.nt = c.nt;
    a.nv = c.nv;
    a.inv_s2 = 1.0 / (c.cfg.sigma_o * c.cfg.sigma_o);
    a.trajx = c.trajx;
    a.trajx_stride = (long long)c.N * c.ext_len;
    a.ext_len = c.ext_len;
    a.pad_l = c.pad_l;
    a.col_member = cols;
    a.active = active;
    a.ubrow = c.ubrow;
    a.band_lo = c.band_lo;
    a.band_hi = c.band_hi;
    return a;
}

int run_tlad(Ctx &c, const TladArgs &a, int mode, bool fp32) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool rec = c.prof && c.in_pcg;
    if (rec) {
        if (c.ev_used + 2 > c.ev.size()) {
            for (int i = 0; i < 64; i++) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                c.ev.push_back(e);
            }
        }
        e0 = c.ev[c.ev_used];
        e1 = c.ev[c.ev_used + 1];
        c.ev_used += 2;
        HIP_TRY(hipEventRecord(e0, c.stream));
    }
    HIP_TRY(launch_tlad(c.stream, a, mode, fp32));
    if (rec) {
        HIP_TRY(hipEventRecord(e1, c.stream));
        c.prof_launches++;
    }
    return EDA_OK;
}

// Batched Hessian product.  Banded U_B: one fused launch (U_B, TL, AD, U_B,
// identity) per call; dense U_B: FP64 MFMA GEMM, TL/AD, GEMM.
int hessvec(Ctx &c, const int32_t *cols, int nb, const double *X, long long ldx, double *Y, long long ldy,
            uint32_t flags, const int32_t *active) {
    if (nb <= 0) return EDA_OK;
    const bool add = (flags & EDA_HV_ADD_IDENTITY) != 0;
    const bool fp32 = (flags & EDA_HV_MIXED) != 0;
    if (c.cfg.ub_mode == EDA_UB_BANDED) {
        TladArgs a = tlad_args(c, nb, cols, active);
        a.V = X;
        a.ldv = ldx;
        a.obs = c.hv_obs;
        a.lam = Y;
        a.ldl = ldy;
        a.add_identity = add ? 1 : 0;
        return run_tlad(c, a, TLAD_HV, fp32);
    }
    EDA_TRY(ub_apply(c, nb, X, ldx, c.hv_v, c.n, nullptr, 0, active, fp32));
    TladArgs a = tlad_args(c, nb, cols, active);
    a.V = c.hv_v;
    a.ldv = c.n;
    a.obs = c.hv_obs;
    a.lam = c.hv_lam;
    a.ldl = c.n;
    EDA_TRY(run_tlad(c, a, TLAD_RAW, fp32));
    EDA_TRY(ub_apply(c, nb, c.hv_lam, c.n, Y, ldy, add ? X : nullptr, ldx, active, fp32));
    return EDA_OK;
}

int sync_read(Ctx &c, void *dst, const void *src, size_t bytes) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    return EDA_OK;
}

// CholQR2 of Y (n x l): Q (n x l) and R_Y = R2 R1 (small slot).  A shifted
// first pass (shifted CholQR3) is used if the plain Gram matrix is not SPD.
int cholqr2(Ctx &c, int l, const double *Y, double *Q, double *R_out) {
    const size_t ls = (size_t)c.max_ell * c.max_ell;
    double *G = c.sk_small + 0 * ls, *R1 = c.sk_small + 1 * ls, *R1i = c.sk_small + 2 * ls;
    double *R2 = c.sk_small + 3 * ls, *R2i = c.sk_small + 4 * ls;
    int32_t *info = c.sk_info;
    // pass 1
    HIP_TRY(gemm_f64(c.stream, true, l, l, c.n, Y, c.n, Y, c.n, G, l, nullptr, 0, nullptr, c.splitk, c.splitk_elems));
    HIP_TRY(launch_chol_inv(c.stream, l, G, 0.0, R1, R1i, info));
    int32_t hinfo = 0;
    EDA_TRY(sync_read(c, &hinfo, info, sizeof(int32_t)));
    int passes = 2;
    if (hinfo != 0) {
        // shifted pass: s = 11 (n l + l (l + 1)) eps trace(G)
        double tr = 0.0;
        std::vector<double> hg((size_t)l * l);
        EDA_TRY(sync_read(c, hg.data(), G, sizeof(double) * l * l));
        for (int i = 0; i < l; i++) tr += hg[(size_t)i * l + i];
        const double shift = 11.0 * ((double)c.n * l + (double)l * (l + 1)) * 2.220446049250313e-16 * tr;
        HIP_TRY(launch_chol_inv(c.stream, l, G, shift, R1, R1i, info));
        EDA_TRY(sync_read(c, &hinfo, info, sizeof(int32_t)));
        if (hinfo != 0) return EDA_ERR_NOT_SPD;
        passes = 3;
    }
    HIP_TRY(gemm_f64(c.stream, false, c.n, l, l, Y, c.n, R1i, l, c.sk_q1, c.n, nullptr, 0, nullptr, nullptr, 0));
    double *Racc = c.sk_small + 5 * ls, *Rtmp = c.sk_small + 6 * ls;
    HIP_TRY(launch_copy_cols(c.stream, l, l, R1, l, Racc, l));
    const double *Qin = c.sk_q1;
    for (int pass = 2; pass <= passes; pass++) {
        double *Qout = (pass == passes) ? Q : (Qin == c.sk_q1 ? c.sk_s : c.sk_q1);
        HIP_TRY(gemm_f64(c.stream, true, l, l, c.n, Qin, c.n, Qin, c.n, G, l, nullptr, 0, nullptr, c.splitk,
                         c.splitk_elems));
        HIP_TRY(launch_chol_inv(c.stream, l, G, 0.0, R2, R2i, info));
        EDA_TRY(sync_read(c, &hinfo, info, sizeof(int32_t)));
        if (hinfo != 0) return EDA_ERR_NOT_SPD;
        HIP_TRY(gemm_f64(c.stream, false, c.n, l, l, Qin, c.n, R2i, l, Qout, c.n, nullptr, 0, nullptr, nullptr, 0));
        HIP_TRY(launch_small_gemm(c.stream, l, false, false, R2, Racc, Rtmp));
        HIP_TRY(launch_copy_cols(c.stream, l, l, Rtmp, l, Racc, l));
        Qin = Qout;
    }
    HIP_TRY(launch_copy_cols(c.stream, l, l, Racc, l, R_out, l));
    return EDA_OK;
}

}  // namespace

extern "C" {

int eda_workspace_bytes(const eda_config *cfg, size_t *bytes) {
    if (!valid_cfg(cfg) || !bytes) return EDA_ERR_INVALID_ARG;
    *bytes = make_plan(cfg).total;
    return EDA_OK;
}

int eda_normals_count(const eda_config *cfg, int64_t *count) {
    if (!valid_cfg(cfg) || !count) return EDA_ERR_INVALID_ARG;
    Plan P = make_plan(cfg);
    *count = 1 + (int64_t)(P.L + 1) * (P.n + P.p);
    return EDA_OK;
}

int eda_setup(const eda_config *cfg, const double *d_normals, void *d_ws, size_t ws_bytes, void *stream,
              eda_ctx **out) {
    if (!valid_cfg(cfg) || !d_normals || !d_ws || !out) return EDA_ERR_INVALID_ARG;
    Plan P = make_plan(cfg);
    if (ws_bytes < P.total) return EDA_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return EDA_ERR_INVALID_ARG;
    eda_ctx *h = new (std::nothrow) eda_ctx();
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    c.cfg = *cfg;
    c.n = P.n;
    c.N = P.N;
    c.L = P.L;
    c.nt = P.nt;
    c.nv = P.nv;
    c.p = P.p;
    c.max_cols = P.maxc;
    c.max_ell = P.maxl;
    c.stream = reinterpret_cast<hipStream_t>(stream);
    c.ws = static_cast<char *>(d_ws);
    c.ws_bytes = ws_bytes;
    char *w = c.ws;
    c.ubrow = at<double>(w, P.off_ubrow);
    c.ub = P.off_ub == (size_t)-1 ? nullptr : at<double>(w, P.off_ub);
    c.ub16 = P.off_ub16 == (size_t)-1 ? nullptr : at<uint16_t>(w, P.off_ub16);
    c.truth = at<double>(w, P.off_truth);
    double *spin = at<double>(w, P.off_spin);
    c.xb = at<double>(w, P.off_xb);
    c.traj = at<double>(w, P.off_traj);
    c.trajx = at<double>(w, P.off_trajx);
    c.ext_len = P.ext_len;
    c.pad_l = P.pad_l;
    c.y = at<double>(w, P.off_y);
    c.d = at<double>(w, P.off_d);
    c.forcing = at<double>(w, P.off_force);
    c.b = at<double>(w, P.off_b);
    c.costc = at<double>(w, P.off_costc);
    c.hv_v = at<double>(w, P.off_hv_v);
    c.hv_obs = at<double>(w, P.off_hv_obs);
    c.hv_lam = at<double>(w, P.off_hv_lam);
    c.zero_members = at<int32_t>(w, P.off_zero);
    c.sk_phi = at<double>(w, P.off_phi);
    c.sk_y = at<double>(w, P.off_sy);
    c.sk_q = at<double>(w, P.off_sq);
    c.sk_q1 = at<double>(w, P.off_sq1);
    c.sk_s = at<double>(w, P.off_ss);
    c.sk_small = at<double>(w, P.off_small);
    c.sk_eig = at<double>(w, P.off_eig);
    c.sk_coef = at<double>(w, P.off_coef);
    c.sk_coefu = at<double>(w, P.off_coefu);
    c.sk_info = at<int32_t>(w, P.off_info);
    c.splitk = at<double>(w, P.off_splitk);
    c.splitk_elems = P.splitk_elems;
    c.lmp_t = at<double>(w, P.off_lmpt);
    c.pc_x = at<double>(w, P.off_x);
    c.pc_r = at<double>(w, P.off_r);
    c.pc_z = at<double>(w, P.off_z);
    c.pc_p = at<double>(w, P.off_pp);
    c.pc_q = at<double>(w, P.off_q);
    c.pc_scal = at<double>(w, P.off_scal);
    c.pc_status = at<int32_t>(w, P.off_status);
    c.pc_iters = at<int32_t>(w, P.off_iters);
    c.pc_members = at<int32_t>(w, P.off_members);
    c.pc_hist = at<double>(w, P.off_hist);
    c.hist_cap = HIST_CAP;
    band_taps(c.n, cfg->len_b, c.band_lo, c.band_hi);

    auto fail = [&](int code) {
        delete h;
        return code;
    };
    hipStream_t s = c.stream;
    const int n = c.n, L = c.L, N = c.N, p = c.p;
    const double F = cfg->F, dt = cfg->dt, hh = 0.5 * dt, c6 = dt / 6.0;
    const double *z = d_normals;
    const double *xi = d_normals + 1;
    const double *eta = d_normals + 1 + (size_t)(L + 1) * n;
    if (hipMemsetAsync(c.zero_members, 0, sizeof(int32_t) * c.max_cols, s) != hipSuccess) return fail(EDA_ERR_HIP);
    // U_B
    if (launch_ub_row(s, n, cfg->sigma_b, cfg->len_b, c.ubrow) != hipSuccess) return fail(EDA_ERR_HIP);
    if (c.ub && launch_ub_fill(s, n, c.ubrow, c.ub) != hipSuccess) return fail(EDA_ERR_HIP);
    if (c.ub16 && launch_to_bf16(s, (long long)n * n, c.ub, c.ub16) != hipSuccess) return fail(EDA_ERR_HIP);
    // truth: spin-up then the window
    if (launch_spin_init(s, n, F, cfg->spin_pert_std, z, spin) != hipSuccess) return fail(EDA_ERR_HIP);
    if (cfg->spinup > 0 && launch_nl(s, n, 1, cfg->spinup, F, hh, dt, c6, spin, nullptr, spin) != hipSuccess)
        return fail(EDA_ERR_HIP);
    if (launch_nl(s, n, 1, N, F, hh, dt, c6, spin, c.truth, nullptr) != hipSuccess) return fail(EDA_ERR_HIP);
    // observations
    if (launch_obs(s, n, L, p, c.nv, cfg->obs_dt, cfg->obs_dx, cfg->obs_x0, cfg->sigma_o, c.truth, eta, c.y) !=
        hipSuccess)
        return fail(EDA_ERR_HIP);
    // backgrounds x^b_j from U_B xi_j
    if (ub_apply(c, L + 1, xi, n, c.hv_v, n, nullptr, 0, nullptr) != EDA_OK) return fail(EDA_ERR_HIP);
    if (launch_xb(s, n, L, c.truth, c.hv_v, c.xb) != hipSuccess) return fail(EDA_ERR_HIP);
    // member trajectories
    if (launch_nl(s, n, L + 1, N, F, hh, dt, c6, c.xb, c.traj, nullptr) != hipSuccess) return fail(EDA_ERR_HIP);
    if (launch_pad_traj(s, n, N, L + 1, c.traj, c.pad_l, c.ext_len, c.trajx) != hipSuccess)
        return fail(EDA_ERR_HIP);
    // innovations, forcing R^-1 d, cost constants
    if (launch_innov(s, n, N, L, p, c.nv, cfg->obs_dt, cfg->obs_dx, cfg->obs_x0, cfg->sigma_o * cfg->sigma_o, c.y,
                     c.traj, c.d, c.forcing, c.costc) != hipSuccess)
        return fail(EDA_ERR_HIP);
    // b_j = U_B^T G_j^T R^-1 d_j: AD run forced by R^-1 d_j, then U_B
    {
        std::vector<int32_t> hm(L + 1);
        for (int j = 0; j <= L; j++) hm[j] = j;
        if (hipMemcpyAsync(c.pc_members, hm.data(), sizeof(int32_t) * (L + 1), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return fail(EDA_ERR_HIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(EDA_ERR_HIP);
        TladArgs a = tlad_args(c, L + 1, c.pc_members, nullptr);
        a.force = c.forcing;
        a.lam = c.hv_lam;
        a.ldl = n;
        if (launch_tlad(s, a, TLAD_ADJ, false) != hipSuccess) return fail(EDA_ERR_HIP);
        if (ub_apply(c, L + 1, c.hv_lam, n, c.b, n, nullptr, 0, nullptr) != EDA_OK) return fail(EDA_ERR_HIP);
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(EDA_ERR_HIP);
    *out = h;
    return EDA_OK;
}

int eda_hessvec(eda_ctx *h, const int32_t *d_col_member, int32_t nb, const double *d_X, int64_t ldx, double *d_Y,
                int64_t ldy, uint32_t flags) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (nb < 0 || nb > c.max_cols || ldx < c.n || ldy < c.n) return EDA_ERR_INVALID_ARG;
    if (nb == 0) return EDA_OK;
    if (!d_col_member || !d_X || !d_Y) return EDA_ERR_INVALID_ARG;
    if (flags & ~(EDA_HV_ADD_IDENTITY | EDA_HV_MIXED)) return EDA_ERR_INVALID_ARG;
    return hessvec(c, d_col_member, nb, d_X, ldx, d_Y, ldy, flags, nullptr);
}

int eda_sketch_evd(eda_ctx *h, int32_t kind, const double *d_phi, int64_t ldphi, int32_t ell, int32_t k, int32_t q,
                   int32_t method, int32_t theta_rule, uint32_t flags, double *h_eig, double *h_theta) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (ell < 1 || ell > c.max_ell || k < 1 || k > ell || q < 1) return EDA_ERR_INVALID_ARG;
    if (method != EDA_METHOD_NYSTROM && method != EDA_METHOD_REVD) return EDA_ERR_INVALID_ARG;
    if (theta_rule < EDA_THETA_MID || theta_rule > EDA_THETA_ONE) return EDA_ERR_INVALID_ARG;
    if (flags & ~EDA_HV_MIXED) return EDA_ERR_INVALID_ARG;
    if (kind == EDA_SKETCH_RHS_DIFF) {
        if (ell > c.L) return EDA_ERR_INVALID_ARG;
    } else if (kind == EDA_SKETCH_USER || kind == EDA_SKETCH_B_PSI || kind == EDA_SKETCH_UBT_PSI) {
        if (!d_phi || ldphi < c.n) return EDA_ERR_INVALID_ARG;
    } else {
        return EDA_ERR_INVALID_ARG;
    }
    hipStream_t s = c.stream;
    const int n = c.n;
    c.have_lmp = false;
    // sketching matrix Phi
    switch (kind) {
        case EDA_SKETCH_RHS_DIFF: HIP_TRY(launch_gamma(s, n, ell, c.b, c.sk_phi)); break;
        case EDA_SKETCH_USER: HIP_TRY(launch_copy_cols(s, n, ell, d_phi, ldphi, c.sk_phi, n)); break;
        case EDA_SKETCH_UBT_PSI: EDA_TRY(ub_apply(c, ell, d_phi, ldphi, c.sk_phi, n, nullptr, 0, nullptr)); break;
        case EDA_SKETCH_B_PSI:
            EDA_TRY(ub_apply(c, ell, d_phi, ldphi, c.sk_s, n, nullptr, 0, nullptr));
            EDA_TRY(ub_apply(c, ell, c.sk_s, n, c.sk_phi, n, nullptr, 0, nullptr));
            break;
    }
    const size_t ls = (size_t)c.max_ell * c.max_ell;
    double *RY = c.sk_small + 7 * ls, *Wm = c.sk_small + 8 * ls, *Cm = c.sk_small + 9 * ls;
    double *Ci = c.sk_small + 1 * ls, *Tm = c.sk_small + 2 * ls, *Um = c.sk_small + 3 * ls;
    double *sig = c.sk_small + 4 * ls;
    double *dscal = reinterpret_cast<double *>(c.sk_info + 16);
    double nu = 0.0;
    const uint32_t hvf = flags & EDA_HV_MIXED;
    if (method == EDA_METHOD_NYSTROM) {
        EDA_TRY(hessvec(c, c.zero_members, ell, c.sk_phi, n, c.sk_y, n, hvf, nullptr));
        EDA_TRY(cholqr2(c, ell, c.sk_y, c.sk_q, RY));
        for (int pass = 2; pass <= q; pass++) {
            HIP_TRY(launch_copy_cols(s, n, ell, c.sk_q, n, c.sk_phi, n));
            EDA_TRY(hessvec(c, c.zero_members, ell, c.sk_phi, n, c.sk_y, n, hvf, nullptr));
            EDA_TRY(cholqr2(c, ell, c.sk_y, c.sk_q, RY));
        }
        // W = Phi^T Y, symmetrised; W = C^T C
        HIP_TRY(gemm_f64(s, true, ell, ell, n, c.sk_phi, n, c.sk_y, n, Wm, ell, nullptr, 0, nullptr, c.splitk,
                         c.splitk_elems));
        HIP_TRY(launch_sym(s, ell, Wm));
        HIP_TRY(launch_chol_inv(s, ell, Wm, 0.0, Cm, Ci, c.sk_info));
        int32_t hinfo = 0;
        EDA_TRY(sync_read(c, &hinfo, c.sk_info, sizeof(int32_t)));
        if (hinfo != 0) {
            // shift (Nystrom-variants appendix): Y <- Y + nu Phi, nu = eps ||Y||_F
            HIP_TRY(gemm_f64(s, true, 1, 1, n * ell, c.sk_y, n * ell, c.sk_y, n * ell, dscal, 1, nullptr, 0,
                             nullptr, c.splitk, c.splitk_elems));
            double fro2 = 0.0;
            EDA_TRY(sync_read(c, &fro2, dscal, sizeof(double)));
            nu = 2.220446049250313e-16 * std::sqrt(fro2);
            HIP_TRY(launch_axpy_cols(s, n, ell, nu, c.sk_phi, n, c.sk_y, n));
            EDA_TRY(cholqr2(c, ell, c.sk_y, c.sk_q, RY));
            HIP_TRY(gemm_f64(s, true, ell, ell, n, c.sk_phi, n, c.sk_y, n, Wm, ell, nullptr, 0, nullptr, c.splitk,
                             c.splitk_elems));
            HIP_TRY(launch_sym(s, ell, Wm));
            HIP_TRY(launch_chol_inv(s, ell, Wm, 0.0, Cm, Ci, c.sk_info));
            EDA_TRY(sync_read(c, &hinfo, c.sk_info, sizeof(int32_t)));
            if (hinfo != 0) return EDA_ERR_NOT_SPD;
        }
        // T = R_Y C^-1, SVD T = U Sigma V^T, S = Q_Y U(:, 1:k), D = Sigma^2 - nu
        HIP_TRY(launch_small_gemm(s, ell, false, false, RY, Ci, Tm));
        HIP_TRY(launch_jacobi_svd_u(s, ell, Tm, Um, sig));
        HIP_TRY(gemm_f64(s, false, n, k, ell, c.sk_q, n, Um, ell, c.sk_s, n, nullptr, 0, nullptr, nullptr, 0));
        HIP_TRY(launch_fix_signs(s, n, k, c.sk_s, n));
        HIP_TRY(launch_lmp_coef(s, k, sig, nu, 1, theta_rule, c.sk_eig, c.sk_coef, c.sk_coefu, dscal + 1));
    } else {
        // REVD: Q = orth(A Phi), T = Q^T A Q, T = V D V^T, S = Q V(:, 1:k)
        EDA_TRY(hessvec(c, c.zero_members, ell, c.sk_phi, n, c.sk_y, n, hvf, nullptr));
        EDA_TRY(cholqr2(c, ell, c.sk_y, c.sk_q, RY));
        EDA_TRY(hessvec(c, c.zero_members, ell, c.sk_q, n, c.sk_y, n, hvf, nullptr));
        HIP_TRY(gemm_f64(s, true, ell, ell, n, c.sk_q, n, c.sk_y, n, Tm, ell, nullptr, 0, nullptr, c.splitk,
                         c.splitk_elems));
        HIP_TRY(launch_sym(s, ell, Tm));
        HIP_TRY(launch_jacobi_eig(s, ell, Tm, Wm, Um, sig));
        HIP_TRY(gemm_f64(s, false, n, k, ell, c.sk_q, n, Um, ell, c.sk_s, n, nullptr, 0, nullptr, nullptr, 0));
        HIP_TRY(launch_fix_signs(s, n, k, c.sk_s, n));
        HIP_TRY(launch_lmp_coef(s, k, sig, 0.0, 0, theta_rule, c.sk_eig, c.sk_coef, c.sk_coefu, dscal + 1));
    }
    double th = 1.0;
    EDA_TRY(sync_read(c, &th, dscal + 1, sizeof(double)));
    if (h_eig) EDA_TRY(sync_read(c, h_eig, c.sk_eig, sizeof(double) * k));
    if (h_theta) *h_theta = th;
    c.theta = th;
    c.k = k;
    c.have_lmp = true;
    return EDA_OK;
}

}  // extern "C"

namespace {

// Y = X + S_k diag(coef) S_k^T X (coef: P_theta or U_theta coefficients).
int lmp_apply(Ctx &c, int which, int nb, const double *X, long long ldx, double *Y, long long ldy) {
    const double *coef = which == EDA_LMP_U ? c.sk_coefu : c.sk_coef;
    HIP_TRY(gemm_f64(c.stream, true, c.k, nb, c.n, c.sk_s, c.n, X, ldx, c.lmp_t, c.k, nullptr, 0, coef, c.splitk,
                     c.splitk_elems));
    HIP_TRY(gemm_f64(c.stream, false, c.n, nb, c.k, c.sk_s, c.n, c.lmp_t, c.k, Y, ldy, X, ldx, nullptr, nullptr, 0));
    return EDA_OK;
}

}  // namespace

extern "C" {

int eda_lmp_apply(eda_ctx *h, int32_t which, int32_t nb, const double *d_X, int64_t ldx, double *d_Y, int64_t ldy) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (which != EDA_LMP_P && which != EDA_LMP_U) return EDA_ERR_INVALID_ARG;
    if (nb < 0 || nb > c.max_cols || ldx < c.n || ldy < c.n) return EDA_ERR_INVALID_ARG;
    if (!c.have_lmp) return EDA_ERR_ORDER;
    if (nb == 0) return EDA_OK;
    if (!d_X || !d_Y) return EDA_ERR_INVALID_ARG;
    return lmp_apply(c, which, nb, d_X, ldx, d_Y, ldy);
}

int eda_pcg_solve(eda_ctx *h, const int32_t *h_members, int32_t nm, double rtol, int32_t maxit, int32_t use_lmp,
                  double *d_DZ, int64_t ldz, int32_t *h_iters, double *h_relres, int32_t *h_status,
                  double *h_cost_hist) {
    if (!h || !h_members || !d_DZ || !h_iters || !h_relres || !h_status) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (nm < 1 || nm > c.max_cols || maxit < 0 || !(rtol >= 0) || ldz < c.n) return EDA_ERR_INVALID_ARG;
    if (h_cost_hist && maxit >= c.hist_cap) return EDA_ERR_UNSUPPORTED;
    for (int i = 0; i < nm; i++)
        if (h_members[i] < 0 || h_members[i] > c.L) return EDA_ERR_INVALID_ARG;
    if (use_lmp && !c.have_lmp) return EDA_ERR_ORDER;
    hipStream_t s = c.stream;
    const int n = c.n;
    HIP_TRY(hipMemcpyAsync(c.pc_members, h_members, sizeof(int32_t) * nm, hipMemcpyHostToDevice, s));
    PcgArgs a{};
    a.n = n;
    a.nb = nm;
    a.members = c.pc_members;
    a.b = c.b;
    a.x = c.pc_x;
    a.r = c.pc_r;
    a.z = use_lmp ? c.pc_z : c.pc_r;
    a.p = c.pc_p;
    a.q = c.pc_q;
    a.scal = c.pc_scal;
    a.status = c.pc_status;
    a.iters = c.pc_iters;
    a.hist = h_cost_hist ? c.pc_hist : nullptr;
    a.hist_cap = c.hist_cap;
    a.rtol = rtol;
    HIP_TRY(launch_pcg_init(s, a));
    if (use_lmp) EDA_TRY(lmp_apply(c, EDA_LMP_P, nm, c.pc_r, n, c.pc_z, n));
    std::vector<int32_t> st(nm);
    const int check_every = 8;
    const bool fused = c.cfg.ub_mode == EDA_UB_BANDED;
    bool stopped_early = false;
    if (!fused) HIP_TRY(launch_pcg_start(s, a));
    struct InPcg {  // profile scope, also left on an error return
        Ctx &c;
        explicit InPcg(Ctx &cc) : c(cc) { c.in_pcg = true; }
        ~InPcg() { c.in_pcg = false; }
    };
    {
        InPcg scope(c);
        for (int it = 1; it <= maxit; it++) {
            if (fused) {
                // one launch: p = z + beta p, q = (I + A) p, alpha, x, r, convergence
                TladArgs t = tlad_args(c, nm, c.pc_members, nullptr);
                t.obs = c.hv_obs;
                t.pcg.members = c.pc_members;
                t.pcg.b = c.b;
                t.pcg.x = c.pc_x;
                t.pcg.r = c.pc_r;
                t.pcg.z = a.z;
                t.pcg.p = c.pc_p;
                t.pcg.scal = c.pc_scal;
                t.pcg.status = c.pc_status;
                t.pcg.iters = c.pc_iters;
                t.pcg.hist = a.hist;
                t.pcg.hist_cap = c.hist_cap;
                t.pcg.rtol = rtol;
                t.pcg.it = it;
                t.pcg.first = it == 1 ? 1 : 0;
                EDA_TRY(run_tlad(c, t, TLAD_PCG, false));
                if (use_lmp) EDA_TRY(lmp_apply(c, EDA_LMP_P, nm, c.pc_r, n, c.pc_z, n));
            } else {
                EDA_TRY(hessvec(c, c.pc_members, nm, c.pc_p, n, c.pc_q, n, EDA_HV_ADD_IDENTITY, c.pc_status));
                HIP_TRY(launch_pcg_alpha(s, a, it));
                if (use_lmp) EDA_TRY(lmp_apply(c, EDA_LMP_P, nm, c.pc_r, n, c.pc_z, n));
                HIP_TRY(launch_pcg_beta(s, a));
            }
            if (it % check_every == 0 || it == maxit) {
                EDA_TRY(sync_read(c, st.data(), c.pc_status, sizeof(int32_t) * nm));
                bool running = false;
                for (int i = 0; i < nm; i++) running |= (st[i] == COL_RUNNING);
                if (!running) {
                    stopped_early = true;
                    break;
                }
            }
        }
    }
    // the fused form tests r^T z for breakdown at the start of the next
    // iteration; after the last one that test runs here (as the textbook loop does)
    if (fused && !stopped_early && maxit > 0) HIP_TRY(launch_pcg_beta(s, a));
    HIP_TRY(launch_pcg_finish(s, a));
    HIP_TRY(launch_copy_cols(s, n, nm, c.pc_x, n, d_DZ, ldz));
    std::vector<double> scal(4 * (size_t)nm);
    EDA_TRY(sync_read(c, h_status, c.pc_status, sizeof(int32_t) * nm));
    EDA_TRY(sync_read(c, h_iters, c.pc_iters, sizeof(int32_t) * nm));
    EDA_TRY(sync_read(c, scal.data(), c.pc_scal, sizeof(double) * 4 * nm));
    int warn = EDA_OK;
    for (int i = 0; i < nm; i++) {
        h_relres[i] = scal[4 * i + 2];
        if (h_status[i] != EDA_MEMBER_CONVERGED) warn = EDA_WARN_NOT_CONVERGED;
    }
    if (h_cost_hist) {
        std::vector<double> hist((size_t)nm * c.hist_cap);
        EDA_TRY(sync_read(c, hist.data(), c.pc_hist, sizeof(double) * hist.size()));
        for (int i = 0; i < nm; i++)
            std::memcpy(h_cost_hist + (size_t)i * (maxit + 1), hist.data() + (size_t)i * c.hist_cap,
                        sizeof(double) * (maxit + 1));
    }
    return warn;
}

int eda_field(const eda_ctx *h, int32_t field, size_t *byte_offset, int64_t *count) {
    if (!h || !byte_offset || !count) return EDA_ERR_INVALID_ARG;
    const Ctx &c = h->c;
    const double *ptr = nullptr;
    int64_t cnt = 0;
    const int64_t n = c.n, L1 = c.L + 1, p = c.p;
    switch (field) {
        case EDA_FIELD_TRUTH: ptr = c.truth; cnt = (c.N + 1) * n; break;
        case EDA_FIELD_XB: ptr = c.xb; cnt = n * L1; break;
        case EDA_FIELD_TRAJ: ptr = c.traj; cnt = L1 * (c.N + 1) * n; break;
        case EDA_FIELD_Y: ptr = c.y; cnt = p * L1; break;
        case EDA_FIELD_D: ptr = c.d; cnt = p * L1; break;
        case EDA_FIELD_B: ptr = c.b; cnt = n * L1; break;
        case EDA_FIELD_COSTC: ptr = c.costc; cnt = L1; break;
        case EDA_FIELD_UBROW: ptr = c.ubrow; cnt = n; break;
        case EDA_FIELD_S:
            if (!c.have_lmp) return EDA_ERR_ORDER;
            ptr = c.sk_s; cnt = n * c.k; break;
        case EDA_FIELD_EIG:
            if (!c.have_lmp) return EDA_ERR_ORDER;
            ptr = c.sk_eig; cnt = c.k; break;
        default: return EDA_ERR_INVALID_ARG;
    }
    *byte_offset = (size_t)(reinterpret_cast<const char *>(ptr) - c.ws);
    *count = cnt;
    return EDA_OK;
}

int eda_profile(eda_ctx *h, int32_t enable) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    HIP_TRY(hipStreamSynchronize(c.stream));
    c.prof = enable != 0;
    c.prof_launches = 0;
    c.ev_used = 0;
    return EDA_OK;
}

int eda_profile_read(eda_ctx *h, int64_t *launches, double *total_ms) {
    if (!h || !launches || !total_ms) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    HIP_TRY(hipStreamSynchronize(c.stream));
    double tot = 0.0;
    for (size_t i = 0; i + 1 < c.ev_used; i += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.ev[i], c.ev[i + 1]));
        tot += ms;
    }
    *launches = c.prof_launches;
    *total_ms = tot;
    return EDA_OK;
}

int eda_destroy(eda_ctx *h) {
    if (!h) return EDA_ERR_INVALID_ARG;
    for (hipEvent_t e : h->c.ev) (void)hipEventDestroy(e);
    delete h;
    return EDA_OK;
}

const char *eda_strerror(int code) {
    switch (code) {
        case EDA_OK: return "ok";
        case EDA_ERR_INVALID_ARG: return "invalid argument";
        case EDA_ERR_WORKSPACE: return "workspace too small";
        case EDA_ERR_HIP: return "HIP runtime error";
        case EDA_ERR_NOT_SPD: return "Cholesky of the sketched matrix failed after the shift";
        case EDA_ERR_ORDER: return "no preconditioner: call eda_sketch_evd first";
        case EDA_ERR_UNSUPPORTED: return "unsupported size or option";
        case EDA_WARN_NOT_CONVERGED: return "some members did not converge";
        default: return "unknown status";
    }
}

}  // extern "C"
