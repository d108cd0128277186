// The C ABI (include/eda.h): workspace planning, problem set-up, Hessian
// products, randomized eigendecomposition, spectral LMP and batched PCG.
// Host code only sequences kernels on the context's stream; every arithmetic
// step of the path runs in this library's HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

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
    if (!(c->sigma_o > 0) || !(c->sigma_b > 0) || !(c->dt > 0)) return false;
    if (c->b_kind == EDA_B_GAUSS) {
        if (!(c->len_b >= 2.0)) return false;
    } else if (c->b_kind == EDA_B_DIFFUSION) {
        if (!(c->len_b > 0) || !(c->len_b <= 1e3) || c->diff_steps < 2 || c->diff_steps > 64 || (c->diff_steps & 1))
            return false;
    } else {
        return false;
    }
    if (c->members < 1 || c->spinup < 0) return false;
    if (c->max_ell < 1 || c->max_ell > 128) return false;
    if (c->max_cols < 0) return false;
    if (c->ub_mode != EDA_UB_DENSE && c->ub_mode != EDA_UB_BANDED) return false;
    return true;
}

struct Plan {
    int n, N, L, nt, nv, p, maxc, maxl;
    int pad_l, ext_len;
    size_t off_trajx, off_ub16, off_ub32;
    size_t off_ubrow, off_ub, off_truth, off_spin, off_xb, off_traj, off_y, off_d, off_force, off_b, off_costc;
    size_t off_hv_v, off_hv_obs, off_hv_lam, off_zero;
    size_t off_phi, off_sy, off_sq, off_sq1, off_ss, off_small, off_eig, off_coef, off_coefu, off_info, off_splitk,
        off_lmpt, off_lmpw, off_sr;
    size_t off_x, off_r, off_z, off_pp, off_q, off_scal, off_status, off_iters, off_start, off_members, off_hist;
    size_t off_p2, off_pqp, off_fin;  // split PCG iterations (banded U_B)
    size_t off_xflags, off_xedges, off_xerr, off_xnseg, off_rzp;  // wave pieces with halo exchange
    size_t off_lsync;                                             // single-launch LMP tile barriers
    size_t splitk_elems;
    size_t total;
};

// Banded U_B taps: offsets o with |r(o)| > 2^-60 r(0), clipped to one full
// period of the ring.  Gaussian B: o^2 < 60 ln 2 len^2.  Diffusion B: the
// offsets where the unbounded line's kernel of (I - kappa Lap)^(-M/2) exceeds
// 2^-60 of its centre (the ring's kernel adds the other periods' tails, which
// are below that wherever the band stops short of a period).  That kernel is
// evaluated here on a window wide enough that its edge is below 2^-80 of the
// centre, only to size the band; the taps themselves are the device's row.
int diffusion_half_width(int n, double daley, int steps) {
    const double kappa = daley * daley / (2.0 * steps - 3.0);
    const double rho = 2.0 * kappa / ((1.0 + 2.0 * kappa) + std::sqrt(1.0 + 4.0 * kappa));
    const int m = steps / 2;
    for (int K = 64;; K *= 2) {
        if (K >= n) return n;  // the band would reach a whole period: it is clipped to one
        const int len = 2 * K + 1;
        std::vector<double> g(len), r(len), t(len);
        for (int i = 0; i < len; i++) g[i] = std::pow(rho, std::abs(i - K));
        r = g;
        for (int step = 1; step < m; step++) {
            for (int i = 0; i < len; i++) {
                double acc = 0.0;
                for (int j = 0; j < len; j++) {
                    const int o = i - j + K;
                    if (o >= 0 && o < len) acc += r[j] * g[o];
                }
                t[i] = acc;
            }
            r.swap(t);
        }
        if (r[len - 1] < std::ldexp(r[K], -80)) {
            int w = 0;
            for (int o = 1; o <= K; o++)
                if (r[K + o] > std::ldexp(r[K], -60)) w = o;
            return w;
        }
    }
}

void band_taps(const eda_config *c, int &lo, int &hi) {
    const int n = c->n;
    int w = 0;
    if (c->b_kind == EDA_B_DIFFUSION) {
        w = diffusion_half_width(n, c->len_b, c->diff_steps);
    } else {
        const double lim = 60.0 * std::log(2.0) * c->len_b * c->len_b;
        while (w + 1 <= n / 2 && (double)(w + 1) * (w + 1) < lim) w++;
    }
    if (2 * w + 1 >= n) {
        lo = -((n - 1) / 2);
        hi = n / 2;
    } else {
        lo = -w;
        hi = w;
    }
}

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
    P.off_ub32 = c->ub_mode == EDA_UB_DENSE ? lay.take(n * n * sizeof(float)) : (size_t)-1;
    P.off_truth = lay.take((P.N + 1) * n * d);
    P.off_spin = lay.take(n * d);
    P.off_xb = lay.take(n * L1 * d);
    P.off_traj = lay.take(L1 * (P.N + 1) * n * d);
    const bool banded = c->ub_mode == EDA_UB_BANDED;
    int band_lo, band_hi;
    band_taps(c, band_lo, band_hi);
    {
        int pl, pr;
        if (banded) {
            tlad_pads_split(P.n, P.N, band_hi, &pl, &pr);
            // the exchange form's windows: up to 8 XCH_TB_MAX before a segment, 64 x 8 after its start
            if (pl < 8 * XCH_TB_MAX) pl = 8 * XCH_TB_MAX;
            if (pr < 64 * 8) pr = 64 * 8;
        } else {
            tlad_pads(P.n, &pl, &pr);
        }
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
    P.off_hv_obs = lay.take(p * mc * (banded ? SPLIT_PMAX : 1) * d);  // split: one block per piece
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
    if (c->ub_mode == EDA_UB_DENSE) {
        // the dense U_B products of up to max(maxl, maxc) columns, K split
        const int nbmax = P.maxl > P.maxc ? P.maxl : P.maxc;
        for (int nb = 1; nb <= nbmax; nb++) {
            const size_t e1 = gemm_splitk_elems(P.n, nb, P.n), e2 = gemm_lowp_splitk_elems(P.n, nb, P.n);
            if (e1 > P.splitk_elems) P.splitk_elems = e1;
            if (e2 > P.splitk_elems) P.splitk_elems = e2;
        }
    }
    P.off_splitk = lay.take((P.splitk_elems ? P.splitk_elems : 1) * d);
    P.off_lmpt = lay.take(ml * mc * d);
    P.off_lmpw = lay.take(lmp_work_doubles(P.n, P.maxl, P.maxc) * d);
    P.off_sr = lay.take(n * ml * d);
    P.off_x = lay.take(n * mc * d);
    P.off_r = lay.take(n * mc * d);
    P.off_z = lay.take(n * mc * d);
    P.off_pp = lay.take(n * mc * d);
    P.off_q = lay.take(n * mc * d);
    P.off_scal = lay.take(4 * mc * d);
    P.off_status = lay.take(mc * sizeof(int32_t));
    P.off_iters = lay.take(mc * sizeof(int32_t));
    P.off_start = lay.take(mc * sizeof(int32_t));
    P.off_members = lay.take(mc * sizeof(int32_t));
    P.off_hist = lay.take(mc * (size_t)HIST_CAP * d);
    P.off_p2 = lay.take((banded ? n * mc : 1) * d);
    P.off_pqp = lay.take(mc * (XCH_SEG_MAX > SPLIT_PMAX ? XCH_SEG_MAX : SPLIT_PMAX) * d);
    P.off_fin = lay.take(lmp_fin_doubles(P.maxc) * d);
    {
        const bool xch = banded && P.n >= XCH_N_MIN;
        const size_t slots = xch ? 8 * (size_t)XCH_GRID_MAX : 1;
        P.off_xflags = lay.take((slots + (xch ? XCH_GRID_MAX : 0)) * sizeof(unsigned long long));
        P.off_xedges = lay.take((xch ? slots * 4 * XCH_E_MAX : 1) * d);
        P.off_xerr = lay.take(sizeof(int32_t));
        P.off_xnseg = lay.take(mc * sizeof(int32_t));
        P.off_rzp = lay.take((size_t)LMP_RB_MAX * ((mc + 15) / 16 * 16) * d);
    }
    P.off_lsync = lay.take(lmp_sync_words(P.maxc) * sizeof(unsigned int));
    P.total = lay.total;
    return P;
}

template <typename T>
T *at(char *ws, size_t off) {
    return reinterpret_cast<T *>(ws + off);
}

// Enqueues launch() with HIP events around it when profiling samples this
// launch (kind EDA_PROF_TLAD: inside eda_pcg_solve only, unless
// EDA_PROF_TLAD_ALL is selected).
template <typename F>
int profiled(Ctx &c, int kind, F launch) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool match = c.prof_kind == kind ? (kind != EDA_PROF_TLAD || c.in_pcg)
                                           : (c.prof_kind == EDA_PROF_TLAD_ALL && kind == EDA_PROF_TLAD);
    const bool rec = c.prof > 0 && match && c.prof_seen++ % c.prof == 0;
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
    HIP_TRY(launch());
    if (rec) {
        HIP_TRY(hipEventRecord(e1, c.stream));
        c.prof_launches++;
    }
    return EDA_OK;
}

// Y = U_B X (+ Add), columns optionally masked.  lowp (reduced-precision
// sketch): the dense product runs on the matrix cores with FP32 accumulation
// and FP32 operands (1) or BF16 operands (2).
int ub_apply(Ctx &c, int nb, const double *X, long long ldx, double *Y, long long ldy, const double *Add,
             long long ldadd, const int32_t *active, int lowp = 0) {
    if (c.cfg.ub_mode == EDA_UB_DENSE && lowp == 2) {
        EDA_TRY(profiled(c, EDA_PROF_UB_GEMM,
                         [&] {
                             return gemm_bf16(c.stream, c.n, nb, c.n, c.ub16, c.n, X, ldx, Y, ldy, Add, ldadd, c.splitk,
                                              c.splitk_elems);
                         }));
    } else if (c.cfg.ub_mode == EDA_UB_DENSE && lowp == 1) {
        EDA_TRY(profiled(c, EDA_PROF_UB_GEMM,
                         [&] {
                             return gemm_f32in(c.stream, c.n, nb, c.n, c.ub32, c.n, X, ldx, Y, ldy, Add, ldadd, c.splitk,
                                               c.splitk_elems);
                         }));
    } else if (c.cfg.ub_mode == EDA_UB_DENSE) {
        EDA_TRY(profiled(c, EDA_PROF_UB_GEMM, [&] {
            return gemm_f64(c.stream, false, c.n, nb, c.n, c.ub, c.n, X, ldx, Y, ldy, Add, ldadd, nullptr, c.splitk,
                            c.splitk_elems);
        }));
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

int run_tlad(Ctx &c, const TladArgs &a, int mode, bool fp32, const SplitCols *sc = nullptr) {
    return profiled(c, EDA_PROF_TLAD,
                    [&] { return launch_tlad(c.stream, a, mode, fp32, c.geo_waves, c.geo_tb, sc); });
}

// Whether a launch of `grid` workgroups with P pieces per column can use
// pieces that share the observed increments: EDA_XCH_OBS, flags for every
// column of the context, every piece co-resident (one per compute unit), and
// pieces long enough for their rings (tlad_split_ring_sh).
bool can_share(const Ctx &c, long long grid, int P) {
    return c.xch_mode == EDA_XCH_OBS && c.xch_flags && (long long)c.max_cols * SPLIT_PMAX <= 8ll * XCH_GRID_MAX &&
           grid <= c.num_cus && tlad_split_ring_sh(c.n, c.N, c.band_hi, P) > 0;
}

// Pieces per column of a split launch over `columns` columns: the forced
// count, else, of 1, 2, 3, 4 and 8 pieces with pieces x columns <= CUs, the
// one whose ring is shortest (shared where can_share, else independent; the
// fewer pieces on a tie).  5 to 7 pieces were measured no faster than 4.
int split_pieces(const Ctx &c, int columns) {
    if (c.split_force != 0) return c.split_force;
    int P = 1, best = c.n;
    for (int cand : {2, 3, 4, 8}) {
        const long long grid = (long long)cand * columns;
        if (grid > c.num_cus) continue;
        const int R = can_share(c, grid, cand) ? tlad_split_ring_sh(c.n, c.N, c.band_hi, cand)
                                               : tlad_split_ring(c.n, c.N, c.band_hi, cand);
        if (R > 0 && R < best) {
            best = R;
            P = cand;
        }
    }
    return P;
}

// Ring pieces of a split launch of `grid` workgroups, P pieces per column:
// pieces that share the observed increments (shorter rings, one bounded wait)
// when can_share, else independent ones.  Returns 1 (shared), 0
// (independent) or -1 when neither ring fits (a forced P that only the
// shared form fits, in a launch that cannot share).
int set_pieces(Ctx &c, TladArgs &a, long long grid, int P) {
    const bool sh = can_share(c, grid, P);
    if (!sh && tlad_split_ring(c.n, c.N, c.band_hi, P) == 0) return -1;
    a.pieces = P;
    a.ring = sh ? tlad_split_ring_sh(c.n, c.N, c.band_hi, P) : tlad_split_ring(c.n, c.N, c.band_hi, P);
    a.halo = sh ? tlad_split_halo_sh(c.N, c.band_hi) : tlad_split_halo(c.N, c.band_hi);
    if (sh) {
        a.pflags = c.xch_flags;
        a.want = (++c.xch_epoch) << 16;
        a.spin_max = c.xch_spin < 0 ? XCH_SPIN_DEFAULT : c.xch_spin;
        a.err = c.xch_err;
    }
    return sh ? 1 : 0;
}

// Batched Hessian product.  Banded U_B: one fused launch (U_B, TL, AD, U_B,
// identity) per call, on pieces of each column when fewer columns than CUs
// run; dense U_B: FP64 MFMA GEMM, TL/AD, GEMM.
int hessvec(Ctx &c, const int32_t *cols, int nb, const double *X, long long ldx, double *Y, long long ldy,
            uint32_t flags, const int32_t *active) {
    if (nb <= 0) return EDA_OK;
    const bool add = (flags & EDA_HV_ADD_IDENTITY) != 0;
    const bool fp32 = (flags & (EDA_HV_MIXED | EDA_HV_BF16)) != 0;
    const int lowp = (flags & EDA_HV_BF16) ? 2 : fp32 ? 1 : 0;
    if (c.cfg.ub_mode == EDA_UB_BANDED) {
        TladArgs a = tlad_args(c, nb, cols, active);
        a.V = X;
        a.ldv = ldx;
        a.obs = c.hv_obs;
        a.lam = Y;
        a.ldl = ldy;
        a.add_identity = add ? 1 : 0;
        const int P = split_pieces(c, nb);
        if (P > 1) {
            const int sh = set_pieces(c, a, (long long)nb * P, P);
            if (sh < 0) return EDA_ERR_UNSUPPORTED;
            return run_tlad(c, a, sh ? TLAD_SPLIT_HV_SH : TLAD_SPLIT_HV, fp32);
        }
        return run_tlad(c, a, TLAD_HV, fp32);
    }
    EDA_TRY(ub_apply(c, nb, X, ldx, c.hv_v, c.n, nullptr, 0, active, lowp));
    TladArgs a = tlad_args(c, nb, cols, active);
    a.V = c.hv_v;
    a.ldv = c.n;
    a.obs = c.hv_obs;
    a.lam = c.hv_lam;
    a.ldl = c.n;
    EDA_TRY(run_tlad(c, a, TLAD_RAW, fp32));
    EDA_TRY(ub_apply(c, nb, c.hv_lam, c.n, Y, ldy, add ? X : nullptr, ldx, active, lowp));
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

// The last stage of the single-problem Nystrom sketch with no host
// synchronisation, in phases around the three Cholesky factorisations and the
// SVD of T (chol_job and jacobi_job give their operands):
//   0: G = Y^T Y                  -> chol 0: R1, R1^-1
//   1: Q1 = Y R1^-1, G = Q1^T Q1  -> chol 1: R2, R2^-1
//   2: Q = Q1 R2^-1, R_Y = R2 R1, W = Phi^T Y (symmetrised) -> chol 2: C, C^-1
//   3: T = R_Y C^-1               -> SVD
// then nystrom_post_svd: S = Q U, signs, theta, the LMP coefficients; then
// the device-side redo (redo_job), which takes over when one of the three
// unshifted Cholesky outcomes (sk_info[0..2]) is nonzero.  Slots of sk_small
// (l_max^2 doubles each): 0 G, 1 R1 then C^-1, 2 R1^-1 then T, 3 R2 then U,
// 4 R2^-1 then sigma, 7 R_Y, 8 W, 9 C.
JacobiJob jacobi_job(const Ctx &c, int l) {
    const size_t ls = (size_t)c.max_ell * c.max_ell;
    return JacobiJob{l, c.sk_small + 2 * ls, c.sk_small + 3 * ls, c.sk_small + 4 * ls};
}

CholJob chol_job(const Ctx &c, int l, int which) {
    const size_t ls = (size_t)c.max_ell * c.max_ell;
    double *m = c.sk_small;
    switch (which) {
        case 0: return CholJob{l, m, 0.0, m + 1 * ls, m + 2 * ls, c.sk_info + 0};
        case 1: return CholJob{l, m, 0.0, m + 3 * ls, m + 4 * ls, c.sk_info + 1};
        default: return CholJob{l, m + 8 * ls, 0.0, m + 9 * ls, m + 1 * ls, c.sk_info + 2};
    }
}

int nystrom_phase(Ctx &c, int l, int phase) {
    hipStream_t s = c.stream;
    const int n = c.n;
    const size_t ls = (size_t)c.max_ell * c.max_ell;
    double *G = c.sk_small, *R1 = c.sk_small + 1 * ls, *R1i = c.sk_small + 2 * ls;
    double *R2 = c.sk_small + 3 * ls, *R2i = c.sk_small + 4 * ls;
    double *RY = c.sk_small + 7 * ls, *Wm = c.sk_small + 8 * ls;
    double *Ci = c.sk_small + 1 * ls, *Tm = c.sk_small + 2 * ls;
    switch (phase) {
        case 0:
            HIP_TRY(gemm_f64(s, true, l, l, n, c.sk_y, n, c.sk_y, n, G, l, nullptr, 0, nullptr, c.splitk,
                             c.splitk_elems));
            break;
        case 1:
            HIP_TRY(gemm_f64(s, false, n, l, l, c.sk_y, n, R1i, l, c.sk_q1, n, nullptr, 0, nullptr, nullptr, 0));
            HIP_TRY(gemm_f64(s, true, l, l, n, c.sk_q1, n, c.sk_q1, n, G, l, nullptr, 0, nullptr, c.splitk,
                             c.splitk_elems));
            break;
        case 2:
            HIP_TRY(gemm_f64(s, false, n, l, l, c.sk_q1, n, R2i, l, c.sk_q, n, nullptr, 0, nullptr, nullptr, 0));
            HIP_TRY(launch_small_gemm(s, l, false, false, R2, R1, RY));
            HIP_TRY(gemm_f64(s, true, l, l, n, c.sk_phi, n, c.sk_y, n, Wm, l, nullptr, 0, nullptr, c.splitk,
                             c.splitk_elems));
            HIP_TRY(launch_sym(s, l, Wm));
            break;
        default:
            HIP_TRY(launch_small_gemm(s, l, false, false, RY, Ci, Tm));
            break;
    }
    return EDA_OK;
}

int nystrom_post_svd(Ctx &c, int l, int k, int rule) {
    hipStream_t s = c.stream;
    const int n = c.n;
    const JacobiJob j = jacobi_job(c, l);
    double *dscal = reinterpret_cast<double *>(c.sk_info + 16);
    HIP_TRY(gemm_f64(s, false, n, k, l, c.sk_q, n, j.U, l, c.sk_s, n, nullptr, 0, nullptr, nullptr, 0));
    HIP_TRY(launch_fix_signs(s, n, k, c.sk_s, n));
    HIP_TRY(launch_lmp_coef(s, k, j.sig, 0.0, 1, rule, c.sk_eig, c.sk_coef, c.sk_coefu, dscal + 1));
    return EDA_OK;
}

// Operands of the device-side shifted sketch (k_nystrom_redo) of this
// context: triggered by the unshifted outcomes sk_info[0..2]; sk_info[3..4]
// receive whether it ran and whether it failed; theta at the same place as
// nystrom_post_svd's.  u: unit roundoff of the products that formed Y.
RedoJob redo_job(const Ctx &c, int l, int k, int rule, double u) {
    RedoJob j{};
    j.n = c.n;
    j.l = l;
    j.k = k;
    j.rule = rule;
    j.u = u;
    j.trigger = c.sk_info;
    j.state = c.sk_info + 3;
    j.phi = c.sk_phi;
    j.y = c.sk_y;
    j.q1 = c.sk_q1;
    j.q2 = c.sk_s;
    j.q = c.sk_q;
    j.s = c.sk_s;
    j.small = c.sk_small;
    j.ls = (long long)c.max_ell * c.max_ell;
    j.eig = c.sk_eig;
    j.coef = c.sk_coef;
    j.coefu = c.sk_coefu;
    j.theta = reinterpret_cast<double *>(c.sk_info + 16) + 1;
    return j;
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
    c.ub32 = P.off_ub32 == (size_t)-1 ? nullptr : at<float>(w, P.off_ub32);
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
    c.lmp_work = at<double>(w, P.off_lmpw);
    c.sk_sr = at<double>(w, P.off_sr);
    c.pc_x = at<double>(w, P.off_x);
    c.pc_r = at<double>(w, P.off_r);
    c.pc_z = at<double>(w, P.off_z);
    c.pc_p = at<double>(w, P.off_pp);
    c.pc_q = at<double>(w, P.off_q);
    c.pc_scal = at<double>(w, P.off_scal);
    c.pc_status = at<int32_t>(w, P.off_status);
    c.pc_iters = at<int32_t>(w, P.off_iters);
    c.pc_start = at<int32_t>(w, P.off_start);
    c.pc_members = at<int32_t>(w, P.off_members);
    c.pc_hist = at<double>(w, P.off_hist);
    c.hist_cap = HIST_CAP;
    c.pc_p2 = at<double>(w, P.off_p2);
    c.pc_pqp = at<double>(w, P.off_pqp);
    c.lmp_fin = at<double>(w, P.off_fin);
    c.pad_r = P.ext_len - P.n - P.pad_l;
    if (cfg->ub_mode == EDA_UB_BANDED && P.n >= XCH_N_MIN) {
        c.xch_flags = at<unsigned long long>(w, P.off_xflags);
        c.xch_edges = at<double>(w, P.off_xedges);
    }
    c.xch_err = at<int32_t>(w, P.off_xerr);
    c.xch_nseg = at<int32_t>(w, P.off_xnseg);
    c.rz_part = at<double>(w, P.off_rzp);
    c.lmp_sync = at<unsigned int>(w, P.off_lsync);
    band_taps(cfg, c.band_lo, c.band_hi);
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c.num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            lmp_noalloc_scratch(&c.lmp_noalloc) != hipSuccess) {
            delete h;
            return EDA_ERR_HIP;
        }
    }

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
    // exchange flags start below every launch's phases; segment counts start empty
    if ((c.xch_flags && hipMemsetAsync(c.xch_flags, 0, sizeof(unsigned long long) * 9 * XCH_GRID_MAX, s) != hipSuccess) ||
        hipMemsetAsync(c.xch_nseg, 0, sizeof(int32_t) * c.max_cols, s) != hipSuccess ||
        hipMemsetAsync(c.xch_err, 0, sizeof(int32_t), s) != hipSuccess ||
        hipMemsetAsync(c.lmp_sync, 0, sizeof(unsigned int) * lmp_sync_words(c.max_cols), s) != hipSuccess)
        return fail(EDA_ERR_HIP);
    // U_B
    if ((cfg->b_kind == EDA_B_DIFFUSION
             ? launch_ub_row_diffusion(s, n, cfg->sigma_b, cfg->len_b, cfg->diff_steps, c.ubrow)
             : launch_ub_row(s, n, cfg->sigma_b, cfg->len_b, c.ubrow)) != hipSuccess)
        return fail(EDA_ERR_HIP);
    if (c.ub && launch_ub_fill(s, n, c.ubrow, c.ub) != hipSuccess) return fail(EDA_ERR_HIP);
    if (c.ub16 && launch_to_bf16(s, (long long)n * n, c.ub, c.ub16) != hipSuccess) return fail(EDA_ERR_HIP);
    if (c.ub32 && launch_to_f32(s, (long long)n * n, c.ub, c.ub32) != hipSuccess) return fail(EDA_ERR_HIP);
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
    if (flags & ~(EDA_HV_ADD_IDENTITY | EDA_HV_MIXED | EDA_HV_BF16)) return EDA_ERR_INVALID_ARG;
    return hessvec(c, d_col_member, nb, d_X, ldx, d_Y, ldy, flags, nullptr);
}

static int sketch_evd_impl(eda_ctx *h, int32_t kind, const double *d_phi, int64_t ldphi, int32_t ell, int32_t k,
                           int32_t q, int32_t method, int32_t theta_rule, uint32_t flags, double *h_eig,
                           double *h_theta) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (ell < 1 || ell > c.max_ell || k < 1 || k > ell || q < 1) return EDA_ERR_INVALID_ARG;
    if (method != EDA_METHOD_NYSTROM && method != EDA_METHOD_REVD) return EDA_ERR_INVALID_ARG;
    if (theta_rule < EDA_THETA_MID || theta_rule > EDA_THETA_ONE) return EDA_ERR_INVALID_ARG;
    if (flags & ~(EDA_HV_MIXED | EDA_HV_BF16)) return EDA_ERR_INVALID_ARG;
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
    c.sr_ready = false;
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
    double *RY = c.sk_small + 7 * ls, *Wm = c.sk_small + 8 * ls;
    double *Tm = c.sk_small + 2 * ls, *Um = c.sk_small + 3 * ls;
    double *sig = c.sk_small + 4 * ls;
    double *dscal = reinterpret_cast<double *>(c.sk_info + 16);
    const uint32_t hvf = flags & (EDA_HV_MIXED | EDA_HV_BF16);
    if (method == EDA_METHOD_NYSTROM) {
        EDA_TRY(hessvec(c, c.zero_members, ell, c.sk_phi, n, c.sk_y, n, hvf, nullptr));
        for (int pass = 2; pass <= q; pass++) {
            // power pass: Phi <- orth(Y), Y = A Phi
            EDA_TRY(cholqr2(c, ell, c.sk_y, c.sk_q, RY));
            HIP_TRY(launch_copy_cols(s, n, ell, c.sk_q, n, c.sk_phi, n));
            EDA_TRY(hessvec(c, c.zero_members, ell, c.sk_phi, n, c.sk_y, n, hvf, nullptr));
        }
        // unshifted CholQR2 of Y, W = Phi^T Y and its Cholesky, T = R_Y C^-1,
        // T = U Sigma V^T, S = Q_Y U(:, 1:k), D = Sigma^2; where one of the
        // Choleskys failed, the device-side redo repeats the stage with the
        // shifts (shifted CholQR3; Y + nu Phi with nu = u ||Y||_F, D = Sigma^2 - nu)
        for (int phase = 0; phase < 4; phase++) {
            EDA_TRY(nystrom_phase(c, ell, phase));
            if (phase < 3) {
                const CholJob j = chol_job(c, ell, phase);
                HIP_TRY(launch_chol_inv(s, j.l, j.W, j.shift, j.C, j.Cinv, j.info));
            }
        }
        const JacobiJob jj = jacobi_job(c, ell);
        HIP_TRY(launch_jacobi_svd_u(s, ell, const_cast<double *>(jj.T), jj.U, jj.sig));
        EDA_TRY(nystrom_post_svd(c, ell, k, theta_rule));
        // the unit roundoff of the products that formed Y: FP64, or FP32 / BF16 operands
        const double u = (hvf & EDA_HV_BF16) ? std::ldexp(1.0, -8)
                         : (hvf & EDA_HV_MIXED) ? std::ldexp(1.0, -24) : 2.220446049250313e-16;
        HIP_TRY(launch_nystrom_redo(s, redo_job(c, ell, k, theta_rule, u)));
        int32_t st[2] = {0, 0};
        EDA_TRY(sync_read(c, st, c.sk_info + 3, sizeof(st)));
        if (st[1] != 0) return EDA_ERR_NOT_SPD;
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
    c.k = k;
    c.have_lmp = true;
    c.sr_ready = false;
    return EDA_OK;
}

// The split products of a sketch wait for each other when their pieces share
// the observed increments; a wait that gave up (NaN in its products) makes
// the call return EDA_ERR_SYNC, whatever the factorisations then did.
int eda_sketch_evd(eda_ctx *h, int32_t kind, const double *d_phi, int64_t ldphi, int32_t ell, int32_t k, int32_t q,
                   int32_t method, int32_t theta_rule, uint32_t flags, double *h_eig, double *h_theta) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    HIP_TRY(hipMemsetAsync(c.xch_err, 0, sizeof(int32_t), c.stream));
    const int rc = sketch_evd_impl(h, kind, d_phi, ldphi, ell, k, q, method, theta_rule, flags, h_eig, h_theta);
    int32_t werr = 0;
    EDA_TRY(sync_read(c, &werr, c.xch_err, sizeof(int32_t)));
    if (werr != 0) {
        c.have_lmp = false;
        return EDA_ERR_SYNC;
    }
    return rc;
}

}  // extern "C"

namespace {

// Y = X + S_k diag(coef) S_k^T X (coef: P_theta or U_theta coefficients);
// inside PCG (status given) tiles of stopped members are skipped.
// The tile barriers of the single-launch LMP (bounded waits report into the
// exchange's error word, which eda_pcg_solve reads at its end).
LmpSync lmp_sync(const Ctx &c) {
    LmpSync y{};
    const int tiles = (int)(lmp_sync_words(c.max_cols) / 2);
    y.arrive = c.lmp_sync;
    y.leave = c.lmp_sync + tiles;
    y.tiles = tiles;
    y.max_blocks = c.num_cus;
    y.spin_max = c.xch_spin < 0 ? XCH_SPIN_DEFAULT : c.xch_spin;
    y.err = c.xch_err;
    return y;
}

// Inside eda_pcg_solve (pcg set) the LMP runs in the context's form; the
// public eda_lmp_apply always takes the two-launch form, which has no wait.
int lmp_apply(Ctx &c, int which, int nb, const double *X, long long ldx, double *Y, long long ldy,
              const int32_t *status = nullptr, double *rz = nullptr, bool pcg = false) {
    const double *coef = which == EDA_LMP_U ? c.sk_coefu : c.sk_coef;
    if (!c.sr_ready) {
        HIP_TRY(launch_lmp_rowmajor(c.stream, c.n, c.k, c.sk_s, c.sk_sr));
        c.sr_ready = true;
    }
    const LmpSync sy = lmp_sync(c);
    const bool one = pcg && c.lmp_form == EDA_LMP_FORM_ONE;
    HIP_TRY(launch_lmp(c.stream, c.n, c.k, nb, c.sk_s, c.sk_sr, coef, X, ldx, Y, ldy, status, c.lmp_work, rz,
                       one ? &sy : nullptr));
    return EDA_OK;
}

// One fused PCG iteration (banded U_B) of every running column: p = z + beta p
// (p updated in place), (I + A) p, alpha, x, r, the convergence test.
// rz_part: the row-block sums of r^T z that the LMP left (null: summed in the kernel).
int fused_iteration(Ctx &c, int nm, const PcgArgs &a, double *p, double rtol, int it,
                    const double *rz_part = nullptr, const int32_t *start = nullptr) {
    TladArgs t = tlad_args(c, nm, c.pc_members, nullptr);
    t.obs = c.hv_obs;
    t.pcg.members = c.pc_members;
    t.pcg.b = c.b;
    t.pcg.x = c.pc_x;
    t.pcg.r = c.pc_r;
    t.pcg.z = a.z;
    t.pcg.p = p;
    t.pcg.scal = c.pc_scal;
    t.pcg.status = c.pc_status;
    t.pcg.iters = c.pc_iters;
    t.pcg.hist = a.hist;
    t.pcg.hist_cap = c.hist_cap;
    t.pcg.rtol = rtol;
    t.pcg.it = it;
    t.pcg.first = it == 1 ? 1 : 0;
    t.pcg.start = start;
    if (rz_part) {
        int rows, nrb;
        lmp_blocks(c.n, &rows, &nrb);
        t.pcg.rz_part = rz_part;
        t.pcg.rz_ld = (nm + 15) / 16 * 16;
        t.pcg.rz_nrb = nrb;
    }
    return run_tlad(c, t, TLAD_PCG, false);
}

// The update half of a split PCG iteration with z = P_theta r of the new r.
int lmp_update(Ctx &c, int nb, const LmpFin &f) {
    if (!c.sr_ready) {
        HIP_TRY(launch_lmp_rowmajor(c.stream, c.n, c.k, c.sk_s, c.sk_sr));
        c.sr_ready = true;
    }
    const LmpSync sy = lmp_sync(c);
    HIP_TRY(launch_lmp_fin(c.stream, c.n, c.k, nb, c.sk_s, c.sk_sr, c.sk_coef, c.pc_r, c.pc_z, c.pc_status,
                           c.lmp_work, f, c.rz_part, c.lmp_form == EDA_LMP_FORM_ONE ? &sy : nullptr));
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

int eda_lmp_apply_noalloc(eda_ctx *h, int32_t which, int32_t nb, const double *d_X, int64_t ldx, double *d_Y,
                          int64_t ldy) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (which != EDA_LMP_P && which != EDA_LMP_U) return EDA_ERR_INVALID_ARG;
    if (nb < 0 || nb > c.max_cols || ldx < c.n || ldy < c.n) return EDA_ERR_INVALID_ARG;
    if (!c.have_lmp) return EDA_ERR_ORDER;
    if (nb == 0) return EDA_OK;
    if (!d_X || !d_Y) return EDA_ERR_INVALID_ARG;
    if (!c.lmp_noalloc) return EDA_ERR_HIP;
    if (lmp_work_doubles(c.n, c.k, nb) > LMP_NOALLOC_DOUBLES) return EDA_ERR_UNSUPPORTED;
    const double *coef = which == EDA_LMP_U ? c.sk_coefu : c.sk_coef;
    if (!c.sr_ready) {
        HIP_TRY(launch_lmp_rowmajor(c.stream, c.n, c.k, c.sk_s, c.sk_sr));
        c.sr_ready = true;
    }
    HIP_TRY(launch_lmp(c.stream, c.n, c.k, nb, c.sk_s, c.sk_sr, coef, d_X, ldx, d_Y, ldy, nullptr, c.lmp_noalloc));
    return EDA_OK;
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
    const bool fused = c.cfg.ub_mode == EDA_UB_BANDED;
    // with the LMP, the banded form runs split iterations: the Hessian part on
    // pieces of every running column (wave pieces with halo exchange, or P ring
    // pieces per column with P * running columns <= compute units), then the
    // update fused with the LMP of the new residual (which also leaves the
    // row-block partials of r^T z for the exchange form)
    const bool split = fused && use_lmp;
    if (use_lmp) {
        // the bounded waits of this solve (halo exchange, LMP tile barriers) start clear
        HIP_TRY(hipMemsetAsync(c.xch_err, 0, sizeof(int32_t), s));
        HIP_TRY(hipMemsetAsync(c.lmp_sync, 0, sizeof(unsigned int) * lmp_sync_words(c.max_cols), s));
        EDA_TRY(lmp_apply(c, EDA_LMP_P, nm, c.pc_r, n, c.pc_z, n, c.pc_status, split ? c.rz_part : nullptr, true));
    }
    const int xch_grid = (c.num_cus < XCH_GRID_MAX ? c.num_cus : XCH_GRID_MAX) & ~7;
    // Admission.  With the automatic piece choice and shared pieces, more
    // running columns than half the CUs would leave whole-column iterations,
    // one column per CU, and so half the device idle.  The solve then starts
    // only `cap` columns; the others wait (COL_PENDING) and are admitted as
    // running ones stop, each from its own first iteration (start[c] holds the
    // loop iteration before it; iteration counts and cost histories are the
    // column's own).  The control member's columns wait first (with the LMP of
    // the control's Hessian they need the fewest iterations), then the last
    // columns; the waiting ones are admitted in column order, the control's
    // last.  A column admitted at loop iteration s has maxit - s + 1 iterations
    // left.  Decisions use the checkpoint lists, so they do not depend on timing.
    const int cap = c.num_cus / 2;
    const bool defer = split && c.split_force == 0 && nm > cap && nm <= SPLIT_LIST_MAX && cap >= 1 &&
                       can_share(c, 2ll * cap, 2);
    std::vector<int16_t> pending;                 // waiting columns, in admission order
    size_t next_pending = 0;                      // pending[next_pending..] still wait
    std::vector<std::pair<int, int16_t>> admits;  // (loop iteration, column) of each admission
    std::vector<char> waits(nm, 0);
    if (defer) {
        std::vector<int16_t> order;  // which columns wait first
        for (int i = 0; i < nm; i++)
            if (h_members[i] == 0) order.push_back((int16_t)i);
        for (int i = nm - 1; i >= 0; i--)
            if (h_members[i] != 0) order.push_back((int16_t)i);
        order.resize(nm - cap);
        for (int16_t col : order) waits[col] = 1;
        for (int i = 0; i < nm; i++)
            if (waits[i] && h_members[i] != 0) pending.push_back((int16_t)i);
        for (int i = 0; i < nm; i++)
            if (waits[i] && h_members[i] == 0) pending.push_back((int16_t)i);
        HIP_TRY(hipMemsetAsync(c.pc_start, 0, sizeof(int32_t) * nm, s));
        SplitCols wl{};
        wl.count = (int32_t)pending.size();
        for (int i = 0; i < wl.count; i++) wl.col[i] = pending[i];
        HIP_TRY(launch_col_status(s, wl, COL_RUNNING, COL_PENDING, c.pc_status, nullptr, 0));
    }
    const int32_t *d_start = defer ? c.pc_start : nullptr;
    // Convergence checks are pipelined: every check_every iterations the status
    // array is copied to a pinned host slot behind an event; the host reads a
    // checkpoint once its event has completed, and waits only when more than
    // max_ahead checkpoints are outstanding, so the GPU always has queued work.
    // Iterations queued after every column stopped return at once.
    const int check_every = 8, max_ahead = 2;
    // (the events first: a context keeps h_ck only with every event created)
    for (int i = 0; i < Ctx::CK_SLOTS; i++)
        if (!c.ck_ev[i]) HIP_TRY(hipEventCreateWithFlags(&c.ck_ev[i], hipEventDisableTiming));
    if (!c.h_ck)
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&c.h_ck),
                              sizeof(int32_t) * Ctx::CK_SLOTS * (size_t)c.max_cols, hipHostMallocDefault));
    int ck_issued = 0, ck_done = 0;
    std::vector<std::vector<int16_t>> ck_running;  // running columns at each checkpoint read
    std::vector<int> ck_iter;                      // loop iteration after which each was taken
    bool none_running = false;
    auto consume = [&](bool block) -> int {  // read the oldest outstanding checkpoint
        const int slot = ck_done % Ctx::CK_SLOTS;
        if (block) {
            HIP_TRY(hipEventSynchronize(c.ck_ev[slot]));
        } else {
            hipError_t q = hipEventQuery(c.ck_ev[slot]);
            if (q == hipErrorNotReady) return 0;
            if (q != hipSuccess) return EDA_ERR_HIP;
        }
        const int32_t *st = c.h_ck + (size_t)slot * c.max_cols;
        std::vector<int16_t> running;
        if (split && nm <= SPLIT_LIST_MAX) {
            for (int i = 0; i < nm; i++)
                if (st[i] == COL_RUNNING) running.push_back((int16_t)i);
        } else {
            for (int i = 0; i < nm; i++)
                if (st[i] == COL_RUNNING) running.push_back(0);  // only the count is used
        }
        // every column stopped: none ran at the checkpoint, none waits, none
        // was admitted after it
        const bool later = !admits.empty() && admits.back().first > ck_iter[ck_done];
        none_running |= running.empty() && next_pending == pending.size() && !later;
        ck_running.push_back(std::move(running));
        ck_done++;
        return 1;
    };
    double *pbuf[2] = {c.pc_p, c.pc_p2};
    int cur = 0;  // pbuf[cur] holds the current p
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
            if (split) {
                // running columns as of the checkpoint 8 .. 15 iterations back (waited
                // for if need be, so that the pieces, and the rounding, of every
                // iteration do not depend on timing; at least 8 iterations stay
                // queued): a superset of the running ones
                SplitCols sc{};
                int active = nm;
                const int j = it / check_every - 2;
                const std::vector<int16_t> *known = nullptr;
                if (j >= 0 && j < ck_issued) {
                    while (ck_done <= j) EDA_TRY(consume(true));
                    known = &ck_running[j];
                    active = (int)known->size();
                }
                if (defer) {
                    // the list, the columns admitted after its checkpoint, and
                    // admissions into the room left
                    std::vector<int16_t> cols;
                    if (known) {
                        cols = *known;
                        for (const auto &ad : admits)
                            if (ad.first > ck_iter[j]) cols.push_back(ad.second);
                    } else {
                        for (int i = 0; i < nm; i++)
                            if (!waits[i]) cols.push_back((int16_t)i);
                    }
                    SplitCols ad{};
                    while ((int)cols.size() < cap && next_pending < pending.size()) {
                        const int16_t col = pending[next_pending++];
                        waits[col] = 0;
                        admits.push_back({it, col});
                        cols.push_back(col);
                        ad.col[ad.count++] = col;
                    }
                    if (ad.count > 0)
                        HIP_TRY(launch_col_status(s, ad, COL_PENDING, COL_RUNNING, c.pc_status, c.pc_start, it - 1));
                    std::sort(cols.begin(), cols.end());
                    sc.count = (int)cols.size();
                    for (int i = 0; i < sc.count; i++) sc.col[i] = cols[i];
                    active = sc.count;
                } else if (nm <= SPLIT_LIST_MAX) {
                    sc.count = known ? (int)known->size() : nm;
                    for (int i = 0; i < sc.count; i++) sc.col[i] = known ? (*known)[i] : (int16_t)i;
                }
                XchPlan xp{};
                if (c.xch_mode == EDA_XCH_ON && c.split_force == 0 && c.xch_flags && active > 0)
                    xp = xch_plan(n, c.N, c.band_hi, sc.count > 0 ? sc.count : nm, xch_grid, c.pad_l, c.pad_r);
                const int P = active == 0 ? 1 : split_pieces(c, active);
                if (xp.ok) {
                    // wave pieces with halo exchange
                    TladArgs t = tlad_args(c, nm, c.pc_members, nullptr);
                    t.obs = c.hv_obs;
                    t.pcg.members = c.pc_members;
                    t.pcg.b = c.b;
                    t.pcg.x = c.pc_x;
                    t.pcg.r = c.pc_r;
                    t.pcg.z = c.pc_z;
                    t.pcg.p = pbuf[cur];
                    t.pcg.p_out = pbuf[cur ^ 1];
                    t.pcg.q = c.pc_q;
                    t.pcg.pq_part = c.pc_pqp;
                    t.pcg.scal = c.pc_scal;
                    t.pcg.status = c.pc_status;
                    t.pcg.iters = c.pc_iters;
                    t.pcg.it = it;
                    t.pcg.first = it == 1 ? 1 : 0;
                    XchArgs xa{};
                    xa.flags = c.xch_flags;
                    xa.claim = c.xch_flags + 8 * XCH_GRID_MAX;
                    xa.edges = c.xch_edges;
                    xa.E = xp.E;
                    xa.tb = xp.tb;
                    xa.grid = xp.grid;
                    xa.max_seg = xp.max_seg;
                    xa.epoch = (++c.xch_epoch) << 16;
                    xa.spin_max = c.xch_spin < 0 ? XCH_SPIN_DEFAULT : c.xch_spin;
                    xa.err = c.xch_err;
                    xa.rz_part = c.rz_part;
                    xa.rz_ld = (nm + 15) / 16 * 16;
                    int rows_, nrb_;
                    lmp_blocks(n, &rows_, &nrb_);
                    xa.nrb = nrb_;
                    xa.nseg = c.xch_nseg;
                    EDA_TRY(profiled(c, EDA_PROF_TLAD, [&] { return launch_tlad_x(s, t, xa, xp, sc); }));
                    LmpFin f{};
                    f.q = c.pc_q;
                    f.p = pbuf[cur ^ 1];
                    f.pq_part = c.pc_pqp;
                    f.b = c.b;
                    f.members = c.pc_members;
                    f.x = c.pc_x;
                    f.scal = c.pc_scal;
                    f.hist = a.hist;
                    f.iters = c.pc_iters;
                    f.pieces = 0;
                    f.nseg = c.xch_nseg;
                    f.it = it;
                    f.hist_cap = c.hist_cap;
                    f.rtol = rtol;
                    f.rr_part = c.lmp_fin;
                    f.xbr_part = c.lmp_fin + lmp_fin_doubles(c.max_cols) / 2;
                    EDA_TRY(lmp_update(c, nm, f));
                    cur ^= 1;
                } else if (P == 1) {
                    // whole columns: the fused iteration (its update hidden under the
                    // TL/AD work), then the LMP of the new residual
                    EDA_TRY(fused_iteration(c, nm, a, pbuf[cur], rtol, it, c.rz_part, d_start));
                    EDA_TRY(lmp_apply(c, EDA_LMP_P, nm, c.pc_r, n, c.pc_z, n, c.pc_status, c.rz_part, true));
                } else {
                    // ring pieces (the flags are indexed by the solve's column)
                    TladArgs t = tlad_args(c, nm, c.pc_members, nullptr);
                    t.obs = c.hv_obs;
                    const int sh = set_pieces(c, t, (long long)(sc.count > 0 ? sc.count : nm) * P, P);
                    if (sh < 0) return EDA_ERR_UNSUPPORTED;
                    t.pcg.members = c.pc_members;
                    t.pcg.b = c.b;
                    t.pcg.x = c.pc_x;
                    t.pcg.r = c.pc_r;
                    t.pcg.z = c.pc_z;
                    t.pcg.p = pbuf[cur];
                    t.pcg.p_out = pbuf[cur ^ 1];
                    t.pcg.q = c.pc_q;
                    t.pcg.pq_part = c.pc_pqp;
                    t.pcg.scal = c.pc_scal;
                    t.pcg.status = c.pc_status;
                    t.pcg.iters = c.pc_iters;
                    t.pcg.it = it;
                    t.pcg.first = it == 1 ? 1 : 0;
                    {  // r^T z from the LMP's row-block sums
                        int rows_, nrb_;
                        lmp_blocks(n, &rows_, &nrb_);
                        t.pcg.rz_part = c.rz_part;
                        t.pcg.rz_ld = (nm + 15) / 16 * 16;
                        t.pcg.rz_nrb = nrb_;
                    }
                    t.pcg.start = d_start;
                    EDA_TRY(run_tlad(c, t, sh ? TLAD_SPLIT_SH : TLAD_SPLIT, false, &sc));
                    LmpFin f{};
                    f.q = c.pc_q;
                    f.p = pbuf[cur ^ 1];
                    f.pq_part = c.pc_pqp;
                    f.b = c.b;
                    f.members = c.pc_members;
                    f.x = c.pc_x;
                    f.scal = c.pc_scal;
                    f.hist = a.hist;
                    f.iters = c.pc_iters;
                    f.pieces = P;
                    f.it = it;
                    f.start = d_start;
                    f.hist_cap = c.hist_cap;
                    f.rtol = rtol;
                    f.rr_part = c.lmp_fin;
                    f.xbr_part = c.lmp_fin + lmp_fin_doubles(c.max_cols) / 2;
                    EDA_TRY(lmp_update(c, nm, f));
                    cur ^= 1;
                }
            } else if (fused) {
                // one launch: p = z + beta p, q = (I + A) p, alpha, x, r, convergence
                EDA_TRY(fused_iteration(c, nm, a, c.pc_p, rtol, it));
                if (use_lmp) EDA_TRY(lmp_apply(c, EDA_LMP_P, nm, c.pc_r, n, c.pc_z, n, c.pc_status, nullptr, true));
            } else {
                EDA_TRY(hessvec(c, c.pc_members, nm, c.pc_p, n, c.pc_q, n, EDA_HV_ADD_IDENTITY, c.pc_status));
                HIP_TRY(launch_pcg_alpha(s, a, it));
                if (use_lmp) EDA_TRY(lmp_apply(c, EDA_LMP_P, nm, c.pc_r, n, c.pc_z, n, c.pc_status, nullptr, true));
                HIP_TRY(launch_pcg_beta(s, a));
            }
            if (it % check_every == 0 || it == maxit) {
                if (ck_issued - ck_done >= Ctx::CK_SLOTS) EDA_TRY(consume(true));
                const int slot = ck_issued % Ctx::CK_SLOTS;
                HIP_TRY(hipMemcpyAsync(c.h_ck + (size_t)slot * c.max_cols, c.pc_status, sizeof(int32_t) * nm,
                                       hipMemcpyDeviceToHost, s));
                HIP_TRY(hipEventRecord(c.ck_ev[slot], s));
                ck_iter.push_back(it);
                ck_issued++;
                int r;
                while (ck_done < ck_issued && (r = consume(false)) == 1) {
                }
                if (ck_done < ck_issued) EDA_TRY(r);
                while (ck_issued - ck_done > max_ahead) EDA_TRY(consume(true));
                if (none_running) {
                    stopped_early = true;
                    break;
                }
            }
        }
        // the remaining checkpoints decide whether every column stopped
        while (ck_done < ck_issued) EDA_TRY(consume(true));
        stopped_early = none_running;
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
    if (use_lmp) {  // the exchange's or the LMP tile barriers' waits
        int32_t err = 0;
        EDA_TRY(sync_read(c, &err, c.xch_err, sizeof(int32_t)));
        if (err != 0) warn = EDA_ERR_SYNC;
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
        case EDA_FIELD_SKETCH_INFO:
            *byte_offset = (size_t)(reinterpret_cast<const char *>(c.sk_info) - c.ws);
            *count = 6;
            return EDA_OK;
        default: return EDA_ERR_INVALID_ARG;
    }
    *byte_offset = (size_t)(reinterpret_cast<const char *>(ptr) - c.ws);
    *count = cnt;
    return EDA_OK;
}

int eda_profile(eda_ctx *h, int32_t every) {
    if (!h || every < 0) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    HIP_TRY(hipStreamSynchronize(c.stream));
    c.prof = every;
    c.prof_seen = 0;
    c.prof_launches = 0;
    c.ev_used = 0;
    return EDA_OK;
}

int eda_profile_select(eda_ctx *h, int32_t kind) {
    if (!h || (kind != EDA_PROF_TLAD && kind != EDA_PROF_UB_GEMM && kind != EDA_PROF_TLAD_ALL))
        return EDA_ERR_INVALID_ARG;
    h->c.prof_kind = kind;
    return EDA_OK;
}

int eda_profile_read(eda_ctx *h, int64_t *timed, int64_t *launches, double *timed_ms) {
    if (!h || !timed || !launches || !timed_ms) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    HIP_TRY(hipStreamSynchronize(c.stream));
    double tot = 0.0;
    for (size_t i = 0; i + 1 < c.ev_used; i += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c.ev[i], c.ev[i + 1]));
        tot += ms;
    }
    *timed = c.prof_launches;
    *launches = c.prof_seen;
    *timed_ms = tot;
    return EDA_OK;
}

int eda_set_geometry(eda_ctx *h, int32_t waves, int32_t tb) {
    if (!h || waves < 0 || tb < 0) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (waves != 0 && !tlad_waves_ok(c.n, waves)) return EDA_ERR_UNSUPPORTED;
    const TladGeom g = tlad_geometry(c.n, waves);
    if (tb > g.tb) return EDA_ERR_UNSUPPORTED;
    c.geo_waves = waves;
    c.geo_tb = tb;
    return EDA_OK;
}

int eda_set_exchange(eda_ctx *h, int32_t mode, int64_t spin_limit) {
    if (!h || (mode != EDA_XCH_ON && mode != EDA_XCH_OFF && mode != EDA_XCH_OBS)) return EDA_ERR_INVALID_ARG;
    h->c.xch_mode = mode;
    h->c.xch_spin = spin_limit < 0 ? -1 : (long long)spin_limit;
    return EDA_OK;
}

int eda_set_lmp_form(eda_ctx *h, int32_t form) {
    if (!h || (form != EDA_LMP_FORM_TWO && form != EDA_LMP_FORM_ONE)) return EDA_ERR_INVALID_ARG;
    h->c.lmp_form = form;
    return EDA_OK;
}

int eda_set_split(eda_ctx *h, int32_t pieces) {
    if (!h) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (pieces < 0 || pieces > SPLIT_PMAX) return EDA_ERR_INVALID_ARG;
    if (c.cfg.ub_mode != EDA_UB_BANDED) return EDA_ERR_UNSUPPORTED;
    if (pieces > 1 && tlad_split_ring(c.n, c.N, c.band_hi, pieces) == 0 &&
        !(c.xch_flags && tlad_split_ring_sh(c.n, c.N, c.band_hi, pieces) > 0))
        return EDA_ERR_UNSUPPORTED;
    c.split_force = pieces;
    return EDA_OK;
}

int eda_destroy(eda_ctx *h) {
    if (!h) return EDA_ERR_INVALID_ARG;
    for (hipEvent_t e : h->c.ev) (void)hipEventDestroy(e);
    if (h->c.h_ck) {
        (void)hipStreamSynchronize(h->c.stream);
        (void)hipHostFree(h->c.h_ck);
    }
    for (hipEvent_t e : h->c.ck_ev)
        if (e) (void)hipEventDestroy(e);
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
        case EDA_ERR_SYNC: return "a wait between exchanging wave pieces gave up, or workgroups ran on unexpected XCDs";
        case EDA_WARN_NOT_CONVERGED: return "some members did not converge";
        default: return "unknown status";
    }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent problems of uneven n, window length and ensemble
// size: the Gamma sketches of every problem, their Nystrom cores and the
// LMP-PCG solves of every member, replayed as one captured graph.  Problems
// with the same n form a class; each class has one multi-problem sketch launch
// and one persistent solve launch (k_solve, a work queue over the class's
// member columns), and the classes run as parallel branches of the graph.
// ---------------------------------------------------------------------------
struct eda_batch {
    std::vector<Ctx *> probs;
    std::vector<eda_ctx *> handles;
    hipStream_t user = nullptr;    // the caller's stream (ordering only)
    hipStream_t stream = nullptr;  // the batch's own capture stream
    hipEvent_t entry = nullptr;
    char *ws = nullptr;
    TladArgs *d_solve = nullptr, *d_hv = nullptr;
    SolveTask *d_stasks = nullptr, *d_htasks = nullptr;
    int *d_counters = nullptr;            // SOLVE_QUEUES queue counters
    int *d_qoff = nullptr;                // SOLVE_QUEUES + 1 queue offsets
    TladGeom *d_geom = nullptr;           // solve geometry of each problem
    RedoJob *d_redo = nullptr;            // last Nystrom pass of every problem (in the sketch launch)
    int *d_done = nullptr;                // finished sketch columns per problem
    int solve_waves = 0, solve_grid = 0;  // the one persistent solve launch
    int sketch_grid = 0;                  // the one persistent sketch launch (solve_waves waves)
    size_t sketch_lds = 0;
    size_t solve_lds = 0;
    const int32_t **d_infoptr = nullptr;  // each problem's sketch outcome slots
    int32_t *d_flags = nullptr;           // gathered sketch states, two per problem
    int32_t *d_titer = nullptr;           // iterations of each solve task in the last call
    std::vector<SolveTask> stasks;        // solve tasks in queue order
    std::vector<int> qoff;                // host copy of d_qoff
    double last_ms[3] = {0.0, 0.0, 0.0};  // sketch launch, prelude, solve launch (one graph)
    long long *d_stamps = nullptr;        // clock at the graph's start, before the sketch, before and after the solve
    double clock_khz = 0.0;               // rate of that clock
    struct Class {
        int n = 0;
        std::vector<int> members;  // problem indices
        int s_cnt = 0, h_off = 0, h_cnt = 0;
        TladGeom g{};   // sketch-product geometry (tuned)
        TladGeom gs{};  // solve geometry (the launch's common waves)
        size_t lds_solve = 0, lds_hv = 0;
        double tune_us = 0.0;
        std::vector<std::pair<TladGeom, float>> timed;  // tuner candidates and their times
    };
    std::vector<Class> classes;
    std::vector<int> ell;
    bool tuned = false;
    int k_cap = -1, maxit = -1, use_lmp = -1;
    double rtol = -1.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

struct BatchPlan {
    size_t off_solve, off_hv, off_st, off_ht, off_cnt, off_qoff, off_geom, off_redo, off_iptr, off_flags, off_titer,
        off_stamps, off_done, total;
};

BatchPlan batch_plan(eda_ctx *const *ctxs, int np) {
    Layout lay;
    BatchPlan P{};
    size_t st = 0, ht = 0;
    for (int i = 0; i < np; i++) {
        const Ctx &c = ctxs[i]->c;
        st += (size_t)c.L + 1;
        ht += (size_t)(c.max_ell < c.L ? c.max_ell : c.L);
    }
    P.off_solve = lay.take(sizeof(TladArgs) * np);
    P.off_hv = lay.take(sizeof(TladArgs) * np);
    P.off_st = lay.take(sizeof(SolveTask) * (st ? st : 1));
    P.off_ht = lay.take(sizeof(SolveTask) * (ht ? ht : 1));
    P.off_cnt = lay.take(sizeof(int) * (SOLVE_QUEUES + 1));
    P.off_qoff = lay.take(sizeof(int) * (SOLVE_QUEUES + 1));
    P.off_geom = lay.take(sizeof(TladGeom) * np);
    P.off_redo = lay.take(sizeof(RedoJob) * np);
    P.off_iptr = lay.take(sizeof(int32_t *) * np);
    P.off_flags = lay.take(2 * sizeof(int32_t) * np);
    P.off_titer = lay.take(2 * sizeof(int32_t) * (st ? st : 1));
    P.off_stamps = lay.take(4 * sizeof(long long));
    P.off_done = lay.take(sizeof(int) * np);
    P.total = lay.total;
    return P;
}

// Device argument blocks of problem i: solve (PCG of members 0..L) and sketch
// (ell columns of Phi on the control trajectory).
void batch_args(eda_batch &b, int i, TladArgs &sa, TladArgs &ha) {
    Ctx &c = *b.probs[i];
    sa = tlad_args(c, c.L + 1, c.pc_members, nullptr);
    sa.obs = c.hv_obs;
    sa.pcg.members = c.pc_members;
    sa.pcg.b = c.b;
    sa.pcg.x = c.pc_x;
    sa.pcg.r = c.pc_r;
    sa.pcg.z = b.use_lmp ? c.pc_z : c.pc_r;
    sa.pcg.p = c.pc_p;
    sa.pcg.scal = c.pc_scal;
    sa.pcg.status = c.pc_status;
    sa.pcg.iters = c.pc_iters;
    sa.pcg.hist = nullptr;
    sa.pcg.hist_cap = c.hist_cap;
    sa.pcg.rtol = b.rtol;
    sa.pcg.maxit = b.maxit;
    sa.pcg.lmp_s = c.sk_s;
    sa.pcg.lmp_c = c.sk_coef;
    sa.pcg.lmp_k = b.use_lmp ? b.ell[i] : 0;
    sa.pcg.lmp_info = b.use_lmp ? c.sk_info + 4 : nullptr;  // set by the shifted redo
    ha = tlad_args(c, b.ell[i], c.zero_members, nullptr);
    ha.V = c.sk_phi;
    ha.ldv = c.n;
    ha.obs = c.hv_obs;
    ha.lam = c.sk_y;
    ha.ldl = c.n;
    ha.add_identity = 0;
}

int batch_class_lds(eda_batch &b, eda_batch::Class &k, const TladGeom &g, size_t &lds_solve, size_t &lds_hv) {
    lds_solve = lds_hv = 0;
    for (int i : k.members) {
        TladArgs sa, ha;
        batch_args(b, i, sa, ha);
        size_t a1 = tlad_lds_bytes(sa, g, TLAD_PCG), a2 = tlad_lds_bytes(ha, g, TLAD_HV);
        if (a1 > lds_solve) lds_solve = a1;
        if (a2 > lds_hv) lds_hv = a2;
    }
    return (lds_solve + 4096 <= 160 * 1024 && lds_hv <= 160 * 1024) ? EDA_OK : EDA_ERR_UNSUPPORTED;
}

// Dynamic LDS and grid of the one persistent solve launch from the classes'
// solve geometries; each class's sketch LDS from its sketch geometry.
int batch_solve_layout(eda_batch &b) {
    size_t lds = 0, slds = 0;
    int cols = 0, scols = 0;
    for (auto &k : b.classes) {
        size_t ls, lh, ls2, lh2;
        EDA_TRY(batch_class_lds(b, k, k.g, ls, lh));
        EDA_TRY(batch_class_lds(b, k, k.gs, ls2, lh2));
        k.lds_hv = lh;
        k.lds_solve = ls2;
        if (ls2 > lds) lds = ls2;
        cols += k.s_cnt;
        // the sketch launch: columns on the solve geometry, and the last Nystrom pass
        if (lh2 > slds) slds = lh2;
        for (int i : k.members) {
            const size_t r = redo_lds(b.ell[i]);
            if (r > slds) slds = r;
            scols += b.ell[i];
        }
    }
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int per_cu = solve_blocks_per_cu(b.solve_waves, lds);
    const int grid = (per_cu > 0 ? per_cu : 1) * cus;
    b.solve_lds = lds;
    b.solve_grid = grid < cols ? grid : cols;
    const int sper_cu = sketch_blocks_per_cu(b.solve_waves, slds);
    const int sgrid = (sper_cu > 0 ? sper_cu : 1) * cus;
    b.sketch_lds = slds;
    b.sketch_grid = sgrid < scols ? sgrid : scols;
    return EDA_OK;
}

// Solve geometry of every class for a common number of waves W: the fastest
// timed candidate with W waves, else the default time block for W.
bool batch_solve_geometry(eda_batch &b, int W) {
    for (auto &k : b.classes) {
        if (!tlad_waves_ok(k.n, W)) return false;
        float best = 1e30f;
        TladGeom g = tlad_geometry(k.n, W);
        for (const auto &c : k.timed)
            if (c.first.waves == W && c.second < best) {
                best = c.second;
                g = c.first;
            }
        size_t ls, lh;
        if (batch_class_lds(b, k, g, ls, lh) != EDA_OK) return false;
        k.gs = g;
    }
    b.solve_waves = W;
    return true;
}

// Autotuner: per class, time the multi-problem sketch launch for each
// candidate geometry (waves per workgroup around the default, time-block
// length at its maximum and at half) and keep the fastest for the sketch.
// The solve is one launch for all classes, so it takes one number of waves:
// that of the class with the most work (members x window x n), each class
// with its fastest time block at that width (8 waves where that width does
// not fit every class).  The persistent grid is what the CUs hold.
int batch_tune(eda_batch &b) {
    hipStream_t s = b.stream;
    for (size_t i = 0; i < b.probs.size(); i++)
        HIP_TRY(launch_gamma(s, b.probs[i]->n, b.ell[i], b.probs[i]->b, b.probs[i]->sk_phi));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return EDA_ERR_HIP;
    }
    int rc = EDA_OK;
    for (auto &k : b.classes) {
        const TladGeom g0 = tlad_geometry(k.n, 0);
        double best = 1e300;
        k.timed.clear();
        for (int w : {g0.waves / 2, g0.waves, g0.waves * 2}) {
            if (w < 1 || !tlad_waves_ok(k.n, w)) continue;
            const TladGeom gw = tlad_geometry(k.n, w);
            for (int tb : {gw.tb, gw.tb / 2}) {
                if (tb < 1) continue;
                const TladGeom g = tlad_geometry(k.n, w, tb);
                size_t ls, lh;
                if (batch_class_lds(b, k, g, ls, lh) != EDA_OK) continue;
                if (launch_hv_multi(s, b.d_hv, b.d_htasks + k.h_off, k.h_cnt, g, lh) != hipSuccess) continue;
                if (hipEventRecord(e0, s) != hipSuccess) { rc = EDA_ERR_HIP; break; }
                for (int r = 0; r < 3; r++)
                    if (launch_hv_multi(s, b.d_hv, b.d_htasks + k.h_off, k.h_cnt, g, lh) != hipSuccess) rc = EDA_ERR_HIP;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) rc = EDA_ERR_HIP;
                if (rc != EDA_OK) break;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                k.timed.push_back({g, ms});
                if (ms < best) {
                    best = ms;
                    k.g = g;
                }
            }
            if (rc != EDA_OK) break;
        }
        if (rc != EDA_OK) break;
        if (best >= 1e300) {
            rc = EDA_ERR_UNSUPPORTED;
            break;
        }
        k.tune_us = 1e3 * best / 3.0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != EDA_OK) return rc;
    const eda_batch::Class *big = nullptr;
    double most = -1.0;
    for (const auto &k : b.classes) {
        double w = 0.0;
        for (int i : k.members) w += (b.probs[i]->L + 1.0) * b.probs[i]->N * k.n;
        if (w > most) {
            most = w;
            big = &k;
        }
    }
    if (!batch_solve_geometry(b, big->g.waves) && !batch_solve_geometry(b, 8)) return EDA_ERR_UNSUPPORTED;
    b.tuned = true;
    return EDA_OK;
}

// Enqueue the batch's sketches (Gamma, products, Nystrom cores) and the
// gathering of their Cholesky outcomes on b.stream (captured by the caller).
// Queue layout of the next persistent solve.  The tasks are grouped by
// problem and the problems dealt to the SOLVE_QUEUES queues, largest total
// cost first, each onto the queue with the least cost so far.  Inside a queue
// the problems come by decreasing cost of their costliest column and each
// problem's columns by decreasing cost, so the longest columns start first.
// cost[t] belongs to b.stasks[t].  b.stasks and b.qoff are rewritten and
// uploaded on b.stream (the caller synchronises).
int batch_schedule(eda_batch &b, const std::vector<long long> &cost) {
    using Item = std::pair<long long, SolveTask>;
    const int np = (int)b.probs.size();
    std::vector<std::vector<Item>> cols(np);
    std::vector<long long> total(np, 0), top(np, 0);
    for (size_t t = 0; t < b.stasks.size(); t++) {
        const int p = b.stasks[t].prob;
        cols[p].push_back({cost[t], b.stasks[t]});
        total[p] += cost[t];
        top[p] = std::max(top[p], cost[t]);
    }
    for (auto &v : cols)
        std::stable_sort(v.begin(), v.end(), [](const Item &x, const Item &y) {
            if (x.first != y.first) return x.first > y.first;
            return x.second.col < y.second.col;
        });
    std::vector<int> by_total;
    for (int p = 0; p < np; p++)
        if (!cols[p].empty()) by_total.push_back(p);
    std::stable_sort(by_total.begin(), by_total.end(), [&](int x, int y) { return total[x] > total[y]; });
    long long load[SOLVE_QUEUES] = {};
    std::vector<std::vector<int>> queue(SOLVE_QUEUES);
    for (int p : by_total) {
        int q = 0;
        for (int r = 1; r < SOLVE_QUEUES; r++)
            if (load[r] < load[q]) q = r;
        load[q] += total[p];
        queue[q].push_back(p);
    }
    std::vector<SolveTask> out;
    out.reserve(b.stasks.size());
    b.qoff.assign(SOLVE_QUEUES + 1, 0);
    for (int q = 0; q < SOLVE_QUEUES; q++) {
        b.qoff[q] = (int)out.size();
        std::stable_sort(queue[q].begin(), queue[q].end(), [&](int x, int y) { return top[x] > top[y]; });
        for (int p : queue[q])
            for (const Item &it : cols[p]) out.push_back(it.second);
    }
    b.qoff[SOLVE_QUEUES] = (int)out.size();
    if (out.size() != b.stasks.size()) return EDA_ERR_INVALID_ARG;
    b.stasks = out;
    HIP_TRY(hipMemcpyAsync(b.d_stasks, b.stasks.data(), sizeof(SolveTask) * b.stasks.size(), hipMemcpyHostToDevice,
                           b.stream));
    HIP_TRY(hipMemcpyAsync(b.d_qoff, b.qoff.data(), sizeof(int) * b.qoff.size(), hipMemcpyHostToDevice, b.stream));
    return EDA_OK;
}

// Expected cost of one iteration of a column of problem p: window steps x
// points per lane of its solve geometry (all classes share the waves).
long long batch_step_cost(const eda_batch &b, int p) {
    for (const auto &k : b.classes)
        if (k.n == b.probs[p]->n) return (long long)b.probs[p]->N * k.gs.q;
    return b.probs[p]->N;
}

// The sketch launch's arguments.
SolveSketch batch_sketch(const eda_batch &b) {
    SolveSketch k{};
    k.hv = b.d_hv;
    k.core = b.d_redo;
    k.done = b.d_done;
    return k;
}

// Enqueue one call's work on b.stream (captured into one graph): with the
// LMP, the prelude (Gamma of every problem, the per-call resets) and one
// persistent sketch launch -- (problem, column) tasks, each problem's last
// Nystrom pass on the workgroup that finishes its last column; then the one
// persistent solve launch over the member columns of every class; then each
// task's iterations and status and each problem's sketch state, gathered for
// one read.  Clock stamps at the start and around the launches.
int batch_enqueue(eda_batch &b) {
    hipStream_t s = b.stream;
    const int np = (int)b.probs.size();
    HIP_TRY(launch_stamp(s, b.d_stamps + 0));
    HIP_TRY(launch_fill_int(s, SOLVE_QUEUES + 1, 0, b.d_counters));
    if (b.use_lmp) {
        const SolveSketch sk = batch_sketch(b);
        HIP_TRY(launch_solve_prelude(s, np, b.d_solve, sk));
        HIP_TRY(launch_stamp(s, b.d_stamps + 1));
        int nh = 0;
        for (const auto &k : b.classes) nh += k.h_cnt;
        HIP_TRY(launch_sketch(s, b.d_geom, b.d_htasks, nh, b.d_counters + SOLVE_QUEUES, b.solve_waves, b.sketch_lds,
                              b.sketch_grid, sk));
    } else {
        HIP_TRY(launch_stamp(s, b.d_stamps + 1));
    }
    HIP_TRY(launch_stamp(s, b.d_stamps + 2));
    HIP_TRY(launch_solve(s, b.d_solve, b.d_geom, b.d_stasks, (int)b.stasks.size(), b.d_qoff, b.d_counters,
                         b.solve_waves, b.solve_lds, b.solve_grid));
    HIP_TRY(launch_stamp(s, b.d_stamps + 3));
    HIP_TRY(launch_task_iters(s, (int)b.stasks.size(), b.d_solve, b.d_stasks, b.d_titer));
    if (b.use_lmp) HIP_TRY(launch_gather_info(s, np, b.d_infoptr, b.d_flags));
    return EDA_OK;
}

void batch_free_graph(eda_batch &b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
}

// Capture what `enqueue` puts on b.stream into an instantiated graph.
int batch_capture(eda_batch &b, int (*enqueue)(eda_batch &), hipGraph_t &graph, hipGraphExec_t &exec) {
    const int np = (int)b.probs.size();
    std::vector<hipStream_t> saved(np);
    for (int i = 0; i < np; i++) saved[i] = b.probs[i]->stream;
    HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(b);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b.stream, &g);
    for (int i = 0; i < np; i++) b.probs[i]->stream = saved[i];
    if (rc != EDA_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != EDA_OK ? rc : EDA_ERR_HIP;
    }
    graph = g;
    if (hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        graph = nullptr;
        exec = nullptr;
        return EDA_ERR_HIP;
    }
    return EDA_OK;
}

}  // namespace

extern "C" {

int eda_batch_workspace_bytes(eda_ctx *const *ctxs, int32_t np, size_t *bytes) {
    if (!ctxs || np < 1 || !bytes) return EDA_ERR_INVALID_ARG;
    for (int i = 0; i < np; i++)
        if (!ctxs[i]) return EDA_ERR_INVALID_ARG;
    *bytes = batch_plan(ctxs, np).total;
    return EDA_OK;
}

int eda_batch_create(eda_ctx *const *ctxs, int32_t np, void *d_ws, size_t ws_bytes, void *stream, eda_batch **out) {
    if (!ctxs || np < 1 || !d_ws || !out) return EDA_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return EDA_ERR_INVALID_ARG;
    for (int i = 0; i < np; i++) {
        if (!ctxs[i]) return EDA_ERR_INVALID_ARG;
        if (ctxs[i]->c.cfg.ub_mode != EDA_UB_BANDED) return EDA_ERR_UNSUPPORTED;
        for (int j = 0; j < i; j++)
            if (ctxs[j] == ctxs[i]) return EDA_ERR_INVALID_ARG;
    }
    const BatchPlan P = batch_plan(ctxs, np);
    if (ws_bytes < P.total) return EDA_ERR_WORKSPACE;
    eda_batch *b = new (std::nothrow) eda_batch();
    if (!b) return EDA_ERR_INVALID_ARG;
    auto fail = [&](int code) {
        if (b->entry) (void)hipEventDestroy(b->entry);
        if (b->stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return code;
    };
    b->user = reinterpret_cast<hipStream_t>(stream);
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return fail(EDA_ERR_HIP);
    if (hipEventCreateWithFlags(&b->entry, hipEventDisableTiming) != hipSuccess) return fail(EDA_ERR_HIP);
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            return fail(EDA_ERR_HIP);
        b->clock_khz = khz;
    }
    // everything already enqueued on the caller's stream (the problems' set-up) comes first
    if (hipEventRecord(b->entry, b->user) != hipSuccess || hipStreamWaitEvent(b->stream, b->entry, 0) != hipSuccess)
        return fail(EDA_ERR_HIP);
    b->ws = static_cast<char *>(d_ws);
    b->d_solve = reinterpret_cast<TladArgs *>(b->ws + P.off_solve);
    b->d_hv = reinterpret_cast<TladArgs *>(b->ws + P.off_hv);
    b->d_stasks = reinterpret_cast<SolveTask *>(b->ws + P.off_st);
    b->d_htasks = reinterpret_cast<SolveTask *>(b->ws + P.off_ht);
    b->d_counters = reinterpret_cast<int *>(b->ws + P.off_cnt);
    b->d_qoff = reinterpret_cast<int *>(b->ws + P.off_qoff);
    b->d_geom = reinterpret_cast<TladGeom *>(b->ws + P.off_geom);
    b->d_redo = reinterpret_cast<RedoJob *>(b->ws + P.off_redo);
    b->d_done = reinterpret_cast<int *>(b->ws + P.off_done);
    b->d_infoptr = reinterpret_cast<const int32_t **>(b->ws + P.off_iptr);
    b->d_flags = reinterpret_cast<int32_t *>(b->ws + P.off_flags);
    b->d_titer = reinterpret_cast<int32_t *>(b->ws + P.off_titer);
    b->d_stamps = reinterpret_cast<long long *>(b->ws + P.off_stamps);
    for (int i = 0; i < np; i++) {
        b->probs.push_back(&ctxs[i]->c);
        b->handles.push_back(ctxs[i]);
    }
    // classes by n, in increasing n
    std::vector<int> ns;
    for (int i = 0; i < np; i++) {
        bool seen = false;
        for (int v : ns) seen |= v == b->probs[i]->n;
        if (!seen) ns.push_back(b->probs[i]->n);
    }
    std::sort(ns.begin(), ns.end());
    for (int v : ns) {
        eda_batch::Class k;
        k.n = v;
        for (int i = 0; i < np; i++)
            if (b->probs[i]->n == v) k.members.push_back(i);
        k.g = tlad_geometry(v, 0);
        b->classes.push_back(k);
    }
    // member lists 0..L of every problem
    std::vector<int32_t> m;
    for (int i = 0; i < np; i++) {
        Ctx &c = *b->probs[i];
        m.resize(c.L + 1);
        for (int j = 0; j <= c.L; j++) m[j] = j;
        if (hipMemcpyAsync(c.pc_members, m.data(), sizeof(int32_t) * m.size(), hipMemcpyHostToDevice, b->stream) !=
                hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess)
            return fail(EDA_ERR_HIP);
    }
    *out = b;
    return EDA_OK;
}

int eda_batch_solve(eda_batch *b, int32_t k_cap, double rtol, int32_t maxit, int32_t use_lmp,
                    int32_t *h_fallbacks) {
    if (!b || k_cap < 1 || !(rtol >= 0) || maxit < 0) return EDA_ERR_INVALID_ARG;
    const int np = (int)b->probs.size();
    HIP_TRY(hipEventRecord(b->entry, b->user));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->entry, 0));
    const bool same = b->exec && k_cap == b->k_cap && rtol == b->rtol && maxit == b->maxit &&
                      (use_lmp != 0) == (b->use_lmp != 0);
    if (!same) {
        batch_free_graph(*b);
        b->k_cap = k_cap;
        b->rtol = rtol;
        b->maxit = maxit;
        b->use_lmp = use_lmp != 0;
        b->ell.assign(np, 0);
        for (int i = 0; i < np; i++) {
            const Ctx &c = *b->probs[i];
            int l = k_cap < c.L ? k_cap : c.L;
            if (l > c.max_ell) l = c.max_ell;
            b->ell[i] = l;
        }
        // argument blocks and task lists, grouped by class
        std::vector<TladArgs> sa(np), ha(np);
        for (int i = 0; i < np; i++) batch_args(*b, i, sa[i], ha[i]);
        std::vector<SolveTask> st, ht;
        for (auto &k : b->classes) {
            const size_t s0 = st.size();
            k.h_off = (int)ht.size();
            for (int i : k.members) {
                for (int j = 0; j <= b->probs[i]->L; j++) st.push_back(SolveTask{i, j});
                for (int j = 0; j < b->ell[i]; j++) ht.push_back(SolveTask{i, j});
            }
            k.s_cnt = (int)(st.size() - s0);
            k.h_cnt = (int)ht.size() - k.h_off;
        }
        hipStream_t s = b->stream;
        HIP_TRY(hipMemcpyAsync(b->d_solve, sa.data(), sizeof(TladArgs) * np, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->d_hv, ha.data(), sizeof(TladArgs) * np, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->d_htasks, ht.data(), sizeof(SolveTask) * ht.size(), hipMemcpyHostToDevice, s));
        std::vector<const int32_t *> ip(np);
        for (int i = 0; i < np; i++) ip[i] = b->probs[i]->sk_info;
        HIP_TRY(hipMemcpyAsync(b->d_infoptr, ip.data(), sizeof(int32_t *) * np, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!b->tuned) EDA_TRY(batch_tune(*b));
        EDA_TRY(batch_solve_layout(*b));
        std::vector<TladGeom> geo(np);
        for (const auto &k : b->classes)
            for (int i : k.members) geo[i] = k.gs;
        HIP_TRY(hipMemcpyAsync(b->d_geom, geo.data(), sizeof(TladGeom) * np, hipMemcpyHostToDevice, s));
        // every problem's last Nystrom pass runs inside the solve, always
        // (the unshifted factorisations first, the shifts where they fail)
        std::vector<RedoJob> rjobs(np);
        for (int i = 0; i < np; i++) {
            rjobs[i] = redo_job(*b->probs[i], b->ell[i], b->ell[i], EDA_THETA_MID, 2.220446049250313e-16);
            rjobs[i].trigger = nullptr;
        }
        HIP_TRY(hipMemcpyAsync(b->d_redo, rjobs.data(), sizeof(RedoJob) * np, hipMemcpyHostToDevice, s));
        // first queue layout from the expected cost of a column (one
        // iteration each); later calls use the measured cost
        b->stasks = st;
        std::vector<long long> cost0(st.size());
        for (size_t t = 0; t < st.size(); t++) cost0[t] = batch_step_cost(*b, st[t].prob);
        EDA_TRY(batch_schedule(*b, cost0));
        HIP_TRY(hipStreamSynchronize(s));
        EDA_TRY(batch_capture(*b, batch_enqueue, b->graph, b->exec));
    }
    // one graph: the sketch launch (sketch columns, each problem's last
    // Nystrom pass with the shifts where a Cholesky fails; a problem whose
    // shifted pass fails too is solved by plain CG), the solve launch
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    const int nt = (int)b->stasks.size();
    std::vector<int32_t> its(2 * (size_t)nt), flags(2 * (size_t)np, 0);
    long long stamps[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(its.data(), b->d_titer, sizeof(int32_t) * 2 * nt, hipMemcpyDeviceToHost, b->stream));
    if (b->use_lmp)
        HIP_TRY(hipMemcpyAsync(flags.data(), b->d_flags, sizeof(int32_t) * 2 * np, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipMemcpyAsync(stamps, b->d_stamps, sizeof(stamps), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->last_ms[0] = (double)(stamps[2] - stamps[1]) / b->clock_khz;
    b->last_ms[1] = (double)(stamps[1] - stamps[0]) / b->clock_khz;
    b->last_ms[2] = (double)(stamps[3] - stamps[2]) / b->clock_khz;
    int fallbacks = 0, unprec = 0;
    for (int i = 0; b->use_lmp && i < np; i++) {
        Ctx &c = *b->probs[i];
        c.sr_ready = false;
        c.k = b->ell[i];
        c.have_lmp = flags[2 * i + 1] == 0;
        fallbacks += flags[2 * i] != 0;
        unprec += flags[2 * i + 1] != 0;
    }
    // queue layout of the next call from the measured cost of each column
    // (iterations x window length)
    bool not_converged = false;
    for (int t = 0; t < nt; t++)
        if (its[nt + t] != EDA_MEMBER_CONVERGED) not_converged = true;
    std::vector<long long> cost(nt);
    for (int t = 0; t < nt; t++) cost[t] = (long long)its[t] * batch_step_cost(*b, b->stasks[t].prob);
    EDA_TRY(batch_schedule(*b, cost));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (h_fallbacks) {
        h_fallbacks[0] = fallbacks;
        h_fallbacks[1] = unprec;
    }
    return not_converged ? EDA_WARN_NOT_CONVERGED : EDA_OK;
}

int eda_batch_result(eda_batch *b, int32_t p, double *d_DZ, int64_t ldz, int32_t *h_iters, double *h_relres,
                     int32_t *h_status) {
    if (!b || p < 0 || p >= (int)b->probs.size() || !h_iters || !h_relres || !h_status) return EDA_ERR_INVALID_ARG;
    Ctx &c = *b->probs[p];
    if (d_DZ && ldz < c.n) return EDA_ERR_INVALID_ARG;
    const int m = c.L + 1;
    hipStream_t s = b->stream;
    if (d_DZ) HIP_TRY(launch_copy_cols(s, c.n, m, c.pc_x, c.n, d_DZ, ldz));
    std::vector<double> scal(4 * (size_t)m);
    HIP_TRY(hipMemcpyAsync(h_iters, c.pc_iters, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_status, c.pc_status, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(scal.data(), c.pc_scal, sizeof(double) * scal.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int warn = EDA_OK;
    for (int j = 0; j < m; j++) {
        h_relres[j] = scal[4 * j + 2];
        if (h_status[j] != EDA_MEMBER_CONVERGED) warn = EDA_WARN_NOT_CONVERGED;
    }
    return warn;
}

int eda_batch_tuning(eda_batch *b, int32_t cls, int32_t *h_out) {
    if (!b || !h_out) return EDA_ERR_INVALID_ARG;
    if (cls < 0 || cls >= (int)b->classes.size()) return EDA_ERR_INVALID_ARG;
    const auto &k = b->classes[cls];
    h_out[0] = k.n;
    h_out[1] = (int32_t)k.members.size();
    h_out[2] = k.gs.waves;
    h_out[3] = k.gs.q;
    h_out[4] = k.gs.tb;
    h_out[5] = b->solve_grid;
    h_out[6] = k.s_cnt;
    h_out[7] = (int32_t)(k.tune_us + 0.5);
    h_out[8] = k.g.waves;
    h_out[9] = k.g.q;
    h_out[10] = k.g.tb;
    return (int32_t)b->classes.size();
}

int eda_batch_timing(eda_batch *b, double *h_ms) {
    if (!b || !h_ms) return EDA_ERR_INVALID_ARG;
    for (int i = 0; i < 3; i++) h_ms[i] = b->last_ms[i];
    return EDA_OK;
}

int eda_batch_destroy(eda_batch *b) {
    if (!b) return EDA_ERR_INVALID_ARG;
    batch_free_graph(*b);
    if (b->entry) (void)hipEventDestroy(b->entry);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return EDA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned sketch: MLP training and inference kernels behind the C ABI
// ---------------------------------------------------------------------------
namespace {

bool mlp_dims_ok(const eda_mlp_dims *d) {
    return d && d->n >= 4 && d->n <= 4096 && d->hidden >= 1 && d->hidden <= 4096 && d->k >= 1 && d->k <= 32;
}

}  // namespace

extern "C" {

int eda_mlp_param_count(const eda_mlp_dims *d, int64_t *count) {
    if (!mlp_dims_ok(d) || !count) return EDA_ERR_INVALID_ARG;
    *count = mlp_layout(d->n, d->hidden, d->k).total;
    return EDA_OK;
}

int eda_mlp_workspace_bytes(const eda_mlp_dims *d, int32_t batch, size_t *bytes) {
    if (!mlp_dims_ok(d) || batch < 1 || !bytes) return EDA_ERR_INVALID_ARG;
    *bytes = sizeof(float) * mlp_ws_floats(d->n, d->hidden, d->k, batch) + sizeof(double) * (size_t)batch + 256;
    return EDA_OK;
}

int eda_mlp_init(const eda_mlp_dims *d, const float *d_normals, float *d_params, void *stream) {
    if (!mlp_dims_ok(d) || !d_normals || !d_params) return EDA_ERR_INVALID_ARG;
    HIP_TRY(mlp_init(reinterpret_cast<hipStream_t>(stream), d->n, d->hidden, d->k, d_normals, d_params));
    return EDA_OK;
}

int eda_mlp_forward(const eda_mlp_dims *d, int32_t batch, const float *d_params, const float *d_X, float *d_O,
                    void *d_ws, size_t ws_bytes, void *stream) {
    if (!mlp_dims_ok(d) || batch < 1 || !d_params || !d_X || !d_O || !d_ws) return EDA_ERR_INVALID_ARG;
    size_t need = 0;
    EDA_TRY(eda_mlp_workspace_bytes(d, batch, &need));
    if (ws_bytes < need) return EDA_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *ws = static_cast<float *>(d_ws);
    HIP_TRY(mlp_forward(s, d->n, d->hidden, d->k, batch, d_params, d_X, ws));
    const size_t kn = (size_t)d->k * d->n, h = d->hidden;
    HIP_TRY(hipMemcpyAsync(d_O, ws + 4 * h * batch, sizeof(float) * kn * batch, hipMemcpyDeviceToDevice, s));
    return EDA_OK;
}

int eda_mlp_loss_grad(const eda_mlp_dims *d, int32_t batch, const float *d_params, const float *d_X,
                      const float *d_S, const float *d_D, float *d_grad, void *d_ws, size_t ws_bytes, void *stream,
                      double *h_loss) {
    if (!mlp_dims_ok(d) || batch < 1 || !d_params || !d_X || !d_S || !d_D || !d_ws || !h_loss)
        return EDA_ERR_INVALID_ARG;
    size_t need = 0;
    EDA_TRY(eda_mlp_workspace_bytes(d, batch, &need));
    if (ws_bytes < need) return EDA_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *ws = static_cast<float *>(d_ws);
    double *lps = reinterpret_cast<double *>(
        (reinterpret_cast<uintptr_t>(ws + mlp_ws_floats(d->n, d->hidden, d->k, batch)) + 255) & ~uintptr_t(255));
    HIP_TRY(mlp_loss_grad(s, d->n, d->hidden, d->k, batch, d_params, d_X, d_S, d_D, d_grad, ws, lps));
    std::vector<double> l(batch);
    HIP_TRY(hipMemcpyAsync(l.data(), lps, sizeof(double) * batch, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double sum = 0.0;
    for (int b = 0; b < batch; b++) sum += l[b];
    *h_loss = sum / batch;
    return EDA_OK;
}

int eda_mlp_adam(int64_t count, float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step, float lr,
                 float beta1, float beta2, float eps, void *stream) {
    if (count < 1 || !d_params || !d_grad || !d_m || !d_v || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return EDA_ERR_INVALID_ARG;
    HIP_TRY(mlp_adam(reinterpret_cast<hipStream_t>(stream), count, d_params, d_grad, d_m, d_v, step, lr, beta1, beta2,
                     eps));
    return EDA_OK;
}

int eda_mlp_to_bf16(int64_t count, const float *d_params, uint16_t *d_params16, void *stream) {
    if (count < 1 || !d_params || !d_params16) return EDA_ERR_INVALID_ARG;
    HIP_TRY(mlp_to_bf16(reinterpret_cast<hipStream_t>(stream), count, d_params, d_params16));
    return EDA_OK;
}

int eda_mlp_input(eda_ctx *h, float *d_x) {
    if (!h || !d_x) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    HIP_TRY(mlp_normalise(c.stream, c.n, 1, c.b, c.n, d_x));
    return EDA_OK;
}

int eda_mlp_infer(eda_ctx *h, const eda_mlp_dims *d, const uint16_t *d_params16, double *d_Z) {
    if (!h || !mlp_dims_ok(d) || !d_params16 || !d_Z) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    if (d->n != c.n) return EDA_ERR_INVALID_ARG;
    if ((size_t)c.n + 2 * (size_t)d->hidden > (size_t)c.n * c.max_cols) return EDA_ERR_UNSUPPORTED;
    HIP_TRY(mlp_infer_bf16(c.stream, c.n, d->hidden, d->k, d_params16, c.b, d_Z, c.hv_v));
    return EDA_OK;
}

int eda_sketch_learned(eda_ctx *h, const eda_mlp_dims *d, const uint16_t *d_params16, int32_t k, int32_t theta_rule,
                       double *h_eig, double *h_theta, int32_t *h_used) {
    if (!h || !mlp_dims_ok(d) || !d_params16) return EDA_ERR_INVALID_ARG;
    Ctx &c = h->c;
    const int l = d->k;
    if (d->n != c.n || l > c.max_ell || k < 1 || k > l) return EDA_ERR_INVALID_ARG;
    if (theta_rule < EDA_THETA_MID || theta_rule > EDA_THETA_ONE) return EDA_ERR_INVALID_ARG;
    // Phi = CholQR2(MLP(b_0)), directions in sk_phi; the Nystrom of the user-sketch path
    EDA_TRY(eda_mlp_infer(h, d, d_params16, c.sk_phi));
    const size_t ls = (size_t)c.max_ell * c.max_ell;
    int r = cholqr2(c, l, c.sk_phi, c.sk_q, c.sk_small + 7 * ls);
    if (r == EDA_OK) {
        HIP_TRY(launch_copy_cols(c.stream, c.n, l, c.sk_q, c.n, c.sk_phi, c.n));
        r = eda_sketch_evd(h, EDA_SKETCH_USER, c.sk_phi, c.n, l, k, 1, EDA_METHOD_NYSTROM, theta_rule, 0, h_eig,
                           h_theta);
    }
    bool ok = r == EDA_OK;
    if (ok && h_eig)
        for (int i = 0; i < k; i++) ok &= std::isfinite(h_eig[i]);
    if (ok) {
        if (h_used) *h_used = 1;
        return EDA_OK;
    }
    if (r < 0 && r != EDA_ERR_NOT_SPD) return r;
    // fallback: the right-hand-side-difference sketch of the same size
    if (l > c.L) return EDA_ERR_NOT_SPD;
    if (h_used) *h_used = 0;
    return eda_sketch_evd(h, EDA_SKETCH_RHS_DIFF, nullptr, 0, l, k, 1, EDA_METHOD_NYSTROM, theta_rule, 0, h_eig,
                          h_theta);
}

}  // extern "C"
