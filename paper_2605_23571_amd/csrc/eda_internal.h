// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/eda.h"

namespace eda {

// Device-side PCG column state.
// Column states besides the EDA_MEMBER_* outcomes: running, or waiting for a
// free slot (a solve admits more columns than its launches hold as others stop).
enum : int32_t { COL_RUNNING = -1, COL_PENDING = -2 };

// Everything a context knows; device pointers point into the caller's workspace.
struct Layout {
    size_t total = 0;
    size_t take(size_t bytes) {  // 256-byte aligned sub-buffer
        size_t off = total;
        total += (bytes + 255) & ~size_t(255);
        return off;
    }
};

struct Ctx {
    eda_config cfg{};
    int n = 0, N = 0, L = 0, nt = 0, nv = 0, p = 0;
    int max_cols = 0, max_ell = 0;
    int band_lo = 0, band_hi = 0;  // tap offsets of the banded U_B product
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;

    // problem data
    double *ubrow = nullptr, *ub = nullptr, *truth = nullptr, *xb = nullptr, *traj = nullptr;
    uint16_t *ub16 = nullptr;  // dense U_B in BF16 (reduced-precision sketch products)
    float *ub32 = nullptr;     // dense U_B in FP32 (reduced-precision sketch products)
    double *trajx = nullptr;  // trajectory rows s < N, periodically padded for the TL/AD windows
    int ext_len = 0, pad_l = 0;
    double *y = nullptr, *d = nullptr, *b = nullptr, *costc = nullptr, *forcing = nullptr;
    // hessvec scratch
    double *hv_v = nullptr, *hv_obs = nullptr, *hv_lam = nullptr;
    int32_t *zero_members = nullptr;  // max_cols zeros (sketch mode)
    // sketch scratch
    double *sk_phi = nullptr, *sk_y = nullptr, *sk_q = nullptr, *sk_q1 = nullptr, *sk_s = nullptr;
    double *sk_small = nullptr;  // 10 ell x ell matrices
    double *sk_eig = nullptr, *sk_coef = nullptr, *sk_coefu = nullptr;
    int32_t *sk_info = nullptr;
    double *lmp_t = nullptr;   // k x max_cols LMP coefficients S_k^T X
    double *lmp_work = nullptr;  // LMP row-block partial projections
    double *lmp_noalloc = nullptr;  // the same, fixed buffer of eda_lmp_apply_noalloc (this device)
    double *sk_sr = nullptr;     // S_k row-major (n x k), made from sk_s on the first LMP use
    bool sr_ready = false;
    double *splitk = nullptr;  // split-K partial sums
    size_t splitk_elems = 0;
    // pcg scratch
    double *pc_x = nullptr, *pc_r = nullptr, *pc_z = nullptr, *pc_p = nullptr, *pc_q = nullptr;
    double *pc_scal = nullptr;  // per column: rho, bnorm, relres, spare
    int32_t *pc_status = nullptr, *pc_iters = nullptr, *pc_members = nullptr, *pc_start = nullptr;
    double *pc_hist = nullptr;
    int hist_cap = 0;
    // split PCG iterations: second p buffer, the pieces' p^T (I + A) p, the
    // update's per-row-block ||r||^2 and x^T (b + r); compute units of the device
    double *pc_p2 = nullptr, *pc_pqp = nullptr, *lmp_fin = nullptr;
    int num_cus = 0;
    int pad_r = 0;  // right pad of the padded trajectory rows
    // wave pieces with halo exchange: flags and edges (banded, n >= XCH_N_MIN),
    // error word, segments per column, r^T z row-block partials, launch epoch,
    // mode and wait limit (eda_set_exchange)
    unsigned long long *xch_flags = nullptr;  // 8 XCH_GRID_MAX slot flags, then XCH_GRID_MAX claims
    double *xch_edges = nullptr;
    int32_t *xch_err = nullptr, *xch_nseg = nullptr;
    double *rz_part = nullptr;
    unsigned int *lmp_sync = nullptr;  // tile barrier counters of the single-launch LMP (2 x tiles)
    int lmp_form = EDA_LMP_FORM_TWO;
    unsigned long long xch_epoch = 0;
    int xch_mode = EDA_XCH_OBS;
    long long xch_spin = -1;
    int split_force = 0;  // pieces per column forced by eda_set_split (0: automatic)
    // pipelined PCG convergence checks: pinned host slots and their events
    static constexpr int CK_SLOTS = 4;
    int32_t *h_ck = nullptr;  // CK_SLOTS x max_cols statuses (pinned host memory)
    hipEvent_t ck_ev[CK_SLOTS] = {};

    // LMP state
    bool have_lmp = false;
    int k = 0;

    // profiling of the TL/AD kernel inside eda_pcg_solve
    int prof = 0;             // time every prof-th launch of the profiled kind (0: off)
    int prof_kind = EDA_PROF_TLAD;
    int64_t prof_seen = 0;
    bool in_pcg = false;
    int geo_waves = 0, geo_tb = 0;  // TL/AD launch geometry override (0: default)
    std::vector<hipEvent_t> ev;
    int64_t prof_launches = 0;
    size_t ev_used = 0;
};

// ---- launchers (each enqueues on s and returns hipGetLastError()) ----

// Nonlinear RK4 integration, one workgroup per vector, bit-for-bit the order
// of operations documented in l96_nl.hip.  x0: n x nvec (ld n).  If store is
// non-null the states after steps 0..nsteps are written to store[v][s][i];
// xend (optional) receives the final states.
hipError_t launch_nl(hipStream_t s, int n, int nvec, int nsteps, double F, double h, double dt,
                     double c6, const double *x0, double *store, double *xend);
// Truth spin-up start: x = F * 1, x[0] = F + std * z[0].
hipError_t launch_spin_init(hipStream_t s, int n, double F, double std_, const double *z, double *x);

// PCG column state used by the fused PCG kernel (column c of every n-vector
// array starts at c * n; scal holds rho, ||b||, relative residual, spare).
struct PcgCols {
    const int32_t *members;
    const double *b;  // n x (L+1) right-hand sides
    double *x, *r, *z, *p;
    double *scal;
    int32_t *status, *iters;
    double *hist;
    int hist_cap;
    double rtol;
    int it;     // iteration number of this launch (1-based)
    int first;  // 1: p = z, rho = r^T z (first iteration)
    int maxit;  // persistent solve: iteration limit
    // persistent solve: LMP z = r + S diag(coef) S^T r (lmp_k = 0: z = r)
    const double *lmp_s, *lmp_c;
    int lmp_k;
    const int32_t *lmp_info;  // persistent solve: nonzero when the problem's sketch gave no LMP
    // split iteration (TLAD_SPLIT): p is read from p and written to p_out (the
    // pieces of a column read each other's halos), (I + A) p goes to q and the
    // pieces' partial sums of p^T (I + A) p to pq_part[c * pieces + piece]
    double *p_out, *q, *pq_part;
    // r^T z per (row block, column), rz_part[b * rz_ld + c] for b < rz_nrb,
    // left by the LMP launch that made z (summed in block order); null: the
    // kernel sums r^T z over the column itself
    const double *rz_part;
    int rz_ld, rz_nrb;
    // per column: the iteration (of this solve's loop) before the column's
    // first, for columns admitted later; null: every column starts at 1
    const int32_t *start;
};
// One task of a batched persistent launch: problem index and column (a PCG
// member column, or a sketch column).
struct SolveTask {
    int prob, col;
};

// Tangent-linear / adjoint kernel modes.
enum TladMode : int {
    TLAD_RAW = 0,   // V (global) -> TL -> AD -> lambda_0 (global)
    TLAD_ADJ = 1,   // forcing (global) -> AD -> lambda_0 (global)
    TLAD_HV = 2,    // X -> U_B X -> TL -> AD -> U_B lambda_0 (+ X) -> Y, banded U_B in-kernel
    TLAD_PCG = 3,   // one fused PCG iteration per member column (banded U_B), see k_tlad
    TLAD_SPLIT = 4, // the Hessian part of a PCG iteration on pieces of each member column, see tlad_column
    TLAD_SPLIT_HV = 5, // TLAD_HV on pieces of each column (ring, halos and pieces as TLAD_SPLIT)
    TLAD_SPLIT_SH = 6, // TLAD_SPLIT with the pieces of a column sharing its observed increments
    TLAD_SPLIT_HV_SH = 7, // TLAD_SPLIT_HV with the pieces sharing the observed increments
};

// A member column split into P pieces: piece i owns the states
// [i n / P, (i + 1) n / P) and integrates a ring of ceil(n / P) + 2 H points
// around them, H = 12 N + 2 band_hi (the TL/AD dependency cone over the window
// plus U_B on both sides), so its owned outputs are exact.
constexpr int SPLIT_PMAX = 8;
// Columns of a split launch: the running columns only (their workgroups are
// contiguous), in groups of eight whose pieces run eight workgroups apart, so
// a column's pieces share one XCD and the XCDs (dealt workgroups in turn) get
// equal shares (split_slot in l96_tlad.hip).  count = 0: every column of the
// launch (col[i] = i).
constexpr int SPLIT_LIST_MAX = 256;
struct SplitCols {
    int32_t count;
    int16_t col[SPLIT_LIST_MAX];
};
int tlad_split_halo(int N, int band_hi);
int tlad_split_ring(int n, int N, int band_hi, int pieces);  // 0: not possible (ring longer than n)
// Pieces that share the column's observed increments (TLAD_SPLIT_SH): piece i
// writes R^-1 H dx at its owned states only, into the column's one buffer of
// observed increments, then waits for its two neighbours' (one bounded wait
// per launch).  Its TL run then needs exact states on the owned range only
// (left halo 8 N + band_hi, right halo 4 N + band_hi: the TL cone grows 8
// states left and 4 right per step, plus U_B), and its AD run, forced from the
// shared buffer, exact lambda on the owned range widened by band_hi (left halo
// 4 N + band_hi, right 8 N + band_hi).  Both rings hold ceil(n / P) + 12 N +
// 2 band_hi points; the AD ring is the TL ring moved 4 N states right.  Every
// piece is at least 8 N + band_hi states long, so the AD run only reads its
// neighbours' increments.
int tlad_split_halo_sh(int N, int band_hi);                     // left halo of the TL ring
int tlad_split_ring_sh(int n, int N, int band_hi, int pieces);  // 0: not possible

// ---- wave pieces with halo exchange (the Hessian part of a PCG iteration) ----
// Every wave of the launch owns one segment of one running column and runs the
// TL/AD windows of its segment alone; at every time-block boundary (and once
// between the TL and AD runs, and once before the outgoing U_B product) it
// publishes the edges of its owned values to device memory and takes its
// neighbours' edges as its window halos.  The running columns are dealt to the
// XCDs in turn (list index i to XCD i mod 8), and an XCD's wave slots
// (workgroups b = x mod 8, eight waves each) are shared among its columns,
// consecutive slots holding one column's consecutive segments, so that
// neighbours exchange through one XCD's L2.
constexpr int XCH_SEG_MAX = 64;     // segments per column at most
constexpr int XCH_GRID_MAX = 1024;  // workgroups of one launch at most
constexpr int XCH_E_MAX = 160;      // edge width at most (doubles per side)
constexpr int XCH_TB_MAX = 16;      // time-block length at most
constexpr size_t XCH_LDS_MIN = 96 * 1024;  // one workgroup per CU: all of a launch's waves co-resident
constexpr int XCH_N_MIN = 512;      // smaller rings keep the whole-column and ring-piece forms
constexpr long long XCH_SPIN_DEFAULT = 1ll << 21;  // polls of one wait (about a second)
struct XchPlan {
    int ok, q, tb, E, max_seg, grid;
};
// The launch shape for m running columns on `grid` workgroups (0 = none fits):
// the most segments per column whose lengths still cover the edge width, the
// fewest points per lane whose window holds the longest segment and its halos,
// and the longest time block that window allows; the windows must lie inside
// the padded trajectory rows (pad_l, pad_r).
XchPlan xch_plan(int n, int N, int band_hi, int m, int grid, int pad_l, int pad_r);
struct XchArgs {
    unsigned long long *flags;  // one per wave slot (8 per workgroup), monotone over launches
    unsigned long long *claim;  // one per workgroup index: the epoch of the launch that took it
    double *edges;              // per slot: 2 parities x 2 sides x E
    int E, tb, grid, max_seg;
    unsigned long long epoch;   // flag base of this launch; phase k publishes epoch + k + 1
    long long spin_max;         // polls of a wait before it gives up
    int32_t *err;               // set to 1 when a wait gave up, 2 when a workgroup ran on another XCD
    const double *rz_part;      // r^T z per (row block, column): nrb x rz_ld
    int rz_ld, nrb;
    int32_t *nseg;              // segments of each column (written by its first segment)
};
// One wave slot: the index of its column in the launch's list (-1: idle), its
// segment, the column's segment count and the neighbouring slots.
struct XSlot {
    int li, seg, nseg, left, right;
};
__host__ __device__ inline XSlot xch_slot(int slot, int m, int grid, int max_seg) {
    XSlot r{-1, 0, 0, 0, 0};
    const int b = slot >> 3, w = slot & 7, x = b & 7;
    const int slots = ((grid - x + 7) >> 3) * 8;
    const int cols = m > x ? (m - x + 7) >> 3 : 0;
    if (cols == 0) return r;
    int base = slots / cols, extra = slots - base * cols;
    if (base >= max_seg) {
        base = max_seg;
        extra = 0;
    }
    if (base < 1) return r;
    const int ls = (b >> 3) * 8 + w;
    int lc, seg, nseg, start;
    if (ls < extra * (base + 1)) {
        lc = ls / (base + 1);
        seg = ls - lc * (base + 1);
        nseg = base + 1;
        start = lc * (base + 1);
    } else {
        const int l2 = ls - extra * (base + 1);
        lc = extra + l2 / base;
        seg = l2 % base;
        nseg = base;
        start = extra * (base + 1) + (lc - extra) * base;
    }
    if (lc >= cols) return r;
    const int lft = start + (seg + nseg - 1) % nseg, rgt = start + (seg + 1) % nseg;
    r.li = x + 8 * lc;
    r.seg = seg;
    r.nseg = nseg;
    r.left = ((x + 8 * (lft >> 3)) << 3) | (lft & 7);
    r.right = ((x + 8 * (rgt >> 3)) << 3) | (rgt & 7);
    return r;
}

// Arguments of the TL/AD kernel.  Columns with active[c] != COL_RUNNING are
// skipped when active is non-null (TLAD_PCG uses pcg.status instead).
struct TladArgs {
    int n, N, nb;
    double F, dt, h, dt6, dt3;
    int obs_dt, obs_dx, obs_x0, nt, nv;
    double inv_s2;
    const double *trajx;    // padded trajectory rows (see launch_pad_traj)
    long long trajx_stride; // per member
    int ext_len, pad_l;     // row length and left pad of the padded rows
    const int32_t *col_member;
    const int32_t *active;
    const double *V;      // RAW: input increments; HV: input X
    long long ldv;
    double *obs;          // p x nb scratch of observed increments (RAW, HV, PCG)
    const double *force;  // ADJ: p x nb forcing
    double *lam;          // RAW/ADJ: lambda_0; HV: output Y
    long long ldl;
    const double *ubrow;  // HV/PCG: U_B first row and tap range
    int band_lo, band_hi;
    int add_identity;     // HV: Y = U_B lambda_0 + X
    int pieces, ring, halo;  // TLAD_SPLIT: pieces per column, ring length, halo
    // TLAD_SPLIT_SH, TLAD_SPLIT_HV_SH: flags per (column, piece) (SPLIT_PMAX
    // per column), the value this launch raises them to (above every earlier
    // launch's), polls of the wait before it gives up, and the error word it
    // then sets
    unsigned long long *pflags;
    unsigned long long want;
    long long spin_max;
    int32_t *err;
    PcgCols pcg;
};
// Launch geometry of the TL/AD kernel: waves per workgroup, ring segment owned
// per wave, points per lane, time-block length and window offsets.
struct TladGeom {
    int waves, S, q, tb, hl_tl, hl_ad;
};
TladGeom tlad_geometry(int n, int waves_hint, int tb_hint = 0);
// Waves per workgroup the geometry accepts for n (1, 2, 4, 8 with Q <= 9).
bool tlad_waves_ok(int n, int waves);
// Bytes of dynamic LDS one column of this problem needs in the given mode.
size_t tlad_lds_bytes(const TladArgs &a, const TladGeom &g, int mode);
// Persistent batched PCG over ntasks tasks cut into SOLVE_QUEUES queues: queue
// q is tasks [qoff[q], qoff[q+1]) (qoff: SOLVE_QUEUES + 1 ints in device
// memory, 0 = qoff[0] <= ... <= qoff[SOLVE_QUEUES] = ntasks) with counter
// counters[q] (zeroed before the launch).  Workgroup b starts on queue
// b mod SOLVE_QUEUES (its XCD) and moves to the next queues as they run dry;
// each task is a whole LMP-PCG solve of one column (init, iterations,
// in-kernel LMP, final status).  probs and geoms hold one TladArgs and one
// geometry per problem (device memory); every geometry has `waves` waves, and
// lds covers the largest problem's dynamic LDS.
constexpr int SOLVE_QUEUES = 8;
// The sketches of a batch (device memory): a task (p, j) computes column j
// of problem p's Y = A Gamma (hv[p], Gamma already in hv[p].V); the
// workgroup that finishes a problem's last column runs its last Nystrom pass
// (core[p], trigger null).  done[] counts finished columns per problem (zero
// at the start of a launch).
struct RedoJob;
struct SolveSketch {
    const TladArgs *hv;
    const RedoJob *core;
    int *done;
};
hipError_t launch_solve(hipStream_t s, const TladArgs *d_probs, const TladGeom *d_geoms, const SolveTask *d_tasks,
                        int ntasks, const int *d_qoff, int *d_counters, int waves, size_t lds, int grid);
// One persistent launch over the sketch tasks of every problem (tasks: ntasks
// (problem, column) pairs, taken from the end; *d_counter zero before the
// launch); geoms and lds as for launch_solve.
hipError_t launch_sketch(hipStream_t s, const TladGeom *d_geoms, const SolveTask *d_tasks, int ntasks, int *d_counter,
                         int waves, size_t lds, int grid, const SolveSketch &sk);
int sketch_blocks_per_cu(int waves, size_t lds);
// Before the sketch launch: Gamma of every problem (hv[p].V column j =
// b_{j+1} - b_0, b = probs[p].pcg.b, ell[p] = core[p].l columns) and done[] = 0.
hipError_t launch_solve_prelude(hipStream_t s, int np, const TladArgs *d_probs, const SolveSketch &sk);
// Hessian products (banded U_B, HV mode) for a list of (problem, column) tasks
// of problems sharing n: one workgroup per task.
hipError_t launch_hv_multi(hipStream_t s, const TladArgs *d_probs, const SolveTask *d_tasks, int ntasks,
                           const TladGeom &g, size_t lds);
// out[t] = iteration count of task t (probs[tasks[t].prob].pcg.iters[col]),
// out[ntasks + t] = its status (out: 2 ntasks ints).
hipError_t launch_task_iters(hipStream_t s, int ntasks, const TladArgs *d_probs, const SolveTask *d_tasks,
                             int32_t *d_out);
// Workgroups of k_solve (waves waves each) one CU holds with this dynamic LDS.
int solve_blocks_per_cu(int waves, size_t lds);
// Bytes of LDS the last Nystrom pass (nystrom_dev.h) needs for ell <= lmax.
size_t redo_lds(int lmax);
// Pads of the periodic row extension that every wave window of the TL/AD
// kernel fits in without wrapping: window points j in [-pad_l, n + pad_r).
void tlad_pads(int n, int *pad_l, int *pad_r);
// The same, also covering the rings of every split (pieces 2 .. SPLIT_PMAX).
void tlad_pads_split(int n, int N, int band_hi, int *pad_l, int *pad_r);
// waves, tb: geometry override (0: the default for n).
// sc: TLAD_SPLIT only (null: every column).
hipError_t launch_tlad(hipStream_t s, const TladArgs &a, int mode, bool fp32, int waves = 0, int tb = 0,
                       const SplitCols *sc = nullptr);
// The Hessian part of a PCG iteration (as TLAD_SPLIT) on wave pieces with halo
// exchange; pq_part holds XCH_SEG_MAX entries per column.  Slots are numbered
// by virtual workgroup index (the dispatch index with its low three bits
// replaced by the XCD the workgroup runs on), so neighbours share an XCD.
hipError_t launch_tlad_x(hipStream_t s, const TladArgs &a, const XchArgs &x, const XchPlan &pl, const SplitCols &sc);

// U_B first row (closed form) and dense fill.
hipError_t launch_ub_row(hipStream_t s, int n, double sigma_b, double len_b, double *row);
hipError_t launch_ub_row_diffusion(hipStream_t s, int n, double sigma_b, double daley, int steps, double *row);
hipError_t launch_ub_fill(hipStream_t s, int n, const double *row, double *ub);
// Y = U_B X (+ Add) with U_B circulant banded: taps o in [lo, hi], r(|o|).
hipError_t launch_band_conv(hipStream_t s, int n, int nb, int lo, int hi, const double *row,
                            const double *X, long long ldx, double *Y, long long ldy,
                            const double *Add, long long ldadd, const int32_t *active);

// FP64 MFMA GEMM: C = op(A) B (+ Add), col-major.  trans_a: op(A) = A^T with
// A stored K x M.  Split-K (when work is K-long and M, N small) uses `part`
// (>= nsplit * M * N doubles) and a deterministic ordered reduction; rowscale
// (optional, M entries) multiplies row i of the product before Add.
hipError_t gemm_f64(hipStream_t s, bool trans_a, int M, int N, int K, const double *A, long long lda,
                    const double *B, long long ldb, double *C, long long ldc, const double *Add,
                    long long ldadd, const double *rowscale, double *part, size_t part_elems);
size_t gemm_splitk_elems(int M, int N, int K);
// C = sum_z part[z] (+ Add), the nsplit partial products (M x N each, in
// order z = 0, 1, ...) of a split-K GEMM.
hipError_t launch_splitk_reduce(hipStream_t s, int M, int N, int nsplit, const double *part, double *C,
                                long long ldc, const double *Add, long long ldadd);

// Spectral LMP on a block: Y = X + S diag(coef) S^T X (S: n x k column-major,
// Sr: the same row-major, from launch_lmp_rowmajor; X, Y: n x nb); column tiles
// whose members all left the running state are skipped (status may be null).
// work: lmp_work_doubles(n, k, ncols); k <= LMP_K_MAX.
constexpr int LMP_RB_MAX = 16;
constexpr int LMP_K_MAX = 128;
void lmp_blocks(int n, int *rows, int *nrb);
size_t lmp_work_doubles(int n, int k, int ncols);
// Size of the fixed partial-projection buffer of eda_lmp_apply_noalloc and its
// device address on the current device (looked up once per device).
constexpr size_t LMP_NOALLOC_DOUBLES = (size_t)EDA_LMP_NOALLOC_SCRATCH_BYTES / sizeof(double);
hipError_t lmp_noalloc_scratch(double **out);
hipError_t launch_lmp_rowmajor(hipStream_t s, int n, int k, const double *S, double *Sr);
// Tile barrier state of the single-launch LMP: per column tile an arrival and
// a departure counter (zero between launches), the tiles provided, the most
// workgroups that are resident at once (one per CU), the wait bound and the
// error word (set to LMP_SYNC_ERR when a wait gives up).
struct LmpSync {
    unsigned int *arrive, *leave;
    int tiles;
    long long max_blocks, spin_max;
    int32_t *err;
};
constexpr int32_t LMP_SYNC_ERR = 4;
size_t lmp_sync_words(int ncols);
// rz (optional): r^T z per (row block, column) with X = r and Y = z, rz[rb *
// ldw + col], ldw = 16 ceil(nb / 16), summed over the block's rows in a fixed order.
// sync (optional): one launch when the grid fits it, else (and without) two.
hipError_t launch_lmp(hipStream_t s, int n, int k, int nb, const double *S, const double *Sr, const double *coef,
                      const double *X, long long ldx, double *Y, long long ldy, const int32_t *status, double *work,
                      double *rz = nullptr, const LmpSync *sync = nullptr);
// The update half of a split PCG iteration, fused with the LMP of the new
// residual: for every running column, alpha = rho / p^T (I + A) p (rho from
// scal[4c + 3], the pieces' partial sums pq_part), x += alpha p, r -= alpha q,
// z = P r, ||r||, the history entry and the status -- what the fused PCG
// kernel does after its Hessian product.  r, z, x: n x nb (ld n).
struct LmpFin {
    const double *q, *p, *pq_part, *b;
    const int32_t *members;
    double *x, *scal, *hist;
    int32_t *iters;
    int pieces, it, hist_cap;  // pieces = 0: wave pieces, nseg[c] per column (stride XCH_SEG_MAX)
    double rtol;
    double *rr_part, *xbr_part;  // LMP_RB_MAX x ldw each
    const int32_t *nseg;
    const int32_t *start;  // as PcgCols::start
};
size_t lmp_fin_doubles(int ncols);
hipError_t launch_lmp_fin(hipStream_t s, int n, int k, int nb, const double *S, const double *Sr, const double *coef,
                          double *r, double *z, int32_t *status, double *work, const LmpFin &f, double *rz = nullptr,
                          const LmpSync *sync = nullptr);
// BF16-operand, FP32-accumulate GEMM C = A B (+ Add): A in BF16 (M x K,
// column-major), B, C, Add in FP64 (B rounded to BF16 as it is staged).
// part (optional, part_elems doubles): FP64 partials of a K split, taken when
// the output has few tiles and part holds gemm_lowp_splitk_elems(M, N, K).
hipError_t gemm_bf16(hipStream_t s, int M, int N, int K, const unsigned short *A, long long lda, const double *B,
                     long long ldb, double *C, long long ldc, const double *Add, long long ldadd,
                     double *part = nullptr, size_t part_elems = 0);
// The same with FP32 operands (A in FP32, B rounded to FP32 when staged).
hipError_t gemm_f32in(hipStream_t s, int M, int N, int K, const float *A, long long lda, const double *B,
                      long long ldb, double *C, long long ldc, const double *Add, long long ldadd,
                      double *part = nullptr, size_t part_elems = 0);
size_t gemm_lowp_splitk_elems(int M, int N, int K);
hipError_t launch_to_f32(hipStream_t s, long long count, const double *x, float *y);
// ---- learned sketch (MLP) ----
struct MlpLayout {
    long long W1, b1, W2, b2, W3, b3, total;  // offsets in the flat parameter array
};
MlpLayout mlp_layout(int n, int h, int k);
size_t mlp_ws_floats(int n, int h, int k, int B);
hipError_t sgemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, float alpha, const float *A, long long lda,
                 const float *B, long long ldb, float beta, float *C, long long ldc, float *part);
hipError_t mlp_normalise(hipStream_t s, int n, int count, const double *b, long long ldb, float *x);
hipError_t mlp_init(hipStream_t s, int n, int h, int k, const float *z, float *th);
hipError_t mlp_forward(hipStream_t s, int n, int h, int k, int B, const float *th, const float *X, float *ws);
hipError_t mlp_loss_grad(hipStream_t s, int n, int h, int k, int B, const float *th, const float *X,
                         const float *S, const float *D, float *grad, float *ws, double *loss_per_sample);
hipError_t mlp_adam(hipStream_t s, long long count, float *th, const float *g, float *m, float *v, int step, float lr,
                    float b1, float b2, float eps);
hipError_t mlp_to_bf16(hipStream_t s, long long count, const float *th, unsigned short *th16);
hipError_t mlp_infer_bf16(hipStream_t s, int n, int h, int k, const unsigned short *th16, const double *b, double *Z,
                          double *tmp);
// y = bf16(x), round to nearest even.
hipError_t launch_to_bf16(hipStream_t s, long long count, const double *x, unsigned short *y);

// Setup helpers.
hipError_t launch_obs(hipStream_t s, int n, int L, int p, int nv, int obs_dt, int obs_dx, int obs_x0,
                      double sigma_o, const double *truth, const double *eta, double *y);
hipError_t launch_xb(hipStream_t s, int n, int L, const double *xt0, const double *ux, double *xb);
hipError_t launch_innov(hipStream_t s, int n, int N, int L, int p, int nv, int obs_dt, int obs_dx,
                        int obs_x0, double s2, const double *y, const double *traj, double *d,
                        double *force, double *costc);
// Periodic extension of trajectory rows: out[m][s][j] = traj[m][s][(j - pad_l) mod n],
// j < ext_len, for states s < N of each of nm members (input rows N + 1 per member).
// out[2 i], out[2 i + 1] = info[i][5], info[i][4]: the shifts problem i's last
// Nystrom pass took, and whether it ended without an LMP.
hipError_t launch_gather_info(hipStream_t s, int np, const int32_t *const *info, int32_t *out);
// *p = the device's constant-rate clock (wall_clock64) when the kernel runs:
// a timestamp that can sit in a captured graph.
hipError_t launch_stamp(hipStream_t s, long long *p);
// p[0 .. count) = value (a kernel, so that it can sit in a captured graph).
hipError_t launch_fill_int(hipStream_t s, int count, int value, int *p);
hipError_t launch_pad_traj(hipStream_t s, int n, int N, int nm, const double *traj, int pad_l, int ext_len,
                           double *out);
hipError_t launch_gamma(hipStream_t s, int n, int ell, const double *b, double *gam);

// Small dense kernels (one workgroup, ell <= 128, matrices col-major ell x ell).
hipError_t launch_chol_inv(hipStream_t s, int l, const double *W, double shift, double *C,
                           double *Cinv, int32_t *info);
hipError_t launch_sym(hipStream_t s, int l, double *W);
hipError_t launch_small_gemm(hipStream_t s, int l, bool ta, bool tb, const double *A, const double *B,
                             double *C);
hipError_t launch_jacobi_svd_u(hipStream_t s, int l, double *T, double *U, double *sig);
// Operands of one Jacobi SVD: T (l x l) -> U, sig as launch_jacobi_svd_u.
struct JacobiJob {
    int l;
    const double *T;
    double *U, *sig;
};
// Operands of one factorisation: as launch_chol_inv(l, W, shift, C, Cinv, info).
struct CholJob {
    int l;
    const double *W;
    double shift;
    double *C, *Cinv;
    int32_t *info;
};
// The shifted Nystrom sketch of one problem on the device (small_la.hip): from
// Y = A Phi, CholQR2 with the shifted first pass when needed, W = Phi^T Y and
// its Cholesky, the Nystrom shift nu = u ||Y||_F when that fails, then T, its
// SVD, S = Q U(:, 1:k), signs and the LMP coefficients.  With trigger set it
// runs only if one of trigger[0..2] (the unshifted Choleskys) is nonzero.
// state[0] = 1 if it ran, state[1] = 1 if it ran and a Cholesky still failed
// (no LMP), state[2] the shifts it took (bit 0: the trace shift of CholQR3,
// bit 1: the Nystrom shift), state[3] its Cholesky scratch.  small: 10 slots of ls doubles
// (slots as the host path: 0 G, 1 R1 then C^-1, 2 R1^-1 then T, 3 R2 then U,
// 4 R2^-1 then sigma, 5-6 R products, 7 R_Y, 8 W, 9 C).
struct RedoJob {
    int n, l, k, rule;
    double u;                 // unit roundoff of the products that formed Y
    const int32_t *trigger;   // null: always run
    int32_t *state;
    const double *phi;        // n x l
    double *y, *q1, *q2, *q;  // n x l: Y (shifted in place), two scratch bases, Q
    double *s;                // n x k: the Ritz basis
    double *small;
    long long ls;
    double *eig, *coef, *coefu, *theta;
};
hipError_t launch_nystrom_redo(hipStream_t s, const RedoJob &job);
hipError_t launch_jacobi_eig(hipStream_t s, int l, double *T, double *Vwork, double *V, double *lam);
hipError_t launch_fix_signs(hipStream_t s, int n, int k, double *S, long long lds);
hipError_t launch_lmp_coef(hipStream_t s, int k, const double *sig, double nu, int square,
                           int theta_rule, double *eig, double *coef, double *coefu, double *theta_out);
hipError_t launch_axpy_cols(hipStream_t s, int n, int nb, double alpha, const double *X, long long ldx,
                            double *Y, long long ldy);
hipError_t launch_copy_cols(hipStream_t s, int n, int nb, const double *X, long long ldx, double *Y,
                            long long ldy);

// PCG kernels (one workgroup per column).
struct PcgArgs {
    int n, nb;
    const int32_t *members;
    const double *b;  // n x (L+1)
    double *x, *r, *z, *p, *q;
    double *scal;      // 4 per column: rho, bnorm, relres, spare
    int32_t *status, *iters;
    double *hist;
    int hist_cap;
    double rtol;
};
hipError_t launch_pcg_init(hipStream_t s, const PcgArgs &a);
hipError_t launch_pcg_start(hipStream_t s, const PcgArgs &a);
hipError_t launch_pcg_alpha(hipStream_t s, const PcgArgs &a, int it);
hipError_t launch_pcg_beta(hipStream_t s, const PcgArgs &a);
hipError_t launch_pcg_finish(hipStream_t s, const PcgArgs &a);
// For the listed columns whose status is `from`: status = to and, when start
// is given, start[c] = start_it (columns made to wait, or admitted).
hipError_t launch_col_status(hipStream_t s, const SplitCols &cols, int32_t from, int32_t to, int32_t *status,
                             int32_t *start, int32_t start_it);

}  // namespace eda
