// api.hip -- C ABI of the library (declared in include/hsf.h): context and
// buffer management, and the host-side sequencing of the kernels.  Every
// numerical step runs in the kernels of prop.hip, ctl.hip and dyn.hip; the host
// only orders launches and reads the per-replica status between line-search
// trials.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <string>
#include <vector>

#include "hsf_internal.h"
#include "prop_block.h"

using namespace hsf;

struct hsf_ctx {
    int n_rep = 0;
    int precision = HSF_FP64;
    int hydro = 1;
    int noise = 0;                   // HSF_NOISE_* flags
    int lb_all = HSF_LB_BGK;         // collision shared by every replica, -1 when mixed
    unsigned long long noise_step = 0;  // generator step word of the next noise draw
    double *noise_flux = nullptr;    // bond fluxes of the composition noise, 3 nsp T (allocated when first on)
    // Crank-Nicolson diffusion (hsf_set_integrator); buffers of n = nsp T doubles
    int integrator = HSF_CD_EXPLICIT;
    double cn_tol = 1e-10, cn_eta = 1e-3;
    int cn_max_newton = 20, cn_m = 40, cn_alloc_m = 0;
    double *cn_rhs = nullptr, *cn_F = nullptr, *cn_Ft = nullptr, *cn_wbase = nullptr, *cn_half = nullptr;
    double *cn_V = nullptr;          // Krylov basis, (m + 1) n
    double *cn_part = nullptr, *cn_dots = nullptr, *cn_coef = nullptr;
    double *cn_dots_h = nullptr;     // pinned host copy of the dot products
    hsf_cn_stats cn_last{};
    Chain ch{};
    long long T = 0;                 // total sites over all replicas
    std::vector<Rep> reps;
    Rep *rep_d = nullptr;
    RepState *st_d = nullptr;
    RepState *st_h = nullptr;        // pinned mirror for status reads (written by the control kernel)
    RepState *st_hd = nullptr;       // the mirror's device-side address
    RepState *st_save = nullptr;     // device copy of the replica states at the start of a coupled step
    double *w_start = nullptr;       // fields at the start of a coupled step (rollback of a failed step)
    int *bad_h = nullptr;            // pinned flag set by the LB and CD kernels on a non-finite result
    int *bad_hd = nullptr;           // its device-side address
    Plan plan;                       // site plan: kBlock consecutive sites per block
    TileCfg tile{8, 8, 8, 2};        // propagator tile configuration in use
    Plan tplan;                      // tile plan of `tile`
    std::vector<int> tile_blk_first; // host copy of the tile plan's first block per replica
    int max_tile_blocks = 0;         // over every configuration (sizes the partials)
    size_t lds_limit = 65536;
    int tuned = 0;
    hipStream_t stream = nullptr;
    int fields_set = 0;              // fields hold a usable warm start
    std::string err;

    // FP64 state and work arrays
    double *w = nullptr, *phi = nullptr, *phi_tmp = nullptr, *mu = nullptr, *eval_out = nullptr;
    double *g = nullptr, *gt = nullptr, *d = nullptr, *acc = nullptr;
    // LB populations: FP64, or with FP32 propagators FP32 deviations from the rest state
    void *nA = nullptr, *nB = nullptr;
    bool lb32 = false;
    double *lb_stage = nullptr;      // FP64 staging of the populations (FP32 storage; allocated at first use)
    double *rho = nullptr, *u = nullptr, *force = nullptr, *uin = nullptr;
    double *part = nullptr, *partG = nullptr;
    int part_cap = 0;                  // doubles in `part`
    double *obs = nullptr;             // observables scratch; results in its last 3 n_rep doubles
    // propagators in the chosen precision
    void *E = nullptr, *G = nullptr, *Gp0 = nullptr, *Gp1 = nullptr, *Gf0 = nullptr, *Gf1 = nullptr;
    // FP64 propagators of the refinement phase of FP32 contexts (HSF_SOLVER_REFINE)
    int refine = 0;
    bool eval64 = false;               // evaluations currently run in FP64
    void *E64 = nullptr, *G64 = nullptr, *Gp64[2] = {nullptr, nullptr}, *Gf64[2] = {nullptr, nullptr};
    std::vector<void *> allocs;

    // hipGraphs of the fixed launch sequences (captured at first use, replayed after)
    hipStream_t cap_stream = nullptr;  // own stream for capture when the caller's is the null stream
    int use_graphs = 1;
    int poison = 0;                    // new buffers filled with NaN bytes (HSF_POISON=1)
    struct EvPair {
        int kind;
        hipEvent_t a, b;
        bool pooled;                   // return to the pool after reading
    };
    struct GraphSlot {
        hipGraphExec_t exec = nullptr;
        const void *key = nullptr;     // the density buffer the sequence was captured with
        bool key64 = false;            // and whether its evaluations ran in FP64
    };
    enum { GK_START = 0, GK_PASS, GK_EVAL, GK_COUNT };
    // a coupled step rotates the densities among four buffers (current, update, two history
    // entries), so each sequence has one captured variant per density buffer, and one per
    // precision of the evaluations
    static constexpr int kGraphVariants = 8;
    GraphSlot graphs[GK_COUNT][kGraphVariants];
    void drop_graphs()
    {
        for (auto &kind : graphs)
            for (auto &g : kind) {
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
                g.exec = nullptr;
                g.key = nullptr;
                g.key64 = false;
            }
    }

    // optional per-launch timing of the hot kernels with HIP events on the context stream
    // warm starts
    int step_warm = HSF_WARM_CURRENT;  // used by hsf_step
    // converged fields and target densities of the last two inversions ([0] the latest)
    double *w_hist[2] = {nullptr, nullptr}, *phi_hist[2] = {nullptr, nullptr};
    int n_hist = 0;                    // how many of them are valid
    hsf_net *net = nullptr;            // attached network (not owned)
    float *net_in = nullptr;           // network input, [channels][V] per replica, replicas in order
    float *net_pred = nullptr;         // network output, [2][V] per replica
    double *net_rms = nullptr;         // per replica: rms of the density difference
    int net_gate = 0;                  // use the network only after inversions of >= this many iterations
    long long work_evals = 0;          // density-functional evaluations, all replicas
    double work_site_evals = 0.0;      // sum over replicas of evaluations x sites
    int timing = 0;
    std::vector<EvPair> pending;       // recorded, not yet read
    std::vector<hipEvent_t> pool;      // free events
    double tot_ms[HSF_K_COUNT] = {0};
    long long tot_cnt[HSF_K_COUNT] = {0};
    // step log (hsf_set_step_log)
    int step_log = 0;
    long long steps_done = 0;          // successful coupled steps
    std::deque<hsf_step_record> log;
    hipEvent_t log_ev[3] = {nullptr, nullptr, nullptr};   // step start, inversion done, dynamics done
    double *log_d = nullptr;           // device: 4 doubles per replica
    std::vector<hsf_invert_stats> log_inv;   // the step's inversion, per replica
    std::vector<double> log_lnq;
};

namespace {

int fail(hsf_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(c, expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((c), HSF_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

int dalloc(hsf_ctx *c, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(c, HSF_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    c->allocs.push_back(*p);
    if (c->poison && (e = hipMemset(*p, 0xff, bytes)) != hipSuccess)
        return fail(c, HSF_EHIP, "hipMemset failed: %s", hipGetErrorString(e));
    return HSF_OK;
}

// Tensor-product reading of the 27-point linkage stencil from the segment length:
// 1-D kernel [al, 1 - 2 al, al] with al = a^2 / 6 (normalised, per-axis variance a^2/3).
void weights_from_segment(double a, double c[4])
{
    const double al = a * a / 6.0, m = 1.0 - 2.0 * al;
    c[0] = m * m * m;
    c[1] = al * m * m;
    c[2] = al * al * m;
    c[3] = al * al * al;
}

size_t real_size(const hsf_ctx *c) { return c->precision == HSF_FP32 ? sizeof(float) : sizeof(double); }

int copy_in(hsf_ctx *c, double *dst, const double *src, size_t n, int where)
{
    if (!src) return fail(c, HSF_EINVAL, "null input pointer");
    if (where == HSF_DEVICE) {
        HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else if (where == HSF_HOST) {
        HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        return fail(c, HSF_EINVAL, "bad memory location %d", where);
    }
    return HSF_OK;
}

int copy_out(hsf_ctx *c, double *dst, const double *src, size_t n, int where)
{
    if (!dst) return fail(c, HSF_EINVAL, "null output pointer");
    if (where == HSF_DEVICE) {
        HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else if (where == HSF_HOST) {
        HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        return fail(c, HSF_EINVAL, "bad memory location %d", where);
    }
    return HSF_OK;
}

// Read the elapsed times of recorded event pairs (the stream has been synchronised).
int harvest(hsf_ctx *c)
{
    for (auto &m : c->pending) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, m.a, m.b));
        c->tot_ms[m.kind] += ms;
        c->tot_cnt[m.kind] += 1;
        if (m.pooled) {
            c->pool.push_back(m.a);
            c->pool.push_back(m.b);
        }
    }
    c->pending.clear();
    return HSF_OK;
}

int sync(hsf_ctx *c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return harvest(c);
}

// The replicas' states as of the last control kernel: it writes them into the pinned
// mirror st_h itself, so reading them takes a stream synchronisation only.
int read_status(hsf_ctx *c) { return sync(c); }

hipEvent_t new_event(hsf_ctx *c, bool pooled)
{
    if (pooled && !c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Events for one launch of kernel family `kind` (HSF_K_*) when timing is on; the
// launcher hands them to hipExtLaunchKernelGGL, which records them around the
// kernel's own execution.
struct Timed {
    hsf_ctx *c;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(hsf_ctx *c_, int k) : c(c_), kind(k)
    {
        if (!c->timing) return;
        a = new_event(c, true);
        b = new_event(c, true);
        if (!a || !b) a = b = nullptr;
    }
    ~Timed()
    {
        if (a) c->pending.push_back({kind, a, b, true});
    }
};

// Run a fixed launch sequence: captured into a hipGraph at its first use, replayed after.
template <class F>
int run_seq(hsf_ctx *c, int kind, F &&body)
{
    if (!c->use_graphs || c->timing) {   // timing mode launches directly, with events per kernel
        body();
        HIPCHK(c, hipGetLastError());
        return HSF_OK;
    }
    hsf_ctx::GraphSlot *slots = c->graphs[kind];
    int v = 0;
    while (v < hsf_ctx::kGraphVariants && slots[v].exec && (slots[v].key != c->phi || slots[v].key64 != c->eval64))
        ++v;
    if (v == hsf_ctx::kGraphVariants) {   // not reached with the four density buffers; recapture
        v = 0;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        (void)hipGraphExecDestroy(slots[0].exec);
        slots[0].exec = nullptr;
    }
    hsf_ctx::GraphSlot &g = slots[v];
    if (!g.exec) {
        g.key = c->phi;
        g.key64 = c->eval64;
        hipStream_t user = c->stream;
        if (!user && !c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = user ? user : c->cap_stream;
        if (!user) HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        c->stream = cs;
        body();
        c->stream = user;
        hipGraph_t graph = nullptr;
        hipError_t e1 = hipGetLastError();
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e1 != hipSuccess || e2 != hipSuccess)
            return fail(c, HSF_EHIP, "graph capture failed: %s / %s", hipGetErrorString(e1), hipGetErrorString(e2));
        hipError_t e3 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) {
            g.exec = nullptr;
            return fail(c, HSF_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
        }
    }
    HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
    return HSF_OK;
}

template <typename real>
PropBufs<real> bufs(hsf_ctx *c)
{
    PropBufs<real> b;
    if (sizeof(real) == sizeof(double) && c->precision == HSF_FP32) {   // refinement phase
        b.E = (real *)c->E64;
        b.G = (real *)c->G64;
        b.Gp[0] = (real *)c->Gp64[0];
        b.Gp[1] = (real *)c->Gp64[1];
        return b;
    }
    b.E = (real *)c->E;
    b.G = (real *)c->G;
    b.Gp[0] = (real *)c->Gp0;
    b.Gp[1] = (real *)c->Gp1;
    return b;
}

// Real size the tilings must fit in LDS: the context's, or FP64 while refinement is on.
size_t lds_real_size(const hsf_ctx *c) { return c->refine ? sizeof(double) : real_size(c); }

// Blocks of the tile plan of configuration t for every replica.
void tile_blocks(const hsf_ctx *c, const TileCfg &t, std::vector<int> &blk_rep, std::vector<int> &blk_first)
{
    blk_rep.clear();
    blk_first.clear();
    for (int r = 0; r < c->n_rep; ++r) {
        const Rep &R = c->reps[r];
        const long long nb = tile_is_stream(t) ? stream_blocks(t, R.Lx, R.Ly, R.Lz)
                                               : (long long)((R.Lx + t.cx - 1) / t.cx) * ((R.Ly + t.cy - 1) / t.cy) *
                                                     ((R.Lz + t.cz - 1) / t.cz);
        blk_first.push_back((int)blk_rep.size());
        for (long long b = 0; b < nb; ++b) blk_rep.push_back(r);
    }
    blk_first.push_back((int)blk_rep.size());
}

bool tile_known(const TileCfg &t)
{
#define HSF_EQ(CX, CY, CZ, K) \
    if (t.cx == CX && t.cy == CY && t.cz == CZ && t.k == K) return true;
#define HSF_EQS(H, CZ, K) HSF_EQ(64, H, CZ, K)
    HSF_TILE_CONFIGS(HSF_EQ)
    HSF_STREAM_CONFIGS(HSF_EQS)
#undef HSF_EQS
#undef HSF_EQ
    return false;
}

// Make t the configuration in use (device tile plan rebuilt; captured graphs dropped).
int set_tile(hsf_ctx *c, const TileCfg &t)
{
    std::vector<int> br, bf;
    tile_blocks(c, t, br, bf);
    if ((int)br.size() > c->max_tile_blocks) return fail(c, HSF_EINVAL, "tile plan larger than sized for");
    HIPCHK(c, hipMemcpy(c->tplan.blk_rep, br.data(), sizeof(int) * br.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->tplan.blk_first, bf.data(), sizeof(int) * bf.size(), hipMemcpyHostToDevice));
    c->tplan.nblocks = (int)br.size();
    c->tplan.n_rep = c->n_rep;
    c->tile_blk_first = bf;
    set_plan_args(c->tplan, c->reps.data(), c->n_rep, bf.data());
    c->tile = t;
    c->drop_graphs();
    return HSF_OK;
}

// One density-functional evaluation for the active replicas.
//   final_mode 0: densities into out (field layout); 1: gradient phi^t - phi into out
//   (polymer layout) with the partial dot products against d.
// Launches with one-step kernels (K = 0): N forward launches, the first also computing
// the field factors, and N backward launches, the first also computing Q and the last
// normalising.  With blocked kernels: exp of the fields, ceil(N/K) forward launches, the
// Q reduction, ceil(N/K) backward launches.
// Paired kernels (K = -1, N >= 2): N launches, launch j taking forward step j and backward
// step N + 1 + (N mod 2) - j (when in 2..N), then backward step 1 alone, which finishes Q
// and normalises; N + 1 launches instead of 2 N.  A bead's two steps never share a launch
// (the backward lag N mod 2 sees to that), and the forward step of bead s runs first exactly
// when s <= se = (N + N mod 2) / 2.  For even N the backward step N would share launch 1
// with forward step 1, which stores the field factors: with N = 2 it forms its factor from
// the fields itself; with N >= 4 it has no launch of its own, and backward step N - 1
// (launch 2) reads G+_N through its stencil as bead N's stored factor times csum and the
// step-N scale, the values step N would have stored.
// Launch j (1..N) of the paired schedule for chains of N >= 2 beads (host only; the
// schedule's read and write sets are checked on the CPU through hsf_paired_schedule).
PairSteps paired_steps(int N, int j)
{
    const int lag = N & 1, se = (N + lag) / 2;
    PairSteps ps{};
    ps.sf = j;
    const int sb = N + 1 + lag - j;
    ps.sb = (sb >= 2 && sb <= N) ? sb : 0;
    ps.f_late = j > se;
    ps.f_from_pp = j >= 2 && j - 1 >= se;
    ps.f_to_pp = j >= se && j < N;
    const bool fold_n = lag == 0 && N >= 4;   // backward step N folded into step N - 1
    if (fold_n && j == 1) ps.sb = 0;
    ps.g_late = ps.sb && ps.sb <= se;
    ps.g_exp = ps.sb == N && j == 1;
    ps.g_from_e = fold_n && j == 2;
    return ps;
}

// Blocks per replica above which the paired sweeps' last launch does not fold Q itself
// (every block re-sums its replica's row of partials, so the reads grow as the square of
// the blocks): a control launch does.  At 2048 blocks (a 128^3 box in 32x8x4 tiles) the
// fold costs the last launch about 2 us and saves the control launch, about 3 us more.
constexpr int kFoldQMaxBlocks = 2048;

template <typename real>
void run_eval_paired(hsf_ctx *c, int use_alpha, int final_mode, double *out, const double *d, int sums)
{
    PropBufs<real> b = bufs<real>(c);
    const int N = c->ch.N;
    const bool alt = sizeof(real) == sizeof(double) && c->precision == HSF_FP32;   // refinement phase
    real *Gf[2] = {(real *)(alt ? c->Gf64[0] : c->Gf0), (real *)(alt ? c->Gf64[1] : c->Gf1)};
    int parity = 0;
    for (int j = 1; j <= N; ++j) {
        const PairSteps ps = paired_steps(N, j);
        const real *gin = b.Gp[parity ^ 1];
        real *gout = b.Gp[parity];
        if (ps.sb) parity ^= 1;
        Timed t(c, HSF_K_PAIR);
        launch_pair_block<real>(c->tile, c->stream, c->tplan, c->rep_d, c->st_d, c->ch, ps, b, Gf[(j - 1) & 1],
                                Gf[j & 1], gin, gout, c->partG, sums, c->w, c->d, use_alpha, t.a, t.b);
    }
    int most = 0;
    for (int r = 0; r < c->n_rep; ++r) most = std::max(most, c->tile_blk_first[r + 1] - c->tile_blk_first[r]);
    const bool fold = most <= kFoldQMaxBlocks;
    if (!fold)
        launch_reduce_ctl(c->stream, c->n_rep, c->tplan, c->st_d, c->rep_d, c->part, PH_Q, c->ch, c->partG, 0.0, 0,
                          c->st_hd);
    Timed t(c, HSF_K_BWD);
    launch_bwd_block<real>(c->tile, c->stream, c->tplan, c->rep_d, c->st_d, c->ch, 1, 1, b, b.Gp[parity ^ 1],
                           b.Gp[parity], c->acc, final_mode, c->phi, d, out, c->part, c->partG, fold ? 2 : 0, t.a,
                           t.b);
}

// Streaming tilings: field factors, ceil(N/K) forward launches, the Q reduction and
// ceil(N/K) backward launches (steps N, N - K, ...; the last one normalises).
template <typename real>
void run_eval_stream(hsf_ctx *c, int use_alpha, int final_mode, double *out, const double *d, int sums)
{
    PropBufs<real> b = bufs<real>(c);
    const int N = c->ch.N, K = c->tile.k;
    {
        Timed t(c, HSF_K_PREP);
        launch_field_exp<real>(c->stream, c->plan, c->rep_d, c->st_d, c->ch, c->w, c->d, use_alpha, b.E, t.a, t.b);
    }
    for (int s0 = 0; s0 < N; s0 += K) {
        Timed t(c, HSF_K_FWD);
        launch_fwd_stream<real>(c->tile, c->stream, c->tplan, c->rep_d, c->st_d, c->ch, s0, std::min(K, N - s0), b,
                                c->partG, sums, t.a, t.b);
    }
    launch_reduce_ctl(c->stream, c->n_rep, c->tplan, c->st_d, c->rep_d, c->part, PH_Q, c->ch, c->partG, 0.0, 0,
                      c->st_hd);
    int parity = 0;
    for (int s_hi = N; s_hi >= 1; s_hi -= K) {
        Timed t(c, HSF_K_BWD);
        launch_bwd_stream<real>(c->tile, c->stream, c->tplan, c->rep_d, c->st_d, c->ch, s_hi, std::min(K, s_hi), b,
                                b.Gp[parity ^ 1], b.Gp[parity], final_mode, c->phi, d, out, c->part, t.a, t.b);
        parity ^= 1;
    }
}

template <typename real>
void run_eval(hsf_ctx *c, int use_alpha, int final_mode, double *out, const double *d, int sums)
{
    if (tile_is_stream(c->tile)) return run_eval_stream<real>(c, use_alpha, final_mode, out, d, sums);
    if (c->tile.k < 0 && c->ch.N >= 2) return run_eval_paired<real>(c, use_alpha, final_mode, out, d, sums);
    PropBufs<real> b = bufs<real>(c);
    const int N = c->ch.N, K = std::max(1, c->tile.k);
    const bool direct = c->tile.k <= 0;
    const bool fold_q = direct && N > 1;   // with N = 1 step 1 is step N: Q first, in its own launch
    if (!direct) {
        Timed t(c, HSF_K_PREP);
        launch_field_exp<real>(c->stream, c->plan, c->rep_d, c->st_d, c->ch, c->w, c->d, use_alpha, b.E, t.a, t.b);
    }
    for (int s0 = 0; s0 < N; s0 += K) {
        Timed t(c, HSF_K_FWD);
        launch_fwd_block<real>(c->tile, c->stream, c->tplan, c->rep_d, c->st_d, c->ch, s0, std::min(K, N - s0), b,
                               c->partG, sums, direct ? c->w : nullptr, c->d, use_alpha, t.a, t.b);
    }
    if (!fold_q)
        launch_reduce_ctl(c->stream, c->n_rep, c->tplan, c->st_d, c->rep_d, c->part, PH_Q, c->ch, c->partG, 0.0, 0,
                          c->st_hd);
    int parity = 0;
    for (int s_hi = N; s_hi >= 1; s_hi -= K) {
        Timed t(c, HSF_K_BWD);
        const real *gin = b.Gp[parity ^ 1];
        real *gout = b.Gp[parity];
        launch_bwd_block<real>(c->tile, c->stream, c->tplan, c->rep_d, c->st_d, c->ch, s_hi, std::min(K, s_hi), b,
                               gin, gout, c->acc, final_mode, c->phi, d, out, c->part, c->partG, fold_q ? 1 : 0,
                               t.a, t.b);
        parity ^= 1;
    }
}

// sums: also produce the per-step propagator sums that update the FP32 scales
void run_eval_any(hsf_ctx *c, int use_alpha, int final_mode, double *out, const double *d, int sums)
{
    if (c->precision == HSF_FP32 && !c->eval64)
        run_eval<float>(c, use_alpha, final_mode, out, d, sums);
    else
        run_eval<double>(c, use_alpha, final_mode, out, d, sums);
}

void target_setup(hsf_ctx *c, double tol, int max_iter)
{
    launch_target_stats(c->stream, c->plan, c->rep_d, c->st_d, c->ch, c->phi, c->w, c->part);
    launch_reduce_ctl(c->stream, c->n_rep, c->plan, c->st_d, c->rep_d, c->part, PH_TARGET, c->ch, c->partG, tol,
                      max_iter, c->st_hd);
}

// Starting fields of an inversion (the warm start), before the gauge is fixed.
//   EXTRAP      w += w^n - w^(n-1)
//   NET         polymer fields = net(phi)
//   NET_DELTA   w += r net(phi^n, (phi - phi^n) / r)
//   NET_EXTRAP  w += w^n - w^(n-1) + r net(phi^n, (phi - 2 phi^n + phi^(n-1)) / r)
// with w^n, phi^n the converged fields and target densities of the latest inversion
// and r the rms of the density difference.  Without enough history the modes fall
// back: NET_EXTRAP to NET_DELTA, NET_DELTA and EXTRAP to the current fields.
int warm_start(hsf_ctx *c, int warm)
{
    hipStream_t s = c->stream;
    const int nsp = c->ch.nsp;
    if (warm == HSF_WARM_EXTRAP) {
        if (c->n_hist >= 2 && c->fields_set)
            for (int r = 0; r < c->n_rep; ++r) {
                const long long fo = (long long)nsp * c->reps[r].site_off;
                net_shift_fields(s, c->w + fo, c->w_hist[0] + fo, c->w_hist[1] + fo, 2 * c->reps[r].V);
            }
        return HSF_OK;
    }
    if (warm != HSF_WARM_NET && warm != HSF_WARM_NET_DELTA && warm != HSF_WARM_NET_EXTRAP) return HSF_OK;
    if (!c->net) return fail(c, HSF_EINVAL, "no network attached");
    if (c->net_gate > 0 && c->n_hist >= 1 && warm != HSF_WARM_NET) {
        // the previous inversions were short: the plain warm start is already close
        int most = 0;
        for (int r = 0; r < c->n_rep; ++r) most = std::max(most, c->st_h[r].iters);
        if (most < c->net_gate) return warm == HSF_WARM_NET_EXTRAP ? warm_start(c, HSF_WARM_EXTRAP) : HSF_OK;
    }
    int mode = 0;   // 0: absolute, 1: first difference, 2: second difference
    if (warm == HSF_WARM_NET_DELTA || warm == HSF_WARM_NET_EXTRAP) {
        if (!c->fields_set || c->n_hist < 1) return HSF_OK;
        mode = (warm == HSF_WARM_NET_EXTRAP && c->n_hist >= 2) ? 2 : 1;
    }
    int in_ch = 0, out_ch = 0, q = 1;
    net_channels(c->net, &in_ch, &out_ch, &q);
    const int want = mode == 0 ? nsp : 2 * nsp;
    if (in_ch != want || out_ch != 2)
        return fail(c, HSF_EINVAL, "network has %d inputs and %d outputs; this warm start needs %d and 2", in_ch,
                    out_ch, want);
    for (int r = 0; r < c->n_rep; ++r) {
        const Rep &R = c->reps[r];
        if (R.Lx != R.Ly || R.Lx != R.Lz || R.Lx % q)
            return fail(c, HSF_EINVAL, "network warm start needs cubic boxes with L a multiple of %d", q);
    }
    const int max_parts = c->part_cap;
    // inputs of every replica, then one network call per run of consecutive replicas
    // with the same box (their inputs and outputs are contiguous)
    for (int r = 0; r < c->n_rep; ++r) {
        const Rep &R = c->reps[r];
        const long long fo = (long long)nsp * R.site_off;
        net_warm_input(s, c->phi + fo, c->phi_hist[0] + fo, c->phi_hist[1] + fo, nsp, R.V, mode, c->part,
                       max_parts, c->net_rms + r, c->net_in + (long long)want * R.site_off);
    }
    for (int r0 = 0; r0 < c->n_rep;) {
        int r1 = r0 + 1;
        while (r1 < c->n_rep && c->reps[r1].Lx == c->reps[r0].Lx) ++r1;
        const Rep &R = c->reps[r0];
        int rc = net_predict(c->net, s, c->net_in + (long long)want * R.site_off, want, r1 - r0, R.Lx,
                             c->net_pred + 2LL * R.site_off);
        if (rc) return fail(c, rc, "network prediction failed");
        r0 = r1;
    }
    for (int r = 0; r < c->n_rep; ++r) {
        const Rep &R = c->reps[r];
        const long long fo = (long long)nsp * R.site_off;
        net_warm_apply(s, c->w + fo, c->net_pred + 2LL * R.site_off, R.V, mode, c->net_rms + r, c->w_hist[0] + fo,
                       c->w_hist[1] + fo);
    }
    c->fields_set = 1;
    HIPCHK(c, hipGetLastError());
    return HSF_OK;
}

// FP64 staging buffer for the FP32 population storage (set/get and checkpoints).
int lb_staging(hsf_ctx *c)
{
    if (c->lb_stage) return HSF_OK;
    return dalloc(c, (void **)&c->lb_stage, sizeof(double) * 19 * c->T);
}

// Keep the latest inversion's result and target for the warm starts of the next ones.
int commit_history(hsf_ctx *c)
{
    std::swap(c->w_hist[0], c->w_hist[1]);
    std::swap(c->phi_hist[0], c->phi_hist[1]);
    HIPCHK(c, hipMemcpyAsync(c->w_hist[0], c->w, sizeof(double) * c->ch.nsp * c->T, hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->phi_hist[0], c->phi, sizeof(double) * c->ch.nsp * c->T, hipMemcpyDeviceToDevice,
                             c->stream));
    c->n_hist = std::min(c->n_hist + 1, 2);
    return HSF_OK;
}

// After a successful explicit coupled step: its inversion's fields become the newest
// history entry (a copy: w stays the current fields), and the densities rotate without
// copies: the step's targets phi become the newest history entry, the updated densities
// phi_tmp the current ones, and the oldest history buffer the next update's target.
int commit_step(hsf_ctx *c)
{
    std::swap(c->w_hist[0], c->w_hist[1]);
    HIPCHK(c, hipMemcpyAsync(c->w_hist[0], c->w, sizeof(double) * c->ch.nsp * c->T, hipMemcpyDeviceToDevice,
                             c->stream));
    double *oldest = c->phi_hist[1];
    c->phi_hist[1] = c->phi_hist[0];
    c->phi_hist[0] = c->phi;
    c->phi = c->phi_tmp;
    c->phi_tmp = oldest;
    c->n_hist = std::min(c->n_hist + 1, 2);
    return HSF_OK;
}

// commit_hist: record the result in the warm-start history here (hsf_invert); a coupled
// step records it only once the whole step has succeeded.
int invert_once(hsf_ctx *c, double tol, int max_iter, int warm, hsf_invert_stats *stats, long long *evals_out,
                bool commit_hist)
{
    if (!(tol >= 0.0) || max_iter < 0) return fail(c, HSF_EINVAL, "bad tol %g or max_iter %d", tol, max_iter);
    if (warm < HSF_WARM_CURRENT || warm > HSF_WARM_NET_EXTRAP) return fail(c, HSF_EINVAL, "bad warm mode %d", warm);
    hipStream_t s = c->stream;
    if (int rc = warm_start(c, warm)) return rc;
    if (warm == HSF_WARM_LOCAL || !c->fields_set)
        launch_local_guess(s, c->plan, c->rep_d, c->ch, c->phi, c->w, c->part);
    target_setup(c, tol, max_iter);
    launch_init_fields(s, c->plan, c->rep_d, c->st_d, c->ch, c->phi, c->w);
    HIPCHK(c, hipGetLastError());
    c->fields_set = 1;
    // starting point: evaluation, residual, first direction, first alpha
    int rc = run_seq(c, hsf_ctx::GK_START, [&] {
        run_eval_any(c, 0, 1, c->g, nullptr, 1);
        launch_reduce_ctl(c->stream, c->n_rep, c->tplan, c->st_d, c->rep_d, c->part, PH_EVAL0, c->ch, c->partG,
                          0.0, 0, c->st_hd);
        launch_cg_update(c->stream, c->plan, c->rep_d, c->st_d, c->ch, 1, c->w, c->g, c->gt, c->d, c->phi,
                         c->part);
        launch_reduce_ctl(c->stream, c->n_rep, c->plan, c->st_d, c->rep_d, c->part, PH_BEGIN, c->ch, c->partG,
                          0.0, 0, c->st_hd);
    });
    if (rc) return rc;
    if ((rc = read_status(c))) return rc;
    bool any = false;
    for (int r = 0; r < c->n_rep; ++r) any |= c->st_h[r].active != 0 || c->st_h[r].pending != 0;
    // A pass is one trial evaluation followed by the update sequence.  The update acts
    // only on replicas whose trial was accepted (the CG step and the start of their next
    // line search); for the others, and for finished replicas, every kernel of a pass
    // does nothing, so each replica advances on its own, without waiting for the line
    // searches of the others.  Passes could be issued several at a time between status
    // reads; measured at 64^3 that gained nothing over one, so the host reads the states
    // after every pass and stops once no replica is active.  Each pass either advances a
    // line-search trial (at most 3 per iteration) or ends an iteration, so 3 * max_iter +
    // 3 passes bound the loop.
    constexpr int kPassesPerRead = 1;
    long long guard = 3LL * max_iter + 3;
    while (any) {
        for (int p = 0; p < kPassesPerRead; ++p) {
            if (--guard < 0)   // the iterate is kept, as at max_iter
                return fail(c, HSF_ENOCONV, "inversion stopped after %lld passes without finishing",
                            3LL * max_iter + 3);
            // the pass (trial evaluation and update) as one captured sequence: one launch
            rc = run_seq(c, hsf_ctx::GK_PASS, [&] {
                run_eval_any(c, 1, 1, c->gt, c->d, 0);
                launch_reduce_ctl(c->stream, c->n_rep, c->tplan, c->st_d, c->rep_d, c->part, PH_TRIAL, c->ch,
                                  c->partG, 0.0, 0, c->st_hd);
                launch_cg_update(c->stream, c->plan, c->rep_d, c->st_d, c->ch, 0, c->w, c->g, c->gt, c->d, c->phi,
                                 c->part);
                launch_reduce_ctl(c->stream, c->n_rep, c->plan, c->st_d, c->rep_d, c->part, PH_BEGIN, c->ch,
                                  c->partG, 0.0, 0, c->st_hd);
            });
            if (rc) return rc;
        }
        if ((rc = read_status(c))) return rc;
        any = false;
        for (int r = 0; r < c->n_rep; ++r) any |= c->st_h[r].active != 0 || c->st_h[r].pending != 0;
    }
    if ((rc = read_status(c))) return rc;
    HIPCHK(c, hipGetLastError());
    int status = HSF_OK;
    long long ev = 0;
    for (int r = 0; r < c->n_rep; ++r) {
        const RepState &S = c->st_h[r];
        ev += S.evals;
        c->work_evals += S.evals;
        c->work_site_evals += (double)S.evals * (double)c->reps[r].V;
        if (stats) {
            stats[r].iterations = S.iters;
            stats[r].evaluations = S.evals;
            stats[r].restarts = S.restarts;
            stats[r].converged = S.converged;
            stats[r].residual = S.res;
        }
        if (S.nonfinite) status = fail(c, HSF_ENONFINITE, "non-finite value in replica %d", r);
        else if (!S.converged && status == HSF_OK)
            status = fail(c, HSF_ENOCONV, "replica %d stopped at %d iterations, residual %g", r, S.iters, S.res);
    }
    if (evals_out) *evals_out += ev;
    if (commit_hist && status != HSF_ENONFINITE)
        if (int rc2 = commit_history(c)) return rc2;
    return status;
}

// Residual down to which an FP32 context with refinement iterates with FP32 evaluations
// before it switches to FP64 ones: above the level where the FP32 evaluations' rounding
// stalls the iteration (measured 1e-7 to 3e-6 relative, by box and composition), so the
// FP32 phase does not stall.
constexpr double kRefineTol = 1e-5;

// The inversion.  FP32 contexts with refinement (HSF_SOLVER_REFINE) asked for a residual
// below kRefineTol run two phases: FP32 evaluations to kRefineTol, then FP64 evaluations
// from those fields (the same Fletcher-Reeves iteration, restarted from its steepest
// descent direction) to tol; the counts of both phases are added.
int invert_impl(hsf_ctx *c, double tol, int max_iter, int warm, hsf_invert_stats *stats, long long *evals_out,
                bool commit_hist = true)
{
    if (!(c->refine && c->precision == HSF_FP32 && tol < kRefineTol))
        return invert_once(c, tol, max_iter, warm, stats, evals_out, commit_hist);
    if (!(tol >= 0.0) || max_iter < 0) return fail(c, HSF_EINVAL, "bad tol %g or max_iter %d", tol, max_iter);
    std::vector<hsf_invert_stats> first(c->n_rep);
    int rc = invert_once(c, kRefineTol, max_iter, warm, first.data(), evals_out, false);
    // a first phase stopped by its iteration limit still hands its fields to the second
    if (rc != HSF_OK && rc != HSF_ENOCONV) return rc;
    c->eval64 = true;
    std::vector<hsf_invert_stats> second(c->n_rep);
    rc = invert_once(c, tol, max_iter, HSF_WARM_CURRENT, second.data(), evals_out, commit_hist);
    c->eval64 = false;
    if (stats)
        for (int r = 0; r < c->n_rep; ++r) {
            stats[r] = second[r];
            stats[r].iterations += first[r].iterations;
            stats[r].evaluations += first[r].evaluations;
            stats[r].restarts += first[r].restarts;
        }
    return rc;
}

// One evaluation of the density functional at the current fields, with phibar from the
// current densities, into eval_out; ln Q, phibar and <exp(-w_S)> stay in the replica
// states.  An evaluation whose propagators left the floating-point range is repeated
// with the per-step scales it adapted (at most three more times).
int evaluate_impl(hsf_ctx *c, bool check_range = true)
{
    hipStream_t s = c->stream;
    for (int attempt = 0; attempt < (check_range ? 4 : 1); ++attempt) {
        int rc0 = run_seq(c, hsf_ctx::GK_EVAL, [&] {
            target_setup(c, 0.0, 0);   // phibar_p, phibar_s from the current densities; all replicas active
            run_eval_any(c, 0, 0, c->eval_out, nullptr, 1);
            launch_reduce_ctl(c->stream, c->n_rep, c->tplan, c->st_d, c->rep_d, c->part, PH_SCALES, c->ch,
                              c->partG, 0.0, 0, c->st_hd);
        });
        if (rc0) return rc0;
        if (!check_range) break;
        if ((rc0 = read_status(c))) return rc0;
        bool bad = false;
        for (int r = 0; r < c->n_rep; ++r) bad |= c->st_h[r].nonfinite != 0;
        if (!bad) break;
    }
    if (c->ch.nsp == 3) {
        launch_solvent(s, c->plan, c->rep_d, c->st_d, c->ch, 0, c->w, c->phi, c->eval_out, c->part);
        launch_reduce_ctl(s, c->n_rep, c->plan, c->st_d, c->rep_d, c->part, PH_SOLVENT, c->ch, c->partG, 0.0, 0, c->st_hd);
        launch_solvent(s, c->plan, c->rep_d, c->st_d, c->ch, 1, c->w, c->phi, c->eval_out, c->part);
    }
    HIPCHK(c, hipGetLastError());
    return HSF_OK;
}

// ---- Crank-Nicolson diffusion: Newton-Krylov solve for the fields of phi^{n+1} ----
//
// F(w) = phi[w] - dt/2 B(phi[w], mu(phi[w], w)) - rhs, rhs = phi^n + dt/2 B^n - div J^C + xi,
// with B the diffusive rate of the explicit step's face fluxes.  Newton's method on the
// fields of all replicas jointly; each correction from restarted GMRES(m) on the
// forward-difference Jacobian J v = (F(w + eps v) - F(w)) / eps, classical Gram-Schmidt
// applied twice, to ||J dw + F|| <= eta ||F||; the correction is halved (at most four
// times) while it does not reduce ||F||.  F keeps each species' amount (its per-species
// sums vanish) and is blind to per-species constants in w, so the Krylov vectors stay
// in the zero-sum subspace.  Stops at rms(F) <= tol.

long long cn_n(const hsf_ctx *c) { return (long long)c->ch.nsp * c->T; }

// out_h[j] = <V_j, x>, j < k
int cn_dots(hsf_ctx *c, const double *V, int k, const double *x, double *out_h)
{
    launch_dots(c->stream, V, k, cn_n(c), x, c->cn_part, c->cn_dots);
    HIPCHK(c, hipMemcpyAsync(c->cn_dots_h, c->cn_dots, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
    int rc = sync(c);
    if (rc) return rc;
    for (int j = 0; j < k; ++j) out_h[j] = c->cn_dots_h[j];
    return HSF_OK;
}

// y += sum_j coef_h[j] V_j
int cn_axpy(hsf_ctx *c, double *y, const double *V, int k, const double *coef_h)
{
    for (int j = 0; j < k; ++j) c->cn_dots_h[j] = coef_h[j];
    HIPCHK(c, hipMemcpyAsync(c->cn_coef, c->cn_dots_h, sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
    launch_multi_axpy(c->stream, y, V, k, cn_n(c), c->cn_coef, 1.0);
    HIPCHK(c, hipGetLastError());
    return sync(c);   // the pinned staging buffer is reused by the next call
}

// F_out = F(current fields c->w); leaves phi[w] in eval_out.  No host round trip: a Q out
// of range makes F non-finite, which the solve detects through ||F|| (and the dot
// products of the Krylov basis).
int cn_residual(hsf_ctx *c, double *F_out, long long *evals)
{
    int rc = evaluate_impl(c, false);
    if (rc) return rc;
    *evals += c->n_rep;
    c->work_evals += c->n_rep;
    for (int r = 0; r < c->n_rep; ++r) c->work_site_evals += (double)c->reps[r].V;
    launch_mu(c->stream, c->plan, c->rep_d, c->ch, c->eval_out, c->w, c->mu);
    launch_cd(c->stream, c->plan, c->rep_d, c->ch, c->eval_out, c->mu, nullptr, c->cn_half, nullptr, 0, nullptr,
              nullptr, 0.5);
    launch_cn_residual(c->stream, F_out, c->eval_out, c->cn_half, c->cn_rhs, cn_n(c));
    HIPCHK(c, hipGetLastError());
    return HSF_OK;
}

double cn_norm(hsf_ctx *c, const double *x, int *rc)
{
    double d = 0.0;
    *rc = cn_dots(c, x, 1, x, &d);
    return sqrt(d);
}

// Solve F(w) = 0 starting from the current fields; on success the fields hold w^{n+1}
// and the densities phi[w^{n+1}].  c->cn_rhs must hold the right-hand side.
int cn_solve(hsf_ctx *c, long long *evals_out)
{
    const long long n = cn_n(c);
    const int m = c->cn_m;
    const double rtn = sqrt((double)n);
    hsf_cn_stats st{};
    long long evals = 0;
    int rc = cn_residual(c, c->cn_F, &evals);
    if (rc) return rc;
    double fnorm = cn_norm(c, c->cn_F, &rc);
    if (rc) return rc;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    for (;;) {
        st.residual = fnorm / rtn;
        if (!std::isfinite(fnorm)) return fail(c, HSF_ENONFINITE, "non-finite Crank-Nicolson residual");
        if (st.residual <= c->cn_tol) {
            st.converged = 1;
            break;
        }
        if (st.newton >= c->cn_max_newton) break;
        ++st.newton;
        const double wnorm = cn_norm(c, c->w, &rc);
        if (rc) return rc;
        // forward-difference step: sqrt(2^-52) (1 + ||w||) with FP64 propagators; with FP32
        // ones the evaluation's rounding (about 1e-7 relative) needs a step large enough
        // that it stays a small part of the difference: 1e-4 (1 + ||w||)
        const double eps = (c->precision == HSF_FP64 ? 1.4901161193847656e-8 : 1e-4) * (1.0 + wnorm);
        // w_base: the Newton iterate; the Krylov basis spans corrections to it
        HIPCHK(c, hipMemcpyAsync(c->cn_wbase, c->w, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        // GMRES(m) for J dw = -F with x0 = 0
        double beta = fnorm;
        launch_lincomb(c->stream, c->cn_V, -1.0 / beta, c->cn_F, 0.0, c->cn_F, n);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double *vj = c->cn_V + (long long)j * n, *vn = c->cn_V + (long long)(j + 1) * n;
            // J v_j by a forward difference (v_j has unit norm)
            launch_lincomb(c->stream, c->w, 1.0, c->cn_wbase, eps, vj, n);
            if ((rc = cn_residual(c, c->cn_Ft, &evals))) return rc;
            launch_lincomb(c->stream, vn, 1.0 / eps, c->cn_Ft, -1.0 / eps, c->cn_F, n);
            ++st.krylov;
            // classical Gram-Schmidt, twice, with the coefficients kept on the device; one
            // copy of both coefficient sets and the norm to the host
            const int stride = kMaxKrylov + 1;
            double *d1 = c->cn_dots, *d2 = c->cn_dots + stride, *dn = c->cn_dots + 2 * stride;
            launch_dots(c->stream, c->cn_V, j + 1, n, vn, c->cn_part, d1);
            launch_multi_axpy(c->stream, vn, c->cn_V, j + 1, n, d1, -1.0);
            launch_dots(c->stream, c->cn_V, j + 1, n, vn, c->cn_part, d2);
            launch_multi_axpy(c->stream, vn, c->cn_V, j + 1, n, d2, -1.0);
            launch_dots(c->stream, vn, 1, n, vn, c->cn_part, dn);
            HIPCHK(c, hipMemcpyAsync(c->cn_dots_h, c->cn_dots, sizeof(double) * 3 * stride, hipMemcpyDeviceToHost,
                                     c->stream));
            if ((rc = sync(c))) return rc;
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = c->cn_dots_h[i] + c->cn_dots_h[stride + i];
            const double hn = sqrt(c->cn_dots_h[2 * stride]);
            if (!std::isfinite(hn)) return fail(c, HSF_ENONFINITE, "non-finite Crank-Nicolson Jacobian product");
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0) launch_lincomb(c->stream, vn, 1.0 / hn, vn, 0.0, vn, n);
            // Givens rotations of the new column
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double r = hypot(a, b);
            cs[j] = r > 0.0 ? a / r : 1.0;
            sn[j] = r > 0.0 ? b / r : 0.0;
            H[(size_t)j * m + j] = r;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            if (fabs(g[j + 1]) <= c->cn_eta * beta || hn == 0.0) break;
        }
        // y = R^-1 g, dw = sum y_i v_i
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int l = i + 1; l < k; ++l) t -= H[(size_t)i * m + l] * y[l];
            y[i] = t / H[(size_t)i * m + i];
        }
        // trial w = w_base + lambda dw, halving lambda while ||F|| does not decrease
        double lambda = 1.0;
        for (int tries = 0;; ++tries) {
            HIPCHK(c, hipMemcpyAsync(c->w, c->cn_wbase, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
            std::vector<double> ly(k);
            for (int i = 0; i < k; ++i) ly[i] = lambda * y[i];
            if ((rc = cn_axpy(c, c->w, c->cn_V, k, ly.data()))) return rc;
            if ((rc = cn_residual(c, c->cn_Ft, &evals))) return rc;
            const double fn = cn_norm(c, c->cn_Ft, &rc);
            if (rc) return rc;
            if ((std::isfinite(fn) && fn < fnorm) || tries == 4) {
                fnorm = fn;
                std::swap(c->cn_F, c->cn_Ft);
                break;
            }
            lambda *= 0.5;
        }
    }
    // eval_out holds phi at the accepted fields: the new densities
    HIPCHK(c, hipMemcpyAsync(c->phi, c->eval_out, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    st.evaluations = evals;
    c->cn_last = st;
    if (evals_out) *evals_out += evals;
    return st.converged ? HSF_OK : fail(c, HSF_ENOCONV, "Crank-Nicolson step: rms residual %.3e after %d Newton "
                                                        "iterations", st.residual, st.newton);
}

int cn_alloc(hsf_ctx *c, int m)
{
    if (c->cn_alloc_m >= m) return HSF_OK;
    const long long n = cn_n(c);
    int rc = HSF_OK;
    if (!c->cn_rhs) {
        for (double **p : {&c->cn_rhs, &c->cn_F, &c->cn_Ft, &c->cn_wbase, &c->cn_half})
            if (rc == HSF_OK) rc = dalloc(c, (void **)p, sizeof(double) * n);
        if (rc == HSF_OK) rc = dalloc(c, (void **)&c->cn_dots, sizeof(double) * 3 * (kMaxKrylov + 1));
        if (rc == HSF_OK) rc = dalloc(c, (void **)&c->cn_coef, sizeof(double) * (kMaxKrylov + 1));
        if (rc == HSF_OK) rc = dalloc(c, (void **)&c->cn_part, sizeof(double) * (kMaxKrylov + 1) * vec_dot_blocks());
        if (rc == HSF_OK && hipHostMalloc((void **)&c->cn_dots_h, sizeof(double) * 3 * (kMaxKrylov + 1),
                                          hipHostMallocDefault) != hipSuccess)
            rc = fail(c, HSF_ENOMEM, "hipHostMalloc failed");
        if (rc) return rc;
    }
    // the Krylov basis grows to the largest dimension asked for (the old one is kept in
    // the allocation list and freed with the context)
    if ((rc = dalloc(c, (void **)&c->cn_V, sizeof(double) * (m + 1) * n))) return rc;
    c->cn_alloc_m = m;
    return HSF_OK;
}

}  // namespace

extern "C" {

int hsf_create(const hsf_params *reps, int n_rep, hsf_ctx **out)
{
    if (!out) return HSF_EINVAL;
    *out = nullptr;
    if (!reps || n_rep <= 0) return HSF_EINVAL;
    const hsf_params &p0 = reps[0];
    if (p0.n_beads < 1 || p0.n_beads > HSF_MAX_BEADS) return HSF_EINVAL;
    if (p0.precision != HSF_FP64 && p0.precision != HSF_FP32) return HSF_EINVAL;
    for (int r = 0; r < n_rep; ++r) {
        const hsf_params &p = reps[r];
        if (p.n_beads != p0.n_beads || p.has_solvent != p0.has_solvent || p.precision != p0.precision ||
            p.hydro != p0.hydro)
            return HSF_EINVAL;
        for (int s = 0; s < p.n_beads; ++s)
            if (p.types[s] != p0.types[s] || p.types[s] < 0 || p.types[s] > 1) return HSF_EINVAL;
        if (p.Lx < 1 || p.Ly < 1 || p.Lz < 1) return HSF_EINVAL;
        if ((long long)p.Lx * p.Ly * p.Lz > HSF_MAX_SITES) return HSF_EINVAL;
        if (!(p.tau > 0.5) || !(p.dt > 0.0)) return HSF_EINVAL;
        if (p.lb_mode != HSF_LB_BGK && p.lb_mode != HSF_LB_MRT) return HSF_EINVAL;
        if (p.lb_mode == HSF_LB_MRT && !(std::fabs(p.gamma_s) < 1.0 && std::fabs(p.gamma_b) < 1.0 &&
                                         std::fabs(p.gamma_ghost) < 1.0))
            return HSF_EINVAL;
    }
    hsf_ctx *c = new hsf_ctx();
    const char *ng = getenv("HSF_NO_GRAPHS");   // debugging aid: launch every kernel directly
    c->use_graphs = (ng && ng[0] == '1') ? 0 : 1;
    // checking aid: every device buffer the context allocates starts filled with NaN bytes
    // (0xff), so a kernel that reads memory no kernel or copy has written yet spreads NaN
    const char *pz = getenv("HSF_POISON");
    c->poison = (pz && pz[0] == '1') ? 1 : 0;
    c->n_rep = n_rep;
    c->precision = p0.precision;
    c->hydro = p0.hydro ? 1 : 0;
    c->ch.N = p0.n_beads;
    c->ch.nsp = p0.has_solvent ? 3 : 2;
    for (int s = 0; s < 64; ++s) c->ch.types[s] = s < p0.n_beads ? p0.types[s] : 0;

    std::vector<int> blk_rep, blk_first;
    long long off = 0;
    for (int r = 0; r < n_rep; ++r) {
        const hsf_params &p = reps[r];
        Rep R{};
        R.Lx = p.Lx;
        R.Ly = p.Ly;
        R.Lz = p.Lz;
        R.hydro = p.hydro;
        R.V = (long long)p.Lx * p.Ly * p.Lz;
        R.site_off = off;
        const bool given = p.stencil[0] != 0.0 || p.stencil[1] != 0.0 || p.stencil[2] != 0.0 || p.stencil[3] != 0.0;
        if (given)
            for (int k = 0; k < 4; ++k) R.c[k] = p.stencil[k];
        else
            weights_from_segment(p.a, R.c);
        R.csum = R.c[0] + 6.0 * R.c[1] + 12.0 * R.c[2] + 8.0 * R.c[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R.chi[i][j] = p.chi[i][j];
        R.kappa = p.kappa;
        R.dt = p.dt;
        R.tau = p.tau;
        R.lb_mode = p.lb_mode;
        R.gamma_s = p.gamma_s;
        R.gamma_b = p.gamma_b;
        R.gamma_ghost = p.gamma_ghost;
        c->reps.push_back(R);
        blk_first.push_back((int)blk_rep.size());
        const long long nb = (R.V + kBlock - 1) / kBlock;
        for (long long b = 0; b < nb; ++b) blk_rep.push_back(r);
        off += R.V;
    }
    blk_first.push_back((int)blk_rep.size());
    c->T = off;
    c->plan.nblocks = (int)blk_rep.size();
    c->plan.n_rep = n_rep;
    set_plan_args(c->plan, c->reps.data(), n_rep, blk_first.data());
    c->lb_all = c->reps[0].lb_mode;
    for (const Rep &R : c->reps)
        if (R.lb_mode != c->lb_all) c->lb_all = -1;
    {
        std::vector<int> br, bf;
#define HSF_SIZE(CX, CY, CZ, K)                                             \
    tile_blocks(c, TileCfg{CX, CY, CZ, K}, br, bf);                         \
    c->max_tile_blocks = std::max(c->max_tile_blocks, (int)br.size());
#define HSF_SIZES(H, CZ, K) HSF_SIZE(64, H, CZ, K)
        HSF_TILE_CONFIGS(HSF_SIZE)
        HSF_STREAM_CONFIGS(HSF_SIZES)
#undef HSF_SIZES
#undef HSF_SIZE
    }
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            c->lds_limit = (size_t)lds;
    }
    const int max_blocks = std::max(c->plan.nblocks, c->max_tile_blocks);

    const long long T = c->T;
    const int nsp = c->ch.nsp, N = c->ch.N;
    const size_t rs = real_size(c);
    int rc = HSF_OK;
#define ALLOC(ptr, bytes)                                          \
    if (rc == HSF_OK) rc = dalloc(c, (void **)&(ptr), (size_t)(bytes));
    ALLOC(c->rep_d, sizeof(Rep) * n_rep);
    ALLOC(c->st_d, sizeof(RepState) * n_rep);
    ALLOC(c->st_save, sizeof(RepState) * n_rep);
    ALLOC(c->plan.blk_rep, sizeof(int) * blk_rep.size());
    ALLOC(c->plan.blk_first, sizeof(int) * blk_first.size());
    ALLOC(c->w, sizeof(double) * nsp * T);
    ALLOC(c->w_start, sizeof(double) * nsp * T);
    ALLOC(c->phi, sizeof(double) * nsp * T);
    ALLOC(c->phi_tmp, sizeof(double) * nsp * T);
    ALLOC(c->mu, sizeof(double) * nsp * T);
    ALLOC(c->eval_out, sizeof(double) * nsp * T);
    ALLOC(c->g, sizeof(double) * 2 * T);
    ALLOC(c->gt, sizeof(double) * 2 * T);
    ALLOC(c->d, sizeof(double) * 2 * T);
    ALLOC(c->acc, sizeof(double) * 2 * T);
    c->lb32 = c->precision == HSF_FP32;
    ALLOC(c->nA, (c->lb32 ? sizeof(float) : sizeof(double)) * 19 * T);
    ALLOC(c->nB, (c->lb32 ? sizeof(float) : sizeof(double)) * 19 * T);
    ALLOC(c->rho, sizeof(double) * T);
    ALLOC(c->u, sizeof(double) * 3 * T);
    ALLOC(c->uin, sizeof(double) * 3 * T);
    ALLOC(c->force, sizeof(double) * 3 * T);
    ALLOC(c->part, sizeof(double) * kNQ * max_blocks);
    c->part_cap = kNQ * max_blocks;
    ALLOC(c->partG, sizeof(double) * (N + 2) * max_blocks);
    ALLOC(c->tplan.blk_rep, sizeof(int) * c->max_tile_blocks);
    ALLOC(c->tplan.blk_first, sizeof(int) * (n_rep + 1));
    ALLOC(c->E, rs * 2 * T);
    ALLOC(c->G, rs * N * T);
    ALLOC(c->Gp0, rs * T);
    ALLOC(c->Gp1, rs * T);
    ALLOC(c->Gf0, rs * T);
    ALLOC(c->Gf1, rs * T);
    for (int h = 0; h < 2; ++h) {
        ALLOC(c->w_hist[h], sizeof(double) * nsp * T);
        ALLOC(c->phi_hist[h], sizeof(double) * nsp * T);
    }
    ALLOC(c->net_in, sizeof(float) * 2 * nsp * T);
    ALLOC(c->net_pred, sizeof(float) * 2 * T);
    ALLOC(c->net_rms, sizeof(double) * n_rep);
    ALLOC(c->obs, sizeof(double) * observables_scratch_doubles(n_rep));
#undef ALLOC
    if (rc == HSF_OK) {
        hipError_t e = hipHostMalloc((void **)&c->st_h, sizeof(RepState) * n_rep, hipHostMallocDefault);
        if (e != hipSuccess) rc = fail(c, HSF_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
        else if ((e = hipHostGetDevicePointer((void **)&c->st_hd, c->st_h, 0)) != hipSuccess)
            rc = fail(c, HSF_EHIP, "hipHostGetDevicePointer failed: %s", hipGetErrorString(e));
        else if ((e = hipHostMalloc((void **)&c->bad_h, sizeof(int), hipHostMallocDefault)) != hipSuccess)
            rc = fail(c, HSF_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
        else if ((e = hipHostGetDevicePointer((void **)&c->bad_hd, c->bad_h, 0)) != hipSuccess)
            rc = fail(c, HSF_EHIP, "hipHostGetDevicePointer failed: %s", hipGetErrorString(e));
        if (c->bad_h) *c->bad_h = 0;
    }
    if (rc != HSF_OK) {
        hsf_destroy(c);
        return rc;
    }
    hipError_t e = hipSuccess;
    std::vector<RepState> st0(n_rep);
    memset(st0.data(), 0, sizeof(RepState) * n_rep);
    if (e == hipSuccess) e = hipMemcpy(c->rep_d, c->reps.data(), sizeof(Rep) * n_rep, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->st_d, st0.data(), sizeof(RepState) * n_rep, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->plan.blk_rep, blk_rep.data(), sizeof(int) * blk_rep.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->plan.blk_first, blk_first.data(), sizeof(int) * blk_first.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->w, 0, sizeof(double) * nsp * T);
    if (e == hipSuccess) e = hipMemset(c->phi, 0, sizeof(double) * nsp * T);
    if (e == hipSuccess) e = hipMemset(c->d, 0, sizeof(double) * 2 * T);
    if (e == hipSuccess) e = hipMemset(c->u, 0, sizeof(double) * 3 * T);
    if (e == hipSuccess) e = hipMemset(c->rho, 0, sizeof(double) * T);
    if (e == hipSuccess) {
        launch_lb_rest(nullptr, c->plan, c->rep_d, c->nA, c->lb32);
        e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        rc = fail(c, HSF_EHIP, "initialisation failed: %s", hipGetErrorString(e));
        hsf_destroy(c);
        return rc;
    }
    // propagator tiles: default, or forced by HSF_TILE=cx,cy,cz,k
    TileCfg t0{8, 8, 8, 2};
    const char *forced = getenv("HSF_TILE");
    if (forced) {
        TileCfg f{0, 0, 0, 0};
        if (sscanf(forced, "%d,%d,%d,%d", &f.cx, &f.cy, &f.cz, &f.k) == 4 && tile_known(f)) t0 = f;
    }
    if (tile_lds_bytes(t0, real_size(c)) > c->lds_limit) t0 = TileCfg{8, 8, 8, 1};
    if ((rc = set_tile(c, t0)) != HSF_OK) {
        hsf_destroy(c);
        return rc;
    }
    *out = c;
    return HSF_OK;
}

void hsf_destroy(hsf_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    c->drop_graphs();
    for (auto &m : c->pending)
        if (m.pooled) {
            (void)hipEventDestroy(m.a);
            (void)hipEventDestroy(m.b);
        }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->log_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (void *p : c->allocs) (void)hipFree(p);
    if (c->st_h) (void)hipHostFree(c->st_h);
    if (c->bad_h) (void)hipHostFree(c->bad_h);
    if (c->cn_dots_h) (void)hipHostFree(c->cn_dots_h);
    delete c;
}

const char *hsf_last_error(const hsf_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

int hsf_set_stream(hsf_ctx *c, void *stream)
{
    if (!c) return HSF_EINVAL;
    c->stream = (hipStream_t)stream;
    return HSF_OK;
}

long long hsf_total_sites(const hsf_ctx *c) { return c ? c->T : -1; }

long long hsf_site_offset(const hsf_ctx *c, int rep)
{
    if (!c || rep < 0 || rep > c->n_rep) return -1;
    return rep == c->n_rep ? c->T : c->reps[rep].site_off;
}

long long hsf_field_offset(const hsf_ctx *c, int rep)
{
    const long long s = hsf_site_offset(c, rep);
    return s < 0 ? -1 : s * c->ch.nsp;
}

int hsf_num_species(const hsf_ctx *c) { return c ? c->ch.nsp : -1; }

int hsf_set_fields(hsf_ctx *c, const double *w, int where)
{
    if (!c) return HSF_EINVAL;
    int rc = copy_in(c, c->w, w, (size_t)c->ch.nsp * c->T, where);
    if (rc == HSF_OK) {
        c->fields_set = 1;
        c->n_hist = 0;   // fields set from outside: the inversion history no longer applies
    }
    return rc;
}

int hsf_get_fields(hsf_ctx *c, double *w, int where)
{
    if (!c) return HSF_EINVAL;
    return copy_out(c, w, c->w, (size_t)c->ch.nsp * c->T, where);
}

int hsf_set_densities(hsf_ctx *c, const double *phi, int where)
{
    if (!c) return HSF_EINVAL;
    return copy_in(c, c->phi, phi, (size_t)c->ch.nsp * c->T, where);
}

int hsf_get_densities(hsf_ctx *c, double *phi, int where)
{
    if (!c) return HSF_EINVAL;
    return copy_out(c, phi, c->phi, (size_t)c->ch.nsp * c->T, where);
}

int hsf_evaluate(hsf_ctx *c, double *phi_out, double *Q_out, int where)
{
    if (!c) return HSF_EINVAL;
    if (!phi_out) return fail(c, HSF_EINVAL, "null output");
    int rc = evaluate_impl(c);
    if (rc) return rc;
    if ((rc = copy_out(c, phi_out, c->eval_out, (size_t)c->ch.nsp * c->T, where))) return rc;
    if ((rc = read_status(c))) return rc;
    for (int r = 0; r < c->n_rep; ++r) {
        if (Q_out) Q_out[r] = exp(c->st_h[r].ln_q);
        if (c->st_h[r].nonfinite) return fail(c, HSF_ENONFINITE, "non-finite Q in replica %d", r);
    }
    return HSF_OK;
}

int hsf_observables(hsf_ctx *c, double *free_energy, double *s_melt, double *s_sol)
{
    if (!c) return HSF_EINVAL;
    int rc = evaluate_impl(c);
    if (rc) return rc;
    double *out = c->obs + observables_scratch_doubles(c->n_rep) - 3 * (size_t)c->n_rep;
    launch_observables(c->stream, c->plan, c->n_rep, c->rep_d, c->st_d, c->ch, c->w, c->phi, c->part, c->obs, out);
    HIPCHK(c, hipGetLastError());
    std::vector<double> h(3 * (size_t)c->n_rep);
    if ((rc = copy_out(c, h.data(), out, h.size(), HSF_HOST))) return rc;
    if ((rc = read_status(c))) return rc;
    for (int r = 0; r < c->n_rep; ++r) {
        if (c->st_h[r].nonfinite) return fail(c, HSF_ENONFINITE, "non-finite Q in replica %d", r);
        if (free_energy) free_energy[r] = h[3 * r];
        if (s_melt) s_melt[r] = h[3 * r + 1];
        if (s_sol) s_sol[r] = h[3 * r + 2];
    }
    return HSF_OK;
}

int hsf_invert(hsf_ctx *c, double tol, int max_iter, int warm, hsf_invert_stats *stats)
{
    if (!c) return HSF_EINVAL;
    return invert_impl(c, tol, max_iter, warm, stats, nullptr);
}

int hsf_mu_force(hsf_ctx *c, double *mu, double *force, int where)
{
    if (!c) return HSF_EINVAL;
    launch_mu(c->stream, c->plan, c->rep_d, c->ch, c->phi, c->w, c->mu);
    launch_force(c->stream, c->plan, c->rep_d, c->ch, c->phi, c->mu, c->force);
    HIPCHK(c, hipGetLastError());
    int rc = HSF_OK;
    if (mu) rc = copy_out(c, mu, c->mu, (size_t)c->ch.nsp * c->T, where);
    if (rc == HSF_OK && force) rc = copy_out(c, force, c->force, (size_t)3 * c->T, where);
    return rc;
}

int hsf_set_lb(hsf_ctx *c, const double *n, int where)
{
    if (!c) return HSF_EINVAL;
    if (!c->lb32) return copy_in(c, (double *)c->nA, n, (size_t)19 * c->T, where);
    const double *src = n;
    if (where == HSF_HOST) {
        int rc = lb_staging(c);
        if (rc == HSF_OK) rc = copy_in(c, c->lb_stage, n, (size_t)19 * c->T, where);
        if (rc) return rc;
        src = c->lb_stage;
    } else if (where != HSF_DEVICE || !n) {
        return fail(c, HSF_EINVAL, "bad populations pointer or location");
    }
    launch_lb_convert(c->stream, c->plan, c->rep_d, true, src, c->nA);
    HIPCHK(c, hipGetLastError());
    return HSF_OK;
}

int hsf_get_lb(hsf_ctx *c, double *n, int where)
{
    if (!c) return HSF_EINVAL;
    if (!c->lb32) return copy_out(c, n, (const double *)c->nA, (size_t)19 * c->T, where);
    if (where == HSF_DEVICE && n) {
        launch_lb_convert(c->stream, c->plan, c->rep_d, false, c->nA, n);
        HIPCHK(c, hipGetLastError());
        return HSF_OK;
    }
    int rc = lb_staging(c);
    if (rc) return rc;
    launch_lb_convert(c->stream, c->plan, c->rep_d, false, c->nA, c->lb_stage);
    HIPCHK(c, hipGetLastError());
    return copy_out(c, n, c->lb_stage, (size_t)19 * c->T, where);
}

int hsf_lb_advance(hsf_ctx *c, int n_steps, const double *force, int where)
{
    if (!c || n_steps < 0) return HSF_EINVAL;
    const double *f = nullptr;
    if (force) {
        int rc = copy_in(c, c->uin, force, (size_t)3 * c->T, where);
        if (rc) return rc;
        f = c->uin;
    }
    for (int k = 0; k < n_steps; ++k) {
        {
            Timed t(c, HSF_K_LB);
            launch_lb(c->stream, c->plan, c->rep_d, c->nA, c->nB, c->lb32, f, c->rho, c->u, (c->noise & HSF_NOISE_LB) != 0,
                      c->noise_step, c->lb_all, t.a, t.b);
        }
        std::swap(c->nA, c->nB);
        if (c->noise) ++c->noise_step;
    }
    HIPCHK(c, hipGetLastError());
    return HSF_OK;
}

int hsf_get_flow(hsf_ctx *c, double *rho, double *u, int where)
{
    if (!c) return HSF_EINVAL;
    int rc = HSF_OK;
    if (rho) rc = copy_out(c, rho, c->rho, (size_t)c->T, where);
    if (rc == HSF_OK && u) rc = copy_out(c, u, c->u, (size_t)3 * c->T, where);
    return rc;
}

int hsf_cd_advance(hsf_ctx *c, const double *mu, const double *u, int where)
{
    if (!c || !mu) return HSF_EINVAL;
    int rc = copy_in(c, c->mu, mu, (size_t)c->ch.nsp * c->T, where);
    if (rc) return rc;
    const double *uu = nullptr;
    if (u) {
        if ((rc = copy_in(c, c->uin, u, (size_t)3 * c->T, where))) return rc;
        uu = c->uin;
    }
    launch_cd(c->stream, c->plan, c->rep_d, c->ch, c->phi, c->mu, uu, c->phi_tmp,
              (c->noise & HSF_NOISE_CD) ? c->noise_flux : nullptr, c->noise_step);
    if (c->noise) ++c->noise_step;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->phi, c->phi_tmp, sizeof(double) * c->ch.nsp * c->T, hipMemcpyDeviceToDevice,
                             c->stream));
    return HSF_OK;
}

// A failed coupled step leaves the state of its start: the fields and replica states
// (scales, control) are copied back, and the densities and LB populations are only
// replaced once the step has finished with finite results.
static int rollback_step(hsf_ctx *c)
{
    HIPCHK(c, hipMemcpyAsync(c->w, c->w_start, sizeof(double) * c->ch.nsp * c->T, hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->st_d, c->st_save, sizeof(RepState) * c->n_rep, hipMemcpyDeviceToDevice, c->stream));
    return sync(c);
}

// Step log: ln Q of the inversion's last evaluation, right after it (later evaluations
// overwrite the replica states); the counts arrive in log_inv from the inversion.
static void log_inversion(hsf_ctx *c)
{
    c->log_lnq.resize(c->n_rep);
    for (int r = 0; r < c->n_rep; ++r) c->log_lnq[r] = c->st_h[r].ln_q;
}

// Step log: amounts and flow speed after a successful step, and the phase times.
static int log_step(hsf_ctx *c, bool flow)
{
    launch_step_moments(c->stream, c->plan, c->n_rep, c->rep_d, c->ch.nsp, c->phi, flow ? c->u : nullptr, c->part,
                        c->log_d);
    HIPCHK(c, hipGetLastError());
    std::vector<double> h(4 * (size_t)c->n_rep);
    if (int rc = copy_out(c, h.data(), c->log_d, h.size(), HSF_HOST)) return rc;
    float t_inv = 0.0f, t_dyn = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&t_inv, c->log_ev[0], c->log_ev[1]));
    HIPCHK(c, hipEventElapsedTime(&t_dyn, c->log_ev[1], c->log_ev[2]));
    constexpr size_t kMaxRecords = (size_t)1 << 20;
    for (int r = 0; r < c->n_rep; ++r) {
        hsf_step_record e{};
        e.step = c->steps_done;
        e.replica = r;
        e.iterations = c->log_inv[r].iterations;
        e.evaluations = c->log_inv[r].evaluations;
        e.converged = c->log_inv[r].converged;
        e.residual = c->log_inv[r].residual;
        e.ln_q = c->log_lnq[r];
        for (int q = 0; q < 3; ++q) e.amount[q] = h[4 * r + q];
        e.max_u = h[4 * r + 3];
        e.ms_inversion = t_inv;
        e.ms_dynamics = t_dyn;
        if (c->log.size() >= kMaxRecords) c->log.pop_front();
        c->log.push_back(e);
    }
    return HSF_OK;
}

int hsf_set_step_log(hsf_ctx *c, int on)
{
    if (!c) return HSF_EINVAL;
    if (on && !c->log_d) {
        if (int rc = dalloc(c, (void **)&c->log_d, sizeof(double) * 4 * c->n_rep)) return rc;
        for (hipEvent_t &e : c->log_ev)
            if (!e) HIPCHK(c, hipEventCreate(&e));
    }
    c->step_log = on ? 1 : 0;
    if (!on) c->log.clear();
    return HSF_OK;
}

int hsf_read_step_log(hsf_ctx *c, hsf_step_record *out, int max_records, int *n_read)
{
    if (!c || !out || !n_read || max_records < 0) return HSF_EINVAL;
    int n = 0;
    while (n < max_records && !c->log.empty()) {
        out[n++] = c->log.front();
        c->log.pop_front();
    }
    *n_read = n;
    return HSF_OK;
}

int hsf_step(hsf_ctx *c, int n_steps, double tol, int max_iter, hsf_invert_stats *stats, long long *total_evals)
{
    if (!c || n_steps < 0) return HSF_EINVAL;
    if (total_evals) *total_evals = 0;
    const bool logging = c->step_log != 0;
    if (logging) c->log_inv.assign(c->n_rep, hsf_invert_stats{});
    // the step log needs the counts of every step's inversion (both phases with refinement)
    hsf_invert_stats *inv = logging ? c->log_inv.data() : stats;
    for (int k = 0; k < n_steps; ++k) {
        if (logging) HIPCHK(c, hipEventRecord(c->log_ev[0], c->stream));
        HIPCHK(c, hipMemcpyAsync(c->w_start, c->w, sizeof(double) * c->ch.nsp * c->T, hipMemcpyDeviceToDevice,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(c->st_save, c->st_d, sizeof(RepState) * c->n_rep, hipMemcpyDeviceToDevice,
                                 c->stream));
        // with Crank-Nicolson the fields of phi^n are already converged (phi^n = phi[w^n]
        // after an implicit step): the inversion only confirms them
        const bool implicit = c->integrator == HSF_CD_CRANK_NICOLSON;
        int rc = invert_impl(c, tol, max_iter, implicit ? HSF_WARM_CURRENT : c->step_warm, inv, total_evals,
                             false);
        if (logging && stats) std::copy(c->log_inv.begin(), c->log_inv.end(), stats);
        if (rc == HSF_ENONFINITE) {
            std::string msg = c->err;
            if (int r2 = rollback_step(c)) return r2;
            return fail(c, HSF_ENONFINITE, "%s; the step was rolled back", msg.c_str());
        }
        if (rc == HSF_ENOCONV) {
            if (int r2 = commit_history(c)) return r2;
            return rc;
        }
        if (rc != HSF_OK) return rc;
        if (logging) {
            log_inversion(c);
            HIPCHK(c, hipEventRecord(c->log_ev[1], c->stream));
        }
        *c->bad_h = 0;   // the kernels below set it on a non-finite result
        launch_mu(c->stream, c->plan, c->rep_d, c->ch, c->phi, c->w, c->mu);
        const double *uu = nullptr;
        if (c->hydro) {
            launch_force(c->stream, c->plan, c->rep_d, c->ch, c->phi, c->mu, c->force);
            {
                Timed t(c, HSF_K_LB);
                launch_lb(c->stream, c->plan, c->rep_d, c->nA, c->nB, c->lb32, c->force, c->rho, c->u,
                          (c->noise & HSF_NOISE_LB) != 0, c->noise_step, c->lb_all, t.a, t.b, c->bad_hd);
            }
            uu = c->u;
        }
        if (c->integrator == HSF_CD_CRANK_NICOLSON) {
            // the inversion's fields are kept for the warm starts (the implicit solve replaces
            // the densities below)
            if ((rc = commit_history(c))) return rc;
            // right-hand side phi^n + dt/2 B^n - div J^C + xi, then the implicit solve
            launch_cd(c->stream, c->plan, c->rep_d, c->ch, c->phi, c->mu, uu, c->cn_rhs,
                      (c->noise & HSF_NOISE_CD) ? c->noise_flux : nullptr, c->noise_step, nullptr, nullptr, 0.5,
                      c->bad_hd);
            long long ev = 0;
            rc = cn_solve(c, &ev);
            if (total_evals) *total_evals += ev;
            if (rc == HSF_OK && *c->bad_h) rc = fail(c, HSF_ENONFINITE, "non-finite LB moment or density");
            if (rc == HSF_ENONFINITE) {   // cn_solve stops before it replaces the densities
                std::string msg = c->err;
                if (int r2 = rollback_step(c)) return r2;
                return fail(c, HSF_ENONFINITE, "%s; the step was rolled back", msg.c_str());
            }
            if (c->hydro) std::swap(c->nA, c->nB);
            if (c->noise) ++c->noise_step;
            if (rc != HSF_OK) return rc;
            ++c->steps_done;
            if (logging) {
                HIPCHK(c, hipEventRecord(c->log_ev[2], c->stream));
                if ((rc = log_step(c, c->hydro != 0))) return rc;
            }
            continue;
        }
        {
            Timed t(c, HSF_K_CD);
            launch_cd(c->stream, c->plan, c->rep_d, c->ch, c->phi, c->mu, uu, c->phi_tmp,
                      (c->noise & HSF_NOISE_CD) ? c->noise_flux : nullptr, c->noise_step, t.a, t.b, 1.0,
                      c->bad_hd);
        }
        HIPCHK(c, hipGetLastError());
        if (logging) HIPCHK(c, hipEventRecord(c->log_ev[2], c->stream));
        if ((rc = sync(c))) return rc;
        if (*c->bad_h) {
            if (int r2 = rollback_step(c)) return r2;
            return fail(c, HSF_ENONFINITE, "non-finite LB moment or updated density; the step was rolled back");
        }
        // the step succeeded: keep its inversion for the warm starts (with the targets phi^n),
        // then the new populations and densities
        if ((rc = commit_step(c))) return rc;
        if (c->hydro) std::swap(c->nA, c->nB);
        if (c->noise) ++c->noise_step;   // both noises of a coupled step share its step word
        ++c->steps_done;
        if (logging && (rc = log_step(c, c->hydro != 0))) return rc;
        HIPCHK(c, hipGetLastError());
    }
    return HSF_OK;
}

int hsf_paired_schedule(int n_beads, int launch, int out[8])
{
    if (!out || n_beads < 2 || n_beads > HSF_MAX_BEADS || launch < 1 || launch > n_beads) return HSF_EINVAL;
    const PairSteps ps = paired_steps(n_beads, launch);
    const int v[8] = {ps.sf, ps.sb, ps.f_late, ps.f_from_pp, ps.f_to_pp, ps.g_late, ps.g_exp, ps.g_from_e};
    for (int k = 0; k < 8; ++k) out[k] = v[k];
    return HSF_OK;
}

int hsf_set_timing(hsf_ctx *c, int on)
{
    if (!c) return HSF_EINVAL;
    c->timing = on ? 1 : 0;
    return HSF_OK;
}

int hsf_get_timing(hsf_ctx *c, double *total_ms, long long *count)
{
    if (!c || !total_ms || !count) return HSF_EINVAL;
    int rc = sync(c);
    if (rc) return rc;
    for (int k = 0; k < HSF_K_COUNT; ++k) {
        total_ms[k] = c->tot_ms[k];
        count[k] = c->tot_cnt[k];
        c->tot_ms[k] = 0.0;
        c->tot_cnt[k] = 0;
    }
    return HSF_OK;
}

int hsf_set_tile(hsf_ctx *c, const int cfg[4])
{
    if (!c || !cfg) return HSF_EINVAL;
    TileCfg t{cfg[0], cfg[1], cfg[2], cfg[3]};
    if (!tile_known(t)) return fail(c, HSF_EINVAL, "tile %d,%d,%d,%d is not instantiated", t.cx, t.cy, t.cz, t.k);
    if (tile_lds_bytes(t, lds_real_size(c)) > c->lds_limit) return fail(c, HSF_EINVAL, "tile exceeds the LDS limit");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return set_tile(c, t);
}

int hsf_get_tile(const hsf_ctx *c, int cfg[4])
{
    if (!c || !cfg) return HSF_EINVAL;
    cfg[0] = c->tile.cx;
    cfg[1] = c->tile.cy;
    cfg[2] = c->tile.cz;
    cfg[3] = c->tile.k;
    return HSF_OK;
}

int hsf_autotune(hsf_ctx *c, int reps, double *best_ms)
{
    if (!c || reps < 1) return HSF_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int saved_timing = c->timing;
    c->timing = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    TileCfg best = c->tile;
    float best_t = 1e30f;
    int rc = HSF_OK;
    std::vector<TileCfg> cands;
#define HSF_CAND(CX, CY, CZ, K) cands.push_back(TileCfg{CX, CY, CZ, K});
#define HSF_CANDS(H, CZ, K) HSF_CAND(64, H, CZ, K)
    HSF_TILE_CONFIGS(HSF_CAND)
    HSF_STREAM_CONFIGS(HSF_CANDS)
#undef HSF_CANDS
#undef HSF_CAND
    for (const TileCfg &t : cands) {
        if (tile_lds_bytes(t, lds_real_size(c)) > c->lds_limit) continue;
        if ((rc = set_tile(c, t)) != HSF_OK) break;
        // `reps` evaluations (exp, sweeps, Q, normalisation; state untouched), captured in a
        // graph and replayed as the inversion replays them
        target_setup(c, 0.0, 0);
        run_eval_any(c, 0, 0, c->eval_out, nullptr, 0);
        hipStream_t user = c->stream;
        if (!user && !c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = user ? user : c->cap_stream;
        HIPCHK(c, hipStreamSynchronize(user));
        HIPCHK(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        c->stream = cs;
        for (int k = 0; k < reps; ++k) run_eval_any(c, 0, 0, c->eval_out, nullptr, 0);
        c->stream = user;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e == hipSuccess) e = hipGraphLaunch(exec, c->stream);   // warm
        float ms = 1e30f;
        for (int trial = 0; trial < 2 && e == hipSuccess; ++trial) {   // best of two replays
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) e = hipGraphLaunch(exec, c->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t_ms = 0.0f;
            if (e == hipSuccess) (void)hipEventElapsedTime(&t_ms, e0, e1);
            ms = std::min(ms, t_ms / reps);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (e != hipSuccess) {
            rc = fail(c, HSF_EHIP, "autotune: %s", hipGetErrorString(e));
            break;
        }
        if (ms < best_t) {
            best_t = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = saved_timing;
    if (rc == HSF_OK) rc = set_tile(c, best);
    c->tuned = 1;
    if (best_ms) *best_ms = best_t;
    return rc;
}

int hsf_set_solver(hsf_ctx *c, int flags)
{
    if (!c || (flags & ~(HSF_SOLVER_PRECOND | HSF_SOLVER_REFINE))) return HSF_EINVAL;
    const int pc = (flags & HSF_SOLVER_PRECOND) ? 1 : 0;
    const int rf = (flags & HSF_SOLVER_REFINE) && c->precision == HSF_FP32 ? 1 : 0;
    if (rf && !c->refine) {
        if (tile_lds_bytes(c->tile, sizeof(double)) > c->lds_limit)
            return fail(c, HSF_EINVAL, "the tiling in use does not fit the LDS in FP64");
        // the FP64 propagators of the refinement phase, made once (each buffer only if a
        // call before ran out of memory before reaching it)
        const size_t T = (size_t)c->T;
        void **bufs64[6] = {&c->E64, &c->G64, &c->Gp64[0], &c->Gp64[1], &c->Gf64[0], &c->Gf64[1]};
        const size_t sizes[6] = {2 * T, (size_t)c->ch.N * T, T, T, T, T};
        for (int k = 0; k < 6; ++k)
            if (!*bufs64[k])
                if (int rc = dalloc(c, bufs64[k], sizeof(double) * sizes[k])) return rc;
    }
    c->refine = rf;
    if (pc != c->ch.precond) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->ch.precond = pc;
        c->drop_graphs();   // the flag is a kernel argument of the captured sequences
    }
    return HSF_OK;
}

int hsf_set_warm(hsf_ctx *c, int warm)
{
    if (!c || warm < HSF_WARM_CURRENT || warm > HSF_WARM_NET_EXTRAP) return HSF_EINVAL;
    c->step_warm = warm;
    return HSF_OK;
}

int hsf_set_net_gate(hsf_ctx *c, int min_iters)
{
    if (!c || min_iters < 0) return HSF_EINVAL;
    c->net_gate = min_iters;
    return HSF_OK;
}

int hsf_attach_net(hsf_ctx *c, hsf_net *net)
{
    if (!c) return HSF_EINVAL;
    c->net = net;
    return HSF_OK;
}

int hsf_get_work(hsf_ctx *c, long long *evals, double *site_evals, int reset)
{
    if (!c) return HSF_EINVAL;
    if (evals) *evals = c->work_evals;
    if (site_evals) *site_evals = c->work_site_evals;
    if (reset) {
        c->work_evals = 0;
        c->work_site_evals = 0.0;
    }
    return HSF_OK;
}

// ---- checkpoint: everything a continuation reads ----------------------------------
//
// Layout: StateHeader, the replicas' RepState (inversion control and the per-step
// power-of-two scales), then the FP64 arrays phi, w (field layout), the LB populations
// (per replica [19][V]) and the warm-start history w_hist[2], phi_hist[2].
namespace {
struct StateHeader {
    unsigned long long magic;        // identifies the layout
    int version;
    int n_rep, nsp, N, precision;
    int types[64];                   // bead species (the per-step scales belong to the chain)
    long long T;
    int tile[4];                     // the propagator tiling (summation order of FP32 runs)
    int n_hist, fields_set;
    unsigned long long noise_step;
};
constexpr unsigned long long kStateMagic = 0x4853465354415445ULL;

long long state_doubles(const hsf_ctx *c) { return (long long)(6 * c->ch.nsp + 19) * c->T; }
}  // namespace

long long hsf_state_size(const hsf_ctx *c)
{
    if (!c) return -1;
    return (long long)sizeof(StateHeader) + (long long)sizeof(RepState) * c->n_rep +
           (long long)sizeof(double) * state_doubles(c);
}

int hsf_get_state(hsf_ctx *c, void *buf, long long size)
{
    if (!c || !buf) return HSF_EINVAL;
    if (size < hsf_state_size(c)) return fail(c, HSF_EINVAL, "state buffer of %lld bytes, %lld needed", size,
                                              hsf_state_size(c));
    int rc = sync(c);
    if (rc) return rc;
    char *p = static_cast<char *>(buf);
    StateHeader h{};
    h.magic = kStateMagic;
    h.version = 1;
    h.n_rep = c->n_rep;
    h.nsp = c->ch.nsp;
    h.N = c->ch.N;
    h.precision = c->precision;
    for (int k = 0; k < 64; ++k) h.types[k] = k < c->ch.N ? c->ch.types[k] : -1;
    h.T = c->T;
    h.tile[0] = c->tile.cx;
    h.tile[1] = c->tile.cy;
    h.tile[2] = c->tile.cz;
    h.tile[3] = c->tile.k;
    h.n_hist = c->n_hist;
    h.fields_set = c->fields_set;
    h.noise_step = c->noise_step;
    memcpy(p, &h, sizeof h);
    p += sizeof h;
    HIPCHK(c, hipMemcpy(p, c->st_d, sizeof(RepState) * c->n_rep, hipMemcpyDeviceToHost));
    p += sizeof(RepState) * c->n_rep;
    const size_t nf = (size_t)c->ch.nsp * c->T;
    const double *lb = (const double *)c->nA;
    if (c->lb32) {   // the populations as FP64 values (exact: every FP32 deviation is a double)
        if ((rc = lb_staging(c))) return rc;
        launch_lb_convert(c->stream, c->plan, c->rep_d, false, c->nA, c->lb_stage);
        if ((rc = sync(c))) return rc;
        lb = c->lb_stage;
    }
    const double *src[] = {c->phi, c->w, lb, c->w_hist[0], c->w_hist[1], c->phi_hist[0], c->phi_hist[1]};
    const size_t cnt[] = {nf, nf, (size_t)19 * c->T, nf, nf, nf, nf};
    for (int k = 0; k < 7; ++k) {
        HIPCHK(c, hipMemcpy(p, src[k], sizeof(double) * cnt[k], hipMemcpyDeviceToHost));
        p += sizeof(double) * cnt[k];
    }
    return HSF_OK;
}

int hsf_set_state(hsf_ctx *c, const void *buf, long long size)
{
    if (!c || !buf) return HSF_EINVAL;
    if (size < (long long)sizeof(StateHeader)) return fail(c, HSF_EINVAL, "state buffer too small");
    StateHeader h;
    memcpy(&h, buf, sizeof h);
    if (h.magic != kStateMagic || h.version != 1) return fail(c, HSF_EINVAL, "not a state written by hsf_get_state");
    bool same = h.n_rep == c->n_rep && h.nsp == c->ch.nsp && h.N == c->ch.N && h.precision == c->precision &&
                h.T == c->T;
    for (int k = 0; same && k < c->ch.N; ++k) same = h.types[k] == c->ch.types[k];
    if (!same) return fail(c, HSF_EINVAL, "state of a different context (replicas, species, chain, precision or sites)");
    if (size < hsf_state_size(c)) return fail(c, HSF_EINVAL, "state buffer truncated");
    int rc = sync(c);
    if (rc) return rc;
    const TileCfg t{h.tile[0], h.tile[1], h.tile[2], h.tile[3]};
    if (!tile_known(t)) return fail(c, HSF_EINVAL, "state names an unknown tiling");
    if (t.cx != c->tile.cx || t.cy != c->tile.cy || t.cz != c->tile.cz || t.k != c->tile.k)
        if ((rc = set_tile(c, t))) return rc;
    const char *p = static_cast<const char *>(buf) + sizeof h;
    HIPCHK(c, hipMemcpy(c->st_d, p, sizeof(RepState) * c->n_rep, hipMemcpyHostToDevice));
    memcpy(c->st_h, p, sizeof(RepState) * c->n_rep);
    p += sizeof(RepState) * c->n_rep;
    const size_t nf = (size_t)c->ch.nsp * c->T;
    if (c->lb32 && (rc = lb_staging(c))) return rc;
    double *dst[] = {c->phi, c->w, c->lb32 ? c->lb_stage : (double *)c->nA, c->w_hist[0], c->w_hist[1],
                     c->phi_hist[0], c->phi_hist[1]};
    const size_t cnt[] = {nf, nf, (size_t)19 * c->T, nf, nf, nf, nf};
    for (int k = 0; k < 7; ++k) {
        HIPCHK(c, hipMemcpy(dst[k], p, sizeof(double) * cnt[k], hipMemcpyHostToDevice));
        p += sizeof(double) * cnt[k];
    }
    if (c->lb32) {
        launch_lb_convert(c->stream, c->plan, c->rep_d, true, c->lb_stage, c->nA);
        if ((rc = sync(c))) return rc;
    }
    c->n_hist = h.n_hist;
    c->fields_set = h.fields_set;
    c->noise_step = h.noise_step;
    return HSF_OK;
}

int hsf_set_integrator(hsf_ctx *c, int scheme, double tol, int max_newton, int krylov_dim)
{
    if (!c) return HSF_EINVAL;
    if (scheme == HSF_CD_EXPLICIT) {
        c->integrator = scheme;
        return HSF_OK;
    }
    if (scheme != HSF_CD_CRANK_NICOLSON) return fail(c, HSF_EINVAL, "unknown integrator %d", scheme);
    if (c->precision != HSF_FP64 && tol < 1e-5)
        return fail(c, HSF_EINVAL, "with FP32 propagators the Crank-Nicolson tolerance must be at least 1e-5");
    if (!(tol > 0.0) || max_newton < 1 || krylov_dim < 2 || krylov_dim > kMaxKrylov)
        return fail(c, HSF_EINVAL, "bad Crank-Nicolson parameters (tol %g, max_newton %d, krylov_dim %d)", tol,
                    max_newton, krylov_dim);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc = cn_alloc(c, krylov_dim);
    if (rc) return rc;
    c->integrator = scheme;
    c->cn_tol = tol;
    c->cn_max_newton = max_newton;
    c->cn_m = krylov_dim;
    return HSF_OK;
}

int hsf_get_cn_stats(const hsf_ctx *c, hsf_cn_stats *st)
{
    if (!c || !st) return HSF_EINVAL;
    *st = c->cn_last;
    return HSF_OK;
}

int hsf_set_noise(hsf_ctx *c, int flags, double omega, unsigned long long seed, unsigned long long step)
{
    if (!c) return HSF_EINVAL;
    if (flags & ~(HSF_NOISE_CD | HSF_NOISE_LB)) return fail(c, HSF_EINVAL, "unknown noise flags %d", flags);
    if (flags && !(omega > 0.0 && std::isfinite(omega))) return fail(c, HSF_EINVAL, "noise needs Omega > 0");
    HIPCHK(c, hipStreamSynchronize(c->stream));   // kernels in flight read the replica table
    if ((flags & HSF_NOISE_CD) && !c->noise_flux) {
        int rc = dalloc(c, (void **)&c->noise_flux, sizeof(double) * 3 * c->ch.nsp * c->T);
        if (rc) return rc;
    }
    for (auto &R : c->reps) {
        R.omega = flags ? omega : 0.0;
        R.seed = seed;
    }
    HIPCHK(c, hipMemcpy(c->rep_d, c->reps.data(), sizeof(Rep) * c->n_rep, hipMemcpyHostToDevice));
    for (Plan *pl : {&c->plan, &c->tplan})
        for (int r = 0; r < pl->args.n; ++r) pl->args.rep[r] = c->reps[r];
    c->noise = flags;
    c->noise_step = step;
    return HSF_OK;
}

int hsf_get_noise_step(const hsf_ctx *c, unsigned long long *step)
{
    if (!c || !step) return HSF_EINVAL;
    *step = c->noise_step;
    return HSF_OK;
}

int hsf_set_hydro(hsf_ctx *c, int on)
{
    if (!c) return HSF_EINVAL;
    c->hydro = on ? 1 : 0;
    return HSF_OK;
}

}  // extern "C"
