// static_eval.hip -- the density functional of hsf_evaluate for callers that cannot
// allocate device memory: one replica, no context, every scratch buffer (propagators,
// partial sums, plans, descriptor and control state) carved out of one file-scope device
// array.  The kernels are the library's own (one contour step per launch, the 32x8
// column tiling with 2 planes per thread).
#include <algorithm>
#include <mutex>

#include "hsf_internal.h"
#include "prop_block.h"

using namespace hsf;

namespace {

// Scratch of the allocation-free entry point.  Each GPU the library runs on holds its own
// copy for the life of the process; calls on one GPU share it.
static __device__ __align__(256) unsigned char scratch[HSF_STATIC_SCRATCH_BYTES];

constexpr TileCfg kStaticTile{32, 8, 2, 0};
constexpr int kMaxDevices = 64;

// Device address of `scratch` per device, taken once with that device current (in host
// code the array's name is only a stand-in, not a device address).
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {nullptr};

int scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HSF_EHIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HSF_EHIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return HSF_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Descriptor, cleared control state and the two one-replica block tables (site plan and
// tile plan), written by a kernel: no host copies and no memset nodes.
__global__ __launch_bounds__(kBlock) void k_static_setup(Rep R, Rep *rep, RepState *st, int *blk_rep, int *blk_first,
                                                         int nbs, int *tblk_rep, int *tblk_first, int nbt)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        rep[0] = R;
        blk_first[0] = 0;
        blk_first[1] = nbs;
        tblk_first[0] = 0;
        tblk_first[1] = nbt;
    }
    int *sw = reinterpret_cast<int *>(st);
    for (int k = t; k < (int)(sizeof(RepState) / 4); k += gridDim.x * blockDim.x) sw[k] = 0;
    for (int k = t; k < nbs; k += gridDim.x * blockDim.x) blk_rep[k] = 0;
    for (int k = t; k < nbt; k += gridDim.x * blockDim.x) tblk_rep[k] = 0;
}

// Q of the evaluation (NaN when it left the floating-point range).
__global__ void k_static_q(const RepState *st, double *q_out)
{
    q_out[0] = st->nonfinite ? __builtin_nan("") : exp(st->ln_q);
}

struct Layout {
    size_t rep, st, blk_rep, blk_first, tblk_rep, tblk_first, part, partG, E, G, Gp0, Gp1, total;
};

Layout layout(long long V, int N, size_t rs, int nbs, int nbt)
{
    Layout L{};
    const int nb = std::max(nbs, nbt);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.rep = take(sizeof(Rep));
    L.st = take(sizeof(RepState));
    L.blk_rep = take(sizeof(int) * nbs);
    L.blk_first = take(sizeof(int) * 2);
    L.tblk_rep = take(sizeof(int) * nbt);
    L.tblk_first = take(sizeof(int) * 2);
    L.part = take(sizeof(double) * kNQ * nb);
    L.partG = take(sizeof(double) * (N + 2) * nb);
    L.E = take(rs * 2 * V);
    L.G = take(rs * (size_t)N * V);
    L.Gp0 = take(rs * V);
    L.Gp1 = take(rs * V);
    L.total = o;
    return L;
}

template <typename real>
void static_pass(hipStream_t s, const Plan &plan, const Plan &tplan, Rep *rep, RepState *st, const Chain &ch,
                 PropBufs<real> b, const double *w, const double *phi, double *phi_out, double *part, double *partG)
{
    const int N = ch.N;
    launch_target_stats(s, plan, rep, st, ch, phi, w, part);
    launch_reduce_ctl(s, 1, plan, st, rep, part, PH_TARGET, ch, partG, 0.0, 0, nullptr);
    for (int s0 = 0; s0 < N; ++s0)
        launch_fwd_block<real>(kStaticTile, s, tplan, rep, st, ch, s0, 1, b, partG, 1, w, nullptr, 0, nullptr,
                               nullptr);
    const bool fold_q = N > 1;   // with N = 1 step 1 is step N: Q first, in its own launch
    if (!fold_q) launch_reduce_ctl(s, 1, tplan, st, rep, part, PH_Q, ch, partG, 0.0, 0, nullptr);
    int parity = 0;
    for (int s_hi = N; s_hi >= 1; --s_hi) {
        launch_bwd_block<real>(kStaticTile, s, tplan, rep, st, ch, s_hi, 1, b, b.Gp[parity ^ 1], b.Gp[parity],
                               nullptr, 0, phi, nullptr, phi_out, part, partG, fold_q ? 1 : 0, nullptr, nullptr);
        parity ^= 1;
    }
    launch_reduce_ctl(s, 1, tplan, st, rep, part, PH_SCALES, ch, partG, 0.0, 0, nullptr);
}

}  // namespace

extern "C" int hsf_evaluate_static(const hsf_params *p, const double *w, const double *phi, double *phi_out,
                                   double *q_out, void *hip_stream)
{
    if (!p || !w || !phi || !phi_out || !q_out) return HSF_EINVAL;
    if (p->n_beads < 1 || p->n_beads > HSF_MAX_BEADS) return HSF_EINVAL;
    if (p->precision != HSF_FP64 && p->precision != HSF_FP32) return HSF_EINVAL;
    if (p->Lx < 1 || p->Ly < 1 || p->Lz < 1) return HSF_EINVAL;
    if ((long long)p->Lx * p->Ly * p->Lz > HSF_MAX_SITES) return HSF_EINVAL;
    for (int s = 0; s < p->n_beads; ++s)
        if (p->types[s] < 0 || p->types[s] > 1) return HSF_EINVAL;
    Rep R{};
    R.Lx = p->Lx;
    R.Ly = p->Ly;
    R.Lz = p->Lz;
    R.V = (long long)p->Lx * p->Ly * p->Lz;
    R.site_off = 0;
    const bool given = p->stencil[0] != 0.0 || p->stencil[1] != 0.0 || p->stencil[2] != 0.0 || p->stencil[3] != 0.0;
    if (given) {
        for (int k = 0; k < 4; ++k) R.c[k] = p->stencil[k];
    } else {   // tensor product of [al, 1 - 2 al, al], al = a^2 / 6
        const double al = p->a * p->a / 6.0, m = 1.0 - 2.0 * al;
        R.c[0] = m * m * m;
        R.c[1] = al * m * m;
        R.c[2] = al * al * m;
        R.c[3] = al * al * al;
    }
    R.csum = R.c[0] + 6.0 * R.c[1] + 12.0 * R.c[2] + 8.0 * R.c[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R.chi[i][j] = p->chi[i][j];
    R.kappa = p->kappa;
    R.dt = p->dt;
    R.tau = p->tau;
    Chain ch{};
    ch.N = p->n_beads;
    ch.nsp = p->has_solvent ? 3 : 2;
    ch.precond = 0;
    for (int s = 0; s < 64; ++s) ch.types[s] = s < ch.N ? p->types[s] : 0;

    const size_t rs = p->precision == HSF_FP32 ? sizeof(float) : sizeof(double);
    const long long nbs_ll = (R.V + kBlock - 1) / kBlock;
    const long long nbt_ll = (long long)((R.Lx + kStaticTile.cx - 1) / kStaticTile.cx) *
                             ((R.Ly + kStaticTile.cy - 1) / kStaticTile.cy) * ((R.Lz + kStaticTile.cz - 1) / kStaticTile.cz);
    if (nbs_ll > (1LL << 30) || nbt_ll > (1LL << 30)) return HSF_EINVAL;
    const int nbs = (int)nbs_ll, nbt = (int)nbt_ll;
    const Layout L = layout(R.V, ch.N, rs, nbs, nbt);
    if (L.total > (size_t)HSF_STATIC_SCRATCH_BYTES) return HSF_EINVAL;

    unsigned char *base = nullptr;
    if (scratch_address((void **)&base) != HSF_OK) return HSF_EHIP;
    hipStream_t s = (hipStream_t)hip_stream;
    Rep *rep = (Rep *)(base + L.rep);
    RepState *st = (RepState *)(base + L.st);
    Plan plan, tplan;
    plan.nblocks = nbs;
    plan.n_rep = 1;
    plan.blk_rep = (int *)(base + L.blk_rep);
    plan.blk_first = (int *)(base + L.blk_first);
    tplan.nblocks = nbt;
    tplan.n_rep = 1;
    tplan.blk_rep = (int *)(base + L.tblk_rep);
    tplan.blk_first = (int *)(base + L.tblk_first);
    const int bf_s[2] = {0, nbs}, bf_t[2] = {0, nbt};
    set_plan_args(plan, &R, 1, bf_s);
    set_plan_args(tplan, &R, 1, bf_t);
    double *part = (double *)(base + L.part), *partG = (double *)(base + L.partG);

    hipLaunchKernelGGL(k_static_setup, dim3(64), dim3(kBlock), 0, s, R, rep, st, plan.blk_rep, plan.blk_first, nbs,
                       tplan.blk_rep, tplan.blk_first, nbt);
    // FP32 propagators: the first pass measures the per-step power-of-two scales, the second
    // evaluates with them (the context-based evaluation carries them between calls)
    const int passes = p->precision == HSF_FP32 ? 2 : 1;
    for (int k = 0; k < passes; ++k) {
        if (p->precision == HSF_FP32) {
            PropBufs<float> b{(float *)(base + L.E), (float *)(base + L.G), {(float *)(base + L.Gp0), (float *)(base + L.Gp1)}};
            static_pass<float>(s, plan, tplan, rep, st, ch, b, w, phi, phi_out, part, partG);
        } else {
            PropBufs<double> b{(double *)(base + L.E), (double *)(base + L.G),
                               {(double *)(base + L.Gp0), (double *)(base + L.Gp1)}};
            static_pass<double>(s, plan, tplan, rep, st, ch, b, w, phi, phi_out, part, partG);
        }
    }
    if (ch.nsp == 3) {
        launch_solvent(s, plan, rep, st, ch, 0, w, phi, phi_out, part);
        launch_reduce_ctl(s, 1, plan, st, rep, part, PH_SOLVENT, ch, partG, 0.0, 0, nullptr);
        launch_solvent(s, plan, rep, st, ch, 1, w, phi, phi_out, part);
    }
    hipLaunchKernelGGL(k_static_q, dim3(1), dim3(1), 0, s, st, q_out);
    return hipGetLastError() == hipSuccess ? HSF_OK : HSF_EHIP;
}
