// prop_block.h -- tile configurations of the temporally blocked propagator kernels.
#pragma once

#include "hsf_internal.h"

namespace hsf {

// Core tile (cx, cy, cz) and contour steps per launch (k).  k = 0 selects the direct
// kernels: one contour step per launch, neighbours read through the caches, a block
// covers cx x cy columns (cx * cy = 256) of cz planes.  k = -1 selects the paired
// direct kernels: a launch takes one forward and one backward step (same tiles).
struct TileCfg {
    int cx, cy, cz, k;
};

// The instantiated configurations (X(cx, cy, cz, k)); the autotuner picks one per context.
#define HSF_TILE_CONFIGS(X) \
    X(64, 4, 1, 0)          \
    X(32, 8, 1, 0)          \
    X(16, 16, 1, 0)         \
    X(64, 4, 2, 0)          \
    X(32, 8, 2, 0)          \
    X(16, 16, 2, 0)         \
    X(64, 4, 4, 0)          \
    X(32, 8, 4, 0)          \
    X(16, 16, 4, 0)         \
    X(64, 4, 8, 0)          \
    X(16, 16, 8, 0)         \
    X(64, 4, 2, -1)         \
    X(64, 4, 4, -1)         \
    X(32, 8, 2, -1)         \
    X(16, 16, 2, -1)        \
    X(32, 8, 4, -1)         \
    X(16, 16, 4, -1)        \
    X(16, 16, 8, -1)        \
    X(8, 8, 8, 1)           \
    X(8, 8, 8, 2)           \
    X(8, 8, 8, 3)           \
    X(8, 8, 8, 4)           \
    X(16, 8, 8, 2)          \
    X(16, 8, 4, 2)          \
    X(32, 8, 4, 1)          \
    X(32, 4, 4, 2)

// The z-streaming sweeps (X(H, CZ, K)): a wavefront's 64 lanes are consecutive x sites,
// each lane holds H rows in y and the wavefront walks a z-chunk of CZ core planes, K contour
// steps per launch; as a tiling they read {64, H, CZ, K}.
#define HSF_STREAM_CONFIGS(X) \
    X(8, 8, 2)                \
    X(8, 16, 2)               \
    X(16, 8, 2)               \
    X(16, 16, 2)              \
    X(16, 32, 2)

inline bool tile_is_stream(const TileCfg &t) { return t.cx == 64 && t.k >= 1; }

// Work items of a streaming tiling in one replica's box: ntx x nty x ntz wavefront tiles
// (the kernels cut the box the same way), four per workgroup.
inline long long stream_blocks(const TileCfg &t, int Lx, int Ly, int Lz)
{
    const int wx = 64 - 2 * t.k, wy = t.cy - 2 * t.k;
    const long long ntiles = (long long)((Lx + wx - 1) / wx) * ((Ly + wy - 1) / wy) * ((Lz + t.cz - 1) / t.cz);
    return (ntiles + 3) / 4;
}

// Bytes of LDS a configuration needs (two staged regions + FP64 core accumulators).
inline size_t tile_lds_bytes(const TileCfg &t, size_t real_bytes)
{
    if (t.k <= 0 || tile_is_stream(t)) return 0;
    const size_t nr = (size_t)(t.cx + 2 * t.k) * (t.cy + 2 * t.k) * (t.cz + 2 * t.k);
    return 2 * nr * real_bytes + 2 * (size_t)t.cx * t.cy * t.cz * sizeof(double);
}

template <typename real>
void launch_field_exp(hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch, const double *w,
                      const double *d, int use_alpha, real *E, hipEvent_t e0, hipEvent_t e1);
// w (may be null): with one-step kernels the first forward launch also computes the field
// factors from w (+ alpha d when use_alpha), in place of launch_field_exp.
template <typename real>
void launch_fwd_block(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                      int s0, int n, PropBufs<real> b, double *partG, int sums, const double *w, const double *d,
                      int use_alpha, hipEvent_t e0, hipEvent_t e1);
// fold_q: with one-step kernels the first backward launch (1), or with paired kernels the
// last one (2), also computes Q from the forward sweep's partials, in place of the control
// launch of that phase.
template <typename real>
void launch_bwd_block(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                      int s_hi, int n, PropBufs<real> b, const real *gin, real *gout, double *acc, int final_mode,
                      const double *phit, const double *d, double *out, double *part, const double *partG,
                      int fold_q, hipEvent_t e0, hipEvent_t e1);

// Streaming sweeps: forward steps s0 + 1 .. s0 + n, and backward steps s_hi .. s_hi - n + 1
// with the density sums of the earlier backward launches in the store (see prop_stream.hip).
template <typename real>
void launch_fwd_stream(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                       int s0, int n, PropBufs<real> b, double *partG, int sums, hipEvent_t e0, hipEvent_t e1);
template <typename real>
void launch_bwd_stream(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                       int s_hi, int n, PropBufs<real> b, const real *gin, real *gout, int final_mode,
                       const double *phit, const double *d, double *out, double *part, hipEvent_t e0, hipEvent_t e1);

// One launch of the paired sweeps: forward step sf and backward step sb (0: none) and
// where each reads and writes its propagators (the schedule is built by the evaluation).
struct PairSteps {
    int sf, sb;
    int f_late, f_from_pp, f_to_pp, g_late, g_exp, g_from_e;
};
template <typename real>
void launch_pair_block(const TileCfg &cfg, hipStream_t s, const Plan &p, const Rep *rep, RepState *st, Chain ch,
                       const PairSteps &ps, PropBufs<real> b, const real *fin, real *fout, const real *gin,
                       real *gout, double *partG, int sums, const double *w, const double *d, int use_alpha,
                       hipEvent_t e0, hipEvent_t e1);

}  // namespace hsf
