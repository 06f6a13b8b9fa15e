// dyn.hip -- the dynamics around the density functional:
//   chemical potential (eq. 4) and thermodynamic force (eq. 8);
//   D3Q19 lattice Boltzmann, moments (eq. 9), equilibrium (eq. 11), single-relaxation
//   collision L_ij = -delta_ij / tau with its forcing term, collide then stream (eq. 10);
//   conservative convection-diffusion update (eq. 3);
//   optional thermal noise: LB mode noise (eq. 13) and composition noise (eq. 5).
#include <hip/hip_ext.h>
#include <math.h>

#include "device_common.h"
#include "philox.h"

namespace hsf {

// D3Q19 velocities: rest, 6 faces, 12 edges (order documented in hsf.h).
constexpr int kCx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Weights of eq. 11.
__host__ __device__ constexpr double lb_w(int q) { return q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// LB populations in memory: FP64 values n_i, or (FP32 storage) the deviations n_i - w_i
// from the rest state, whose magnitude is that of the flow and density perturbations, so
// FP32 keeps about 7 significant digits of the perturbation rather than of n_i.  All
// arithmetic is FP64.
__device__ __forceinline__ double pop_load(const double *p, long long k, int) { return p[k]; }
__device__ __forceinline__ double pop_load(const float *p, long long k, int q) { return lb_w(q) + (double)p[k]; }
__device__ __forceinline__ void pop_store(double *p, long long k, int, double v) { p[k] = v; }
__device__ __forceinline__ void pop_store(float *p, long long k, int q, double v) { p[k] = (float)(v - lb_w(q)); }

__device__ __forceinline__ void site_xyz(const Rep &R, long long i, int &x, int &y, int &z)
{
    x = (int)(i % R.Lx);
    y = (int)((i / R.Lx) % R.Ly);
    z = (int)(i / ((long long)R.Lx * R.Ly));
}

__device__ __forceinline__ long long sidx(const Rep &R, int x, int y, int z)
{
    return (long long)x + (long long)R.Lx * ((long long)y + (long long)R.Ly * z);
}

// x-neighbours by lane exchange.  In a site plan the lanes of a wavefront hold
// consecutive sites of one replica, so the lane to the left holds site x - 1 of the same
// row unless the site is the first of its row or the lane the first of its wavefront,
// and likewise to the right; those lanes load the neighbour instead.  Every lane takes
// part in the exchange (lanes past the box's end work on its last site and store
// nothing); the values are the loads they replace, so results are unchanged bit for bit.
struct XLanes {
    bool lw, rw;   // the neighbour is held by the adjacent lane
    int dl, dr;    // offsets of the periodic x - 1 and x + 1 from the site
};

__device__ __forceinline__ XLanes x_lanes(int x, int Lx)
{
    const int lane = threadIdx.x & 63;
    XLanes n;
    n.lw = lane > 0 && x > 0;
    n.rw = lane < 63 && x < Lx - 1;
    n.dl = x > 0 ? -1 : Lx - 1;
    n.dr = x < Lx - 1 ? 1 : 1 - Lx;
    return n;
}

// f at x - 1 and x + 1 of site k, given c = f[k].
template <typename Idx>
__device__ __forceinline__ void x_pair(const double *f, Idx k, double c, const XLanes &n, double &l, double &r)
{
    l = from_left(c);
    r = from_right(c);
    if (!n.lw) l = f[k + n.dl];
    if (!n.rw) r = f[k + n.dr];
}

// The same for NR rows at once, in one round trip to memory: with every row's centre each
// lane also loads one more value, its outer x neighbour if it is an edge lane (the left one
// if it lacks the left, else the right one) and its own site otherwise, so the edge values
// arrive with the centres; only a lane lacking both neighbours (rows shorter than a
// wavefront) loads its right neighbour afterwards.
template <int NR, typename Idx>
__device__ __forceinline__ void x_rows(const double *f, const Idx (&k)[NR], const XLanes &n, double (&c)[NR],
                                       double (&l)[NR], double (&r)[NR])
{
    const int eo = !n.lw ? n.dl : (!n.rw ? n.dr : 0);
    double e[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        c[q] = f[k[q]];
        e[q] = f[k[q] + eo];
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const double fl = from_left(c[q]), fr = from_right(c[q]);
        l[q] = n.lw ? fl : e[q];
        r[q] = n.rw ? fr : e[q];
    }
    if (!n.lw && !n.rw) {
#pragma unroll
        for (int q = 0; q < NR; ++q) r[q] = f[k[q] + n.dr];
    }
}

// mu_I = -w_I + sum_J chi_IJ sigma[phi_J] + kappa (sum_J phi_J - 1); the stencil sums
// are formed per class (centre, faces, edges, corners) as in stencil27.  Sites are
// addressed by 32-bit offsets from each species' base (a replica holds fewer than 2^31
// sites), and the nine rows of every species are loaded together.
template <int NSP>
__global__ __launch_bounds__(kBlock) void k_mu(const int *__restrict__ blk_rep, const int *__restrict__ blk_first,
                                               const Rep *__restrict__ rep, Chain ch,
                                               const double *__restrict__ phi, const double *__restrict__ w,
                                               double *__restrict__ mu)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const int V = (int)R.V, Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const bool live = sr.i < V;
    const int i = live ? (int)sr.i : V - 1;
    const int x = i % Lx, y = (i / Lx) % Ly, z = i / (Lx * Ly);
    const XLanes xn = x_lanes(x, Lx);
    const long long fo = off_field(R, NSP);
    const int dym = (wrap1(y - 1, Ly) - y) * Lx, dyp = (wrap1(y + 1, Ly) - y) * Lx;
    const int dzm = (wrap1(z - 1, Lz) - z) * Lx * Ly, dzp = (wrap1(z + 1, Lz) - z) * Lx * Ly;
    // rows: the site's, four with exactly one of (dy, dz) non-zero, four with both
    const int k[9] = {i, i + dym, i + dyp, i + dzm, i + dzp, i + dym + dzm, i + dym + dzp, i + dyp + dzm, i + dyp + dzp};
    double sp[3] = {0, 0, 0}, tot = 0.0;
#pragma unroll 1
    for (int J = 0; J < NSP; ++J) {
        const double *f = phi + fo + (long long)J * V;
        double c[9], l[9], r[9];
        x_rows(f, k, xn, c, l, r);
        double s0 = c[0], s1 = l[0] + r[0], s2 = 0, s3 = 0;
        tot += c[0];
#pragma unroll
        for (int q = 1; q < 5; ++q) {
            s1 += c[q];
            s2 += l[q] + r[q];
        }
#pragma unroll
        for (int q = 5; q < 9; ++q) {
            s2 += c[q];
            s3 += l[q] + r[q];
        }
        sp[J] = R.c[0] * s0 + R.c[1] * s1 + R.c[2] * s2 + R.c[3] * s3;
    }
    if (!live) return;
#pragma unroll
    for (int I = 0; I < NSP; ++I) {
        double inter = 0.0;
#pragma unroll
        for (int J = 0; J < NSP; ++J) inter += R.chi[I][J] * sp[J];
        const long long k = fo + (long long)I * V;
        mu[k + i] = -w[k + i] + inter + R.kappa * (tot - 1.0);
    }
}

// f = -dt^2 sum_I phi_I (mu_I(r + e) - mu_I(r - e)) / 2 per axis (LB units).
__global__ __launch_bounds__(kBlock) void k_force(const int *__restrict__ blk_rep,
                                                  const int *__restrict__ blk_first, const Rep *__restrict__ rep,
                                                  Chain ch, const double *__restrict__ phi,
                                                  const double *__restrict__ mu, double *__restrict__ f)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    if (i >= V) return;
    int x, y, z;
    site_xyz(R, i, x, y, z);
    const long long fo = off_field(R, ch.nsp);
    const long long nb[6] = {sidx(R, wrap1(x + 1, R.Lx), y, z), sidx(R, wrap1(x - 1, R.Lx), y, z),
                             sidx(R, x, wrap1(y + 1, R.Ly), z), sidx(R, x, wrap1(y - 1, R.Ly), z),
                             sidx(R, x, y, wrap1(z + 1, R.Lz)), sidx(R, x, y, wrap1(z - 1, R.Lz))};
    double acc[3] = {0, 0, 0};
    for (int I = 0; I < ch.nsp; ++I) {
        const double *m = mu + fo + I * V;
        const double p = phi[fo + I * V + i];
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a] += p * (0.5 * (m[nb[2 * a]] - m[nb[2 * a + 1]]));
    }
    const double k = -R.dt * R.dt;
    const long long vo = 3LL * R.site_off;
#pragma unroll
    for (int a = 0; a < 3; ++a) f[vo + a * V + i] = k * acc[a];
}

// Multiple-relaxation-time collision (eq. 12-14) in the orthogonal basis of Table 1:
// e_k(c) for k = 0..18, orthogonal under the weights w_i; b_k = sum_i w_i e_k(c_i)^2.
__host__ __device__ constexpr double mrt_e(int k, int cx, int cy, int cz)
{
    const double x = cx, y = cy, z = cz, c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return x * x - y * y;
    case 6: return c2 - 3.0 * z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (x * x - y * y);
    default: return (2.0 * c2 - 3.0) * (c2 - 3.0 * z * z);
    }
}


// The basis at the 19 velocities and 1 / b_k, as compile-time tables (the unrolled
// projections below index them with constants).
struct MrtTable {
    double e[19][19];   // [k][q]
    double binv[19];
};

constexpr MrtTable make_mrt_table()
{
    MrtTable t{};
    for (int k = 0; k < 19; ++k) {
        double b = 0.0;
        for (int q = 0; q < 19; ++q) {
            t.e[k][q] = mrt_e(k, kCx[q], kCy[q], kCz[q]);
            b += lb_w(q) * t.e[k][q] * t.e[k][q];
        }
        t.binv[k] = 1.0 / b;
    }
    return t;
}

__device__ constexpr MrtTable kMrt = make_mrt_table();

// Post-collision populations of one site for the MRT scheme: n* = n_eq + w_i sum_k
// e_k(c_i) m*_k / b_k with m*_k = gamma_k (n - n_eq)_k + (Delta^f)_k, where the forcing
// Delta^f_i = (w_i / c_s^2) [f.c_i + Sigma : (c_i c_i - c_s^2 1) / (2 c_s^2)] and
// Sigma = (1 + gamma_s)/2 (u f + f u - 2/3 (u.f) 1) + (1 + gamma_b)/3 (u.f) 1 (eq. 14).
__device__ __forceinline__ void mrt_collide(const double *n, double rho, double ux, double uy, double uz, double fx,
                                            double fy, double fz, const Rep &R, double *ns)
{
    const double gs = R.gamma_s, gb = R.gamma_b, gg = R.gamma_ghost;
    const double uu = ux * ux + uy * uy + uz * uz, uf = ux * fx + uy * fy + uz * fz;
    // Sigma (symmetric)
    const double as = 0.5 * (1.0 + gs), ab = (1.0 + gb) / 3.0;
    const double sxx = as * (2.0 * ux * fx - 2.0 / 3.0 * uf) + ab * uf;
    const double syy = as * (2.0 * uy * fy - 2.0 / 3.0 * uf) + ab * uf;
    const double szz = as * (2.0 * uz * fz - 2.0 / 3.0 * uf) + ab * uf;
    const double sxy = as * (ux * fy + uy * fx), sxz = as * (ux * fz + uz * fx), syz = as * (uy * fz + uz * fy);
    const double trs = sxx + syy + szz;
    double dn[19], df[19], neq[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const double cx = kCx[q], cy = kCy[q], cz = kCz[q];
        const double cu = cx * ux + cy * uy + cz * uz;
        neq[q] = rho * lb_w(q) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        dn[q] = n[q] - neq[q];
        // Sigma : (c c - 1/3) = c.Sigma.c - tr(Sigma)/3
        const double scc = cx * cx * sxx + cy * cy * syy + cz * cz * szz +
                           2.0 * (cx * cy * sxy + cx * cz * sxz + cy * cz * syz) - trs / 3.0;
        df[q] = 3.0 * lb_w(q) * (cx * fx + cy * fy + cz * fz + 1.5 * scc);
    }
    double ms[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) {
        double m = 0.0, mf = 0.0;
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const double e = kMrt.e[k][q];
            m += e * dn[q];
            mf += e * df[q];
        }
        const double g = k <= 3 ? 1.0 : (k == 4 ? gb : (k <= 9 ? gs : gg));
        ms[k] = (g * m + mf) * kMrt.binv[k];
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < 19; ++k) a += kMrt.e[k][q] * ms[k];
        ns[q] = neq[q] + lb_w(q) * a;
    }
}

// Mode noise of eq. 13 added to the post-collision populations ns of site i of replica r:
// mode k >= 4 receives phi_k r_k, phi_k = sqrt(rho kT b_k (1 - gamma_k^2) / c_s^2), carried
// to the populations as w_q e_k(c_q) phi_k r_k / b_k.  kT = dt^2 / Omega in LB units;
// gamma_k of the collision (BGK: 1 - 1/tau for every non-conserved mode).  r_k are the
// normal numbers of purposes 0-3 (mode k takes number k - 4).
__device__ __forceinline__ void lb_mode_noise(const Rep &R, int r, long long i, unsigned long long step,
                                              double rho, double *ns)
{
    double z[16];
#pragma unroll
    for (int p = 0; p < 4; ++p) normals4(R.seed, (uint64_t)r, (uint64_t)i, step, (uint64_t)p, z + 4 * p);
    const double rk = 3.0 * fmax(rho, 0.0) * (R.dt * R.dt / R.omega);
    const bool mrt = R.lb_mode == HSF_LB_MRT;
    const double gbgk = 1.0 - 1.0 / R.tau;
    double a[19];
#pragma unroll
    for (int k = 4; k < 19; ++k) {
        const double g = mrt ? (k == 4 ? R.gamma_b : (k <= 9 ? R.gamma_s : R.gamma_ghost)) : gbgk;
        a[k] = sqrt(rk * (1.0 - g * g) * kMrt.binv[k]) * z[k - 4];
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int k = 4; k < 19; ++k) acc += kMrt.e[k][q] * a[k];
        ns[q] += lb_w(q) * acc;
    }
}

// One LB step, push form: read the 19 pre-collision populations of this site,
// take the moments of eq. 9 (u with the half-force shift), relax towards the
// equilibrium of eq. 11 with rate 1/tau, add the forcing term
//   F_i = (1 - 1/(2 tau)) w_i [3 (c_i - u).f + 9 (c_i.u)(c_i.f)],
// and write each post-collision population to the neighbour it streams to.  NOISE adds
// the mode noise of eq. 13 before streaming.  MODE: HSF_LB_BGK or HSF_LB_MRT when every
// replica uses that collision (each variant needs only its own registers), -1 for a batch
// that mixes them (chosen per replica).
template <bool NOISE, int MODE, typename pop_t>
__global__ __launch_bounds__(kBlock) void k_lb(const int *__restrict__ blk_rep, const int *__restrict__ blk_first,
                                               const Rep *__restrict__ rep, const pop_t *__restrict__ nsrc,
                                               pop_t *__restrict__ ndst, const double *__restrict__ f,
                                               double *__restrict__ rho_out, double *__restrict__ u_out,
                                               unsigned long long step, int *__restrict__ bad)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    if (i >= V) return;
    int x, y, z;
    site_xyz(R, i, x, y, z);
    const long long base = 19LL * R.site_off, vo = 3LL * R.site_off;
    double n[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) n[q] = pop_load(nsrc, base + q * V + i, q);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (f) {
        fx = f[vo + i];
        fy = f[vo + V + i];
        fz = f[vo + 2 * V + i];
    }
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        rho += n[q];
        jx += kCx[q] * n[q];
        jy += kCy[q] * n[q];
        jz += kCz[q] * n[q];
    }
    const double ux = (jx + 0.5 * fx) / rho, uy = (jy + 0.5 * fy) / rho, uz = (jz + 0.5 * fz) / rho;
    // a non-finite population or force shows in the moments; the host rolls the step back
    if (bad && !(isfinite(rho) && isfinite(ux) && isfinite(uy) && isfinite(uz))) bad[0] = 1;
    double ns[19];
    const bool mrt = MODE == HSF_LB_MRT || (MODE < 0 && R.lb_mode == HSF_LB_MRT);
    if (mrt) {
        mrt_collide(n, rho, ux, uy, uz, fx, fy, fz, R, ns);
    } else {
        const double om = 1.0 / R.tau, fp = 1.0 - 0.5 / R.tau;
        const double uu = ux * ux + uy * uy + uz * uz;
        const double uf = ux * fx + uy * fy + uz * fz;
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const double cu = kCx[q] * ux + kCy[q] * uy + kCz[q] * uz;
            const double cf = kCx[q] * fx + kCy[q] * fy + kCz[q] * fz;
            const double wq = lb_w(q);
            const double neq = rho * wq * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            const double F = fp * wq * (3.0 * (cf - uf) + 9.0 * cu * cf);
            ns[q] = n[q] - om * (n[q] - neq) + F;
            if (!NOISE) {   // stored at once: fewer live registers
                const int xd = wrap1(x + kCx[q], R.Lx), yd = wrap1(y + kCy[q], R.Ly), zd = wrap1(z + kCz[q], R.Lz);
                pop_store(ndst, base + q * V + sidx(R, xd, yd, zd), q, ns[q]);
            }
        }
    }
    if (NOISE) lb_mode_noise(R, sr.r, i, step, rho, ns);
    if (NOISE || mrt) {
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const int xd = wrap1(x + kCx[q], R.Lx), yd = wrap1(y + kCy[q], R.Ly), zd = wrap1(z + kCz[q], R.Lz);
            pop_store(ndst, base + q * V + sidx(R, xd, yd, zd), q, ns[q]);
        }
    }
    rho_out[R.site_off + i] = rho;
    u_out[vo + i] = ux;
    u_out[vo + V + i] = uy;
    u_out[vo + 2 * V + i] = uz;
}

// Conservative convection-diffusion update.  Face between r and r + e_a:
//   J = dt * (-(phi_r + phi_e)/2 (mu_e - mu_r))
//     + [(phi_r + phi_e)/2 - ((phi u_a)_e - (phi u_a)_r)/2] (u_a,r + u_a,e)/2
// phi_new(r) = phi(r) - sum_a (J(r + e_a/2) - J(r - e_a/2)).
// NOISE adds the composition noise of eq. 5 as a random flux on every bond, drawn
// beforehand by k_cd_noise into jn.
template <bool NOISE, int NSP>
__global__ __launch_bounds__(kBlock) void k_cd(const int *__restrict__ blk_rep, const int *__restrict__ blk_first,
                                               const Rep *__restrict__ rep, Chain ch,
                                               const double *__restrict__ phi, const double *__restrict__ mu,
                                               const double *__restrict__ u, double *__restrict__ phi_out,
                                               const double *__restrict__ jn, double diff_scale,
                                               int *__restrict__ bad)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const int V = (int)R.V, Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const bool live = sr.i < V;
    const int i = live ? (int)sr.i : V - 1;
    const int x = i % Lx, y = (i / Lx) % Ly, z = i / (Lx * Ly);
    const XLanes xn = x_lanes(x, Lx);
    const long long fo = off_field(R, NSP), vo = 3LL * R.site_off;
    // y and z neighbours (32-bit offsets: a replica holds fewer than 2^31 sites)
    const int nb[6] = {i + xn.dl, i + xn.dr,
                       i + (wrap1(y - 1, Ly) - y) * Lx, i + (wrap1(y + 1, Ly) - y) * Lx,
                       i + (wrap1(z - 1, Lz) - z) * Lx * Ly, i + (wrap1(z + 1, Lz) - z) * Lx * Ly};
    const double dt = R.dt * diff_scale;   // diffusive flux over dt (or dt/2 in the CN step)
    // Every load is issued before the first lane exchange: the rows that take their x
    // neighbours from the adjacent lanes (phi and mu of each species, u_x) with one more
    // value per row (an edge lane's outer x neighbour, else its own site), and the y and z
    // neighbours of all of them.  Without a velocity field the u rows read phi and are
    // replaced by zero.
    constexpr int NR = 2 * NSP + 1;
    const double *rows[NR];
#pragma unroll
    for (int I = 0; I < NSP; ++I) {
        rows[2 * I] = phi + fo + (long long)I * V;
        rows[2 * I + 1] = mu + fo + (long long)I * V;
    }
    const double *ub = u ? u + vo : phi + fo;
    rows[2 * NSP] = ub;
    double c[NR], lo[NR], hi[NR], ex[NR];
    const int eo = !xn.lw ? xn.dl : (!xn.rw ? xn.dr : 0);   // an edge lane's outer neighbour
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        c[q] = rows[q][i];
        ex[q] = rows[q][i + eo];
    }
    double uyz[2][3];   // u_y, u_z at (lower neighbour, site, upper neighbour)
#pragma unroll
    for (int a = 1; a < 3; ++a) {
        const double *ua = u ? ub + (long long)a * V : ub;
        uyz[a - 1][0] = ua[nb[2 * a]];
        uyz[a - 1][1] = ua[i];
        uyz[a - 1][2] = ua[nb[2 * a + 1]];
    }
    double pyz[NSP][4], myz[NSP][4];   // (y-, y+, z-, z+)
#pragma unroll
    for (int I = 0; I < NSP; ++I) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pyz[I][q] = rows[2 * I][nb[2 + q]];
            myz[I][q] = rows[2 * I + 1][nb[2 + q]];
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const double fl = from_left(c[q]), fr = from_right(c[q]);
        lo[q] = xn.lw ? fl : ex[q];
        hi[q] = xn.rw ? fr : ex[q];
    }
    if (!xn.lw && !xn.rw) {   // rows shorter than a wavefront: both neighbours from memory
#pragma unroll
        for (int q = 0; q < NR; ++q) hi[q] = rows[q][nb[1]];
    }
    // the velocity at the site and its six neighbours, shared by the species
    double ul[3] = {0, 0, 0}, ur[3] = {0, 0, 0}, uh[3] = {0, 0, 0};
    if (u) {
        ul[0] = lo[2 * NSP];
        ur[0] = c[2 * NSP];
        uh[0] = hi[2 * NSP];
#pragma unroll
        for (int a = 1; a < 3; ++a) {
            ul[a] = uyz[a - 1][0];
            ur[a] = uyz[a - 1][1];
            uh[a] = uyz[a - 1][2];
        }
    }
#pragma unroll
    for (int I = 0; I < NSP; ++I) {
        const double pr = c[2 * I], mr = c[2 * I + 1];
        const double pn_l[3] = {lo[2 * I], pyz[I][0], pyz[I][2]}, pn_h[3] = {hi[2 * I], pyz[I][1], pyz[I][3]};
        const double mn_l[3] = {lo[2 * I + 1], myz[I][0], myz[I][2]},
                     mn_h[3] = {hi[2 * I + 1], myz[I][1], myz[I][3]};
        double div = 0.0;
        const double *jI = NOISE ? jn + 3 * fo + 3 * (long long)I * V : nullptr;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // face between lo and r, then between r and hi
            const double pl = pn_l[a], ph = pn_h[a];
            double jl = dt * (-0.5 * (pl + pr) * (mr - mn_l[a]));
            double jh = dt * (-0.5 * (pr + ph) * (mn_h[a] - mr));
            if (u) {
                jl += (0.5 * (pl + pr) - 0.5 * (pr * ur[a] - pl * ul[a])) * (0.5 * (ul[a] + ur[a]));
                jh += (0.5 * (pr + ph) - 0.5 * (ph * uh[a] - pr * ur[a])) * (0.5 * (ur[a] + uh[a]));
            }
            if (NOISE) {
                jl += jI[(long long)a * V + nb[2 * a]];
                jh += jI[(long long)a * V + i];
            }
            div += jh - jl;
        }
        const double pn = pr - div;
        if (!live) continue;
        if (bad && !isfinite(pn)) bad[0] = 1;
        phi_out[fo + (long long)I * V + i] = pn;
    }
}

// Composition noise of eq. 5 as random bond fluxes: the bond between site s and
// s + e_a of species I carries jn = sqrt(2 dt max(phi_bond, 0) / Omega) g with
// phi_bond = (phi_I(s) + phi_I(s + e_a)) / 2 and g number a of the normal numbers of
// (site s, purpose 4 + I).  Its divergence conserves each species exactly and has the
// covariance (2 dt / Omega)(-div phi grad) of eq. 5 over a step.
// Layout of jn: per replica [species][3][V] at 3 nsp site_off.
__global__ __launch_bounds__(kBlock) void k_cd_noise(const int *__restrict__ blk_rep,
                                                     const int *__restrict__ blk_first,
                                                     const Rep *__restrict__ rep, Chain ch,
                                                     const double *__restrict__ phi, double *__restrict__ jn,
                                                     unsigned long long step)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    if (i >= V) return;
    int x, y, z;
    site_xyz(R, i, x, y, z);
    const long long fo = off_field(R, ch.nsp);
    const long long up[3] = {sidx(R, wrap1(x + 1, R.Lx), y, z), sidx(R, x, wrap1(y + 1, R.Ly), z),
                             sidx(R, x, y, wrap1(z + 1, R.Lz))};
    for (int I = 0; I < ch.nsp; ++I) {
        const double *p = phi + fo + I * V;
        double g[4];
        normals4(R.seed, (uint64_t)sr.r, (uint64_t)i, step, (uint64_t)(4 + I), g);
        const double pr = p[i];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            jn[3 * fo + (3 * I + a) * V + i] = sqrt(2.0 * R.dt * fmax(0.5 * (pr + p[up[a]]), 0.0) / R.omega) * g[a];
    }
}

// Fluid at rest with density 1: n_i = w_i.
template <typename pop_t>
__global__ __launch_bounds__(kBlock) void k_lb_rest(const int *__restrict__ blk_rep,
                                                    const int *__restrict__ blk_first, const Rep *__restrict__ rep,
                                                    pop_t *__restrict__ n)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    if (i >= V) return;
#pragma unroll
    for (int q = 0; q < 19; ++q) pop_store(n, 19LL * R.site_off + q * V + i, q, lb_w(q));
}

// FP64 populations to the FP32 deviation storage (to_f32) or back.
__global__ __launch_bounds__(kBlock) void k_lb_convert(const int *__restrict__ blk_rep,
                                                       const int *__restrict__ blk_first,
                                                       const Rep *__restrict__ rep, int to_f32,
                                                       const void *__restrict__ src, void *__restrict__ dst)
{
    const SiteRef sr = site_ref(blk_rep, blk_first);
    const Rep &R = rep[sr.r];
    const long long V = R.V, i = sr.i;
    if (i >= V) return;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const long long k = 19LL * R.site_off + q * V + i;
        if (to_f32) pop_store((float *)dst, k, q, ((const double *)src)[k]);
        else ((double *)dst)[k] = pop_load((const float *)src, k, q);
    }
}

void launch_mu(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phi, const double *w,
               double *mu)
{
    hipLaunchKernelGGL(ch.nsp == 3 ? k_mu<3> : k_mu<2>, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first,
                       rep, ch, phi, w, mu);
}

void launch_force(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phi, const double *mu,
                  double *f)
{
    hipLaunchKernelGGL(k_force, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, ch, phi, mu, f);
}

template <typename pop_t>
static void launch_lb_t(hipStream_t s, const Plan &p, const Rep *rep, const pop_t *nsrc, pop_t *ndst,
                        const double *f, double *rho, double *u, bool noise, unsigned long long step, int lb_mode,
                        hipEvent_t e0, hipEvent_t e1, int *bad)
{
    auto pick = [&](auto bgk, auto mrt, auto mixed) { return lb_mode == HSF_LB_BGK ? bgk : lb_mode == HSF_LB_MRT ? mrt : mixed; };
    auto kern = noise ? pick(k_lb<true, HSF_LB_BGK, pop_t>, k_lb<true, HSF_LB_MRT, pop_t>, k_lb<true, -1, pop_t>)
                      : pick(k_lb<false, HSF_LB_BGK, pop_t>, k_lb<false, HSF_LB_MRT, pop_t>, k_lb<false, -1, pop_t>);
    if (e0)
        hipExtLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, e0, e1, 0, p.blk_rep, p.blk_first, rep,
                              nsrc, ndst, f, rho, u, step, bad);
    else
        hipLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, nsrc, ndst, f,
                           rho, u, step, bad);
}

void launch_lb(hipStream_t s, const Plan &p, const Rep *rep, const void *nsrc, void *ndst, bool f32, const double *f,
               double *rho, double *u, bool noise, unsigned long long step, int lb_mode, hipEvent_t e0,
               hipEvent_t e1, int *bad)
{
    if (f32)
        launch_lb_t<float>(s, p, rep, (const float *)nsrc, (float *)ndst, f, rho, u, noise, step, lb_mode, e0, e1,
                           bad);
    else
        launch_lb_t<double>(s, p, rep, (const double *)nsrc, (double *)ndst, f, rho, u, noise, step, lb_mode, e0,
                            e1, bad);
}

void launch_lb_convert(hipStream_t s, const Plan &p, const Rep *rep, bool to_f32, const void *src, void *dst)
{
    hipLaunchKernelGGL(k_lb_convert, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep,
                       to_f32 ? 1 : 0, src, dst);
}

void launch_cd(hipStream_t s, const Plan &p, const Rep *rep, Chain ch, const double *phi, const double *mu,
               const double *u, double *phi_out, double *noise_flux, unsigned long long step, hipEvent_t e0,
               hipEvent_t e1, double diff_scale, int *bad)
{
    // with noise the events bracket both kernels: e0 at the start of the flux draw
    if (noise_flux) {
        if (e0)
            hipExtLaunchKernelGGL(k_cd_noise, dim3(p.nblocks), dim3(kBlock), 0, s, e0, nullptr, 0, p.blk_rep,
                                  p.blk_first, rep, ch, phi, noise_flux, step);
        else
            hipLaunchKernelGGL(k_cd_noise, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, ch,
                               phi, noise_flux, step);
        e0 = nullptr;
    }
    auto kern = noise_flux ? (ch.nsp == 3 ? k_cd<true, 3> : k_cd<true, 2>) : (ch.nsp == 3 ? k_cd<false, 3> : k_cd<false, 2>);
    if (e0 || e1)
        hipExtLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, e0, e1, 0, p.blk_rep, p.blk_first, rep,
                              ch, phi, mu, u, phi_out, (const double *)noise_flux, diff_scale, bad);
    else
        hipLaunchKernelGGL(kern, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep, ch, phi, mu, u,
                           phi_out, (const double *)noise_flux, diff_scale, bad);
}

void launch_lb_rest(hipStream_t s, const Plan &p, const Rep *rep, void *n, bool f32)
{
    if (f32)
        hipLaunchKernelGGL(k_lb_rest<float>, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep,
                           (float *)n);
    else
        hipLaunchKernelGGL(k_lb_rest<double>, dim3(p.nblocks), dim3(kBlock), 0, s, p.blk_rep, p.blk_first, rep,
                           (double *)n);
}

}  // namespace hsf
