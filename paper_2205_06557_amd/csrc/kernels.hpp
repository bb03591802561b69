// kernels.hpp -- the HIP kernels of one time step.
//
//   pair_forces_f32 / pair_forces_f64   forces on every ion (Section 2):
//       screened (Yukawa) ion-ion sum over all other ions, bare Coulomb pull
//       of each grain, homogeneous drive; plus the per-grain sum of Eq. (1)
//       over all ions, reduced per block and added to int64 fixed-point
//       accumulators.
//   step_tail_kernel<T, FIX>  the rest of the step, per ion: acceleration
//       from the symmetric pair sum's totals plus the grain terms and the
//       Eq. (1) summands (FIX), kick, charge exchange, drift, absorption test
//       against every grain along the drift segment, exit test, per-ion
//       event byte, list of lost ions; the system's last block to finish
//       updates the charges (the three
//       charging models of Section 2), assembles the four force parts of
//       Eqs. (1)-(4) in SI, records the step, keeps the time averages,
//       clears the accumulators and advances the step counter.
//   reinject_kernel<T>  new boundary position and velocity of every listed
//       ion (Appendix B).
//   init_kernel<T>      initial uniform positions and shifted-Maxwellian
//       velocities.
//   conf_grid_kernel<T> potential of the plasma outside the domain on the
//       (r, z) grid of Appendix A, from the ions at the time of the call.
//
// Dimensionless units: length r_De, time 1/omega_pi, velocity c_s, charge e.
#pragma once

#include "device_common.hpp"

namespace odk {

struct DustSet {
    int nd;
    int pad_;
    double pos[kMaxDust][3];
    double rad2[kMaxDust];
};

// Confinement field of the plasma outside the domain (Appendix A), in
// dimensionless form: potential in k_B T_e / e and lengths in r_De, so that
// the field is the ion's dimensionless acceleration.  The fitted potential is
// P = sum_m c[m] u^a_m v^b_m with u = (x^2 + y^2) iu, v = z^2 iv, the terms in
// the order of Eq. (A.3): (a, b) = (0,0) (1,0) (0,1) (1,1) (2,0) (0,2) (2,1)
// (1,2) (3,0) (0,3) (2,2) (3,1) (1,3) (4,0) (0,4).
struct ConfField {
    int on, pad_;
    double c[15];
    double iu, iv;      // 1 / rs^2, 1 / zs^2 (rs = R, zs = H / 2)
};

// E = -grad P at (x, y, z), Eq. (A.4); the u and v derivatives written out
// term by term.
__host__ __device__ inline void conf_field(const ConfField& f, double x, double y, double z,
                                           double& ex, double& ey, double& ez)
{
#pragma clang fp contract(off)
    const double* c = f.c;
    const double u = (x * x + y * y) * f.iu, v = z * z * f.iv;
    const double u2 = u * u, v2 = v * v;
    const double dPu = c[1] + c[3] * v + 2.0 * c[4] * u + 2.0 * c[6] * u * v + c[7] * v2 +
                       3.0 * c[8] * u2 + 2.0 * c[10] * u * v2 + 3.0 * c[11] * u2 * v +
                       c[12] * v2 * v + 4.0 * c[13] * u2 * u;
    const double dPv = c[2] + c[3] * u + 2.0 * c[5] * v + c[6] * u2 + 2.0 * c[7] * u * v +
                       3.0 * c[9] * v2 + 2.0 * c[10] * u2 * v + c[11] * u2 * u +
                       3.0 * c[12] * u * v2 + 4.0 * c[14] * v2 * v;
    const double gu = -2.0 * dPu * f.iu;
    ex = gu * x;
    ey = gu * y;
    ez = -2.0 * dPv * f.iv * z;
}

struct PairArgs {
    int N, Npad, nd, ion_ion;
    float C;        // ion-ion coupling: (superparticle weight)/(4 pi n r_De^3) = V/(4 pi N)
    float pad_;
    double Cd;      // same in FP64
    double Kq;      // ion<-grain coupling per unit grain charge (e): 1/(4 pi n r_De^3)
    double Ez;      // homogeneous drive along z (dimensionless acceleration)
    double sym_scale;   // fixed-point scale of the symmetric kernel's raw pair sums
    ConfField cf;   // confinement field, added to every ion when cf.on
};

constexpr unsigned kFlagLiteralSide = 1u;   // side injection without the tangential part
constexpr unsigned kFlagFieldDriven = 8u;   // field-driven collisional flow distribution

struct PushArgs {
    int N, Npad, nd;
    unsigned flags;
    double dt, sig, ubar, R, H;
    uint64_t k0, k1, Tc, Tb, Tbt;
    double ufd;     // field-driven flow: mean drift gained between collisions, a / nu
};

struct FinalArgs {
    int nd, mode;
    long long n_discard;
    double dt;                      // dimensionless step
    double w;                       // superparticle weight (ions per superparticle)
    double Ie0[kMaxDust];           // electron random current at phi = 0, e per unit time
    double Ii0[kMaxDust];           // ion thermal current factor pi a^2 n v_t, e per unit time
    double psi[kMaxDust];           // e phi / kB Te per unit charge (e)
    double s_oml, te_over_ti;       // drift / v_t ; Te/Ti
    double c_orbit;                 // N per (e * dimensionless Eq.(1) sum), times w
    double c_dd;                    // N per e^2 per dimensionless 1/r^2
    double c_coll;                  // N per (dimensionless velocity sum)
    double c_ext;                   // N per e (e * E_SI)
    double eout[kMaxDust][3];       // N per e: e * E_out(r_d) of the confinement field, or 0
    double* hist;                   // per-step records [hist_cap][nd][kHistWords], or null
    long long hist_start, hist_cap; // steps hist_start .. hist_start + hist_cap - 1 are recorded
};

// Words of one per-step record: Q^n (e), the twelve force components (SI),
// the absorbed count.
constexpr int kHistWords = 14;

// ---------------------------------------------------------------------------
// End of a block of 256 target ions: adds (when epi) the grain terms in FP64
// (N_d per ion), the drive and the confinement field to the ion-ion sum
// (gx, gy, gz), writes the acceleration to slot `out` of the output planes,
// and adds the block's share of the Eq. (1) sums to the int64 fixed-point
// accumulators.
template <int BLOCK>
__device__ __forceinline__ void pair_epilogue(float xi, float yi, float zi, int out, bool live,
                                              double gx, double gy, double gz, bool epi,
                                              const PairArgs& p, const DustSet& ds,
                                              Ctl* __restrict__ ctl, float* __restrict__ oX,
                                              float* __restrict__ oY, float* __restrict__ oZ,
                                              double (*red)[kMaxDust][3])
{
    if (epi) {
        const double xd = xi, yd = yi, zd = zi;
        gz += p.Ez;
        if (p.cf.on) {
            double ex, ey, ez;
            conf_field(p.cf, xd, yd, zd, ex, ey, ez);
            gx += ex; gy += ey; gz += ez;
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int d = 0; d < ds.nd; ++d) {
            const double rx = xd - ds.pos[d][0], ry = yd - ds.pos[d][1], rz = zd - ds.pos[d][2];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double r = sqrt(r2);
            const double ir3 = 1.0 / (r2 * r);
            const double kq = p.Kq * ctl->Q[d] * ir3;               // bare Coulomb on the ion
            gx += kq * rx; gy += kq * ry; gz += kq * rz;
            // Eq. (1) summand: (1 + rho) e^-rho / rho^3 (r_d - x_i)
            double f = live ? -(1.0 + r) * exp(-r) * ir3 : 0.0;
            double fx = wave_sum(f * rx), fy = wave_sum(f * ry), fz = wave_sum(f * rz);
            if (lane == 0) {
                red[wv][d][0] = fx;
                red[wv][d][1] = fy;
                red[wv][d][2] = fz;
            }
        }
    }
    if (live) {
        oX[out] = (float)gx;
        oY[out] = (float)gy;
        oZ[out] = (float)gz;
    }
    if (epi) {
        __syncthreads();
        for (int t = threadIdx.x; t < ds.nd * 3; t += BLOCK) {
            const int d = t / 3, c = t % 3;
            double s = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) s += red[w][d][c];
            atomicAdd(&ctl->part[blockIdx.x % kSlots][d][c], to_fixed(s, kForceScale, &ctl->status));
        }
    }
    __syncthreads();
}

// Forces, FP32 tiles.  One block's share of the pair sum: target ions
// [i0, i0 + BLOCK) of one system (planes X/Y/Z, local indices) against the
// sources [jb, je), one target per lane.  The block stages TJ sources at a
// time in LDS as float4 and every lane reads them with a broadcast load;
// sums run in FP32 over a tile and are added to FP64 totals per tile.  The
// result (times the ion-ion coupling) goes to out planes oX/oY/oZ.  With
// `epi` set, the grain and drive terms are added and the Eq. (1) sums of the
// block are reduced and added to the system's fixed-point accumulators.
template <int BLOCK, int TJ>
__device__ __forceinline__ void pair_block_f32(const float* __restrict__ X,
                                               const float* __restrict__ Y,
                                               const float* __restrict__ Z, int i0, int jb,
                                               int je, const PairArgs& p, const DustSet& ds,
                                               Ctl* __restrict__ ctl, float* __restrict__ oX,
                                               float* __restrict__ oY, float* __restrict__ oZ,
                                               bool epi, float4* tile,
                                               double (*red)[kMaxDust][3])
{
    const int i = i0 + threadIdx.x;
    const float xi = X[i], yi = Y[i], zi = Z[i];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    const float kNegLog2e = -1.4426950408889634f;

    if (p.ion_ion) {
        for (int j0 = jb; j0 < je; j0 += TJ) {
            __syncthreads();
            for (int t = threadIdx.x; t < TJ; t += BLOCK)
                tile[t] = make_float4(X[j0 + t], Y[j0 + t], Z[j0 + t], 0.0f);
            __syncthreads();
            float ax = 0.0f, ay = 0.0f, az = 0.0f;
            const bool diag = (j0 < i0 + BLOCK) && (i0 < j0 + TJ);
            if (!diag) {
#pragma unroll 8
                for (int k = 0; k < TJ; ++k) {
                    const float4 q = tile[k];
                    const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float ri = __builtin_amdgcn_rsqf(r2);
                    const float r = r2 * ri;
                    const float e = __builtin_amdgcn_exp2f(r * kNegLog2e);
                    const float ri2 = ri * ri;
                    const float f = fmaf(ri2, ri, ri2) * e;      // (1 + r) e^-r / r^3
                    ax = fmaf(f, dx, ax);
                    ay = fmaf(f, dy, ay);
                    az = fmaf(f, dz, az);
                }
            } else {
                const int kself = i - j0;
                for (int k = 0; k < TJ; ++k) {
                    const float4 q = tile[k];
                    const float dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float ri = __builtin_amdgcn_rsqf(r2);
                    const float r = r2 * ri;
                    const float e = __builtin_amdgcn_exp2f(r * kNegLog2e);
                    const float ri2 = ri * ri;
                    float f = fmaf(ri2, ri, ri2) * e;
                    f = (k == kself) ? 0.0f : f;
                    ax = fmaf(f, dx, ax);
                    ay = fmaf(f, dy, ay);
                    az = fmaf(f, dz, az);
                }
            }
            sx += (double)ax;
            sy += (double)ay;
            sz += (double)az;
        }
    }

    pair_epilogue<BLOCK>(xi, yi, zi, i, i < p.N, p.Cd * sx, p.Cd * sy, p.Cd * sz, epi, p, ds, ctl,
                         oX, oY, oZ, red);
}

template <int BLOCK, int TJ>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8)))
void pair_forces_f32(const float* __restrict__ xs,
                                                         float* __restrict__ acc,
                                                         PairArgs p, DustSet ds,
                                                         Ctl* __restrict__ ctl, int nsplit)
{
    __shared__ float4 tile[TJ];
    __shared__ double red[BLOCK / 64][kMaxDust][3];
    const int Npad = p.Npad;
    const int nib = Npad / BLOCK, tiles = Npad / TJ;
    const int ib = blockIdx.x % nib, k = blockIdx.x / nib;
    const int jb = (tiles * k / nsplit) * TJ, je = (tiles * (k + 1) / nsplit) * TJ;
    float* o = acc + (long long)k * 3 * Npad;
    pair_block_f32<BLOCK, TJ>(xs, xs + Npad, xs + 2 * Npad, ib * BLOCK, jb, je, p, ds, ctl, o,
                              o + Npad, o + 2 * Npad, k == 0, tile, red);
}

// Forces, FP64 throughout (precision mode OD_PREC_FP64).
// FP64 pair terms of one target against a staged tile of TJ sources;
// Self: the tile holds the target itself (source index `self`), whose term
// is dropped.
template <int TJ, bool Self>
__device__ __forceinline__ void f64_tile(const double4* __restrict__ tile, double xi, double yi, double zi,
                                         int self, double& sx, double& sy, double& sz)
{
    for (int k = 0; k < TJ; ++k) {
        const double4 q = tile[k];
        const double dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double ri = rsq_f64(r2);
        const double r = r2 * ri;
        const double e = exp_neg_f64(r);
        double f = fma(r, e, e) * (ri * ri * ri);         // (1 + r) e^-r / r^3
        if (Self) f = (k == self) ? 0.0 : f;
        sx += f * dx;
        sy += f * dy;
        sz += f * dz;
    }
}

template <int BLOCK, int TJ>
__global__ __launch_bounds__(BLOCK) void pair_forces_f64(const double* __restrict__ xs,
                                                         double* __restrict__ acc,
                                                         PairArgs p, DustSet ds,
                                                         Ctl* __restrict__ ctl)
{
    static_assert(BLOCK == TJ, "the block's own tile is the one source tile holding its targets");
    __shared__ double4 tile[TJ];
    __shared__ double red[BLOCK / 64][kMaxDust][3];
    const int Npad = p.Npad;
    const double* X = xs;
    const double* Y = xs + Npad;
    const double* Z = xs + 2 * Npad;
    const int i0 = blockIdx.x * BLOCK;
    const int i = i0 + threadIdx.x;
    const double xi = X[i], yi = Y[i], zi = Z[i];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (p.ion_ion) {
        for (int j0 = 0; j0 < Npad; j0 += TJ) {
            __syncthreads();
            for (int t = threadIdx.x; t < TJ; t += BLOCK) {
                double4 q;
                q.x = X[j0 + t]; q.y = Y[j0 + t]; q.z = Z[j0 + t]; q.w = 0.0;
                tile[t] = q;
            }
            __syncthreads();
            if (j0 == i0)      // the block's own tile holds the self-pair
                f64_tile<TJ, true>(tile, xi, yi, zi, threadIdx.x, sx, sy, sz);
            else
                f64_tile<TJ, false>(tile, xi, yi, zi, threadIdx.x, sx, sy, sz);
        }
    }
    const bool live = i < p.N;
    double gx = p.Cd * sx, gy = p.Cd * sy, gz = p.Cd * sz + p.Ez;
    if (p.cf.on) {
        double ex, ey, ez;
        conf_field(p.cf, xi, yi, zi, ex, ey, ez);
        gx += ex; gy += ey; gz += ez;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int d = 0; d < ds.nd; ++d) {
        const double rx = xi - ds.pos[d][0], ry = yi - ds.pos[d][1], rz = zi - ds.pos[d][2];
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double r = sqrt(r2);
        const double ir3 = 1.0 / (r2 * r);
        const double kq = p.Kq * ctl->Q[d] * ir3;
        gx += kq * rx; gy += kq * ry; gz += kq * rz;
        double f = live ? -(1.0 + r) * exp(-r) * ir3 : 0.0;
        double fx = wave_sum(f * rx), fy = wave_sum(f * ry), fz = wave_sum(f * rz);
        if (lane == 0) {
            red[wv][d][0] = fx;
            red[wv][d][1] = fy;
            red[wv][d][2] = fz;
        }
    }
    if (live) {
        acc[i] = gx;
        acc[Npad + i] = gy;
        acc[2 * Npad + i] = gz;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ds.nd * 3; t += BLOCK) {
        const int d = t / 3, c = t % 3;
        double s = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) s += red[w][d][c];
        atomicAdd(&ctl->part[blockIdx.x % kSlots][d][c], to_fixed(s, kForceScale, &ctl->status));
    }
}

// ---------------------------------------------------------------------------
// Boundary sampling helpers (Appendix B), dimensionless, FP64.

__device__ inline double npdf(double t) { return 0.3989422804014326779 * exp(-0.5 * t * t); }

// Inflow per unit area through a face whose inward normal velocity is
// N(m, s^2): int_0^inf v phi(v) dv.
__device__ inline double inflow(double m, double s)
{
    return m * 0.5 * erfc(-m / (s * 1.4142135623730950488)) + s * npdf(m / s);
}

// Flux-weighted normal speed on a face: the v >= 0 whose flux tail
// int_v^inf v' phi(v') dv' equals uu times the total inflow.  Newton on the
// tail (slope -v phi(v)) inside a shrinking bracket, bisection when a Newton
// step would not land strictly inside it; stops when a step is below
// 1e-13 s, or when the tail equals the goal to within the rounding of its
// own evaluation, 8 ulp of the magnitudes of its terms (where the flux
// density is tiny the root is resolved no further than that).
__device__ double flux_speed(double uu, double m, double s)
{
    const double goal = uu * inflow(m, s);
    double lo = 0.0;
    double hi = fmax(m, 0.0) + 40.0 * s;
    double v = fmax(m, 0.0) + s;
    for (int it = 0; it < 400; ++it) {
        const double t = (v - m) / s;
        const double t1 = m * 0.5 * erfc(t * 0.70710678118654752440), t2 = s * npdf(t);
        const double g = (t1 + t2) - goal;
        if (fabs(g) <= 8.0 * 2.220446049250313e-16 * (fabs(t1) + t2)) break;
        if (g > 0.0) lo = v; else hi = v;
        const double slope = -v * npdf(t) / s;
        double nv = 0.5 * (lo + hi);
        if (slope < 0.0) {
            const double cand = v - g / slope;
            if (cand > lo && cand < hi) nv = cand;
        }
        const bool done = fabs(nv - v) <= 1e-13 * s;
        v = nv;
        if (done) break;
    }
    return v;
}

// Field-driven collisional flow (constant-frequency charge exchange in a
// homogeneous field): in the stationary flow v_z = sig g + ufd T with g
// standard normal and T ~ Exp(1) the time since the last collision in units
// of 1/nu.  With A(x) = exp(c - x/ufd) Phi(x/sig - sig/ufd), c = sig^2 /
// (2 ufd^2), its density is A(x)/ufd and, integrating by parts,
//   int_x^inf v phi dv      = (x + ufd) A(x) + sig pdf(x/sig) + ufd Phic(x/sig),
//   -int_-inf^-w v phi dv   = (ufd - w) A(-w) + sig pdf(w/sig) - ufd Phic(w/sig).
// A is evaluated through erfcx where its argument is non-negative, so that
// neither factor overflows.
__device__ inline double fd_A(double x, double ufd, double sig)
{
    const double z = (sig / ufd - x / sig) * 0.70710678118654752440;
    if (z >= 0.0) return 0.5 * exp(-0.5 * (x / sig) * (x / sig)) * erfcx(z);
    const double r = sig / ufd;
    return 0.5 * exp(0.5 * r * r - x / ufd) * erfc(z);
}

// Flux-weighted inward speed at the bottom (top = false, v_z = s) or top
// (v_z = -s) face for the field-driven distribution: the s >= 0 whose flux
// tail is uu times the face's inflow.  Safeguarded Newton as flux_speed.
__device__ double fd_speed(double uu, double ufd, double sig, bool top)
{
    const double k = 0.70710678118654752440;
    // tail at v, its slope and the magnitude of its terms (rounding scale)
    auto tail = [&](double v, double& slope, double& mag) {
        const double A = fd_A(top ? -v : v, ufd, sig);
        slope = -v * A / ufd;
        const double t1 = (top ? ufd - v : v + ufd) * A, t2 = sig * npdf(v / sig);
        const double t3 = ufd * 0.5 * erfc(v / sig * k);
        mag = fabs(t1) + t2 + t3;
        return top ? (t1 + t2) - t3 : (t1 + t2) + t3;
    };
    double slope, mag;
    const double goal = uu * tail(0.0, slope, mag);
    double lo = 0.0, hi = 40.0 * sig + (top ? 0.0 : 50.0 * ufd);
    double v = top ? sig : ufd + sig;
    for (int it = 0; it < 400; ++it) {
        const double g = tail(v, slope, mag) - goal;
        if (fabs(g) <= 8.0 * 2.220446049250313e-16 * mag) break;   // as flux_speed
        if (g > 0.0) lo = v; else hi = v;
        double nv = 0.5 * (lo + hi);
        if (slope < 0.0) {
            const double cand = v - g / slope;
            if (cand > lo && cand < hi) nv = cand;
        }
        const bool done = fabs(nv - v) <= 1e-13 * sig;
        v = nv;
        if (done) break;
    }
    return v;
}

// New position and velocity of a lost ion, from blocks (i, n, REINJ, 0/1).
__device__ void reinject(const PushArgs& p, uint64_t ion, uint64_t n, double o[6])
{
    const U64x4 a = philox(ion, n, kReinj, 0, p.k0, p.k1);
    const U64x4 b = philox(ion, n, kReinj, 1, p.k0, p.k1);
    double g1, g2;
    gauss2(unit(b.w[0]), unit(b.w[1]), g1, g2);
    if (a.w[0] < p.Tbt) {                       // bottom or top disk
        const bool bottom = a.w[0] < p.Tb;
        const double rr = p.R * sqrt(unit(a.w[1]));
        double sn, cs;
        sincos(2.0 * kPi * unit(a.w[2]), &sn, &cs);
        o[0] = rr * cs;
        o[1] = rr * sn;
        o[2] = bottom ? -0.5 * p.H : 0.5 * p.H;
        o[3] = p.sig * g1;
        o[4] = p.sig * g2;
        if (p.flags & kFlagFieldDriven)
            o[5] = bottom ? fd_speed(unit(a.w[3]), p.ufd, p.sig, false)
                          : -fd_speed(unit(a.w[3]), p.ufd, p.sig, true);
        else
            o[5] = bottom ? flux_speed(unit(a.w[3]), p.ubar, p.sig)
                          : -flux_speed(unit(a.w[3]), -p.ubar, p.sig);
    } else {                                    // side wall
        double sn, cs;
        sincos(2.0 * kPi * unit(a.w[1]), &sn, &cs);
        o[0] = p.R * cs;
        o[1] = p.R * sn;
        o[2] = p.H * (unit(a.w[2]) - 0.5);
        const double vr = p.sig * sqrt(-2.0 * log(unit(a.w[3])));
        const double vt = (p.flags & kFlagLiteralSide) ? 0.0 : p.sig * g2;
        o[3] = -vr * cs - vt * sn;
        o[4] = -vr * sn + vt * cs;
        // v_z from phi(v_z); the field-driven flow adds T = -ln u2 of block 1
        o[5] = (p.flags & kFlagFieldDriven) ? p.sig * g1 - p.ufd * log(unit(b.w[2]))
                                            : p.ubar + p.sig * g1;
    }
}

// ---------------------------------------------------------------------------
// The per-ion tail of a step, one kernel: acceleration (for the symmetric
// pair sum: its fixed-point totals plus the grain, drive and confinement
// terms, and the ion's share of the Eq. (1) sums), kick, charge exchange,
// drift, absorption test against every grain along the drift segment, exit
// test, reinjection of a lost ion on the boundary (Appendix B) by the thread
// that lost it, and, in the last block of the system to finish, the charge
// update and force assembly.

// Charge exchange of ion i in step n (Section 2, constant frequency): the
// first word of block (i, n, COLL, 0) below Tc = floor(P 2^64), P = 1 - e^(-nu dt).
// It depends on no ion data, so the step's tail evaluates it while the ion's
// loads are in flight.
__device__ __forceinline__ bool collision_decision(int i, uint64_t n, const PushArgs& p)
{
    return p.Tc != 0 && philox((uint64_t)i, n, kColl, 0, p.k0, p.k1).w[0] < p.Tc;
}

// Kick, charge exchange (collide: the decision of collision_decision) and
// drift of one ion from x with velocity v and acceleration a; absorption (the
// earliest grain met along the drift segment, ties to the lower index) and
// exit tests.  Returns the new x, v in y, w; absorbed ions add to the grain's
// count and momentum.
template <typename T>
__device__ __forceinline__ void push_core(const T x[3], const T v[3], const T a[3], int i, uint64_t n,
                                          const PushArgs& p, const DustSet& ds, Ctl* __restrict__ ctl,
                                          bool collide, T y[3], T w[3], uint8_t& code, bool& coll, bool& lost)
{
#pragma clang fp contract(off)      // the same rounding in every kernel that inlines it
    const T dt = (T)p.dt;
    // kick and drift with one rounding each (fused multiply-add)
    T v0 = fma(dt, a[0], v[0]);
    T v1 = fma(dt, a[1], v[1]);
    T v2 = fma(dt, a[2], v[2]);
    if (collide) {      // see collision_decision; the new velocity from the block after it
        const U64x4 g = philox((uint64_t)i, n, kColl, 1, p.k0, p.k1);
        double g1, g2, g3, g4;
        gauss2(unit(g.w[0]), unit(g.w[1]), g1, g2);
        gauss2(unit(g.w[2]), unit(g.w[3]), g3, g4);
        v0 = (T)(p.sig * g1);
        v1 = (T)(p.sig * g2);
        v2 = (T)(p.sig * g3);
        coll = true;
    }
    const T y0 = fma(dt, v0, x[0]), y1 = fma(dt, v1, x[1]), y2 = fma(dt, v2, x[2]);
    // Absorption: does the drift segment x -> y meet a grain?  FP64 on
    // the stored values; the earliest entry wins, ties to the lower index.
    int hit = -1;
    double tbest = 2.0;
    const double D0 = (double)y0 - (double)x[0], D1 = (double)y1 - (double)x[1],
                 D2 = (double)y2 - (double)x[2];
    const double DD = D0 * D0 + D1 * D1 + D2 * D2;
    for (int d = 0; d < ds.nd; ++d) {
        const double s0 = (double)x[0] - ds.pos[d][0], s1 = (double)x[1] - ds.pos[d][1],
                     s2 = (double)x[2] - ds.pos[d][2];
        const double a2 = ds.rad2[d];
        const double ss = s0 * s0 + s1 * s1 + s2 * s2;
        const double sD = s0 * D0 + s1 * D1 + s2 * D2;
        // squared closest approach of the segment, without a division:
        // at the start if moving away, at the end if the foot of the
        // perpendicular lies beyond it, else ss - sD^2/DD (scaled by DD)
        bool in;
        if (DD == 0.0 || sD >= 0.0) {
            in = ss <= a2;
        } else if (-sD >= DD) {
            const double e0 = (double)y0 - ds.pos[d][0], e1 = (double)y1 - ds.pos[d][1],
                         e2 = (double)y2 - ds.pos[d][2];
            in = e0 * e0 + e1 * e1 + e2 * e2 <= a2;
        } else {
            in = ss * DD - sD * sD <= a2 * DD;
        }
        if (in) {   // rare: entry parameter of the first crossing
            double th = 0.0;
            if (DD > 0.0) {
                const double disc = fmax(sD * sD - DD * (ss - a2), 0.0);
                th = fmax((-sD - sqrt(disc)) / DD, 0.0);
            }
            if (th < tbest) {
                tbest = th;
                hit = d;
            }
        }
    }
    if (hit >= 0) {
        code = (uint8_t)(kEvAbsBase + hit);
        atomicAdd(&ctl->acc[hit][3], 1ull);
        atomicAdd(&ctl->acc[hit][4], to_fixed((double)v0, kMomScale, &ctl->status));
        atomicAdd(&ctl->acc[hit][5], to_fixed((double)v1, kMomScale, &ctl->status));
        atomicAdd(&ctl->acc[hit][6], to_fixed((double)v2, kMomScale, &ctl->status));
        lost = true;
    } else {
        const double rr = (double)y0 * (double)y0 + (double)y1 * (double)y1;
        if (rr > p.R * p.R || fabs((double)y2) > 0.5 * p.H) {
            code = kEvExit;
            lost = true;
        }
    }
    y[0] = y0; y[1] = y1; y[2] = y2;
    w[0] = v0; w[1] = v1; w[2] = v2;
}

// Acceleration of an ion from the symmetric pair sum's fixed-point totals
// fx (read by the caller), the homogeneous drive, the
// confinement field and the bare Coulomb pull of every grain (FP32 terms of
// FP64 differences, summed in FP64).  When `eq1` is set the ion's Eq. (1)
// summands (1 + rho) e^-rho / rho^3 (r_d - x_i), FP32 terms, are reduced over
// the wave in FP64 into red[wave][d][c] (zero for a padding slot).  All lanes
// of the wave must call it.  Floating-point contraction is off here (the only
// fused operations are the written fmaf), so that every kernel that inlines
// it rounds alike: a system in a batch reproduces the same system run alone.
__device__ __forceinline__ void accel_from_fixed(const float x[3], bool live, const unsigned long long fx[3],
                                                 const PairArgs& pa, const DustSet& ds,
                                                 const double* __restrict__ Q, float a[3],
                                                 double (*red)[kMaxDust][3])
{
#pragma clang fp contract(off)
    double g[3];
    for (int c = 0; c < 3; ++c) g[c] = live ? pa.Cd * from_fixed(fx[c], pa.sym_scale) : 0.0;
    g[2] += pa.Ez;
    if (pa.cf.on) {
        double ex, ey, ez;
        conf_field(pa.cf, x[0], x[1], x[2], ex, ey, ez);
        g[0] += ex; g[1] += ey; g[2] += ez;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const float kNegLog2e = -1.4426950408889634f;
    for (int d = 0; d < ds.nd; ++d) {
        const float rx = (float)((double)x[0] - ds.pos[d][0]);
        const float ry = (float)((double)x[1] - ds.pos[d][1]);
        const float rz = (float)((double)x[2] - ds.pos[d][2]);
        const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ir3 = ri * ri * ri;
        const float kq = (float)(pa.Kq * Q[d]) * ir3;                 // bare Coulomb on the ion
        g[0] += (double)(kq * rx); g[1] += (double)(kq * ry); g[2] += (double)(kq * rz);
        // Eq. (1) summand, the grain's side: -(1 + rho) e^-rho / rho^3 (x_i - r_d)
        const float rho = r2 * ri;
        const float e = __builtin_amdgcn_exp2f(rho * kNegLog2e);
        const float f = live ? -(fmaf(rho, e, e) * ir3) : 0.0f;
        const double fx = wave_sum((double)(f * rx)), fy = wave_sum((double)(f * ry)),
                     fz = wave_sum((double)(f * rz));
        if (lane == 0) {
            red[wv][d][0] = fx;
            red[wv][d][1] = fy;
            red[wv][d][2] = fz;
        }
    }
    a[0] = (float)g[0]; a[1] = (float)g[1]; a[2] = (float)g[2];
}

// Ions lost in a step (absorbed or exited), as (system, ion) pairs, for the
// reinjection kernel.  The list is cut into kSlots segments of `cap` entries;
// block b of the tail appends its lost ions to segment b mod kSlots
// (seg[slot * kPad32] counts them), so that blocks do not all add to one counter.
struct LostList {
    unsigned int* seg;       // [kSlots * kPad32] segment lengths, one cache line each
    unsigned int* ticket;    // reinjection blocks that have finished
    int2* item;              // [kSlots * cap]
    long long cap;
};

// Segment capacity for a tail grid of nblk blocks of 256 ions: the blocks of
// one slot hold at most this many ions, so no segment can overflow.
__host__ __device__ inline long long lost_cap(long long nblk)
{
    return (nblk + kSlots - 1) / kSlots * 256;
}

// Wave64 sum of an unsigned 64-bit integer (two's-complement wrap, so the
// fixed-point words add exactly).
__device__ inline unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Charge update (the three charging models of Section 2), the four force
// parts of Eqs. (1)-(4) in SI, recording of step n (the charge Q^n used in
// the step and the forces of the step), running sums over n >= n_discard,
// optional history, counters cleared, step counter advanced.  Run by one
// wave (lane d handles grain d; lane l also sums slot l of the per-slot
// counters), after every contribution to the counters is visible; no block
// barrier, so the block's other waves may have left.
__device__ void finalize_wave(const FinalArgs& f, const DustSet& ds, Ctl* __restrict__ ctl)
{
    const int lane = threadIdx.x & 63;
    const int d = lane;
    const long long n = ctl->step;
    // Every load is issued before its value is used, so that their latencies
    // (atomics live beyond the per-XCD caches) overlap instead of adding up.
    const double Qn = d < f.nd ? ctl->Q[d] : 0.0;
    const unsigned long long ex = __hip_atomic_load(&ctl->n_exit[lane][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long co = __hip_atomic_load(&ctl->n_coll[lane][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long acc[4] = {0ull, 0ull, 0ull, 0ull};
    if (d < f.nd)
        for (int c = 0; c < 4; ++c)
            acc[c] = __hip_atomic_load(&ctl->acc[d][3 + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Eq. (1) sums: slot `lane` of every grain's three words, summed over the
    // wave (integers, so the order does not matter), cleared for the next
    // step; two grains' words loaded at a time
    double S[3] = {0.0, 0.0, 0.0};
    for (int g0 = 0; g0 < f.nd; g0 += 2) {
        unsigned long long v[2][3];
#pragma unroll
        for (int gg = 0; gg < 2; ++gg)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                v[gg][c] = g0 + gg < f.nd ? __hip_atomic_load(&ctl->part[lane][g0 + gg][c], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT) : 0ull;
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            const int g = g0 + gg;
            if (g >= f.nd) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ctl->part[lane][g][c] = 0ull;
                const unsigned long long t = wave_sum_u64(v[gg][c]);
                if (g == d) S[c] = from_fixed(t, kForceScale);
            }
        }
    }
    // event counters: one slot per lane
    const double ne = wave_sum((double)ex);
    const double nc = wave_sum((double)co);
    ctl->n_exit[lane][0] = 0ull;
    ctl->n_coll[lane][0] = 0ull;
    ctl->ticket_slot[lane][0] = 0u;
    // the other grains' charges Q^n for Eq. (2)
    double px = 0.0, py = 0.0, pz = 0.0;
    for (int q = 0; q < f.nd; ++q) {
        const double Qq = __shfl(Qn, q, 64);
        if (q == d || d >= f.nd) continue;
        const double rx = ds.pos[d][0] - ds.pos[q][0], ry = ds.pos[d][1] - ds.pos[q][1],
                     rz = ds.pos[d][2] - ds.pos[q][2];
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double k = Qq / (r2 * sqrt(r2));
        px += k * rx; py += k * ry; pz += k * rz;
    }
    if (d < f.nd) {
        const double cntd = (double)(long long)acc[0];
        const double P0 = from_fixed(acc[1], kMomScale);
        const double P1 = from_fixed(acc[2], kMomScale);
        const double P2 = from_fixed(acc[3], kMomScale);
        for (int c = 0; c < 8; ++c) ctl->acc[d][c] = 0ull;

        // charge update
        const double psi = f.psi[d] * Qn;                     // e phi / kB Te
        const double Ie = -f.Ie0[d] * (psi < 0.0 ? exp(psi) : 1.0 + psi);
        double Qnew = Qn;
        if (f.mode == 2) {
            Qnew = Qn + f.w * cntd + Ie * f.dt;
        } else if (f.mode == 1) {
            const double chi = psi < 0.0 ? -psi * f.te_over_ti : 0.0;
            const double s = f.s_oml;
            const double br = s < 1e-6 ? 1.1283791670955125739 * (1.0 + chi)
                                       : exp(-s * s) * 0.5641895835477562869 +
                                             (s * s + 0.5 + chi) * erf(s) / s;
            Qnew = Qn + (f.Ii0[d] * br + Ie) * f.dt;
        }

        // forces, SI
        double F[12];
        const double co = f.c_orbit * Qn;
        F[0] = co * S[0] + Qn * f.eout[d][0];
        F[1] = co * S[1] + Qn * f.eout[d][1];
        F[2] = co * S[2] + Qn * f.eout[d][2];
        const double cd = f.c_dd * Qn;
        F[3] = cd * px; F[4] = cd * py; F[5] = cd * pz;
        F[6] = f.c_coll * P0; F[7] = f.c_coll * P1; F[8] = f.c_coll * P2;
        F[9] = 0.0; F[10] = 0.0; F[11] = f.c_ext * Qn;

        bool bad = !(Qnew == Qnew) || (Qnew - Qnew != 0.0);
        ctl->last[d][0] = Qn;
        for (int c = 0; c < 12; ++c) {
            ctl->last[d][1 + c] = F[c];
            bad = bad || (F[c] - F[c] != 0.0);
        }
        ctl->last[d][13] = cntd;
        if (n >= f.n_discard) {
            ctl->sums[d][0] += Qn;
            for (int c = 0; c < 12; ++c) ctl->sums[d][1 + c] += F[c];
        }
        if (f.hist && n >= f.hist_start && n < f.hist_start + f.hist_cap) {
            double* h = f.hist + ((n - f.hist_start) * f.nd + d) * kHistWords;
            h[0] = Qn;
            for (int c = 0; c < 12; ++c) h[1 + c] = F[c];
            h[13] = cntd;
        }
        ctl->Q[d] = Qnew;
        if (bad) atomicOr(&ctl->status, kStNaN);
    }
    if (lane == 0) {
        ctl->last_exit = (long long)ne;
        ctl->last_coll = (long long)nc;
        if (n >= f.n_discard) ctl->nrec += 1;
        ctl->ticket = 0u;
        ctl->step = n + 1;
    }
}

// The tail of one block of 256 ions of one system (planes X.. of the
// system, local ion index i = i0 + threadIdx.x): FIX selects the symmetric
// pair sum (acceleration assembled here from fix, written to AX..) over
// precomputed acceleration planes (AX.. plus nsplit - 1 partial planes
// sstride apart).  nblk: the system's number of tail blocks.  After the
// block's counters are added, the last block of the system to finish (a
// ticket counter in the control block) runs finalize_wave.
template <typename T, bool FIX, bool INL = false>
__device__ __forceinline__ void tail_block(T* __restrict__ X, T* __restrict__ Y, T* __restrict__ Z,
                                           T* __restrict__ VX, T* __restrict__ VY, T* __restrict__ VZ,
                                           T* __restrict__ AX, T* __restrict__ AY, T* __restrict__ AZ,
                                           long long sstride, int nsplit, unsigned long long* __restrict__ fix,
                                           long long fstride, uint8_t* __restrict__ ev, int i0, int nblk,
                                           const PairArgs& pa, const PushArgs& pu, const DustSet& ds,
                                           const FinalArgs& fa, Ctl* __restrict__ ctl, int sys,
                                           LostList lost_list)
{
    __shared__ double red[4][kMaxDust][3];
    __shared__ unsigned int wtally[3][4];
    __shared__ unsigned int lbase;
    const int i = i0 + threadIdx.x;
    const bool live = i < pu.N;
    const uint64_t n = (uint64_t)ctl->step;
    T x[3], v[3], a[3];
    unsigned long long fx[3];
    x[0] = X[i]; x[1] = Y[i]; x[2] = Z[i];
    v[0] = VX[i]; v[1] = VY[i]; v[2] = VZ[i];   // padding slots hold zeros
    if (FIX)
        for (int c = 0; c < 3; ++c) fx[c] = fix[c * fstride + i];
    // the collision decision needs none of the loaded values: its Philox
    // block runs while the loads are in flight
    const bool collide = live && collision_decision(i, n, pu);
    if (FIX) {
        for (int c = 0; c < 3; ++c) fix[c * fstride + i] = 0ull;   // cleared for the next step
        float xf[3] = {(float)x[0], (float)x[1], (float)x[2]}, af[3];
        accel_from_fixed(xf, live, fx, pa, ds, ctl->Q, af, red);
        a[0] = af[0]; a[1] = af[1]; a[2] = af[2];
        if (live) {
            AX[i] = a[0]; AY[i] = a[1]; AZ[i] = a[2];
        }
    } else {
        a[0] = AX[i]; a[1] = AY[i]; a[2] = AZ[i];
        for (int k = 1; k < nsplit; ++k) {
            a[0] += AX[i + k * sstride];
            a[1] += AY[i + k * sstride];
            a[2] += AZ[i + k * sstride];
        }
    }
    bool coll = false, lost = false;
    uint8_t code = kEvNone;
    if (live) {
        T y[3], w[3];
        push_core<T>(x, v, a, i, n, pu, ds, ctl, collide, y, w, code, coll, lost);
        if (INL && lost) {          // new boundary ion (Appendix B), here
            double o[6];
            reinject(pu, (uint64_t)i, n, o);
            for (int c = 0; c < 3; ++c) {
                y[c] = (T)o[c];
                w[c] = (T)o[3 + c];
            }
        }
        // else a lost ion is overwritten by the reinjection kernel
        X[i] = y[0]; Y[i] = y[1]; Z[i] = y[2];
        VX[i] = w[0]; VY[i] = w[1]; VZ[i] = w[2];
        ev[i] = code | (coll ? kEvCollBit : 0);
    }
    // Block totals: exits, collisions and lost ions per wave, then one
    // atomic per counter and block, on the block's slot.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long mex = __ballot(code == kEvExit), mcl = __ballot(coll), mls = __ballot(lost);
    if (lane == 0) {
        wtally[0][wv] = (unsigned int)__popcll(mex);
        wtally[1][wv] = (unsigned int)__popcll(mcl);
        wtally[2][wv] = (unsigned int)__popcll(mls);
    }
    __syncthreads();
    const int lblk = i0 / 256;                   // the block's index within its system
    const int slot = lblk % kSlots;
    if (threadIdx.x == 0) {
        const unsigned int ne = wtally[0][0] + wtally[0][1] + wtally[0][2] + wtally[0][3];
        const unsigned int nc = wtally[1][0] + wtally[1][1] + wtally[1][2] + wtally[1][3];
        const unsigned int nl = wtally[2][0] + wtally[2][1] + wtally[2][2] + wtally[2][3];
        if (ne) atomicAdd(&ctl->n_exit[slot][0], (unsigned long long)ne);
        if (nc) atomicAdd(&ctl->n_coll[slot][0], (unsigned long long)nc);
        lbase = (nl && !INL) ? atomicAdd(&lost_list.seg[(blockIdx.x % kSlots) * kPad32], nl) : 0u;
    }
    if (FIX && ds.nd > 0) {
        for (int t = threadIdx.x; t < ds.nd * 3; t += blockDim.x) {
            const int d = t / 3, c = t % 3;
            const double sum = ((red[0][d][c] + red[1][d][c]) + red[2][d][c]) + red[3][d][c];
            atomicAdd(&ctl->part[slot][d][c], to_fixed(sum, kForceScale, &ctl->status));
        }
    }
    __syncthreads();
    if (lost && !INL) {
        unsigned int r = lbase + (unsigned int)__popcll(mls & ((1ull << lane) - 1ull));
        for (int k = 0; k < wv; ++k) r += wtally[2][k];
        lost_list.item[(long long)(blockIdx.x % kSlots) * lost_list.cap + r] = make_int2(sys, i);
    }
    // The last block of the system to get here finalizes the step.  Every
    // contribution to the counters is a device-scope atomic, performed where
    // all blocks see it; each wave waits until its own have completed before
    // the block takes its ticket (also an atomic).  With more blocks than
    // slots, tickets are counted per slot and the block that completes a slot
    // adds to the system's ticket, so that no counter takes one atomic per
    // block.  When the system's ticket is complete every contribution is in
    // place; only that block then fences (one cache invalidation per step, not
    // one per wave).
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (wv != 0) return;            // the ticket and the finalize need one wave
    int is_last = 0;
    if (lane == 0) {
        if (nblk <= kSlots) {
            is_last = atomicAdd(&ctl->ticket, 1u) == (unsigned int)(nblk - 1);
        } else {
            const int per_slot = nblk / kSlots + (slot < nblk % kSlots ? 1 : 0);
            if (atomicAdd(&ctl->ticket_slot[slot][0], 1u) == (unsigned int)(per_slot - 1))
                is_last = atomicAdd(&ctl->ticket, 1u) == (unsigned int)(kSlots - 1);
        }
    }
    if (__shfl(is_last, 0, 64)) {
        __threadfence();
        finalize_wave(fa, ds, ctl);
    }
}

// The tail of one system: block b handles ions [256 b, 256 b + 256); lost
// ions are listed for reinject_kernel.  Seven waves per SIMD: the per-ion
// path fits them without spilling (only the single finalizing wave of the
// last block may spill a register).
template <typename T, bool FIX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8)))
void step_tail_kernel(T* __restrict__ xs, T* __restrict__ vs, T* __restrict__ as,
                      unsigned long long* __restrict__ fix, uint8_t* __restrict__ ev, int nsplit, PairArgs pa,
                      PushArgs pu, DustSet ds, FinalArgs fa, Ctl* __restrict__ ctl, LostList lost_list)
{
    const long long P = pu.Npad;
    tail_block<T, FIX, false>(xs, xs + P, xs + 2 * P, vs, vs + P, vs + 2 * P, as, as + P, as + 2 * P, 3 * P,
                              nsplit, fix, P, ev, blockIdx.x * 256, gridDim.x, pa, pu, ds, fa, ctl, 0, lost_list);
}

// The same tail for small systems: lost ions are reinjected by the thread
// that lost them, where a step is a chain of short kernels and a separate
// reinjection launch would lengthen it (the FP64 sampling then sets the
// kernel's register budget).
template <typename T, bool FIX>
__global__ __launch_bounds__(256) void step_tail_inl_kernel(T* __restrict__ xs, T* __restrict__ vs,
                                                            T* __restrict__ as, unsigned long long* __restrict__ fix,
                                                            uint8_t* __restrict__ ev, int nsplit, PairArgs pa,
                                                            PushArgs pu, DustSet ds, FinalArgs fa,
                                                            Ctl* __restrict__ ctl, LostList lost_list)
{
    const long long P = pu.Npad;
    tail_block<T, FIX, true>(xs, xs + P, xs + 2 * P, vs, vs + P, vs + 2 * P, as, as + P, as + 2 * P, 3 * P,
                             nsplit, fix, P, ev, blockIdx.x * 256, gridDim.x, pa, pu, ds, fa, ctl, 0, lost_list);
}

// Reinjection (Appendix B) of the ions the step's tail listed: a grid-stride
// walk of the list; the new position and velocity of ion i of system s come
// from the blocks (i, n, REINJ, 0/1) of that system's stream, n the step
// just finalized.  The last block to finish empties the list for the next
// step.  sysp(s) gives the system's planes and constants.
template <typename T, typename Sys>
__device__ __forceinline__ void reinject_list(LostList L, const Sys& sysp)
{
    static_assert(kSlots == 64, "one segment per lane");
    __shared__ unsigned int pre[kSlots + 1];
    __shared__ int last;
    if (threadIdx.x < kSlots) {        // segment offsets of the listed ions: a wave scan
        const unsigned int len = L.seg[threadIdx.x * kPad32];
        unsigned int inc = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned int u = __shfl_up(inc, o, 64);
            if ((int)threadIdx.x >= o) inc += u;
        }
        pre[threadIdx.x] = inc - len;
        if (threadIdx.x == kSlots - 1) pre[kSlots] = inc;
    }
    __syncthreads();
    const unsigned int cnt = pre[kSlots];
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
        int lo = 0, hi = kSlots;       // the segment holding entry k: pre[lo] <= k < pre[lo + 1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= k) lo = mid; else hi = mid;
        }
        const int2 e = L.item[(long long)lo * L.cap + (k - pre[lo])];
        T *X, *V;
        const PushArgs* pu;
        const Ctl* ctl;
        long long P;
        sysp(e.x, X, V, pu, ctl, P);
        double o[6];
        reinject(*pu, (uint64_t)e.y, (uint64_t)(ctl->step - 1), o);
        X[e.y] = (T)o[0]; X[P + e.y] = (T)o[1]; X[2 * P + e.y] = (T)o[2];
        V[e.y] = (T)o[3]; V[P + e.y] = (T)o[4]; V[2 * P + e.y] = (T)o[5];
    }
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(L.ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (last && threadIdx.x < kSlots) {     // every block has read the lengths
        L.seg[threadIdx.x * kPad32] = 0u;
        if (threadIdx.x == 0) *L.ticket = 0u;
    }
}

template <typename T>
struct OneSystem {
    T* xs;
    T* vs;
    const PushArgs* pu;
    const Ctl* ctl;
    long long P;
    __device__ void operator()(int, T*& X, T*& V, const PushArgs*& p, const Ctl*& c, long long& Pp) const
    {
        X = xs; V = vs; p = pu; c = ctl; Pp = P;
    }
};

template <typename T>
__global__ __launch_bounds__(64) void reinject_kernel(T* __restrict__ xs, T* __restrict__ vs, PushArgs pu,
                                                     const Ctl* __restrict__ ctl, LostList lost_list)
{
    reinject_list<T>(lost_list, OneSystem<T>{xs, vs, &pu, ctl, pu.Npad});
}
// ---------------------------------------------------------------------------
// Initial state of ion i: uniform in the cylinder outside every grain,
// velocity from N((0,0,u), sig^2).  Padding slots get a far-away sentinel
// position that contributes exactly zero to every pair sum.
template <typename T>
__device__ __forceinline__ void init_ion(T* __restrict__ X, T* __restrict__ Y, T* __restrict__ Z,
                                         T* __restrict__ VX, T* __restrict__ VY,
                                         T* __restrict__ VZ, int i, const PushArgs& p,
                                         const DustSet& ds, Ctl* __restrict__ ctl)
{
    if (i >= p.N) {
        const T far = (T)1.0e18;
        X[i] = far; Y[i] = far; Z[i] = far;
        VX[i] = 0; VY[i] = 0; VZ[i] = 0;
        return;
    }
    double px = 0.0, py = 0.0, pz = 0.0;
    bool ok = false;
    for (uint64_t k = 0; k < 1000 && !ok; ++k) {
        const U64x4 r = philox((uint64_t)i, 0, kInitPos, k, p.k0, p.k1);
        const double rr = p.R * sqrt(unit(r.w[0]));
        double sn, cs;
        sincos(2.0 * kPi * unit(r.w[1]), &sn, &cs);
        px = rr * cs;
        py = rr * sn;
        pz = p.H * (unit(r.w[2]) - 0.5);
        ok = true;
        for (int d = 0; d < ds.nd; ++d) {
            const double a0 = px - ds.pos[d][0], a1 = py - ds.pos[d][1], a2 = pz - ds.pos[d][2];
            if (a0 * a0 + a1 * a1 + a2 * a2 <= ds.rad2[d]) ok = false;
        }
    }
    if (!ok) atomicOr(&ctl->status, kStPlace);
    const U64x4 g = philox((uint64_t)i, 0, kInitVel, 0, p.k0, p.k1);
    double g1, g2, g3, g4;
    gauss2(unit(g.w[0]), unit(g.w[1]), g1, g2);
    gauss2(unit(g.w[2]), unit(g.w[3]), g3, g4);
    double vz = p.ubar + p.sig * g3;
    if (p.flags & kFlagFieldDriven) {
        // time since the last collision from block (i, 0, INIT_VEL, 1)
        const U64x4 t = philox((uint64_t)i, 0, kInitVel, 1, p.k0, p.k1);
        vz = p.sig * g3 - p.ufd * log(unit(t.w[0]));
    }
    X[i] = (T)px; Y[i] = (T)py; Z[i] = (T)pz;
    VX[i] = (T)(p.sig * g1); VY[i] = (T)(p.sig * g2); VZ[i] = (T)vz;
}

template <typename T>
__global__ __launch_bounds__(256) void init_kernel(T* __restrict__ xs, T* __restrict__ vs,
                                                   T* __restrict__ as, PushArgs p, DustSet ds,
                                                   Ctl* __restrict__ ctl)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int Npad = p.Npad;
    if (i >= Npad) return;
    init_ion<T>(xs, xs + Npad, xs + 2 * Npad, vs, vs + Npad, vs + 2 * Npad, i, p, ds, ctl);
    as[i] = 0; as[Npad + i] = 0; as[2 * Npad + i] = 0;
}

// Confinement potential (Appendix A, Eqs. (A.1)-(A.2)), dimensionless:
// out[(nz + 1) k + p] = 1 - C sum_l exp(-d_l) / d_l at the node
// (k R / nx, 0, p (H/2) / nz), the sum over the N ions of one system at
// X, Y, Z; 1 is the screened potential of the infinite background and C the
// ion-ion coupling.  One block per node; an ion exactly on a node is left
// out.  Grid: (nx + 1) (nz + 1) blocks of 256.
template <typename T>
__global__ __launch_bounds__(256) void conf_grid_kernel(const T* __restrict__ X,
                                                        const T* __restrict__ Y,
                                                        const T* __restrict__ Z, int N, double C,
                                                        double R, double Hh, int nx, int nz,
                                                        double* __restrict__ out)
{
    __shared__ double part[4];
    const int g = blockIdx.x;
    const double gx = R * (double)(g / (nz + 1)) / (double)nx;
    const double gz = Hh * (double)(g % (nz + 1)) / (double)nz;
    double s = 0.0;
    for (int l = threadIdx.x; l < N; l += 256) {
        const double dx = (double)X[l] - gx, dy = (double)Y[l], dz = (double)Z[l] - gz;
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        s += d > 0.0 ? exp(-d) / d : 0.0;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[g] = 1.0 - C * (((part[0] + part[1]) + part[2]) + part[3]);
}

__global__ void rng_kernel(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2,
                           uint64_t c3, uint64_t* out)
{
    if (threadIdx.x == 0) {
        const U64x4 r = philox(c0, c1, c2, c3, k0, k1);
        for (int k = 0; k < 4; ++k) out[k] = r.w[k];
    }
}

}  // namespace odk
