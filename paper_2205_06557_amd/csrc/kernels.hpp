// kernels.hpp -- the HIP kernels of one time step.
//
//   pair_forces_f32 / pair_forces_f64   forces on every ion (Section 2):
//       screened (Yukawa) ion-ion sum over all other ions, bare Coulomb pull
//       of each grain, homogeneous drive; plus the per-grain sum of Eq. (1)
//       over all ions, reduced per block and added to int64 fixed-point
//       accumulators.
//   push_kernel<T>      kick, charge exchange, drift, absorption test against
//       every grain along the drift segment, exit test, per-ion event byte;
//       lost ions are appended to a list.
//   reinject_kernel<T>  new boundary position and velocity for every listed
//       ion (Appendix B).
//   finalize_kernel     one wave: charge update (the three charging models of
//       Section 2), the four force parts of Eqs. (1)-(4) in SI, recording,
//       time averages, clearing of the accumulators, step counter.
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
};

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
            atomicAdd(&ctl->acc[d][c], to_fixed(s, kForceScale, &ctl->status));
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
        atomicAdd(&ctl->acc[d][c], to_fixed(s, kForceScale, &ctl->status));
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
// step leaves it; stops when a step is below 1e-13 s.
__device__ double flux_speed(double uu, double m, double s)
{
    const double goal = uu * inflow(m, s);
    double lo = 0.0;
    double hi = fmax(m, 0.0) + 40.0 * s;
    double v = fmax(m, 0.0) + s;
    for (int it = 0; it < 400; ++it) {
        const double t = (v - m) / s;
        const double tail = m * 0.5 * erfc(t * 0.70710678118654752440) + s * npdf(t);
        const double g = tail - goal;
        if (g > 0.0) lo = v; else hi = v;
        const double slope = -v * npdf(t) / s;
        double nv = 0.5 * (lo + hi);
        if (slope < 0.0) {
            // a converged step lands on the bracket end it just moved: keep it
            const double cand = v - g / slope;
            if (cand >= lo && cand <= hi) nv = cand;
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
    auto tail = [&](double v, double& slope) {
        if (top) {
            const double A = fd_A(-v, ufd, sig);
            slope = -v * A / ufd;
            return (ufd - v) * A + sig * npdf(v / sig) - ufd * 0.5 * erfc(v / sig * k);
        }
        const double A = fd_A(v, ufd, sig);
        slope = -v * A / ufd;
        return (v + ufd) * A + sig * npdf(v / sig) + ufd * 0.5 * erfc(v / sig * k);
    };
    double slope;
    const double goal = uu * tail(0.0, slope);
    double lo = 0.0, hi = 40.0 * sig + (top ? 0.0 : 50.0 * ufd);
    double v = top ? sig : ufd + sig;
    for (int it = 0; it < 400; ++it) {
        const double g = tail(v, slope) - goal;
        if (g > 0.0) lo = v; else hi = v;
        double nv = 0.5 * (lo + hi);
        if (slope < 0.0) {
            const double cand = v - g / slope;
            if (cand >= lo && cand <= hi) nv = cand;
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
// Push of one ion: kick with the acceleration (the sum of `nsplit` partial
// planes `sstride` apart), charge exchange, drift, absorption test against
// every grain along the drift segment, exit test.  Planes use the system's
// local ion index.  Absorbed ions add to the grain's count and momentum.
template <typename T>
__device__ __forceinline__ void push_ion(T* __restrict__ X, T* __restrict__ Y, T* __restrict__ Z,
                                         T* __restrict__ VX, T* __restrict__ VY,
                                         T* __restrict__ VZ, const T* __restrict__ AX,
                                         const T* __restrict__ AY, const T* __restrict__ AZ,
                                         long long sstride, int nsplit, int i, uint64_t n,
                                         const PushArgs& p, const DustSet& ds,
                                         Ctl* __restrict__ ctl, uint8_t& code, bool& coll,
                                         bool& lost)
{
    const T dt = (T)p.dt;
    T ax = AX[i], ay = AY[i], az = AZ[i];
    for (int k = 1; k < nsplit; ++k) {
        ax += AX[i + k * sstride];
        ay += AY[i + k * sstride];
        az += AZ[i + k * sstride];
    }
    const T x0 = X[i], x1 = Y[i], x2 = Z[i];
    T v0 = VX[i] + dt * ax;
    T v1 = VY[i] + dt * ay;
    T v2 = VZ[i] + dt * az;
    if (p.Tc != 0) {
        const U64x4 r = philox((uint64_t)i, n, kColl, 0, p.k0, p.k1);
        if (r.w[0] < p.Tc) {
            const U64x4 g = philox((uint64_t)i, n, kColl, 1, p.k0, p.k1);
            double g1, g2, g3, g4;
            gauss2(unit(g.w[0]), unit(g.w[1]), g1, g2);
            gauss2(unit(g.w[2]), unit(g.w[3]), g3, g4);
            v0 = (T)(p.sig * g1);
            v1 = (T)(p.sig * g2);
            v2 = (T)(p.sig * g3);
            coll = true;
        }
    }
    const T y0 = x0 + dt * v0, y1 = x1 + dt * v1, y2 = x2 + dt * v2;
    // Absorption: does the drift segment x -> y meet a grain?  FP64 on
    // the stored values; the earliest entry wins, ties to the lower index.
    int hit = -1;
    double tbest = 2.0;
    const double D0 = (double)y0 - (double)x0, D1 = (double)y1 - (double)x1,
                 D2 = (double)y2 - (double)x2;
    const double DD = D0 * D0 + D1 * D1 + D2 * D2;
    for (int d = 0; d < ds.nd; ++d) {
        const double s0 = (double)x0 - ds.pos[d][0], s1 = (double)x1 - ds.pos[d][1],
                     s2 = (double)x2 - ds.pos[d][2];
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
    // lost ions are overwritten by the reinjection kernel
    X[i] = y0; Y[i] = y1; Z[i] = y2;
    VX[i] = v0; VY[i] = v1; VZ[i] = v2;
}

// Capacity of one lost-list segment for a push grid of nblk blocks of 256
// ions: the blocks of a slot hold at most this many ions, so no segment can
// overflow.
__host__ __device__ inline long long seg_cap(int nblk)
{
    return (long long)((nblk + kSlots - 1) / kSlots) * 256;
}

// Wave totals of exits and collisions into the system's counters (slot of
// this block), and a place in the slot's segment of the lost list (segment
// lengths in seg_len[kSlots], capacity cap) for every lane with `lost` set.
// All lanes of the wave must call it.  Returns the lane's list index (valid
// if `lost`).
__device__ __forceinline__ long long wave_tally(Ctl* __restrict__ ctl, uint8_t code, bool coll,
                                                bool lost, unsigned long long* seg_len, long long cap)
{
    const int slot = blockIdx.x % kSlots;
    const unsigned long long ex = __ballot(code == kEvExit);
    const unsigned long long cl = __ballot(coll);
    const unsigned long long ls = __ballot(lost);
    const int lane = threadIdx.x & 63;
    unsigned long long base = 0;
    if (lane == 0) {
        if (ex) atomicAdd(&ctl->n_exit[slot], (unsigned long long)__popcll(ex));
        if (cl) atomicAdd(&ctl->n_coll[slot], (unsigned long long)__popcll(cl));
        if (ls) base = atomicAdd(&seg_len[slot], (unsigned long long)__popcll(ls));
    }
    base = __shfl(base, 0, 64);
    return slot * cap + (long long)base + __popcll(ls & ((1ull << lane) - 1ull));
}

// Push of one system: one ion per thread.
template <typename T>
__global__ __launch_bounds__(256) void push_kernel(T* __restrict__ xs, T* __restrict__ vs,
                                                   const T* __restrict__ as,
                                                   uint8_t* __restrict__ ev,
                                                   int* __restrict__ lost_list, PushArgs p,
                                                   DustSet ds, Ctl* __restrict__ ctl, int nsplit)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int Npad = p.Npad;
    const uint64_t n = (uint64_t)ctl->step;
    bool coll = false, lost = false;
    uint8_t code = kEvNone;
    if (i < p.N) {
        push_ion<T>(xs, xs + Npad, xs + 2 * Npad, vs, vs + Npad, vs + 2 * Npad, as, as + Npad,
                    as + 2 * Npad, 3LL * Npad, nsplit, i, n, p, ds, ctl, code, coll, lost);
        ev[i] = code | (coll ? kEvCollBit : 0);
    }
    const long long at = wave_tally(ctl, code, coll, lost, ctl->n_lost, seg_cap(gridDim.x));
    if (lost) lost_list[at] = i;
}

// New boundary position and velocity of listed ion i (Appendix B).
template <typename T>
__device__ __forceinline__ void reinject_ion(T* __restrict__ X, T* __restrict__ Y,
                                             T* __restrict__ Z, T* __restrict__ VX,
                                             T* __restrict__ VY, T* __restrict__ VZ, int i,
                                             uint64_t n, const PushArgs& p)
{
    double o[6];
    reinject(p, (uint64_t)i, n, o);
    X[i] = (T)o[0]; Y[i] = (T)o[1]; Z[i] = (T)o[2];
    VX[i] = (T)o[3]; VY[i] = (T)o[4]; VZ[i] = (T)o[5];
}

// Reinjection of the ions the push listed.  Block b walks segment
// b mod kSlots of the list (length left by the push in n_lost); the grid is
// a multiple of kSlots.  cap: segment capacity of the push grid.
template <typename T>
__global__ __launch_bounds__(64) void reinject_kernel(T* __restrict__ xs, T* __restrict__ vs,
                                                     const int* __restrict__ lost_list, PushArgs p,
                                                     long long cap, Ctl* __restrict__ ctl)
{
    const int slot = blockIdx.x % kSlots, part = blockIdx.x / kSlots, parts = gridDim.x / kSlots;
    const long long cnt = (long long)ctl->n_lost[slot];
    const uint64_t n = (uint64_t)ctl->step;
    const int Npad = p.Npad;
    const int* seg = lost_list + slot * cap;
    for (long long k = part * 64 + threadIdx.x; k < cnt; k += (long long)parts * 64)
        reinject_ion<T>(xs, xs + Npad, xs + 2 * Npad, vs, vs + Npad, vs + 2 * Npad, seg[k], n, p);
}

// ---------------------------------------------------------------------------
// Finalize of one system by one wave (lane d handles grain d): charge update,
// the four force parts in SI, recording, running sums, counters cleared,
// step counter advanced.
__device__ __forceinline__ void finalize_sys(const FinalArgs& f, const DustSet& ds,
                                             Ctl* __restrict__ ctl, double* Qs)
{
    const int d = threadIdx.x;
    if (d < f.nd) Qs[d] = ctl->Q[d];
    __syncthreads();
    const long long n = ctl->step;
    if (d < f.nd) {
        const double Qn = Qs[d];
        const double S0 = from_fixed(ctl->acc[d][0], kForceScale);
        const double S1 = from_fixed(ctl->acc[d][1], kForceScale);
        const double S2 = from_fixed(ctl->acc[d][2], kForceScale);
        const double cntd = (double)(long long)ctl->acc[d][3];
        const double P0 = from_fixed(ctl->acc[d][4], kMomScale);
        const double P1 = from_fixed(ctl->acc[d][5], kMomScale);
        const double P2 = from_fixed(ctl->acc[d][6], kMomScale);
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
        F[0] = co * S0 + Qn * f.eout[d][0];
        F[1] = co * S1 + Qn * f.eout[d][1];
        F[2] = co * S2 + Qn * f.eout[d][2];
        double px = 0.0, py = 0.0, pz = 0.0;
        for (int q = 0; q < f.nd; ++q) {
            if (q == d) continue;
            const double rx = ds.pos[d][0] - ds.pos[q][0], ry = ds.pos[d][1] - ds.pos[q][1],
                         rz = ds.pos[d][2] - ds.pos[q][2];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double k = Qs[q] / (r2 * sqrt(r2));
            px += k * rx; py += k * ry; pz += k * rz;
        }
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
        ctl->Q[d] = Qnew;
        if (bad) atomicOr(&ctl->status, kStNaN);
    }
    __syncthreads();
    // event counters: one slot per lane (blockDim.x == kSlots == 64)
    const double ne = wave_sum((double)ctl->n_exit[d]);
    const double nc = wave_sum((double)ctl->n_coll[d]);
    ctl->n_exit[d] = 0ull;
    ctl->n_coll[d] = 0ull;
    ctl->n_lost[d] = 0ull;
    if (d == 0) {
        ctl->last_exit = (long long)ne;
        ctl->last_coll = (long long)nc;
        if (n >= f.n_discard) ctl->nrec += 1;
        ctl->step = n + 1;
    }
}

__global__ __launch_bounds__(64) void finalize_kernel(FinalArgs f, DustSet ds,
                                                      Ctl* __restrict__ ctl)
{
    __shared__ double Qs[kMaxDust];
    finalize_sys(f, ds, ctl, Qs);
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
