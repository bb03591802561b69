// odust.hip -- host runtime and C-ABI of libodust (declarations and the
// meaning of every argument: include/odust.h).
//
// One od_system owns, on one HIP stream:
//   x, v      [3][Npad] structure-of-arrays state, float (FP32 mode) or double
//             (FP64 mode); Npad = N rounded up to the pair tile, padding slots
//             parked at a far-away sentinel;
//   a         [nsplit][3][Npad] partial accelerations of the source splits;
//   ev        [Npad] per-ion event byte of the last step;
//   lost      [Npad] (system, ion) pairs of the ions the step lost;
//   ctl       small control block (charges, int64 fixed-point accumulators,
//             last-step record, running sums, step counter, status word).
// All per-step state stays on the device; a step is three launches (pair sum;
// the per-ion tail, whose last block finalizes the step; reinjection of the
// ions the tail listed; a cutoff adds the slab sort and its epilogue) and
// needs no host synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/odust.h"
#include "kernels.hpp"
#include "cutoff.hpp"
#include "pairsym.hpp"
#include "worksplit.hpp"

namespace {

constexpr double kQE = 1.602176634e-19;
constexpr double kKB = 1.380649e-23;
constexpr double kEPS0 = 8.8541878128e-12;
constexpr double kME = 9.1093837015e-31;
constexpr double kPI = 3.14159265358979323846;

constexpr int kPairBlock = 256;
constexpr int kPairTile = 256;
constexpr int kPad = 256;
constexpr int kMaxSplitSingle = 4;             // source splits of one system's pair sum
constexpr int kConfNr = 32, kConfNz = 32;      // intervals of the confinement grid along r, z
constexpr int kConfNodes = (kConfNr + 1) * (kConfNz + 1);

thread_local std::string g_err;

od_status fail(od_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(OD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

uint64_t prob_to_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    const double t = p * 18446744073709551616.0;
    if (t >= 18446744073709551615.0) return ~0ull;
    return (uint64_t)t;
}

double normal_cdf(double t) { return 0.5 * std::erfc(-t / std::sqrt(2.0)); }
double normal_pdf(double t) { return std::exp(-0.5 * t * t) / std::sqrt(2.0 * kPI); }

struct SysConsts {
    double lam = 0, wpi = 0, cs = 0;
    odk::DustSet ds{};
    odk::PairArgs pa{};
    odk::PushArgs pu{};
    odk::FinalArgs fa{};
};

}  // namespace

struct od_system {
    hipStream_t stream = nullptr;
    // steps captured as one HIP graph (od_set_graph); re-captured on demand
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_steps = 0;
    od_allocator alloc{};
    bool custom_alloc = false;
    od_plasma pl{};
    od_sim sim{};
    int nd = 0;
    od_dust dust[OD_MAX_DUST]{};
    int prec = 0;
    int64_t N = 0, Npad = 0;
    size_t esz = 4;
    int nsplit = 1;
    // units
    double lam = 0, wpi = 0, cs = 0;
    odk::DustSet ds{};
    odk::PairArgs pa{};
    odk::PushArgs pu{};
    odk::FinalArgs fa{};
    std::vector<double> conf_grid;      // dimensionless confinement potentials
    // ion-ion cutoff (FP32): slab sort buffers
    bool cut = false;
    odk::CutArgs ca{};
    float* xs_sorted = nullptr;         // [3][Npad] positions in slab order
    int* idx_sorted = nullptr;          // [Npad] ion of each sorted slot
    int* slab = nullptr;                // [Npad] slab of each ion
    int* table = nullptr;               // [nslab][nblk] per-block counts, then offsets
    int* slab_total = nullptr;          // [nslab]
    int* slab_start = nullptr;          // [nslab + 1]
    unsigned long long* cut_fix = nullptr;  // [3][Npad] fixed-point sums by sorted slot
    // all-pairs sum with each pair evaluated once
    int pair_kind = OD_PAIR_AUTO;
    bool sym = false;
    unsigned long long* acc_fix = nullptr;  // [3][Npad] int64 fixed-point pair sums
    odk::SymItem* sym_items = nullptr;
    int n_sym_items = 0;
    // device memory
    void* x = nullptr;
    void* v = nullptr;
    void* a = nullptr;
    uint8_t* ev = nullptr;
    int2* lost = nullptr;                // ions lost in the step, for the reinjection kernel
    odk::Ctl* ctl = nullptr;
    double* hist = nullptr;              // per-step records (od_set_history), or null
    // timing
    bool timing = false;
    std::vector<hipEvent_t> evpool;
    std::vector<std::pair<int, int>> marks[4];   // (start idx, stop idx) per class
    size_t evnext = 0;
};

namespace {

void* dev_alloc(od_system* s, size_t bytes)
{
    if (s->custom_alloc) return s->alloc.alloc(s->alloc.ctx, bytes);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(od_system* s, void* p)
{
    if (!p) return;
    if (s->custom_alloc)
        s->alloc.release(s->alloc.ctx, p);
    else
        (void)hipFree(p);
}

void free_cutoff(od_system* s)
{
    dev_free(s, s->xs_sorted);
    dev_free(s, s->idx_sorted);
    dev_free(s, s->slab);
    dev_free(s, s->table);
    dev_free(s, s->slab_total);
    dev_free(s, s->slab_start);
    dev_free(s, s->cut_fix);
    s->cut_fix = nullptr;
    s->xs_sorted = nullptr;
    s->idx_sorted = s->slab = s->table = s->slab_total = s->slab_start = nullptr;
    s->cut = false;
}

void free_sym(od_system* s)
{
    dev_free(s, s->acc_fix);
    dev_free(s, s->sym_items);
    s->acc_fix = nullptr;
    s->sym_items = nullptr;
    s->n_sym_items = 0;
    s->sym = false;
}

// Sets up the symmetric pair sum: its fixed-point totals and work items.  In
// test-particle mode there are no items (no pair kernel runs); the totals stay
// zero and the step's tail adds the grain, drive and confinement terms.
od_status setup_sym(od_system* s)
{
    if (s->sym) return OD_OK;
    const int T = (int)(s->Npad / kPairBlock);
    std::vector<odk::SymItem> items;
    if (s->pa.ion_ion) items = sym_items(T);
    s->acc_fix = (unsigned long long*)dev_alloc(s, 3 * (size_t)s->Npad * sizeof(unsigned long long));
    if (!items.empty()) s->sym_items = (odk::SymItem*)dev_alloc(s, items.size() * sizeof(odk::SymItem));
    if (!s->acc_fix || (!items.empty() && !s->sym_items)) {
        free_sym(s);
        return fail(OD_ENOMEM, "device allocation of the symmetric pair sum failed");
    }
    if (!items.empty())
        HIPCHK(hipMemcpyAsync(s->sym_items, items.data(), items.size() * sizeof(odk::SymItem),
                              hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemsetAsync(s->acc_fix, 0, 3 * (size_t)s->Npad * sizeof(unsigned long long), s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->n_sym_items = (int)items.size();
    s->sym = true;
    return OD_OK;
}

// Chooses the all-pairs kernel for the system's kind: the symmetric one
// unless one-sided is asked for (it is the faster at every size).
od_status apply_pair_kind(od_system* s)
{
    const bool able = s->prec == OD_PREC_FP32;
    const bool want = able && (s->pair_kind == OD_PAIR_SYMMETRIC || s->pair_kind == OD_PAIR_AUTO);
    if (want && !s->sym) {
        od_status st = setup_sym(s);
        if (st != OD_OK) return st;
    } else if (!want && s->sym) {
        free_sym(s);
    }
    return OD_OK;
}

od_status check_params(const od_plasma* pl, const od_sim* sim, const od_dust* dust, int nd)
{
    if (!pl || !sim) return fail(OD_EINVAL, "null plasma or sim");
    if (nd < 0 || nd > OD_MAX_DUST) return fail(OD_EINVAL, "n_dust %d out of [0,%d]", nd, OD_MAX_DUST);
    if (nd > 0 && !dust) return fail(OD_EINVAL, "null dust array");
    if (!(pl->T_e > 0) || !(pl->T_i > 0) || !(pl->n_inf > 0) || !(pl->m_i > 0))
        return fail(OD_EINVAL, "temperatures, density and ion mass must be positive");
    if (!(pl->mach >= 0) || !(pl->nu_in >= 0) || std::isinf(pl->E_ext))
        return fail(OD_EINVAL, "mach and nu_in must be >= 0 and E_ext finite or NaN");
    if (!(sim->R > 0) || !(sim->H > 0) || !(sim->dt > 0))
        return fail(OD_EINVAL, "R, H and dt must be positive");
    // 2^29 keeps every plane offset c * Npad + i (c < 3) of the kernels in int range
    if (sim->n_ions < 2 || sim->n_ions > (int64_t)1 << 29)
        return fail(OD_EINVAL, "n_ions %lld out of [2, 2^29]", (long long)sim->n_ions);
    if (sim->n_discard < 0) return fail(OD_EINVAL, "n_discard must be >= 0");
    if (sim->charge_mode < 0 || sim->charge_mode > 2) return fail(OD_EINVAL, "bad charge_mode");
    if (sim->precision != OD_PREC_FP32 && sim->precision != OD_PREC_FP64)
        return fail(OD_EINVAL, "bad precision");
    if (sim->flags & ~(OD_FLAG_LITERAL_SIDE | OD_FLAG_NO_ION_ION | OD_FLAG_CONFINEMENT | OD_FLAG_FIELD_DRIVEN))
        return fail(OD_EINVAL, "unknown flags");
    if (sim->flags & OD_FLAG_FIELD_DRIVEN) {
        // drift gained between collisions a / nu against the thermal speed
        const double cs = std::sqrt(kKB * pl->T_e / pl->m_i);
        const double E = std::isnan(pl->E_ext) ? pl->m_i * pl->nu_in * pl->mach * cs / kQE : pl->E_ext;
        const double ufd = pl->nu_in > 0 ? kQE * E / (pl->m_i * pl->nu_in) : 0.0;
        const double sig = std::sqrt(kKB * pl->T_i / pl->m_i);
        if (!(pl->nu_in > 0) || !(ufd > 0) || sig > 30.0 * ufd)
            return fail(OD_EINVAL, "field-driven flow needs nu_in > 0 and a drift a/nu above sigma/30");
    }
    if (sim->reserved != 0) return fail(OD_EINVAL, "reserved must be 0");
    for (int d = 0; d < nd; ++d) {
        const od_dust& g = dust[d];
        if (!(g.radius > 0) || !std::isfinite(g.q0) || !std::isfinite(g.x) || !std::isfinite(g.y) ||
            !std::isfinite(g.z))
            return fail(OD_EINVAL, "grain %d: bad radius, charge or position", d);
        const double rho = std::sqrt(g.x * g.x + g.y * g.y);
        if (rho + g.radius >= sim->R || std::fabs(g.z) + g.radius >= 0.5 * sim->H)
            return fail(OD_EINVAL, "grain %d crosses the domain boundary", d);
        for (int q = 0; q < d; ++q) {
            const double dx = g.x - dust[q].x, dy = g.y - dust[q].y, dz = g.z - dust[q].z;
            if (std::sqrt(dx * dx + dy * dy + dz * dz) <= g.radius + dust[q].radius)
                return fail(OD_EINVAL, "grains %d and %d overlap", q, d);
        }
    }
    return OD_OK;
}

// SI -> dimensionless constants of every kernel.
void derive_consts(const od_plasma& P, const od_sim& S, const od_dust* dust, int nd, int64_t N,
                   int64_t Npad, SysConsts& c)
{
    const double lam = std::sqrt(kEPS0 * kKB * P.T_e / (P.n_inf * kQE * kQE));
    const double wpi = std::sqrt(P.n_inf * kQE * kQE / (kEPS0 * P.m_i));
    const double cs = lam * wpi;
    c.lam = lam;
    c.wpi = wpi;
    c.cs = cs;
    const double sig = std::sqrt(P.T_i / P.T_e);
    const double ubar = P.mach;
    const double R = S.R / lam, H = S.H / lam, dt = S.dt * wpi, nu = P.nu_in / wpi;
    const double nl3 = P.n_inf * lam * lam * lam;          // ions per Debye cube
    const double Vt = kPI * R * R * H;
    const double w = nl3 * Vt / (double)S.n_ions;           // ions per superparticle
    double Ez, E_si;
    if (std::isnan(P.E_ext)) {
        Ez = nu > 0 ? nu * ubar : 0.0;
        E_si = P.nu_in > 0 ? P.m_i * P.nu_in * ubar * cs / kQE : 0.0;
    } else {
        E_si = P.E_ext;
        Ez = kQE * P.E_ext / (P.m_i * lam * wpi * wpi);
    }
    const double Pc = -std::expm1(-nu * dt);

    odk::DustSet& ds = c.ds;
    ds.nd = nd;
    for (int d = 0; d < nd; ++d) {
        ds.pos[d][0] = dust[d].x / lam;
        ds.pos[d][1] = dust[d].y / lam;
        ds.pos[d][2] = dust[d].z / lam;
        const double a = dust[d].radius / lam;
        ds.rad2[d] = a * a;
    }

    odk::PairArgs& pa = c.pa;
    pa.N = (int)N;
    pa.Npad = (int)Npad;
    pa.nd = nd;
    pa.ion_ion = (S.flags & OD_FLAG_NO_ION_ION) ? 0 : 1;
    pa.Cd = Vt / (4.0 * kPI * (double)S.n_ions);
    pa.C = (float)pa.Cd;
    pa.Kq = 1.0 / (4.0 * kPI * nl3);
    pa.Ez = Ez;
    {
        // fixed-point scale of the symmetric sums: 2^(27 - (2/3) log2 n), n ions per r_De^3
        const double n_ions = (double)S.n_ions / Vt;
        const double e = std::round(27.0 - (2.0 / 3.0) * std::log2(n_ions));
        pa.sym_scale = std::ldexp(1.0, (int)std::min(40.0, std::max(10.0, e)));
    }

    // face inflows per unit density (Appendix B), dimensionless
    auto face = [&](double m) { return m * normal_cdf(m / sig) + sig * normal_pdf(m / sig); };
    double Jb = kPI * R * R * face(ubar);
    double Jt = kPI * R * R * face(-ubar);
    const double ufd = nu > 0 ? Ez / nu : 0.0;
    if (S.flags & OD_FLAG_FIELD_DRIVEN) {
        // inflows of the field-driven distribution: A(0) = e^c Phi(-sig/ufd)
        const double r = sig / ufd;
        const double A0 = std::exp(0.5 * r * r) * normal_cdf(-r);
        const double tail0 = ufd * A0 + sig * normal_pdf(0.0) + 0.5 * ufd;
        Jb = kPI * R * R * tail0;
        Jt = kPI * R * R * (tail0 - ufd);
    }
    const double Js = 2.0 * kPI * R * H * sig / std::sqrt(2.0 * kPI);
    const double J = Jb + Jt + Js;

    odk::PushArgs& pu = c.pu;
    pu.N = (int)N;
    pu.Npad = (int)Npad;
    pu.nd = nd;
    pu.flags = S.flags;
    pu.dt = dt;
    pu.sig = sig;
    pu.ubar = ubar;
    pu.R = R;
    pu.H = H;
    pu.k0 = S.seed;
    pu.k1 = S.system_id;
    pu.Tc = prob_to_threshold(Pc);
    pu.Tb = prob_to_threshold(Jb / J);
    pu.Tbt = prob_to_threshold((Jb + Jt) / J);
    pu.ufd = ufd;

    odk::FinalArgs& fa = c.fa;
    fa.nd = nd;
    fa.mode = S.charge_mode;
    fa.n_discard = S.n_discard;
    fa.dt = dt;
    fa.w = w;
    const double ve = std::sqrt(8.0 * kKB * P.T_e / (kPI * kME));
    const double vt = std::sqrt(2.0 * kKB * P.T_i / P.m_i);
    for (int d = 0; d < nd; ++d) {
        const double a = dust[d].radius;
        fa.Ie0[d] = kPI * a * a * P.n_inf * ve / wpi;
        fa.Ii0[d] = kPI * a * a * P.n_inf * vt / wpi;
        fa.psi[d] = kQE * kQE / (4.0 * kPI * kEPS0 * a * kKB * P.T_e);
    }
    fa.s_oml = ubar * cs / vt;
    fa.te_over_ti = P.T_e / P.T_i;
    const double k_e2 = kQE * kQE / (4.0 * kPI * kEPS0 * lam * lam);
    fa.c_orbit = w * k_e2;
    fa.c_dd = k_e2;
    fa.c_coll = w * P.m_i * cs / S.dt;
    fa.c_ext = kQE * E_si;
}

// Exponents of u = (r/R)^2 and v = (z/(H/2))^2 in the fifteen terms of
// Eq. (A.3), in the order of the coefficients alpha_0 .. alpha_14.
constexpr int kTermU[15] = {0, 1, 0, 1, 2, 0, 2, 1, 3, 0, 2, 3, 1, 4, 0};
constexpr int kTermV[15] = {0, 0, 1, 1, 0, 2, 1, 2, 0, 3, 2, 1, 3, 0, 4};

double ipow(double x, int k)
{
    double r = 1.0;
    while (k-- > 0) r *= x;
    return r;
}

// Least-squares fit of Eq. (A.3) to the confinement grid (node (k, p) at
// index (kConfNz + 1) k + p), every node weighted alike: Householder QR of
// the (nodes x 15) design matrix in the scaled variables u = (k/nr)^2,
// v = (p/nz)^2, then back substitution.  False if the matrix is singular.
bool fit_confinement(const double* grid, double* coef)
{
    const int m = kConfNodes, n = 15;
    std::vector<double> A((size_t)m * n), b(grid, grid + m), rdiag(n);   // A column-major
    for (int g = 0; g < m; ++g) {
        const double r = (double)(g / (kConfNz + 1)) / kConfNr, z = (double)(g % (kConfNz + 1)) / kConfNz;
        for (int j = 0; j < n; ++j) A[(size_t)j * m + g] = ipow(r * r, kTermU[j]) * ipow(z * z, kTermV[j]);
    }
    for (int j = 0; j < n; ++j) {
        double* a = &A[(size_t)j * m];
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += a[i] * a[i];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) return false;
        const double alpha = a[j] > 0.0 ? -nrm : nrm;
        a[j] -= alpha;                                  // Householder vector in a[j..m)
        double vv = 0.0;
        for (int i = j; i < m; ++i) vv += a[i] * a[i];
        auto reflect = [&](double* col) {
            double dot = 0.0;
            for (int i = j; i < m; ++i) dot += a[i] * col[i];
            const double f = 2.0 * dot / vv;
            for (int i = j; i < m; ++i) col[i] -= f * a[i];
        };
        for (int k = j + 1; k < n; ++k) reflect(&A[(size_t)k * m]);
        reflect(b.data());
        rdiag[j] = alpha;
    }
    for (int j = n - 1; j >= 0; --j) {
        double t = b[j];
        for (int k = j + 1; k < n; ++k) t -= A[(size_t)k * m + j] * coef[k];
        coef[j] = t / rdiag[j];
        if (!std::isfinite(coef[j])) return false;
    }
    return true;
}

// Confinement field of one system (Appendix A), from its ions at X, Y, Z:
// the grid on the device into dbuf (kConfNodes doubles), the fit on the host.
// Fills grid (dimensionless potentials), the field of the pair kernels and
// e E_out at every grain for the force of Eq. (1).  Synchronises the stream.
template <typename T>
od_status setup_confinement(hipStream_t st, const T* X, const T* Y, const T* Z, int N,
                            double* dbuf, SysConsts& c, double Te, std::vector<double>& grid)
{
    const double R = c.pu.R, Hh = 0.5 * c.pu.H;
    odk::conf_grid_kernel<T><<<kConfNodes, 256, 0, st>>>(X, Y, Z, N, c.pa.Cd, R, Hh, kConfNr, kConfNz, dbuf);
    HIPCHK(hipGetLastError());
    grid.assign(kConfNodes, 0.0);
    HIPCHK(hipMemcpyAsync(grid.data(), dbuf, kConfNodes * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    odk::ConfField& cf = c.pa.cf;
    if (!fit_confinement(grid.data(), cf.c)) return fail(OD_ENUMERIC, "confinement fit failed");
    cf.on = 1;
    cf.iu = 1.0 / (R * R);
    cf.iv = 1.0 / (Hh * Hh);
    const double e_unit = kKB * Te / c.lam;          // N per e per unit dimensionless field
    for (int d = 0; d < c.ds.nd; ++d) {
        double e[3];
        odk::conf_field(cf, c.ds.pos[d][0], c.ds.pos[d][1], c.ds.pos[d][2], e[0], e[1], e[2]);
        for (int k = 0; k < 3; ++k) c.fa.eout[d][k] = e[k] * e_unit;
    }
    return OD_OK;
}

// Coefficients (volts) and grid (volts, may be null) of a fitted field.
od_status report_confinement(const odk::ConfField& cf, const std::vector<double>& grid, double Te,
                             double* coef, double* grid_out, int32_t* nr, int32_t* nz)
{
    if (!cf.on) return fail(OD_ESTATE, "the confinement field is not enabled for this system");
    const double volt = kKB * Te / kQE;
    if (coef)
        for (int m = 0; m < 15; ++m) coef[m] = cf.c[m] * volt;
    if (grid_out)
        for (int g = 0; g < kConfNodes; ++g) grid_out[g] = grid[g] * volt;
    if (nr) *nr = kConfNr;
    if (nz) *nz = kConfNz;
    return OD_OK;
}

void derive(od_system* s)
{
    SysConsts c;
    derive_consts(s->pl, s->sim, s->dust, s->nd, s->N, s->Npad, c);
    s->lam = c.lam;
    s->wpi = c.wpi;
    s->cs = c.cs;
    s->ds = c.ds;
    s->pa = c.pa;
    s->pu = c.pu;
    s->fa = c.fa;
}

// Partial-acceleration planes the push adds: the chosen source split for the
// one-sided all-pairs kernel, one plane for the symmetric and cutoff paths.
int eff_split(const od_system* s) { return (s->cut || s->sym) ? 1 : s->nsplit; }

hipEvent_t next_event(od_system* s)
{
    if (s->evnext == s->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        s->evpool.push_back(e);
    }
    return s->evpool[s->evnext++];
}

od_status launch_step(od_system* s, bool timed);

// Blocks of 64 threads of the reinjection kernel for `ions` ions: one thread
// per 128 ions, several times the ions lost in a step of the configurations
// (about 0.2 % of N at Mach 1); the kernel walks the list with a grid stride,
// so a longer list is still covered.
// Systems up to this size reinject their lost ions inside the tail kernel
// (a step is then two launches); larger ones list them for reinject_kernel,
// which keeps the FP64 sampling out of the streaming tail's register budget.
constexpr int64_t kInlineReinjectMaxN = 16384;

int reinject_grid(int64_t ions) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (ions + 8191) / 8192)); }

void drop_graph(od_system* s)
{
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
}

// Captures s->graph_steps steps of the system's stream as one graph.
od_status capture_graph(od_system* s)
{
    drop_graph(s);
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < s->graph_steps; ++k) {
        od_status st = launch_step(s, false);
        if (st != OD_OK) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
    }
    HIPCHK(hipStreamEndCapture(s->stream, &s->graph));
    HIPCHK(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
    return OD_OK;
}

od_status launch_step(od_system* s, bool timed)
{
    const int gp = (int)(s->Npad / kPairBlock);
    const int gt = (int)(s->Npad / 256);      // tail blocks
    const odk::LostList lost{s->ctl->lost_seg, &s->ctl->lost_ticket, s->lost, odk::lost_cap(gt)};
    const bool inl = s->N <= kInlineReinjectMaxN;
    for (int k = 0; k < (inl ? 2 : 3); ++k) {
        int e0 = -1, e1 = -1;
        if (timed) {
            e0 = (int)s->evnext;
            hipEvent_t e = next_event(s);
            if (!e) return fail(OD_EDEVICE, "hipEventCreate failed");
            HIPCHK(hipEventRecord(e, s->stream));
        }
        if (k == 0 && s->cut) {
            const float* x = (const float*)s->x;
            const int64_t P = s->Npad;
            const int nb = s->ca.nblk;
            odk::slab_count_kernel<<<nb, 256, 0, s->stream>>>(x + 2 * P, (int)s->N, s->ca, s->slab, s->table);
            odk::slab_scan_kernel<<<s->ca.nslab, 256, 0, s->stream>>>(s->table, nb, s->slab_total);
            odk::slab_start_kernel<<<1, odk::kMaxSlabs, 0, s->stream>>>(s->slab_total, s->ca.nslab, s->slab_start);
            odk::slab_scatter_kernel<<<nb, 256, 0, s->stream>>>(
                x, x + P, x + 2 * P, (int)s->N, s->ca, s->slab, s->table, s->slab_start, s->xs_sorted,
                s->xs_sorted + P, s->xs_sorted + 2 * P, s->idx_sorted);
            odk::pair_cut_kernel<kPairBlock><<<nb, kPairBlock, 0, s->stream>>>(
                s->xs_sorted, s->slab_start, s->cut_fix, s->pa, s->ca, s->ctl);
            odk::pair_cut_epilogue<<<nb, 256, 0, s->stream>>>(s->xs_sorted, s->idx_sorted, s->cut_fix,
                                                               (float*)s->a, s->pa, s->ds, s->ctl);
        } else if (k == 0 && s->sym) {
            if (s->n_sym_items > 0)     // none in test-particle mode
                odk::pair_sym_kernel<kPairBlock><<<s->n_sym_items, kPairBlock, 0, s->stream>>>(
                    (const float*)s->x, (int)s->Npad, (int)s->N, s->pa.sym_scale, s->sym_items, s->acc_fix,
                    s->ctl);
        } else if (k == 0) {
            if (s->prec == OD_PREC_FP32)
                odk::pair_forces_f32<kPairBlock, kPairTile><<<gp * s->nsplit, kPairBlock, 0, s->stream>>>(
                    (const float*)s->x, (float*)s->a, s->pa, s->ds, s->ctl, s->nsplit);
            else
                odk::pair_forces_f64<kPairBlock, kPairTile><<<gp, kPairBlock, 0, s->stream>>>(
                    (const double*)s->x, (double*)s->a, s->pa, s->ds, s->ctl);
        } else if (k == 1 && s->sym && !s->cut && inl) {
            odk::step_tail_inl_kernel<float, true><<<gt, 256, 0, s->stream>>>(
                (float*)s->x, (float*)s->v, (float*)s->a, s->acc_fix, s->ev, 1, s->pa, s->pu, s->ds, s->fa,
                s->ctl, lost);
        } else if (k == 1 && s->sym && !s->cut) {
            odk::step_tail_kernel<float, true><<<gt, 256, 0, s->stream>>>(
                (float*)s->x, (float*)s->v, (float*)s->a, s->acc_fix, s->ev, 1, s->pa, s->pu, s->ds, s->fa,
                s->ctl, lost);
        } else if (k == 1 && s->prec == OD_PREC_FP32 && inl) {
            odk::step_tail_inl_kernel<float, false><<<gt, 256, 0, s->stream>>>(
                (float*)s->x, (float*)s->v, (float*)s->a, nullptr, s->ev, eff_split(s), s->pa, s->pu, s->ds,
                s->fa, s->ctl, lost);
        } else if (k == 1 && s->prec == OD_PREC_FP32) {
            odk::step_tail_kernel<float, false><<<gt, 256, 0, s->stream>>>(
                (float*)s->x, (float*)s->v, (float*)s->a, nullptr, s->ev, eff_split(s), s->pa, s->pu, s->ds,
                s->fa, s->ctl, lost);
        } else if (k == 1 && inl) {
            odk::step_tail_inl_kernel<double, false><<<gt, 256, 0, s->stream>>>(
                (double*)s->x, (double*)s->v, (double*)s->a, nullptr, s->ev, 1, s->pa, s->pu, s->ds, s->fa,
                s->ctl, lost);
        } else if (k == 1) {
            odk::step_tail_kernel<double, false><<<gt, 256, 0, s->stream>>>(
                (double*)s->x, (double*)s->v, (double*)s->a, nullptr, s->ev, 1, s->pa, s->pu, s->ds, s->fa,
                s->ctl, lost);
        } else if (inl) {
            // reinjected inside the tail
        } else if (s->prec == OD_PREC_FP32) {
            odk::reinject_kernel<float><<<reinject_grid(s->Npad), 64, 0, s->stream>>>(
                (float*)s->x, (float*)s->v, s->pu, s->ctl, lost);
        } else {
            odk::reinject_kernel<double><<<reinject_grid(s->Npad), 64, 0, s->stream>>>(
                (double*)s->x, (double*)s->v, s->pu, s->ctl, lost);
        }
        HIPCHK(hipGetLastError());
        if (timed) {
            e1 = (int)s->evnext;
            hipEvent_t e = next_event(s);
            if (!e) return fail(OD_EDEVICE, "hipEventCreate failed");
            HIPCHK(hipEventRecord(e, s->stream));
            s->marks[k].push_back({e0, e1});
        }
    }
    return OD_OK;
}

// OD_EDEVICE with a plain message when no HIP device is visible, so that a
// missing GPU is not reported as a failed allocation further on.
od_status need_device()
{
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || nd < 1) {
        (void)hipGetLastError();
        return fail(OD_EDEVICE, "no HIP device is visible");
    }
    return OD_OK;
}

od_status read_status(od_system* s)
{
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, &s->ctl->status, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (st & odk::kStPlace) return fail(OD_ESTATE, "an ion could not be placed outside the grains");
    if (st & odk::kStNaN) return fail(OD_ENUMERIC, "non-finite charge or force on the device");
    if (st & odk::kStOverflow) return fail(OD_ENUMERIC, "fixed-point accumulator overflow");
    return OD_OK;
}

}  // namespace

extern "C" {

const char* od_last_error(void) { return g_err.c_str(); }

od_status od_init_system(const od_plasma* plasma, const od_sim* sim, const od_dust* dust,
                         int32_t n_dust, void* hip_stream, const od_allocator* allocator,
                         od_system** out)
{
    if (!out) return fail(OD_EINVAL, "null out");
    *out = nullptr;
    od_status st = check_params(plasma, sim, dust, n_dust);
    if (st != OD_OK) return st;
    if (allocator && (!allocator->alloc || !allocator->release))
        return fail(OD_EINVAL, "allocator needs alloc and release");
    st = need_device();
    if (st != OD_OK) return st;
    od_system* s = new (std::nothrow) od_system();
    if (!s) return fail(OD_ENOMEM, "host allocation failed");
    s->stream = (hipStream_t)hip_stream;
    if (allocator) {
        s->alloc = *allocator;
        s->custom_alloc = true;
    }
    s->pl = *plasma;
    s->sim = *sim;
    s->nd = n_dust;
    for (int d = 0; d < n_dust; ++d) s->dust[d] = dust[d];
    s->prec = sim->precision;
    s->esz = s->prec == OD_PREC_FP32 ? 4 : 8;
    s->N = sim->n_ions;
    s->Npad = (s->N + kPad - 1) / kPad * kPad;
    derive(s);
    // Source splits of the pair sum: enough blocks for about four per CU.
    {
        int dev = 0;
        hipDeviceProp_t prop{};
        (void)hipGetDevice(&dev);
        (void)hipGetDeviceProperties(&prop, dev);
        const int64_t nib = s->Npad / kPairBlock;
        const int64_t want = 4 * (int64_t)std::max(prop.multiProcessorCount, 1);
        s->nsplit = s->prec == OD_PREC_FP32
                        ? (int)std::min<int64_t>(kMaxSplitSingle, std::max<int64_t>(1, (want + nib - 1) / nib))
                        : 1;
        s->nsplit = (int)std::min<int64_t>(s->nsplit, nib);
    }

    const size_t vec = 3 * (size_t)s->Npad * s->esz;
    s->x = dev_alloc(s, vec);
    s->v = dev_alloc(s, vec);
    s->a = dev_alloc(s, vec * (s->prec == OD_PREC_FP32 ? kMaxSplitSingle : 1));
    s->ev = (uint8_t*)dev_alloc(s, (size_t)s->Npad);
    s->lost = (int2*)dev_alloc(s, (size_t)odk::kSlots * odk::lost_cap(s->Npad / 256) * sizeof(int2));
    s->ctl = (odk::Ctl*)dev_alloc(s, sizeof(odk::Ctl));
    if (!s->x || !s->v || !s->a || !s->ev || !s->lost || !s->ctl) {
        od_destroy(s);
        return fail(OD_ENOMEM, "device allocation of %zu bytes failed", 3 * vec);
    }
    odk::Ctl h{};
    std::memset(&h, 0, sizeof h);
    for (int d = 0; d < n_dust; ++d) h.Q[d] = dust[d].q0 / kQE;
    hipError_t e = hipMemcpyAsync(s->ctl, &h, sizeof h, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->ev, 0, (size_t)s->Npad, s->stream);
    if (e != hipSuccess) {
        od_destroy(s);
        return fail(OD_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    const int gi = (int)((s->Npad + 255) / 256);
    if (s->prec == OD_PREC_FP32)
        odk::init_kernel<float><<<gi, 256, 0, s->stream>>>((float*)s->x, (float*)s->v, (float*)s->a,
                                                           s->pu, s->ds, s->ctl);
    else
        odk::init_kernel<double><<<gi, 256, 0, s->stream>>>((double*)s->x, (double*)s->v,
                                                            (double*)s->a, s->pu, s->ds, s->ctl);
    e = hipGetLastError();
    if (e != hipSuccess) {
        od_destroy(s);
        return fail(OD_EDEVICE, "init kernel launch failed: %s", hipGetErrorString(e));
    }
    st = read_status(s);
    if (st == OD_OK && (sim->flags & OD_FLAG_CONFINEMENT)) {
        double* dbuf = (double*)dev_alloc(s, kConfNodes * sizeof(double));
        if (!dbuf) st = fail(OD_ENOMEM, "device allocation of the confinement grid failed");
        SysConsts c;
        c.lam = s->lam; c.ds = s->ds; c.pa = s->pa; c.pu = s->pu; c.fa = s->fa;
        const int64_t P = s->Npad;
        if (st == OD_OK && s->prec == OD_PREC_FP32) {
            const float* x = (const float*)s->x;
            st = setup_confinement<float>(s->stream, x, x + P, x + 2 * P, (int)s->N, dbuf, c, plasma->T_e, s->conf_grid);
        } else if (st == OD_OK) {
            const double* x = (const double*)s->x;
            st = setup_confinement<double>(s->stream, x, x + P, x + 2 * P, (int)s->N, dbuf, c, plasma->T_e, s->conf_grid);
        }
        if (dbuf) {
            (void)hipStreamSynchronize(s->stream);
            dev_free(s, dbuf);
        }
        s->pa = c.pa;
        s->fa = c.fa;
    }
    if (st == OD_OK) st = apply_pair_kind(s);
    if (st != OD_OK) {
        od_destroy(s);
        return st;
    }
    *out = s;
    return OD_OK;
}

od_status od_step(od_system* s, int64_t n_steps)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (n_steps < 0) return fail(OD_EINVAL, "n_steps < 0");
    int64_t left = n_steps;
    if (s->graph_steps > 0 && !s->timing) {
        if (!s->gexec && left >= s->graph_steps) {
            od_status st = capture_graph(s);
            if (st != OD_OK) return st;
        }
        for (; s->gexec && left >= s->graph_steps; left -= s->graph_steps)
            HIPCHK(hipGraphLaunch(s->gexec, s->stream));
    }
    for (; left > 0; --left) {
        od_status st = launch_step(s, s->timing);
        if (st != OD_OK) return st;
    }
    return OD_OK;
}

od_status od_set_graph(od_system* s, int32_t steps_per_graph)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (steps_per_graph < 0 || steps_per_graph > 1000) return fail(OD_EINVAL, "steps_per_graph out of [0,1000]");
    if (steps_per_graph > 0 && s->stream == nullptr)
        return fail(OD_ESTATE, "graph capture needs a stream of the system's own (not the null stream)");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->graph_steps = steps_per_graph;
    return OD_OK;
}

od_status od_sync(od_system* s)
{
    if (!s) return fail(OD_EINVAL, "null system");
    return read_status(s);
}

od_status od_get_dust_charges(od_system* s, double* q_now, double* q_avg)
{
    if (!s) return fail(OD_EINVAL, "null system");
    odk::Ctl h;
    HIPCHK(hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int d = 0; d < s->nd; ++d) {
        if (q_now) q_now[d] = h.Q[d] * kQE;
        if (q_avg) q_avg[d] = h.nrec ? h.sums[d][0] / (double)h.nrec * kQE : 0.0;
    }
    return read_status(s);
}

od_status od_get_dust_forces(od_system* s, int32_t which, double* f)
{
    if (!s || !f) return fail(OD_EINVAL, "null argument");
    if (which != 0 && which != 1) return fail(OD_EINVAL, "which must be 0 or 1");
    odk::Ctl h;
    HIPCHK(hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int d = 0; d < s->nd; ++d)
        for (int c = 0; c < 12; ++c) {
            if (which == 0)
                f[12 * d + c] = h.last[d][1 + c];
            else
                f[12 * d + c] = h.nrec ? h.sums[d][1 + c] / (double)h.nrec : 0.0;
        }
    return read_status(s);
}

void od_destroy(od_system* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    drop_graph(s);
    free_cutoff(s);
    free_sym(s);
    dev_free(s, s->x);
    dev_free(s, s->v);
    dev_free(s, s->a);
    dev_free(s, s->ev);
    dev_free(s, s->lost);
    dev_free(s, s->hist);
    dev_free(s, s->ctl);
    for (hipEvent_t e : s->evpool) (void)hipEventDestroy(e);
    delete s;
}

od_status od_set_cutoff(od_system* s, double r_switch, double r_cut)
{
    if (!s) return fail(OD_EINVAL, "null system");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    if (!(r_cut > 0.0)) {
        if (s->cut) free_cutoff(s);
        return OD_OK;
    }
    if (s->prec != OD_PREC_FP32) return fail(OD_EINVAL, "the cutoff path runs in FP32 only");
    if (!(r_switch >= 0.0) || !(r_switch < r_cut)) return fail(OD_EINVAL, "need 0 <= r_switch < r_cut");
    const double H = s->sim.H / s->lam, rc = r_cut / s->lam, rs = r_switch / s->lam;
    // Slabs of about r_cut / 16, so that the blocks within reach overshoot the
    // cutoff sphere by little; where that many would pass kMaxSlabs, r_cut / 8
    // (timed faster there than the capped finer width).  reach = ceil(r_cut / width).
    const double per = std::floor(16.0 * H / rc) <= odk::kMaxSlabs ? 16.0 : 8.0;
    const int nslab = (int)std::min<double>(odk::kMaxSlabs, std::max(1.0, std::floor(per * H / rc)));
    const int reach = (int)std::ceil(rc * nslab / H);
    const int nblk = (int)(s->Npad / 256);
    if (s->cut) free_cutoff(s);
    const size_t P = (size_t)s->Npad;
    s->xs_sorted = (float*)dev_alloc(s, 3 * P * sizeof(float));
    s->idx_sorted = (int*)dev_alloc(s, P * sizeof(int));
    s->slab = (int*)dev_alloc(s, P * sizeof(int));
    s->table = (int*)dev_alloc(s, (size_t)nslab * nblk * sizeof(int));
    s->slab_total = (int*)dev_alloc(s, (size_t)nslab * sizeof(int));
    s->slab_start = (int*)dev_alloc(s, (size_t)(nslab + 1) * sizeof(int));
    s->cut_fix = (unsigned long long*)dev_alloc(s, 3 * P * sizeof(unsigned long long));
    if (!s->xs_sorted || !s->idx_sorted || !s->slab || !s->table || !s->slab_total || !s->slab_start ||
        !s->cut_fix) {
        free_cutoff(s);
        return fail(OD_ENOMEM, "device allocation of the slab sort failed");
    }
    HIPCHK(hipMemset(s->cut_fix, 0, 3 * P * sizeof(unsigned long long)));
    // padding slots of the sorted copy sit far away and are never overwritten
    const size_t npad = P - (size_t)s->N;
    if (npad) {
        std::vector<float> far(npad, 1.0e18f);
        std::vector<int> none(npad, -1);
        for (int c = 0; c < 3; ++c)
            HIPCHK(hipMemcpy(s->xs_sorted + c * P + s->N, far.data(), npad * sizeof(float), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(s->idx_sorted + s->N, none.data(), npad * sizeof(int), hipMemcpyHostToDevice));
    }
    s->ca.nslab = nslab;
    s->ca.nblk = nblk;
    s->ca.reach = std::max(reach, 1);
    s->ca.z0 = (float)(-0.5 * H);
    s->ca.inv_w = (float)(nslab / H);
    s->ca.rsw = (float)rs;
    s->ca.inv_sw = (float)(1.0 / (rc - rs));
    s->cut = true;
    return OD_OK;
}

od_status od_get_cutoff_info(od_system* s, int32_t* nslab, int64_t* pairs_evaluated)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (!s->cut) return fail(OD_ESTATE, "no cutoff is set");
    const int ns = s->ca.nslab;
    std::vector<int> start(ns + 1);
    HIPCHK(hipMemcpyAsync(start.data(), s->slab_start, (ns + 1) * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (nslab) *nslab = ns;
    if (pairs_evaluated) {
        // slab of sorted slot p: the s with start[s] <= p < start[s + 1]
        auto slab_at = [&](int64_t p) {
            return (int)(std::upper_bound(start.begin(), start.end(), (int)p) - start.begin()) - 1;
        };
        // tile I meets tiles I .. J1 - 1; off-diagonal tile pairs count both ways
        int64_t total = 0;
        for (int64_t i0 = 0; i0 < s->N; i0 += 256) {
            const int hi = slab_at(std::min<int64_t>(i0 + 256, s->N) - 1);
            const int64_t je = start[std::min(hi + s->ca.reach + 1, ns)];
            const int64_t tiles = (je + 255) / 256 - i0 / 256;
            total += 256 * 256 * (2 * tiles - 1);
        }
        *pairs_evaluated = total;
    }
    return OD_OK;
}

od_status od_get_confinement(od_system* s, double* coef, double* grid, int32_t* nr, int32_t* nz)
{
    if (!s) return fail(OD_EINVAL, "null system");
    return report_confinement(s->pa.cf, s->conf_grid, s->pl.T_e, coef, grid, nr, nz);
}

od_status od_get_units(od_system* s, double* u)
{
    if (!s || !u) return fail(OD_EINVAL, "null argument");
    u[0] = s->lam;
    u[1] = 1.0 / s->wpi;
    u[2] = s->cs;
    u[3] = s->lam * s->wpi * s->wpi;
    return OD_OK;
}

od_status od_get_sizes(od_system* s, int64_t* o)
{
    if (!s || !o) return fail(OD_EINVAL, "null argument");
    o[0] = s->N;
    o[1] = s->nd;
    o[2] = s->prec;
    o[3] = s->Npad;
    return OD_OK;
}

static od_status copy_soa_out(od_system* s, const void* dev, void* host)
{
    const size_t row = (size_t)s->N * s->esz;
    const size_t drow = (size_t)s->Npad * s->esz;
    for (int c = 0; c < 3; ++c)
        HIPCHK(hipMemcpyAsync((char*)host + c * row, (const char*)dev + c * drow, row,
                              hipMemcpyDeviceToHost, s->stream));
    return OD_OK;
}

od_status od_get_state(od_system* s, void* x, void* v, double* q, int64_t* step)
{
    if (!s) return fail(OD_EINVAL, "null system");
    od_status st;
    if (x && (st = copy_soa_out(s, s->x, x)) != OD_OK) return st;
    if (v && (st = copy_soa_out(s, s->v, v)) != OD_OK) return st;
    odk::Ctl h;
    HIPCHK(hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (q)
        for (int d = 0; d < s->nd; ++d) q[d] = h.Q[d] * kQE;
    if (step) *step = h.step;
    return OD_OK;
}

od_status od_set_state(od_system* s, const void* x, const void* v, const double* q, int64_t step)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (step < 0) return fail(OD_EINVAL, "step < 0");
    const int64_t N = s->N;
    auto val = [&](const void* p, int64_t k) {
        return s->prec == OD_PREC_FP32 ? (double)((const float*)p)[k] : ((const double*)p)[k];
    };
    for (const void* p : {x, v}) {
        if (!p) continue;
        for (int64_t k = 0; k < 3 * N; ++k)
            if (!std::isfinite(val(p, k))) return fail(OD_ENUMERIC, "non-finite state value at %lld", (long long)k);
    }
    if (x) {
        for (int64_t i = 0; i < N; ++i) {
            const double px = val(x, i), py = val(x, N + i), pz = val(x, 2 * N + i);
            for (int d = 0; d < s->nd; ++d) {
                const double a0 = px - s->ds.pos[d][0], a1 = py - s->ds.pos[d][1], a2 = pz - s->ds.pos[d][2];
                if (a0 * a0 + a1 * a1 + a2 * a2 <= s->ds.rad2[d])
                    return fail(OD_ESTATE, "ion %lld lies inside grain %d", (long long)i, d);
            }
        }
    }
    if (q)
        for (int d = 0; d < s->nd; ++d)
            if (!std::isfinite(q[d])) return fail(OD_ENUMERIC, "non-finite charge");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    const size_t row = (size_t)N * s->esz;
    const size_t drow = (size_t)s->Npad * s->esz;
    for (int c = 0; c < 3; ++c) {
        if (x)
            HIPCHK(hipMemcpyAsync((char*)s->x + c * drow, (const char*)x + c * row, row,
                                  hipMemcpyHostToDevice, s->stream));
        if (v)
            HIPCHK(hipMemcpyAsync((char*)s->v + c * drow, (const char*)v + c * row, row,
                                  hipMemcpyHostToDevice, s->stream));
    }
    odk::Ctl h;
    HIPCHK(hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (q)
        for (int d = 0; d < s->nd; ++d) h.Q[d] = q[d] / kQE;
    h.step = step;
    HIPCHK(hipMemcpyAsync(s->ctl, &h, sizeof h, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return OD_OK;
}

od_status od_get_accelerations(od_system* s, void* a)
{
    if (!s || !a) return fail(OD_EINVAL, "null argument");
    od_status st = copy_soa_out(s, s->a, a);
    if (st != OD_OK) return st;
    HIPCHK(hipStreamSynchronize(s->stream));
    if (eff_split(s) > 1) {   // add the partial planes in the push's order
        std::vector<float> part(3 * (size_t)s->N);
        float* out = (float*)a;
        for (int k = 1; k < eff_split(s); ++k) {
            st = copy_soa_out(s, (const char*)s->a + (size_t)k * 3 * s->Npad * s->esz, part.data());
            if (st != OD_OK) return st;
            HIPCHK(hipStreamSynchronize(s->stream));
            for (size_t i = 0; i < part.size(); ++i) out[i] += part[i];
        }
    }
    return OD_OK;
}

od_status od_set_pair_kernel(od_system* s, int32_t kind)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (kind != OD_PAIR_AUTO && kind != OD_PAIR_ONE_SIDED && kind != OD_PAIR_SYMMETRIC)
        return fail(OD_EINVAL, "unknown pair kernel kind %d", kind);
    if (kind == OD_PAIR_SYMMETRIC && s->prec != OD_PREC_FP32)
        return fail(OD_EINVAL, "the symmetric sum needs FP32");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    const int old = s->pair_kind;
    s->pair_kind = kind;
    od_status st = apply_pair_kind(s);
    if (st != OD_OK) s->pair_kind = old;
    return st;
}

od_status od_get_pair_kernel(od_system* s, int32_t* kind)
{
    if (!s || !kind) return fail(OD_EINVAL, "null argument");
    *kind = s->sym ? OD_PAIR_SYMMETRIC : OD_PAIR_ONE_SIDED;
    return OD_OK;
}

od_status od_set_pair_split(od_system* s, int32_t nsplit)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (s->cut && nsplit != 1) return fail(OD_ESTATE, "the pair sum is not split while a cutoff is set");
    if (s->sym && nsplit != 1) return fail(OD_ESTATE, "the symmetric pair sum is not split");
    if (nsplit < 1 || nsplit > kMaxSplitSingle) return fail(OD_EINVAL, "nsplit must be in [1,%d]", kMaxSplitSingle);
    if (s->prec != OD_PREC_FP32 && nsplit != 1) return fail(OD_EINVAL, "the FP64 mode does not split");
    if (nsplit > s->Npad / kPairBlock) return fail(OD_EINVAL, "more splits than source tiles");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->nsplit = nsplit;
    return OD_OK;
}

od_status od_get_pair_split(od_system* s, int32_t* nsplit)
{
    if (!s || !nsplit) return fail(OD_EINVAL, "null argument");
    *nsplit = eff_split(s);
    return OD_OK;
}

od_status od_get_step_events(od_system* s, uint8_t* ev, int64_t* n_abs, int64_t* n_exit, int64_t* n_coll)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (ev) HIPCHK(hipMemcpyAsync(ev, s->ev, (size_t)s->N, hipMemcpyDeviceToHost, s->stream));
    odk::Ctl h;
    HIPCHK(hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (n_abs)
        for (int d = 0; d < s->nd; ++d) n_abs[d] = (int64_t)h.last[d][13];
    if (n_exit) *n_exit = h.last_exit;
    if (n_coll) *n_coll = h.last_coll;
    return OD_OK;
}

od_status od_get_absorbed(od_system* s, int64_t* absorbed, int32_t* by_dust, int64_t cap, int64_t* n_absorbed,
                          int64_t* n_exited)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (cap < 0) return fail(OD_EINVAL, "cap < 0");
    std::vector<uint8_t> ev((size_t)s->N);
    HIPCHK(hipMemcpyAsync(ev.data(), s->ev, (size_t)s->N, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    int64_t na = 0, ne = 0;
    for (int64_t i = 0; i < s->N; ++i) {
        const int code = ev[(size_t)i] & 0x7f;
        if (code == odk::kEvExit) {
            ++ne;
        } else if (code >= odk::kEvAbsBase) {
            if (na < cap) {
                if (absorbed) absorbed[na] = i;
                if (by_dust) by_dust[na] = code - odk::kEvAbsBase;
            }
            ++na;
        }
    }
    if (n_absorbed) *n_absorbed = na;
    if (n_exited) *n_exited = ne;
    return OD_OK;
}

od_status od_set_history(od_system* s, int64_t capacity)
{
    if (!s) return fail(OD_EINVAL, "null system");
    if (capacity < 0 || capacity > ((int64_t)1 << 30)) return fail(OD_EINVAL, "capacity out of [0, 2^30]");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    dev_free(s, s->hist);
    s->hist = nullptr;
    s->fa.hist = nullptr;
    s->fa.hist_cap = 0;
    if (capacity == 0 || s->nd == 0) return OD_OK;
    s->hist = (double*)dev_alloc(s, (size_t)capacity * s->nd * odk::kHistWords * sizeof(double));
    if (!s->hist) return fail(OD_ENOMEM, "device allocation of the history failed");
    odk::Ctl h;
    HIPCHK(hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->fa.hist = s->hist;
    s->fa.hist_start = h.step;
    s->fa.hist_cap = capacity;
    return OD_OK;
}

od_status od_get_history(od_system* s, double* rec, int64_t* n_recorded)
{
    if (!s) return fail(OD_EINVAL, "null system");
    odk::Ctl h;
    HIPCHK(hipMemcpyAsync(&h, s->ctl, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const int64_t n = s->hist ? std::max<int64_t>(0, std::min<int64_t>(h.step - s->fa.hist_start, s->fa.hist_cap)) : 0;
    if (n_recorded) *n_recorded = n;
    if (rec && n > 0) {
        const size_t words = (size_t)n * s->nd * odk::kHistWords;
        HIPCHK(hipMemcpyAsync(rec, s->hist, words * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        for (size_t k = 0; k < words; k += odk::kHistWords) rec[k] *= kQE;   // charge e -> C
    }
    return OD_OK;
}

od_status od_rng_block(uint64_t seed, uint64_t system, const uint64_t* ctr, uint64_t* out)
{
    if (!ctr || !out) return fail(OD_EINVAL, "null argument");
    uint64_t* d = nullptr;
    HIPCHK(hipMalloc(&d, 4 * sizeof(uint64_t)));
    odk::rng_kernel<<<1, 64>>>(seed, system, ctr[0], ctr[1], ctr[2], ctr[3], d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(out, d, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(OD_EDEVICE, "rng kernel: %s", hipGetErrorString(e));
    return OD_OK;
}

od_status od_set_timing(od_system* s, int32_t enable)
{
    if (!s) return fail(OD_EINVAL, "null system");
    HIPCHK(hipStreamSynchronize(s->stream));
    s->timing = enable != 0;
    for (auto& m : s->marks) m.clear();
    s->evnext = 0;
    return OD_OK;
}

od_status od_get_kernel_times(od_system* s, double* ms, int64_t* launches)
{
    if (!s) return fail(OD_EINVAL, "null system");
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int k = 0; k < 4; ++k) {
        double tot = 0.0;
        for (auto& m : s->marks[k]) {
            float t = 0.0f;
            HIPCHK(hipEventElapsedTime(&t, s->evpool[m.first], s->evpool[m.second]));
            tot += t;
        }
        if (ms) ms[k] = tot;
        if (launches) launches[k] = (int64_t)s->marks[k].size();
        s->marks[k].clear();
    }
    s->evnext = 0;
    return OD_OK;
}

}  // extern "C"

#include "batch_api.inc"
#include "mlp_api.inc"

extern "C" od_status od_oml_floating_charge(const od_plasma* P, double a, double* q)
{
    if (!P || !q || !(a > 0) || !(P->T_e > 0) || !(P->T_i > 0) || !(P->n_inf > 0) || !(P->m_i > 0))
        return fail(OD_EINVAL, "bad argument");
    // currents in A as functions of the grain charge Q (C); OML forms of the
    // "oml" charging model: electrons Boltzmann-repelled, ions collected with
    // the OML cross-section from the drifting Maxwellian.
    const double ve = std::sqrt(8.0 * kKB * P->T_e / (kPI * kME));
    const double vt = std::sqrt(2.0 * kKB * P->T_i / P->m_i);
    const double cs = std::sqrt(kKB * P->T_e / P->m_i);
    const double s = P->mach * cs / vt;
    auto total = [&](double Q) {
        const double phi = Q / (4.0 * kPI * kEPS0 * a);
        const double x = kQE * phi / (kKB * P->T_e);
        const double Ie = -kPI * a * a * P->n_inf * kQE * ve * (phi < 0 ? std::exp(x) : 1.0 + x);
        const double chi = phi < 0 ? -kQE * phi / (kKB * P->T_i) : 0.0;
        const double br = s < 1e-6 ? 2.0 / std::sqrt(kPI) * (1.0 + chi)
                                   : std::exp(-s * s) / std::sqrt(kPI) + (s * s + 0.5 + chi) * std::erf(s) / s;
        return kPI * a * a * P->n_inf * kQE * vt * br + Ie;
    };
    // bracket: total(0) < 0 (electrons dominate); grow a negative bound
    double lo = -kQE, hi = 0.0;
    int guard = 0;
    while (total(lo) < 0.0 && guard++ < 200) lo *= 2.0;
    if (total(lo) < 0.0) return fail(OD_ENUMERIC, "no floating charge found");
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (total(mid) > 0.0) lo = mid; else hi = mid;
        if (hi - lo <= 1e-15 * std::fabs(lo)) break;
    }
    *q = 0.5 * (lo + hi);
    return OD_OK;
}
