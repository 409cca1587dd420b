// ez_api.hip -- C ABI of libezeta: argument validation, programs (which
// products are integrated), quadrature plans and rule tables, the per-device
// workspace, and the launch sequence  setup -> nodes -> hadamard -> finalize.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ezeta.h"
#include "ez_internal.h"
#include "ez_kernels.h"
#include "ez_grid.h"
#include "ep_f32_rational.h"

namespace {

thread_local std::string g_err = "";

ez_status fail(ez_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define EZ_HIP_TRY(call)                                                             \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(EZ_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// Gauss-Legendre nodes on [lo, hi]: Newton's method on P_n (three-term
// recurrence), started from Tricomi's asymptotic root estimate.
void gauss_legendre(int n, double lo, double hi, double *x, double *w) {
    for (int k = 1; k <= n; ++k) {
        double th = M_PI * (4.0 * k - 1.0) / (4.0 * n + 2.0);
        double t = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(th);
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p_prev = 1.0, p = t;
            for (int j = 1; j < n; ++j) {
                double p_next = ((2.0 * j + 1.0) * t * p - j * p_prev) / (j + 1.0);
                p_prev = p;
                p = p_next;
            }
            if (n == 1) { p = t; p_prev = 1.0; }
            dp = n * (p_prev - t * p) / (1.0 - t * t);
            double dt = p / dp;
            t -= dt;
            if (std::fabs(dt) <= 1e-16) {
                // refresh dp at the final t
                p_prev = 1.0; p = t;
                for (int j = 1; j < n; ++j) {
                    double p_next = ((2.0 * j + 1.0) * t * p - j * p_prev) / (j + 1.0);
                    p_prev = p;
                    p = p_next;
                }
                if (n == 1) { p = t; p_prev = 1.0; }
                dp = n * (p_prev - t * p) / (1.0 - t * t);
                break;
            }
        }
        // roots come out in decreasing t; store ascending
        int idx = n - k;
        x[idx] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * t;
        w[idx] = (hi - lo) / ((1.0 - t * t) * dp * dp);
    }
}

// ---------------------------------------------------------------------------
// Least squares: pinv (n x P, row-major) with pinv M = I for M (P x n, row-major,
// full column rank), by modified Gram-Schmidt QR (two passes) and back substitution.
void lstsq_pinv(int P, int n, const std::vector<double> &M, std::vector<double> &pinv) {
    std::vector<double> Q(M), R((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                double r = 0.0;
                for (int p = 0; p < P; ++p) r += Q[(size_t)p * n + i] * Q[(size_t)p * n + j];
                for (int p = 0; p < P; ++p) Q[(size_t)p * n + j] -= r * Q[(size_t)p * n + i];
                R[(size_t)i * n + j] += r;
            }
        double nr = 0.0;
        for (int p = 0; p < P; ++p) nr += Q[(size_t)p * n + j] * Q[(size_t)p * n + j];
        nr = std::sqrt(nr);
        R[(size_t)j * n + j] = nr;
        for (int p = 0; p < P; ++p) Q[(size_t)p * n + j] /= nr;
    }
    // pinv = R^{-1} Q^T
    pinv.assign((size_t)n * P, 0.0);
    for (int p = 0; p < P; ++p)
        for (int i = n - 1; i >= 0; --i) {
            double v = Q[(size_t)p * n + i];
            for (int j = i + 1; j < n; ++j) v -= R[(size_t)i * n + j] * pinv[(size_t)j * P + p];
            pinv[(size_t)i * P + p] = v / R[(size_t)i * n + i];
        }
}

int n_mono(int d, int g) { return d == 1 ? 1 : (d == 2 ? g + 1 : (g + 1) * (g + 2) / 2); }

// monomials of degree g of x (order: a0 descending, then a1 descending)
void monomials(int d, int g, const double *x, std::vector<double> &out) {
    out.clear();
    if (d == 1) { out.push_back(std::pow(x[0], g)); return; }
    if (d == 2) { for (int a = g; a >= 0; --a) out.push_back(std::pow(x[0], a) * std::pow(x[1], g - a)); return; }
    for (int a = g; a >= 0; --a)
        for (int b = g - a; b >= 0; --b) out.push_back(std::pow(x[0], a) * std::pow(x[1], b) * std::pow(x[2], g - a - b));
}

// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// bumped whenever device memory the library owns is freed or moved (a buffer
// grown, a plan evicted, ez_finalize): device pointers recorded earlier, e.g. in
// a captured HIP graph, are valid while it is unchanged
std::atomic<uint64_t> g_generation{1};

ez_status grow(DevBuf &b, size_t bytes) {
    if (bytes <= b.bytes && b.p) return EZ_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        g_generation.fetch_add(1);
    }
    size_t want = std::max<size_t>(bytes, 256);
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        return fail(EZ_ERR_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    b.bytes = want;
    return EZ_OK;
}

// Device pointers and counts of a plan, wherever it lives (cached plan buffers,
// or the static scratch of the no-allocation entry point).
struct PlanView {
    const double *rules = nullptr;
    const EzInstPlan *plans = nullptr;
    const int *tile_begin = nullptr, *dir_begin = nullptr, *htile_begin = nullptr, *tile_order = nullptr;
    int n_tiles = 0, n_dirs = 0, n_htiles = 0;
    int n_probe = 0, ell_probe = 0, probe_off = 0;
    int pinv_off[EZ_ELL_MAX + 1] = {0};
};
using PlanViewBase = PlanView;

// A plan depends only on (d, batch, specs): rule tables, per-lattice plans, prefixes.
struct DevPlan {
    DevBuf rules, plans, tile_begin, dir_begin, htile_begin, tile_order;
    int n_tiles = 0, n_dirs = 0, n_htiles = 0;
    int n_probe = 0, ell_probe = 0, probe_off = 0;
    int pinv_off[EZ_ELL_MAX + 1] = {0};
    std::vector<EzInstPlan> host_plans;
};

// Signal words for stream-ordered edges between the caller's stream and the second
// stream: a stream writes the next value of a word after its prior work, the other
// waits until the word reaches it.  A value wait resumes sooner than an event wait
// (about 5 against 8.5 µs per edge between two streams, measured with 100 µs kernels
// on the MI355X).  64-bit values only grow.  Word 1 joins the node kernels' stream
// into the caller's; word 0 is allocated but unused.
struct StreamSignals {
    uint64_t *p[2] = {nullptr, nullptr};
    uint64_t seq[2] = {0, 0};
    bool ok = false;
};

struct DeviceState {
    std::map<std::string, DevPlan *> plans;
    std::vector<std::string> plan_order;
    DevBuf meta, real, rn, rows, rec, tile_part, sub_part, tail_acc, tail_cnt, dir_part, dir_flag, probe_val, tensor,
        tile_grad, dir_grad;
    DevBuf gmeta, greal, grec;   // general-x Epstein tables
    DevBuf queue;                // work-queue position of the persistent node kernel
    DevBuf tile_bound;           // mixed-precision bound partials per tile
    DevBuf dxlist, dpart;        // direct ATM sum: outer points and partial sums
    // Epstein grid workspace
    DevBuf g_pts_x, g_pts_y, g_perm, g_counts, g_A64r, g_B64r, g_A64k, g_B64k, g_R, g_Q, g_wsum, g_stat;
    long long grid_nr = 0, grid_nk = 0;          // table sizes of the last grid call
    long long sum_tiles = 0, sum_main = 0;       // node tiles of the last lattice-sum call
    int sum_tail = 0;                            // and its tail (0 none, 1 split kernel, 2 halves)
    DevBuf g_Ahr, g_Alr, g_Bhr, g_Blr, g_Ahk, g_Alk, g_Bhk, g_Blk;
    int n_cu = 0;
    hipStream_t side = nullptr;  // second stream: Hadamard branch concurrent with the nodes
    hipEvent_t ev_setup = nullptr, ev_had = nullptr;
    StreamSignals sig;           // value-wait edges between the two streams (small value calls)
    // no-allocation entry point: this device's address of the static scratch array,
    // and the plan currently resident at its start
    void *scratch = nullptr;
    std::string scratch_key;
    PlanViewBase scratch_plan;
    size_t scratch_plan_bytes = 0;
};

std::mutex g_mu;
std::map<int, DeviceState *> g_dev;

// ---- optional per-kernel timing with HIP events on the launch stream ----
struct TimedLaunch { hipEvent_t a, b; int kernel; };
bool g_timing = false;
std::vector<TimedLaunch> g_pending;
double g_ms[EZ_KERNEL_COUNT] = {0};
long long g_calls[EZ_KERNEL_COUNT] = {0};

void timing_flush() {
    for (auto &t : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            g_ms[t.kernel] += ms;
            g_calls[t.kernel] += 1;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_pending.clear();
}

// records an event pair around `launch` when timing is on
template <class F>
hipError_t timed(int kernel, hipStream_t s, F launch) {
    if (!g_timing) return launch();
    if (g_pending.size() >= 4096) timing_flush();
    TimedLaunch t;
    t.kernel = kernel;
    if (hipEventCreate(&t.a) != hipSuccess) return launch();
    if (hipEventCreate(&t.b) != hipSuccess) { (void)hipEventDestroy(t.a); return launch(); }
    (void)hipEventRecord(t.a, s);
    hipError_t e = launch();
    (void)hipEventRecord(t.b, s);
    g_pending.push_back(t);
    return e;
}

DeviceState *device_state(int dev) {
    auto it = g_dev.find(dev);
    if (it != g_dev.end()) return it->second;
    DeviceState *s = new DeviceState();
    g_dev[dev] = s;
    return s;
}

void free_buf(DevBuf &b) {
    if (b.p) {
        (void)hipFree(b.p);
        g_generation.fetch_add(1);
    }
    b.p = nullptr;
    b.bytes = 0;
}

void free_plan(DevPlan *p) {
    free_buf(p->rules); free_buf(p->plans); free_buf(p->tile_begin); free_buf(p->dir_begin);
    free_buf(p->htile_begin); free_buf(p->tile_order);
    delete p;
}

// ---------------------------------------------------------------------------
ez_status check_spec(const ez_quad_spec &s) {
    if (s.n_q < 1 || s.n_q > 64) return fail(EZ_ERR_INVALID_ARG, "spec.n_q must be in [1, 64]");
    if (s.n_panels < 1 || s.n_panels > 256) return fail(EZ_ERR_INVALID_ARG, "spec.n_panels must be in [1, 256]");
    if (s.n_g < 1 || s.n_g > 128) return fail(EZ_ERR_INVALID_ARG, "spec.n_g must be in [1, 128]");
    // Taylor orders up to 6 (the paper's reference order for its cutoff study, Sec. 4.1,
    // Table 1): beyond it the least-squares recovery of the degree-2 ell coefficient
    // polynomials from the probe values loses digits (condition ~1e6 at ell = 8)
    if (s.ell < 0 || s.ell > 6) return fail(EZ_ERR_INVALID_ARG, "spec.ell must be in [0, 6]");
    if (!(s.eps > 0.0 && s.eps < 0.5)) return fail(EZ_ERR_INVALID_ARG, "spec.eps must be in (0, 1/2)");
    if (!(s.lam >= 0.0 && s.lam <= 8.0)) return fail(EZ_ERR_INVALID_ARG, "spec.lam must be in [0, 8]");
    if (!(s.a_cut >= 0.0 && s.a_cut <= 200.0)) return fail(EZ_ERR_INVALID_ARG, "spec.a_cut must be in [0, 200]");
    if (s.precision != EZ_PREC_FP64 && s.precision != EZ_PREC_MIXED)
        return fail(EZ_ERR_INVALID_ARG, "spec.precision must be EZ_PREC_FP64 or EZ_PREC_MIXED");
    if (s.flags & ~(EZ_SPEC_PERSISTENT | EZ_SPEC_SERIAL | EZ_SPEC_NO_SPLIT | 0xFF00 | 0xFF0000 | 0x7000000))
        return fail(EZ_ERR_INVALID_ARG, "spec.flags: unknown bits");
    if (((s.flags >> 24) & 0x7) > 4) return fail(EZ_ERR_INVALID_ARG, "EZ_SPEC_WAVE_U(k): k must be in [0, 4]");
    const int amix = (s.flags >> 16) & 0xFF;
    if (amix != 0 && amix < (int)EZ_EPF_XMIN)
        return fail(EZ_ERR_INVALID_ARG, "EZ_SPEC_MIX_A(n): n must be 0 or >= 8");
    return EZ_OK;
}

double spec_lam(const ez_quad_spec &s) { return s.lam > 0.0 ? s.lam : 1.0; }
double spec_acut(const ez_quad_spec &s) { return s.a_cut > 0.0 ? s.a_cut : 36.0; }

struct Term {
    int res;
    double coef;
    std::vector<std::pair<int, int>> fac;   // (nu index, multiplicity)
};

ez_status build_program(int d, const std::vector<double> &nu, const std::vector<Term> &terms, int n_res,
                        int ell_max, EzProgram &P, std::vector<EzCombo> &combos) {
    combos.clear();
    std::memset(&P, 0, sizeof(P));
    if ((int)nu.size() < 1 || (int)nu.size() > EZ_NU_MAX) return fail(EZ_ERR_INVALID_ARG, "1 <= n_nu <= 8");
    if ((int)terms.size() < 1 || (int)terms.size() > EZ_TERM_MAX) return fail(EZ_ERR_INVALID_ARG, "1 <= n_terms <= 8");
    if (n_res < 1 || n_res > EZ_RES_MAX) return fail(EZ_ERR_INVALID_ARG, "1 <= n_results <= 8");
    P.d = d;
    P.n_nu = (int)nu.size();
    P.n_res = n_res;
    P.n_terms = (int)terms.size();
    for (int i = 0; i < P.n_nu; ++i) {
        const double v = nu[i];
        if (!std::isfinite(v) || std::fabs(v) > 64.0)
            return fail(EZ_ERR_INVALID_ARG, "quadrature exponents must be finite with |nu| <= 64");
        if (v != std::floor(v)) P.real_nu = 1;
    }
    for (int i = 0; i < P.n_nu; ++i) {
        double v = nu[i];
        P.nu[i] = v;
        P.preal[i] = 0.5 * (v - d + 2.0);
        P.e[i] = v - d;
        if (P.real_nu) {                 // E_p of every exponent from its own incomplete gamma
            P.p2[i] = 0;
            P.logm[i] = -1;
            if (v == std::floor(v) && (int)v - d >= 0 && ((int)v - d) % 2 == 0)
                return fail(EZ_ERR_UNSUPPORTED, "an integer exponent nu = d + 2m (logarithmic singular part) "
                                                "cannot share a call with non-integer exponents");
            continue;
        }
        P.p2[i] = (int)v - d + 2;
        int em = (int)v - d;
        P.logm[i] = (em >= 0 && em % 2 == 0) ? em / 2 : -1;
        if ((P.p2[i] & 1) == 0 && P.p2[i] / 2 >= 1) P.need_e1 = 1;
        if (P.p2[i] & 1) P.need_half = 1;
    }
    P.pset = 0;
    for (int id = 1; id < EZ_NPSETS && !P.real_nu; ++id) {
        EzPSet ps = ez_pset(id);
        if (ps.n != P.n_nu) continue;
        bool same = true;
        for (int i = 0; i < ps.n; ++i) same = same && ps.p2[i] == P.p2[i];
        if (same) { P.pset = id; break; }
    }
    for (int t = 0; t < P.n_terms; ++t) {
        const Term &T = terms[t];
        if (T.res < 0 || T.res >= n_res) return fail(EZ_ERR_INVALID_ARG, "term_result out of range");
        if (T.fac.empty() || (int)T.fac.size() > EZ_FAC_MAX) return fail(EZ_ERR_INVALID_ARG, "1 <= term_nfac <= 4");
        P.term_res[t] = T.res;
        P.term_coef[t] = T.coef;
        P.term_nfac[t] = (int)T.fac.size();
        int deg = 0;
        for (size_t f = 0; f < T.fac.size(); ++f) {
            int fi = T.fac[f].first, m = T.fac[f].second;
            if (fi < 0 || fi >= P.n_nu) return fail(EZ_ERR_INVALID_ARG, "term_fac out of range");
            if (m < 1) return fail(EZ_ERR_INVALID_ARG, "term_mult must be >= 1");
            P.term_fac[t][f] = fi;
            P.term_mult[t][f] = m;
            deg += m;
        }
        if (deg > EZ_MULT_MAX) return fail(EZ_ERR_INVALID_ARG, "total degree of a term must be <= 64");
        // expansion of the product of (singular + Taylor) factors into combinations;
        // Hadamard exponents mu = d + sum_f j_f (nu_f - d) + 2J must avoid 0 (paper, Sec. 3)
        std::vector<int> jj(T.fac.size(), 0);
        while (true) {
            double E = 0.0;
            int rest = 0, Q = 0;
            double coef = T.coef;
            for (size_t f = 0; f < T.fac.size(); ++f) {
                E += jj[f] * (P.nu[T.fac[f].first] - d);
                Q += jj[f] * (P.logm[T.fac[f].first] >= 0 ? 1 : 0);
                rest += T.fac[f].second - jj[f];
                double bn = 1.0;
                for (int q = 1; q <= jj[f]; ++q) bn = bn * (double)(T.fac[f].second - jj[f] + q) / (double)q;
                coef *= bn;
            }
            if ((int)combos.size() >= EZ_COMBO_MAX)
                return fail(EZ_ERR_UNSUPPORTED, "more than 64 expansion terms on (0, eps)");
            EzCombo cb;
            std::memset(&cb, 0, sizeof(cb));
            cb.coef = coef;
            cb.E = E;
            cb.Q = Q;
            cb.t = (signed char)t;
            cb.res = (signed char)T.res;
            for (size_t f = 0; f < T.fac.size(); ++f) cb.j[f] = (signed char)jj[f];
            combos.push_back(cb);
            int Jmax = std::min(rest * ell_max, 32);
            for (int J = 0; J <= Jmax; ++J)
                if (std::fabs(d + E + 2.0 * J) < 1e-12)
                    return fail(EZ_ERR_UNSUPPORTED, "Hadamard exponent mu + 2k = 0 (logarithmic correction not implemented)");
            size_t f = 0;
            while (f < T.fac.size()) {
                if (++jj[f] <= T.fac[f].second) break;
                jj[f] = 0;
                ++f;
            }
            if (f == T.fac.size()) break;
        }
    }
    return EZ_OK;
}

std::string plan_key(int d, int batch, const ez_quad_spec *specs, int n_specs, int ndb) {
    std::string k(reinterpret_cast<const char *>(&d), sizeof(d));
    k.append(reinterpret_cast<const char *>(&ndb), sizeof(ndb));
    k.append(reinterpret_cast<const char *>(&batch), sizeof(batch));
    k.append(reinterpret_cast<const char *>(&n_specs), sizeof(n_specs));
    k.append(reinterpret_cast<const char *>(specs), sizeof(ez_quad_spec) * (size_t)n_specs);
    return k;
}

// volume of the unit ball in d dimensions
const double kOmega[4] = {0.0, 2.0, M_PI, 4.0 * M_PI / 3.0};

// Host part of a plan: rule tables, per-lattice plans, prefixes, the persistent
// kernel's tile order, probe directions and least-squares inverses.
struct HostPlan {
    std::vector<double> rules;
    std::vector<EzInstPlan> plans;
    std::vector<int> tb, db, hb, order;
    int n_tiles = 0, n_dirs = 0, n_htiles = 0;
    int n_probe = 0, ell_probe = 0, probe_off = 0;
    int pinv_off[EZ_ELL_MAX + 1] = {0};
};

// ndb: directions per workgroup of the Hadamard direction kernel
ez_status build_host_plan(int d, int batch, const ez_quad_spec *specs, int n_specs, int ndb, HostPlan &H) {
    // rule tables: one v-rule per distinct n_q, one u-rule per distinct (n_panels, n_g, eps)
    std::vector<double> &rules = H.rules;
    rules.clear();
    std::map<int, int> vrule_of;
    std::map<std::string, int> urule_of;
    H.plans.assign(batch, EzInstPlan());
    H.tb.assign(batch + 1, 0);
    H.db.assign(batch + 1, 0);
    H.hb.assign(batch + 1, 0);
    std::vector<int> &tb = H.tb, &db = H.db, &hb = H.hb;
    long long tiles = 0, dirs = 0, htiles = 0;
    for (int b = 0; b < batch; ++b) {
        const ez_quad_spec &s = specs[n_specs == 1 ? 0 : b];
        EzInstPlan &ip = H.plans[b];
        std::memset(&ip, 0, sizeof(ip));
        ip.n_q = s.n_q;
        ip.ell = s.ell;
        ip.eps = s.eps;
        ip.lam_rel = spec_lam(s);
        int nq = (d == 1) ? 1 : s.n_q;
        if (!vrule_of.count(nq)) {
            vrule_of[nq] = (int)rules.size();
            std::vector<double> x(nq), w(nq);
            gauss_legendre(nq, 0.0, 1.0, x.data(), w.data());
            if (d == 1) { x[0] = 0.0; w[0] = 1.0; }
            rules.insert(rules.end(), x.begin(), x.end());
            rules.insert(rules.end(), w.begin(), w.end());
        }
        ip.vrule = vrule_of[nq];
        if (d == 1) ip.n_q = 1;
        std::string uk(reinterpret_cast<const char *>(&s.n_panels), sizeof(int));
        uk.append(reinterpret_cast<const char *>(&s.n_g), sizeof(int));
        uk.append(reinterpret_cast<const char *>(&s.eps), sizeof(double));
        const int n_u = s.n_panels * s.n_g;
        if (!urule_of.count(uk)) {
            urule_of[uk] = (int)rules.size();
            std::vector<double> ux(n_u), uw(n_u), gx(s.n_g), gw(s.n_g);
            const double r = std::pow(0.5 / s.eps, 1.0 / s.n_panels);
            for (int p = 0; p < s.n_panels; ++p) {
                double lo = s.eps * std::pow(r, (double)p);
                double hi = (p == s.n_panels - 1) ? 0.5 : s.eps * std::pow(r, (double)(p + 1));
                gauss_legendre(s.n_g, lo, hi, gx.data(), gw.data());
                for (int g = 0; g < s.n_g; ++g) { ux[p * s.n_g + g] = gx[g]; uw[p * s.n_g + g] = gw[g]; }
            }
            rules.insert(rules.end(), ux.begin(), ux.end());
            rules.insert(rules.end(), uw.begin(), uw.end());
        }
        ip.urule = urule_of[uk];
        ip.n_u = n_u;
        long long nd = (long long)d * (1ll << (d - 1));
        for (int i = 0; i < d - 1; ++i) nd *= s.n_q;
        ip.n_dir = (int)nd;
        // wave blocks of 64 nodes: ub consecutive u-nodes (one u-panel when n_g = 16)
        // across db = 64/ub neighbouring directions, so that each wave's k lie in a
        // small box; the shape with the fewest empty lanes, 16 x 4 on ties
        {
            const int cand[4] = {4, 3, 5, 6};     // log2 ub: 16, 8, 32, 64
            const int forced = (s.flags >> 24) & 0x7;  // EZ_SPEC_WAVE_U: 1..4 -> log2 ub = 3..6
            long long best = -1;
            for (int ci = 0; ci < 4; ++ci) {
                const int lg = (d == 1) ? 6 : (forced ? forced + 2 : cand[ci]);
                const long long ub = 1ll << lg, dbk = 64 / ub;
                const long long slots = ((n_u + ub - 1) / ub) * ub * ((nd + dbk - 1) / dbk) * dbk;
                if (best < 0 || slots < best) {
                    best = slots;
                    ip.ub_log2 = lg;
                    ip.db = (int)dbk;
                }
                if (d == 1 || forced) break;
            }
            ip.n_ublk = (n_u + (1 << ip.ub_log2) - 1) >> ip.ub_log2;
            const long long nblk = (long long)ip.n_ublk * ((nd + ip.db - 1) / ip.db);
            if (nblk > (1ll << 30)) return fail(EZ_ERR_INVALID_ARG, "quadrature too large for one call");
            ip.n_wblk = (int)nblk;
        }
        ip.tile_begin = (int)tiles;
        ip.dir_begin = (int)dirs;
        tb[b] = (int)tiles;
        db[b] = (int)dirs;
        hb[b] = (int)htiles;
        tiles += (ip.n_wblk + EZ_TILE / 64 - 1) / (EZ_TILE / 64);
        dirs += nd;
        htiles += (nd + ndb - 1) / ndb;
        if (tiles > (1ll << 30) || dirs > (1ll << 30)) return fail(EZ_ERR_INVALID_ARG, "quadrature too large for one call");
    }
    tb[batch] = (int)tiles;
    db[batch] = (int)dirs;
    hb[batch] = (int)htiles;
    // order in which the persistent node kernel takes the tiles: costliest first
    // (nodes in the tile x model cost of one node at the lattice's lam)
    std::vector<int> &order = H.order;
    order.resize((size_t)tiles);
    {
        std::vector<double> cost((size_t)tiles);
        for (int b = 0; b < batch; ++b) {
            const ez_quad_spec &s = specs[n_specs == 1 ? 0 : b];
            const EzInstPlan &ip = H.plans[b];
            const double R = std::sqrt(spec_acut(s) / M_PI), lam = spec_lam(s);
            const double per_node = kOmega[d] * (std::pow(R / lam, d) * 108.0 + 0.5 * std::pow(R * lam, d) * 14.0);
            for (int t = tb[b]; t < tb[b + 1]; ++t) {
                const long long first = (long long)(t - tb[b]) * (EZ_TILE / 64);
                cost[t] = (double)std::min<long long>(EZ_TILE / 64, ip.n_wblk - first) * 64.0 * per_node;
            }
        }
        for (size_t t = 0; t < order.size(); ++t) order[t] = (int)t;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    }
    // probe directions and least-squares inverses for the Taylor coefficients
    {
        int lp = 0;
        for (int b = 0; b < batch; ++b) lp = std::max(lp, H.plans[b].ell);
        const int np = (d == 1) ? 1 : (d == 2 ? n_mono(2, 2 * lp) + 8 : n_mono(3, 2 * lp) + 32);
        std::vector<double> probes((size_t)np * d);
        for (int p = 0; p < np; ++p) {
            if (d == 1) {
                probes[p] = 1.0;
            } else if (d == 2) {
                const double th = M_PI * (p + 0.5) / np;
                probes[2 * p] = std::cos(th);
                probes[2 * p + 1] = std::sin(th);
            } else {          // Fibonacci points on the unit sphere
                const double z = 1.0 - 2.0 * (p + 0.5) / np, r = std::sqrt(1.0 - z * z);
                const double th = M_PI * (1.0 + std::sqrt(5.0)) * (p + 0.5);
                probes[3 * p] = r * std::cos(th);
                probes[3 * p + 1] = r * std::sin(th);
                probes[3 * p + 2] = z;
            }
        }
        H.n_probe = np;
        H.ell_probe = lp;
        H.probe_off = (int)rules.size();
        rules.insert(rules.end(), probes.begin(), probes.end());
        std::vector<double> mono, Mk, pinv;
        for (int k = 0; k <= lp; ++k) {
            const int nm = n_mono(d, 2 * k);
            Mk.assign((size_t)np * nm, 0.0);
            for (int p = 0; p < np; ++p) {
                monomials(d, 2 * k, &probes[(size_t)p * d], mono);
                for (int a = 0; a < nm; ++a) Mk[(size_t)p * nm + a] = mono[a];
            }
            lstsq_pinv(np, nm, Mk, pinv);
            H.pinv_off[k] = (int)rules.size();
            rules.insert(rules.end(), pinv.begin(), pinv.end());
        }
    }
    H.n_tiles = (int)tiles;
    H.n_dirs = (int)dirs;
    H.n_htiles = (int)htiles;
    return EZ_OK;
}

void fill_plan_view(const HostPlan &H, PlanView &v) {
    v.n_tiles = H.n_tiles;
    v.n_dirs = H.n_dirs;
    v.n_htiles = H.n_htiles;
    v.n_probe = H.n_probe;
    v.ell_probe = H.ell_probe;
    v.probe_off = H.probe_off;
    for (int k = 0; k <= EZ_ELL_MAX; ++k) v.pinv_off[k] = H.pinv_off[k];
}

// Quadrature plans are cached per device, at most EZ_PLAN_CACHE of them; evicting
// one frees its buffers and bumps the workspace generation.
#define EZ_PLAN_CACHE 128
ez_status get_plan(DeviceState *S, int d, int batch, const ez_quad_spec *specs, int n_specs, int ndb, DevPlan **out) {
    std::string key = plan_key(d, batch, specs, n_specs, ndb);
    auto it = S->plans.find(key);
    if (it != S->plans.end()) {
        // least recently used order: a hit moves the key to the back
        auto pos = std::find(S->plan_order.begin(), S->plan_order.end(), key);
        if (pos != S->plan_order.end() && pos + 1 != S->plan_order.end()) {
            S->plan_order.erase(pos);
            S->plan_order.push_back(key);
        }
        *out = it->second;
        return EZ_OK;
    }
    HostPlan H;
    ez_status st = build_host_plan(d, batch, specs, n_specs, ndb, H);
    if (st) return st;
    DevPlan *P = new DevPlan();
    P->host_plans = H.plans;
    P->n_tiles = H.n_tiles;
    P->n_dirs = H.n_dirs;
    P->n_htiles = H.n_htiles;
    P->n_probe = H.n_probe;
    P->ell_probe = H.ell_probe;
    P->probe_off = H.probe_off;
    for (int k = 0; k <= EZ_ELL_MAX; ++k) P->pinv_off[k] = H.pinv_off[k];
    if ((st = grow(P->rules, H.rules.size() * sizeof(double))) ||
        (st = grow(P->plans, sizeof(EzInstPlan) * batch)) ||
        (st = grow(P->tile_begin, sizeof(int) * (batch + 1))) ||
        (st = grow(P->dir_begin, sizeof(int) * (batch + 1))) ||
        (st = grow(P->htile_begin, sizeof(int) * (batch + 1))) ||
        (st = grow(P->tile_order, sizeof(int) * std::max<size_t>(1, H.order.size())))) {
        free_plan(P);
        return st;
    }
    // one-time synchronous uploads (plans are cached and reused)
    if (hipMemcpy(P->rules.p, H.rules.data(), H.rules.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->plans.p, H.plans.data(), sizeof(EzInstPlan) * batch, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->tile_begin.p, H.tb.data(), sizeof(int) * (batch + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->dir_begin.p, H.db.data(), sizeof(int) * (batch + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->htile_begin.p, H.hb.data(), sizeof(int) * (batch + 1), hipMemcpyHostToDevice) != hipSuccess ||
        (!H.order.empty() &&
         hipMemcpy(P->tile_order.p, H.order.data(), sizeof(int) * H.order.size(), hipMemcpyHostToDevice) != hipSuccess)) {
        free_plan(P);
        return fail(EZ_ERR_HIP, "upload of the quadrature plan failed");
    }
    if (S->plans.size() >= EZ_PLAN_CACHE) {      // bounded cache, least recently used out
        std::string old = S->plan_order.front();
        S->plan_order.erase(S->plan_order.begin());
        free_plan(S->plans[old]);
        S->plans.erase(old);
    }
    S->plans[key] = P;
    S->plan_order.push_back(key);
    *out = P;
    return EZ_OK;
}

const double kSkew = 2.5;   // bound on (1/2) sum |a_i| / V^{1/d} assumed for table capacity

// 1/Gamma(x), zero at the poles
double rgamma_host(double x) { return (x <= 0.0 && x == std::floor(x)) ? 0.0 : 1.0 / std::tgamma(x); }

// lattice-independent factors of the per-exponent constants of the split: the
// reciprocal prefactor pi^{nu-d/2}/Gamma(nu/2) (times alpha^{(d-nu)/2}/V on the
// device), the self-term factor 1/Gamma(nu/2+1), and V times the coefficient of
// the singular part |k|^{nu-d}: Gamma((d-nu)/2) pi^{nu-d/2}/Gamma(nu/2), or for
// nu = d + 2m the coefficient of |k|^{2m} log(pi |k|^2),
// (-1)^{m+1} pi^{2m+d/2} / (Gamma(m+d/2) m!)
void fill_nu_constants(const EzProgram &prog, EzSetupArgs &sa) {
    std::memset(sa.nuc, 0, sizeof(sa.nuc));
    const double d = (double)prog.d;
    for (int i = 0; i < prog.n_nu; ++i) {
        const double nu = prog.nu[i];
        const double rg = rgamma_host(0.5 * nu);
        const double c0 = std::pow(M_PI, nu - 0.5 * d) * rg;
        sa.nuc[i][0] = c0;
        sa.nuc[i][1] = rgamma_host(0.5 * nu + 1.0);
        const int m = prog.logm[i];
        if (m >= 0) {
            double mf = 1.0;
            for (int j = 2; j <= m; ++j) mf *= (double)j;
            sa.nuc[i][2] = std::pow(M_PI, 2.0 * m + 0.5 * d) * rgamma_host(m + 0.5 * d) *
                           (((m + 1) & 1) ? -1.0 : 1.0) / mf;
        } else {
            sa.nuc[i][2] = c0 * std::tgamma(0.5 * (d - nu));
        }
        sa.nuc[i][3] = rg;
    }
}

int real_capacity(int d, double lam, double acut, bool general) {
    double R = lam * std::sqrt(acut / M_PI) + (general ? kSkew : 0.0);
    double n = kOmega[d] * std::pow(R + kSkew, d);
    return (int)std::ceil(general ? n : 0.5 * n) + 16;
}
int rec_capacity(int d, double lam, double acut) {
    double R = std::sqrt(acut / M_PI) / lam + kSkew;
    return (int)std::ceil(kOmega[d] * std::pow(R + kSkew, d)) + 16;
}

// What one lattice-sum call needs besides its plan: checked options, the table
// capacities and the sizes that follow from them (no allocation, no launch).
struct CallInfo {
    bool grad = false;
    int ndb = 0, n_ch = 1, maxdeg = 0, flags = 0;
    double acut = 36.0;
    EzTables tab;
    // mixed precision: requested, and active (FP32 far field in the node kernel)
    bool mixed = false, mixed_active = false;
    double a_mix = 16.0;
    int top2[2] = {-1, -1};
    double eps[EZ_NU_MAX] = {0.0};
    // tail tiles [n_main, n_tiles) taken as two half-tile workgroups each by the tile kernel
    bool tail_halves = false;
};

// Relative error bound of one FP32 chunk sum of the far field, per exponent, first
// order in u = 2^-24 (the terms of a chunk are positive):
//   e^{-a}: the fraction x - n rounded to FP32 (0.35 u), v_exp_f32 (1 u): 2 u;
//   t = 1/a: a rounded to FP32 (0.5 u), v_rcp_f32 (1 u): 1.5 u;  e^{-a} t: 0.5 u;
//   the fit at a chain's top: its error with FP32 coefficients (EZ_EPF_FIT_ERR) plus
//   Horner of degree 3 with positive terms in P and Q (6 u each), v_rcp_f32 and the
//   product (1.5 u), and the product with e^{-a} t (0.5 u);
//   a downward step E_{p-1} = fma(-(p-1), E_p, e^{-a}) t: with r = (p-1)/a_mix >=
//   (p-1) E_p / e^{-a} (E_p <= e^{-a}/a for p >= 0), the difference carries
//   (2 u + r e_p)/(1 - r) + 0.5 u when p - 1 > 0 and max(2 u, e_p) + 0.5 u otherwise,
//   then t and the product add 2 u;
//   the FP32 sum of at most 64 terms: 63 u;
// and 1% for the second-order terms.
void mixed_bounds(const EzProgram &prog, double a_mix, const int *top2, double *eps) {
    const double u = std::ldexp(1.0, -24);
    const double e_ex = 2.0, e_t = 1.5, e_fit = EZ_EPF_FIT_ERR / u + 13.5;
    for (int i = 0; i < EZ_NU_MAX; ++i) eps[i] = 0.0;
    for (int i = 0; i < prog.n_nu; ++i) {
        const int p2 = prog.p2[i];
        const int odd = p2 & 1;
        const int top = top2[odd];
        double e = e_ex + e_t + 0.5;
        if (top >= (odd ? 1 : 2)) e += e_fit + 0.5;
        for (int q2 = top; q2 > p2; q2 -= 2) {
            const double q = 0.5 * (q2 - 2);
            double eD;
            if (q > 0.0) {
                const double r = q / a_mix;
                eD = (e_ex + r * e) / (1.0 - r) + 0.5;
            } else {
                eD = std::max(e_ex, e) + 0.5;
            }
            e = eD + e_t + 0.5;
        }
        eps[i] = 1.01 * (e + 63.0) * u;
    }
}

ez_status prepare_call(int batch, int d, const EzProgram &prog, const std::vector<EzCombo> &combos,
                       const ez_quad_spec *specs, int n_specs, bool grad, CallInfo &C) {
    (void)batch; (void)d;
    if (combos.size() < 2) return fail(EZ_ERR_INVALID_ARG, "internal: expansion with fewer than 2 terms");
    C.grad = grad;
    if (grad && prog.n_res > EZ_GRAD_RES_MAX)
        return fail(EZ_ERR_INVALID_ARG, "derivatives are available for at most 2 results per call");
    // 64 directions per direction workgroup (one per lane, the combinations shared out
    // over its waves), values and derivatives alike
    C.ndb = EZ_HDIR;
    C.n_ch = grad ? 1 + d * (d + 1) / 2 : 1;
    int ell_max = 0;
    for (int i = 0; i < n_specs; ++i) ell_max = std::max(ell_max, specs[i].ell);
    C.maxdeg = 0;          // highest power of u^2 in the (0, eps) product polynomials
    for (const EzCombo &cb : combos) {
        int rest = 0;
        for (int f = 0; f < prog.term_nfac[cb.t]; ++f) rest += prog.term_mult[cb.t][f] - cb.j[f];
        C.maxdeg = std::max(C.maxdeg, rest * ell_max);
    }
    // the product polynomials on (0, eps) keep powers up to u^64: a dropped power u^{2K},
    // K > 32, integrates to a part of relative size below (C eps^2)^33 with C the
    // ratio of successive Taylor coefficients (below 1e-40 at eps = 1e-2 for the
    // lattices here), so many-factor products (n up to 64) are truncated there
    C.maxdeg = std::min(C.maxdeg, 32);
    C.flags = specs[0].flags;
    for (int i = 1; i < n_specs; ++i)
        if (specs[i].flags != C.flags) return fail(EZ_ERR_INVALID_ARG, "all specs of one call must share flags");
    C.mixed = specs[0].precision == EZ_PREC_MIXED;
    for (int i = 1; i < n_specs; ++i)
        if ((specs[i].precision == EZ_PREC_MIXED) != C.mixed)
            return fail(EZ_ERR_INVALID_ARG, "all specs of one call must share the precision");
    if (C.mixed && grad) return fail(EZ_ERR_UNSUPPORTED, "derivatives are computed in FP64 only (EZ_PREC_FP64)");
    double lam_min = 1e300, lam_max = 0.0;
    C.acut = spec_acut(specs[0]);
    for (int i = 0; i < n_specs; ++i) {
        lam_min = std::min(lam_min, spec_lam(specs[i]));
        lam_max = std::max(lam_max, spec_lam(specs[i]));
        if (spec_acut(specs[i]) != C.acut) return fail(EZ_ERR_INVALID_ARG, "all specs of one call must share a_cut");
    }
    C.tab.real_cap = real_capacity(d, lam_max, C.acut, false);
    C.tab.rec_cap = rec_capacity(d, lam_min, C.acut);
    if (C.tab.rec_cap > EZ_KCULL)
        return fail(EZ_ERR_UNSUPPORTED, "reciprocal table too large for this lam and a_cut (raise spec.lam)");
    C.tab.rstride = 4 * ((3 + (grad ? 2 : 1) * prog.n_nu + 3) / 4);
    C.tab.row_cap = C.tab.real_cap;
    if (C.mixed) {
        // the FP32 far field needs the fits of every chain top (2p <= EZ_EPF_P2MAX) and
        // e^{-a} well inside the FP32 range (a_cut <= 80); otherwise the call stays FP64
        const int amix = (C.flags >> 16) & 0xFF;
        C.a_mix = amix ? (double)amix : 16.0;
        for (int i = 0; i < prog.n_nu; ++i) {
            const int odd = prog.p2[i] & 1;
            C.top2[odd] = std::max(C.top2[odd], std::max(prog.p2[i], odd));
        }
        C.mixed_active = !prog.real_nu && C.top2[0] <= EZ_EPF_P2MAX && C.top2[1] <= EZ_EPF_P2MAX &&
                         C.acut <= 80.0 && C.a_mix < C.acut;
        if (C.mixed_active) mixed_bounds(prog, C.a_mix, C.top2, C.eps);
    }
    return EZ_OK;
}

// Workspace of one call: the buffers the kernels write and read back.
enum WsSlot {
    WS_META, WS_SUB_PART, WS_TAIL_ACC, WS_REAL, WS_RN, WS_ROWS, WS_REC, WS_TILE_PART, WS_DIR_PART, WS_DIR_FLAG,
    WS_PROBE_VAL, WS_TENSOR, WS_TILE_GRAD, WS_DIR_GRAD, WS_TAIL_CNT, WS_QUEUE, WS_TILE_BOUND, WS_COUNT
};

struct Workspace {
    size_t bytes[WS_COUNT];
    void *ptr[WS_COUNT];
};

int probe_slices(int batch, int n_probe) {
    const int n_pblk = (n_probe + 63) / 64;
    return std::max(1, std::min(EZ_SLICE_MAX, 512 / std::max(1, batch * n_pblk)));
}

// The tail of the tile kernel: with round = the tile-kernel workgroups resident on the
// device at once, the last n_tiles % round tiles form a partly filled last round.
//  - A few tiles (16 split-kernel workgroups per tile fit one per CU): they go to the
//    split kernel, launched after the tile kernel with one workgroup per CU; each
//    64-node group is shared by 16 waves of four workgroups.
//  - Up to about half a round: the tile kernel takes each of them as two workgroups of
//    half the terms (C.tail_halves), so that the last round runs at the occupancy of
//    the others (three-lattice ATM call, 3087 tiles over rounds of 2048).
//  - More: the tile kernel as it is.
// Value calls only, without EZ_SPEC_NO_SPLIT; the persistent schedule takes no halves,
// mixed-precision calls no split kernel.
int main_tiles(CallInfo &C, const EzProgram &prog, int n_cu, int n_tiles) {
    int round = 0;                     // tile-kernel workgroups resident on the device at once
    {
        EzQuadArgs probe_args;
        std::memset(&probe_args, 0, sizeof(probe_args));
        probe_args.prog = prog;
        round = n_cu * ez_nodes_tile_blocks_per_cu(probe_args);
    }
    int n_main = n_tiles;
    C.tail_halves = false;
    if (!C.grad && !prog.real_nu && !(C.flags & EZ_SPEC_NO_SPLIT)) {
        const int tail = round > 0 ? n_tiles % round : 0;
        const int per_tile = (EZ_TILE / 64) * EZ_TAIL_PARTS;     // split-kernel workgroups per tail tile
        if (n_tiles > round && tail > 0) {
            if (tail * per_tile <= n_cu) {
                if (!C.mixed_active) n_main = n_tiles - tail;     // the split kernel is FP64 only
            } else if (!(C.flags & EZ_SPEC_PERSISTENT) && 2 * tail <= round + round / 4) {
                n_main = n_tiles - tail;
                C.tail_halves = true;
            }
        }
    }
    return n_main;
}

// the node tiles of a lattice-sum call and its tail, for ez_last_sum_tiles
void note_tiles(DeviceState *S, const CallInfo &C, int n_tiles, int n_main) {
    S->sum_tiles = n_tiles;
    S->sum_main = n_main;
    S->sum_tail = n_main == n_tiles ? 0 : (C.tail_halves ? 2 : 1);
}

void workspace_sizes(int batch, const EzProgram &prog, const CallInfo &C, const PlanView &P, int n_main, Workspace &W) {
    const size_t ntail = (size_t)std::max(1, P.n_tiles - n_main);
    // the split kernel's part sums and counters (half-tile tails combine in LDS)
    const size_t nsplit = C.tail_halves ? 1 : ntail;
    const int n_slice = probe_slices(batch, P.n_probe);
    W.bytes[WS_META] = sizeof(EzLatMeta) * batch;
    W.bytes[WS_SUB_PART] = sizeof(double) * 2 * (EZ_TILE / 64) * ntail * prog.n_res;
    W.bytes[WS_TAIL_ACC] = sizeof(double) * (EZ_TILE / 64) * EZ_TAIL_PARTS * 2 * 64 * nsplit * prog.n_nu;
    W.bytes[WS_REAL] = sizeof(double) * (size_t)batch * C.tab.real_cap * C.tab.rstride;
    W.bytes[WS_RN] = sizeof(int) * 4 * (size_t)batch * C.tab.real_cap;
    W.bytes[WS_ROWS] = sizeof(int) * 8 * (size_t)batch * C.tab.row_cap;
    W.bytes[WS_REC] = sizeof(double) * (size_t)batch * C.tab.rec_cap * 4;
    W.bytes[WS_TILE_PART] = sizeof(double) * 2 * (size_t)P.n_tiles * prog.n_res;
    W.bytes[WS_DIR_PART] = sizeof(double) * (size_t)P.n_dirs * prog.n_res;
    W.bytes[WS_DIR_FLAG] = sizeof(uint32_t) * (size_t)P.n_dirs;
    W.bytes[WS_PROBE_VAL] =
        sizeof(double) * (size_t)batch * n_slice * P.n_probe * C.n_ch * prog.n_nu * (EZ_ELL_MAX + 1);
    W.bytes[WS_TENSOR] = sizeof(double) * (size_t)batch * C.n_ch * prog.n_nu * EZ_TDIM;
    W.bytes[WS_TILE_GRAD] = C.grad ? sizeof(double) * 12 * (size_t)P.n_tiles * prog.n_res : 0;
    W.bytes[WS_DIR_GRAD] = C.grad ? sizeof(double) * 6 * (size_t)P.n_dirs * prog.n_res : 0;
    W.bytes[WS_TAIL_CNT] = sizeof(int) * (EZ_TILE / 64) * nsplit;
    W.bytes[WS_QUEUE] = 256;
    // mixed calls: one bound per tile, and one more per tail tile taken in halves
    W.bytes[WS_TILE_BOUND] =
        C.mixed_active ? sizeof(double) * ((size_t)P.n_tiles + (C.tail_halves ? ntail : 0)) * prog.n_res : 0;
    for (int i = 0; i < WS_COUNT; ++i) W.ptr[i] = nullptr;
}

// The launch sequence of one lattice-sum call: setup, Taylor/Hadamard branch,
// node kernels, finalize.  `side` (may be NULL) is the second stream for the
// Hadamard branch with its two events; without it, or with EZ_SPEC_SERIAL, the
// whole branch runs on `stream` before the nodes.  tail_cnt must hold zeros.
ez_status enqueue_sums(int batch, const double *A_dev, const EzProgram &prog, const std::vector<EzCombo> &combos,
                       const CallInfo &C, const PlanView &P, int n_main, int n_cu, const Workspace &W,
                       double *out_dev, uint32_t *status_dev, double *grad_dev, hipStream_t stream, hipStream_t side,
                       hipEvent_t ev_setup, hipEvent_t ev_had, bool timing_ok = true, double *bound_dev = nullptr,
                       StreamSignals *sig = nullptr) {
    const bool grad = C.grad;
    // the timing hooks create events; the no-allocation entry point launches without them
    auto tm = [&](int kernel, hipStream_t st, auto launch) { return timing_ok ? timed(kernel, st, launch) : launch(); };
    EzTables tab = C.tab;
    tab.real = (double *)W.ptr[WS_REAL];
    tab.rn = (int *)W.ptr[WS_RN];
    tab.rows = (int *)W.ptr[WS_ROWS];
    tab.rec = (double *)W.ptr[WS_REC];

    EzSetupArgs sa;
    sa.prog = prog;
    sa.A = A_dev;
    sa.plans = P.plans;
    sa.meta = (EzLatMeta *)W.ptr[WS_META];
    sa.tab = tab;
    sa.a_cut = C.acut;
    sa.general_x = 0;
    sa.grad = grad ? 1 : 0;
    sa.status_out = nullptr;
    fill_nu_constants(prog, sa);
    const bool two = side && !(C.flags & EZ_SPEC_SERIAL);
    // Derivative calls keep the (seven-channel) probe and the tensor kernel on the
    // caller's stream before the adjoint node kernel unless the batch's tiles fill
    // more than eight rounds of the device (throughput-bound: the 4096-lattice scan).
    int round = 0;
    {
        EzQuadArgs probe_args;
        std::memset(&probe_args, 0, sizeof(probe_args));
        probe_args.prog = prog;
        round = n_cu * ez_nodes_tile_blocks_per_cu(probe_args);
    }
    // Value calls whose tiles fill at most eight rounds swap the streams: the Hadamard
    // branch on the caller's stream right behind the setup, so that its probe kernel is
    // dispatched before the node kernel fills the device, and the node kernels on the
    // second stream (three-lattice ATM call: the branch no longer ends after the nodes)
    const bool swap = two && !grad && P.n_tiles <= 8 * round;
    const bool big = two && !swap && (!grad || P.n_tiles > 8 * round);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    EZ_HIP_TRY(hipStreamIsCapturing(stream, &cap));
    // the fork event after the setup is recorded by the setup launch itself (no marker
    // packet between the setup and the node kernel), or by hipEventRecord under capture
    // small value calls outside capture join the streams at the end with a value wait
    // (the setup edge stays an event recorded by the setup launch: a value write there
    // is a runtime kernel that would hold the probe back behind the setup)
    const bool use_sig = swap && sig && sig->ok && cap == hipStreamCaptureStatusNone;
    const bool ext_setup = (big || swap) && cap == hipStreamCaptureStatusNone;
    EZ_HIP_TRY(tm(EZ_KERNEL_SETUP, stream,
                  [&] { return ez_launch_setup(sa, batch, stream, ext_setup ? ev_setup : nullptr); }));

    EzQuadArgs qa;
    qa.prog = prog;
    qa.batch = batch;
    qa.plans = P.plans;
    qa.tile_begin = P.tile_begin;
    qa.dir_begin = P.dir_begin;
    qa.htile_begin = P.htile_begin;
    qa.n_dir_blk = C.ndb;
    qa.poly_deg = C.maxdeg <= 12 ? 13 : 33;
    qa.n_slice = probe_slices(batch, P.n_probe);
    qa.n_ch = C.n_ch;
    qa.n_probe = P.n_probe;
    qa.ell_probe = P.ell_probe;
    qa.probe_off = P.probe_off;
    for (int k = 0; k <= EZ_ELL_MAX; ++k) qa.pinv_off[k] = P.pinv_off[k];
    qa.probe_val = (double *)W.ptr[WS_PROBE_VAL];
    qa.tensor = (double *)W.ptr[WS_TENSOR];
    qa.n_combo = (int)combos.size();
    for (size_t c = 0; c < combos.size(); ++c) qa.combo[c] = combos[c];
    qa.meta = (const EzLatMeta *)W.ptr[WS_META];
    qa.tab = tab;
    qa.rules = P.rules;
    qa.tile_part = (double *)W.ptr[WS_TILE_PART];
    qa.mixed = C.mixed_active ? 1 : 0;
    qa.a_mix = C.a_mix;
    qa.mix_top2[0] = C.top2[0];
    qa.mix_top2[1] = C.top2[1];
    for (int i = 0; i < EZ_NU_MAX; ++i) qa.mix_eps[i] = C.eps[i];
    qa.tile_bound = (double *)W.ptr[WS_TILE_BOUND];
    qa.bound_out = bound_dev;
    qa.dir_part = (double *)W.ptr[WS_DIR_PART];
    qa.dir_flag = (uint32_t *)W.ptr[WS_DIR_FLAG];
    qa.out = out_dev;
    qa.status = status_dev;
    qa.tile_grad = grad ? (double *)W.ptr[WS_TILE_GRAD] : nullptr;
    qa.dir_grad = grad ? (double *)W.ptr[WS_DIR_GRAD] : nullptr;
    qa.grad_out = grad_dev;
    qa.n_tiles = P.n_tiles;
    qa.n_main = n_main;
    qa.tail_halves = C.tail_halves ? 1 : 0;
    qa.sub_part = (double *)W.ptr[WS_SUB_PART];
    qa.tail_acc = (double *)W.ptr[WS_TAIL_ACC];
    qa.tail_cnt = (int *)W.ptr[WS_TAIL_CNT];
    qa.tile_order = P.tile_order;
    qa.queue = (int *)W.ptr[WS_QUEUE];

    // The Taylor/Hadamard branch depends only on the setup.  Its probe, tensor and
    // direction kernels run concurrently with the node kernel on the other stream:
    // they take the workgroup slots that the node kernel leaves free.  Small value
    // calls (`swap`) keep the branch on the caller's stream and put the nodes on the
    // second one; the probe, queued right behind the setup, then starts before the
    // node kernel fills the device (three-lattice ATM call, 263424 nodes each: 0.2458
    // ms per step against 0.2489 ms with the nodes on the caller's stream, where the
    // probe waited for the node kernel's drain and the branch ended after the nodes).
    // Large scans and derivative calls keep the nodes on the caller's stream.  The
    // caller's stream joins the other before the final reduction (event edges, so the
    // sequence can be captured into a graph).  EZ_SPEC_SERIAL keeps everything on
    // `stream`.
    auto had = [&](hipStream_t s, int part, hipEvent_t done) {
        return grad ? ez_launch_hadamard_adj(qa, P.n_htiles, s, part, done)
                    : ez_launch_hadamard(qa, P.n_htiles, s, part, done);
    };
    // The fork event is recorded by the tensor launch itself (no marker packet between
    // the tensors and the node kernel), or by hipEventRecord while the stream is captured.
    // With derivatives the direction kernel only gets slots as the adjoint node kernel
    // drains, and runs beside its last, partly filled round of tiles (three-lattice ATM
    // derivative, 263424 nodes each: 0.869 ms per step, 0.901 ms with the direction
    // kernel before the nodes).
    hipStream_t hs = stream;                      // the Hadamard branch
    hipStream_t ns = stream;                      // the node kernels
    if (swap) {
        if (!ext_setup) EZ_HIP_TRY(hipEventRecord(ev_setup, stream));
        EZ_HIP_TRY(hipStreamWaitEvent(side, ev_setup, 0));
        ns = side;
        EZ_HIP_TRY(tm(EZ_KERNEL_TAYLOR, stream, [&] { return had(stream, EZ_HAD_PRE, nullptr); }));
    } else if (big) {
        if (!ext_setup) EZ_HIP_TRY(hipEventRecord(ev_setup, stream));
        EZ_HIP_TRY(hipStreamWaitEvent(side, ev_setup, 0));
        hs = side;
        EZ_HIP_TRY(tm(EZ_KERNEL_TAYLOR, hs, [&] { return had(hs, EZ_HAD_PRE, nullptr); }));
    } else {
        const bool ext = two && cap == hipStreamCaptureStatusNone;
        EZ_HIP_TRY(tm(EZ_KERNEL_TAYLOR, stream, [&] { return had(stream, EZ_HAD_PRE, ext ? ev_setup : nullptr); }));
        if (two) {
            if (!ext) EZ_HIP_TRY(hipEventRecord(ev_setup, stream));
            EZ_HIP_TRY(hipStreamWaitEvent(side, ev_setup, 0));
            hs = side;
        }
    }
    EZ_HIP_TRY(tm(EZ_KERNEL_HADAMARD, hs, [&] { return had(hs, EZ_HAD_DIR, nullptr); }));
    if (grad) {
        EZ_HIP_TRY(tm(EZ_KERNEL_NODES_ADJ, ns, [&] { return ez_launch_nodes_adj(qa, P.n_tiles, ns); }));
    } else if ((C.flags & EZ_SPEC_PERSISTENT) && !C.mixed_active && !prog.real_nu) {
        int bpc = (C.flags >> 8) & 0xFF;
        if (bpc == 0) bpc = ez_nodes_blocks_per_cu(qa);
        const int nblk = std::max(1, std::min(P.n_tiles, n_cu * bpc));
        EZ_HIP_TRY(ez_launch_fill_int(qa.queue, 1, 0, ns));
        EZ_HIP_TRY(tm(EZ_KERNEL_NODES, ns, [&] { return ez_launch_nodes_persistent(qa, nblk, ns); }));
    } else {
        const int n_wg = C.tail_halves ? n_main + 2 * (P.n_tiles - n_main) : n_main;
        EZ_HIP_TRY(tm(EZ_KERNEL_NODES, ns, [&] { return ez_launch_nodes(qa, n_wg, ns); }));
    }
    if (n_main < P.n_tiles && !C.tail_halves)
        EZ_HIP_TRY(tm(EZ_KERNEL_NODES_TAIL, ns, [&] { return ez_launch_nodes_split(qa, ns); }));
    // join the second stream before the final reduction
    if (use_sig) {
        const uint64_t v = sig->seq[1] + 1;
        EZ_HIP_TRY(hipStreamWriteValue64(ns, sig->p[1], v, 0));
        sig->seq[1] = v;
        EZ_HIP_TRY(hipStreamWaitValue64(stream, sig->p[1], v, hipStreamWaitValueGte, ~0ull));
    } else if (hs != stream || ns != stream) {
        EZ_HIP_TRY(hipEventRecord(ev_had, hs != stream ? hs : ns));
        EZ_HIP_TRY(hipStreamWaitEvent(stream, ev_had, 0));
    }
    EZ_HIP_TRY(tm(EZ_KERNEL_FINALIZE, stream, [&] { return ez_launch_finalize(qa, stream); }));
    return EZ_OK;
}

// grad_dev (may be NULL): batch x n_res x d x d derivatives of the results with respect to A
ez_status run_sums(int batch, int d, const double *A_dev, const EzProgram &prog, const std::vector<EzCombo> &combos,
                   const ez_quad_spec *specs, int n_specs, double *out_dev, uint32_t *status_dev, hipStream_t stream,
                   double *grad_dev = nullptr, double *bound_dev = nullptr) {
    int dev = 0;
    EZ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState *S = device_state(dev);
    CallInfo C;
    ez_status st = prepare_call(batch, d, prog, combos, specs, n_specs, grad_dev != nullptr, C);
    if (st) return st;
    DevPlan *P = nullptr;
    if ((st = get_plan(S, d, batch, specs, n_specs, C.ndb, &P))) return st;
    if (!S->side) {
        EZ_HIP_TRY(hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking));
        EZ_HIP_TRY(hipEventCreate(&S->ev_setup));     // recorded by a kernel launch (needs timing)
        EZ_HIP_TRY(hipEventCreateWithFlags(&S->ev_had, hipEventDisableTiming));
        EZ_HIP_TRY(hipDeviceGetAttribute(&S->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        // the signal words, zeroed once (outside capture only: otherwise the calls keep events)
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        int can = 0;
        if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
            hipDeviceGetAttribute(&can, hipDeviceAttributeCanUseStreamWaitValue, dev) == hipSuccess && can) {
            bool good = true;
            for (int i = 0; i < 2 && good; ++i) {
                void *w = nullptr;
                good = hipExtMallocWithFlags(&w, 8, hipMallocSignalMemory) == hipSuccess;
                if (good) {
                    S->sig.p[i] = (uint64_t *)w;
                    good = hipMemset(w, 0, 8) == hipSuccess;
                }
            }
            if (good) good = hipDeviceSynchronize() == hipSuccess;
            S->sig.ok = good;
            if (!good) (void)hipGetLastError();
        }
    }
    PlanView pv;
    pv.rules = (const double *)P->rules.p;
    pv.plans = (const EzInstPlan *)P->plans.p;
    pv.tile_begin = (const int *)P->tile_begin.p;
    pv.dir_begin = (const int *)P->dir_begin.p;
    pv.htile_begin = (const int *)P->htile_begin.p;
    pv.tile_order = (const int *)P->tile_order.p;
    pv.n_tiles = P->n_tiles;
    pv.n_dirs = P->n_dirs;
    pv.n_htiles = P->n_htiles;
    pv.n_probe = P->n_probe;
    pv.ell_probe = P->ell_probe;
    pv.probe_off = P->probe_off;
    for (int k = 0; k <= EZ_ELL_MAX; ++k) pv.pinv_off[k] = P->pinv_off[k];
    const int n_main = main_tiles(C, prog, S->n_cu, P->n_tiles);
    note_tiles(S, C, P->n_tiles, n_main);
    Workspace W;
    workspace_sizes(batch, prog, C, pv, n_main, W);
    DevBuf *bufs[WS_COUNT] = {&S->meta, &S->sub_part, &S->tail_acc, &S->real, &S->rn, &S->rows, &S->rec,
                              &S->tile_part, &S->dir_part, &S->dir_flag, &S->probe_val, &S->tensor,
                              &S->tile_grad, &S->dir_grad, &S->tail_cnt, &S->queue, &S->tile_bound};
    for (int i = 0; i < WS_COUNT; ++i) {
        if (W.bytes[i] == 0) continue;
        const size_t had = bufs[i]->bytes;
        if ((st = grow(*bufs[i], W.bytes[i]))) return st;
        W.ptr[i] = bufs[i]->p;
        // the tail group counters are zero between calls: zeroed when allocated,
        // then reset by the kernel that uses them
        if (i == WS_TAIL_CNT && bufs[i]->bytes != had)
            EZ_HIP_TRY(ez_launch_fill_int((int *)bufs[i]->p, (int)(bufs[i]->bytes / sizeof(int)), 0, stream));
    }
    return enqueue_sums(batch, A_dev, prog, combos, C, pv, n_main, S->n_cu, W, out_dev, status_dev, grad_dev, stream,
                        S->side, S->ev_setup, S->ev_had, true, bound_dev, &S->sig);
}

// tables of one lattice for general shifts x (every z, every m*, no weights)
ez_status general_setup(DeviceState *S, int d, const double *A_dev, double lam, double a_cut, uint32_t *status_dev,
                        hipStream_t s, EzTables *tab_out) {
    EzProgram prog;
    std::memset(&prog, 0, sizeof(prog));
    prog.d = d;
    prog.n_nu = 0;   // general-x tables carry no weights
    EzTables tab;
    tab.real_cap = real_capacity(d, lam, a_cut, true);
    tab.rec_cap = rec_capacity(d, lam, a_cut);
    tab.rstride = 4;
    tab.row_cap = 0;
    tab.rn = nullptr;
    tab.rows = nullptr;
    ez_status st;
    if ((st = grow(S->gmeta, sizeof(EzLatMeta))) ||
        (st = grow(S->greal, sizeof(double) * (size_t)tab.real_cap * tab.rstride)) ||
        (st = grow(S->grec, sizeof(double) * (size_t)tab.rec_cap * 4)))
        return st;
    tab.real = (double *)S->greal.p;
    tab.rec = (double *)S->grec.p;
    // a one-lattice plan carrying lam
    ez_quad_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.n_q = 1; sp.n_panels = 1; sp.n_g = 1; sp.ell = 0; sp.eps = 0.01; sp.lam = lam; sp.a_cut = a_cut;
    DevPlan *P = nullptr;
    if ((st = get_plan(S, d, 1, &sp, 1, 256, &P))) return st;
    EzSetupArgs sa;
    sa.prog = prog;
    sa.A = A_dev;
    sa.plans = (const EzInstPlan *)P->plans.p;
    sa.meta = (EzLatMeta *)S->gmeta.p;
    sa.tab = tab;
    sa.a_cut = a_cut;
    sa.general_x = 1;
    sa.grad = 0;
    sa.status_out = status_dev;
    fill_nu_constants(prog, sa);
    EZ_HIP_TRY(timed(EZ_KERNEL_SETUP, s, [&] { return ez_launch_setup(sa, 1, s); }));
    *tab_out = tab;
    return EZ_OK;
}

ez_status check_common(int batch, int d, const double *A_dev, const ez_quad_spec *spec, const void *out) {
    if (d < 1 || d > 3) return fail(EZ_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (batch < 1) return fail(EZ_ERR_INVALID_ARG, "batch must be >= 1");
    if (!A_dev || !spec || !out) return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    return EZ_OK;
}

// host checks and the program of a general lattice-sum call
ez_status sums_program(int batch, int d, const double *A_dev, int n_nu, const double *nu_host, int n_terms,
                       const int *term_result, const double *term_coef, const int *term_nfac, const int *term_fac,
                       const int *term_mult, int n_results, const ez_quad_spec *specs, int n_specs,
                       const double *out_dev, bool grad, EzProgram &prog, std::vector<EzCombo> &combos) {
    ez_status st = check_common(batch, d, A_dev, specs, out_dev);
    if (st) return st;
    if (!nu_host || !term_result || !term_coef || !term_nfac || !term_fac || !term_mult)
        return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    if (n_specs != 1 && n_specs != batch) return fail(EZ_ERR_INVALID_ARG, "n_specs must be 1 or batch");
    if (grad && n_results > EZ_GRAD_RES_MAX)
        return fail(EZ_ERR_INVALID_ARG, "derivatives are available for at most 2 results per call");
    if (n_nu < 1 || n_nu > EZ_NU_MAX || n_terms < 1 || n_terms > EZ_TERM_MAX)
        return fail(EZ_ERR_INVALID_ARG, "n_nu and n_terms must be in [1, 8]");
    int ell_max = 0;
    for (int i = 0; i < n_specs; ++i) {
        if ((st = check_spec(specs[i]))) return st;
        if (grad && specs[i].precision != EZ_PREC_FP64)
            return fail(EZ_ERR_UNSUPPORTED, "derivatives are computed in FP64 only (EZ_PREC_FP64)");
        ell_max = std::max(ell_max, specs[i].ell);
    }
    std::vector<double> nu(nu_host, nu_host + n_nu);
    std::vector<Term> terms(n_terms);
    for (int t = 0; t < n_terms; ++t) {
        terms[t].res = term_result[t];
        terms[t].coef = term_coef[t];
        if (term_nfac[t] < 1 || term_nfac[t] > EZ_FAC_MAX) return fail(EZ_ERR_INVALID_ARG, "term_nfac must be in [1, 4]");
        for (int f = 0; f < term_nfac[t]; ++f)
            terms[t].fac.push_back({term_fac[EZ_FAC_MAX * t + f], term_mult[EZ_FAC_MAX * t + f]});
    }
    if ((st = build_program(d, nu, terms, n_results, ell_max, prog, combos))) return st;
    if (grad && prog.real_nu)
        return fail(EZ_ERR_UNSUPPORTED, "derivatives need integer exponents");
    return EZ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the no-allocation entry point: file-scope device memory, one copy
// per GPU, held until the process ends.  Host code never passes `scratch` itself
// (in host code its name is a host-side stand-in, not a device address); it
// uses the address hipGetSymbolAddress returns for the current device.
#define EZ_SCRATCH_BYTES (64u << 20)
static __device__ __align__(256) unsigned char scratch[EZ_SCRATCH_BYTES];

namespace {

// this device's address of `scratch` (looked up once per device, with that device current)
ez_status scratch_address(DeviceState *S, void **out) {
    if (!S->scratch) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(EZ_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        S->scratch = ptr;
    }
    *out = S->scratch;
    return EZ_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

const char *ez_last_error(void) { return g_err.c_str(); }

const char *ez_version(void) { return "libezeta 0.3 (gfx950, FP64 and mixed precision)"; }

uint64_t ez_workspace_generation(void) { return g_generation.load(); }

ez_status ez_finalize(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    timing_flush();
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_dev) {
        (void)hipSetDevice(kv.first);
        DeviceState *S = kv.second;
        for (auto &p : S->plans) free_plan(p.second);
        free_buf(S->meta); free_buf(S->real); free_buf(S->rec); free_buf(S->rn); free_buf(S->rows);
        free_buf(S->tile_part); free_buf(S->sub_part); free_buf(S->tail_acc); free_buf(S->tail_cnt); free_buf(S->dir_part); free_buf(S->dir_flag); free_buf(S->probe_val); free_buf(S->tensor);
        free_buf(S->tile_grad); free_buf(S->dir_grad); free_buf(S->queue); free_buf(S->tile_bound);
        free_buf(S->dxlist); free_buf(S->dpart);
        for (DevBuf *b : {&S->g_pts_x, &S->g_pts_y, &S->g_perm, &S->g_counts, &S->g_A64r, &S->g_B64r, &S->g_A64k,
                          &S->g_B64k, &S->g_R, &S->g_Q, &S->g_wsum, &S->g_stat, &S->g_Ahr, &S->g_Alr, &S->g_Bhr,
                          &S->g_Blr, &S->g_Ahk, &S->g_Alk, &S->g_Bhk, &S->g_Blk})
            free_buf(*b);
        if (S->side) {
            (void)hipStreamSynchronize(S->side);
            (void)hipStreamDestroy(S->side);
            (void)hipEventDestroy(S->ev_setup);
            (void)hipEventDestroy(S->ev_had);
        }
        for (int i = 0; i < 2; ++i)
            if (S->sig.p[i]) (void)hipFree(S->sig.p[i]);
        free_buf(S->gmeta); free_buf(S->greal); free_buf(S->grec);
        delete S;
    }
    g_dev.clear();
    (void)hipSetDevice(cur);
    return EZ_OK;
}

ez_status ez_lattice_sums_grad(int batch, int d, const double *A_dev, int n_nu, const double *nu_host, int n_terms,
                               const int *term_result, const double *term_coef, const int *term_nfac,
                               const int *term_fac, const int *term_mult, int n_results, const ez_quad_spec *specs,
                               int n_specs, double *out_dev, double *grad_dev, uint32_t *status_dev, void *stream) {
    EzProgram prog;
    std::vector<EzCombo> combos;
    ez_status st = sums_program(batch, d, A_dev, n_nu, nu_host, n_terms, term_result, term_coef, term_nfac, term_fac,
                                term_mult, n_results, specs, n_specs, out_dev, grad_dev != nullptr, prog, combos);
    if (st) return st;
    return run_sums(batch, d, A_dev, prog, combos, specs, n_specs, out_dev, status_dev, (hipStream_t)stream, grad_dev);
}

ez_status ez_lattice_sums_noalloc(int batch, int d, const double *A_dev, int n_nu, const double *nu_host, int n_terms,
                                  const int *term_result, const double *term_coef, const int *term_nfac,
                                  const int *term_fac, const int *term_mult, int n_results, const ez_quad_spec *specs,
                                  int n_specs, double *out_dev, uint32_t *status_dev, void *stream) {
    EzProgram prog;
    std::vector<EzCombo> combos;
    ez_status st = sums_program(batch, d, A_dev, n_nu, nu_host, n_terms, term_result, term_coef, term_nfac, term_fac,
                                term_mult, n_results, specs, n_specs, out_dev, false, prog, combos);
    if (st) return st;
    for (int i = 0; i < n_specs; ++i)
        if (specs[i].precision != EZ_PREC_FP64)
            return fail(EZ_ERR_UNSUPPORTED, "the no-allocation entry point computes in FP64 only");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    EZ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState *S = device_state(dev);
    void *base = nullptr;
    if ((st = scratch_address(S, &base))) return st;
    if (!S->n_cu) EZ_HIP_TRY(hipDeviceGetAttribute(&S->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    CallInfo C;
    if ((st = prepare_call(batch, d, prog, combos, specs, n_specs, false, C))) return st;
    // the plan at the start of the scratch; uploaded unless it is the resident one
    const std::string key = plan_key(d, batch, specs, n_specs, C.ndb);
    HostPlan H;
    const bool resident = S->scratch_key == key && S->scratch_plan_bytes > 0;
    if (!resident && (st = build_host_plan(d, batch, specs, n_specs, C.ndb, H))) return st;
    unsigned char *p0 = (unsigned char *)base;
    size_t off = 0;
    PlanView pv;
    size_t sz[6] = {0, 0, 0, 0, 0, 0}, o[6] = {0, 0, 0, 0, 0, 0};
    if (resident) {
        pv = S->scratch_plan;
        off = S->scratch_plan_bytes;
    } else {
        sz[0] = H.rules.size() * sizeof(double);
        sz[1] = sizeof(EzInstPlan) * (size_t)batch;
        sz[2] = sz[3] = sz[4] = sizeof(int) * (size_t)(batch + 1);
        sz[5] = sizeof(int) * std::max<size_t>(1, H.order.size());
        for (int i = 0; i < 6; ++i) { o[i] = off; off += align256(sz[i]); }
        fill_plan_view(H, pv);
        pv.rules = (const double *)(p0 + o[0]);
        pv.plans = (const EzInstPlan *)(p0 + o[1]);
        pv.tile_begin = (const int *)(p0 + o[2]);
        pv.dir_begin = (const int *)(p0 + o[3]);
        pv.htile_begin = (const int *)(p0 + o[4]);
        pv.tile_order = (const int *)(p0 + o[5]);
    }
    const size_t plan_bytes = off;
    const int n_main = main_tiles(C, prog, S->n_cu, pv.n_tiles);
    note_tiles(S, C, pv.n_tiles, n_main);
    Workspace W;
    workspace_sizes(batch, prog, C, pv, n_main, W);
    for (int i = 0; i < WS_COUNT; ++i) {
        if (W.bytes[i] == 0) continue;
        W.ptr[i] = p0 + off;
        off += align256(W.bytes[i]);
    }
    if (off > EZ_SCRATCH_BYTES)   // checked before anything is copied or launched
        return fail(EZ_ERR_INVALID_ARG, "the call needs " + std::to_string(off) +
                                            " bytes for its plan and workspace; the no-allocation scratch holds " +
                                            std::to_string(EZ_SCRATCH_BYTES));
    if (!resident) {
        // pageable host sources: each copy has completed when hipMemcpyAsync returns
        const void *src[6] = {H.rules.data(), H.plans.data(), H.tb.data(), H.db.data(), H.hb.data(), H.order.data()};
        S->scratch_key.clear();
        for (int i = 0; i < 6; ++i)
            if (sz[i] && !(i == 5 && H.order.empty()))
                EZ_HIP_TRY(hipMemcpyAsync(p0 + o[i], src[i], sz[i], hipMemcpyHostToDevice, s));
        S->scratch_key = key;
        S->scratch_plan = pv;
        S->scratch_plan_bytes = plan_bytes;
    }
    // the tail group counters must start at zero (the scratch keeps the last call's contents)
    EZ_HIP_TRY(ez_launch_fill_int((int *)W.ptr[WS_TAIL_CNT], (int)(W.bytes[WS_TAIL_CNT] / sizeof(int)), 0, s));
    // one stream, no events: the Hadamard branch runs before the nodes
    return enqueue_sums(batch, A_dev, prog, combos, C, pv, n_main, S->n_cu, W, out_dev, status_dev, nullptr, s,
                        nullptr, nullptr, nullptr, false);
}

ez_status ez_lattice_sums(int batch, int d, const double *A_dev, int n_nu, const double *nu_host, int n_terms,
                          const int *term_result, const double *term_coef, const int *term_nfac,
                          const int *term_fac, const int *term_mult, int n_results, const ez_quad_spec *specs,
                          int n_specs, double *out_dev, uint32_t *status_dev, void *stream) {
    return ez_lattice_sums_grad(batch, d, A_dev, n_nu, nu_host, n_terms, term_result, term_coef, term_nfac, term_fac,
                                term_mult, n_results, specs, n_specs, out_dev, nullptr, status_dev, stream);
}

ez_status ez_lattice_sums_bound(int batch, int d, const double *A_dev, int n_nu, const double *nu_host, int n_terms,
                                const int *term_result, const double *term_coef, const int *term_nfac,
                                const int *term_fac, const int *term_mult, int n_results, const ez_quad_spec *specs,
                                int n_specs, double *out_dev, double *bound_dev, uint32_t *status_dev, void *stream) {
    if (!bound_dev) return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    EzProgram prog;
    std::vector<EzCombo> combos;
    ez_status st = sums_program(batch, d, A_dev, n_nu, nu_host, n_terms, term_result, term_coef, term_nfac, term_fac,
                                term_mult, n_results, specs, n_specs, out_dev, false, prog, combos);
    if (st) return st;
    return run_sums(batch, d, A_dev, prog, combos, specs, n_specs, out_dev, status_dev, (hipStream_t)stream, nullptr,
                    bound_dev);
}

ez_status ez_nbody_lattice_sum(int batch, int d, const double *A_dev, int n, const double *nu_host,
                               const ez_quad_spec *spec, double *out_dev, uint32_t *status_dev, void *stream) {
    ez_status st = check_common(batch, d, A_dev, spec, out_dev);
    if (st) return st;
    if (!nu_host || n < 1 || n > EZ_MULT_MAX) return fail(EZ_ERR_INVALID_ARG, "need 1 <= n <= 64 exponents");
    if ((st = check_spec(*spec))) return st;
    std::vector<double> distinct;
    std::vector<int> mult;
    for (int i = 0; i < n; ++i) {
        auto it = std::find(distinct.begin(), distinct.end(), nu_host[i]);
        if (it == distinct.end()) { distinct.push_back(nu_host[i]); mult.push_back(1); }
        else mult[it - distinct.begin()]++;
    }
    if ((int)distinct.size() > EZ_FAC_MAX)
        return fail(EZ_ERR_INVALID_ARG, "at most 4 distinct exponents per n-body sum");
    Term T;
    T.res = 0;
    T.coef = 1.0;
    for (size_t i = 0; i < distinct.size(); ++i) T.fac.push_back({(int)i, mult[i]});
    EzProgram prog;
    std::vector<EzCombo> combos;
    if ((st = build_program(d, distinct, {T}, 1, spec->ell, prog, combos))) return st;
    return run_sums(batch, d, A_dev, prog, combos, spec, 1, out_dev, status_dev, (hipStream_t)stream);
}

ez_status ez_atm_energy(int batch, int d, const double *A_dev, const ez_quad_spec *spec, double *E_dev,
                        double *dEdA_dev, uint32_t *status_dev, void *stream) {
    ez_status st = check_common(batch, d, A_dev, spec, E_dev);
    if (st) return st;
    if ((st = check_spec(*spec))) return st;
    if (dEdA_dev && spec->precision != EZ_PREC_FP64)
        return fail(EZ_ERR_UNSUPPORTED, "derivatives are computed in FP64 only (EZ_PREC_FP64)");
    // nu set {-1, 1, 3, 5};  E = 1/24 Z3^3 - 3/16 Z-1 Z5^2 + 3/8 Z1 Z3 Z5
    std::vector<double> nu = {-1.0, 1.0, 3.0, 5.0};
    Term t0{0, 1.0 / 24.0, {{2, 3}}};
    Term t1{0, -3.0 / 16.0, {{0, 1}, {3, 2}}};
    Term t2{0, 3.0 / 8.0, {{1, 1}, {2, 1}, {3, 1}}};
    EzProgram prog;
    std::vector<EzCombo> combos;
    if ((st = build_program(d, nu, {t0, t1, t2}, 1, spec->ell, prog, combos))) return st;
    return run_sums(batch, d, A_dev, prog, combos, spec, 1, E_dev, status_dev, (hipStream_t)stream, dEdA_dev);
}

ez_status ez_direct_atm(int d, const double *A_host, int L, int use_symmetry, double *out_dev, void *stream) {
    if (d < 1 || d > 3) return fail(EZ_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (!A_host || !out_dev) return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    const long long Lmax = d == 1 ? (1ll << 28) : (d == 2 ? 8192 : 512);
    if (L < 1 || L > Lmax) return fail(EZ_ERR_INVALID_ARG, "L out of range for this d");
    double G[9] = {0}, tr = 0.0;
    for (int i = 0; i < d * d; ++i)
        if (!std::isfinite(A_host[i])) return fail(EZ_ERR_INVALID_ARG, "A not finite");
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double g = 0.0;
            for (int k = 0; k < d; ++k) g += A_host[k * d + i] * A_host[k * d + j];
            G[i * 3 + j] = g;
        }
    for (int i = 0; i < d; ++i) tr += G[i * 3 + i];
    if (!(tr > 0.0)) return fail(EZ_ERR_INVALID_ARG, "A is singular");
    if (use_symmetry) {
        // the metric must be c I so that the signed coordinate permutations are isometries
        const double c = tr / d;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                if (std::fabs(G[i * 3 + j] - (i == j ? c : 0.0)) > 1e-14 * c)
                    return fail(EZ_ERR_INVALID_ARG, "use_symmetry needs A^T A = c I (square or cubic lattice)");
    }
    EzDirectArgs g;
    std::memset(&g, 0, sizeof(g));
    g.d = d;
    g.L = L;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) g.A[i * 3 + j] = A_host[i * d + j];
    const long long M = 2ll * L + 1;
    long long nbox = 1;
    for (int i = 0; i < d; ++i) nbox *= M;
    g.n_box = nbox;
    // outer points with weights
    std::vector<int> xl;
    if (use_symmetry) {
        // 0 <= n_1 <= ... <= n_d <= L, n != 0; weight 2^{#nonzero} d! / prod(multiplicities!)
        int n[3] = {0, 0, 0};
        std::function<void(int, int)> rec = [&](int j, int lo) {
            if (j == d) {
                int nz = 0;
                for (int i = 0; i < d; ++i) nz += n[i] != 0;
                if (nz == 0) return;
                long long wgt = 1ll << nz, perm = 1, run = 1;
                for (int i = 2; i <= d; ++i) perm *= i;
                for (int i = 1; i < d; ++i) {
                    if (n[i] == n[i - 1]) { ++run; perm /= run; } else run = 1;
                }
                xl.insert(xl.end(), {n[0], n[1], n[2], (int)(wgt * perm)});
                return;
            }
            for (int v = lo; v <= L; ++v) { n[j] = v; rec(j + 1, v); }
            n[j] = 0;
        };
        rec(0, 0);
    } else {
        for (long long k = 0; k < nbox; ++k) {
            long long q = k;
            int n[3] = {0, 0, 0};
            bool zero = true;
            for (int j = 0; j < d; ++j) { n[j] = (int)(q % M) - L; q /= M; zero = zero && n[j] == 0; }
            if (!zero) xl.insert(xl.end(), {n[0], n[1], n[2], 1});
        }
    }
    g.n_x = (long long)(xl.size() / 4);
    const long long xblocks = (g.n_x + 255) / 256;
    long long chunks = std::max<long long>(1, (nbox + 32767) / 32768);
    chunks = std::max<long long>(chunks, (4096 + xblocks - 1) / xblocks);
    chunks = std::min<long long>(chunks, std::min<long long>(65535, nbox));
    g.per_chunk = (nbox + chunks - 1) / chunks;
    int dev = 0;
    EZ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState *S = device_state(dev);
    ez_status st;
    const long long nparts = ez_direct_parts(g.n_x, (int)chunks);
    if ((st = grow(S->dxlist, sizeof(int) * xl.size())) || (st = grow(S->dpart, sizeof(double) * 2 * nparts)))
        return st;
    hipStream_t hs = (hipStream_t)stream;
    // pageable host source: the copy has completed when the call returns
    EZ_HIP_TRY(hipMemcpyAsync(S->dxlist.p, xl.data(), sizeof(int) * xl.size(), hipMemcpyHostToDevice, hs));
    g.xlist = (const int *)S->dxlist.p;
    g.part = (double *)S->dpart.p;
    EZ_HIP_TRY(ez_launch_direct_atm(g, (int)chunks, out_dev, hs));
    return EZ_OK;
}

ez_status ez_epstein_zeta(int d, const double *A_dev, int n_nu, const double *nu_host, int64_t n_pts,
                          const double *x_dev, const double *y_dev, double lam, double a_cut, double *out_dev,
                          uint32_t *status_dev, void *stream) {
    if (d < 1 || d > 3) return fail(EZ_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (!A_dev || !nu_host || (n_pts > 0 && (!x_dev || !y_dev || !out_dev)))
        return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    if (n_nu < 1 || n_nu > EZ_NU_MAX) return fail(EZ_ERR_INVALID_ARG, "n_nu must be in [1, 8]");
    if (n_pts < 0) return fail(EZ_ERR_INVALID_ARG, "n_pts must be >= 0");
    if (!(lam >= 0.0 && lam <= 8.0) || !(a_cut >= 0.0 && a_cut <= 200.0))
        return fail(EZ_ERR_INVALID_ARG, "lam in [0, 8], a_cut in [0, 200]");
    for (int i = 0; i < n_nu; ++i)
        if (!std::isfinite(nu_host[i]) || std::fabs(nu_host[i]) > 64.0)
            return fail(EZ_ERR_INVALID_ARG, "nu must be finite, |nu| <= 64");
    if (lam == 0.0) lam = 1.0;
    if (a_cut == 0.0) a_cut = 36.0;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    EZ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState *S = device_state(dev);
    EzTables tab;
    ez_status st = general_setup(S, d, A_dev, lam, a_cut, status_dev, s, &tab);
    if (st) return st;
    EzEpsteinArgs ea;
    std::memset(&ea, 0, sizeof(ea));
    ea.d = d;
    ea.n_nu = n_nu;
    for (int i = 0; i < n_nu; ++i) ea.nu[i] = nu_host[i];
    ea.n_pts = n_pts;
    ea.x = x_dev;
    ea.y = y_dev;
    ea.meta = (const EzLatMeta *)S->gmeta.p;
    ea.tab = tab;
    ea.out = out_dev;
    ea.status = status_dev;
    EZ_HIP_TRY(timed(EZ_KERNEL_EPSTEIN, s, [&] { return ez_launch_epstein(ea, s); }));
    return EZ_OK;
}

ez_status ez_epstein_grid(int d, const double *A_dev, int n_nu, const double *nu_host, int n_x, const double *x_dev,
                          int n_y, const double *y_dev, double lam, double a_cut, int precision, double *out_dev,
                          double *bound_dev, uint32_t *status_dev, void *stream) {
    if (d < 1 || d > 3) return fail(EZ_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (!A_dev || !nu_host || !x_dev || !y_dev || !out_dev) return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    if (n_nu < 1 || n_nu > EZ_NU_MAX) return fail(EZ_ERR_INVALID_ARG, "n_nu must be in [1, 8]");
    if (n_x < 1 || n_y < 1 || n_x > (1 << 16) || n_y > (1 << 22))
        return fail(EZ_ERR_INVALID_ARG, "need 1 <= n_x <= 65536 and 1 <= n_y <= 4194304");
    if (precision != EZ_PREC_FP64 && precision != EZ_PREC_MIXED)
        return fail(EZ_ERR_INVALID_ARG, "precision must be EZ_PREC_FP64 or EZ_PREC_MIXED");
    if (!(lam >= 0.0 && lam <= 8.0) || !(a_cut >= 0.0 && a_cut <= 200.0))
        return fail(EZ_ERR_INVALID_ARG, "lam in [0, 8], a_cut in [0, 200]");
    for (int i = 0; i < n_nu; ++i)
        if (!std::isfinite(nu_host[i]) || std::fabs(nu_host[i]) > 64.0)
            return fail(EZ_ERR_INVALID_ARG, "nu must be finite, |nu| <= 64");
    if (lam == 0.0) lam = 1.0;
    if (a_cut == 0.0) a_cut = 36.0;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    EZ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState *S = device_state(dev);
    ez_status st;
    if ((st = grow(S->g_stat, 256))) return st;
    uint32_t *stat = status_dev ? status_dev : (uint32_t *)S->g_stat.p;
    EzTables tab;
    if ((st = general_setup(S, d, A_dev, lam, a_cut, stat, s, &tab))) return st;
    // table sizes size the products: one read-back after the setup
    EzLatMeta meta;
    EZ_HIP_TRY(hipMemcpyAsync(&meta, S->gmeta.p, sizeof(EzLatMeta), hipMemcpyDeviceToHost, s));
    EZ_HIP_TRY(hipStreamSynchronize(s));
    const int nr = meta.status ? 0 : meta.n_real, nk = meta.status ? 0 : meta.n_rec;
    EzGridArgs g;
    std::memset(&g, 0, sizeof(g));
    g.d = d;
    g.n_nu = n_nu;
    for (int i = 0; i < n_nu; ++i) g.nu[i] = nu_host[i];
    g.n_x = n_x;
    g.n_y = n_y;
    g.Mp = (n_x + 127) / 128 * 128;
    g.Np = (n_y + 127) / 128 * 128;
    g.Kr_pad = (nr + 31) / 32 * 32 + 32;
    g.Kk_pad = (nk + 31) / 32 * 32 + 32;
    g.Krn_pad = g.Krf_pad = g.Kr_pad;
    g.Kkn_pad = g.Kkf_pad = g.Kk_pad;
    g.mixed = precision == EZ_PREC_MIXED ? 1 : 0;
    g.a_near = 21.0;
    g.ladder = 1;
    for (int i = 0; i < n_nu; ++i) {
        const double p2 = nu_host[i] - d + 2.0;
        if (p2 != std::floor(p2) || std::fabs(p2) > 64.0) g.ladder = 0;
        g.p2[i] = g.ladder ? (int)p2 : 0;
    }
    g.meta = (const EzLatMeta *)S->gmeta.p;
    g.tab = tab;
    g.x = x_dev;
    g.y = y_dev;
    const size_t Mp = g.Mp, Np = g.Np, Kr = g.Kr_pad, Kk = g.Kk_pad, nn = n_nu;
    if ((st = grow(S->g_pts_x, sizeof(double) * 8 * (size_t)n_x)) ||
        (st = grow(S->g_pts_y, sizeof(double) * 4 * (size_t)n_y)) ||
        (st = grow(S->g_perm, sizeof(int) * (Kr + Kk))) ||
        (st = grow(S->g_counts, sizeof(int) * 8 + sizeof(double) * EZ_NU_MAX)) ||
        (st = grow(S->g_A64r, sizeof(double) * nn * Mp * Kr)) ||
        (st = grow(S->g_B64r, sizeof(double) * Kr * 2 * Np)) ||
        (st = grow(S->g_A64k, sizeof(double) * 2 * Mp * Kk)) ||
        (st = grow(S->g_B64k, sizeof(double) * Kk * nn * Np)) ||
        (st = grow(S->g_R, sizeof(double) * nn * Mp * 2 * Np)) ||
        (st = grow(S->g_Q, sizeof(double) * 2 * Mp * nn * Np)) ||
        (st = grow(S->g_wsum, sizeof(double) * 2 * (nn * Mp + nn * Np))))
        return st;
    if (g.mixed &&
        ((st = grow(S->g_Ahr, 2 * nn * Mp * Kr)) || (st = grow(S->g_Alr, 2 * nn * Mp * Kr)) ||
         (st = grow(S->g_Bhr, 2 * 2 * Np * Kr)) || (st = grow(S->g_Blr, 2 * 2 * Np * Kr)) ||
         (st = grow(S->g_Ahk, 2 * 2 * Mp * Kk)) || (st = grow(S->g_Alk, 2 * 2 * Mp * Kk)) ||
         (st = grow(S->g_Bhk, 2 * nn * Np * Kk)) || (st = grow(S->g_Blk, 2 * nn * Np * Kk))))
        return st;
    g.pts_x = (double *)S->g_pts_x.p;
    g.pts_y = (double *)S->g_pts_y.p;
    g.perm_real = (int *)S->g_perm.p;
    g.perm_rec = g.perm_real + Kr;
    g.counts = (int *)S->g_counts.p;
    g.kpref = (double *)(g.counts + 8);
    g.A64r = (double *)S->g_A64r.p;
    g.B64r = (double *)S->g_B64r.p;
    g.A64k = (double *)S->g_A64k.p;
    g.B64k = (double *)S->g_B64k.p;
    g.R = (double *)S->g_R.p;
    g.Q = (double *)S->g_Q.p;
    g.wsum = (double *)S->g_wsum.p;
    g.gfar = g.wsum + nn * Mp;
    g.wall = g.gfar + nn * Np;
    g.gall = g.wall + nn * Mp;
    if (g.mixed) {
        g.Ahr = (__bf16 *)S->g_Ahr.p; g.Alr = (__bf16 *)S->g_Alr.p;
        g.Bhr = (__bf16 *)S->g_Bhr.p; g.Blr = (__bf16 *)S->g_Blr.p;
        g.Ahk = (__bf16 *)S->g_Ahk.p; g.Alk = (__bf16 *)S->g_Alk.p;
        g.Bhk = (__bf16 *)S->g_Bhk.p; g.Blk = (__bf16 *)S->g_Blk.p;
    }
    g.out = out_dev;
    g.bound = bound_dev;
    g.status_acc = stat;
    S->grid_nr = nr;
    S->grid_nk = nk;
    EZ_HIP_TRY(timed(EZ_KERNEL_GRID, s, [&] { return ez_grid_launch(g, s, EZ_GRID_PRE); }));
    EZ_HIP_TRY(timed(EZ_KERNEL_GRID_GEMM, s, [&] { return ez_grid_launch(g, s, EZ_GRID_GEMM); }));
    EZ_HIP_TRY(timed(EZ_KERNEL_GRID, s, [&] { return ez_grid_launch(g, s, EZ_GRID_POST); }));
    return EZ_OK;
}

ez_status ez_grid_last_tables(int64_t *n_real, int64_t *n_rec) {
    if (!n_real || !n_rec) return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    int dev = 0;
    EZ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState *S = device_state(dev);
    *n_real = S->grid_nr;
    *n_rec = S->grid_nk;
    return EZ_OK;
}

ez_status ez_last_sum_tiles(int64_t *n_tiles, int64_t *n_main, int *tail_mode) {
    if (!n_tiles || !n_main || !tail_mode) return fail(EZ_ERR_INVALID_ARG, "null pointer argument");
    int dev = 0;
    EZ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState *S = device_state(dev);
    *n_tiles = S->sum_tiles;
    *n_main = S->sum_main;
    *tail_mode = S->sum_tail;
    return EZ_OK;
}

ez_status ez_timing_enable(int enable) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_timing = enable != 0;
    return EZ_OK;
}

ez_status ez_timing_reset(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    timing_flush();
    for (int i = 0; i < EZ_KERNEL_COUNT; ++i) { g_ms[i] = 0.0; g_calls[i] = 0; }
    return EZ_OK;
}

ez_status ez_timing_read(int kernel, double *total_ms, int64_t *launches) {
    if (kernel < 0 || kernel >= EZ_KERNEL_COUNT || !total_ms || !launches)
        return fail(EZ_ERR_INVALID_ARG, "kernel id out of range or null pointer");
    std::lock_guard<std::mutex> lock(g_mu);
    timing_flush();
    *total_ms = g_ms[kernel];
    *launches = g_calls[kernel];
    return EZ_OK;
}

}  // extern "C"
