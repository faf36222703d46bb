// api.hip -- the C ABI of libgrpic.so (declared in include/grpic.h):
// argument validation, launch configuration and error reporting.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <algorithm>
#include <mutex>
#include <string>
#include <tuple>

#include "grpic.h"
#include "grpic_fields.hpp"
#include "grpic_launch.hpp"
#include "grpic_qed.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return GRPIC_OK;
    return fail(GRPIC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int check_metric(const grpic_metric* m) {
    if (!m) return fail(GRPIC_EINVAL, "metric is NULL");
    if (!isfinite(m->a) || !isfinite(m->M) || m->M < 0.0 || fabs(m->a) > m->M)
        return fail(GRPIC_EINVAL, "metric: need M >= 0 and |a| <= M (a=%g, M=%g)", m->a, m->M);
    return GRPIC_OK;
}

int check_grid(const grpic_grid* g) {
    if (!g) return fail(GRPIC_EINVAL, "grid is NULL");
    if (g->nr <= 0 || g->nth <= 0) return fail(GRPIC_EINVAL, "grid: nr, nth must be positive");
    if ((int64_t)g->nr * g->nth >= (int64_t)INT32_MAX) return fail(GRPIC_EINVAL, "grid: nr*nth too large");
    if (g->guard < 2) return fail(GRPIC_EINVAL, "grid: guard must be >= 2 (got %d)", g->guard);
    if (g->pitch < g->nth + 1 + 2 * g->guard)
        return fail(GRPIC_EINVAL, "grid: pitch %d < nth + 1 + 2*guard", g->pitch);
    if ((int64_t)(g->nr + 1 + 2 * g->guard) * g->pitch * (int64_t)sizeof(double) > (int64_t)UINT32_MAX)
        return fail(GRPIC_EINVAL, "grid: arrays of (nr + 1 + 2*guard) x pitch doubles must stay below 4 GiB");
    if (!isfinite(g->lnr0) || !(g->dlnr > 0.0) || !isfinite(g->dlnr))
        return fail(GRPIC_EINVAL, "grid: lnr0 must be finite and dlnr > 0");
    const double dth = M_PI / g->nth;
    if (!(fabs(g->dth - dth) <= 1e-12 * dth)) return fail(GRPIC_EINVAL, "grid: dth must equal pi/nth");
    return GRPIC_OK;
}

int check_species(const grpic_species* sp, int nsp) {
    if (!sp) return fail(GRPIC_EINVAL, "species is NULL");
    if (nsp < 1 || nsp > GRPIC_MAX_SPECIES) return fail(GRPIC_EINVAL, "nsp must be in [1, %d]", GRPIC_MAX_SPECIES);
    for (int s = 0; s < nsp; ++s) {
        if (!isfinite(sp[s].q) || !isfinite(sp[s].m)) return fail(GRPIC_EINVAL, "species %d: q, m not finite", s);
        if (!sp[s].massless && !(sp[s].m > 0.0)) return fail(GRPIC_EINVAL, "species %d: m must be > 0", s);
    }
    return GRPIC_OK;
}

int check_particles(const grpic_particles* p, const char* name) {
    if (!p) return fail(GRPIC_EINVAL, "%s is NULL", name);
    if (p->n < 0) return fail(GRPIC_EINVAL, "%s: n < 0", name);
    if (p->precision != GRPIC_FP64 && p->precision != GRPIC_FP32_SPLIT)
        return fail(GRPIC_EINVAL, "%s: unknown precision %d", name, p->precision);
    if (p->n > 0 && (!p->cell || !p->xr || !p->xth || !p->ur || !p->uth || !p->uph || !p->w || !p->sp))
        return fail(GRPIC_EINVAL, "%s: NULL particle array", name);
    return GRPIC_OK;
}

// Host evaluation of the light-crossing bound (own formulas of App. A).
double crossing_time_uncached(const grpic_metric* m, const grpic_grid* g) {
    double best = INFINITY;
    const double a = m->a, M = m->M;
    for (int i = 0; i < g->nr; ++i) {
        const double r = exp(g->lnr0 + (i + 0.5) * g->dlnr);
        for (int j = 0; j < g->nth; ++j) {
            const double th = (j + 0.5) * g->dth;
            const double c = cos(th);
            const double rho2 = r * r + a * a * c * c;
            const double z = 2.0 * M * r / rho2;
            const double alpha = 1.0 / sqrt(1.0 + z);
            const double beta = z / (1.0 + z);
            const double h_rr = (r * r + a * a) / rho2 - beta;
            const double v_xi = (alpha * sqrt(h_rr) + fabs(beta)) / (r * g->dlnr);
            const double v_eta = alpha / sqrt(rho2) / g->dth;
            const double v = v_xi > v_eta ? v_xi : v_eta;
            if (1.0 / v < best) best = 1.0 / v;
        }
    }
    return best;
}

std::mutex g_cache_mu;
std::map<std::tuple<double, double, int, int, double, double>, double> g_cross_cache;

double crossing_time_cached(const grpic_metric* m, const grpic_grid* g) {
    const auto key = std::make_tuple(m->a, m->M, g->nr, g->nth, g->lnr0, g->dlnr);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cross_cache.find(key);
        if (it != g_cross_cache.end()) return it->second;
    }
    const double t = crossing_time_uncached(m, g);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_cross_cache.size() > 64) g_cross_cache.clear();
    g_cross_cache[key] = t;
    return t;
}

// Host-side record of the tilings written by grpic_sort, so that a push can
// check without a device round trip that a tiling describes its particles.
struct TilingInfo {
    int64_t n;
    int nr, nth;
    double lnr0, dlnr, dth;          // the grid its anchor table was computed for
};
bool tiling_matches(const TilingInfo& t, int64_t n, const grpic_grid* g) {
    return t.n == n && t.nr == g->nr && t.nth == g->nth && t.lnr0 == g->lnr0 && t.dlnr == g->dlnr && t.dth == g->dth;
}
std::mutex g_tiling_mu;
std::map<const void*, TilingInfo> g_tilings;

void fill_common(grpic::StepArgs& A, const grpic_metric* m, const grpic_grid* g,
                 const grpic_species* sp, int nsp, const grpic_particles* p) {
    memset(&A, 0, sizeof A);
    A.a = m ? m->a : 0.0;
    A.M = m ? m->M : 0.0;
    A.nr = g->nr; A.nth = g->nth; A.guard = g->guard; A.pitch = g->pitch;
    A.lnr0 = g->lnr0; A.dlnr = g->dlnr; A.dth = g->dth;
    A.idlnr = 1.0 / g->dlnr; A.idth = 1.0 / g->dth;
    A.inv_nth = 1.0 / g->nth;
    A.inv_tpr = 1.0 / grpic::tiles_per_row(g->nth);
    A.small_steps = (2.0 * g->dlnr <= grpic::kTinyArg && 2.0 * g->dth <= grpic::kTinyArg)     ? 2
                  : (2.0 * g->dlnr <= grpic::kSmallArg && 2.0 * g->dth <= grpic::kSmallArg) ? 1
                                                                                             : 0;
    // split precision: FP64 where a step can reach r < 2M (the strong-field
    // region) and within a sin(theta) < kPoleSin band of the axis (+2 cells of reach)
    const double M = m ? m->M : 0.0;
    const double i2 = M > 0.0 ? (log(2.0 * M) - g->lnr0) / g->dlnr : -1e9;
    A.fp64_rows = i2 < 0.0 ? 0 : (int)fmin((double)g->nr, ceil(i2) + 2.0);
    // rounded up to whole tiles, so that no tile mixes float and double lanes
    const int pole = (int)ceil(asin(grpic::kPoleSin) / g->dth) + 2;
    A.pole_cols = std::min(g->nth, (pole + grpic::kTileCells - 1) / grpic::kTileCells * grpic::kTileCells);
    A.nsp = nsp;
    for (int s = 0; s < nsp; ++s) {
        A.q[s] = sp[s].q;
        A.m[s] = sp[s].m;
        A.qm[s] = sp[s].massless ? 0.0 : sp[s].q / sp[s].m;
        A.massless[s] = sp[s].massless;
    }
    A.n = p->n;
    A.cell = p->cell;
    A.xr = p->xr; A.xth = p->xth; A.ur = p->ur; A.uth = p->uth; A.uph = p->uph; A.w = p->w;
    A.sp = p->sp;
    A.phi = p->phi;
}

// Host-side record of the field tables written by grpic_field_tables: the
// metric and grid they describe, so that a step can check them.
struct FieldTablesInfo {
    double a, M, lnr0, dlnr, dth;
    int nr, nth, guard, pitch;
};
std::mutex g_ftab_mu;
std::map<const void*, FieldTablesInfo> g_ftabs;

// 10-point Gauss-Legendre nodes and weights on [-1, 1] by the Golub-Welsch
// method: the nodes are the eigenvalues of the symmetric tridiagonal Jacobi
// matrix of the Legendre recurrence (zero diagonal, off-diagonal
// k / sqrt(4 k^2 - 1), k = 1 .. 9), and each weight is 2 (the integral of 1)
// times the squared first component of its unit eigenvector.  The
// eigenproblem is solved by cyclic Jacobi rotations, which keep the
// eigenvectors orthonormal to rounding.
void gauss_legendre10(double* x, double* w) {
    const int n = 10;
    double A[n][n] = {}, V[n][n] = {};
    for (int k = 1; k < n; ++k) A[k - 1][k] = A[k][k - 1] = k / sqrt(4.0 * k * k - 1.0);
    for (int i = 0; i < n; ++i) V[i][i] = 1.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p][q] * A[p][q];
        if (off < 1e-60) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (A[p][q] == 0.0) continue;
                // rotation angle that zeroes A[p][q]: t = tan(angle)
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {          // A <- A R (columns p, q)
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {          // A <- R^T A (rows p, q)
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {          // V <- V R
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    // eigenpairs in ascending node order
    int order[n];
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order, order + n, [&](int a, int b) { return A[a][a] < A[b][b]; });
    for (int i = 0; i < n; ++i) {
        const int e = order[i];
        double norm = 0.0;
        for (int k = 0; k < n; ++k) norm += V[k][e] * V[k][e];
        x[i] = A[e][e];
        w[i] = 2.0 * V[0][e] * V[0][e] / norm;
    }
}

void fill_field_args(grpic::FieldArgs& F, const grpic_metric* m, const grpic_grid* g) {
    memset(&F, 0, sizeof F);
    F.a = m->a;
    F.M = m->M;
    F.lnr0 = g->lnr0;
    F.dlnr = g->dlnr;
    F.dth = g->dth;
    F.nr = g->nr;
    F.nth = g->nth;
    F.guard = g->guard;
    F.pitch = g->pitch;
    F.plane = grpic::field_plane(g->nr, g->pitch, g->guard);
    F.nrow = g->nr + 4;
}

}  // namespace

extern "C" {

const char* grpic_last_error(void) { return g_last_error.c_str(); }

const char* grpic_version(void) { return "grpic 0.1 (gfx950)"; }

double grpic_crossing_time(const grpic_metric* metric, const grpic_grid* grid) {
    if (check_metric(metric) || check_grid(grid)) return -1.0;
    return crossing_time_cached(metric, grid);
}

static int push_deposit(const grpic_metric* metric, const grpic_grid* grid, const grpic_species* species, int nsp,
                        grpic_particles* parts, const grpic_fields* fields, grpic_current* J, void* tiling, double dt,
                        int nsteps, int ncorr, void* ckpt, size_t ckpt_bytes, int ckpt_every, int64_t* counters,
                        void* stream, int kick, int order = 1) {
    int rc;
    if ((rc = check_metric(metric)) || (rc = check_grid(grid)) || (rc = check_species(species, nsp)) ||
        (rc = check_particles(parts, "parts")))
        return rc;
    if (!fields) return fail(GRPIC_EINVAL, "fields is NULL");
    for (int c = 0; c < 3; ++c)
        if (!fields->D[c] || !fields->B[c]) return fail(GRPIC_EINVAL, "fields: NULL component");
    if (!J || !J->Fr || !J->Fth || !J->Gph) return fail(GRPIC_EINVAL, "current: NULL array");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(GRPIC_EINVAL, "dt must be positive and finite");
    if (nsteps < 0) return fail(GRPIC_EINVAL, "nsteps < 0");
    if (ncorr < 0 || ncorr > 16) return fail(GRPIC_EINVAL, "ncorr must be in [0, 16]");
    if (ckpt) {
        if (ckpt_every < 1 || nsteps % ckpt_every != 0)
            return fail(GRPIC_EINVAL, "ckpt_every must be >= 1 and divide nsteps");
        const size_t need = grpic_checkpoint_bytes(parts->n, nsteps, ckpt_every);
        if (ckpt_bytes < need) return fail(GRPIC_ENOMEM, "checkpoints need %zu bytes, got %zu", need, ckpt_bytes);
    }
    const double tc = crossing_time_cached(metric, grid);
    if (dt > tc * (1.0 + 1e-12))
        return fail(GRPIC_ERANGE, "dt = %.17g exceeds the cell light-crossing time %.17g", dt, tc);
    if (tiling) {
        std::lock_guard<std::mutex> lk(g_tiling_mu);
        auto it = g_tilings.find(tiling);
        if (it == g_tilings.end() || !tiling_matches(it->second, parts->n, grid))
            return fail(GRPIC_EINVAL, "tiling was not written by grpic_sort for %lld particles on this grid",
                        (long long)parts->n);
    }
    if (parts->n == 0 || nsteps == 0) return GRPIC_OK;

    grpic::StepArgs A;
    fill_common(A, metric, grid, species, nsp, parts);
    A.dt = dt;
    A.idt = 1.0 / dt;
    A.ncorr = ncorr;
    for (int c = 0; c < 3; ++c) { A.F[c] = fields->D[c]; A.F[3 + c] = fields->B[c]; }
    A.Fr = J->Fr; A.Fth = J->Fth; A.Gph = J->Gph;
    A.counters = reinterpret_cast<unsigned long long*>(counters);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t slot = grpic::checkpoint_slot_bytes(parts->n);
    for (int step = 0; step < nsteps; ++step) {
        if (ckpt && step % ckpt_every == 0) {
            void* dst = static_cast<char*>(ckpt) + (size_t)(step / ckpt_every) * slot;
            if ((rc = hip_status(grpic::launch_save_state(A, parts->precision == GRPIC_FP32_SPLIT, dst, s),
                                 "checkpoint launch")))
                return rc;
        }
        const bool split = parts->precision == GRPIC_FP32_SPLIT;
        const hipError_t e = tiling ? grpic::launch_push_deposit_tiled(A, split, tiling, s, kick, order)
                                    : grpic::launch_push_deposit(A, split, s, kick, order);
        if ((rc = hip_status(e, "push_deposit launch"))) return rc;
    }
    return GRPIC_OK;
}

int grpic_push_deposit(const grpic_metric* metric, const grpic_grid* grid,
                       const grpic_species* species, int nsp,
                       grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                       void* tiling, double dt, int nsteps, int ncorr,
                       void* ckpt, size_t ckpt_bytes, int ckpt_every,
                       int64_t* counters, void* stream) {
    return push_deposit(metric, grid, species, nsp, parts, fields, J, tiling, dt, nsteps, ncorr, ckpt, ckpt_bytes,
                        ckpt_every, counters, stream, grpic::kBoris);
}

int grpic_push_deposit_spline3(const grpic_metric* metric, const grpic_grid* grid,
                               const grpic_species* species, int nsp,
                               grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                               void* tiling, double dt, int nsteps, int ncorr, int64_t* counters, void* stream) {
    if (parts && parts->precision != GRPIC_FP64)
        return fail(GRPIC_EINVAL, "grpic_push_deposit_spline3: GRPIC_FP64 particles only");
    if (grid && grid->guard < 3) return fail(GRPIC_EINVAL, "grpic_push_deposit_spline3: the cubic shape needs guard >= 3");
    if (grid && grid->nth < 4)     // the folded 5 x 5 window stays inside columns 0 .. nth
        return fail(GRPIC_EINVAL, "grpic_push_deposit_spline3: nth must be >= 4");
    return push_deposit(metric, grid, species, nsp, parts, fields, J, tiling, dt, nsteps, ncorr, nullptr, 0, 0,
                        counters, stream, grpic::kBoris, 3);
}

int grpic_push_deposit_vay(const grpic_metric* metric, const grpic_grid* grid,
                           const grpic_species* species, int nsp,
                           grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                           void* tiling, double dt, int nsteps, int ncorr,
                           int64_t* counters, void* stream) {
    if (parts && parts->precision != GRPIC_FP64)
        return fail(GRPIC_EINVAL, "grpic_push_deposit_vay: GRPIC_FP64 particles only");
    return push_deposit(metric, grid, species, nsp, parts, fields, J, tiling, dt, nsteps, ncorr, nullptr, 0, 0,
                        counters, stream, grpic::kVay);
}

size_t grpic_qed_workspace_bytes(const grpic_grid* grid, int64_t n) {
    if (!grid || grid->nr <= 0 || grid->nth <= 0 || n < 0) return 0;
    return grpic::qed_workspace_bytes(grpic::slice_capacity(n, grid->nr, grid->nth));
}

int grpic_push_deposit_qed(const grpic_metric* metric, const grpic_grid* grid,
                           const grpic_species* species, int nsp,
                           grpic_particles* parts, const grpic_fields* fields, grpic_current* J,
                           void* tiling, double dt, int64_t step, int ncorr, const grpic_qed* qed,
                           int64_t* n_used, void* ws, size_t ws_bytes, int64_t* counters, int64_t* qcounters,
                           void* stream) {
    int rc;
    if ((rc = check_metric(metric)) || (rc = check_grid(grid)) || (rc = check_species(species, nsp)) ||
        (rc = check_particles(parts, "parts")))
        return rc;
    if (parts->precision != GRPIC_FP64) return fail(GRPIC_EINVAL, "grpic_push_deposit_qed: GRPIC_FP64 particles only");
    if (parts->n > 0 && !parts->tag) return fail(GRPIC_EINVAL, "grpic_push_deposit_qed: the particles need tags");
    if (!qed) return fail(GRPIC_EINVAL, "qed is NULL");
    if (!n_used) return fail(GRPIC_EINVAL, "n_used is NULL");
    const int sp_e = qed->electron_sp, sp_p = qed->positron_sp, sp_g = qed->photon_sp;
    if (sp_e < 0 || sp_e >= nsp || sp_p < 0 || sp_p >= nsp || sp_g < 0 || sp_g >= nsp)
        return fail(GRPIC_EINVAL, "qed: species indices must lie in [0, %d)", nsp);
    if (!species[sp_g].massless) return fail(GRPIC_EINVAL, "qed: the photon species must be massless");
    if (species[sp_e].massless || species[sp_p].massless)
        return fail(GRPIC_EINVAL, "qed: the electron and positron species must be massive");
    if (!(qed->gamma_thr > 1.0) || !isfinite(qed->gamma_thr)) return fail(GRPIC_EINVAL, "qed: gamma_thr must be > 1");
    if (!(qed->eps_ph > 0.0) || !(qed->eps_ph < sqrt(qed->gamma_thr * qed->gamma_thr - 1.0)))
        return fail(GRPIC_EINVAL, "qed: need 0 < eps_ph < sqrt(gamma_thr^2 - 1)");
    if (!(qed->tau >= 0.0) || !isfinite(qed->tau)) return fail(GRPIC_EINVAL, "qed: tau must be >= 0 and finite");
    if (step < 0) return fail(GRPIC_EINVAL, "step must be >= 0");
    // the push's own checks (one step, no checkpoints); nothing is enqueued
    // for an empty set
    grpic_particles none = *parts;
    none.n = 0;
    if ((rc = push_deposit(metric, grid, species, nsp, &none, fields, J, nullptr, dt, 1, ncorr, nullptr, 0, 0,
                           counters, stream, grpic::kBoris)))
        return rc;
    if (tiling) {
        std::lock_guard<std::mutex> lk(g_tiling_mu);
        auto it = g_tilings.find(tiling);
        if (it == g_tilings.end() || !tiling_matches(it->second, parts->n, grid))
            return fail(GRPIC_EINVAL, "tiling was not written by grpic_sort for %lld particles on this grid",
                        (long long)parts->n);
    }
    if (ws && tiling && ws_bytes < grpic_qed_workspace_bytes(grid, parts->n))
        return fail(GRPIC_ENOMEM, "qed workspace needs %zu bytes, got %zu", grpic_qed_workspace_bytes(grid, parts->n),
                    ws_bytes);
    if (parts->n == 0) return GRPIC_OK;
    grpic::StepArgs A;
    fill_common(A, metric, grid, species, nsp, parts);
    A.dt = dt;
    A.idt = 1.0 / dt;
    A.ncorr = ncorr;
    for (int c = 0; c < 3; ++c) { A.F[c] = fields->D[c]; A.F[3 + c] = fields->B[c]; }
    A.Fr = J->Fr; A.Fth = J->Fth; A.Gph = J->Gph;
    A.counters = reinterpret_cast<unsigned long long*>(counters);
    grpic::QedArgs Q;
    memset(&Q, 0, sizeof Q);
    Q.gamma_thr = qed->gamma_thr;
    Q.eps_ph = qed->eps_ph;
    Q.P = 1.0 - exp(-qed->tau * dt);                          // eq. optical-depth
    Q.seed = qed->seed;
    Q.step = (uint64_t)step;
    Q.electron_sp = sp_e; Q.positron_sp = sp_p; Q.photon_sp = sp_g;
    Q.tag = parts->tag;
    Q.n_used = n_used;
    Q.cap = parts->n;
    Q.qcounters = reinterpret_cast<unsigned long long*>(qcounters);
    const int64_t cap = grpic::slice_capacity(parts->n, grid->nr, grid->nth);
    return hip_status(grpic::launch_push_deposit_qed(A, Q, tiling, cap, ws, static_cast<hipStream_t>(stream)),
                      "push_deposit_qed launch");
}

size_t grpic_checkpoint_bytes(int64_t n, int nsteps, int ckpt_every) {
    if (n < 0 || ckpt_every < 1 || nsteps < 0 || nsteps % ckpt_every != 0) return 0;
    return (size_t)(nsteps / ckpt_every) * grpic::checkpoint_slot_bytes(n);
}

static size_t backward_state_bytes(int64_t n, int ckpt_every) {
    return ((size_t)ckpt_every * 5 * sizeof(double) * (size_t)n + 255) / 256 * 256;
}

size_t grpic_backward_workspace_bytes(const grpic_grid* grid, int64_t n, int ckpt_every) {
    if (!grid || grid->nr <= 0 || grid->guard < 0 || grid->pitch <= 0 || n < 0 || ckpt_every < 1) return 0;
    return backward_state_bytes(n, ckpt_every) + grpic::backward_aux_bytes(grid->nr + 1 + 2 * grid->guard, grid->pitch);
}

static int backward_checked(const grpic_metric* metric, const grpic_grid* grid, const grpic_species* species,
                            int nsp, const grpic_particles* parts, const grpic_fields* fields,
                            const grpic_current* lambda, double dt, int nsteps, int ncorr, const void* ckpt,
                            size_t ckpt_bytes, int ckpt_every, const grpic_backward_range* range, void* ws,
                            size_t ws_bytes, const grpic_momentum_grads* grad_u,
                            const grpic_field_grads* grad_fields, void* stream) {
    int rc;
    if ((rc = check_metric(metric)) || (rc = check_grid(grid)) || (rc = check_species(species, nsp)))
        return rc;
    // the reverse reads w and sp of the particles (their states come from the checkpoints)
    if (!parts) return fail(GRPIC_EINVAL, "parts is NULL");
    if (parts->n < 0) return fail(GRPIC_EINVAL, "parts: n < 0");
    if (parts->precision != GRPIC_FP64) return fail(GRPIC_EINVAL, "the adjoint needs GRPIC_FP64 particles");
    const int64_t first = range ? range->first : 0, count = range ? range->count : parts->n;
    if (first < 0 || count < 0 || first > parts->n || count > parts->n - first)
        return fail(GRPIC_EINVAL, "range: [first, first + count) must lie in [0, n)");
    if (!fields) return fail(GRPIC_EINVAL, "fields is NULL");
    for (int c = 0; c < 3; ++c)
        if (!fields->D[c] || !fields->B[c]) return fail(GRPIC_EINVAL, "fields: NULL component");
    if (!lambda || !lambda->Fr || !lambda->Fth || !lambda->Gph) return fail(GRPIC_EINVAL, "lambda: NULL array");
    if (!grad_u) return fail(GRPIC_EINVAL, "grad_u is NULL");
    if (count > 0 && (!grad_u->ur || !grad_u->uth || !grad_u->uph))
        return fail(GRPIC_EINVAL, "grad_u: NULL array");
    const bool want_fields = grad_fields != nullptr;
    if (!range && !want_fields) return fail(GRPIC_EINVAL, "grad_fields is NULL");
    if (want_fields)
        for (int c = 0; c < 3; ++c)
            if (!grad_fields->D[c] || !grad_fields->B[c]) return fail(GRPIC_EINVAL, "grad_fields: NULL component");
    const size_t plane = (size_t)(grid->nr + 1 + 2 * grid->guard) * (size_t)grid->pitch;
    if (range && ((range->field_step_stride != 0 && range->field_step_stride < plane) ||
                  (range->grad_step_stride != 0 && range->grad_step_stride < plane)))
        return fail(GRPIC_EINVAL, "range: step strides must be 0 or at least one grid array (%zu elements)", plane);
    if (!(dt > 0.0) || !isfinite(dt)) return fail(GRPIC_EINVAL, "dt must be positive and finite");
    if (ncorr < 0 || ncorr > grpic::adj_max_corr()) return fail(GRPIC_EINVAL, "ncorr must be in [0, %d] for the adjoint",
                                                                 grpic::adj_max_corr());
    if (ckpt_every < 1 || nsteps < 1 || nsteps % ckpt_every != 0)
        return fail(GRPIC_EINVAL, "need nsteps >= 1 and ckpt_every >= 1 dividing nsteps");
    if ((parts->n > 0 && !ckpt) || ckpt_bytes < grpic_checkpoint_bytes(parts->n, nsteps, ckpt_every))
        return fail(GRPIC_ENOMEM, "checkpoint buffer too small or NULL");
    if ((count > 0 && !ws) || ws_bytes < grpic_backward_workspace_bytes(grid, count, ckpt_every))
        return fail(GRPIC_ENOMEM, "backward workspace needs %zu bytes, got %zu",
                    grpic_backward_workspace_bytes(grid, count, ckpt_every), ws_bytes);
    const double tc = crossing_time_cached(metric, grid);
    if (dt > tc * (1.0 + 1e-12))
        return fail(GRPIC_ERANGE, "dt = %.17g exceeds the cell light-crossing time %.17g", dt, tc);
    if (parts->n > 0 && (!parts->w || !parts->sp)) return fail(GRPIC_EINVAL, "parts: NULL w or sp");
    grpic::BackArgs B;
    memset(&B, 0, sizeof B);
    B.a = metric->a; B.M = metric->M;
    B.lnr0 = grid->lnr0; B.dlnr = grid->dlnr; B.dth = grid->dth;
    B.nr = grid->nr; B.nth = grid->nth; B.guard = grid->guard; B.pitch = grid->pitch;
    B.dt = dt; B.ncorr = ncorr; B.nsteps = nsteps; B.ckpt_every = ckpt_every; B.nsp = nsp;
    for (int i = 0; i < nsp; ++i) { B.q[i] = species[i].q; B.m[i] = species[i].m; B.massless[i] = species[i].massless; }
    B.n = parts->n;
    B.first = first;
    B.count = count;
    B.fstride = range ? range->field_step_stride : 0;
    B.gstride = range ? range->grad_step_stride : 0;
    B.w = static_cast<const double*>(parts->w);
    B.sp = parts->sp;
    for (int c = 0; c < 3; ++c) {
        B.F[c] = static_cast<const double*>(fields->D[c]);
        B.F[3 + c] = static_cast<const double*>(fields->B[c]);
        B.gradF[c] = want_fields ? grad_fields->D[c] : nullptr;
        B.gradF[3 + c] = want_fields ? grad_fields->B[c] : nullptr;
    }
    B.lam[0] = lambda->Fr; B.lam[1] = lambda->Fth; B.lam[2] = lambda->Gph;
    B.ckpt = ckpt;
    B.slot_bytes = grpic::checkpoint_slot_bytes(parts->n);
    B.ws = static_cast<double*>(ws);
    B.rows = grid->nr + 1 + 2 * grid->guard;
    void* aux = static_cast<char*>(ws) + backward_state_bytes(count, ckpt_every);
    B.grad_u[0] = grad_u->ur; B.grad_u[1] = grad_u->uth; B.grad_u[2] = grad_u->uph;
    return hip_status(grpic::launch_push_deposit_backward(B, aux, static_cast<hipStream_t>(stream)), "backward launch");
}

int grpic_push_deposit_backward(const grpic_metric* metric, const grpic_grid* grid,
                                const grpic_species* species, int nsp, const grpic_particles* parts,
                                const grpic_fields* fields, const grpic_current* lambda,
                                double dt, int nsteps, int ncorr, const void* ckpt, size_t ckpt_bytes,
                                int ckpt_every, void* ws, size_t ws_bytes,
                                const grpic_momentum_grads* grad_u, const grpic_field_grads* grad_fields,
                                void* stream) {
    return backward_checked(metric, grid, species, nsp, parts, fields, lambda, dt, nsteps, ncorr, ckpt, ckpt_bytes,
                            ckpt_every, nullptr, ws, ws_bytes, grad_u, grad_fields, stream);
}

int grpic_push_deposit_backward_range(const grpic_metric* metric, const grpic_grid* grid,
                                      const grpic_species* species, int nsp, const grpic_particles* parts,
                                      const grpic_fields* fields, const grpic_current* lambda,
                                      double dt, int nsteps, int ncorr, const void* ckpt, size_t ckpt_bytes,
                                      int ckpt_every, const grpic_backward_range* range, void* ws,
                                      size_t ws_bytes, const grpic_momentum_grads* grad_u,
                                      const grpic_field_grads* grad_fields, void* stream) {
    if (!range) return fail(GRPIC_EINVAL, "range is NULL");
    return backward_checked(metric, grid, species, nsp, parts, fields, lambda, dt, nsteps, ncorr, ckpt, ckpt_bytes,
                            ckpt_every, range, ws, ws_bytes, grad_u, grad_fields, stream);
}

static int charge(const grpic_grid* grid, const grpic_species* species, int nsp,
                 const grpic_particles* parts, double* Q, void* stream, int order) {
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_species(species, nsp)) || (rc = check_particles(parts, "parts")))
        return rc;
    if (!Q) return fail(GRPIC_EINVAL, "Q is NULL");
    grpic::StepArgs A;
    fill_common(A, nullptr, grid, species, nsp, parts);
    return hip_status(grpic::launch_charge(A, parts->precision == GRPIC_FP32_SPLIT, Q,
                                           static_cast<hipStream_t>(stream), order), "charge launch");
}

int grpic_charge(const grpic_grid* grid, const grpic_species* species, int nsp, const grpic_particles* parts,
                 double* Q, void* stream) {
    return charge(grid, species, nsp, parts, Q, stream, 1);
}

int grpic_charge3(const grpic_grid* grid, const grpic_species* species, int nsp, const grpic_particles* parts,
                  double* Q, void* stream) {
    if (grid && grid->guard < 3) return fail(GRPIC_EINVAL, "grpic_charge3: the cubic shape needs guard >= 3");
    return charge(grid, species, nsp, parts, Q, stream, 3);
}

size_t grpic_sort_workspace_bytes(const grpic_grid* grid, int64_t n) {
    (void)n;
    if (!grid || grid->nr <= 0 || grid->nth <= 0) return 0;
    return grpic::sort_workspace_bytes(grid->nr, grid->nth);
}

size_t grpic_tiling_bytes(const grpic_grid* grid, int64_t n) {
    if (!grid || grid->nr <= 0 || grid->nth <= 0 || n < 0) return 0;
    return grpic::tiling_bytes(n, grid->nr, grid->nth);
}

static int sort_checked(const grpic_grid* grid, const grpic_particles* in, grpic_particles* out,
                        int64_t* cell_offsets, void* tiling, size_t tiling_bytes, void* ws, size_t ws_bytes,
                        int64_t* n_alive_dev, void* stream, bool noalloc) {
    int rc;
    if ((rc = check_grid(grid)) || (rc = check_particles(in, "in")) || (rc = check_particles(out, "out")))
        return rc;
    if (in->precision != out->precision) return fail(GRPIC_EINVAL, "in and out precision differ");
    if (in->n > 0 && (!out->cell || !out->xr || !out->xth || !out->ur || !out->uth || !out->uph || !out->w ||
                      !out->sp))
        return fail(GRPIC_EINVAL, "out: NULL particle array");
    if ((in->phi == nullptr) != (out->phi == nullptr)) return fail(GRPIC_EINVAL, "phi given for only one of in/out");
    if ((in->tag == nullptr) != (out->tag == nullptr)) return fail(GRPIC_EINVAL, "tag given for only one of in/out");
    if (in->n > 0 && (in->cell == out->cell || in->xr == out->xr)) return fail(GRPIC_EINVAL, "in and out alias");
    if (!n_alive_dev) return fail(GRPIC_EINVAL, "n_alive_dev is NULL");
    const size_t need = grpic_sort_workspace_bytes(grid, in->n);
    if (noalloc) {
        if (need > grpic::kSortScratchBytes)
            return fail(GRPIC_ENOMEM, "grpic_sort_noalloc: this grid's sort needs %zu bytes of scratch, above its "
                        "maximum of %zu (2048 x 2048 grids and smaller fit); use grpic_sort", need,
                        grpic::kSortScratchBytes);
        if ((rc = hip_status(grpic::sort_scratch(&ws), "sort scratch address"))) return rc;
        ws_bytes = grpic::kSortScratchBytes;
    }
    if (!ws || ws_bytes < need) return fail(GRPIC_ENOMEM, "sort workspace needs %zu bytes, got %zu", need, ws_bytes);
    if (tiling) {
        const size_t tneed = grpic_tiling_bytes(grid, in->n);
        if (tiling_bytes < tneed) return fail(GRPIC_ENOMEM, "tiling needs %zu bytes, got %zu", tneed, tiling_bytes);
    }
    grpic::SortArgs S;
    memset(&S, 0, sizeof S);
    S.n = in->n;
    S.nr = grid->nr;
    S.nth = grid->nth;
    S.ncell = grid->nr * grid->nth;
    S.elem = in->precision == GRPIC_FP64 ? 8 : 4;
    S.cell_in = in->cell;
    const void* ins[6] = {in->xr, in->xth, in->ur, in->uth, in->uph, in->w};
    void* outs[6] = {out->xr, out->xth, out->ur, out->uth, out->uph, out->w};
    for (int k = 0; k < 6; ++k) { S.in[k] = ins[k]; S.out[k] = outs[k]; }
    S.sp_in = in->sp;
    S.phi_in = in->phi;
    S.cell_out = out->cell;
    S.sp_out = out->sp;
    S.phi_out = out->phi;
    S.tag_in = in->tag;
    S.tag_out = out->tag;
    S.counts = static_cast<unsigned long long*>(ws);
    S.blocksums = S.counts + (S.ncell + 1);
    S.tile_slices = S.blocksums + grpic::sort_scan_blocks((int64_t)S.ncell + 1) + 1;
    S.cell_offsets = cell_offsets;
    S.n_alive = n_alive_dev;
    S.tiling = tiling;
    S.lnr0 = grid->lnr0;
    S.dlnr = grid->dlnr;
    S.dth = grid->dth;
    if ((rc = hip_status(grpic::launch_sort(S, static_cast<hipStream_t>(stream)), "sort launch"))) return rc;
    if (tiling) {
        std::lock_guard<std::mutex> lk(g_tiling_mu);
        if (g_tilings.size() > 4096) g_tilings.clear();
        g_tilings[tiling] = TilingInfo{in->n, grid->nr, grid->nth, grid->lnr0, grid->dlnr, grid->dth};
    }
    return GRPIC_OK;
}

int grpic_sort(const grpic_grid* grid, const grpic_particles* in, grpic_particles* out,
               int64_t* cell_offsets, void* tiling, size_t tiling_bytes, void* ws, size_t ws_bytes,
               int64_t* n_alive_dev, void* stream) {
    return sort_checked(grid, in, out, cell_offsets, tiling, tiling_bytes, ws, ws_bytes, n_alive_dev, stream, false);
}

int grpic_sort_noalloc(const grpic_grid* grid, const grpic_particles* in, grpic_particles* out,
                       int64_t* cell_offsets, void* tiling, size_t tiling_bytes, int64_t* n_alive_dev,
                       void* stream) {
    return sort_checked(grid, in, out, cell_offsets, tiling, tiling_bytes, nullptr, 0, n_alive_dev, stream, true);
}

size_t grpic_field_tables_bytes(const grpic_grid* grid) {
    if (check_grid(grid)) return 0;
    return grpic::field_tables_bytes(grid->nr, grid->nth, grid->pitch, grid->guard);
}

size_t grpic_field_workspace_bytes(const grpic_grid* grid) {
    if (check_grid(grid)) return 0;
    return grpic::field_workspace_bytes(grid->nr, grid->pitch, grid->guard);
}

int grpic_field_tables(const grpic_metric* metric, const grpic_grid* grid, void* tables, size_t tables_bytes,
                       void* stream) {
    int rc;
    if ((rc = check_metric(metric)) || (rc = check_grid(grid))) return rc;
    if (!tables) return fail(GRPIC_EINVAL, "tables is NULL");
    const size_t need = grpic_field_tables_bytes(grid);
    if (tables_bytes < need) return fail(GRPIC_ENOMEM, "field tables need %zu bytes, got %zu", need, tables_bytes);
    grpic::FieldArgs F;
    fill_field_args(F, metric, grid);
    F.tab = static_cast<double*>(tables);
    F.drow = F.tab + grpic::kTablePlanes * F.plane;
    F.rad = F.drow + grpic::kDrRows * F.nrow;
    F.sn = F.rad + grpic::field_nrad(F.nr);
    double gx[10], gw[10];
    gauss_legendre10(gx, gw);
    if ((rc = hip_status(grpic::launch_field_tables(F, gx, gw, static_cast<hipStream_t>(stream)), "field tables")))
        return rc;
    std::lock_guard<std::mutex> lk(g_ftab_mu);
    g_ftabs[tables] = FieldTablesInfo{metric->a, metric->M, grid->lnr0, grid->dlnr, grid->dth,
                                      grid->nr, grid->nth, grid->guard, grid->pitch};
    return GRPIC_OK;
}

int grpic_field_step(const grpic_metric* metric, const grpic_grid* grid, const void* tables,
                     const grpic_field_state* state, const grpic_current* J, double dt, double w1, int ncorr,
                     int damp_cells, double damp_max, void* ws, size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_metric(metric)) || (rc = check_grid(grid))) return rc;
    if (!state) return fail(GRPIC_EINVAL, "state is NULL");
    if (grid->nth < 2 * grid->guard)
        return fail(GRPIC_EINVAL, "field step: nth (%d) must be at least 2*guard (the columns beyond the axes mirror "
                                  "physical ones)", grid->nth);
    for (int c = 0; c < 3; ++c)
        if (!state->D[c] || !state->B[c]) return fail(GRPIC_EINVAL, "state: NULL component");
    if (J && (!J->Fr || !J->Fth || !J->Gph)) return fail(GRPIC_EINVAL, "current: NULL array");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(GRPIC_EINVAL, "dt must be positive and finite");
    if (!(w1 >= 0.0 && w1 <= 1.0)) return fail(GRPIC_EINVAL, "w1 must lie in [0, 1]");
    if (ncorr < 0 || ncorr > 64) return fail(GRPIC_EINVAL, "ncorr must be in [0, 64]");
    if (damp_cells < 0 || damp_cells > grid->nr) return fail(GRPIC_EINVAL, "damp_cells must be in [0, nr]");
    if (!(damp_max >= 0.0 && damp_max <= 1.0)) return fail(GRPIC_EINVAL, "damp_max must lie in [0, 1]");
    {
        std::lock_guard<std::mutex> lk(g_ftab_mu);
        auto it = g_ftabs.find(tables);
        const FieldTablesInfo want{metric->a, metric->M, grid->lnr0, grid->dlnr, grid->dth,
                                   grid->nr, grid->nth, grid->guard, grid->pitch};
        if (!tables || it == g_ftabs.end() || memcmp(&it->second, &want, sizeof want) != 0)
            return fail(GRPIC_EINVAL, "tables were not written by grpic_field_tables for this metric and grid");
    }
    const size_t need = grpic_field_workspace_bytes(grid);
    if (!ws || ws_bytes < need) return fail(GRPIC_ENOMEM, "field workspace needs %zu bytes, got %zu", need, ws_bytes);
    grpic::FieldArgs F;
    fill_field_args(F, metric, grid);
    F.tab = const_cast<double*>(static_cast<const double*>(tables));
    F.drow = F.tab + grpic::kTablePlanes * F.plane;
    F.rad = F.drow + grpic::kDrRows * F.nrow;
    F.sn = F.rad + grpic::field_nrad(F.nr);
    if (J) {
        F.J[0] = J->Fr;
        F.J[1] = J->Fth;
        F.J[2] = J->Gph;
    }
    F.dt = dt;
    F.w1 = w1;
    F.w0 = 1.0 - w1;
    grpic::FieldPtrs X, R, W1, W2;
    for (int c = 0; c < 3; ++c) {
        X.c[c] = state->D[c];
        X.c[3 + c] = state->B[c];
    }
    double* w = static_cast<double*>(ws);
    for (int c = 0; c < 6; ++c) {
        R.c[c] = w + (size_t)c * F.plane;
        W1.c[c] = w + (size_t)(6 + c) * F.plane;
        W2.c[c] = w + (size_t)(12 + c) * F.plane;
    }
    return hip_status(grpic::launch_field_step(F, X, R, W1, W2, ncorr, damp_cells, damp_max,
                                               static_cast<hipStream_t>(stream)),
                      "field step");
}

}  // extern "C"
