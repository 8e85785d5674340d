// Host FP64 equilibria: measured f_eq from counts (Eq.(theory_feq)), the
// single-Gaussian (Eq.(feq_gaussian)) and Poisson-WSG (Eq.(f_eq_wsg)) closed
// forms, and lambda from the displacement moments (Eq.(lambda_eq)).
//
// The one-axis closed form is evaluated through the second difference of the
// ramp expectation h(c) = E[(Z - c)_+], Z ~ N(0, s^2):
//     g(w; s^2) = h(w - 1) - 2 h(w) + h(w + 1),
//     h(c) = s phi(c/s) - c Q(c/s)   (phi: normal density, Q: upper tail),
// which is Eq.(feq_gaussian) rearranged (with a^2 = s^2 and
// N = a / sqrt(2 pi)): the exponentials are the s phi terms and the erf
// differences are the c Q terms.  Written this way every term is evaluated
// with erfc of a non-negative argument, so nothing cancels between nearly
// equal erf values when s is small.
#include <cmath>
#include <cstring>

#include "mdlg_internal.h"

namespace {

constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kInvSqrt2 = 0.70710678118654752440;

// E[(Z - c)_+] for Z ~ N(0, s^2), c >= 0.
double ramp_pos(double c, double s) {
    if (s <= 0.0) return 0.0;
    double z = c / s;
    return s * kInvSqrt2Pi * std::exp(-0.5 * z * z) - c * 0.5 * std::erfc(z * kInvSqrt2);
}

// E[(Z - c)_+] for any c, using E[(Z - c)_+] = -c + E[(Z + c)_+] for c < 0.
double ramp(double c, double s) { return c >= 0.0 ? ramp_pos(c, s) : -c + ramp_pos(-c, s); }

// Probability of lattice displacement w (= v - u, in cells) along one axis
// for a Gaussian displacement of variance s2 (cells^2) and a start position
// uniform in its cell.  Symmetric in w; evaluated at |w|.
double g1(double w, double s2) {
    double aw = std::fabs(w);
    if (s2 <= 0.0) return aw < 1.0 ? 1.0 - aw : 0.0;
    double s = std::sqrt(s2);
    return ramp(aw - 1.0, s) - 2.0 * ramp(aw, s) + ramp(aw + 1.0, s);
}

void gauss2d(double s2, const double* u, double w, double* acc) {
    double ux = u ? u[0] : 0.0, uy = u ? u[1] : 0.0;
    double gx[7], gy[7];
    for (int v = -3; v <= 3; ++v) {
        gx[v + 3] = g1(v - ux, s2);
        gy[v + 3] = g1(v - uy, s2);
    }
    for (int i = 0; i < MDLG_NQ; ++i)
        acc[i] += w * gx[mdlg::kVel.v[i][0] + 3] * gy[mdlg::kVel.v[i][1] + 3];
}

bool finite_u(const double* u) { return !u || (std::isfinite(u[0]) && std::isfinite(u[1])); }

}  // namespace

extern "C" mdlg_status mdlg_feq_measured(const int64_t* counts, int64_t n_particles, int64_t n_events,
                                         int32_t symmetrize, double* g_out, double* overflow_frac) {
    if (!counts || !g_out) return mdlg::fail(MDLG_EINVAL, "mdlg_feq_measured: NULL pointer");
    if (n_particles <= 0 || n_events <= 0)
        return mdlg::fail(MDLG_EINVAL, "mdlg_feq_measured: n_particles and n_events must be > 0");
    double denom = (double)n_particles * (double)n_events;
    for (int i = 0; i < MDLG_NQ; ++i) g_out[i] = (double)counts[i] / denom;
    if (overflow_frac) *overflow_frac = (double)counts[MDLG_NQ] / denom;
    if (symmetrize) {
        // shells of equal |v|^2 (each is one orbit of the square's symmetry group here)
        double sum[19] = {0};
        int num[19] = {0};
        for (int i = 0; i < MDLG_NQ; ++i) {
            int r2 = mdlg::kVel.v[i][0] * mdlg::kVel.v[i][0] + mdlg::kVel.v[i][1] * mdlg::kVel.v[i][1];
            sum[r2] += g_out[i];
            num[r2] += 1;
        }
        for (int i = 0; i < MDLG_NQ; ++i) {
            int r2 = mdlg::kVel.v[i][0] * mdlg::kVel.v[i][0] + mdlg::kVel.v[i][1] * mdlg::kVel.v[i][1];
            g_out[i] = sum[r2] / num[r2];
        }
    }
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_moments(const double* moments, double dx, double* mu2, double* mu4,
                                    double* a2) {
    if (!moments) return mdlg::fail(MDLG_EINVAL, "mdlg_moments: moments is NULL");
    if (!(moments[0] > 0.0)) return mdlg::fail(MDLG_EINVAL, "mdlg_moments: no samples");
    if (a2 && !(dx > 0.0)) return mdlg::fail(MDLG_EINVAL, "mdlg_moments: dx must be > 0");
    double m2 = moments[1] / moments[0];
    if (mu2) *mu2 = m2;
    if (mu4) *mu4 = moments[2] / moments[0];
    if (a2) *a2 = m2 / (dx * dx);
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_lambda_from_moments(double mu2, double mu4, int32_t branch, double* lambda,
                                                double* r_out) {
    if (!lambda) return mdlg::fail(MDLG_EINVAL, "mdlg_lambda_from_moments: lambda is NULL");
    if (!(mu2 > 0.0) || !(mu4 >= 0.0) || !std::isfinite(mu2) || !std::isfinite(mu4))
        return mdlg::fail(MDLG_EINVAL, "mdlg_lambda_from_moments: need finite mu2 > 0, mu4 >= 0");
    if (branch != 1 && branch != 2)
        return mdlg::fail(MDLG_EINVAL, "mdlg_lambda_from_moments: branch must be 1 or 2");
    // mu4 = 3 mu2^2 (l^2 + 3 l + 1) / (l + 1)^2  <=>  (1 - r) l^2 + (3 - 2r) l + (1 - r) = 0,
    // r = mu4 / (3 mu2^2): roots l and 1/l, real for 1 <= r <= 5/4.
    double r = mu4 / (3.0 * mu2 * mu2);
    if (r_out) *r_out = r;
    if (r <= 1.0) {
        *lambda = 0.0;
        return MDLG_OK;
    }
    if (r >= 1.25) {
        *lambda = 1.0;
        return MDLG_OK;
    }
    // larger root without cancellation: (3 - 2r + sqrt(5 - 4r)) / (2 (r - 1))
    double big = (3.0 - 2.0 * r + std::sqrt(5.0 - 4.0 * r)) / (2.0 * (r - 1.0));
    *lambda = (branch == 2) ? big : 1.0 / big;
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_feq_gauss(double a2, const double* u, double* g_out) {
    if (!g_out) return mdlg::fail(MDLG_EINVAL, "mdlg_feq_gauss: g_out is NULL");
    if (!(a2 >= 0.0) || !std::isfinite(a2) || !finite_u(u))
        return mdlg::fail(MDLG_EINVAL, "mdlg_feq_gauss: need finite a2 >= 0 and finite u");
    for (int i = 0; i < MDLG_NQ; ++i) g_out[i] = 0.0;
    gauss2d(a2, u, 1.0, g_out);
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_feq_wsg(double a2, double lambda, const double* u, double* g_out) {
    if (!g_out) return mdlg::fail(MDLG_EINVAL, "mdlg_feq_wsg: g_out is NULL");
    if (!(a2 >= 0.0) || !std::isfinite(a2) || !(lambda >= 0.0) || !std::isfinite(lambda) || !finite_u(u))
        return mdlg::fail(MDLG_EINVAL, "mdlg_feq_wsg: need finite a2 >= 0, lambda >= 0 and finite u");
    if (lambda > 1e8) return mdlg::fail(MDLG_EINVAL, "mdlg_feq_wsg: lambda above 1e8");
    for (int i = 0; i < MDLG_NQ; ++i) g_out[i] = 0.0;
    if (lambda == 0.0) {
        gauss2d(a2, u, 1.0, g_out);
        return MDLG_OK;
    }
    // Poisson weights e^-l l^c / c! over the window holding all but < 1e-20 of the mass
    long lo = (long)std::floor(lambda - 12.0 * std::sqrt(lambda) - 10.0);
    if (lo < 0) lo = 0;
    long hi = (long)std::ceil(lambda + 12.0 * std::sqrt(lambda) + 40.0);
    double ll = std::log(lambda);
    for (long c = lo; c <= hi; ++c) {
        double w = std::exp((double)c * ll - lambda - std::lgamma((double)c + 1.0));
        if (w == 0.0) continue;
        gauss2d(a2 * ((double)c + 1.0) / (lambda + 1.0), u, w, g_out);
    }
    return MDLG_OK;
}

// ------------------------------------------------------ displacement PDF ---

namespace {

// Mass of N(mean, s^2) on [a, b) (a may be -inf, b +inf).  Each case keeps the
// erfc arguments non-negative, so tail bins keep their relative accuracy.
double normal_mass(double a, double b, double mean, double s) {
    const double za = (a - mean) / s * kInvSqrt2, zb = (b - mean) / s * kInvSqrt2;
    if (za >= 0.0) return 0.5 * (std::erfc(za) - std::erfc(zb));
    if (zb <= 0.0) return 0.5 * (std::erfc(-zb) - std::erfc(-za));
    return 1.0 - 0.5 * (std::erfc(-za) + std::erfc(zb));
}

// acc[k] += w * mass of bin k (k < n_bin), acc[n_bin] below, acc[n_bin + 1] above.
void normal_bins(double var, double mean, double h, int n_bin, double w, double* acc) {
    const double s = std::sqrt(var);
    const double half = 0.5 * (double)n_bin;
    double lo = (0.0 - half) * h;
    for (int k = 0; k < n_bin; ++k) {
        const double hi = ((double)(k + 1) - half) * h;
        acc[k] += w * normal_mass(lo, hi, mean, s);
        lo = hi;
    }
    acc[n_bin] += w * normal_mass(-INFINITY, (0.0 - half) * h, mean, s);
    acc[n_bin + 1] += w * normal_mass(((double)n_bin - half) * h, INFINITY, mean, s);
}

}  // namespace

extern "C" mdlg_status mdlg_pdf_bins(double msd, double lambda, double mean, double h, int32_t n_bin,
                                     double* p_gauss, double* p_wsg) {
    const char* who = "mdlg_pdf_bins: ";
    if (!p_gauss && !p_wsg) return mdlg::fail(MDLG_EINVAL, std::string(who) + "both outputs are NULL");
    if (!(msd > 0.0) || !std::isfinite(msd) || !(h > 0.0) || !std::isfinite(h) || !std::isfinite(mean) ||
        !(lambda >= 0.0) || !(lambda <= 1e8))
        return mdlg::fail(MDLG_EINVAL, std::string(who) + "need finite msd > 0, h > 0, mean and 0 <= lambda <= 1e8");
    if (n_bin < 1 || n_bin > MDLG_HIST_MAX_BINS)
        return mdlg::fail(MDLG_EINVAL, std::string(who) + "n_bin must be in [1, MDLG_HIST_MAX_BINS]");
    if (p_gauss) {
        for (int k = 0; k < n_bin + 2; ++k) p_gauss[k] = 0.0;
        normal_bins(msd, mean, h, n_bin, 1.0, p_gauss);
    }
    if (p_wsg) {
        for (int k = 0; k < n_bin + 2; ++k) p_wsg[k] = 0.0;
        if (lambda == 0.0) {
            normal_bins(msd, mean, h, n_bin, 1.0, p_wsg);
            return MDLG_OK;
        }
        // the Poisson window of mdlg_feq_wsg; component c has variance msd (c + 1) / (lambda + 1)
        long lo = (long)std::floor(lambda - 12.0 * std::sqrt(lambda) - 10.0);
        if (lo < 0) lo = 0;
        long hi = (long)std::ceil(lambda + 12.0 * std::sqrt(lambda) + 40.0);
        const double ll = std::log(lambda);
        for (long c = lo; c <= hi; ++c) {
            const double w = std::exp((double)c * ll - lambda - std::lgamma((double)c + 1.0));
            if (w == 0.0) continue;
            normal_bins(msd * ((double)c + 1.0) / (lambda + 1.0), mean, h, n_bin, w, p_wsg);
        }
    }
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_pdf_measured(const int64_t* hist, int32_t n_hist, int32_t n, double* p_out) {
    const char* who = "mdlg_pdf_measured: ";
    if (!hist || !p_out || n_hist < 1 || n < 1)
        return mdlg::fail(MDLG_EINVAL, std::string(who) + "NULL argument, n_hist < 1 or n < 1");
    int64_t total = 0;
    for (int k = 0; k < n; ++k) {
        int64_t s = 0;
        for (int j = 0; j < n_hist; ++j) {
            const int64_t c = hist[(int64_t)j * n + k];
            if (c < 0) return mdlg::fail(MDLG_EINVAL, std::string(who) + "negative count");
            s += c;
        }
        p_out[k] = (double)s;
        total += s;
    }
    if (total <= 0) return mdlg::fail(MDLG_EINVAL, std::string(who) + "empty histogram");
    for (int k = 0; k < n; ++k) p_out[k] /= (double)total;
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_kl_divergence(const double* r, const double* q, int32_t n, double* k_out,
                                          double* d_kl) {
    const char* who = "mdlg_kl_divergence: ";
    if (!r || !q || n < 1) return mdlg::fail(MDLG_EINVAL, std::string(who) + "NULL argument or n < 1");
    double s = 0.0, comp = 0.0;  // Neumaier-compensated sum in index order
    bool inf = false;
    for (int i = 0; i < n; ++i) {
        if (!(r[i] >= 0.0) || !std::isfinite(r[i]) || !(q[i] >= 0.0) || !std::isfinite(q[i]))
            return mdlg::fail(MDLG_EINVAL, std::string(who) + "probabilities must be finite and >= 0");
        double k;
        if (r[i] == 0.0) {
            k = 0.0;  // r log r -> 0
        } else if (q[i] == 0.0) {
            k = INFINITY;
            inf = true;
        } else {
            const double ratio = r[i] / q[i];
            k = (std::isnormal(ratio) && std::isfinite(ratio)) ? r[i] * std::log(ratio)
                                                                : r[i] * (std::log(r[i]) - std::log(q[i]));
        }
        if (k_out) k_out[i] = k;
        if (!inf) {
            const double t = s + k;
            comp += std::fabs(s) >= std::fabs(k) ? (s - t) + k : (k - t) + s;
            s = t;
        }
    }
    if (d_kl) *d_kl = inf ? INFINITY : s + comp;
    return MDLG_OK;
}
