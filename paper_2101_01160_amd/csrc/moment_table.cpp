// Displacement moments at new parameter points, without molecular dynamics:
// the Poisson-WSG closed form (Eq.(f_eq_wsg)) needs a^2 and lambda, which
// the method measures from a trajectory (Eq.(theory_a), Eq.(lambda_eq)).  A
// table fitted to the moments of the training runs supplies them wherever
// the surrogate network is used, so that its guard needs no trajectory.
//
// Fitted fields: y0 = ln a^2 and y1 = r = mu4 / (3 mu2^2), on a regular
// grid over the coordinates (phi, ln kT, ln(dt_cg/dx)).  The fit minimises
//     sum_s (sum_p B_p(c_s) y_p - y_s)^2 + w sum (second differences of y)^2
// with tensor-product hat functions B_p (multilinear interpolation between
// the nodes) and the second differences taken along each axis in node
// units, w = smooth * n / P.  The penalty fixes nodes that no sample
// touches (extending the fit linearly beyond the samples, up to the edges of
// a caller-given box) and vanishes for every multilinear function, which the
// fit therefore reproduces exactly.  ln a^2 is close to linear in the two
// logarithms in the ballistic limit (a^2 = kT (dt_cg/dx)^2 there).
#include <cmath>
#include <string>
#include <vector>

#include "mdlg_internal.h"

struct mdlg_moment_table {
    int dims[3];
    double lo[3], hi[3];
    int32_t branch;
    std::vector<double> y[2];  // node values, index (i0 * dims[1] + i1) * dims[2] + i2
};

namespace {

constexpr int kMaxNodes = 2048;

bool coords(const double* x, double c[3]) {
    if (!(x[1] > 0.0) || !(x[2] > 0.0) || !std::isfinite(x[0]) || !std::isfinite(x[1]) || !std::isfinite(x[2]))
        return false;
    c[0] = x[0];
    c[1] = std::log(x[1]);
    c[2] = std::log(x[2]);
    return true;
}

// Multilinear weights of coordinate c: the 8 (or fewer) nodes and weights;
// returns their number, or -1 when c lies outside the grid (beyond a relative 1e-9 of the
// span, which absorbs the rounding of the bounds themselves).
int stencil(const mdlg_moment_table* t, const double c[3], int idx[8], double w[8]) {
    int base[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double span = t->hi[a] - t->lo[a];
        const double eps = 1e-9 * (span > 0.0 ? span : std::fmax(1.0, std::fabs(t->lo[a])));
        if (c[a] < t->lo[a] - eps || c[a] > t->hi[a] + eps) return -1;
        if (t->dims[a] == 1) {
            base[a] = 0;
            f[a] = 0.0;
            continue;
        }
        double s = (c[a] - t->lo[a]) / span * (t->dims[a] - 1);
        s = std::fmin(std::fmax(s, 0.0), (double)(t->dims[a] - 1));
        int b = (int)std::floor(s);
        if (b > t->dims[a] - 2) b = t->dims[a] - 2;
        base[a] = b;
        f[a] = s - b;
    }
    int k = 0;
    for (int d0 = 0; d0 < (t->dims[0] > 1 ? 2 : 1); ++d0)
        for (int d1 = 0; d1 < (t->dims[1] > 1 ? 2 : 1); ++d1)
            for (int d2 = 0; d2 < (t->dims[2] > 1 ? 2 : 1); ++d2) {
                idx[k] = ((base[0] + d0) * t->dims[1] + (base[1] + d1)) * t->dims[2] + (base[2] + d2);
                w[k] = (t->dims[0] > 1 ? (d0 ? f[0] : 1.0 - f[0]) : 1.0) *
                       (t->dims[1] > 1 ? (d1 ? f[1] : 1.0 - f[1]) : 1.0) *
                       (t->dims[2] > 1 ? (d2 ? f[2] : 1.0 - f[2]) : 1.0);
                ++k;
            }
    return k;
}

// In-place Cholesky factorisation of the symmetric positive definite P x P
// matrix A (lower triangle used) and the solution of A x = b for nrhs
// right-hand sides stored column after column in b.  False if A is not
// numerically positive definite.
bool cholesky_solve(std::vector<double>& A, int P, std::vector<double>& b, int nrhs) {
    for (int j = 0; j < P; ++j) {
        double d = A[(size_t)j * P + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * P + k] * A[(size_t)j * P + k];
        if (!(d > 1e-300)) return false;
        d = std::sqrt(d);
        A[(size_t)j * P + j] = d;
        for (int i = j + 1; i < P; ++i) {
            double s = A[(size_t)i * P + j];
            const double* ri = &A[(size_t)i * P];
            const double* rj = &A[(size_t)j * P];
            for (int k = 0; k < j; ++k) s -= ri[k] * rj[k];
            A[(size_t)i * P + j] = s / d;
        }
    }
    for (int r = 0; r < nrhs; ++r) {
        double* x = &b[(size_t)r * P];
        for (int i = 0; i < P; ++i) {
            double s = x[i];
            for (int k = 0; k < i; ++k) s -= A[(size_t)i * P + k] * x[k];
            x[i] = s / A[(size_t)i * P + i];
        }
        for (int i = P - 1; i >= 0; --i) {
            double s = x[i];
            for (int k = i + 1; k < P; ++k) s -= A[(size_t)k * P + i] * x[k];
            x[i] = s / A[(size_t)i * P + i];
        }
    }
    return true;
}

}  // namespace

extern "C" void mdlg_moment_table_destroy(mdlg_moment_table* t) { delete t; }

extern "C" mdlg_status mdlg_moment_table_create(mdlg_moment_table** out, const double* samples, int64_t n,
                                                const int32_t* dims, const double* lo, const double* hi,
                                                double smooth, int32_t branch) {
    if (!out || !samples || !dims) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: NULL argument");
    *out = nullptr;
    if (n < 1) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: need at least one sample");
    if (branch != 1 && branch != 2) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: branch must be 1 or 2");
    if (!(smooth >= 0.0) || !std::isfinite(smooth))
        return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: smooth must be finite and >= 0");
    long P = 1;
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < 1 || dims[a] > 64) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: dims in [1, 64]");
        P *= dims[a];
    }
    if (P > kMaxNodes) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: more than 2048 nodes");
    auto* t = new mdlg_moment_table();
    t->branch = branch;
    for (int a = 0; a < 3; ++a) {
        t->dims[a] = dims[a];
        t->lo[a] = INFINITY;
        t->hi[a] = -INFINITY;
    }
    std::vector<double> cs((size_t)n * 3), ys((size_t)n * 2);
    for (int64_t s = 0; s < n; ++s) {
        const double* row = samples + s * 5;
        double c[3];
        if (!coords(row, c) || !(row[3] > 0.0) || !std::isfinite(row[3]) || !std::isfinite(row[4])) {
            delete t;
            return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: sample " + std::to_string(s) +
                                               " needs finite phi, kT > 0, dt_cg/dx > 0, a2 > 0 and finite r");
        }
        for (int a = 0; a < 3; ++a) {
            cs[(size_t)s * 3 + a] = c[a];
            t->lo[a] = std::fmin(t->lo[a], c[a]);
            t->hi[a] = std::fmax(t->hi[a], c[a]);
        }
        ys[(size_t)s * 2] = std::log(row[3]);
        ys[(size_t)s * 2 + 1] = row[4];
    }
    if ((lo == nullptr) != (hi == nullptr)) {
        delete t;
        return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: give both lo and hi, or neither");
    }
    if (lo) {
        // a caller-given box (the design's parameter range): it must hold every sample
        double clo[3], chi[3];
        if (!coords(lo, clo) || !coords(hi, chi)) {
            delete t;
            return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: lo and hi need finite phi, kT > 0, dt_cg/dx > 0");
        }
        for (int a = 0; a < 3; ++a) {
            const double eps = 1e-9 * std::fmax(chi[a] - clo[a], 1e-300);
            if (!(chi[a] >= clo[a]) || t->lo[a] < clo[a] - eps || t->hi[a] > chi[a] + eps) {
                delete t;
                return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: the box lo..hi must hold every sample");
            }
            t->lo[a] = clo[a];
            t->hi[a] = chi[a];
        }
    }
    for (int a = 0; a < 3; ++a)
        if (dims[a] > 1 && !(t->hi[a] > t->lo[a])) {
            delete t;
            return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: axis " + std::to_string(a) +
                                               " has no spread in the samples; give it one node");
        }
    // normal equations of the penalised least-squares fit
    std::vector<double> A((size_t)P * P, 0.0), b((size_t)2 * P, 0.0);
    for (int64_t s = 0; s < n; ++s) {
        int idx[8];
        double w[8];
        const int k = stencil(t, &cs[(size_t)s * 3], idx, w);
        for (int i = 0; i < k; ++i) {
            for (int j = 0; j < k; ++j) A[(size_t)idx[i] * P + idx[j]] += w[i] * w[j];
            b[idx[i]] += w[i] * ys[(size_t)s * 2];
            b[P + idx[i]] += w[i] * ys[(size_t)s * 2 + 1];
        }
    }
    const double pen = smooth * (double)n / (double)P;
    if (pen > 0.0) {
        const int stride[3] = {dims[1] * dims[2], dims[2], 1};
        for (int i0 = 0; i0 < dims[0]; ++i0)
            for (int i1 = 0; i1 < dims[1]; ++i1)
                for (int i2 = 0; i2 < dims[2]; ++i2) {
                    const int ii[3] = {i0, i1, i2};
                    const int p = i0 * stride[0] + i1 * stride[1] + i2;
                    for (int a = 0; a < 3; ++a) {
                        if (ii[a] == 0 || ii[a] == dims[a] - 1) continue;
                        const int q[3] = {p - stride[a], p, p + stride[a]};
                        const double c[3] = {1.0, -2.0, 1.0};
                        for (int u = 0; u < 3; ++u)
                            for (int v = 0; v < 3; ++v) A[(size_t)q[u] * P + q[v]] += pen * c[u] * c[v];
                    }
                }
    }
    if (!cholesky_solve(A, (int)P, b, 2)) {
        delete t;
        return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_create: the fit is singular (nodes no sample reaches; "
                                       "raise smooth or use fewer nodes)");
    }
    t->y[0].assign(b.begin(), b.begin() + P);
    t->y[1].assign(b.begin() + P, b.end());
    *out = t;
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_moment_table_eval(const mdlg_moment_table* t, const double* x, double* a2,
                                              double* lambda, double* r) {
    if (!t || !x) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_eval: NULL argument");
    double c[3];
    if (!coords(x, c)) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_eval: need finite phi, kT > 0, dt_cg/dx > 0");
    int idx[8];
    double w[8];
    const int k = stencil(t, c, idx, w);
    if (k < 0)
        return mdlg::fail(MDLG_ERANGE, "mdlg_moment_table_eval: (phi, kT, dt_cg/dx) outside the range of the table");
    double y0 = 0.0, y1 = 0.0;
    for (int i = 0; i < k; ++i) {
        y0 += w[i] * t->y[0][idx[i]];
        y1 += w[i] * t->y[1][idx[i]];
    }
    if (a2) *a2 = std::exp(y0);
    if (r) *r = y1;
    if (lambda) {
        // mu2 = 1, mu4 = 3 r: the ratio alone fixes lambda (Eq.(lambda_eq))
        mdlg_status s = mdlg_lambda_from_moments(1.0, std::fmax(3.0 * y1, 0.0), t->branch, lambda, nullptr);
        if (s != MDLG_OK) return s;
    }
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_moment_table_info(const mdlg_moment_table* t, int32_t* dims, double* lo, double* hi,
                                              double* nodes) {
    if (!t) return mdlg::fail(MDLG_EINVAL, "mdlg_moment_table_info: NULL handle");
    const size_t P = t->y[0].size();
    for (int a = 0; a < 3; ++a) {
        if (dims) dims[a] = t->dims[a];
        if (lo) lo[a] = t->lo[a];
        if (hi) hi[a] = t->hi[a];
    }
    if (nodes)
        for (size_t p = 0; p < P; ++p) {
            nodes[2 * p] = t->y[0][p];
            nodes[2 * p + 1] = t->y[1][p];
        }
    return MDLG_OK;
}
