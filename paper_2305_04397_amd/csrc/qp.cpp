// Projections of Alg. 1 (Sec. 3.3) on the host, FP64.
//
// With M = L L^T and y = L^T (x - t) (so ||x - t||_M = ||y||_2) both
// projections are least-distance problems  min ||z||_2  s.t.  G z >= h :
//   outer:  z minimising ||t - z||_M s.t. w'.z <= w'.r' for all (w', r'):
//           rows -(L^{-1} w')^T, right-hand sides w'.(t - r'); z = t + L^{-T} y.
//   inner:  x in down(conv Phi) minimising ||t - x||_M is t + L^{-T} y* where
//           y* is the minimum-norm point of conv{L^T (r_i - t)} + cone{-L^T e_k}.
//           A point y* of that set is minimal iff y*.v >= ||y*||^2 for every
//           point generator v and y*.g >= 0 for every ray g, so y* = z*/||z*||^2
//           with z* = argmin ||z|| s.t. v_i.z >= 1, g_k.z >= 0; that problem has
//           no solution exactly when t lies in down(Phi) (then x = t).  The
//           convex weights of the points are the normalised multipliers of
//           their constraints.
// Each least-distance problem is solved exactly (finite active-set steps) by
// the dual method of Goldfarb and Idnani (1983) for a unit Hessian: start at
// z = 0, add the most violated constraint, and keep the active constraint
// normals in a QR form N = J [R; 0] updated by Givens rotations.
#include "common.h"

#include <algorithm>
#include <cmath>

namespace morap {

namespace {

bool cholesky(std::vector<double>& A, int n) {
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(s > 0)) return false;
        const double d = std::sqrt(s);
        A[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = t / d;
        }
        for (int i = 0; i < j; ++i) A[(size_t)i * n + j] = 0.0;
    }
    return true;
}

// L (lower, row-major) solves
void lower_solve(const std::vector<double>& L, int n, double* b) {   // L b' = b
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * b[k];
        b[i] = t / L[(size_t)i * n + i];
    }
}
void lower_t_solve(const std::vector<double>& L, int n, double* b) { // L^T b' = b
    for (int i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * b[k];
        b[i] = t / L[(size_t)i * n + i];
    }
}

std::vector<double> factor_norm(const double* M, int d) {
    std::vector<double> L((size_t)d * d, 0.0);
    if (!M) {
        for (int i = 0; i < d; ++i) L[(size_t)i * d + i] = 1.0;
        return L;
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            const double a = M[(size_t)i * d + j], b = M[(size_t)j * d + i];
            MORAP_CHECK(std::isfinite(a), MORAP_E_INVALID, "M must be finite");
            MORAP_CHECK(std::fabs(a - b) <= 1e-12 * std::max(1.0, std::fabs(a)), MORAP_E_INVALID,
                        "M must be symmetric");
            L[(size_t)i * d + j] = a;
        }
    MORAP_CHECK(cholesky(L, d), MORAP_E_INVALID, "M must be positive definite");
    return L;
}

// min 1/2 ||z||^2 s.t. G z >= h (G: nc x n row-major).  Returns false when
// the constraints are inconsistent.  u receives the multipliers (nc) of the
// solution, or a certificate y >= 0 with G^T y = 0, h.y > 0 when there is none.
bool least_distance(const std::vector<double>& G, const std::vector<double>& h, int nc, int n,
                    std::vector<double>& z, std::vector<double>& u) {
    z.assign(n, 0.0);
    u.assign(nc, 0.0);
    std::vector<double> J((size_t)n * n, 0.0);   // column j at J[j*n ..] (column-major)
    for (int i = 0; i < n; ++i) J[(size_t)i * n + i] = 1.0;
    std::vector<double> R((size_t)n * n, 0.0);   // R[i*n + j], upper triangular q x q
    std::vector<int> act;                        // active constraint ids
    std::vector<double> ua;                      // their multipliers
    std::vector<double> d(n), zs(n), r(n);
    std::vector<char> is_act(nc, 0);
    std::vector<double> gnorm(nc);
    for (int i = 0; i < nc; ++i) {
        double s = 0;
        for (int k = 0; k < n; ++k) s += G[(size_t)i * n + k] * G[(size_t)i * n + k];
        gnorm[i] = std::sqrt(s);
    }
    // a zero normal with a positive right-hand side can never be met: y = e_i
    for (int i = 0; i < nc; ++i)
        if (gnorm[i] == 0.0 && h[i] > 0.0) {
            u[i] = 1.0;
            return false;
        }
    auto slack = [&](int i) {
        double s = -h[i];
        for (int k = 0; k < n; ++k) s += G[(size_t)i * n + k] * z[k];
        return s;
    };
    auto rot = [](double a, double b, double& c, double& s) {
        const double rho = std::hypot(a, b);
        if (rho == 0.0) {
            c = 1.0;
            s = 0.0;
        } else {
            c = a / rho;
            s = b / rho;
        }
        return rho;
    };
    auto rotate_cols = [&](int j0, int j1, double c, double s) {
        double* a = &J[(size_t)j0 * n];
        double* b = &J[(size_t)j1 * n];
        for (int k = 0; k < n; ++k) {
            const double x = a[k], y = b[k];
            a[k] = c * x + s * y;
            b[k] = -s * x + c * y;
        }
    };
    auto drop = [&](int l) {
        const int q = (int)act.size();
        // remove column l of R, then restore the triangle with row rotations
        for (int j = l; j < q - 1; ++j)
            for (int i = 0; i < q; ++i) R[(size_t)i * n + j] = R[(size_t)i * n + j + 1];
        for (int i = 0; i < q; ++i) R[(size_t)i * n + q - 1] = 0.0;
        for (int j = l; j < q - 1; ++j) {
            double c, s;
            R[(size_t)j * n + j] = rot(R[(size_t)j * n + j], R[(size_t)(j + 1) * n + j], c, s);
            R[(size_t)(j + 1) * n + j] = 0.0;
            for (int k = j + 1; k < q - 1; ++k) {
                const double x = R[(size_t)j * n + k], y = R[(size_t)(j + 1) * n + k];
                R[(size_t)j * n + k] = c * x + s * y;
                R[(size_t)(j + 1) * n + k] = -s * x + c * y;
            }
            rotate_cols(j, j + 1, c, s);
        }
        is_act[act[l]] = 0;
        act.erase(act.begin() + l);
        ua.erase(ua.begin() + l);
    };
    const int max_steps = 50 * (nc + n) + 100;
    for (int step = 0; step < max_steps; ++step) {
        // most violated constraint (scaled by its norm)
        int p = -1;
        double worst = 0.0;
        for (int i = 0; i < nc; ++i) {
            if (is_act[i] || gnorm[i] == 0.0) continue;
            const double s = slack(i);
            const double tol = 1e-13 * std::max(1.0, std::fabs(h[i]));
            if (s < -tol && s / gnorm[i] < worst) {
                worst = s / gnorm[i];
                p = i;
            }
        }
        if (p < 0) {
            for (size_t a = 0; a < act.size(); ++a) u[act[a]] = ua[a];
            return true;
        }
        double sp = slack(p);
        double up = 0.0;   // multiplier of p
        for (int inner = 0; inner < max_steps; ++inner) {
            const int q = (int)act.size();
            // d = J^T n_p
            for (int j = 0; j < n; ++j) {
                double s = 0;
                const double* col = &J[(size_t)j * n];
                for (int k = 0; k < n; ++k) s += col[k] * G[(size_t)p * n + k];
                d[j] = s;
            }
            // primal direction z_s = J2 d2, dual direction r = R^{-1} d1
            double zn = 0;
            for (int k = 0; k < n; ++k) {
                double s = 0;
                for (int j = q; j < n; ++j) s += J[(size_t)j * n + k] * d[j];
                zs[k] = s;
                zn += s * s;
            }
            zn = std::sqrt(zn);
            for (int i = q - 1; i >= 0; --i) {
                double s = d[i];
                for (int k = i + 1; k < q; ++k) s -= R[(size_t)i * n + k] * r[k];
                r[i] = s / R[(size_t)i * n + i];
            }
            double t1 = INFINITY;
            int l = -1;
            for (int i = 0; i < q; ++i)
                if (r[i] > 0 && ua[i] / r[i] < t1) {
                    t1 = ua[i] / r[i];
                    l = i;
                }
            double t2 = INFINITY;
            if (zn > 1e-12 * gnorm[p]) {
                double zg = 0;
                for (int k = 0; k < n; ++k) zg += zs[k] * G[(size_t)p * n + k];
                if (zg > 0) t2 = -sp / zg;
            }
            const double t = std::min(t1, t2);
            if (!std::isfinite(t)) {
                // n_p = N_A r with r <= 0 while the active constraints are
                // tight and p is violated: y = (1 for p, -r for the active
                // set) is a Farkas certificate, G^T y = 0 and h.y > 0
                std::fill(u.begin(), u.end(), 0.0);
                u[p] = 1.0;
                for (int i = 0; i < q; ++i) u[act[i]] = std::max(0.0, -r[i]);
                return false;
            }
            for (int i = 0; i < q; ++i) ua[i] -= t * r[i];
            up += t;
            if (std::isfinite(t2)) {
                for (int k = 0; k < n; ++k) z[k] += t * zs[k];
            }
            if (t == t2) {
                // add p: rotate d[q+1..n-1] into d[q]
                for (int j = n - 1; j > q; --j) {
                    double c, s;
                    d[j - 1] = rot(d[j - 1], d[j], c, s);
                    d[j] = 0.0;
                    rotate_cols(j - 1, j, c, s);
                }
                for (int i = 0; i <= q; ++i) R[(size_t)i * n + q] = d[i];
                act.push_back(p);
                ua.push_back(up);
                is_act[p] = 1;
                break;
            }
            // partial step: constraint l leaves the active set
            drop(l);
            sp = std::min(slack(p), 0.0);
        }
    }
    fail(MORAP_E_NOT_CONVERGED, "least-distance problem: too many active-set steps");
}

}  // namespace

void project_inner(const double* Phi, int m, int d, const double* t, const double* M, double* x, double* lam) {
    MORAP_CHECK(Phi && t && x && m >= 1 && d >= 1, MORAP_E_INVALID, "bad projection arguments");
    const auto L = factor_norm(M, d);
    // constraints: v_i = L^T (r_i - t) (>= 1), g_k = -L^T e_k (>= 0)
    const int nc = m + d;
    std::vector<double> G((size_t)nc * d, 0.0), h(nc, 0.0);
    for (int i = 0; i < m; ++i) {
        for (int c = 0; c < d; ++c) {
            double s = 0;
            for (int k = c; k < d; ++k) s += L[(size_t)k * d + c] * (Phi[(size_t)i * d + k] - t[k]);
            G[(size_t)i * d + c] = s;
        }
        h[i] = 1.0;
    }
    for (int k = 0; k < d; ++k)
        for (int c = 0; c < d; ++c) G[(size_t)(m + k) * d + c] = -L[(size_t)k * d + c];
    std::vector<double> z, u;
    if (!least_distance(G, h, nc, d, z, u)) {
        // t lies in down(Phi): it is its own projection, and the point part of
        // the certificate, normalised, is a convex combination dominating t
        std::copy(t, t + d, x);
        if (lam) {
            double s = 0;
            for (int i = 0; i < m; ++i) s += u[i];
            for (int i = 0; i < m; ++i) lam[i] = s > 0 ? u[i] / s : 1.0 / m;
        }
        return;
    }
    double zz = 0;
    for (double v : z) zz += v * v;
    std::vector<double> y(d);
    for (int c = 0; c < d; ++c) y[c] = z[c] / zz;
    lower_t_solve(L, d, y.data());   // L^{-T} y
    for (int k = 0; k < d; ++k) x[k] = t[k] + y[k];
    if (lam) {
        double s = 0;
        for (int i = 0; i < m; ++i) s += u[i];
        for (int i = 0; i < m; ++i) lam[i] = s > 0 ? u[i] / s : 1.0 / m;
    }
}

void project_outer(const double* W, const double* R, int nc, int d, const double* t, const double* M, double* z) {
    MORAP_CHECK(W && R && t && z && nc >= 1 && d >= 1, MORAP_E_INVALID, "bad projection arguments");
    const auto L = factor_norm(M, d);
    std::vector<double> G((size_t)nc * d), h(nc);
    bool any = false;
    std::vector<double> col(d);
    for (int l = 0; l < nc; ++l) {
        double hv = 0;
        for (int k = 0; k < d; ++k) {
            col[k] = W[(size_t)l * d + k];
            hv += W[(size_t)l * d + k] * (t[k] - R[(size_t)l * d + k]);
        }
        lower_solve(L, d, col.data());   // L^{-1} w'
        for (int k = 0; k < d; ++k) G[(size_t)l * d + k] = -col[k];
        h[l] = hv;
        any |= hv > 0;
    }
    if (!any) {
        std::copy(t, t + d, z);
        return;
    }
    std::vector<double> y, u;
    MORAP_CHECK(least_distance(G, h, nc, d, y, u), MORAP_E_NOT_CONVERGED, "outer approximation is empty");
    lower_t_solve(L, d, y.data());
    for (int k = 0; k < d; ++k) z[k] = t[k] + y[k];
}

}  // namespace morap
