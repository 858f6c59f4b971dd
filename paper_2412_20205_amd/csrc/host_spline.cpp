// Host-side univariate B-spline machinery (see host_spline.hpp).
#include "host_spline.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace igamg {

std::vector<double> open_knots(int ne, int p) {
    std::vector<double> t;
    t.reserve(ne + 2 * p + 1);
    for (int k = 0; k <= p; ++k) t.push_back(0.0);
    for (int e = 1; e < ne; ++e) t.push_back((double)e / ne);
    for (int k = 0; k <= p; ++k) t.push_back(1.0);
    return t;
}

void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < (m + 1) / 2; ++i) {
        // initial guess from the asymptotic node distribution
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            // three-term recurrence for P_m(z) and its derivative
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= m; ++k) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = m * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged node
        {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= m; ++k) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = m * (z * p0 - p1) / (z * z - 1.0);
        }
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (m % 2 == 1) x[m / 2] = 0.0;
}

void basis_and_derivs(const std::vector<double>& t, int p, int s, double u, double* N,
                      double* dN) {
    // ndu[j][r]: triangle of basis values of increasing degree j (p <= 9)
    double ndu[10][10], left[10], right[10];
    ndu[0][0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = u - t[s + 1 - j];
        right[j] = t[s + j] - u;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double den = right[r + 1] + left[j - r];
            double tmp = den != 0.0 ? ndu[j - 1][r] / den : 0.0;
            ndu[j][r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        ndu[j][j] = saved;
    }
    for (int r = 0; r <= p; ++r) N[r] = ndu[p][r];
    if (p == 0) {
        dN[0] = 0.0;
        return;
    }
    // derivative from the degree p-1 row: function s-p+r
    for (int r = 0; r <= p; ++r) {
        int f = s - p + r;
        double a = 0.0, b = 0.0;
        double dl = t[f + p] - t[f];
        double dr = t[f + p + 1] - t[f + 1];
        // N_f^{p-1} is entry r-1 of the degree p-1 row, N_{f+1}^{p-1} entry r
        if (r >= 1 && dl != 0.0) a = ndu[p - 1][r - 1] / dl;
        if (r <= p - 1 && dr != 0.0) b = ndu[p - 1][r] / dr;
        dN[r] = p * (a - b);
    }
}

static int find_span(const std::vector<double>& t, int p, int ne, double u) {
    // span index s with t[s] <= u < t[s+1]; u == 1 maps to the last element
    int s = p + (int)std::floor(u * ne);
    if (s > p + ne - 1) s = p + ne - 1;
    if (s < p) s = p;
    while (s < p + ne - 1 && u >= t[s + 1]) ++s;
    while (s > p && u < t[s]) --s;
    return s;
}

ElementTables element_tables(int ne, int p, int nq) {
    ElementTables T;
    T.ne = ne;
    T.nq = nq;
    T.p = p;
    std::vector<double> gx, gw;
    gauss_legendre(nq, gx, gw);
    std::vector<double> t = open_knots(ne, p);
    T.pts.resize((size_t)ne * nq);
    T.wts.resize((size_t)ne * nq);
    T.V.resize((size_t)ne * nq * (p + 1));
    T.D.resize((size_t)ne * nq * (p + 1));
    for (int e = 0; e < ne; ++e) {
        double a = (double)e / ne, b = (double)(e + 1) / ne;
        for (int q = 0; q < nq; ++q) {
            double u = 0.5 * (a + b) + 0.5 * (b - a) * gx[q];
            T.pts[e * nq + q] = u;
            T.wts[e * nq + q] = 0.5 * (b - a) * gw[q];
            basis_and_derivs(t, p, p + e, u, &T.V[((size_t)e * nq + q) * (p + 1)],
                             &T.D[((size_t)e * nq + q) * (p + 1)]);
        }
    }
    return T;
}

void eval_at_points(int ne, int p, const std::vector<double>& x, std::vector<int>& span,
                    std::vector<double>& V, std::vector<double>& D) {
    std::vector<double> t = open_knots(ne, p);
    span.resize(x.size());
    V.resize(x.size() * (p + 1));
    D.resize(x.size() * (p + 1));
    for (size_t k = 0; k < x.size(); ++k) {
        int s = find_span(t, p, ne, x[k]);
        span[k] = s - p;  // element index
        basis_and_derivs(t, p, s, x[k], &V[k * (p + 1)], &D[k * (p + 1)]);
    }
}

Prolong1D prolongation_boehm(int nc_el, int p) {
    Prolong1D P;
    P.nc_el = nc_el;
    P.p = p;
    P.nc_fun = nc_el + p;
    P.nf_fun = 2 * nc_el + p;
    std::vector<double> t = open_knots(nc_el, p);
    // each coarse function starts as a unit coefficient vector
    P.col_start.resize(P.nc_fun);
    P.col_val.resize(P.nc_fun);
    for (int J = 0; J < P.nc_fun; ++J) {
        P.col_start[J] = J;
        P.col_val[J] = {1.0};
    }
    for (int e = 0; e < nc_el; ++e) {
        double u = (2.0 * e + 1.0) / (2.0 * nc_el);
        // span k in the current knot vector: t[k] <= u < t[k+1]
        int k = (int)(std::upper_bound(t.begin(), t.end(), u) - t.begin()) - 1;
        for (int J = 0; J < P.nc_fun; ++J) {
            int s = P.col_start[J];
            std::vector<double>& v = P.col_val[J];
            int last = s + (int)v.size() - 1;
            if (last < k - p) continue;          // entirely before the change
            if (s > k) {                          // entirely after: index shift
                P.col_start[J] = s + 1;
                continue;
            }
            auto old = [&](int i) { return (i >= s && i <= last) ? v[i - s] : 0.0; };
            int ns = std::max(0, s), ne2 = last + 1;
            std::vector<double> q(ne2 - ns + 1, 0.0);
            for (int i = ns; i <= ne2; ++i) {
                double val;
                if (i <= k - p) {
                    val = old(i);
                } else if (i <= k) {
                    double den = t[i + p] - t[i];
                    double al = den > 0.0 ? (u - t[i]) / den : 0.0;
                    val = al * old(i) + (1.0 - al) * old(i - 1);
                } else {
                    val = old(i - 1);
                }
                q[i - ns] = val;
            }
            // trim exact zeros at both ends
            int a = 0, b = (int)q.size() - 1;
            while (a < b && q[a] == 0.0) ++a;
            while (b > a && q[b] == 0.0) --b;
            P.col_start[J] = ns + a;
            v.assign(q.begin() + a, q.begin() + b + 1);
        }
        t.insert(t.begin() + k + 1, u);
    }
    return P;
}

TransferTables transfer_tables(const Prolong1D& P) {
    TransferTables T;
    T.nf = P.nf_fun - 2;
    T.nc = P.nc_fun - 2;
    // interior columns J = 1 .. nc_fun-2; interior rows i = 1 .. nf_fun-2
    int RW = 0;
    std::vector<std::vector<std::pair<int, double>>> rows(T.nf);
    for (int J = 1; J <= P.nc_fun - 2; ++J) {
        int s = P.col_start[J];
        const auto& v = P.col_val[J];
        for (size_t a = 0; a < v.size(); ++a) {
            int i = s + (int)a;
            if (i < 1 || i > P.nf_fun - 2) {
                if (v[a] != 0.0 && (i == 0 || i == P.nf_fun - 1))
                    throw std::runtime_error("interior coarse function touches a Dirichlet fine function");
                continue;
            }
            if (v[a] != 0.0) rows[i - 1].push_back({J - 1, v[a]});
        }
        RW = std::max(RW, (int)v.size());
    }
    T.RW = std::max(RW, 1);
    int PW = 1;
    for (auto& r : rows) {
        if (!r.empty()) PW = std::max(PW, r.back().first - r.front().first + 1);
    }
    T.PW = PW;
    T.r_start.assign(T.nc, 0);
    T.r_w.assign((size_t)T.nc * T.RW, 0.0);
    for (int J = 1; J <= P.nc_fun - 2; ++J) {
        int I = J - 1;
        int s = P.col_start[J] - 1;  // interior fine index of the first entry
        int st = std::min(std::max(s, 0), std::max(T.nf - T.RW, 0));
        T.r_start[I] = st;
        const auto& v = P.col_val[J];
        for (size_t a = 0; a < v.size(); ++a) {
            int i = s + (int)a;
            if (i < 0 || i >= T.nf) continue;
            int slot = i - st;
            if (slot < 0 || slot >= T.RW) throw std::runtime_error("restriction window");
            T.r_w[(size_t)I * T.RW + slot] = v[a];
        }
    }
    T.p_start.assign(T.nf, 0);
    T.p_w.assign((size_t)T.nf * T.PW, 0.0);
    for (int i = 0; i < T.nf; ++i) {
        if (rows[i].empty()) continue;
        int s = rows[i].front().first;
        int st = std::min(std::max(s, 0), std::max(T.nc - T.PW, 0));
        T.p_start[i] = st;
        for (auto& e : rows[i]) {
            int slot = e.first - st;
            if (slot < 0 || slot >= T.PW) throw std::runtime_error("prolongation window");
            T.p_w[(size_t)i * T.PW + slot] = e.second;
        }
    }
    return T;
}

void stiffness_mass_bands(int ne, int p, Band1D& K, Band1D& M) {
    ElementTables E = element_tables(ne, p, p + 1);
    int n = ne + p - 2, W = 2 * p + 1;
    K.n = M.n = n;
    K.p = M.p = p;
    K.v.assign((size_t)n * W, 0.0);
    M.v.assign((size_t)n * W, 0.0);
    for (int e = 0; e < ne; ++e)
        for (int q = 0; q < p + 1; ++q) {
            double w = E.wts[e * (p + 1) + q];
            const double* V = &E.V[((size_t)e * (p + 1) + q) * (p + 1)];
            const double* D = &E.D[((size_t)e * (p + 1) + q) * (p + 1)];
            for (int a = 0; a <= p; ++a) {
                int i = e + a - 1;
                if (i < 0 || i >= n) continue;
                for (int b = 0; b <= p; ++b) {
                    int j = e + b - 1;
                    if (j < 0 || j >= n) continue;
                    K.v[(size_t)i * W + (j - i) + p] += w * D[a] * D[b];
                    M.v[(size_t)i * W + (j - i) + p] += w * V[a] * V[b];
                }
            }
        }
}

Band1D galerkin_band(const Band1D& Af, const TransferTables& T, int p) {
    Band1D Ac;
    Ac.n = T.nc;
    Ac.p = p;
    int W = 2 * p + 1;
    Ac.v.assign((size_t)T.nc * W, 0.0);
    for (int I = 0; I < T.nc; ++I)
        for (int d = -p; d <= p; ++d) {
            int J = I + d;
            if (J < 0 || J >= T.nc) continue;
            double s = 0.0;
            for (int a = 0; a < T.RW; ++a) {
                int i = T.r_start[I] + a;
                double wi = T.r_w[(size_t)I * T.RW + a];
                if (wi == 0.0) continue;
                for (int b = 0; b < T.RW; ++b) {
                    int j = T.r_start[J] + b;
                    double wj = T.r_w[(size_t)J * T.RW + b];
                    if (wj == 0.0) continue;
                    int dd = j - i;
                    if (dd < -p || dd > p) continue;
                    s += wi * Af.at(i, dd) * wj;
                }
            }
            Ac.v[(size_t)I * W + d + p] = s;
        }
    return Ac;
}

bool cholesky_inplace(std::vector<double>& A, int n) {
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        A[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = s / d;
        }
        for (int i = 0; i < j; ++i) A[(size_t)i * n + j] = 0.0;
    }
    return true;
}

std::vector<double> inverse_from_cholesky(const std::vector<double>& L, int n) {
    // solve L L^T X = I column by column
    std::vector<double> X((size_t)n * n, 0.0), y(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * X[(size_t)k * n + c];
            X[(size_t)i * n + c] = s / L[(size_t)i * n + i];
        }
    }
    return X;
}

bool inverse_lu(const std::vector<double>& A, int n, std::vector<double>& inv) {
    std::vector<double> M(A);
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    double scale = 0.0;
    for (double v : A) scale = std::max(scale, std::fabs(v));
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(M[(size_t)i * n + k]) > std::fabs(M[(size_t)piv * n + k])) piv = i;
        const double d = M[(size_t)piv * n + k];
        if (!(std::fabs(d) > 1e-14 * scale)) return false;
        if (piv != k)
            for (int j = 0; j < n; ++j) {
                std::swap(M[(size_t)k * n + j], M[(size_t)piv * n + j]);
                std::swap(inv[(size_t)k * n + j], inv[(size_t)piv * n + j]);
            }
        for (int j = 0; j < n; ++j) {
            M[(size_t)k * n + j] /= d;
            inv[(size_t)k * n + j] /= d;
        }
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            const double f = M[(size_t)i * n + k];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
                inv[(size_t)i * n + j] -= f * inv[(size_t)k * n + j];
            }
        }
    }
    return true;
}

int coarse_inverse(std::vector<double> A, int n, bool symmetric, std::vector<double>& inv) {
    if (!symmetric) {
        std::vector<double> r;
        if (!inverse_lu(A, n, r)) return -4;
        inv.swap(r);
        return 0;
    }
    if (!cholesky_inplace(A, n)) return -4;
    inv = inverse_from_cholesky(A, n);
    return 0;
}

}  // namespace igamg

// ---------------------------------------------------------------------------
// host-only C entry points (include/igamg_host.h)

#include "../../include/igamg_host.h"

extern "C" {

int igamg_host_gauss_legendre(int m, double* x, double* w) {
    if (m < 1 || !x || !w) return -1;
    std::vector<double> xs, ws;
    igamg::gauss_legendre(m, xs, ws);
    for (int i = 0; i < m; ++i) {
        x[i] = xs[i];
        w[i] = ws[i];
    }
    return 0;
}

int igamg_host_basis(int ne, int p, double u, double* N, double* dN, int* first) {
    if (ne < 1 || p < 0 || p > 9 || !N || !dN || !first || !(u >= 0.0 && u <= 1.0)) return -1;
    std::vector<int> span;
    std::vector<double> V, D;
    igamg::eval_at_points(ne, p, std::vector<double>{u}, span, V, D);
    for (int a = 0; a <= p; ++a) {
        N[a] = V[a];
        dN[a] = D[a];
    }
    *first = span[0];
    return 0;
}

int igamg_host_prolongation_1d(int ne_coarse, int p, double* out) {
    if (ne_coarse < 1 || p < 1 || p > 9 || !out) return -1;
    igamg::Prolong1D P = igamg::prolongation_boehm(ne_coarse, p);
    for (size_t k = 0; k < (size_t)P.nf_fun * P.nc_fun; ++k) out[k] = 0.0;
    for (int J = 0; J < P.nc_fun; ++J)
        for (size_t a = 0; a < P.col_val[J].size(); ++a)
            out[(size_t)(P.col_start[J] + (int)a) * P.nc_fun + J] = P.col_val[J][a];
    return 0;
}

int igamg_host_bands(int ne, int ne_coarsest, int level, int p, double* K, double* M) {
    if (ne < 1 || ne_coarsest < 1 || ne % ne_coarsest || p < 1 || p > 9 || !K || !M) return -1;
    int nlev = 1;
    for (int m = ne / ne_coarsest; m > 1; m /= 2) {
        if (m % 2) return -1;
        ++nlev;
    }
    if (level < 0 || level >= nlev) return -1;
    igamg::Band1D Kb, Mb;
    igamg::stiffness_mass_bands(ne, p, Kb, Mb);
    for (int l = nlev - 1, e = ne; l > level; --l, e /= 2) {
        igamg::TransferTables T = igamg::transfer_tables(igamg::prolongation_boehm(e / 2, p));
        Kb = igamg::galerkin_band(Kb, T, p);
        Mb = igamg::galerkin_band(Mb, T, p);
    }
    for (size_t k = 0; k < Kb.v.size(); ++k) {
        K[k] = Kb.v[k];
        M[k] = Mb.v[k];
    }
    return 0;
}

int igamg_host_coarse_inverse(int n, const double* A, int symmetric, double* inv) {
    if (n < 1 || !A || !inv) return -1;
    std::vector<double> M(A, A + (size_t)n * n), r;
    int st = igamg::coarse_inverse(std::move(M), n, symmetric != 0, r);
    if (st != 0) return st;
    std::copy(r.begin(), r.end(), inv);
    return 0;
}

}  // extern "C"
