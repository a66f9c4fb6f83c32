// Reference triangle of the nodal DG discretisation, built on the host in FP64.
//
// Section 3 of the paper: degree-N Lagrange polynomials on Warp & Blend
// interpolation nodes (the node family of the nodal DG book it cites).  With
// the volume and surface terms evaluated by collocation the solver needs the
// differentiation matrices Dr, Ds, the lift operator LIFT = M^{-1} E of the
// three faces, the cell-integral weights w = M 1, and linear-polynomial tools
// for the limiters of Section 5 (P1 projection evaluated at the edge
// midpoints, and the midpoint-Lagrange basis at the nodes).
//
// Numerics chosen for this library: orthonormal Jacobi polynomials by their
// three-term recurrence, Gauss-Lobatto-Legendre nodes by Newton iteration on
// P_N', Lagrange interpolation in barycentric form, dense inverses by
// Gauss-Jordan elimination with partial pivoting.
#include "host_refelem.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace dgswe {

namespace {

// Orthonormal Jacobi polynomial P_n^{(a,b)} and its derivative at x.
double jacobi(double x, double a, double b, int n) {
    const double g0 = std::exp((a + b + 1.0) * std::log(2.0) + std::lgamma(a + 1.0) +
                               std::lgamma(b + 1.0) - std::lgamma(a + b + 2.0));
    double pm1 = 1.0 / std::sqrt(g0);
    if (n == 0) return pm1;
    const double g1 = (a + 1.0) * (b + 1.0) / (a + b + 3.0) * g0;
    double p = ((a + b + 2.0) * x / 2.0 + (a - b) / 2.0) / std::sqrt(g1);
    if (n == 1) return p;
    // x p_k = c_{k+1} p_{k+1} + d_k p_k + c_k p_{k-1}
    auto c = [&](int k) {
        const double s = 2.0 * k + a + b;
        return 2.0 / s * std::sqrt(k * (k + a + b) * (k + a) * (k + b) / ((s - 1.0) * (s + 1.0)));
    };
    auto d = [&](int k) {
        const double s = 2.0 * k + a + b;
        return (b * b - a * a) / (s * (s + 2.0));
    };
    for (int k = 1; k < n; ++k) {
        const double pn = ((x - d(k)) * p - c(k) * pm1) / c(k + 1);
        pm1 = p;
        p = pn;
    }
    return p;
}

double jacobi_deriv(double x, double a, double b, int n) {
    if (n == 0) return 0.0;
    return std::sqrt(n * (n + a + b + 1.0)) * jacobi(x, a + 1.0, b + 1.0, n - 1);
}

// Legendre P_n and P_n' (classical normalisation) at x.
void legendre(int n, double x, double& p, double& dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    p = p1;
    dp = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.0;
}

Mat inverse(const Mat& A) {
    const int n = A.rows;
    Mat a = A, inv = Mat::identity(n);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a(r, c)) > std::fabs(a(piv, c))) piv = r;
        if (a(piv, c) == 0.0) throw std::runtime_error("singular matrix in reference element");
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a(c, k), a(piv, k));
                std::swap(inv(c, k), inv(piv, k));
            }
        const double d = a(c, c);
        for (int k = 0; k < n; ++k) { a(c, k) /= d; inv(c, k) /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a(r, c);
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) { a(r, k) -= f * a(c, k); inv(r, k) -= f * inv(c, k); }
        }
    }
    return inv;
}

// Collapsed coordinates of the reference triangle.
void collapse(double r, double s, double& a, double& b) {
    a = (std::fabs(1.0 - s) > 1e-14) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
    b = s;
}

double mode(double r, double s, int i, int j) {
    double a, b;
    collapse(r, s, a, b);
    return std::sqrt(2.0) * jacobi(a, 0, 0, i) * jacobi(b, 2.0 * i + 1.0, 0, j) *
           std::pow(1.0 - b, i);
}

void mode_grad(double r, double s, int i, int j, double& dr, double& ds) {
    double a, b;
    collapse(r, s, a, b);
    const double fa = jacobi(a, 0, 0, i), dfa = jacobi_deriv(a, 0, 0, i);
    const double gb = jacobi(b, 2.0 * i + 1.0, 0, j), dgb = jacobi_deriv(b, 2.0 * i + 1.0, 0, j);
    // psi = sqrt2 f(a) g(b) (1-b)^i, da/dr = 2/(1-b), da/ds = (1+a)/(1-b)
    if (i == 0) {
        dr = 0.0;
        ds = fa * dgb;
    } else {
        const double om = 1.0 - b;
        const double omi1 = std::pow(om, i - 1);
        dr = 2.0 * dfa * gb * omi1;
        ds = dfa * gb * (1.0 + a) * omi1 + fa * dgb * omi1 * om - i * fa * gb * omi1;
    }
    dr *= std::sqrt(2.0);
    ds *= std::sqrt(2.0);
}

// Gauss points and weights of the weight (1-x)^a (1+x)^b on [-1, 1]: roots
// of the orthonormal Jacobi polynomial of degree q by Newton iteration with
// the roots already found divided out, weights from the Christoffel numbers
// w_i = 1 / sum_{k<q} p_k(x_i)^2 of the orthonormal family.
void gauss_jacobi(int q, double a, double b, std::vector<double>& x, std::vector<double>& w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int i = 0; i < q; ++i) {
        double t = -std::cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 200; ++it) {
            const double f = jacobi(t, a, b, q), df = jacobi_deriv(t, a, b, q);
            double defl = 0.0;
            for (int j = 0; j < i; ++j) defl += 1.0 / (t - x[j]);
            const double dt = f / (df - f * defl);
            t -= dt;
            if (std::fabs(dt) < 1e-16 * std::max(1.0, std::fabs(t))) break;
        }
        x[i] = t;
    }
    std::sort(x.begin(), x.end());
    for (int i = 0; i < q; ++i) {
        double sum = 0.0;
        for (int k = 0; k < q; ++k) {
            const double p = jacobi(x[i], a, b, k);
            sum += p * p;
        }
        w[i] = 1.0 / sum;
    }
}

}  // namespace

std::vector<double> gauss_lobatto(int N) {
    std::vector<double> x(N + 1);
    x[0] = -1.0;
    x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double t = -std::cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, t, p, dp);
            // (1 - t^2) P'' = 2 t P' - N(N+1) P
            const double d2 = (2.0 * t * dp - N * (N + 1.0) * p) / (1.0 - t * t);
            const double dt = dp / d2;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[j] = t;
    }
    for (int j = 0; j <= N / 2; ++j) {  // exact symmetry
        const double m = 0.5 * (x[N - j] - x[j]);
        x[j] = -m;
        x[N - j] = m;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    return x;
}

// Warp function: displacement of the equidistant edge nodes onto the GLL
// nodes, interpolated at t in barycentric form, divided by 1 - t^2.
static double warp(int N, double t, const std::vector<double>& gll) {
    if (std::fabs(t) >= 1.0 - 1e-10) return 0.0;
    std::vector<double> xe(N + 1), wb(N + 1);
    for (int i = 0; i <= N; ++i) xe[i] = -1.0 + 2.0 * i / N;
    for (int i = 0; i <= N; ++i) {
        double p = 1.0;
        for (int k = 0; k <= N; ++k)
            if (k != i) p *= (xe[i] - xe[k]);
        wb[i] = 1.0 / p;
    }
    double num = 0.0, den = 0.0;
    for (int i = 0; i <= N; ++i) {
        const double d = t - xe[i];
        if (d == 0.0) return (gll[i] - xe[i]) / (1.0 - t * t);
        num += wb[i] / d * (gll[i] - xe[i]);
        den += wb[i] / d;
    }
    return num / den / (1.0 - t * t);
}

static const double kAlphaOpt[15] = {0.0,    0.0,    1.4152, 0.1001, 0.2751,
                                     0.9800, 1.0999, 1.2832, 1.3648, 1.4773,
                                     1.4959, 1.5743, 1.5770, 1.6223, 1.6258};

RefElement build_reference(int N) {
    if (N < 1 || N > 10) throw std::invalid_argument("N must be in 1..10");
    RefElement re;
    re.N = N;
    re.Np = (N + 1) * (N + 2) / 2;
    re.Nfp = N + 1;
    const int Np = re.Np, Nfp = re.Nfp;
    const double alpha = N <= 15 ? kAlphaOpt[N - 1] : 5.0 / 3.0;
    const std::vector<double> gll = gauss_lobatto(N);
    re.r.resize(Np);
    re.s.resize(Np);
    // equilateral triangle with vertices (-1,-1/sqrt3), (1,-1/sqrt3), (0,2/sqrt3)
    int n = 0;
    const double sq3 = std::sqrt(3.0);
    for (int row = 0; row <= N; ++row) {
        for (int col = 0; col <= N - row; ++col, ++n) {
            const double L1 = double(row) / N, L3 = double(col) / N, L2 = 1.0 - L1 - L3;
            double x = -L2 + L3, y = (-L2 - L3 + 2.0 * L1) / sq3;
            const double w1 = 4.0 * L2 * L3 * warp(N, L3 - L2, gll) * (1.0 + (alpha * L1) * (alpha * L1));
            const double w2 = 4.0 * L1 * L3 * warp(N, L1 - L3, gll) * (1.0 + (alpha * L2) * (alpha * L2));
            const double w3 = 4.0 * L1 * L2 * warp(N, L2 - L1, gll) * (1.0 + (alpha * L3) * (alpha * L3));
            x += w1 + std::cos(2.0 * M_PI / 3.0) * w2 + std::cos(4.0 * M_PI / 3.0) * w3;
            y += std::sin(2.0 * M_PI / 3.0) * w2 + std::sin(4.0 * M_PI / 3.0) * w3;
            const double l1 = (sq3 * y + 1.0) / 3.0;
            const double l2 = (-3.0 * x - sq3 * y + 2.0) / 6.0;
            const double l3 = (3.0 * x - sq3 * y + 2.0) / 6.0;
            re.r[n] = -l2 + l3 - l1;
            re.s[n] = -l2 - l3 + l1;
        }
    }
    // modes (i, j) with i + j <= N, i outer
    std::vector<std::pair<int, int>> modes;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j) modes.push_back({i, j});
    Mat V(Np, Np), Vr(Np, Np), Vs(Np, Np);
    for (int p = 0; p < Np; ++p)
        for (int m = 0; m < Np; ++m) {
            V(p, m) = mode(re.r[p], re.s[p], modes[m].first, modes[m].second);
            mode_grad(re.r[p], re.s[p], modes[m].first, modes[m].second, Vr(p, m), Vs(p, m));
        }
    const Mat Vinv = inverse(V);
    re.Dr = Vr * Vinv;
    re.Ds = Vs * Vinv;
    re.M = Vinv.transpose() * Vinv;
    // faces in counter-clockwise traversal: f0 s=-1 (r up), f1 r+s=0 (s up), f2 r=-1 (s down)
    re.fmask.assign(3 * Nfp, -1);
    std::vector<std::pair<double, int>> f[3];
    for (int p = 0; p < Np; ++p) {
        if (std::fabs(re.s[p] + 1.0) < 1e-10) f[0].push_back({re.r[p], p});
        if (std::fabs(re.r[p] + re.s[p]) < 1e-10) f[1].push_back({re.s[p], p});
        if (std::fabs(re.r[p] + 1.0) < 1e-10) f[2].push_back({-re.s[p], p});
    }
    for (int k = 0; k < 3; ++k) {
        if ((int)f[k].size() != Nfp) throw std::runtime_error("face node detection failed");
        std::sort(f[k].begin(), f[k].end());
        for (int j = 0; j < Nfp; ++j) re.fmask[k * Nfp + j] = f[k][j].second;
    }
    // 1D mass matrix on the GLL face nodes
    Mat V1(Nfp, Nfp);
    for (int a = 0; a < Nfp; ++a)
        for (int m = 0; m < Nfp; ++m) V1(a, m) = jacobi(gll[a], 0, 0, m);
    const Mat V1i = inverse(V1);
    const Mat M1 = V1i.transpose() * V1i;
    Mat E(Np, 3 * Nfp);
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < Nfp; ++a)
            for (int b = 0; b < Nfp; ++b) E(re.fmask[k * Nfp + a], k * Nfp + b) = M1(a, b);
    re.LIFT = V * (V.transpose() * E);
    re.w.assign(Np, 0.0);
    for (int p = 0; p < Np; ++p)
        for (int q = 0; q < Np; ++q) re.w[p] += re.M(p, q);
    // P1 projection (modes (0,0), (0,1), (1,0)) evaluated at the face midpoints
    const double mid[3][2] = {{0.0, -1.0}, {0.0, 0.0}, {-1.0, 0.0}};
    int lin[3] = {-1, -1, -1};
    for (int m = 0; m < Np; ++m) {
        if (modes[m] == std::make_pair(0, 0)) lin[0] = m;
        if (modes[m] == std::make_pair(0, 1)) lin[1] = m;
        if (modes[m] == std::make_pair(1, 0)) lin[2] = m;
    }
    re.p1_mid = Mat(3, Np);
    for (int e = 0; e < 3; ++e)
        for (int p = 0; p < Np; ++p) {
            double acc = 0.0;
            for (int t = 0; t < 3; ++t)
                acc += mode(mid[e][0], mid[e][1], modes[lin[t]].first, modes[lin[t]].second) *
                       Vinv(lin[t], p);
            re.p1_mid(e, p) = acc;
        }
    // midpoint-Lagrange P1 basis at the nodes: phi_i = 1 - 2 lambda_(vertex opposite edge i)
    re.phi_mid = Mat(3, Np);
    for (int p = 0; p < Np; ++p) {
        const double lam[3] = {-(re.r[p] + re.s[p]) / 2.0, (1.0 + re.r[p]) / 2.0,
                               (1.0 + re.s[p]) / 2.0};
        for (int e = 0; e < 3; ++e) re.phi_mid(e, p) = 1.0 - 2.0 * lam[(e + 2) % 3];
    }
    return re;
}

OverInt build_overint(const RefElement& re) {
    const int N = re.N, Np = re.Np, Nfp = re.Nfp;
    OverInt oi;
    oi.q = (3 * N + 2) / 2;
    const int q = oi.q;
    oi.Ncub = q * q;
    oi.NG = q;
    std::vector<double> xa, wa, xb, wb;
    gauss_jacobi(q, 0.0, 0.0, xa, wa);
    gauss_jacobi(q, 1.0, 0.0, xb, wb);
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            oi.rc.push_back(0.5 * (1.0 + xa[i]) * (1.0 - xb[j]) - 1.0);
            oi.sc.push_back(xb[j]);
            oi.wc.push_back(0.5 * wa[i] * wb[j]);
        }
    oi.xg = xa;
    oi.wg = wa;
    std::vector<std::pair<int, int>> modes;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j) modes.push_back({i, j});
    Mat V(Np, Np);
    for (int p = 0; p < Np; ++p)
        for (int m = 0; m < Np; ++m) V(p, m) = mode(re.r[p], re.s[p], modes[m].first, modes[m].second);
    const Mat Vinv = inverse(V);
    const int Nc = oi.Ncub;
    Mat Vc(Nc, Np), Vrc(Nc, Np), Vsc(Nc, Np);
    for (int c = 0; c < Nc; ++c)
        for (int m = 0; m < Np; ++m) {
            Vc(c, m) = mode(oi.rc[c], oi.sc[c], modes[m].first, modes[m].second);
            mode_grad(oi.rc[c], oi.sc[c], modes[m].first, modes[m].second, Vrc(c, m), Vsc(c, m));
        }
    oi.Ic = Vc * Vinv;
    const Mat Drc = Vrc * Vinv, Dsc = Vsc * Vinv;
    const Mat Minv = inverse(re.M);
    Mat DrW = Drc.transpose(), DsW = Dsc.transpose(), IW = oi.Ic.transpose();   // Np x Nc
    for (int i = 0; i < Np; ++i)
        for (int c = 0; c < Nc; ++c) {
            DrW(i, c) *= oi.wc[c];
            DsW(i, c) *= oi.wc[c];
            IW(i, c) *= oi.wc[c];
        }
    oi.Pr = Minv * DrW;
    oi.Ps = Minv * DsW;
    oi.P = Minv * IW;
    // face-node Lagrange basis (GLL nodes) at the Gauss points, barycentric form
    const std::vector<double> gll = gauss_lobatto(N);
    std::vector<double> bw(Nfp, 1.0);
    for (int j = 0; j < Nfp; ++j)
        for (int k = 0; k < Nfp; ++k)
            if (k != j) bw[j] /= (gll[j] - gll[k]);
    oi.I1 = Mat(q, Nfp);
    for (int g = 0; g < q; ++g) {
        double den = 0.0;
        for (int j = 0; j < Nfp; ++j) den += bw[j] / (oi.xg[g] - gll[j]);
        for (int j = 0; j < Nfp; ++j) oi.I1(g, j) = bw[j] / (oi.xg[g] - gll[j]) / den;
    }
    // L^g = M^-1 E_g with E_g(node, f q + g) = sum_j I1(g, j) Wg(g) [node = fmask(f, j)]
    Mat Eg(Np, 3 * q);
    for (int f = 0; f < 3; ++f)
        for (int g = 0; g < q; ++g)
            for (int j = 0; j < Nfp; ++j) Eg(re.fmask[f * Nfp + j], f * q + g) += oi.I1(g, j) * oi.wg[g];
    oi.Lg = Minv * Eg;
    return oi;
}

}  // namespace dgswe
