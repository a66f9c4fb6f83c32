// Host-side dense matrices and the reference-triangle data of the DG solver.
#pragma once

#include <vector>

namespace dgswe {

struct Mat {
    int rows = 0, cols = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int r, int c) : rows(r), cols(c), a(size_t(r) * c, 0.0) {}
    static Mat identity(int n) {
        Mat m(n, n);
        for (int i = 0; i < n; ++i) m(i, i) = 1.0;
        return m;
    }
    double& operator()(int i, int j) { return a[size_t(i) * cols + j]; }
    double operator()(int i, int j) const { return a[size_t(i) * cols + j]; }
    Mat transpose() const {
        Mat t(cols, rows);
        for (int i = 0; i < rows; ++i)
            for (int j = 0; j < cols; ++j) t(j, i) = (*this)(i, j);
        return t;
    }
    Mat operator*(const Mat& b) const {
        Mat c(rows, b.cols);
        for (int i = 0; i < rows; ++i)
            for (int k = 0; k < cols; ++k) {
                const double v = (*this)(i, k);
                if (v == 0.0) continue;
                for (int j = 0; j < b.cols; ++j) c(i, j) += v * b(k, j);
            }
        return c;
    }
};

struct RefElement {
    int N = 0, Np = 0, Nfp = 0;
    std::vector<double> r, s;   // Warp & Blend nodes on (-1,-1),(1,-1),(-1,1)
    Mat Dr, Ds, M, LIFT;        // LIFT: Np x 3Nfp
    std::vector<int> fmask;     // 3 x Nfp, counter-clockwise face traversal
    std::vector<double> w;      // cell-integral weights, sum 2
    Mat p1_mid;                 // 3 x Np: P1 projection at the face midpoints
    Mat phi_mid;                // 3 x Np: midpoint-Lagrange P1 basis at the nodes
};

// Over-integrated weak-form operators (the cubature and Gauss rules of the
// paper's volume and surface integrals): rules exact to degree 3N with q =
// ceil((3N+1)/2) points per direction (cubature: Stroud's conical product of
// q Gauss-Legendre by q Gauss-Jacobi(1,0) points) and per face (Gauss-Legendre,
// counter-clockwise along the face).
struct OverInt {
    int q = 0, Ncub = 0, NG = 0;
    std::vector<double> rc, sc, wc;   // cubature nodes and weights (sum 2)
    std::vector<double> xg, wg;       // Gauss points and weights on [-1, 1]
    Mat Ic;                           // Ncub x Np: nodal basis at the cubature nodes
    Mat Pr, Ps, P;                    // Np x Ncub: M^-1 Dr_c^T W, M^-1 Ds_c^T W, M^-1 Ic^T W
    Mat I1;                           // NG x Nfp: face-node Lagrange basis at the Gauss points
    Mat Lg;                           // Np x 3NG: M^-1 [I_g0^T Wg, I_g1^T Wg, I_g2^T Wg]
};

std::vector<double> gauss_lobatto(int N);
RefElement build_reference(int N);
OverInt build_overint(const RefElement& re);

}  // namespace dgswe
