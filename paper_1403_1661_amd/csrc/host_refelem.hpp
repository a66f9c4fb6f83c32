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

std::vector<double> gauss_lobatto(int N);
RefElement build_reference(int N);

}  // namespace dgswe
