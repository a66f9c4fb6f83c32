// Mesh setup on the host (FP64).
//
// * Connectivity of a conforming triangulation (Section 3): face f of an
//   element joins its vertices f and f+1; faces are matched through a hash of
//   the unordered vertex pair.  A face met a third time, or met twice with the
//   same orientation, is a mesh error; an unmatched face is a reflective wall.
// * Affine map x = -(r+s)/2 x1 + (1+r)/2 x2 + (1+s)/2 x3; outward normals from
//   the reference-face tangents, Fscale = sJ / J, inradius 2 J / sum(sJ) (the
//   element length H^k of Eq. 4.1).
// * Levels (Section 4): dt_k = CFL r_k / ((N+1)^2 a) with one global wave
//   speed, so level l_k = 1 + max{j : 2^j r_min <= r_k (1 + 1e-12)} capped at
//   the level count, then lowered to the fixed point l_k <= l_nbr + 1.
// * TVB stencil (Section 5.3 and the Cockburn-Shu limiter it cites): for
//   edge i, non-negative alpha_j, alpha_k with
//   m_i - b0 = alpha_j (b_j - b0) + alpha_k (b_k - b0); pairs tried in the
//   order (i,i+1), (i,i+2), (i+1,i+2); a wall neighbour's barycentre is b0
//   mirrored in the wall; fallback: the face neighbour alone scaled by
//   |m_i - b0| / |b_i - b0|.
#include "host_mesh.hpp"

#include <cmath>
#include <unordered_map>

namespace dgswe {

std::string build_host_mesh(int nv, const double* vx, const double* vy, int K,
                            const int32_t* etov, const int8_t* bc, HostMesh& m) {
    if (nv < 3 || K < 1 || !vx || !vy || !etov) return "empty or null mesh";
    m.K = K;
    m.Nv = nv;
    m.vx.assign(vx, vx + nv);
    m.vy.assign(vy, vy + nv);
    m.etov.assign(etov, etov + 3 * size_t(K));
    for (size_t i = 0; i < m.etov.size(); ++i)
        if (m.etov[i] < 0 || m.etov[i] >= nv)
            return "vertex index out of range in element " + std::to_string(i / 3);
    m.rx.resize(K); m.ry.resize(K); m.sx.resize(K); m.sy.resize(K); m.J.resize(K);
    m.nx.resize(3 * size_t(K)); m.ny.resize(3 * size_t(K));
    m.sJ.resize(3 * size_t(K)); m.fscale.resize(3 * size_t(K));
    m.inradius.resize(K); m.dk.resize(K);
    for (int k = 0; k < K; ++k) {
        const int a = m.etov[3 * k], b = m.etov[3 * k + 1], c = m.etov[3 * k + 2];
        if (a == b || b == c || a == c) return "element " + std::to_string(k) + " repeats a vertex";
        const double xr = 0.5 * (vx[b] - vx[a]), xs = 0.5 * (vx[c] - vx[a]);
        const double yr = 0.5 * (vy[b] - vy[a]), ys = 0.5 * (vy[c] - vy[a]);
        const double J = xr * ys - xs * yr;
        if (!(J > 0.0))
            return "element " + std::to_string(k) + " is clockwise or degenerate";
        m.J[k] = J;
        m.rx[k] = ys / J; m.ry[k] = -xs / J; m.sx[k] = -yr / J; m.sy[k] = xr / J;
        const double fnx[3] = {yr, ys - yr, -ys};
        const double fny[3] = {-xr, xr - xs, xs};
        double per = 0.0, longest = 0.0;
        for (int f = 0; f < 3; ++f) {
            const double sJ = std::sqrt(fnx[f] * fnx[f] + fny[f] * fny[f]);
            m.nx[3 * k + f] = fnx[f] / sJ;
            m.ny[3 * k + f] = fny[f] / sJ;
            m.sJ[3 * k + f] = sJ;
            m.fscale[3 * k + f] = sJ / J;
            per += sJ;
            longest = std::fmax(longest, 2.0 * sJ);
        }
        m.inradius[k] = 2.0 * J / per;
        m.dk[k] = longest;
    }
    // face matching
    m.etoe.resize(3 * size_t(K));
    m.etof.resize(3 * size_t(K));
    m.wall.assign(3 * size_t(K), 1);
    std::unordered_map<uint64_t, int64_t> open;
    open.reserve(size_t(K) * 2);
    std::vector<uint8_t> closed_use(3 * size_t(K), 0);
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < 3; ++f) {
            m.etoe[3 * k + f] = k;
            m.etof[3 * k + f] = int8_t(f);
        }
    std::unordered_map<uint64_t, int> closed;
    for (int k = 0; k < K; ++k) {
        for (int f = 0; f < 3; ++f) {
            const int64_t a = m.etov[3 * k + f], b = m.etov[3 * k + (f + 1) % 3];
            const uint64_t key = uint64_t(std::min(a, b)) * uint64_t(nv) + uint64_t(std::max(a, b));
            if (closed.count(key)) return "a face is shared by more than two elements";
            auto it = open.find(key);
            if (it == open.end()) {
                open.emplace(key, int64_t(k) * 3 + f);
                continue;
            }
            const int k2 = int(it->second / 3), f2 = int(it->second % 3);
            open.erase(it);
            const int a2 = m.etov[3 * k2 + f2], b2 = m.etov[3 * k2 + (f2 + 1) % 3];
            if (!(a2 == b && b2 == a))
                return "elements " + std::to_string(k2) + " and " + std::to_string(k) +
                       " traverse a shared face the same way";
            m.etoe[3 * k + f] = k2; m.etof[3 * k + f] = int8_t(f2);
            m.etoe[3 * k2 + f2] = k; m.etof[3 * k2 + f2] = int8_t(f);
            m.wall[3 * k + f] = 0;
            m.wall[3 * k2 + f2] = 0;
            closed.emplace(key, 1);
        }
    }
    // tagged walls: a shared face tagged on either side becomes a wall on both
    if (bc) {
        for (int k = 0; k < K; ++k)
            for (int f = 0; f < 3; ++f) {
                const int8_t t = bc[3 * k + f];
                if (t != 0 && t != 1) return "boundary tag of element " + std::to_string(k) + " is not 0 or 1";
                if (t == 0 || m.wall[3 * k + f]) continue;
                const int k2 = m.etoe[3 * k + f], f2 = m.etof[3 * k + f];
                m.etoe[3 * k + f] = k; m.etof[3 * k + f] = int8_t(f); m.wall[3 * k + f] = 1;
                m.etoe[3 * k2 + f2] = k2; m.etof[3 * k2 + f2] = int8_t(f2); m.wall[3 * k2 + f2] = 1;
            }
    }
    return "";
}

void assign_levels(HostMesh& m, int max_levels) {
    double rmin = m.inradius[0];
    for (int k = 1; k < m.K; ++k) rmin = std::fmin(rmin, m.inradius[k]);
    m.level.assign(m.K, 1);
    for (int k = 0; k < m.K; ++k) {
        int j = 0;
        while (j + 1 < max_levels && std::ldexp(rmin, j + 1) <= m.inradius[k] * (1.0 + 1e-12)) ++j;
        m.level[k] = int8_t(1 + j);
    }
    bool changed = true;
    while (changed) {
        changed = false;
        std::vector<int8_t> nxt(m.level);
        for (int k = 0; k < m.K; ++k)
            for (int f = 0; f < 3; ++f) {
                const int nb = m.etoe[3 * k + f];
                if (m.level[nb] + 1 < nxt[k]) nxt[k] = int8_t(m.level[nb] + 1);
            }
        for (int k = 0; k < m.K; ++k)
            if (nxt[k] != m.level[k]) changed = true;
        m.level.swap(nxt);
    }
}

void build_tvb_stencil(HostMesh& m) {
    const int K = m.K;
    m.pair.assign(6 * size_t(K), 0);
    m.alpha.assign(6 * size_t(K), 0.0);
    m.dir.assign(6 * size_t(K), 0.0);
    auto bary = [&](int k, double& x, double& y) {
        const int* v = &m.etov[3 * size_t(k)];
        x = (m.vx[v[0]] + m.vx[v[1]] + m.vx[v[2]]) / 3.0;
        y = (m.vy[v[0]] + m.vy[v[1]] + m.vy[v[2]]) / 3.0;
    };
    for (int k = 0; k < K; ++k) {
        double b0x, b0y;
        bary(k, b0x, b0y);
        double nbx[3], nby[3];
        for (int f = 0; f < 3; ++f) {
            if (m.wall[3 * k + f]) {
                const int v = m.etov[3 * k + f];
                const double n_x = m.nx[3 * k + f], n_y = m.ny[3 * k + f];
                const double d = (b0x - m.vx[v]) * n_x + (b0y - m.vy[v]) * n_y;
                nbx[f] = b0x - 2.0 * d * n_x;
                nby[f] = b0y - 2.0 * d * n_y;
            } else {
                bary(m.etoe[3 * k + f], nbx[f], nby[f]);
            }
        }
        for (int i = 0; i < 3; ++i) {
            const int va = m.etov[3 * k + i], vb = m.etov[3 * k + (i + 1) % 3];
            const double dx = 0.5 * (m.vx[va] + m.vx[vb]) - b0x;
            const double dy = 0.5 * (m.vy[va] + m.vy[vb]) - b0y;
            const double dl = std::sqrt(dx * dx + dy * dy);
            m.dir[6 * k + 2 * i] = dx / dl;
            m.dir[6 * k + 2 * i + 1] = dy / dl;
            const int cand[3][2] = {{i, (i + 1) % 3}, {i, (i + 2) % 3}, {(i + 1) % 3, (i + 2) % 3}};
            bool found = false;
            for (int c = 0; c < 3 && !found; ++c) {
                const int j = cand[c][0], l = cand[c][1];
                const double ax = nbx[j] - b0x, ay = nby[j] - b0y;
                const double bx = nbx[l] - b0x, by = nby[l] - b0y;
                const double det = ax * by - ay * bx;
                const double scale = std::sqrt(ax * ax + ay * ay) * std::sqrt(bx * bx + by * by);
                if (!(std::fabs(det) > 1e-12 * scale)) continue;
                const double aj = (dx * by - dy * bx) / det;
                const double al = (ax * dy - ay * dx) / det;
                if (aj >= -1e-10 && al >= -1e-10) {
                    m.pair[6 * k + 2 * i] = int8_t(j);
                    m.pair[6 * k + 2 * i + 1] = int8_t(l);
                    m.alpha[6 * k + 2 * i] = aj;
                    m.alpha[6 * k + 2 * i + 1] = al;
                    found = true;
                }
            }
            if (!found) {
                const double bx = nbx[i] - b0x, by = nby[i] - b0y;
                m.pair[6 * k + 2 * i] = int8_t(i);
                m.pair[6 * k + 2 * i + 1] = int8_t(i);
                m.alpha[6 * k + 2 * i] = dl / std::sqrt(bx * bx + by * by);
                m.alpha[6 * k + 2 * i + 1] = 0.0;
            }
        }
    }
}

void node_coords(const HostMesh& m, const RefElement& re, double* x, double* y) {
    for (int k = 0; k < m.K; ++k) {
        const int* v = &m.etov[3 * size_t(k)];
        for (int p = 0; p < re.Np; ++p) {
            const double r = re.r[p], s = re.s[p];
            x[size_t(k) * re.Np + p] =
                0.5 * (-(r + s) * m.vx[v[0]] + (1.0 + r) * m.vx[v[1]] + (1.0 + s) * m.vx[v[2]]);
            y[size_t(k) * re.Np + p] =
                0.5 * (-(r + s) * m.vy[v[0]] + (1.0 + r) * m.vy[v[1]] + (1.0 + s) * m.vy[v[2]]);
        }
    }
}

}  // namespace dgswe
