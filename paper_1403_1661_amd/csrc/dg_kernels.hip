// HIP kernels (gfx950) of the nodal DG shallow-water step.
//
// Step kernel (one workgroup = E consecutive elements, one lane per node):
//   1. stage eta, hu, hv, B of the block's elements in LDS (coalesced
//      element-major loads);
//   2. volume fluxes at the nodes in contravariant form X_r = rx F + ry G,
//      velocities 2 h m / (h^2 + max(h^2, hvel^2)) (m/h for h >= hvel),
//      X_s = sx F + sy G (Section 2, Eq. 2.3), with the momentum pressure and
//      the split bathymetry source in perturbation form about the element's
//      first-node surface level eta_k:  with d = eta - eta_k,
//        -(g/2) grad(h^2) - g eta grad B + (g/2) grad(B^2)
//          = -(g/2) grad(d (2h - d)) - g d grad B,
//      which is algebraically identical (grad of a constant is zero) and is
//      exactly zero for still water in any precision;
//   3. face traces: interior values from LDS, exterior values gathered from
//      the neighbour through EToE/EToF (node j meets node Nfp-1-j) or the
//      reflective wall ghost; hydrostatic reconstruction h* (Eq. 5.1) and the
//      well-balanced Lax-Friedrichs flux (Eq. 5.2) with the wave speed maxed
//      over the face; the (g/2) h^2 terms of F(Q-).n and of the pressure
//      correction cancel symbolically and the rest is formed from h*- - h*+;
//   4. R = -Dr X_r - Ds X_s + LIFT (Fscale dF) + S (Section 3, Eq. 3.3);
//   5. Adams-Bashforth update with the level's weights (Algorithm 4.1), RHS
//      written to the ring, half-step face traces for finer neighbours;
//   6. per-element FP64 reductions (min depth, means, P1 edge-midpoint
//      deviations) and the positivity limiter of Algorithm 5.2.
// TVB kernel (one lane per element, FP64): characteristic minmod on the
// edge-midpoint deviations against the neighbours' means, balancing, and the
// depth rescaling of Eq. 5.3 (Section 5.3).
#include <hip/hip_runtime.h>

#include <cstdio>

#include "dg_launch.hpp"

namespace dgswe {

template <int N>
struct Shape {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int nF = 3 * (N + 1);
    static constexpr int E = 256 / Np;   // elements per 256-lane workgroup
};

__device__ __forceinline__ int xcd_remap(int b, int n) {
    // Dispatch sends block b to XCD b % 8; give each XCD one contiguous run of
    // element blocks so neighbour gathers hit its own L2.
    const int full = n & ~7;
    if (b >= full) return b;
    const int per = full >> 3;
    return (b & 7) * per + (b >> 3);
}

// Desingularised velocity factor 2h / (h^2 + max(h^2, hvel^2)): u = hu * f
// equals hu/h for h >= hvel and goes continuously to zero with h.
__device__ __forceinline__ float vel_factor(float h, float hvel) {
    const float h2 = h * h;
    return 2.f * h / (h2 + fmaxf(h2, hvel * hvel));
}

template <typename A>
__device__ __forceinline__ int level_of(const A& a, int k) {
    int l = 0;
#pragma unroll
    for (int q = 0; q < kMaxLevels - 1; ++q) l += (q + 1 < a.nlev && k >= a.lev[q].end) ? 1 : 0;
    return l;
}

template <typename A>
__device__ __forceinline__ LevelArgs pick_level(const A& a, int l) {
    LevelArgs L = a.lev[0];
#pragma unroll
    for (int q = 1; q < kMaxLevels; ++q)
        if (l == q) L = a.lev[q];
    return L;
}

// ---------------------------------------------------------------------------
// step kernel
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(256) step_kernel(StepArgs a) {
    using S = Shape<N>;
    constexpr int Np = S::Np, Nfp = S::Nfp, nF = S::nF, E = S::E;
    __shared__ float sDr[Np * Np], sDs[Np * Np], sL[Np * nF];
    __shared__ int sFm[nF];
    __shared__ float sQ[4][E * Np];       // eta, hu, hv, B
    __shared__ float sX[7][E * Np];       // X_r (3 fields), X_s (3 fields), B - B_k
    __shared__ float sT[4][E * nF];       // exterior eta, hu, hv, B
    __shared__ float sLam[E * nF];
    __shared__ float sF[3][E * nF];
    __shared__ double sRed[E][16];

    const int tid = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int k0 = a.k_begin + blk * E;
    const int mode = a.mode;
    const bool rhs = (mode == MODE_FUSED || mode == MODE_RHS_ONLY);

    if (rhs) {
        for (int t = tid; t < Np * Np; t += 256) {
            sDr[t] = a.ops.Dr[t];
            sDs[t] = a.ops.Ds[t];
        }
        for (int t = tid; t < Np * nF; t += 256) sL[t] = a.ops.LIFT[t];
    }
    for (int t = tid; t < nF; t += 256) sFm[t] = a.ops.fmask[t];

    const int e = tid / Np;
    const int i = tid - e * Np;
    const int k = k0 + e;
    const bool live = (e < E) && (k < a.k_end);
    const long long KNp = a.KNp;
    const float g = a.g, hvel = a.hvel;

    LevelArgs L = a.lev[0];
    float eta = 0.f, hu = 0.f, hv = 0.f, Bn = 0.f;
    float4 g0 = make_float4(0, 0, 0, 0), g3 = make_float4(0, 0, 0, 0);
    const long long idx = (long long)k * Np + i;
    if (live) {
        L = pick_level(a, level_of(a, k));
        const float* Q = a.Q[L.parity];
        eta = Q[idx];
        hu = Q[KNp + idx];
        hv = Q[2 * KNp + idx];
        Bn = a.B[idx];
        sQ[0][tid] = eta;
        sQ[1][tid] = hu;
        sQ[2][tid] = hv;
        sQ[3][tid] = Bn;
        const float4* gp = reinterpret_cast<const float4*>(a.geo) + 4LL * k;
        g0 = gp[0];   // rx, ry, sx, sy
        g3 = gp[3];   // fs2, J, dt_min of the instance, instance id
    }
    __syncthreads();

    float Rn[3] = {0.f, 0.f, 0.f};
    float dlt = 0.f;
    if (rhs) {
        // ---- volume fluxes at the nodes
        if (live) {
            const float h = eta - Bn;
            dlt = eta - sQ[0][e * Np];
            // bed relative to the element's first node: the gradient of B is
            // taken from O(H |grad B|) values instead of O(|B|) ones
            sX[6][tid] = Bn - sQ[3][e * Np];
            const float fv = vel_factor(h, hvel);
            const float u = hu * fv;
            const float v = hv * fv;
            const float p = 0.5f * g * (dlt * (2.f * h - dlt));
            const float Fh = hu, Gh = hv;
            const float Fu = hu * u + p, Gu = hv * u;
            const float Fv = hu * v, Gv = hv * v + p;
            const float rx = g0.x, ry = g0.y, sx = g0.z, sy = g0.w;
            sX[0][tid] = rx * Fh + ry * Gh;
            sX[1][tid] = rx * Fu + ry * Gu;
            sX[2][tid] = rx * Fv + ry * Gv;
            sX[3][tid] = sx * Fh + sy * Gh;
            sX[4][tid] = sx * Fu + sy * Gu;
            sX[5][tid] = sx * Fv + sy * Gv;
        }
        // ---- exterior traces and nodal wave speeds
        for (int t = tid; t < E * nF; t += 256) {
            const int fe = t / nF;
            const int fn = t - fe * nF;
            const int f = fn / Nfp;
            const int j = fn - f * Nfp;
            const int kk = k0 + fe;
            if (kk >= a.k_end) continue;
            const int4 cn = reinterpret_cast<const int4*>(a.conn)[kk];
            const int nb = f == 0 ? cn.x : (f == 1 ? cn.y : cn.z);
            const int n = sFm[fn];
            const float etaM = sQ[0][fe * Np + n], huM = sQ[1][fe * Np + n];
            const float hvM = sQ[2][fe * Np + n], BM = sQ[3][fe * Np + n];
            float etaP, huP, hvP, BP;
            if (nb < 0) {
                const float* gk = a.geo + 16LL * kk;
                const float nx = gk[4 + f], ny = gk[7 + f];
                const float mn = huM * nx + hvM * ny;
                etaP = etaM;
                BP = BM;
                huP = huM - 2.f * mn * nx;
                hvP = hvM - 2.f * mn * ny;
            } else {
                const int f2 = (cn.w >> (2 * f)) & 3;
                const int l2 = level_of(a, nb);
                const LevelArgs L2 = pick_level(a, l2);
                const int n2 = sFm[f2 * Nfp + (Nfp - 1 - j)];
                const long long id2 = (long long)nb * Np + n2;
                BP = a.B[id2];
                if (L2.active || a.half == nullptr) {
                    const float* Q2 = a.Q[L2.parity];
                    etaP = Q2[id2];
                    huP = Q2[KNp + id2];
                    hvP = Q2[2 * KNp + id2];
                } else {
                    const long long hid = (long long)nb * nF + f2 * Nfp + (Nfp - 1 - j);
                    etaP = a.half[hid];
                    huP = a.half[a.KnF + hid];
                    hvP = a.half[2 * a.KnF + hid];
                }
            }
            sT[0][t] = etaP;
            sT[1][t] = huP;
            sT[2][t] = hvP;
            sT[3][t] = BP;
            // nodal wave speed of the reconstructed states
            const float* gk = a.geo + 16LL * kk;
            const float nx = gk[4 + f], ny = gk[7 + f];
            const float hM = etaM - BM, hP = etaP - BP;
            const float fM = vel_factor(hM, hvel), fP = vel_factor(hP, hvel);
            const float uM = huM * fM, vM = hvM * fM;
            const float uP = huP * fP, vP = hvP * fP;
            const float Bmax = fmaxf(BM, BP);
            const float hsM = fmaxf(0.f, etaM - Bmax), hsP = fmaxf(0.f, etaP - Bmax);
            const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
            sLam[t] = fmaxf(fabsf(unM) + sqrtf(g * hsM), fabsf(unP) + sqrtf(g * hsP));
        }
        __syncthreads();
        // ---- numerical flux differences, scaled by Fscale
        for (int t = tid; t < E * nF; t += 256) {
            const int fe = t / nF;
            const int fn = t - fe * nF;
            const int f = fn / Nfp;
            const int kk = k0 + fe;
            if (kk >= a.k_end) continue;
            float lam = sLam[fe * nF + f * Nfp];
#pragma unroll
            for (int q = 1; q < Nfp; ++q) lam = fmaxf(lam, sLam[fe * nF + f * Nfp + q]);
            const int n = sFm[fn];
            const float etaM = sQ[0][fe * Np + n], huM = sQ[1][fe * Np + n];
            const float hvM = sQ[2][fe * Np + n], BM = sQ[3][fe * Np + n];
            const float etaP = sT[0][t], huP = sT[1][t], hvP = sT[2][t], BP = sT[3][t];
            const float* gk = a.geo + 16LL * kk;
            const float nx = gk[4 + f], ny = gk[7 + f], fs = gk[10 + f];
            const float hM = etaM - BM, hP = etaP - BP;
            const float fM = vel_factor(hM, hvel), fP = vel_factor(hP, hvel);
            const float uM = huM * fM, vM = hvM * fM;
            const float uP = huP * fP, vP = hvP * fP;
            const float Bmax = fmaxf(BM, BP);
            const float hsM = fmaxf(0.f, etaM - Bmax), hsP = fmaxf(0.f, etaP - Bmax);
            const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
            // F(Q-).n - F*.n.  The (g/2)(h-)^2 of F(Q-).n cancels the one in the
            // pressure correction of Eq. 5.2, and the remaining (g/2) h*^2 terms
            // combine into (g/4)(h*- - h*+)(h*- + h*+): no O(1) quantities are
            // subtracted, and the difference is exactly zero for still water.
            const float dp = 0.25f * g * (hsM - hsP) * (hsM + hsP);
            const float ah = hsM * unM + hsP * unP;
            const float au = hsM * uM * unM + hsP * uP * unP;
            const float av = hsM * vM * unM + hsP * vP * unP;
            sF[0][t] = fs * ((huM * nx + hvM * ny) - 0.5f * ah + 0.5f * lam * (hsP - hsM));
            sF[1][t] = fs * (huM * unM - 0.5f * au + dp * nx + 0.5f * lam * (hsP * uP - hsM * uM));
            sF[2][t] = fs * (hvM * unM - 0.5f * av + dp * ny + 0.5f * lam * (hsP * vP - hsM * vM));
        }
        __syncthreads();
        // ---- R = -(Dr X_r + Ds X_s) + LIFT dF + source
        if (live) {
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, br = 0.f, bs = 0.f;
#pragma unroll
            for (int j = 0; j < Np; ++j) {
                const float dr = sDr[i * Np + j], ds = sDs[i * Np + j];
                const int b = e * Np + j;
                a0 += dr * sX[0][b] + ds * sX[3][b];
                a1 += dr * sX[1][b] + ds * sX[4][b];
                a2 += dr * sX[2][b] + ds * sX[5][b];
                br += dr * sX[6][b];
                bs += ds * sX[6][b];
            }
            float l0 = 0.f, l1 = 0.f, l2 = 0.f;
#pragma unroll
            for (int m = 0; m < nF; ++m) {
                const float lm = sL[i * nF + m];
                const int b = e * nF + m;
                l0 += lm * sF[0][b];
                l1 += lm * sF[1][b];
                l2 += lm * sF[2][b];
            }
            const float rx = g0.x, ry = g0.y, sx = g0.z, sy = g0.w;
            Rn[0] = l0 - a0;
            Rn[1] = l1 - a1 - g * dlt * (rx * br + sx * bs);
            Rn[2] = l2 - a2 - g * dlt * (ry * br + sy * bs);
        }
    }
    if (mode == MODE_RHS_ONLY) {
        if (live) {
            float* R0 = a.R[L.slot[0]];
            R0[idx] = Rn[0];
            R0[KNp + idx] = Rn[1];
            R0[2 * KNp + idx] = Rn[2];
        }
        return;
    }
    // ---- Adams-Bashforth update
    float qn[3] = {eta, hu, hv};
    if (live && mode != MODE_LIMIT_ONLY) {
        float* R0 = a.R[L.slot[0]];
        if (mode == MODE_UPDATE_ONLY) {
            Rn[0] = R0[idx];
            Rn[1] = R0[KNp + idx];
            Rn[2] = R0[2 * KNp + idx];
        } else {
            R0[idx] = Rn[0];
            R0[KNp + idx] = Rn[1];
            R0[2 * KNp + idx] = Rn[2];
        }
        const float dt = g3.z * L.scale;
        float r1[3] = {0.f, 0.f, 0.f}, r2[3] = {0.f, 0.f, 0.f};
        if (L.ab[1] != 0.f) {
            const float* R1 = a.R[L.slot[1]];
            r1[0] = R1[idx]; r1[1] = R1[KNp + idx]; r1[2] = R1[2 * KNp + idx];
        }
        if (L.ab[2] != 0.f) {
            const float* R2 = a.R[L.slot[2]];
            r2[0] = R2[idx]; r2[1] = R2[KNp + idx]; r2[2] = R2[2 * KNp + idx];
        }
        const float q0[3] = {eta, hu, hv};
#pragma unroll
        for (int c = 0; c < 3; ++c)
            qn[c] = q0[c] + dt * (L.ab[0] * Rn[c] + L.ab[1] * r1[c] + L.ab[2] * r2[c]);
        if (L.write_half && a.half != nullptr) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int slot = a.ops.nodeface[2 * i + s];
                if (slot < 0) continue;
                const long long hid = (long long)k * nF + slot;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    a.half[c * a.KnF + hid] =
                        q0[c] + dt * (L.half[0] * Rn[c] + L.half[1] * r1[c] + L.half[2] * r2[c]);
            }
        }
    }
    __syncthreads();
    if (live) {
        sQ[0][tid] = qn[0];
        sQ[1][tid] = qn[1];
        sQ[2][tid] = qn[2];
    }
    __syncthreads();
    // ---- per-element FP64 reductions: 0 min h, 1-3 means, 4-12 midpoint deviations
    if (live) {
        for (int q = i; q < 13; q += Np) {
            double acc;
            if (q == 0) {
                acc = 1e300;
                for (int j = 0; j < Np; ++j)
                    acc = fmin(acc, (double)sQ[0][e * Np + j] - (double)sQ[3][e * Np + j]);
            } else if (q < 4) {
                const int c = q - 1;
                acc = 0.0;
                for (int j = 0; j < Np; ++j) {
                    const double val = c == 0 ? (double)sQ[0][e * Np + j] - (double)sQ[3][e * Np + j]
                                              : (double)sQ[c][e * Np + j];
                    acc += a.ops.wh[j] * val;
                }
            } else {
                const int c = (q - 4) / 3, ed = (q - 4) % 3;
                acc = 0.0;
                for (int j = 0; j < Np; ++j) {
                    const double val = c == 0 ? (double)sQ[0][e * Np + j] - (double)sQ[3][e * Np + j]
                                              : (double)sQ[c][e * Np + j];
                    acc += a.ops.pmid[ed * Np + j] * val;
                }
            }
            sRed[e][q] = acc;
        }
    }
    __syncthreads();
    // ---- positivity limiter decision (Algorithm 5.2), one lane per element
    if (live && i == 0) {
        const double hmin = sRed[e][0], hb = sRed[e][1];
        double mean[3] = {hb, sRed[e][2], sRed[e][3]};
        double scale = 1.0;
        int code = 0;
        double hdry = 0.0;
        if (a.pp_on && hmin <= (double)a.eps) {
            if (hb < (double)a.h0) {
                code = 2;
                if (hb < 0.0) atomicAdd(&a.counters[0], 1ULL);
                hdry = a.dry_literal ? (double)a.h0 : fmax(hb, 0.0);
                mean[0] = hdry;
                mean[1] = 0.0;
                mean[2] = 0.0;
                scale = 0.0;
            } else {
                code = 1;
                const double d0 = sRed[e][4], d1 = sRed[e][5], d2 = sRed[e][6];
                const double Ssum = d0 + d1 + d2;
                const double vmin = hb + fmin(Ssum - 2.0 * d0, fmin(Ssum - 2.0 * d1, Ssum - 2.0 * d2));
                const double den = hb - vmin;
                scale = den > 0.0 ? fmin(1.0, (hb - (double)a.h0) / den) : 1.0;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) a.means[c * (long long)a.K + k] = mean[c];
#pragma unroll
        for (int q = 0; q < 9; ++q) a.devs[q * (long long)a.K + k] = (float)(scale * sRed[e][4 + q]);
        a.flags[k] = (uint8_t)code;
        sRed[e][13] = (double)code;
        sRed[e][14] = scale;
        sRed[e][15] = hdry;
    }
    __syncthreads();
    if (!live) return;
    const int code = (int)sRed[e][13];
    float out[3] = {qn[0], qn[1], qn[2]};
    if (code == 2) {
        out[0] = (float)(sRed[e][15] + (double)Bn);
        out[1] = 0.f;
        out[2] = 0.f;
    } else if (code == 1) {
        const double th = sRed[e][14];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double val = sRed[e][1 + c];
#pragma unroll
            for (int ed = 0; ed < 3; ++ed) val += th * sRed[e][4 + 3 * c + ed] * a.ops.phi[ed * Np + i];
            out[c] = c == 0 ? (float)(val + (double)Bn) : (float)val;
        }
    }
    float* Qo = a.Q[1 - L.parity];
    Qo[idx] = out[0];
    Qo[KNp + idx] = out[1];
    Qo[2 * KNp + idx] = out[2];
}

// ---------------------------------------------------------------------------
// step kernel with the contraction on the matrix cores (N <= 4, Np <= 16)
//
// Lanes are element-aligned: a wave holds 4 elements, lane 16q + j is node j
// of element q.  The volume and lift terms of all three fields are one
// product  R^T = X^T [Dr Ds LIFT]^T  per wave on v_mfma_f32_16x16x4f32:
// rows are (element q, field f) pairs, columns are nodes, so lane 16q + j
// receives R of element q at node j for f = 0..3 in its four accumulators.
// X^T rows: f = 0..2 hold (-X_r, -X_s, dF) of h, hu, hv; f = 3 holds
// (rx (B - B_k), sx (B - B_k), 0), whose product is dB/dx at the nodes; a
// second, shorter pass over the Dr/Ds columns gives dB/dy.  The operator is
// held in registers in B-operand order, 0 beyond Np rows / K columns.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int N>
struct MShape {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int nF = 3 * (N + 1);
    static constexpr int KT = 2 * Np + nF;        // contraction length
    static constexpr int KS = (KT + 3) / 4;       // MFMA steps of K = 4
    static constexpr int KB = (2 * Np + 3) / 4;   // steps covering the Dr/Ds columns
    // LDS row stride (floats); at least 24 so the rows can later hold the
    // per-element reduction scratch
    static constexpr int RS = (4 * KS + 4) > 24 ? (4 * KS + 4) : 24;
    static_assert(Np <= 16 && nF <= 16, "element must fit a 16-lane group");
};

template <int KS>
__device__ __forceinline__ int kperm(int k) {
    // K index k is supplied by lane group k % 4 at step k / 4; each group's
    // values are stored contiguously so a lane reads its row slice in order
    return (k & 3) * KS + (k >> 2);
}

template <int N>
__global__ void __launch_bounds__(256) step_mfma_kernel(StepArgs a) {
    using S = MShape<N>;
    constexpr int Np = S::Np, Nfp = S::Nfp, nF = S::nF, KS = S::KS, KB = S::KB, RS = S::RS;
    // X^T rows per element (permuted K order); after the contraction the same
    // storage holds the updated nodal values and the per-element reductions
    __shared__ float sA[16][4][RS];
    __shared__ float sD[16][16];          // B - B_k per node
    __shared__ float sG[16][4];           // rx, ry, sx, sy
    static_assert(sizeof(float) * 16 * 4 * RS >= sizeof(float) * 16 * 4 * 16 + sizeof(double) * 16 * 16,
                  "reduction scratch must fit in the X^T rows");
    float (*sV)[4][16] = reinterpret_cast<float (*)[4][16]>(&sA[0][0][0]);
    double (*sRed)[16] = reinterpret_cast<double (*)[16]>(&sA[0][0][0] + 16 * 4 * 16);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, j = lane & 15;
    const int el = wave * 4 + q;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int k = a.k_begin + blk * 16 + el;
    const bool live = k < a.k_end;
    const bool node = live && j < Np;
    const long long KNp = a.KNp;
    const float g = a.g, hvel = a.hvel;
    const long long idx = (long long)k * Np + j;

    // ---- issue every independent global load first
    LevelArgs L = a.lev[0];
    float eta = 0.f, hu = 0.f, hv = 0.f, Bn = 0.f;
    float r1[3] = {0.f, 0.f, 0.f}, r2[3] = {0.f, 0.f, 0.f};
    float4 g0 = make_float4(0, 0, 0, 0), g3 = make_float4(0, 0, 0, 0);
    int4 cn = make_int4(-1, -1, -1, 0);
    const bool fnode = live && j < nF;
    const int fn = j < nF ? j : 0;
    const int f = fn / Nfp, jj = fn - f * Nfp;
    float nx = 0.f, ny = 0.f, fs = 0.f;
    if (live) {
        L = pick_level(a, level_of(a, k));
        const float4* gp = reinterpret_cast<const float4*>(a.geo) + 4LL * k;
        g0 = gp[0];
        g3 = gp[3];
        cn = reinterpret_cast<const int4*>(a.conn)[k];
        if (j < Np) {
            const float* Q = a.Q[L.parity];
            eta = Q[idx];
            hu = Q[KNp + idx];
            hv = Q[2 * KNp + idx];
            Bn = a.B[idx];
            if (L.ab[1] != 0.f) {
                const float* R1 = a.R[L.slot[1]];
                r1[0] = R1[idx]; r1[1] = R1[KNp + idx]; r1[2] = R1[2 * KNp + idx];
            }
            if (L.ab[2] != 0.f) {
                const float* R2 = a.R[L.slot[2]];
                r2[0] = R2[idx]; r2[1] = R2[KNp + idx]; r2[2] = R2[2 * KNp + idx];
            }
        }
        if (j < nF) {
            const float* gk = a.geo + 16LL * k;
            nx = gk[4 + f];
            ny = gk[7 + f];
            fs = gk[10 + f];
        }
    }
    const int n = a.ops.fmask[fn];
    // exterior trace of face node fn: neighbour gather (depends only on conn)
    const int nb = f == 0 ? cn.x : (f == 1 ? cn.y : cn.z);
    float etaP = 0.f, huP = 0.f, hvP = 0.f, BP = 0.f;
    if (fnode && nb >= 0) {
        const int f2 = (cn.w >> (2 * f)) & 3;
        const LevelArgs L2 = pick_level(a, level_of(a, nb));
        const int n2 = a.ops.fmask[f2 * Nfp + (Nfp - 1 - jj)];
        const long long id2 = (long long)nb * Np + n2;
        BP = a.B[id2];
        if (L2.active || a.half == nullptr) {
            const float* Q2 = a.Q[L2.parity];
            etaP = Q2[id2];
            huP = Q2[KNp + id2];
            hvP = Q2[2 * KNp + id2];
        } else {
            const long long hid = (long long)nb * nF + f2 * Nfp + (Nfp - 1 - jj);
            etaP = a.half[hid];
            huP = a.half[a.KnF + hid];
            hvP = a.half[2 * a.KnF + hid];
        }
    }
    float opB[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) opB[s] = a.ops.Amfma[s * 64 + lane];
    for (int t = j; t < 4 * RS; t += 16) (&sA[el][0][0])[t] = 0.f;

    const float eta0 = __shfl(eta, lane & ~15);
    const float B0 = __shfl(Bn, lane & ~15);
    const float dlt = eta - eta0;

    // ---- volume fluxes, written negated as X^T rows 0..2; bed gradient row 3
    if (node) {
        const float h = eta - Bn;
        const float fv = vel_factor(h, hvel);
        const float u = hu * fv, v = hv * fv;
        const float p = 0.5f * g * (dlt * (2.f * h - dlt));
        const float F[3] = {hu, hu * u + p, hu * v};
        const float G[3] = {hv, hv * u, hv * v + p};
        const float rx = g0.x, ry = g0.y, sx = g0.z, sy = g0.w;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sA[el][c][kperm<KS>(j)] = -(rx * F[c] + ry * G[c]);
            sA[el][c][kperm<KS>(Np + j)] = -(sx * F[c] + sy * G[c]);
        }
        const float bb = Bn - B0;
        sA[el][3][kperm<KS>(j)] = rx * bb;
        sA[el][3][kperm<KS>(Np + j)] = sx * bb;
        sD[el][j] = bb;
        if (j == 0) {
            sG[el][0] = rx; sG[el][1] = ry; sG[el][2] = sx; sG[el][3] = sy;
        }
    }

    // ---- face node fn = j of element q
    const float etaM = __shfl(eta, (lane & ~15) + n);
    const float huM = __shfl(hu, (lane & ~15) + n);
    const float hvM = __shfl(hv, (lane & ~15) + n);
    const float BM = __shfl(Bn, (lane & ~15) + n);
    if (fnode && nb < 0) {
        const float mn = huM * nx + hvM * ny;
        etaP = etaM;
        BP = BM;
        huP = huM - 2.f * mn * nx;
        hvP = hvM - 2.f * mn * ny;
    }
    const float hM = etaM - BM, hP = etaP - BP;
    const float fM = vel_factor(hM, hvel), fP = vel_factor(hP, hvel);
    const float uM = huM * fM, vM = hvM * fM, uP = huP * fP, vP = hvP * fP;
    const float Bmax = fmaxf(BM, BP);
    const float hsM = fmaxf(0.f, etaM - Bmax), hsP = fmaxf(0.f, etaP - Bmax);
    const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
    const float lamN = fnode ? fmaxf(fabsf(unM) + sqrtf(g * hsM), fabsf(unP) + sqrtf(g * hsP)) : 0.f;
    float lam = lamN;
    const int fbase = (lane & ~15) + f * Nfp;
#pragma unroll
    for (int t = 0; t < Nfp; ++t) lam = fmaxf(lam, __shfl(lamN, fbase + t));
    if (fnode) {
        const float dp = 0.25f * g * (hsM - hsP) * (hsM + hsP);
        const float ah = hsM * unM + hsP * unP;
        const float au = hsM * uM * unM + hsP * uP * unP;
        const float av = hsM * vM * unM + hsP * vP * unP;
        const int kp = kperm<KS>(2 * Np + fn);
        sA[el][0][kp] = fs * ((huM * nx + hvM * ny) - 0.5f * ah + 0.5f * lam * (hsP - hsM));
        sA[el][1][kp] = fs * (huM * unM - 0.5f * au + dp * nx + 0.5f * lam * (hsP * uP - hsM * uM));
        sA[el][2][kp] = fs * (hvM * unM - 0.5f * av + dp * ny + 0.5f * lam * (hsP * vP - hsM * vM));
    }
    __syncthreads();

    // ---- contraction on the matrix cores
    const int ar = lane & 15;           // A-operand row: (element ar/4, field ar%4) of this wave
    const int ag = lane >> 4;           // K group supplied by this lane
    const float* arow = &sA[wave * 4 + (ar >> 2)][ar & 3][ag * KS];
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[s], opB[s], acc, 0, 0, 0);
    floatx4 accy = {0.f, 0.f, 0.f, 0.f};
    {
        const int eA = wave * 4 + (ar >> 2);
        const bool rowy = (ar & 3) == 0;
        const float ry = sG[eA][1], sy = sG[eA][3];
#pragma unroll
        for (int s = 0; s < KB; ++s) {
            const int kk = 4 * s + ag;
            float av = 0.f;
            if (rowy) av = kk < Np ? ry * sD[eA][kk] : (kk < 2 * Np ? sy * sD[eA][kk - Np] : 0.f);
            accy = __builtin_amdgcn_mfma_f32_16x16x4f32(av, opB[s], accy, 0, 0, 0);
        }
    }
    float Rn[3];
    Rn[0] = acc[0];
    Rn[1] = acc[1] - g * dlt * acc[3];
    Rn[2] = acc[2] - g * dlt * accy[0];

    // ---- Adams-Bashforth update
    float qn[3] = {eta, hu, hv};
    __syncthreads();   // X^T rows are consumed; their storage is reused below
    if (node) {
        float* R0 = a.R[L.slot[0]];
        R0[idx] = Rn[0];
        R0[KNp + idx] = Rn[1];
        R0[2 * KNp + idx] = Rn[2];
        const float dt = g3.z * L.scale;
        const float q0[3] = {eta, hu, hv};
#pragma unroll
        for (int c = 0; c < 3; ++c)
            qn[c] = q0[c] + dt * (L.ab[0] * Rn[c] + L.ab[1] * r1[c] + L.ab[2] * r2[c]);
        if (L.write_half && a.half != nullptr) {
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const int slot = a.ops.nodeface[2 * j + sl];
                if (slot < 0) continue;
                const long long hid = (long long)k * nF + slot;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    a.half[c * a.KnF + hid] =
                        q0[c] + dt * (L.half[0] * Rn[c] + L.half[1] * r1[c] + L.half[2] * r2[c]);
            }
        }
        sV[el][0][j] = qn[0];
        sV[el][1][j] = qn[1];
        sV[el][2][j] = qn[2];
        sV[el][3][j] = Bn;
    }
    __syncthreads();
    // ---- per-element FP64 reductions: 0 min h, 1-3 means, 4-12 midpoint deviations
    if (live && j < 13) {
        double acc64;
        if (j == 0) {
            acc64 = 1e300;
            for (int t = 0; t < Np; ++t) acc64 = fmin(acc64, (double)sV[el][0][t] - (double)sV[el][3][t]);
        } else {
            const int c = j < 4 ? j - 1 : (j - 4) / 3;
            const double* w = j < 4 ? a.ops.wh : a.ops.pmid + ((j - 4) % 3) * Np;
            acc64 = 0.0;
            for (int t = 0; t < Np; ++t) {
                const double val = c == 0 ? (double)sV[el][0][t] - (double)sV[el][3][t] : (double)sV[el][c][t];
                acc64 += w[t] * val;
            }
        }
        sRed[el][j] = acc64;
    }
    __syncthreads();
    // ---- positivity limiter decision (Algorithm 5.2)
    if (live && j == 0) {
        const double hmin = sRed[el][0], hb = sRed[el][1];
        double mean[3] = {hb, sRed[el][2], sRed[el][3]};
        double scale = 1.0, hdry = 0.0;
        int code = 0;
        if (a.pp_on && hmin <= (double)a.eps) {
            if (hb < (double)a.h0) {
                code = 2;
                if (hb < 0.0) atomicAdd(&a.counters[0], 1ULL);
                hdry = a.dry_literal ? (double)a.h0 : fmax(hb, 0.0);
                mean[0] = hdry;
                mean[1] = 0.0;
                mean[2] = 0.0;
                scale = 0.0;
            } else {
                code = 1;
                const double d0 = sRed[el][4], d1 = sRed[el][5], d2 = sRed[el][6];
                const double Ssum = d0 + d1 + d2;
                const double vmin = hb + fmin(Ssum - 2.0 * d0, fmin(Ssum - 2.0 * d1, Ssum - 2.0 * d2));
                const double den = hb - vmin;
                scale = den > 0.0 ? fmin(1.0, (hb - (double)a.h0) / den) : 1.0;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) a.means[c * (long long)a.K + k] = mean[c];
#pragma unroll
        for (int t = 0; t < 9; ++t) a.devs[t * (long long)a.K + k] = (float)(scale * sRed[el][4 + t]);
        a.flags[k] = (uint8_t)code;
        sRed[el][13] = (double)code;
        sRed[el][14] = scale;
        sRed[el][15] = hdry;
    }
    __syncthreads();
    if (!node) return;
    const int code = (int)sRed[el][13];
    float out[3] = {qn[0], qn[1], qn[2]};
    if (code == 2) {
        out[0] = (float)(sRed[el][15] + (double)Bn);
        out[1] = 0.f;
        out[2] = 0.f;
    } else if (code == 1) {
        const double th = sRed[el][14];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double val = sRed[el][1 + c];
#pragma unroll
            for (int ed = 0; ed < 3; ++ed) val += th * sRed[el][4 + 3 * c + ed] * a.ops.phi[ed * Np + j];
            out[c] = c == 0 ? (float)(val + (double)Bn) : (float)val;
        }
    }
    float* Qo = a.Q[1 - L.parity];
    Qo[idx] = out[0];
    Qo[KNp + idx] = out[1];
    Qo[2 * KNp + idx] = out[2];
}

// ---------------------------------------------------------------------------
// TVB limiter with the positivity modification of Eq. 5.3, one lane per element
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) tvb_kernel(TvbArgs a) {
    const int k = a.k_begin + blockIdx.x * 256 + threadIdx.x;
    if (k >= a.k_end) return;
    const int K = a.K;
    const uint8_t pp = a.flags[k] & 3;
    if (pp == 2) {
        a.flags[k] = pp;
        return;
    }
    const int4 cn = reinterpret_cast<const int4*>(a.conn)[k];
    const int nbs[3] = {cn.x, cn.y, cn.z};
#pragma unroll
    for (int f = 0; f < 3; ++f)
        if (nbs[f] >= 0 && (a.flags[nbs[f]] & 3) == 2) {
            a.flags[k] = pp;
            return;
        }
    const double qb[3] = {a.means[k], a.means[(long long)K + k], a.means[2LL * K + k]};
    double dev[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int ed = 0; ed < 3; ++ed) dev[c][ed] = (double)a.devs[(3 * c + ed) * (long long)K + k];
    const float* gk = a.geo + 16LL * k;
    double diff[3][3];   // [face][field]
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        if (nbs[f] < 0) {
            const double nx = gk[4 + f], ny = gk[7 + f];
            const double mn = qb[1] * nx + qb[2] * ny;
            diff[f][0] = 0.0;
            diff[f][1] = -2.0 * mn * nx;
            diff[f][2] = -2.0 * mn * ny;
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) diff[f][c] = a.means[c * (long long)K + nbs[f]] - qb[c];
        }
    }
    const float* st = a.stencil + 16LL * k;
    const int pairs = __float_as_int(st[13]);
    const double M2 = st[12];
    const double hb = qb[0];
    const double ub = qb[1] / hb, vb = qb[2] / hb;
    const double c = sqrt(a.g * hb);
    double D[3][3];   // [field][edge]
    bool all_a1 = true;
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
        const int pj = (pairs >> (4 * ed)) & 3, pk = (pairs >> (4 * ed + 2)) & 3;
        const double aj = st[4 * ed], ak = st[4 * ed + 1];
        const double ex = st[4 * ed + 2], ey = st[4 * ed + 3];
        double dbar[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) dbar[q] = aj * diff[pj][q] + ak * diff[pk][q];
        const double un = ub * ex + vb * ey, ut = -ub * ey + vb * ex;
        const double i2c = 0.5 / c;
        const double Lm[3][3] = {{(un + c) * i2c, -ex * i2c, -ey * i2c},
                                 {-ut, -ey, ex},
                                 {-(un - c) * i2c, ex * i2c, ey * i2c}};
        const double Rm[3][3] = {{1.0, 0.0, 1.0},
                                 {ub - c * ex, -ey, ub + c * ex},
                                 {vb - c * ey, ex, vb + c * ey}};
        double mt[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double a1 = Lm[r][0] * dev[0][ed] + Lm[r][1] * dev[1][ed] + Lm[r][2] * dev[2][ed];
            const double a2 = a.nu * (Lm[r][0] * dbar[0] + Lm[r][1] * dbar[1] + Lm[r][2] * dbar[2]);
            const bool small = fabs(a1) <= M2;
            const bool same = (a1 > 0.0 && a2 > 0.0) || (a1 < 0.0 && a2 < 0.0);
            const double mm = same ? copysign(fmin(fabs(a1), fabs(a2)), a1) : 0.0;
            mt[r] = small ? a1 : mm;
            all_a1 = all_a1 && (small || a1 == 0.0 || (same && fabs(a1) <= fabs(a2)));
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) D[q][ed] = Rm[q][0] * mt[0] + Rm[q][1] * mt[1] + Rm[q][2] * mt[2];
    }
    if (all_a1) {
        a.flags[k] = pp | (1 << 2);
        return;
    }
    // balance each conserved component
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double pos = 0.0, neg = 0.0;
#pragma unroll
        for (int ed = 0; ed < 3; ++ed) {
            pos += fmax(D[q][ed], 0.0);
            neg += fmax(-D[q][ed], 0.0);
        }
        const double thp = pos > 0.0 ? fmin(1.0, neg / pos) : 1.0;
        const double thm = neg > 0.0 ? fmin(1.0, pos / neg) : 1.0;
#pragma unroll
        for (int ed = 0; ed < 3; ++ed) D[q][ed] = thp * fmax(D[q][ed], 0.0) - thm * fmax(-D[q][ed], 0.0);
    }
    // Eq. 5.3 on the depth increments
    int code = 2;
    {
        const double Ssum = D[0][0] + D[0][1] + D[0][2];
        const double dbh = Ssum / 3.0;
        const double vmin = fmin(Ssum - 2.0 * D[0][0], fmin(Ssum - 2.0 * D[0][1], Ssum - 2.0 * D[0][2]));
        if (hb + vmin < a.h0) {
            const double den = dbh - vmin;
            double th = den > 0.0 ? (hb + dbh - a.h0) / den : 0.0;
            th = fmin(1.0, fmax(0.0, th));
#pragma unroll
            for (int ed = 0; ed < 3; ++ed) D[0][ed] = dbh + th * (D[0][ed] - dbh);
            code = 3;
        }
    }
    // P1 output: mean + sum_i D_i phi_i at every node
    int l = 0;
#pragma unroll
    for (int q = 0; q < kMaxLevels - 1; ++q) l += (q + 1 < a.nlev && k >= a.lev[q].end) ? 1 : 0;
    const LevelArgs L = pick_level(a, l);
    float* Qo = a.Q[1 - L.parity];
    const int Np = a.Np;
    for (int j = 0; j < Np; ++j) {
        const double p0 = a.phi[j], p1 = a.phi[Np + j], p2 = a.phi[2 * Np + j];
        const long long id = (long long)k * Np + j;
        const double hval = qb[0] + D[0][0] * p0 + D[0][1] * p1 + D[0][2] * p2;
        Qo[id] = (float)(hval + (double)a.B[id]);
        Qo[a.KNp + id] = (float)(qb[1] + D[1][0] * p0 + D[1][1] * p1 + D[1][2] * p2);
        Qo[2 * a.KNp + id] = (float)(qb[2] + D[2][0] * p0 + D[2][1] * p1 + D[2][2] * p2);
    }
    a.flags[k] = pp | (code << 2);
}

// ---------------------------------------------------------------------------
// deterministic FP64 diagnostics: mass, min depth, flag histograms
// ---------------------------------------------------------------------------
constexpr int kDiagBlocks = 256;

__global__ void __launch_bounds__(256) diag_partial_kernel(DiagArgs a) {
    __shared__ double sm[256][9];
    double mass = 0.0, hmin = 1e300;
    double cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = a.k_begin + blockIdx.x * 256 + threadIdx.x; k < a.k_end; k += gridDim.x * 256) {
        const float* gk = a.geo + 16LL * k;
        if (__float_as_int(gk[15]) != a.inst) continue;
        int l = 0;
#pragma unroll
        for (int q = 0; q < kMaxLevels - 1; ++q) l += (q + 1 < a.nlev && k >= a.lev[q].end) ? 1 : 0;
        const LevelArgs L = pick_level(a, l);
        const float* Q = L.parity ? a.Q2 : a.Q;
        double wh = 0.0;
        for (int j = 0; j < a.Np; ++j) {
            const long long id = (long long)k * a.Np + j;
            const double h = (double)Q[id] - (double)a.B[id];
            wh += a.wfull[j] * h;
            hmin = fmin(hmin, h);
        }
        mass += (double)gk[13] * wh;
        const int fl = a.flags[k];
        cnt[fl & 3] += 1.0;
        cnt[3 + ((fl >> 2) & 3)] += 1.0;
    }
    sm[threadIdx.x][0] = mass;
    sm[threadIdx.x][1] = hmin;
    for (int q = 0; q < 7; ++q) sm[threadIdx.x][2 + q] = cnt[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sm[threadIdx.x][0] += sm[threadIdx.x + s][0];
            sm[threadIdx.x][1] = fmin(sm[threadIdx.x][1], sm[threadIdx.x + s][1]);
            for (int q = 2; q < 9; ++q) sm[threadIdx.x][q] += sm[threadIdx.x + s][q];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9) a.partial[blockIdx.x * 16 + threadIdx.x] = sm[0][threadIdx.x];
}

__global__ void diag_final_kernel(DiagArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double out[9] = {0.0, 1e300, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < kDiagBlocks; ++b) {
        out[0] += a.partial[b * 16 + 0];
        out[1] = fmin(out[1], a.partial[b * 16 + 1]);
        for (int q = 2; q < 9; ++q) out[q] += a.partial[b * 16 + q];
    }
    for (int q = 0; q < 9; ++q) a.out[q] = out[q];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static thread_local char g_dev_err[256];

const char* device_error_string() { return g_dev_err; }

static int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::snprintf(g_dev_err, sizeof(g_dev_err), "%s: %s", what, hipGetErrorString(e));
        return -1;
    }
    return 0;
}

int step_elems_per_block(int N, int engine) {
    (void)engine;
    const int Np = (N + 1) * (N + 2) / 2;
    return 256 / Np;
}

template <int N>
static int launch_step_n(const StepArgs& a, hipStream_t s) {
    const int n = a.k_end - a.k_begin;
    if (n <= 0) return 0;
    if constexpr (N <= 4) {
        if (a.engine == ENGINE_MFMA_F32 && a.mode == MODE_FUSED) {
            hipLaunchKernelGGL(step_mfma_kernel<N>, dim3((n + 15) / 16), dim3(256), 0, s, a);
            return check_launch("step mfma kernel");
        }
    }
    const int E = Shape<N>::E;
    const int blocks = (n + E - 1) / E;
    hipLaunchKernelGGL(step_kernel<N>, dim3(blocks), dim3(256), 0, s, a);
    return check_launch("step kernel");
}

int mfma_steps(int N) {
    const int Np = (N + 1) * (N + 2) / 2, nF = 3 * (N + 1);
    return (2 * Np + nF + 3) / 4;
}

int launch_step(const StepArgs& a, void* stream, int elems_per_block) {
    (void)elems_per_block;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (a.N) {
        case 1: return launch_step_n<1>(a, s);
        case 2: return launch_step_n<2>(a, s);
        case 3: return launch_step_n<3>(a, s);
        case 4: return launch_step_n<4>(a, s);
        case 5: return launch_step_n<5>(a, s);
        case 6: return launch_step_n<6>(a, s);
        default:
            std::snprintf(g_dev_err, sizeof(g_dev_err), "unsupported N=%d", a.N);
            return -1;
    }
}

int launch_tvb(const TvbArgs& a, void* stream) {
    const int n = a.k_end - a.k_begin;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(tvb_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), a);
    return check_launch("tvb kernel");
}

int launch_diag(const DiagArgs& a, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(diag_partial_kernel, dim3(kDiagBlocks), dim3(256), 0, s, a);
    if (check_launch("diag kernel")) return -1;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, s, a);
    return check_launch("diag final kernel");
}

}  // namespace dgswe
