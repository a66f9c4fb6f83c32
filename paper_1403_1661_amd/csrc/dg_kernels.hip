// HIP kernels (gfx950) of the nodal DG shallow-water step.
//
// Step kernel (one workgroup = E consecutive elements, one lane per node):
//   1. stage eta and B (each an FP32 hi + lo pair), hu, hv of the block's
//      elements in LDS (coalesced element-major loads);
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
//      deviations) and the positivity limiter of Algorithm 5.2; the element
//      leaves a record of its FP64 means and positivity code, and its
//      deviations (stored in FP32) unless it is dry.
// TVB kernel (three lanes per element, FP64 arithmetic): characteristic minmod
// on the edge-midpoint deviations against the neighbours' means, balancing,
// and the depth rescaling of Eq. 5.3 (Section 5.3).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

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

// Compensated surface level: the state keeps eta as an FP32 pair hi + lo with
// |lo| <= ulp(hi)/2, so that rounding the stored level to FP32 once per step
// does not accumulate over a run.  eta_add adds an increment with the
// two-sum of Knuth (the rounding error of hi + d is recovered exactly) and
// renormalises with the fast two-sum of Dekker; eta_split rounds an FP64
// value to the pair.
__device__ __forceinline__ void eta_add(float& hi, float& lo, float d) {
    const float s = hi + d;
    const float bp = s - hi;
    const float err = (hi - (s - bp)) + (d - bp);
    const float l = lo + err;
    hi = s + l;
    lo = l - (hi - s);
}

// The low word is stored as a 16-bit integer in units of 2^-15 ulp(hi):
// |lo| <= ulp(hi)/2 fits in +-2^14, and the stored pair keeps the level to
// 2^-16 ulp(hi) (ulp(hi) = 2^(e-24) with hi = m 2^e, 1/2 <= |m| < 1).
__device__ __forceinline__ short lo_encode(float hi, float lo) {
    const int e = __builtin_amdgcn_frexp_expf(hi);
    const float s = __builtin_rintf(__builtin_amdgcn_ldexpf(lo, 39 - e));
    return (short)fminf(fmaxf(s, -32767.f), 32767.f);
}
__device__ __forceinline__ float lo_decode(float hi, short s) {
    return __builtin_amdgcn_ldexpf((float)s, __builtin_amdgcn_frexp_expf(hi) - 39);
}

__device__ __forceinline__ void eta_split(double v, float& hi, float& lo) {
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

// Jump h*- - h*+ of the reconstructed depths (Eq. 5.1).  Where both sides
// are wet they share max(B-, B+), so the jump is the difference of the two
// compensated surface levels, formed without rounding the O(1) depths first
// (the level difference of nearby values is exact in FP32); where one side
// is clipped to zero the plain difference has no cancellation.
__device__ __forceinline__ float depth_jump(float etaM, float loM, float etaP, float loP,
                                            float hsM, float hsP) {
    return (hsM > 0.f && hsP > 0.f) ? (etaM - etaP) + (loM - loP) : hsM - hsP;
}

// Higher of two compensated bed values (hi + lo), for h* = eta - max(B-, B+)
// of Eq. 5.1: equal high words compare by the low words.
__device__ __forceinline__ void bed_max(float bM, float lM, float bP, float lP, float& b, float& l) {
    const bool m = bM > bP || (bM == bP && lM >= lP);
    b = m ? bM : bP;
    l = m ? lM : lP;
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
    __shared__ float sQ[6][E * Np];       // eta (hi), hu, hv, B (hi), eta (lo), B (lo)
    __shared__ float sX[6][E * Np];       // X_r (3 fields), X_s (3 fields)
    __shared__ float sT[6][E * nF];       // exterior eta (hi), hu, hv, B (hi), eta (lo), B (lo)
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
    float eta = 0.f, hu = 0.f, hv = 0.f, Bn = 0.f, lo = 0.f, bl = 0.f;
    float4 g0 = make_float4(0, 0, 0, 0), g3 = make_float4(0, 0, 0, 0);
    const long long idx = (long long)k * Np + i;
    if (live) {
        L = pick_level(a, level_of(a, k));
        const float* Q = a.Q[L.parity];
        eta = Q[idx];
        hu = Q[KNp + idx];
        hv = Q[2 * KNp + idx];
        lo = lo_decode(eta, reinterpret_cast<const short*>(Q + 3 * KNp)[idx]);
        Bn = a.B[idx];
        bl = lo_decode(Bn, a.Blo[idx]);
        sQ[0][tid] = eta;
        sQ[1][tid] = hu;
        sQ[2][tid] = hv;
        sQ[3][tid] = Bn;
        sQ[4][tid] = lo;
        sQ[5][tid] = bl;
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
            const float h = (eta - Bn) + (lo - bl);
            dlt = (eta - sQ[0][e * Np]) + (lo - sQ[4][e * Np]);
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
            const float loM = sQ[4][fe * Np + n], blM = sQ[5][fe * Np + n];
            float etaP, huP, hvP, BP, loP = 0.f, blP;
            if (nb < 0) {
                const float* gk = a.geo + 16LL * kk;
                const float nx = gk[4 + f], ny = gk[7 + f];
                const float mn = huM * nx + hvM * ny;
                etaP = etaM;
                loP = loM;
                BP = BM;
                blP = blM;
                huP = huM - 2.f * mn * nx;
                hvP = hvM - 2.f * mn * ny;
            } else {
                const int f2 = (cn.w >> (2 * f)) & 3;
                const int l2 = level_of(a, nb);
                const LevelArgs L2 = pick_level(a, l2);
                const int n2 = sFm[f2 * Nfp + (Nfp - 1 - j)];
                const long long id2 = (long long)nb * Np + n2;
                BP = a.B[id2];
                blP = lo_decode(BP, a.Blo[id2]);
                if (L2.active || a.half == nullptr) {
                    const float* Q2 = a.Q[L2.parity];
                    etaP = Q2[id2];
                    huP = Q2[KNp + id2];
                    hvP = Q2[2 * KNp + id2];
                    loP = lo_decode(etaP, reinterpret_cast<const short*>(Q2 + 3 * KNp)[id2]);
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
            sT[4][t] = loP;
            sT[5][t] = blP;
            // nodal wave speed of the reconstructed states
            const float* gk = a.geo + 16LL * kk;
            const float nx = gk[4 + f], ny = gk[7 + f];
            const float hM = (etaM - BM) + (loM - blM), hP = (etaP - BP) + (loP - blP);
            const float fM = vel_factor(hM, hvel), fP = vel_factor(hP, hvel);
            const float uM = huM * fM, vM = hvM * fM;
            const float uP = huP * fP, vP = hvP * fP;
            float Bmax, bmlo;
            bed_max(BM, blM, BP, blP, Bmax, bmlo);
            const float hsM = fmaxf(0.f, (etaM - Bmax) + (loM - bmlo));
            const float hsP = fmaxf(0.f, (etaP - Bmax) + (loP - bmlo));
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
            const float loM = sQ[4][fe * Np + n], loP = sT[4][t];
            const float blM = sQ[5][fe * Np + n], blP = sT[5][t];
            const float* gk = a.geo + 16LL * kk;
            const float nx = gk[4 + f], ny = gk[7 + f], fs = gk[10 + f];
            const float hM = (etaM - BM) + (loM - blM), hP = (etaP - BP) + (loP - blP);
            const float fM = vel_factor(hM, hvel), fP = vel_factor(hP, hvel);
            const float uM = huM * fM, vM = hvM * fM;
            const float uP = huP * fP, vP = hvP * fP;
            float Bmax, bmlo;
            bed_max(BM, blM, BP, blP, Bmax, bmlo);
            const float hsM = fmaxf(0.f, (etaM - Bmax) + (loM - bmlo));
            const float hsP = fmaxf(0.f, (etaP - Bmax) + (loP - bmlo));
            const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
            // F(Q-).n - F*.n.  The (g/2)(h-)^2 of F(Q-).n cancels the one in the
            // pressure correction of Eq. 5.2, and the remaining (g/2) h*^2 terms
            // combine into (g/4)(h*- - h*+)(h*- + h*+): no O(1) quantities are
            // subtracted, and the difference is exactly zero for still water.
            const float dh = depth_jump(etaM, loM, etaP, loP, hsM, hsP);
            const float dp = 0.25f * g * dh * (hsM + hsP);
            const float ah = hsM * unM + hsP * unP;
            const float au = hsM * uM * unM + hsP * uP * unP;
            const float av = hsM * vM * unM + hsP * vP * unP;
            sF[0][t] = fs * ((huM * nx + hvM * ny) - 0.5f * ah - 0.5f * lam * dh);
            sF[1][t] = fs * (huM * unM - 0.5f * au + dp * nx + 0.5f * lam * (hsP * uP - hsM * uM));
            sF[2][t] = fs * (hvM * unM - 0.5f * av + dp * ny + 0.5f * lam * (hsP * vP - hsM * vM));
        }
        __syncthreads();
        // ---- R = -(Dr X_r + Ds X_s) + LIFT dF + source
        if (live) {
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
            for (int j = 0; j < Np; ++j) {
                const float dr = sDr[i * Np + j], ds = sDs[i * Np + j];
                const int b = e * Np + j;
                a0 += dr * sX[0][b] + ds * sX[3][b];
                a1 += dr * sX[1][b] + ds * sX[4][b];
                a2 += dr * sX[2][b] + ds * sX[5][b];
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
            Rn[0] = l0 - a0;
            Rn[1] = l1 - a1 - g * dlt * a.dB[idx];
            Rn[2] = l2 - a2 - g * dlt * a.dB[KNp + idx];
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
    float qlo = lo;
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
        const float q0lo[3] = {lo, 0.f, 0.f};
        const float d0 = dt * (L.ab[0] * Rn[0] + L.ab[1] * r1[0] + L.ab[2] * r2[0]);
        eta_add(qn[0], qlo, d0);
#pragma unroll
        for (int c = 1; c < 3; ++c)
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
                        q0[c] + (q0lo[c] + dt * (L.half[0] * Rn[c] + L.half[1] * r1[c] + L.half[2] * r2[c]));
            }
        }
    }
    __syncthreads();
    if (live) {
        sQ[0][tid] = qn[0];
        sQ[1][tid] = qn[1];
        sQ[2][tid] = qn[2];
        sQ[4][tid] = qlo;
    }
    __syncthreads();
    // ---- per-element FP64 reductions: 0 min h, 1-3 means, 4-12 midpoint deviations
    if (live) {
        for (int q = i; q < 13; q += Np) {
            double acc;
            if (q == 0) {
                acc = 1e300;
                for (int j = 0; j < Np; ++j)
                    acc = fmin(acc, ((double)sQ[0][e * Np + j] - (double)sQ[3][e * Np + j]) + ((double)sQ[4][e * Np + j] - (double)sQ[5][e * Np + j]));
            } else if (q < 4) {
                const int c = q - 1;
                acc = 0.0;
                for (int j = 0; j < Np; ++j) {
                    const double val = c == 0 ? ((double)sQ[0][e * Np + j] - (double)sQ[3][e * Np + j]) + ((double)sQ[4][e * Np + j] - (double)sQ[5][e * Np + j])
                                              : (double)sQ[c][e * Np + j];
                    acc += a.ops.wh[j] * val;
                }
            } else {
                const int c = (q - 4) / 3, ed = (q - 4) % 3;
                acc = 0.0;
                for (int j = 0; j < Np; ++j) {
                    const double val = c == 0 ? ((double)sQ[0][e * Np + j] - (double)sQ[3][e * Np + j]) + ((double)sQ[4][e * Np + j] - (double)sQ[5][e * Np + j])
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
        // a mean below h0 with every node above eps (negative vertex weights
        // of the nodal mean at N = 4, 6) also takes the dry branch
        if (a.pp_on && (hmin <= (double)a.eps || hb < (double)a.h0)) {
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
        for (int c = 0; c < 3; ++c) a.mrec[4 * (long long)k + c] = mean[c];
        a.mrec[4 * (long long)k + 3] = (double)code;
        if (code != 2) {
#pragma unroll
            for (int q = 0; q < 9; ++q) a.devs[q * (long long)a.K + k] = (float)(scale * sRed[e][4 + q]);
        }
        a.flags[k] = (uint8_t)code;
        sRed[e][13] = (double)code;
        sRed[e][14] = scale;
        sRed[e][15] = hdry;
    }
    __syncthreads();
    if (!live) return;
    const int code = (int)sRed[e][13];
    float out[3] = {qn[0], qn[1], qn[2]};
    float olo = qlo;
    if (code == 2) {
        eta_split(sRed[e][15] + ((double)Bn + (double)bl), out[0], olo);
        out[1] = 0.f;
        out[2] = 0.f;
    } else if (code == 1) {
        const double th = sRed[e][14];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double val = sRed[e][1 + c];
#pragma unroll
            for (int ed = 0; ed < 3; ++ed) val += th * sRed[e][4 + 3 * c + ed] * a.ops.phi[ed * Np + i];
            if (c == 0)
                eta_split(val + ((double)Bn + (double)bl), out[0], olo);
            else
                out[c] = (float)val;
        }
    }
    if (a.thin_cut > 0.f && (out[0] - Bn) + (olo - bl) < a.thin_cut) {   // thin film: no momentum
        out[1] = 0.f;
        out[2] = 0.f;
    }
    float* Qo = a.Q[1 - L.parity];
    Qo[idx] = out[0];
    Qo[KNp + idx] = out[1];
    Qo[2 * KNp + idx] = out[2];
    reinterpret_cast<short*>(Qo + 3 * KNp)[idx] = lo_encode(out[0], olo);
}


// ---------------------------------------------------------------------------
// right-hand side of the over-integrated weak form (Section 3, Eq. 3.2 with
// cubature and Gauss rules; Section 7, Volume and Surface kernels):
//   R = Pr cF1 + Ps cF2 + P cS - L^g (Fscale Fn*)
// with cF1 = rx F + ry G, cF2 = sx F + sy G and cS at the Ncub cubature
// nodes and Fn* at the 3 NG Gauss nodes of the faces.  The pressure and the
// bed source are taken in perturbation form about the element's first-node
// level eta_k (d = eta - eta_k): volume pressure (g/2) d (2h - d), source
// -g d grad B, and on the faces the flux minus (g/2)(eta_k - B-)^2 n, i.e.
// (g/2) d- (2h- - d-) + (g/4)(h*+ - h*-)(h*+ + h*-) in the momentum flux.
// Under rules exact to degree 3N this differs from the plain form (pressure
// (g/2) h^2, source -g h grad B) only by that face term, which it carries, so
// both are the same scheme; still water gives d = 0 and a zero jump exactly.
// Element data are interpolated as d, h, hu, hv (and the bed slope from the
// nodes) so that every term of still water is zero in any precision.
// One block = E elements, W = max(Ncub, Np, 3 NG) lanes per element.
// ---------------------------------------------------------------------------
template <int N>
struct OShape {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int nF = 3 * (N + 1);
    static constexpr int Q = overint_points(N);
    static constexpr int NC = Q * Q;
    static constexpr int NG = Q;
    static constexpr int NGF = 3 * Q;
    static constexpr int W0 = NC > Np ? NC : Np;
    static constexpr int W = W0 > NGF ? W0 : NGF;
    static constexpr int E = 256 / W;
};

template <int N>
__global__ void __launch_bounds__(256) rhs_overint_kernel(StepArgs a) {
    using S = OShape<N>;
    constexpr int Np = S::Np, Nfp = S::Nfp, nF = S::nF, NC = S::NC, NG = S::NG, NGF = S::NGF;
    constexpr int W = S::W, E = S::E;
    __shared__ float sIc[NC * Np], sPr[Np * NC], sPs[Np * NC], sP[Np * NC], sLg[Np * NGF], sI1[NG * Nfp];
    __shared__ float sN[6][E][Np];      // h, d, hu, hv, dB/dx, dB/dy at the nodes
    __shared__ float sT[5][E][nF];      // exterior h, hu, hv, d (about the own eta_k), B+ - B- at own face nodes
    __shared__ float sC[8][E][NC];      // cF1 (3), cF2 (3), cS (hu, hv) at the cubature nodes
    __shared__ float sF[3][E][NGF];     // Fscale Fn* at the Gauss nodes
    __shared__ float sLam[E][NGF];

    const int tid = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int k0 = a.k_begin + blk * E;
    for (int t = tid; t < NC * Np; t += 256) {
        sIc[t] = a.ops.oIc[t];
        sPr[t] = a.ops.oPr[t];
        sPs[t] = a.ops.oPs[t];
        sP[t] = a.ops.oP[t];
    }
    for (int t = tid; t < Np * NGF; t += 256) sLg[t] = a.ops.oLg[t];
    for (int t = tid; t < NG * Nfp; t += 256) sI1[t] = a.ops.oI1[t];

    const int e = tid / W;
    const int i = tid - e * W;
    const int k = k0 + e;
    const bool live = e < E && k < a.k_end;
    const long long KNp = a.KNp;
    const float g = a.g, hvel = a.hvel;
    // ---- nodal data of the element (lanes i < Np)
    float etak = 0.f, lok = 0.f;
    LevelArgs L = a.lev[0];
    if (live) {
        L = pick_level(a, level_of(a, k));
        const float* Q = a.Q[L.parity];
        const long long b0 = (long long)k * Np;
        etak = Q[b0];
        lok = lo_decode(etak, reinterpret_cast<const short*>(Q + 3 * KNp)[b0]);
        if (i < Np) {
            const long long idx = b0 + i;
            const float eta = Q[idx];
            const float lo = lo_decode(eta, reinterpret_cast<const short*>(Q + 3 * KNp)[idx]);
            const float Bn = a.B[idx];
            const float bl = lo_decode(Bn, a.Blo[idx]);
            sN[0][e][i] = (eta - Bn) + (lo - bl);
            sN[1][e][i] = (eta - etak) + (lo - lok);
            sN[2][e][i] = Q[KNp + idx];
            sN[3][e][i] = Q[2 * KNp + idx];
            sN[4][e][i] = a.dB[idx];
            sN[5][e][i] = a.dB[KNp + idx];
        }
    }
    // ---- exterior values at the own face nodes (lanes i < 3 (N+1))
    if (live && i < nF) {
        const int f = i / Nfp, j = i - f * Nfp;
        const int4 cn = reinterpret_cast<const int4*>(a.conn)[k];
        const int nb = f == 0 ? cn.x : (f == 1 ? cn.y : cn.z);
        if (nb >= 0) {
            const int f2 = (cn.w >> (2 * f)) & 3;
            const int l2 = level_of(a, nb);
            const LevelArgs L2 = pick_level(a, l2);
            const long long id2 = (long long)nb * Np + a.ops.fmask[f2 * Nfp + (Nfp - 1 - j)];
            const float BP = a.B[id2];
            const float blP = lo_decode(BP, a.Blo[id2]);
            const long long idM = (long long)k * Np + a.ops.fmask[i];
            const float BM = a.B[idM];
            const float blM = lo_decode(BM, a.Blo[idM]);
            float etaP, loP = 0.f, huP, hvP;
            if (L2.active || a.half == nullptr) {
                const float* Q2 = a.Q[L2.parity];
                etaP = Q2[id2];
                huP = Q2[KNp + id2];
                hvP = Q2[2 * KNp + id2];
                loP = lo_decode(etaP, reinterpret_cast<const short*>(Q2 + 3 * KNp)[id2]);
            } else {
                const long long hid = (long long)nb * nF + f2 * Nfp + (Nfp - 1 - j);
                etaP = a.half[hid];
                huP = a.half[a.KnF + hid];
                hvP = a.half[2 * a.KnF + hid];
            }
            sT[0][e][i] = (etaP - BP) + (loP - blP);
            sT[1][e][i] = huP;
            sT[2][e][i] = hvP;
            sT[3][e][i] = (etaP - etak) + (loP - lok);
            sT[4][e][i] = (BP - BM) + (blP - blM);
        }
    }
    __syncthreads();
    if (live && i < nF) {
        const int f = i / Nfp;
        const int4 cn = reinterpret_cast<const int4*>(a.conn)[k];
        const int nb = f == 0 ? cn.x : (f == 1 ? cn.y : cn.z);
        if (nb < 0) {   // reflective wall: the mirror state, same bed
            const int n = a.ops.fmask[i];
            const float* gk = a.geo + 16LL * k;
            const float nx = gk[4 + f], ny = gk[7 + f];
            const float huM = sN[2][e][n], hvM = sN[3][e][n];
            const float mn = huM * nx + hvM * ny;
            sT[0][e][i] = sN[0][e][n];
            sT[1][e][i] = huM - 2.f * mn * nx;
            sT[2][e][i] = hvM - 2.f * mn * ny;
            sT[3][e][i] = sN[1][e][n];
            sT[4][e][i] = 0.f;
        }
    }
    // ---- volume fluxes and source at the cubature nodes (lanes i < Ncub)
    if (live && i < NC) {
        float h = 0.f, d = 0.f, hu = 0.f, hv = 0.f, bx = 0.f, by = 0.f;
#pragma unroll
        for (int n = 0; n < Np; ++n) {
            const float c = sIc[i * Np + n];
            h += c * sN[0][e][n];
            d += c * sN[1][e][n];
            hu += c * sN[2][e][n];
            hv += c * sN[3][e][n];
            bx += c * sN[4][e][n];
            by += c * sN[5][e][n];
        }
        const float4 g0 = reinterpret_cast<const float4*>(a.geo)[4LL * k];   // rx, ry, sx, sy
        const float fv = vel_factor(h, hvel);
        const float u = hu * fv, v = hv * fv;
        const float p = 0.5f * g * (d * (2.f * h - d));
        const float F[3] = {hu, hu * u + p, hu * v};
        const float G[3] = {hv, hv * u, hv * v + p};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sC[c][e][i] = g0.x * F[c] + g0.y * G[c];
            sC[3 + c][e][i] = g0.z * F[c] + g0.w * G[c];
        }
        sC[6][e][i] = -g * d * bx;
        sC[7][e][i] = -g * d * by;
    }
    __syncthreads();
    // ---- numerical flux at the Gauss nodes (lanes i < 3 NG)
    float hsM = 0.f, hsP = 0.f, uM = 0.f, vM = 0.f, uP = 0.f, vP = 0.f, jump = 0.f;
    float hM = 0.f, dM = 0.f, huM = 0.f, hvM = 0.f, huP = 0.f, hvP = 0.f, nx = 0.f, ny = 0.f, fs = 0.f;
    if (live && i < NGF) {
        const int f = i / NG, gq = i - f * NG;
        float hP = 0.f, dP = 0.f, dB = 0.f;
#pragma unroll
        for (int j = 0; j < Nfp; ++j) {
            const float c = sI1[gq * Nfp + j];
            const int n = a.ops.fmask[f * Nfp + j];
            const int t = f * Nfp + j;
            hM += c * sN[0][e][n];
            dM += c * sN[1][e][n];
            huM += c * sN[2][e][n];
            hvM += c * sN[3][e][n];
            hP += c * sT[0][e][t];
            huP += c * sT[1][e][t];
            hvP += c * sT[2][e][t];
            dP += c * sT[3][e][t];
            dB += c * sT[4][e][t];
        }
        const float* gk = a.geo + 16LL * k;
        nx = gk[4 + f];
        ny = gk[7 + f];
        fs = gk[10 + f];
        // Eq. 5.1 with max(B-, B+) - B- = max(0, dB), max(B-, B+) - B+ = max(0, -dB)
        hsM = fmaxf(0.f, hM - fmaxf(0.f, dB));
        hsP = fmaxf(0.f, hP - fmaxf(0.f, -dB));
        // both sides wet: h*+ - h*- = eta+ - eta-, formed from the levels
        jump = (hsM > 0.f && hsP > 0.f) ? dP - dM : hsP - hsM;
        const float fM = vel_factor(hM, hvel), fP = vel_factor(hP, hvel);
        uM = huM * fM;
        vM = hvM * fM;
        uP = huP * fP;
        vP = hvP * fP;
        const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
        sLam[e][i] = fmaxf(fabsf(unM) + sqrtf(g * hsM), fabsf(unP) + sqrtf(g * hsP));
    }
    __syncthreads();
    if (live && i < NGF) {
        const int f = i / NG;
        float lam = sLam[e][f * NG];
#pragma unroll
        for (int t = 1; t < NG; ++t) lam = fmaxf(lam, sLam[e][f * NG + t]);
        const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
        const float pc = 0.5f * g * (dM * (2.f * hM - dM)) + 0.25f * g * jump * (hsP + hsM);
        sF[0][e][i] = fs * (0.5f * (hsM * unM + hsP * unP) - 0.5f * lam * jump);
        sF[1][e][i] = fs * (0.5f * (hsM * uM * unM + hsP * uP * unP) + pc * nx - 0.5f * lam * (hsP * uP - hsM * uM));
        sF[2][e][i] = fs * (0.5f * (hsM * vM * unM + hsP * vP * unP) + pc * ny - 0.5f * lam * (hsP * vP - hsM * vM));
    }
    __syncthreads();
    // ---- projection to the nodes (lanes i < Np)
    if (!live || i >= Np) return;
    float r0 = 0.f, r1 = 0.f, r2 = 0.f;
#pragma unroll 4
    for (int c = 0; c < NC; ++c) {
        const float pr = sPr[i * NC + c], ps = sPs[i * NC + c], pp = sP[i * NC + c];
        r0 += pr * sC[0][e][c] + ps * sC[3][e][c];
        r1 += pr * sC[1][e][c] + ps * sC[4][e][c] + pp * sC[6][e][c];
        r2 += pr * sC[2][e][c] + ps * sC[5][e][c] + pp * sC[7][e][c];
    }
#pragma unroll
    for (int t = 0; t < NGF; ++t) {
        const float lg = sLg[i * NGF + t];
        r0 -= lg * sF[0][e][t];
        r1 -= lg * sF[1][e][t];
        r2 -= lg * sF[2][e][t];
    }
    float* R0 = a.R[L.slot[0]];
    const long long idx = (long long)k * Np + i;
    R0[idx] = r0;
    R0[KNp + idx] = r1;
    R0[2 * KNp + idx] = r2;
}

// ---------------------------------------------------------------------------
// characteristic rows L of the flux Jacobian in direction (ex, ey) at a cell
// mean (Section 5.3, Cockburn-Shu), FP64
// ---------------------------------------------------------------------------
__device__ __forceinline__ void char_left(double hb, double mu, double mv, double g, double ex,
                                          double ey, double Lm[3][3]) {
    const double ub = mu / hb, vb = mv / hb;
    const double c = sqrt(g * hb);
    const double un = ub * ex + vb * ey, ut = -ub * ey + vb * ex;
    const double i2c = 0.5 / c;
    Lm[0][0] = (un + c) * i2c; Lm[0][1] = -ex * i2c; Lm[0][2] = -ey * i2c;
    Lm[1][0] = -ut;            Lm[1][1] = -ey;       Lm[1][2] = ex;
    Lm[2][0] = -(un - c) * i2c; Lm[2][1] = ex * i2c; Lm[2][2] = ey * i2c;
}

// ---------------------------------------------------------------------------
// step kernel with the contraction on the matrix cores (N <= 4, Np <= 16)
//
// Lanes are element-aligned: a wave holds 4 elements, lane 16q + j is node j
// of element q, and every LDS row a wave touches is its own, so waves only
// order their own LDS traffic (no block barriers).
// Contraction: R^T = X^T [Dr Ds LIFT]^T on the matrix cores with rows
// (element q, field f) and columns = nodes, so lane 16q + j receives R of
// element q at node j for f = 0..2.  X^T rows = (-X_r, -X_s, Fscale dF) of h,
// hu, hv (row 3 of each element is not contracted).  Engines: FP32 on
// v_mfma_f32_16x16x4f32, or BF16 on v_mfma_f32_16x16x32_bf16 with both
// operands split into two or three BF16 parts and the split products
// accumulated in FP32.  The bed gradient of the source term is static and
// comes from the host (FP64).  Element reductions (means and P1
// edge-midpoint deviations of h, hu, hv) are W V on v_mfma_f64_16x16x4f64 in
// FP64 (W rows: w/2 and the three midpoint functionals).
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// K layout of the X^T rows in LDS.  FP32 engine (v_mfma_f32_16x16x4f32): K
// index k is supplied by lane group k % 4 at step k / 4.  BF16 engine
// (v_mfma_f32_16x16x32_bf16): lane group g supplies K = 32 s + 8 g .. +7 at
// step s.  Each group's values are contiguous so a lane reads its slice of a
// row with float4 loads.
template <int N, int BF>
struct MShape {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int nF = 3 * (N + 1);
    static constexpr int LPE = mfma_lanes(N);                         // lanes per element
    static constexpr int EPW = 64 / LPE;                              // elements per wave
    static constexpr int NT = mfma_tiles(N);                          // 16-node column tiles
    static constexpr bool CMP = mfma_compact(N);                      // packed lane groups
    static constexpr int KQ = BF ? 32 : 4;                            // K per MFMA step
    static constexpr int KV = mfma_kv(N);                             // first LIFT column
    static constexpr int KS = BF ? (KV + nF + 31) / 32 : mfma_steps(N);
    static constexpr int SV = KV / KQ;                                // volume-only steps
    static constexpr int KSP = BF ? KS : (KS + 3) & ~3;               // FP32: steps padded to float4
    static constexpr int RL = BF ? 32 * KS : 4 * KSP;                 // row length (floats)
    static constexpr int RS = RL + 4;                                 // LDS row stride (floats)
    static constexpr int KR = (Np + 3) / 4;                           // FP64 reduction steps
    static_assert(Np <= LPE && nF <= LPE, "element must fit its lane group");
    static_assert(CMP ? 3 * EPW <= 16 : (LPE == 16 && NT == 1), "one 16-row tile of element x field rows");
    static constexpr int OR = 20;   // row stride (floats) of the packed layout's result transpose
    // load schedule, chosen per order by measurement: EARLY issues the
    // operator table's loads first and writes them to LDS before the
    // neighbour loads, issues every element-indexed load before the wait for
    // the connectivity, and loads the reduction weights ahead of the
    // reduction (N = 4: 41 -> 35 us per C2 step, N = 5: 668 -> 619 us per C4
    // step); at N = 3 the compiler's own order with the table copied after
    // the neighbour loads is faster (1045 against 1124 us per C5 step)
    static constexpr bool EARLY = N != 3;
    // packed groups: element r / 3 and field r % 3 of row r < 3 EPW from
    // 4-bit and 2-bit tables (rows past 3 EPW map to element 0, field 0)
    static constexpr unsigned long long row_element_bits() {
        unsigned long long b = 0;
        for (int r = 0; r < 16; ++r) b |= (unsigned long long)(r < 3 * EPW ? r / 3 : 0) << (4 * r);
        return b;
    }
    static constexpr unsigned row_field_bits() {
        unsigned b = 0;
        for (int r = 0; r < 16; ++r) b |= (unsigned)(r < 3 * EPW ? r % 3 : 0) << (2 * r);
        return b;
    }
    static __device__ __forceinline__ int row_element(int r) { return (int)((row_element_bits() >> (4 * r)) & 15ull); }
    static __device__ __forceinline__ int row_field(int r) { return (int)((row_field_bits() >> (2 * r)) & 3u); }
    static __device__ __forceinline__ int perm(int k) {
        if constexpr (BF) return ((k >> 3) & 3) * (8 * KS) + (k >> 5) * 8 + (k & 7);
        else return (k & 3) * KSP + (k >> 2);
    }
};

// BF16 split of eight FP32 values into P parts: x_0 = bf16(x), x_1 =
// bf16(x - x_0), x_2 = bf16(x - x_0 - x_1) (each remainder is exact in FP32)
template <int P>
__device__ __forceinline__ void bf16_split(const float4& x0, const float4& x1, bf16x8 (&part)[P]) {
    const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        float r = v[i];
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const __bf16 b = (__bf16)r;
            part[t][i] = b;
            if (t + 1 < P) r -= (float)b;
        }
    }
}

// split-precision products of one K = 32 step, accumulated in FP32 from the
// smallest term up: P = 2: x1 o0 + x0 o1 + x0 o0; P = 3: x2 o0 + x1 o1 +
// x0 o2 + x1 o0 + x0 o1 + x0 o0 (terms below 2^-24 of the product dropped)
template <int P>
__device__ __forceinline__ floatx4 bf16_products(const bf16x8 (&x)[P], const bf16x8* o, floatx4 acc) {
    if constexpr (P == 2) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], o[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], o[1], acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[2], o[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], o[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], o[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1], o[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], o[1], acc, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0], o[0], acc, 0, 0, 0);
}

// face node fn of the reference element from a 4-bit packed table (N <= 4)
template <int N>
__device__ __forceinline__ int face_node(int fn) {
    if constexpr (N <= 4) {   // 3(N+1) entries of 4 bits fit 64 bits
        constexpr unsigned long long bits = face_node_bits(N);
        return (int)((bits >> (4 * fn)) & 15ull);
    } else if constexpr (N == 5) {   // 18 entries of 5 bits in two words
        constexpr unsigned long long b0 = face_node_bits5(N, 0), b1 = face_node_bits5(N, 1);
        const bool up = fn >= 12;
        return (int)(((up ? b1 : b0) >> (5 * (up ? fn - 12 : fn))) & 31ull);
    } else {
        return face_node_index(N, fn);
    }
}

// value of x in the lane whose byte address (4 x lane) is given; every lane
// of the wave active
__device__ __forceinline__ float lane_f32(float x, int byte_addr) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(byte_addr, __builtin_bit_cast(int, x)));
}

__device__ __forceinline__ void wave_lds_sync() {
    // order this wave's LDS writes before its reads of other lanes' data
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// element load at a 32-bit element index from a uniform base
template <typename T>
__device__ __forceinline__ T ldg(const T* base, unsigned i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T* base, unsigned i, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T)) = v;
}

// Raw buffer view of an FP32 array: a resource descriptor in scalar
// registers and 32-bit byte offsets (element offset in a vector register,
// field offset in a scalar one), so no 64-bit address arithmetic per lane;
// accesses beyond `bytes` read 0 and write nothing.
struct BufF32 {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BufF32(const float* p, unsigned bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, (int)bytes, 0x00020000)) {}
    __device__ __forceinline__ float ld(unsigned i, unsigned field_bytes) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(i * 4u), (int)field_bytes, 0));
    }
    __device__ __forceinline__ float ldb(unsigned byte_off, unsigned field_bytes) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, (int)field_bytes, 0));
    }
    // 16-bit field (the level's low word): element i at field_bytes + 2 i
    __device__ __forceinline__ short ld16(unsigned i, unsigned field_bytes) const {
        return (short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)(i * 2u), (int)field_bytes, 0);
    }
    __device__ __forceinline__ short ldb16(unsigned byte_off, unsigned field_bytes) const {
        return (short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)byte_off, (int)field_bytes, 0);
    }
    __device__ __forceinline__ void st16(unsigned i, unsigned field_bytes, short v) const {
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, (int)(i * 2u), (int)field_bytes, 0);
    }
    __device__ __forceinline__ void st(unsigned i, unsigned field_bytes, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)(i * 4u), (int)field_bytes, 0);
    }
};


// ---------------------------------------------------------------------------
// The same right-hand side with its contractions on the matrix cores
// (v_mfma_f32_16x16x4f32).  One wave = 4 elements, lane 16 e + c; blocks of
// one wave, so waves never wait on each other.
//  * stage 1: [h, d, hu, hv] and [dB/dx, dB/dy] at the cubature nodes as
//    X1^T Ic^T, rows (element, field) and columns the cubature nodes, so lane
//    16 e + c receives element e's values at cubature node 16 t + c of
//    column tile t;
//  * stage 2: that lane forms cF1, cF2 and cS there (perturbation form as in
//    the vector kernel);
//  * faces: exterior traces at the face nodes and the numerical flux at the
//    Gauss points, lanes looping over the element's points;
//  * stage 3: R^T = X3^T [Pr Ps P -L^g]^T, rows (element, field) and columns
//    the nodes, the K range cF1 | cF2 | cS | Fscale Fn* passed through one
//    LDS buffer in four chunks; lane 16 e + c receives R of element e at node
//    16 tn + c.
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(64) rhs_overint_mfma_kernel(StepArgs a) {
    constexpr int Np = (N + 1) * (N + 2) / 2, Nfp = N + 1, nF = 3 * (N + 1);
    constexpr int Q = overint_points(N), NC = Q * Q, NG = Q, NGF = 3 * Q;
    constexpr int S1 = overint_mfma_s1(N), T1 = overint_mfma_t1(N), SC = overint_mfma_sc(N);
    constexpr int SG = overint_mfma_sg(N), TN = overint_mfma_tn(N), ST3 = overint_mfma_t3_steps(N);
    constexpr int KC = 4 * SC, KG = 4 * SG;
    // row strides: odd multiples of 4 dwords, so that the 16 rows x 4 k of an
    // A-operand read, and the four elements' rows of a write, fall in
    // distinct banks
    constexpr int X1S = 4 * ((S1 + 1) | 1);
    constexpr int XS = 4 * (((KC > KG ? KC : KG) / 4 + 1) | 1);
    constexpr int NI = (NGF + 15) / 16;                 // Gauss points per lane
    __shared__ __attribute__((aligned(16))) float sX1[2][16][X1S];
    __shared__ __attribute__((aligned(16))) float sX3[16][XS];
    __shared__ float sNd[4][4][Np];                     // own h, d, hu, hv at the nodes
    __shared__ float sFn[4][5][nF];                     // exterior h, hu, hv, d; B+ - B-, own face nodes
    __shared__ float sFg[4][3][NGF];                    // Fscale Fn* at the Gauss points
    __shared__ float sLam[4][NGF];

    const int lane = threadIdx.x;
    const int e = lane >> 4, c = lane & 15;
    const int k = a.k_begin + xcd_remap(blockIdx.x, gridDim.x) * 4 + e;
    const bool live = k < a.k_end;
    const int kc = live ? k : a.k_end - 1;            // clamped: loads stay in range
    const long long KNp = a.KNp;
    const float g = a.g, hvel = a.hvel;
    const LevelArgs L = pick_level(a, level_of(a, kc));
    const float* Qs = a.Q[L.parity];
    const short* Qlo = reinterpret_cast<const short*>(Qs + 3 * KNp);
    const long long b0 = (long long)kc * Np;
    const float etak = Qs[b0];
    const float lok = lo_decode(etak, Qlo[b0]);
    // loads that depend on the element alone go out first: the metric terms,
    // the connectivity and (where they fit in registers) the stage-1 B operands
    const float4 g0 = ldg(reinterpret_cast<const float4*>(a.geo), 4u * (unsigned)kc);   // rx, ry, sx, sy
    const int4 cn = ldg(reinterpret_cast<const int4*>(a.conn), (unsigned)kc);
    constexpr bool PF1 = T1 * S1 <= 8;
    float b1[PF1 ? T1 : 1][PF1 ? S1 : 1];
    if constexpr (PF1) {
#pragma unroll
        for (int t = 0; t < T1; ++t)
#pragma unroll
            for (int st = 0; st < S1; ++st) b1[t][st] = ldg(a.ops.oT1, (unsigned)((t * S1 + st) * 64 + lane));
    }
    // ---- nodal data into the stage-1 rows and the node table
    for (int j = c; j < 4 * S1; j += 16) {
        float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (j < Np) {
            const long long idx = b0 + j;
            const float eta = Qs[idx];
            const float lo = lo_decode(eta, Qlo[idx]);
            const float Bn = a.B[idx];
            const float bl = lo_decode(Bn, a.Blo[idx]);
            v[0] = (eta - Bn) + (lo - bl);
            v[1] = (eta - etak) + (lo - lok);
            v[2] = Qs[KNp + idx];
            v[3] = Qs[2 * KNp + idx];
            v[4] = a.dB[idx];
            v[5] = a.dB[KNp + idx];
#pragma unroll
            for (int f = 0; f < 4; ++f) sNd[e][f][j] = v[f];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) sX1[0][4 * e + f][j] = v[f];
        sX1[1][4 * e + 0][j] = v[4];
        sX1[1][4 * e + 1][j] = v[5];
        sX1[1][4 * e + 2][j] = 0.f;
        sX1[1][4 * e + 3][j] = 0.f;
    }
    wave_lds_sync();
    // ---- stage 1 on the matrix cores
    const int ar = lane & 15, ak = lane >> 4;
    floatx4 acc1[2][T1];
#pragma unroll
    for (int tr = 0; tr < 2; ++tr)
#pragma unroll
        for (int t = 0; t < T1; ++t) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < S1; ++st)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(
                    sX1[tr][ar][4 * st + ak],
                    PF1 ? b1[PF1 ? t : 0][PF1 ? st : 0] : ldg(a.ops.oT1, (unsigned)((t * S1 + st) * 64 + lane)),
                    acc, 0, 0, 0);
            acc1[tr][t] = acc;
        }
    // ---- stage 2: fluxes and source at this lane's cubature nodes
    float cf[T1][8];
#pragma unroll
    for (int t = 0; t < T1; ++t) {
        const bool on = 16 * t + c < NC;
        const float h = acc1[0][t][0], d = acc1[0][t][1], hu = acc1[0][t][2], hv = acc1[0][t][3];
        const float bx = acc1[1][t][0], by = acc1[1][t][1];
        const float fv = vel_factor(h, hvel);
        const float u = hu * fv, v = hv * fv;
        const float pr = 0.5f * g * (d * (2.f * h - d));
        const float F[3] = {hu, hu * u + pr, hu * v};
        const float G[3] = {hv, hv * u, hv * v + pr};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            cf[t][r] = on ? g0.x * F[r] + g0.y * G[r] : 0.f;
            cf[t][3 + r] = on ? g0.z * F[r] + g0.w * G[r] : 0.f;
        }
        cf[t][6] = on ? -g * d * bx : 0.f;
        cf[t][7] = on ? -g * d * by : 0.f;
    }
    // ---- faces: exterior traces at the own face nodes
    const float* gk = a.geo + 16LL * kc;
    for (int pn = c; pn < nF; pn += 16) {
        const int f = pn / Nfp, j = pn - f * Nfp;
        const int n = face_node_index(N, pn);
        const int nb = f == 0 ? cn.x : (f == 1 ? cn.y : cn.z);
        float hP, huP, hvP, dP, dB;
        if (nb >= 0) {
            const int f2 = (cn.w >> (2 * f)) & 3;
            const LevelArgs L2 = pick_level(a, level_of(a, nb));
            const long long id2 = (long long)nb * Np + face_node_index(N, f2 * Nfp + (Nfp - 1 - j));
            const float BP = a.B[id2];
            const float blP = lo_decode(BP, a.Blo[id2]);
            const long long idM = b0 + n;
            const float BM = a.B[idM];
            const float blM = lo_decode(BM, a.Blo[idM]);
            float etaP, loP = 0.f;
            if (L2.active || a.half == nullptr) {
                const float* Q2 = a.Q[L2.parity];
                etaP = Q2[id2];
                huP = Q2[KNp + id2];
                hvP = Q2[2 * KNp + id2];
                loP = lo_decode(etaP, reinterpret_cast<const short*>(Q2 + 3 * KNp)[id2]);
            } else {
                const long long hid = (long long)nb * nF + f2 * Nfp + (Nfp - 1 - j);
                etaP = a.half[hid];
                huP = a.half[a.KnF + hid];
                hvP = a.half[2 * a.KnF + hid];
            }
            hP = (etaP - BP) + (loP - blP);
            dP = (etaP - etak) + (loP - lok);
            dB = (BP - BM) + (blP - blM);
        } else {   // reflective wall: the mirror state, same bed
            const float nx = gk[4 + f], ny = gk[7 + f];
            const float huM = sNd[e][2][n], hvM = sNd[e][3][n];
            const float mn = huM * nx + hvM * ny;
            hP = sNd[e][0][n];
            huP = huM - 2.f * mn * nx;
            hvP = hvM - 2.f * mn * ny;
            dP = sNd[e][1][n];
            dB = 0.f;
        }
        sFn[e][0][pn] = hP;
        sFn[e][1][pn] = huP;
        sFn[e][2][pn] = hvP;
        sFn[e][3][pn] = dP;
        sFn[e][4][pn] = dB;
    }
    wave_lds_sync();
    // ---- numerical flux at the Gauss points (lanes loop over the element's points)
    float gh[NI][8];   // hsM, hsP, uM, vM, uP, vP, jump, pressure part (without the jump term)
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int pg = c + 16 * it;
        for (int q = 0; q < 8; ++q) gh[it][q] = 0.f;
        if (pg >= NGF) continue;
        const int f = pg / NG, gq = pg - f * NG;
        float hM = 0.f, dM = 0.f, huM = 0.f, hvM = 0.f, hP = 0.f, huP = 0.f, hvP = 0.f, dP = 0.f, dB = 0.f;
#pragma unroll
        for (int j = 0; j < Nfp; ++j) {
            const float w = ldg(a.ops.oI1, (unsigned)(gq * Nfp + j));
            const int n = face_node_index(N, f * Nfp + j);
            const int t = f * Nfp + j;
            hM += w * sNd[e][0][n];
            dM += w * sNd[e][1][n];
            huM += w * sNd[e][2][n];
            hvM += w * sNd[e][3][n];
            hP += w * sFn[e][0][t];
            huP += w * sFn[e][1][t];
            hvP += w * sFn[e][2][t];
            dP += w * sFn[e][3][t];
            dB += w * sFn[e][4][t];
        }
        const float nx = gk[4 + f], ny = gk[7 + f];
        const float hsM = fmaxf(0.f, hM - fmaxf(0.f, dB));
        const float hsP = fmaxf(0.f, hP - fmaxf(0.f, -dB));
        const float jump = (hsM > 0.f && hsP > 0.f) ? dP - dM : hsP - hsM;
        const float fM = vel_factor(hM, hvel), fP = vel_factor(hP, hvel);
        const float uM = huM * fM, vM = hvM * fM, uP = huP * fP, vP = hvP * fP;
        const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
        sLam[e][pg] = fmaxf(fabsf(unM) + sqrtf(g * hsM), fabsf(unP) + sqrtf(g * hsP));
        gh[it][0] = hsM;
        gh[it][1] = hsP;
        gh[it][2] = uM;
        gh[it][3] = vM;
        gh[it][4] = uP;
        gh[it][5] = vP;
        gh[it][6] = jump;
        gh[it][7] = 0.5f * g * (dM * (2.f * hM - dM));
    }
    wave_lds_sync();
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int pg = c + 16 * it;
        if (pg >= NGF) continue;
        const int f = pg / NG;
        float lam = sLam[e][f * NG];
#pragma unroll
        for (int t = 1; t < NG; ++t) lam = fmaxf(lam, sLam[e][f * NG + t]);
        const float nx = gk[4 + f], ny = gk[7 + f], fs = gk[10 + f];
        const float hsM = gh[it][0], hsP = gh[it][1], uM = gh[it][2], vM = gh[it][3];
        const float uP = gh[it][4], vP = gh[it][5], jump = gh[it][6];
        const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
        const float pc = gh[it][7] + 0.25f * g * jump * (hsP + hsM);
        sFg[e][0][pg] = fs * (0.5f * (hsM * unM + hsP * unP) - 0.5f * lam * jump);
        sFg[e][1][pg] = fs * (0.5f * (hsM * uM * unM + hsP * uP * unP) + pc * nx - 0.5f * lam * (hsP * uP - hsM * uM));
        sFg[e][2][pg] = fs * (0.5f * (hsM * vM * unM + hsP * vP * unP) + pc * ny - 0.5f * lam * (hsP * vP - hsM * vM));
    }
    // ---- stage 3: four K chunks through the LDS buffer
    floatx4 acc3[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) acc3[tn] = floatx4{0.f, 0.f, 0.f, 0.f};
    // the chunk's B operands are loaded before its LDS round trip so that
    // their latency overlaps it (where they fit in registers: N <= 4)
    constexpr int SM = SC > SG ? SC : SG;
    constexpr bool PF = TN * SM <= 16;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        const int nst = ch < 3 ? SC : SG;
        const int off = ch < 3 ? ch * SC : 3 * SC;
        float bop[PF ? TN : 1][PF ? SM : 1];
        if constexpr (PF) {
#pragma unroll
            for (int tn = 0; tn < TN; ++tn)
#pragma unroll
                for (int st = 0; st < SM; ++st)
                    if (st < nst) bop[tn][st] = ldg(a.ops.oT3, (unsigned)(((tn * ST3) + off + st) * 64 + lane));
        }
        wave_lds_sync();   // the previous chunk's reads (and the flux writes) are done
        if (ch < 3) {
            // rows (e, r): cF1_r, cF2_r or cS_r (cS_h = 0) at cubature node 16 t + c
#pragma unroll
            for (int t = 0; t < T1; ++t) {
                const int cp = 16 * t + c;
                if (cp < KC) {
#pragma unroll
                    for (int r = 0; r < 3; ++r)
                        sX3[4 * e + r][cp] = ch == 0 ? cf[t][r] : (ch == 1 ? cf[t][3 + r] : (r == 0 ? 0.f : cf[t][5 + r]));
                    sX3[4 * e + 3][cp] = 0.f;
                }
            }
        } else {
            for (int pg = c; pg < KG; pg += 16) {
#pragma unroll
                for (int r = 0; r < 3; ++r) sX3[4 * e + r][pg] = pg < NGF ? sFg[e][r][pg] : 0.f;
                sX3[4 * e + 3][pg] = 0.f;
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
#pragma unroll
            for (int st = 0; st < SM; ++st) {
                if (st >= nst) break;
                const float bv = PF ? bop[PF ? tn : 0][PF ? st : 0]
                                    : ldg(a.ops.oT3, (unsigned)(((tn * ST3) + off + st) * 64 + lane));
                acc3[tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(sX3[ar][4 * st + ak], bv, acc3[tn], 0, 0, 0);
            }
    }
    // ---- lane 16 e + c holds R of element e at node 16 tn + c (rows 4 e .. 4 e + 2)
    if (!live) return;
    float* R0 = a.R[L.slot[0]];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const int node = 16 * tn + c;
        if (node >= Np) continue;
        const long long idx = (long long)k * Np + node;
        R0[idx] = acc3[tn][0];
        R0[KNp + idx] = acc3[tn][1];
        R0[2 * KNp + idx] = acc3[tn][2];
    }
}

// occupancy target (waves per SIMD) of the matrix-core kernel: what its
// register use allows without spills (the BF16 splits and the multi-rate
// bookkeeping hold more live values; N = 5 holds two accumulator tiles)
constexpr int mfma_waves_target(int N, bool multi, int bf) {
    return (bf == 2 ? (multi ? 4 : 5) : (bf ? (multi ? 5 : 6) : (multi ? 6 : 7))) - (N == 5 ? 1 : 0);
}

// UPD: the update alone (MODE_UPDATE_ONLY of the over-integrated form): the
// right-hand side is read from the ring slot another kernel wrote, and the
// AB update, the FP64 reductions, the positivity limiter and the hand-off to
// the TVB kernel run as in the fused kernel
template <int N, bool MULTI, int WPB, int BF, bool UPD = false>
__global__ void __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(mfma_waves_target(N, MULTI, BF), 8)))
step_mfma_kernel(StepArgs a) {
    using S = MShape<N, BF>;
    constexpr int Np = S::Np, Nfp = S::Nfp, nF = S::nF, KV = S::KV, KS = S::KS, SV = S::SV;
    constexpr int KSP = S::KSP, RS = S::RS, RL = S::RL, LPE = S::LPE, EPW = S::EPW, NT = S::NT;
    // LDS is per wave (its EPW elements): the X^T rows, and after they have
    // been read into registers, the FP64 node values and reductions in the
    // same bytes
    struct WaveLds {
        union {
            float A[EPW][3][RS];
            float O[NT * 16][S::OR];   // packed layout: contraction result, node-major
            struct {
                double Vd[EPW][3][LPE + 1];   // updated h, hu, hv per node (rows padded
                                              // so the reduction's column reads
                                              // fall in distinct banks)
                double Red[EPW][16];      // 1-3 means, 4-12 deviations
            } r;
        };
    };
    __shared__ __attribute__((aligned(16))) WaveLds lds[WPB];
    // FP32 operator table of the block: lane l of tile t reads its KS steps
    // as float4 chunks from row t * 64 + l (row stride padded so that the
    // 128-bit reads of consecutive lanes fall in distinct banks)
    // (blocks of four or eight waves; smaller blocks read the table from global
    // memory, so the launch-shape search covers both ways)
    constexpr bool OPL = !BF && WPB >= 4 && !UPD;
    constexpr int OPS = (S::KSP % 8 == 0) ? S::KSP + 4 : S::KSP;
    static_assert(BF || OPS == mfma_lds_row(N), "LDS image row stride");
    // blocks that stage the operator table also stage the FP64 reduction
    // weights (one float4 per thread) after it, so that no wave loads them
    // from global memory (C4: 607 -> 580 us, C3: 126 -> 120 us per tick)
    constexpr bool WL = OPL;
    constexpr int WOFF = S::NT * 64 * OPS;   // reduction weights after the operator table
    __shared__ __attribute__((aligned(16))) float sOp[OPL ? WOFF + (WL ? 2 * 64 * S::KR : 0) : 4];

    const int tid = threadIdx.x;
    // the block's operator table (four-wave blocks) is copied from its LDS
    // image in global memory as float4 chunks; these loads go out before any
    // other, so that waiting for them does not wait for the state loads
    constexpr int NV4 = OPL ? NT * 64 * OPS / 4 : 1;
    constexpr int SIT = (NV4 + 64 * WPB - 1) / (64 * WPB);
    float4 opv[SIT];
    if constexpr (OPL && S::EARLY) {
#pragma unroll
        for (int i = 0; i < SIT; ++i) {
            const int e = tid + i * 64 * WPB;
            opv[i] = ldg(reinterpret_cast<const float4*>(a.ops.AmfmaL), (unsigned)(e < NV4 ? e : NV4 - 1));
        }
    }
    constexpr int NW4 = 32 * S::KR;   // float4 chunks of the reduction weights
    static_assert(!WL || NW4 <= 64 * WPB, "one chunk of the weights per thread");
    float4 wv = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (WL && S::EARLY) wv = ldg(reinterpret_cast<const float4*>(a.ops.Wred), (unsigned)(tid < NW4 ? tid : 0));
    const int lane = tid & 63, wave = tid >> 6;
    // packed layout: lanes past EPW * LPE are spare; they shadow the wave's
    // last element with the group index LPE (a padding slot everywhere) and
    // are never live
    const bool spare = S::CMP && lane >= EPW * LPE;
    const int q = spare ? EPW - 1 : lane / LPE;
    const int j = spare ? LPE : lane - q * LPE;
    const int gbase = q * LPE;   // first lane of the element
    const int el = wave * EPW + q;
    float (&sA)[EPW][3][RS] = lds[wave].A;
    double (&sVd)[EPW][3][LPE + 1] = lds[wave].r.Vd;
    double (&sRed)[EPW][16] = lds[wave].r.Red;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    // multi-rate: the block's level (uniform) from the launcher's cut of the
    // element range into whole blocks per level
    int lv = 0;
    if constexpr (MULTI) {
#pragma unroll
        for (int t = 1; t < kMaxLevels; ++t) lv += (t < a.nlev && blk >= a.seg_block[t]) ? 1 : 0;
    }
    const LevelArgs L = a.lev[lv];
    const int sbeg = MULTI ? a.seg_begin[lv] : a.k_begin, send = MULTI ? a.seg_end[lv] : a.k_end;
    const int k = sbeg + (blk - (MULTI ? a.seg_block[lv] : 0)) * (EPW * WPB) + el;
    const bool live = !spare && k < send;
    const bool node = live && j < Np;
    // loads are unconditional: lanes past the last element of the block's
    // range read that element and lanes j >= Np read node Np - 1; their
    // results are never stored
    const int kc = live ? k : send - 1;
    const unsigned KNp = (unsigned)a.KNp;
    const float g = a.g, hvel = a.hvel;
    const unsigned idx = (unsigned)kc * Np + (j < Np ? j : Np - 1);

    // ---- independent global loads first
    const float4 g0 = ldg(reinterpret_cast<const float4*>(a.gm), (unsigned)kc);   // rx, ry, sx, sy
    const int4 cn = ldg(reinterpret_cast<const int4*>(a.conn), (unsigned)kc);
    // buffer views of the block's level arrays (byte offsets < 2^32, checked
    // by the host): resolved on the host for single rate, from the level's
    // parity and ring slots for multi-rate
    const unsigned FB = 4u * KNp;   // bytes of one nodal field
    const float* q_in = MULTI ? a.Q[L.parity] : a.q_in;
    float* q_out = MULTI ? a.Q[1 - L.parity] : a.q_out;
    float* r_now = MULTI ? a.R[L.slot[0]] : a.r_now;
    const float* r_prev1 = MULTI ? a.R[L.slot[1]] : a.r_prev1;
    const float* r_prev2 = MULTI ? a.R[L.slot[2]] : a.r_prev2;
    const unsigned QB = 3u * FB + 2u * KNp;   // state buffer: hi, hu, hv (FP32), lo (16-bit)
    const BufF32 bQi(q_in, QB), bQo(q_out, QB), bB(a.B, FB), bdB(a.dB, 2u * FB);
    const BufF32 bBl(reinterpret_cast<const float*>(a.Blo), 2u * KNp);
    const BufF32 bR0(r_now, 3u * FB), bR1(r_prev1, 3u * FB), bR2(r_prev2, 3u * FB);
    float r1[3], r2[3];
    const float eta = bQi.ld(idx, 0);
    const float hu = bQi.ld(idx, FB);
    const float hv = bQi.ld(idx, 2u * FB);
    const float lo = lo_decode(eta, bQi.ld16(idx, 3u * FB));
    const float Bn = bB.ld(idx, 0);
    const float bl = lo_decode(Bn, bBl.ld16(idx, 0));
    const float dBx = UPD ? 0.f : bdB.ld(idx, 0);   // static bed gradient
    const float dBy = UPD ? 0.f : bdB.ld(idx, FB);
    // the RHS history is read unconditionally (slots hold zeros or finite RHS
    // values) and weighted by the level's AB coefficients
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        r1[c] = bR1.ld(idx, c * FB);
        r2[c] = bR2.ld(idx, c * FB);
    }
    const int ag = lane >> 4;   // K group supplied by this lane (contraction, reductions)
    const unsigned HB = 4u * (unsigned)a.KnF;   // bytes of one half-trace field
    const BufF32 bH(a.half, 3u * HB);
    float Rn[3];
    float dtmin;   // the instance's FP32 time step, by the instance id in the connectivity record
    if constexpr (UPD) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Rn[c] = bR0.ld(idx, c * FB);
        dtmin = ldg(a.idt, (unsigned)cn.w >> kConnInstShift);
    } else {
    const bool fnode = live && j < nF;
    const int fn = j < nF ? j : 0;
    const int f = fn / Nfp, jj = fn - f * Nfp;
    // outward normal and Fscale = sJ / J of face f from the metric terms
    // (straight-sided element): the gradient of the coordinate that is
    // constant on the face, -grad s, grad(r + s), -grad r for faces 0, 1, 2,
    // has length sJ / J and points outward
    const float gx = f == 0 ? -g0.z : (f == 1 ? g0.x + g0.z : -g0.x);
    const float gy = f == 0 ? -g0.w : (f == 1 ? g0.y + g0.w : -g0.y);
    const float fs = __builtin_amdgcn_sqrtf(gx * gx + gy * gy);
    const float rfs = __builtin_amdgcn_rcpf(fs);
    const float nx = gx * rfs, ny = gy * rfs;
    if constexpr (S::EARLY) {
        // every load indexed by the element alone goes out before anything
        // waits for the connectivity (loads complete in issue order, so that
        // wait covers none of them), and the operator table, loaded first, is
        // written to LDS
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (OPL) {
            float4* sOp4 = reinterpret_cast<float4*>(sOp);
#pragma unroll
            for (int i = 0; i < SIT; ++i) {
                const int e = tid + i * 64 * WPB;
                if (e < NV4) sOp4[e] = opv[i];
            }
            if constexpr (WL) {
                if (tid < NW4) sOp4[WOFF / 4 + tid] = wv;
            }
        }
    }
    const int n = face_node<N>(fn);
    const int nb = f == 0 ? cn.x : (f == 1 ? cn.y : cn.z);
    // exterior node: node Nfp-1-jj of the neighbour's face f2 (a wall face
    // reads its own face here and is replaced by the mirror state below)
    const int f2 = nb >= 0 ? (cn.w >> (2 * f)) & 3 : f;
    const int nbc = nb >= 0 ? nb : kc;
    const unsigned id2 = (unsigned)nbc * Np + face_node<N>(f2 * Nfp + (Nfp - 1 - jj));
    float BP = bB.ld(id2, 0);
    float blP = lo_decode(BP, bBl.ld16(id2, 0));
    float etaP, huP, hvP, loP = 0.f;
    if constexpr (!MULTI) {
        etaP = bQi.ld(id2, 0);
        huP = bQi.ld(id2, FB);
        hvP = bQi.ld(id2, 2u * FB);
        loP = lo_decode(etaP, bQi.ld16(id2, 3u * FB));
    } else {
        // the neighbour's level: its state buffer (one view spans both
        // parities) or, when it does not step at this tick, its half-step
        // traces
        const int l2 = level_of(a, nbc);
        if (((a.active_bits >> l2) & 1u) || a.half == nullptr) {
            const BufF32 bQ2(a.Q[0], a.q_pair_bytes + QB);
            const unsigned par = ((a.parity_bits >> l2) & 1u) ? a.q_pair_bytes : 0u;
            const unsigned off = id2 * 4u + par;
            etaP = bQ2.ldb(off, 0);
            huP = bQ2.ldb(off, FB);
            hvP = bQ2.ldb(off, 2u * FB);
            loP = lo_decode(etaP, bQ2.ldb16(id2 * 2u + par, 3u * FB));
        } else {
            const unsigned hid = (unsigned)nbc * nF + f2 * Nfp + (Nfp - 1 - jj);
            etaP = bH.ld(hid, 0);
            huP = bH.ld(hid, HB);
            hvP = bH.ld(hid, 2u * HB);
        }
    }
    dtmin = ldg(a.idt, (unsigned)cn.w >> kConnInstShift);

    if constexpr (OPL && !S::EARLY) {
        // the operator table in global order (tile, step, lane) to the LDS
        // rows, after every other load has been issued
        for (int e = tid; e < NT * KS * 64; e += 64 * WPB) {
            const int t = e / (KS * 64), r = e - t * (KS * 64);
            sOp[(t * 64 + (r & 63)) * OPS + (r >> 6)] = ldg(a.ops.Amfma, (unsigned)e);
        }
        if (tid < NW4)
            reinterpret_cast<float4*>(sOp)[WOFF / 4 + tid] = ldg(reinterpret_cast<const float4*>(a.ops.Wred), (unsigned)tid);
    }
    if constexpr (OPL) __syncthreads();   // the block's operator table is in LDS

    const int g4 = 4 * gbase;   // byte address of the element's first lane
    const float eta0 = lane_f32(eta, g4);
    const float lo0 = lane_f32(lo, g4);
    const float dlt = (eta - eta0) + (lo - lo0);

    // ---- X^T rows: volume fluxes (negated), zero padding.  Every lane
    // computes (lanes that are not nodes hold a clamped node's finite data)
    // and lanes that are not nodes store into the unread padding of the row.
    {
        const float h = (eta - Bn) + (lo - bl);
        const float fv = 2.f * h * __builtin_amdgcn_rcpf(h * h + fmaxf(h * h, hvel * hvel));
        const float u = hu * fv, v = hv * fv;
        const float p = 0.5f * g * (dlt * (2.f * h - dlt));
        const float F[3] = {hu, hu * u + p, hu * v};
        const float G[3] = {hv, hv * u, hv * v + p};
        const float rx = g0.x, ry = g0.y, sx = g0.z, sy = g0.w;
        const int nm = -(int)node, pd = RL + (j & 3);   // branch-free selects
        const int cr = pd ^ ((S::perm(j) ^ pd) & nm);
        const int cs = pd ^ ((S::perm(Np + j) ^ pd) & nm);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sA[q][c][cr] = -(rx * F[c] + ry * G[c]);
            sA[q][c][cs] = -(sx * F[c] + sy * G[c]);
        }
    }
    // padding after the volume and after the lift columns (finite: the
    // operator is zero there); one column per lane where they are fewer
    // than the lanes of the element
    constexpr int PV = KV - 2 * Np, PL = RL - (KV + nF);
    static_assert(PV < LPE, "one volume padding column per lane at most");
    if constexpr (PV > 0) {
        if (j < PV) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sA[q][c][S::perm(2 * Np + j)] = 0.f;
        }
    }
    if constexpr (PL > 0 && PL <= LPE) {
        if (j < PL) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sA[q][c][S::perm(KV + nF + j)] = 0.f;
        }
    } else if constexpr (PL > 0) {
        for (int t = j; t < PL; t += LPE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sA[q][c][S::perm(KV + nF + t)] = 0.f;
        }
    }
    wave_lds_sync();

    // ---- volume part of the contraction on the matrix cores, issued before
    // the face flux so that it overlaps the neighbour loads
    // A-operand row r = lane % 16: 16-lane groups: field r % 4 of element
    // r / 4 (field row 3 reads field 0, its results unused), so the result
    // of node j lands in the lane of node j; packed groups: field r % 3 of
    // element r / 3 (rows past 3 EPW read element 0, unused).
    const int ar = lane & 15;
    const int ae = S::CMP ? S::row_element(ar) : (ar >> 2);
    const int arow = S::CMP ? S::row_field(ar) : ((ar & 3) == 3 ? 0 : (ar & 3));
    floatx4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF) {
        constexpr int SV4 = (SV + 3) / 4;   // float4 chunks covering the volume steps
        float av[4 * SV4];
#pragma unroll
        for (int s4 = 0; s4 < SV4; ++s4) {
            const float4 v4 = *reinterpret_cast<const float4*>(&sA[ae][arow][ag * KSP + 4 * s4]);
            av[4 * s4] = v4.x; av[4 * s4 + 1] = v4.y; av[4 * s4 + 2] = v4.z; av[4 * s4 + 3] = v4.w;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float ov[4 * SV4];
#pragma unroll
            for (int s4 = 0; s4 < SV4; ++s4) {
                if constexpr (OPL) {
                    const float4 o4 = *reinterpret_cast<const float4*>(&sOp[(t * 64 + lane) * OPS + 4 * s4]);
                    ov[4 * s4] = o4.x; ov[4 * s4 + 1] = o4.y; ov[4 * s4 + 2] = o4.z; ov[4 * s4 + 3] = o4.w;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (4 * s4 + i < KS) ov[4 * s4 + i] = ldg(a.ops.Amfma, (unsigned)((t * KS + 4 * s4 + i) * 64 + lane));
                }
            }
#pragma unroll
            for (int s = 0; s < SV; ++s) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], ov[s], acc[t], 0, 0, 0);
        }
    } else {
        // X and the operator split into P = BF + 1 BF16 parts; the operator
        // table holds hi, mid, lo parts (the two-part split uses hi, mid)
        constexpr int P = BF + 1;
        const bf16x8* tab = reinterpret_cast<const bf16x8*>(a.ops.Abf);
#pragma unroll
        for (int s = 0; s < SV; ++s) {
            const float* xp = &sA[ae][arow][ag * 8 * KS + 8 * s];
            bf16x8 xs[P];
            bf16_split<P>(*reinterpret_cast<const float4*>(xp), *reinterpret_cast<const float4*>(xp + 4), xs);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                bf16x8 o[P];
#pragma unroll
                for (int u = 0; u < P; ++u) o[u] = ldg(tab, (unsigned)(3 * ((t * KS + s) * 64 + lane) + u));
                acc[t] = bf16_products<P>(xs, o, acc[t]);
            }
        }
    }

    // ---- face node fn = j of element q: reconstructed states, LLF flux
    const int n4 = g4 + 4 * n;
    const float etaM = lane_f32(eta, n4);
    const float huM = lane_f32(hu, n4);
    const float hvM = lane_f32(hv, n4);
    const float BM = lane_f32(Bn, n4);
    const float loM = lane_f32(lo, n4);
    const float blM = lane_f32(bl, n4);
    if (nb < 0) {
        const float mn = huM * nx + hvM * ny;
        etaP = etaM;
        loP = loM;
        BP = BM;
        blP = blM;
        huP = huM - 2.f * mn * nx;
        hvP = hvM - 2.f * mn * ny;
    }
    const float hM = (etaM - BM) + (loM - blM), hP = (etaP - BP) + (loP - blP);
    const float fM = 2.f * hM * __builtin_amdgcn_rcpf(hM * hM + fmaxf(hM * hM, hvel * hvel));
    const float fP = 2.f * hP * __builtin_amdgcn_rcpf(hP * hP + fmaxf(hP * hP, hvel * hvel));
    const float uM = huM * fM, vM = hvM * fM, uP = huP * fP, vP = hvP * fP;
    float Bmax, bmlo;
    bed_max(BM, blM, BP, blP, Bmax, bmlo);
    const float hsM = fmaxf(0.f, (etaM - Bmax) + (loM - bmlo));
    const float hsP = fmaxf(0.f, (etaP - Bmax) + (loP - bmlo));
    const float unM = uM * nx + vM * ny, unP = uP * nx + vP * ny;
    const float lamN = fnode ? fmaxf(fabsf(unM) + __builtin_amdgcn_sqrtf(g * hsM),
                                     fabsf(unP) + __builtin_amdgcn_sqrtf(g * hsP))
                             : 0.f;
    float lam = lamN;
    const int f4 = g4 + 4 * f * Nfp;   // the face's first lane
#pragma unroll
    for (int t = 0; t < Nfp; ++t) lam = fmaxf(lam, lane_f32(lamN, f4 + 4 * t));
    if (fnode) {
        const float dh = depth_jump(etaM, loM, etaP, loP, hsM, hsP);
        const float dp = 0.25f * g * dh * (hsM + hsP);
        const float ah = hsM * unM + hsP * unP;
        const float au = hsM * uM * unM + hsP * uP * unP;
        const float av = hsM * vM * unM + hsP * vP * unP;
        const int kp = S::perm(KV + fn);
        sA[q][0][kp] = fs * ((huM * nx + hvM * ny) - 0.5f * ah - 0.5f * lam * dh);
        sA[q][1][kp] = fs * (huM * unM - 0.5f * au + dp * nx + 0.5f * lam * (hsP * uP - hsM * uM));
        sA[q][2][kp] = fs * (hvM * unM - 0.5f * av + dp * ny + 0.5f * lam * (hsP * vP - hsM * vM));
    }
    wave_lds_sync();

    // ---- lift part of the contraction (steps SV .. KS-1)
    if constexpr (!BF) {
        constexpr int F0 = SV / 4, F1 = (KS + 3) / 4;   // float4 chunks holding the lift steps
        float af[4 * (F1 - F0)];
#pragma unroll
        for (int s4 = F0; s4 < F1; ++s4) {
            const float4 v4 = *reinterpret_cast<const float4*>(&sA[ae][arow][ag * KSP + 4 * s4]);
            af[4 * (s4 - F0)] = v4.x; af[4 * (s4 - F0) + 1] = v4.y;
            af[4 * (s4 - F0) + 2] = v4.z; af[4 * (s4 - F0) + 3] = v4.w;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float ov[4 * (F1 - F0)];
#pragma unroll
            for (int s4 = F0; s4 < F1; ++s4) {
                if constexpr (OPL) {
                    const float4 o4 = *reinterpret_cast<const float4*>(&sOp[(t * 64 + lane) * OPS + 4 * s4]);
                    ov[4 * (s4 - F0)] = o4.x; ov[4 * (s4 - F0) + 1] = o4.y;
                    ov[4 * (s4 - F0) + 2] = o4.z; ov[4 * (s4 - F0) + 3] = o4.w;
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (4 * s4 + i >= SV && 4 * s4 + i < KS)
                            ov[4 * (s4 - F0) + i] = ldg(a.ops.Amfma, (unsigned)((t * KS + 4 * s4 + i) * 64 + lane));
                }
            }
#pragma unroll
            for (int s = SV; s < KS; ++s)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[s - 4 * F0], ov[s - 4 * F0], acc[t], 0, 0, 0);
        }
    } else {
        constexpr int P = BF + 1;
        const bf16x8* tab = reinterpret_cast<const bf16x8*>(a.ops.Abf);
#pragma unroll
        for (int s = SV; s < KS; ++s) {
            const float* xp = &sA[ae][arow][ag * 8 * KS + 8 * s];
            bf16x8 xs[P];
            bf16_split<P>(*reinterpret_cast<const float4*>(xp), *reinterpret_cast<const float4*>(xp + 4), xs);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                bf16x8 o[P];
#pragma unroll
                for (int u = 0; u < P; ++u) o[u] = ldg(tab, (unsigned)(3 * ((t * KS + s) * 64 + lane) + u));
                acc[t] = bf16_products<P>(xs, o, acc[t]);
            }
        }
    }
    if constexpr (!S::CMP) {   // the lane of node j holds rows 4 q .. 4 q + 2 of column j
        Rn[0] = acc[0][0];
        Rn[1] = acc[0][1];
        Rn[2] = acc[0][2];
    } else {
        // packed groups: D[row][node] to LDS node-major (lane c + 16 g of tile
        // t holds rows 4 g .. 4 g + 3 of node column 16 t + c), then each lane
        // reads rows 3 q .. 3 q + 2 of its node
        float (&sO)[NT * 16][S::OR] = lds[wave].O;
        wave_lds_sync();   // X^T reads done before the results overwrite them
#pragma unroll
        for (int t = 0; t < NT; ++t)
            *reinterpret_cast<float4*>(&sO[16 * t + (lane & 15)][4 * (lane >> 4)]) =
                make_float4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]);
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < 3; ++c) Rn[c] = sO[j][3 * q + c];
    }
    Rn[1] -= g * dlt * dBx;
    Rn[2] -= g * dlt * dBy;
    }   // right-hand side (fused kernel)

    // the reduction weights are loaded before the kernel's first store: every
    // store comes at the end, so no wait for a load covers a store
    double wr[S::KR];
    if constexpr (S::EARLY && !WL) {
#pragma unroll
        for (int s = 0; s < S::KR; ++s) wr[s] = ldg(a.ops.Wred, (unsigned)(s * 64 + lane));
    }

    // ---- Adams-Bashforth update and half-step traces (stored at the end)
    float qn[3] = {eta, hu, hv};
    float qlo = lo;
    float hh[3] = {0.f, 0.f, 0.f};
    if (node) {
        const float dt = dtmin * L.scale;
        const float q0[3] = {eta, hu, hv};
        const float q0lo[3] = {lo, 0.f, 0.f};
        eta_add(qn[0], qlo, dt * (L.ab[0] * Rn[0] + L.ab[1] * r1[0] + L.ab[2] * r2[0]));
#pragma unroll
        for (int c = 1; c < 3; ++c)
            qn[c] = q0[c] + dt * (L.ab[0] * Rn[c] + L.ab[1] * r1[c] + L.ab[2] * r2[c]);
        if constexpr (MULTI) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                hh[c] = q0[c] + (q0lo[c] + dt * (L.half[0] * Rn[c] + L.half[1] * r1[c] + L.half[2] * r2[c]));
        }
    }
    // ---- FP64 element reductions on the matrix cores
    const double h64 = node ? ((double)qn[0] - (double)Bn) + ((double)qlo - (double)bl) : 0.0;
    wave_lds_sync();   // X^T / result reads done before the node values overwrite them
    sVd[q][0][j] = h64;
    sVd[q][1][j] = node ? (double)qn[1] : 0.0;
    sVd[q][2][j] = node ? (double)qn[2] : 0.0;
    // a node of the element at or below eps (the positivity test needs only
    // that, not the minimum itself): one ballot bit per lane
    const unsigned long long lowm = __ballot(node && h64 <= (double)a.eps);
    const bool any_low = ((lowm >> gbase) & ((1ull << LPE) - 1ull)) != 0ull;
    wave_lds_sync();
    doublex4 red = {0.0, 0.0, 0.0, 0.0};
    {
        // column c: element c / 4, field c % 4 (16-lane groups) or element
        // c / 3, field c % 3 (packed groups); node rows past Np read nothing
        const int c = lane & 15;
        const int ec = S::CMP ? S::row_element(c) : c >> 2, fc = S::CMP ? S::row_field(c) : c & 3;
        const bool col = S::CMP ? c < 3 * EPW : (fc < 3 && ec < EPW);
        const int ecc = ec < EPW ? ec : 0, fcc = fc < 3 ? fc : 0;
#pragma unroll
        for (int s = 0; s < S::KR; ++s) {
            const int nd = 4 * s + ag;
            if constexpr (S::EARLY) {
                const double raw = sVd[ecc][fcc][nd < Np ? nd : 0];   // always a valid row
                const double bv = (col && nd < Np) ? raw : 0.0;
                const double w = WL ? reinterpret_cast<const double*>(sOp + WOFF)[s * 64 + lane] : wr[s];
                red = __builtin_amdgcn_mfma_f64_16x16x4f64(w, bv, red, 0, 0, 0);
            } else {
                const double bv = (col && nd < Np) ? sVd[ecc][fcc][nd < Np ? nd : 0] : 0.0;
                const double w = WL ? reinterpret_cast<const double*>(sOp + WOFF)[s * 64 + lane]
                                    : ldg(a.ops.Wred, (unsigned)(s * 64 + lane));
                red = __builtin_amdgcn_mfma_f64_16x16x4f64(w, bv, red, 0, 0, 0);
            }
        }
        // lane 16 g + c holds row g (0: mean, 1-3: midpoint deviation g-1) of column c
        if (col) sRed[ec][ag == 0 ? 1 + fc : 4 + 3 * fc + (ag - 1)] = red[0];
    }
    wave_lds_sync();
    // ---- positivity limiter decision (Algorithm 5.2), taken by all lanes of
    // the element
    const double hb = sRed[q][1];
    double scale = 1.0, hdry = 0.0;
    int code = 0;
    // a mean below h0 with every node above eps (negative vertex weights of
    // the nodal mean at N = 4, 6) also takes the dry branch
    if (a.pp_on && (any_low || hb < (double)a.h0)) {
        if (hb < (double)a.h0) {
            code = 2;
            hdry = a.dry_literal ? (double)a.h0 : fmax(hb, 0.0);
            scale = 0.0;
        } else {
            code = 1;
            const double d0 = sRed[q][4], d1 = sRed[q][5], d2 = sRed[q][6];
            const double Ssum = d0 + d1 + d2;
            const double vmin = hb + fmin(Ssum - 2.0 * d0, fmin(Ssum - 2.0 * d1, Ssum - 2.0 * d2));
            const double den = hb - vmin;
            scale = den > 0.0 ? fmin(1.0, (hb - (double)a.h0) / den) : 1.0;
        }
    }
    // ---- limited nodal values and the new state
    float out[3] = {qn[0], qn[1], qn[2]};
    float olo = qlo;
    if (node) {
        if (code == 2) {
            eta_split(hdry + ((double)Bn + (double)bl), out[0], olo);
            out[1] = 0.f;
            out[2] = 0.f;
        } else if (code == 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double val = sRed[q][1 + c];
#pragma unroll
                for (int ed = 0; ed < 3; ++ed) val += scale * sRed[q][4 + 3 * c + ed] * a.ops.phi[ed * Np + j];
                if (c == 0)
                    eta_split(val + ((double)Bn + (double)bl), out[0], olo);
                else
                    out[c] = (float)val;
            }
        }
        if (a.thin_cut > 0.f && (out[0] - Bn) + (olo - bl) < a.thin_cut) {   // thin film: no momentum
            out[1] = 0.f;
            out[2] = 0.f;
        }
    }
    // ---- stores: RHS ring, half-step traces, new state; then the hand-off
    // to the TVB kernel (a 32-byte record of post-limiter means and
    // positivity code for every element, P1 midpoint deviations (FP32) of
    // every element that is not dry) and the flags
    if (node) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if constexpr (!UPD) bR0.st(idx, c * FB, Rn[c]);
        if (MULTI && L.write_half && a.half != nullptr) {
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const int slot = a.ops.nodeface[2 * j + sl];
                if (slot < 0) continue;
                const unsigned hid = (unsigned)k * nF + slot;
#pragma unroll
                for (int c = 0; c < 3; ++c) bH.st(hid, c * HB, hh[c]);
            }
        }
        bQo.st(idx, 0, out[0]);
        bQo.st(idx, FB, out[1]);
        bQo.st(idx, 2u * FB, out[2]);
        bQo.st16(idx, 3u * FB, lo_encode(out[0], olo));
    }
    if (live && j < 4) {
        const double mv = code == 2 ? (j == 0 ? hdry : 0.0) : (j < 3 ? sRed[q][1 + j] : 0.0);
        stg(a.mrec, 4u * (unsigned)k + j, j == 3 ? (double)code : mv);
    }
    if (live && j < 9 && code != 2) {
        const int ed = j / 3, r = j % 3;   // field r at edge ed
        stg(a.devs, (unsigned)(3 * r + ed) * (unsigned)a.K + k, (float)(scale * sRed[q][4 + 3 * r + ed]));
    }
    if (live && j == 0) {
        a.flags[k] = (uint8_t)code;
        if (code == 2 && hb < 0.0) atomicAdd(&a.counters[0], 1ULL);
    }
}

// ---------------------------------------------------------------------------
// TVB limiter with the positivity modification of Eq. 5.3 (Section 5.3),
// FP64.  Three lanes per element (21 elements per wave, lane 63 idle): lane
// t owns edge t (its neighbour t, its stencil row, its characteristic
// decomposition); the balancing and the P1 output are shared by the three
// (lane t writes nodes t, t+3, ...).
// Means and positivity codes come from the step kernel's per-element records,
// which this kernel only reads, so the order in which elements are limited
// does not matter.
// ---------------------------------------------------------------------------
constexpr int kTvbElems = 84;   // elements per 256-lane block: four waves of 21

__global__ void __launch_bounds__(256) tvb_kernel(TvbArgs a) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int grp = lane / 3, t = lane - 3 * grp, gb = 3 * grp;   // element of the wave, edge, first lane
    // XCD-contiguous block order, as in the step kernel: the neighbour records
    // a mesh row away are then mostly in the same XCD's L2
    const int k = a.k_begin + xcd_remap(blockIdx.x, gridDim.x) * kTvbElems + wave * 21 + grp;
    if (grp == 21 || k >= a.k_end) return;   // the three lanes of an element leave together
    const unsigned K = (unsigned)a.K;
    const int ed = t;
    // first load round: everything indexed by k alone; the element's record holds its
    // post-positivity means and positivity code (the step kernel's snapshot)
    const double2* rec = reinterpret_cast<const double2*>(a.mrec);
    const double2 r01 = ldg(rec, 2u * k), r23 = ldg(rec, 2u * k + 1u);
    const int4 cn = ldg(reinterpret_cast<const int4*>(a.conn), (unsigned)k);
    const uint8_t pp = (uint8_t)r23.y;
    if (pp == 2) {
        if (t == 0) a.flags[k] = pp;
        return;
    }
    const double qb[3] = {r01.x, r01.y, r23.x};
    double dev[3];   // field c at edge ed
#pragma unroll
    for (int c = 0; c < 3; ++c) dev[c] = (double)ldg(a.devs, (3 * c + ed) * K + k);
    const float4 st = ldg(reinterpret_cast<const float4*>(a.stencil), 4u * k + ed);   // alpha_j, alpha_k, ex, ey
    const float2 mp = ldg(reinterpret_cast<const float2*>(a.stencil), 8u * k + 6u);
    const float M2 = mp.x;
    const int pairs = __float_as_int(mp.y);
    // second load round: neighbour t's record (means, and its code for the dry test)
    const int nbt = t == 0 ? cn.x : (t == 1 ? cn.y : cn.z);
    bool dry_t = false;
    double nm[3] = {0.0, 0.0, 0.0};
    if (nbt >= 0) {
        const double2 n01 = ldg(rec, 2u * (unsigned)nbt), n23 = ldg(rec, 2u * (unsigned)nbt + 1u);
        dry_t = n23.y == 2.0;
        nm[0] = n01.x;
        nm[1] = n01.y;
        nm[2] = n23.x;
    }
    if (((__ballot(dry_t) >> gb) & 0x7ull) != 0) {   // a face neighbour is dry: skipped
        if (t == 0) a.flags[k] = pp;
        return;
    }
    // mean difference across face t (a wall mirrors the momentum mean)
    double df[3] = {0.0, 0.0, 0.0};
    if (nbt < 0) {
        const float* gk = a.geo + 16LL * k;
        const double nx = gk[4 + ed], ny = gk[7 + ed];
        const double mn = qb[1] * nx + qb[2] * ny;
        df[0] = 0.0;
        df[1] = -2.0 * mn * nx;
        df[2] = -2.0 * mn * ny;
    } else if (nbt >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) df[c] = nm[c] - qb[c];
    }
    // edge ed: neighbour-mean increment from the faces of its stencil pair
    const int pj = (pairs >> (4 * ed)) & 3, pk = (pairs >> (4 * ed + 2)) & 3;
    double dbar[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        dbar[c] = (double)st.x * __shfl(df[c], gb + pj) + (double)st.y * __shfl(df[c], gb + pk);
    const double hb = qb[0];
    const double ub = qb[1] / hb, vb = qb[2] / hb;
    const double cc = sqrt(a.g * hb);
    const double ex = st.z, ey = st.w;
    double Lm[3][3];
    char_left(qb[0], qb[1], qb[2], a.g, ex, ey, Lm);
    const double Rm[3][3] = {{1.0, 0.0, 1.0},
                             {ub - cc * ex, -ey, ub + cc * ex},
                             {vb - cc * ey, ex, vb + cc * ey}};
    double mt[3];
    bool all_a1 = true;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double a1 = Lm[r][0] * dev[0] + Lm[r][1] * dev[1] + Lm[r][2] * dev[2];
        const double a2 = a.nu * (Lm[r][0] * dbar[0] + Lm[r][1] * dbar[1] + Lm[r][2] * dbar[2]);
        const bool small = fabs(a1) <= (double)M2;
        const bool same = (a1 > 0.0 && a2 > 0.0) || (a1 < 0.0 && a2 < 0.0);
        const double mm = same ? copysign(fmin(fabs(a1), fabs(a2)), a1) : 0.0;
        mt[r] = small ? a1 : mm;
        all_a1 = all_a1 && (small || a1 == 0.0 || (same && fabs(a1) <= fabs(a2)));
    }
    if (((__ballot(!all_a1) >> gb) & 0x7ull) == 0) {   // nothing limited: keep P^N
        if (t == 0) a.flags[k] = pp | (1 << 2);
        return;
    }
    double Dl[3];   // increments of edge ed in conserved variables
#pragma unroll
    for (int q = 0; q < 3; ++q) Dl[q] = Rm[q][0] * mt[0] + Rm[q][1] * mt[1] + Rm[q][2] * mt[2];
    double D[3][3];   // [field][edge], gathered by every lane of the element
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int e = 0; e < 3; ++e) D[q][e] = __shfl(Dl[q], gb + e);
    // balance each conserved component
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double pos = 0.0, neg = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            pos += fmax(D[q][e], 0.0);
            neg += fmax(-D[q][e], 0.0);
        }
        const double thp = pos > 0.0 ? fmin(1.0, neg / pos) : 1.0;
        const double thm = neg > 0.0 ? fmin(1.0, pos / neg) : 1.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) D[q][e] = thp * fmax(D[q][e], 0.0) - thm * fmax(-D[q][e], 0.0);
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
            for (int e = 0; e < 3; ++e) D[0][e] = dbh + th * (D[0][e] - dbh);
            code = 3;
        }
    }
    // P1 output: mean + sum_i D_i phi_i, nodes t, t+4, ... of the element
    const LevelArgs L = pick_level(a, level_of(a, k));
    float* Qo = a.Q[1 - L.parity];
    const int Np = a.Np;
    for (int j = t; j < Np; j += 3) {
        const double p0 = a.phi[j], p1 = a.phi[Np + j], p2 = a.phi[2 * Np + j];
        const long long id = (long long)k * Np + j;
        const double hval = qb[0] + D[0][0] * p0 + D[0][1] * p1 + D[0][2] * p2;
        float hi, lo;
        const float bh = a.B[id];
        eta_split(hval + ((double)bh + (double)lo_decode(bh, a.Blo[id])), hi, lo);
        Qo[id] = hi;
        reinterpret_cast<short*>(Qo + 3 * a.KNp)[id] = lo_encode(hi, lo);
        const bool thin = a.thin_cut > 0.0 && hval < a.thin_cut;   // thin film: no momentum
        Qo[a.KNp + id] = thin ? 0.f : (float)(qb[1] + D[1][0] * p0 + D[1][1] * p1 + D[1][2] * p2);
        Qo[2 * a.KNp + id] = thin ? 0.f : (float)(qb[2] + D[2][0] * p0 + D[2][1] * p1 + D[2][2] * p2);
    }
    if (t == 0) a.flags[k] = pp | (code << 2);
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
            const double h = ((double)Q[id] - (double)a.B[id]) +
                             ((double)lo_decode(Q[id], reinterpret_cast<const short*>(Q + 3 * a.KNp)[id]) -
                              (double)lo_decode(a.B[id], a.Blo[id]));
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
    if (engine != ENGINE_VALU && N <= 5) return mfma_default_waves(N) * (64 / mfma_lanes(N));
    return 256 / ((N + 1) * (N + 2) / 2);
}

// kernel launch; with a start/stop event pair the events take the kernel's
// own start and end timestamps from its dispatch (no queue or launch gaps)
template <typename K>
static void dispatch(K kernel, int blocks, int threads, hipStream_t s, const StepArgs& a, hipEvent_t e0,
                     hipEvent_t e1) {
    if (e0 != nullptr)
        hipExtLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), 0, s, a);
}

// matrix-core step kernel with W waves (EPW W elements) per block
template <int N, int W, bool UPD = false>
static int dispatch_mfma(int n, hipStream_t s, const StepArgs& a, hipEvent_t e0, hipEvent_t e1) {
    constexpr int EPW = 64 / mfma_lanes(N), EPB = EPW * W;
    const int bf = a.engine == ENGINE_MFMA_BF16X3 ? 1 : (a.engine == ENGINE_MFMA_BF16X6 ? 2 : 0);
    if (a.nlev > 1) {
        // cut [k_begin, k_end) at the level boundaries into whole blocks
        StepArgs m = a;
        int blocks = 0;
        m.parity_bits = 0;
        m.active_bits = 0;
        for (int l = 0; l < kMaxLevels; ++l) {
            int lo = a.k_begin, hi = a.k_begin;
            if (l < a.nlev) {
                lo = a.lev[l].begin > a.k_begin ? a.lev[l].begin : a.k_begin;
                hi = a.lev[l].end < a.k_end ? a.lev[l].end : a.k_end;
                if (hi < lo) hi = lo;
                m.parity_bits |= (unsigned)(a.lev[l].parity & 1) << l;
                m.active_bits |= (unsigned)(a.lev[l].active & 1) << l;
            }
            m.seg_begin[l] = lo;
            m.seg_end[l] = hi;
            m.seg_block[l] = blocks;
            blocks += (hi - lo + EPB - 1) / EPB;
        }
        m.seg_block[kMaxLevels] = blocks;
        const long long qd = reinterpret_cast<const char*>(a.Q[1]) - reinterpret_cast<const char*>(a.Q[0]);
        if (qd < 14 * a.KNp || qd + 14 * a.KNp >= (1ll << 32)) {
            std::snprintf(g_dev_err, sizeof(g_dev_err), "state buffers out of one 32-bit view");
            return -1;
        }
        m.q_pair_bytes = (unsigned)qd;
        if constexpr (UPD) dispatch(step_mfma_kernel<N, true, W, 0, true>, blocks, 64 * W, s, m, e0, e1);
        else if (bf == 1) dispatch(step_mfma_kernel<N, true, W, 1>, blocks, 64 * W, s, m, e0, e1);
        else if (bf == 2) dispatch(step_mfma_kernel<N, true, W, 2>, blocks, 64 * W, s, m, e0, e1);
        else dispatch(step_mfma_kernel<N, true, W, 0>, blocks, 64 * W, s, m, e0, e1);
    } else {
        const int blocks = (n + EPB - 1) / EPB;
        if constexpr (UPD) dispatch(step_mfma_kernel<N, false, W, 0, true>, blocks, 64 * W, s, a, e0, e1);
        else if (bf == 1) dispatch(step_mfma_kernel<N, false, W, 1>, blocks, 64 * W, s, a, e0, e1);
        else if (bf == 2) dispatch(step_mfma_kernel<N, false, W, 2>, blocks, 64 * W, s, a, e0, e1);
        else dispatch(step_mfma_kernel<N, false, W, 0>, blocks, 64 * W, s, a, e0, e1);
    }
    return 0;
}

template <int N>
static int launch_step_n(const StepArgs& a, hipStream_t s, int epb, hipEvent_t e0, hipEvent_t e1) {
    const int n = a.k_end - a.k_begin;
    if (n <= 0) return 0;
    if constexpr (N <= 5) {
        if (a.engine == ENGINE_MFMA_F32 && a.mode == MODE_UPDATE_ONLY) {
            // the over-integrated form's update on the matrix-core kernel
            if (dispatch_mfma<N, 4, true>(n, s, a, e0, e1)) return -1;
            return check_launch("update mfma kernel");
        }
        if (a.engine != ENGINE_VALU && a.mode == MODE_FUSED) {
            constexpr int EPW = 64 / mfma_lanes(N);
            const int w = epb % EPW == 0 ? epb / EPW : 0;
            switch (w) {
                case 1: if (dispatch_mfma<N, 1>(n, s, a, e0, e1)) return -1; break;
                case 2: if (dispatch_mfma<N, 2>(n, s, a, e0, e1)) return -1; break;
                case 4: if (dispatch_mfma<N, 4>(n, s, a, e0, e1)) return -1; break;
                case 8: if (dispatch_mfma<N, 8>(n, s, a, e0, e1)) return -1; break;
                default:
                    std::snprintf(g_dev_err, sizeof(g_dev_err),
                                  "elements per block %d is not 1, 2, 4 or 8 waves of %d elements", epb, EPW);
                    return -1;
            }
            return check_launch("step mfma kernel");
        }
    }
    const int E = Shape<N>::E;
    dispatch(step_kernel<N>, (n + E - 1) / E, 256, s, a, e0, e1);
    return check_launch("step kernel");
}

int launch_step(const StepArgs& a, void* stream, int elems_per_block, void* ev_start, void* ev_stop) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = static_cast<hipEvent_t>(ev_start), e1 = static_cast<hipEvent_t>(ev_stop);
    const int epb = elems_per_block > 0 ? elems_per_block : step_elems_per_block(a.N, a.engine);
    switch (a.N) {
        case 1: return launch_step_n<1>(a, s, epb, e0, e1);
        case 2: return launch_step_n<2>(a, s, epb, e0, e1);
        case 3: return launch_step_n<3>(a, s, epb, e0, e1);
        case 4: return launch_step_n<4>(a, s, epb, e0, e1);
        case 5: return launch_step_n<5>(a, s, epb, e0, e1);
        case 6: return launch_step_n<6>(a, s, epb, e0, e1);
        default:
            std::snprintf(g_dev_err, sizeof(g_dev_err), "unsupported N=%d", a.N);
            return -1;
    }
}

template <int N>
static int launch_rhs_overint_n(const StepArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int n = a.k_end - a.k_begin;
    if (n <= 0) return 0;
    if (a.engine == ENGINE_MFMA_F32) {
        dispatch(rhs_overint_mfma_kernel<N>, (n + 3) / 4, 64, s, a, e0, e1);
        return check_launch("over-integrated rhs kernel (matrix cores)");
    }
    constexpr int E = OShape<N>::E;
    dispatch(rhs_overint_kernel<N>, (n + E - 1) / E, 256, s, a, e0, e1);
    return check_launch("over-integrated rhs kernel");
}

int launch_rhs_overint(const StepArgs& a, void* stream, void* ev_start, void* ev_stop) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = static_cast<hipEvent_t>(ev_start), e1 = static_cast<hipEvent_t>(ev_stop);
    switch (a.N) {
        case 1: return launch_rhs_overint_n<1>(a, s, e0, e1);
        case 2: return launch_rhs_overint_n<2>(a, s, e0, e1);
        case 3: return launch_rhs_overint_n<3>(a, s, e0, e1);
        case 4: return launch_rhs_overint_n<4>(a, s, e0, e1);
        case 5: return launch_rhs_overint_n<5>(a, s, e0, e1);
        default:
            std::snprintf(g_dev_err, sizeof(g_dev_err), "over-integration supports N <= 5, got N=%d", a.N);
            return -1;
    }
}

int launch_tvb(const TvbArgs& a, void* stream, void* ev_start, void* ev_stop) {
    const int n = a.k_end - a.k_begin;
    if (n <= 0) return 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ev_start)
        hipExtLaunchKernelGGL(tvb_kernel, dim3((n + kTvbElems - 1) / kTvbElems), dim3(256), 0, s,
                              static_cast<hipEvent_t>(ev_start), static_cast<hipEvent_t>(ev_stop), 0, a);
    else
        hipLaunchKernelGGL(tvb_kernel, dim3((n + kTvbElems - 1) / kTvbElems), dim3(256), 0, s, a);
    return check_launch("tvb kernel");
}

// ---------------------------------------------------------------------------
// Allocation-free diagnostics: the per-block partial sums of the reduction go
// to a fixed device array instead of the bound workspace.  Its size does not
// depend on the input (the partial kernel always runs kDiagBlocks blocks of
// 16 values); every call on a device shares that device's copy.
// ---------------------------------------------------------------------------
constexpr int kScratchDoubles = kDiagBlocks * 16;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch`, looked up once per device
// with the device current (the host-side name of the array is not a device
// address)
static int scratch_on_current_device(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        std::snprintf(g_dev_err, sizeof(g_dev_err), "hipGetDevice: %s", hipGetErrorString(e));
        return -1;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        std::snprintf(g_dev_err, sizeof(g_dev_err), "device %d beyond the scratch table (%d)", dev, kMaxDevices);
        return -1;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            std::snprintf(g_dev_err, sizeof(g_dev_err), "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return -1;
        }
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

int diag_scratch_doubles() { return kScratchDoubles; }

int launch_diag_static(const DiagArgs& args, double* out, void* stream) {
    static_assert(kDiagBlocks * 16 <= kScratchDoubles, "diagnostics partials exceed the scratch array");
    double* part = nullptr;
    if (scratch_on_current_device(&part)) return -1;
    DiagArgs a = args;
    a.partial = part;   // every slot is written by the partial kernel: nothing to clear
    a.out = out;
    return launch_diag(a, stream);
}

int launch_diag(const DiagArgs& a, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(diag_partial_kernel, dim3(kDiagBlocks), dim3(256), 0, s, a);
    if (check_launch("diag kernel")) return -1;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, s, a);
    return check_launch("diag final kernel");
}

}  // namespace dgswe
