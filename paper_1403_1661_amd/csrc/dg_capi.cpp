// C ABI of the DG shallow-water solver: setup, device binding, time stepping,
// read-back.  Host work is FP64; the device path is the HIP step/TVB kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/dgswe.h"
#include "dg_launch.hpp"
#include "host_mesh.hpp"
#include "host_refelem.hpp"

using namespace dgswe;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHECK(call)                                                               \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) return fail(DG_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t Q[2], R[3], half, mrec, devs, flags, counters;   // dynamic (checkpointed)
    size_t dyn_begin, dyn_end;
    size_t B, Blo, dB, geo, gm, idt, conn, stencil;
    size_t Dr, Ds, LIFT, Amfma, AmfmaL, Abf, Wred, fmask, nodeface, wh, pmid, phi, wfull;
    size_t oIc, oPr, oPs, oP, oLg, oI1, oT1, oT3;
    size_t diag_partial, diag_out;
    size_t total;
};

struct Inst {
    HostMesh mesh;
    int offset = 0;          // first global (unsorted) element index
    bool has_B = false, has_state = false;
    double dt_min = 0.0, a_max = 0.0;
    // Vertical datum of the instance: the device stores eta - datum and
    // B - datum in FP32.  Every formula of the scheme depends on depths and
    // surface-level differences only, so the shift changes nothing but the
    // FP32 rounding of the stored surface level, which shrinks with |eta - datum|.
    float datum = 0.f;
    // datum, time step and wave speed of the state staged by dg_set_state
    // (dg_prepare starts from them; a restored checkpoint brings its own)
    float staged_datum = 0.f;
    double staged_dt_min = 0.0, staged_a_max = 0.0;
    std::vector<double> speed0;   // per-element wave speed of the staged state (regrouping)
    // simulated time: t_base + (ticks - tick_base) dt_min (dt_min changes at regroups)
    double t_base = 0.0;
    int64_t tick_base = 0;
};

}  // namespace

struct dg_solver {
    dg_params p{};
    RefElement re;
    OverInt oi;               // cubature / Gauss operators (built for every solver)
    std::vector<Inst> inst;
    int K = 0, Np = 0, Nfp = 0, nF = 0, L = 1;
    std::vector<int> perm, inv, inst_of;     // sorted -> global, global -> sorted
    std::vector<int> lev_begin, lev_end;     // per level (0-based) in sorted order
    Layout lay{};
    char* ws = nullptr;
    bool bound = false, prepared = false;
    int device = 0;
    // host staging (sorted order, FP32)
    std::vector<float> gmh, idth;   // staging of the compact metric terms and per-instance time steps
    std::vector<float> geo, stencil, Bh, Qh, dBh;   // dBh: [2][K*Np] bed gradient; Qh: [3][K*Np] (eta hi, hu, hv); Bh, eta relative to the datum
    std::vector<int16_t> Ql;                         // [K*Np] eta lo, 16-bit (see lo_encode)
    std::vector<int16_t> Bl;                         // [K*Np] bed (relative to the datum) lo, 16-bit
    std::vector<double> B64;                   // bed elevation, FP64, sorted order
    std::vector<int> conn;
    // time stepping state
    int parity[kMaxLevels] = {0}, head[kMaxLevels] = {0}, nhist[kMaxLevels] = {0};
    long long steps = 0;     // coarse steps since dg_prepare
    int64_t ticks = 0;       // finest-level ticks since dg_prepare (simulated time = ticks * dt_min)
    int64_t regroups = 0;    // regroupings since dg_prepare
    // execution
    hipStream_t exec = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_key[3 * kMaxLevels] = {0};
    bool have_graph = false;
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events, prof_tvb_events;
    size_t prof_used = 0, prof_tvb_used = 0;
    double prof_avg_us = 0.0;
    long long prof_launches = 0, prof_elems = 0;
};

// ---------------------------------------------------------------------------
static const float kAB[3][3] = {{1.f, 0.f, 0.f}, {1.5f, -0.5f, 0.f},
                                {23.f / 12.f, -16.f / 12.f, 5.f / 12.f}};
static const float kHalf[3][3] = {{0.5f, 0.f, 0.f}, {5.f / 8.f, -1.f / 8.f, 0.f},
                                  {17.f / 24.f, -7.f / 24.f, 2.f / 24.f}};

// bfloat16 of an FP32 value, round to nearest even (finite inputs), and back
static uint16_t bf16_round(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
static float bf16_value(uint16_t b) {
    const uint32_t u = uint32_t(b) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// The level's low word travels as a 16-bit integer in units of 2^-15 ulp(hi)
// (ulp(hi) = 2^(e-24) with hi = m 2^e, 1/2 <= |m| < 1); the kernels use the
// same encoding.
static int16_t lo_encode(float hi, float lo) {
    int e = 0;
    std::frexp(hi, &e);
    const float s = std::nearbyint(std::ldexp(lo, 39 - e));
    return int16_t(std::fmin(std::fmax(s, -32767.f), 32767.f));
}
static float lo_decode(float hi, int16_t s) {
    int e = 0;
    std::frexp(hi, &e);
    return std::ldexp(float(s), e - 39);
}

// The instance's bed relative to a datum as an FP32 pair hi + lo (lo in the
// 16-bit encoding), so that depths keep the caller's FP64 bed to 2^-16 ulp.
static void shift_bed(dg_solver* h, const Inst& I, double datum) {
    const int Np = h->Np;
    for (int k = 0; k < I.mesh.K; ++k) {
        const size_t s0 = size_t(h->inv[I.offset + k]) * Np;
        for (int j = 0; j < Np; ++j) {
            const double b = h->B64[s0 + j] - datum;
            const float bh = float(b);
            h->Bh[s0 + j] = bh;
            h->Bl[s0 + j] = lo_encode(bh, float(b - double(bh)));
        }
    }
}

// Geometry records on the device: the 64-byte rows (with each instance's
// FP32 time step in slot 14), the compact rx, ry, sx, sy array that the
// matrix-core step kernel reads instead (16 bytes per element), and the
// per-instance time steps it finds through the connectivity record.  async:
// on stream s (the host vectors live in the handle until the next call).
static int upload_geometry(dg_solver* h, hipStream_t s, bool async) {
    const size_t K = size_t(h->K);
    for (size_t sidx = 0; sidx < K; ++sidx) h->geo[16 * sidx + 14] = float(h->inst[h->inst_of[sidx]].dt_min);
    h->gmh.resize(4 * K);
    for (size_t sidx = 0; sidx < K; ++sidx)
        for (int c = 0; c < 4; ++c) h->gmh[4 * sidx + c] = h->geo[16 * sidx + c];
    h->idth.resize(h->inst.size());
    for (size_t i = 0; i < h->inst.size(); ++i) h->idth[i] = float(h->inst[i].dt_min);
    const Layout& l = h->lay;
    const std::pair<size_t, const std::vector<float>*> up[3] = {{l.geo, &h->geo}, {l.gm, &h->gmh}, {l.idt, &h->idth}};
    for (const auto& u : up) {
        if (async)
            HIPCHECK(hipMemcpyAsync(h->ws + u.first, u.second->data(), u.second->size() * 4, hipMemcpyHostToDevice, s));
        else
            HIPCHECK(hipMemcpy(h->ws + u.first, u.second->data(), u.second->size() * 4, hipMemcpyHostToDevice));
    }
    return DG_OK;
}

static int engine_of(int precision) {
    switch (precision) {
        case DG_FUSED_MFMA32: return ENGINE_MFMA_F32;
        case DG_FUSED_BF16X3: return ENGINE_MFMA_BF16X3;
        case DG_FUSED_BF16X6: return ENGINE_MFMA_BF16X6;
        default: return ENGINE_VALU;
    }
}

// Morton (Z-order) key of every element's centroid, 16 bits per axis over
// the instance's bounding box: elements close on the mesh get close keys.
static std::vector<uint32_t> morton_keys(const HostMesh& m) {
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    for (int v = 0; v < m.Nv; ++v) {
        x0 = std::fmin(x0, m.vx[v]);
        x1 = std::fmax(x1, m.vx[v]);
        y0 = std::fmin(y0, m.vy[v]);
        y1 = std::fmax(y1, m.vy[v]);
    }
    const double sx = 65535.0 / std::fmax(x1 - x0, 1e-300), sy = 65535.0 / std::fmax(y1 - y0, 1e-300);
    auto spread = [](uint32_t v) {
        v &= 0xFFFFu;
        v = (v | (v << 8)) & 0x00FF00FFu;
        v = (v | (v << 4)) & 0x0F0F0F0Fu;
        v = (v | (v << 2)) & 0x33333333u;
        v = (v | (v << 1)) & 0x55555555u;
        return v;
    };
    std::vector<uint32_t> key(m.K);
    for (int k = 0; k < m.K; ++k) {
        const int* t = &m.etov[3 * size_t(k)];
        const double cx = (m.vx[t[0]] + m.vx[t[1]] + m.vx[t[2]]) / 3.0;
        const double cy = (m.vy[t[0]] + m.vy[t[1]] + m.vy[t[2]]) / 3.0;
        const uint32_t qx = uint32_t(std::lround((cx - x0) * sx)), qy = uint32_t(std::lround((cy - y0) * sy));
        key[k] = spread(qx) | (spread(qy) << 1);
    }
    return key;
}

// Element order of the device arrays: by level, then instance, then the
// Morton key of the centroid (ties by local index), so that every level is
// one contiguous range and face neighbours are mostly close in memory (their
// face values are then still in the L2 cache when a neighbour gathers them).
static void sort_elements(dg_solver* h) {
    h->perm.resize(h->K);
    h->inv.resize(h->K);
    h->inst_of.resize(h->K);
    std::vector<std::vector<int>> order(h->inst.size());
    for (size_t i = 0; i < h->inst.size(); ++i) {
        const HostMesh& m = h->inst[i].mesh;
        const std::vector<uint32_t> key = morton_keys(m);
        order[i].resize(m.K);
        for (int k = 0; k < m.K; ++k) order[i][k] = k;
        std::stable_sort(order[i].begin(), order[i].end(), [&](int a, int b) { return key[a] < key[b]; });
    }
    int pos = 0;
    h->lev_begin.assign(h->L, 0);
    h->lev_end.assign(h->L, 0);
    for (int l = 1; l <= h->L; ++l) {
        h->lev_begin[l - 1] = pos;
        for (size_t i = 0; i < h->inst.size(); ++i) {
            const Inst& I = h->inst[i];
            for (int k : order[i]) {
                if (I.mesh.level[k] != l) continue;
                const int gidx = I.offset + k;
                h->perm[pos] = gidx;
                h->inv[gidx] = pos;
                h->inst_of[pos] = int(i);
                ++pos;
            }
        }
        h->lev_end[l - 1] = pos;
    }
}

// Wave speed of every element for grouping: max |(u,v)| + sqrt(g h) over
// its nodes and its face neighbours' nodes (desingularised velocity),
// floored at 1e-12.  State in the instance's element order, [K][Np].
static void element_speeds(const HostMesh& m, int Np, const double* hh, const double* hu, const double* hv,
                           double g, double hvel, std::vector<double>& a) {
    std::vector<double> node(m.K, 0.0);
    for (int k = 0; k < m.K; ++k) {
        double mx = 0.0;
        for (int j = 0; j < Np; ++j) {
            const size_t t = size_t(k) * Np + j;
            const double d = hh[t];
            const double f = 2.0 * d / (d * d + std::fmax(d * d, hvel * hvel));
            mx = std::fmax(mx, std::hypot(hu[t] * f, hv[t] * f) + std::sqrt(g * std::fmax(d, 0.0)));
        }
        node[k] = mx;
    }
    a.assign(m.K, 0.0);
    for (int k = 0; k < m.K; ++k) {
        double mx = node[k];
        for (int f = 0; f < 3; ++f) mx = std::fmax(mx, node[m.etoe[3 * k + f]]);
        a[k] = std::fmax(mx, 1e-12);
    }
}

// Levels from each element's own step dt_k = cfl r_k / ((N+1)^2 a_k) (Eq. 4.1
// with a per element): 2^(l-1) dt_min <= dt_k < 2^l dt_min with a tie
// tolerance of 1e-12, capped at L, then the 2:1 rule across faces.  Writes
// m.level and returns dt_min.
static double speed_levels(HostMesh& m, int N, double cfl, const std::vector<double>& a, int L) {
    std::vector<double> dt(m.K);
    double dtmin = 1e300;
    for (int k = 0; k < m.K; ++k) {
        dt[k] = cfl * m.inradius[k] / (double((N + 1) * (N + 1)) * a[k]);
        dtmin = std::fmin(dtmin, dt[k]);
    }
    m.level.assign(m.K, 1);
    for (int k = 0; k < m.K; ++k) {
        int j = 0;
        while (j + 1 < L && std::ldexp(dtmin, j + 1) <= dt[k] * (1.0 + 1e-12)) ++j;
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
    return dtmin;
}

// After the instances' levels changed: new element order, and every host
// staging array moved to it.  Returns, for every old sorted position, its
// new one (for the caller's own arrays).
template <typename T>
static void move_rows(std::vector<T>& v, size_t row, size_t fields, const std::vector<int>& to) {
    if (v.empty()) return;
    const size_t K = to.size();
    std::vector<T> out(v.size());
    for (size_t c = 0; c < fields; ++c)
        for (size_t o = 0; o < K; ++o)
            std::copy(v.begin() + (c * K + o) * row, v.begin() + (c * K + o + 1) * row,
                      out.begin() + (c * K + size_t(to[o])) * row);
    v.swap(out);
}

static std::vector<int> resort(dg_solver* h) {
    const std::vector<int> old_perm = h->perm;
    sort_elements(h);
    const int K = h->K;
    std::vector<int> to(K);
    for (int o = 0; o < K; ++o) to[o] = h->inv[old_perm[o]];
    const size_t Np = size_t(h->Np);
    move_rows(h->geo, 16, 1, to);
    move_rows(h->stencil, 16, 1, to);
    move_rows(h->conn, 4, 1, to);
    for (int sidx = 0; sidx < K; ++sidx)
        for (int f = 0; f < 3; ++f) {
            int& c = h->conn[4 * size_t(sidx) + f];
            if (c >= 0) c = to[c];
        }
    move_rows(h->B64, Np, 1, to);
    move_rows(h->Bh, Np, 1, to);
    move_rows(h->Bl, Np, 1, to);
    move_rows(h->dBh, Np, 2, to);
    move_rows(h->Qh, Np, 3, to);
    move_rows(h->Ql, Np, 1, to);
    return to;
}

static void compute_layout(dg_solver* h) {
    Layout& l = h->lay;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t KNp = size_t(h->K) * h->Np, KnF = size_t(h->K) * h->nF;
    l.dyn_begin = o;
    // state: eta hi, hu, hv (FP32) then the level's low word (16-bit)
    l.Q[0] = take(14 * KNp);
    l.Q[1] = take(14 * KNp);
    for (int s = 0; s < 3; ++s) l.R[s] = take(3 * KNp * 4);
    l.half = take(h->L > 1 ? 3 * KnF * 4 : 0);
    l.mrec = take(4 * size_t(h->K) * 8);
    l.devs = take(9 * size_t(h->K) * 4);
    l.flags = take(size_t(h->K));
    l.counters = take(64);
    l.dyn_end = o;
    l.B = take(KNp * 4);
    l.Blo = take(KNp * 2);
    l.dB = take(2 * KNp * 4);
    l.geo = take(size_t(h->K) * 64);
    l.gm = take(size_t(h->K) * 16);
    l.idt = take(h->inst.size() * 4);
    l.conn = take(size_t(h->K) * 16);
    l.stencil = take(size_t(h->K) * 64);
    const int Np = h->Np, nF = h->nF;
    l.Dr = take(size_t(Np) * Np * 4);
    l.Ds = take(size_t(Np) * Np * 4);
    l.LIFT = take(size_t(Np) * nF * 4);
    l.Amfma = take(size_t(64) * 256 * 4 * 2);
    l.AmfmaL = take(size_t(2) * 64 * 24 * 4);
    l.Abf = take(size_t(8) * 64 * 48);
    l.Wred = take(size_t(8) * 64 * 8);
    l.fmask = take(size_t(nF) * 4);
    l.nodeface = take(size_t(Np) * 2 * 4);
    l.wh = take(size_t(Np) * 8);
    l.pmid = take(3 * size_t(Np) * 8);
    l.phi = take(3 * size_t(Np) * 8);
    l.wfull = take(size_t(Np) * 8);
    {
        const size_t nc = size_t(h->oi.Ncub), ng = size_t(h->oi.NG);
        l.oIc = take(nc * Np * 4);
        l.oPr = take(nc * Np * 4);
        l.oPs = take(nc * Np * 4);
        l.oP = take(nc * Np * 4);
        l.oLg = take(size_t(Np) * 3 * ng * 4);
        l.oI1 = take(ng * size_t(h->Nfp) * 4);
        const int N = h->p.N;
        if (N <= 5) {
            l.oT1 = take(size_t(overint_mfma_t1(N)) * overint_mfma_s1(N) * 64 * 4);
            l.oT3 = take(size_t(overint_mfma_tn(N)) * overint_mfma_t3_steps(N) * 64 * 4);
        } else {
            l.oT1 = l.oT3 = take(0);
        }
    }
    l.diag_partial = take(256 * 16 * 8);
    l.diag_out = take(16 * 8);
    l.total = o;
}

// ---------------------------------------------------------------------------
extern "C" {

const char* dg_last_error(void) { return g_err.c_str(); }

int32_t dg_default_params(int32_t N, dg_params* p) {
    if (!p) return fail(DG_EINVAL, "null params");
    std::memset(p, 0, sizeof(*p));
    p->N = N;
    p->g = 9.81;
    p->cfl = 0.5;
    p->h0 = 1e-5;
    p->eps = 1e-5;
    p->hvel = 1e-3;
    p->tvb_M = 10.0;
    p->tvb_nu = 1.5;
    p->limiter_mask = DG_LIMIT_PP | DG_LIMIT_TVB;
    p->max_levels = 1;
    p->precision = DG_FUSED_FP32;
    p->dry_literal = 0;
    p->use_graph = 1;
    p->elems_per_block = 0;
    return DG_OK;
}

int32_t dg_create(const dg_mesh_desc* meshes, int32_t n_inst, const dg_params* p, dg_solver** out) {
    if (!meshes || !p || !out || n_inst < 1) return fail(DG_EINVAL, "null argument or n_inst < 1");
    if (n_inst > kMaxInstances) return fail(DG_EINVAL, "n_inst must be at most 2^23");
    *out = nullptr;
    if (p->N < 1 || p->N > 6) return fail(DG_EINVAL, "N must be in 1..6");
    if (!(p->thin_cut >= 0)) return fail(DG_EINVAL, "thin_cut must be >= 0");
    if (!(p->g > 0) || !(p->cfl > 0) || !(p->h0 > 0) || !(p->eps >= 0) || !(p->hvel > 0) ||
        !(p->tvb_M >= 0) ||
        !(p->tvb_nu >= 1.0))
        return fail(DG_EINVAL, "bad physical or limiter parameter");
    if (p->max_levels < 1 || p->max_levels > kMaxLevels)
        return fail(DG_EINVAL, "max_levels must be in 1..6");
    if (p->precision < DG_PLAIN_FP32 || p->precision > DG_FUSED_BF16X6)
        return fail(DG_EINVAL, "unknown precision/path");
    if (p->precision >= DG_FUSED_MFMA32 && p->N > 5)
        return fail(DG_EINVAL, "the MFMA contraction supports N <= 5");
    if (p->overint != 0 && p->overint != 1) return fail(DG_EINVAL, "overint must be 0 or 1");
    if (p->regroup_every < 0 || (p->regroup_every > 0 && p->regroup_every < 3))
        return fail(DG_EINVAL, "regroup_every must be 0 or at least 3 coarse steps");
    if (p->regroup_every > 0 && p->max_levels < 2)
        return fail(DG_EINVAL, "regrouping needs max_levels >= 2");
    if (p->overint && (p->N > 5 || p->precision > DG_FUSED_MFMA32))
        return fail(DG_EINVAL, "over-integration runs for N <= 5 on DG_PLAIN_FP32, DG_FUSED_FP32 or DG_FUSED_MFMA32");
    if (p->elems_per_block != 0) {
        const bool mfma = p->precision >= DG_FUSED_MFMA32;
        const int valu_e = 256 / ((p->N + 1) * (p->N + 2) / 2);
        const int epw = 64 / mfma_lanes(p->N);
        const int e = p->elems_per_block;
        const bool ok = mfma ? (e == epw || e == 2 * epw || e == 4 * epw || e == 8 * epw) : e == valu_e;
        if (!ok)
            return fail(DG_EINVAL, mfma ? "elems_per_block must be 0 or 1, 2, 4, 8 waves of 64/lanes elements on "
                                          "the MFMA paths (N = 1, 2, 4: 4, 8, 16, 32; N = 3: 5, 10, 20, 40; "
                                          "N = 5: 3, 6, 12, 24)"
                                        : "elems_per_block must be 0 or floor(256 / Np) on the VALU paths");
    }
    std::unique_ptr<dg_solver> h;
    try {
        h.reset(new dg_solver());
        h->p = *p;
        h->re = build_reference(p->N);
        h->oi = build_overint(h->re);
    } catch (const std::bad_alloc&) {
        return fail(DG_ENOMEM, "out of host memory");
    } catch (const std::exception& ex) {
        return fail(DG_EINVAL, ex.what());
    }
    h->Np = h->re.Np;
    h->Nfp = h->re.Nfp;
    h->nF = 3 * h->Nfp;
    h->L = p->max_levels;
    h->inst.resize(n_inst);
    long long total = 0;
    for (int i = 0; i < n_inst; ++i) {
        const dg_mesh_desc& m = meshes[i];
        if (!m.vx || !m.vy || !m.etov || m.n_elements < 1 || m.n_vertices < 3)
            return fail(DG_EINVAL, "instance " + std::to_string(i) + ": null or empty mesh");
        std::string err;
        try {
            err = build_host_mesh(m.n_vertices, m.vx, m.vy, m.n_elements, m.etov, m.bc, h->inst[i].mesh);
        } catch (const std::bad_alloc&) {
            return fail(DG_ENOMEM, "out of host memory");
        }
        if (!err.empty()) return fail(DG_EMESH, "instance " + std::to_string(i) + ": " + err);
        assign_levels(h->inst[i].mesh, h->L);
        build_tvb_stencil(h->inst[i].mesh);
        h->inst[i].offset = int(total);
        total += m.n_elements;
    }
    if (total > (1LL << 30)) return fail(DG_EINVAL, "too many elements");
    h->K = int(total);
    sort_elements(h.get());
    // static per-element device records
    const int K = h->K;
    h->geo.assign(size_t(K) * 16, 0.f);
    h->conn.assign(size_t(K) * 4, 0);
    h->stencil.assign(size_t(K) * 16, 0.f);
    for (int s = 0; s < K; ++s) {
        const int gidx = h->perm[s], i = h->inst_of[s];
        const HostMesh& m = h->inst[i].mesh;
        const int k = gidx - h->inst[i].offset;
        float* gk = &h->geo[16 * size_t(s)];
        gk[0] = float(m.rx[k]); gk[1] = float(m.ry[k]); gk[2] = float(m.sx[k]); gk[3] = float(m.sy[k]);
        for (int f = 0; f < 3; ++f) {
            gk[4 + f] = float(m.nx[3 * k + f]);
            gk[7 + f] = float(m.ny[3 * k + f]);
            gk[10 + f] = float(m.fscale[3 * k + f]);
        }
        gk[13] = float(m.J[k]);
        gk[14] = 0.f;
        int iid = i;
        std::memcpy(&gk[15], &iid, 4);
        int* cn = &h->conn[4 * size_t(s)];
        int packed = 0;
        for (int f = 0; f < 3; ++f) {
            if (m.wall[3 * k + f]) {
                cn[f] = -1;
            } else {
                cn[f] = h->inv[h->inst[i].offset + m.etoe[3 * k + f]];
                packed |= (m.etof[3 * k + f] & 3) << (2 * f);
            }
        }
        cn[3] = packed | (i << kConnInstShift);
        float* st = &h->stencil[16 * size_t(s)];
        int pairs = 0;
        for (int e = 0; e < 3; ++e) {
            st[4 * e] = float(m.alpha[6 * k + 2 * e]);
            st[4 * e + 1] = float(m.alpha[6 * k + 2 * e + 1]);
            st[4 * e + 2] = float(m.dir[6 * k + 2 * e]);
            st[4 * e + 3] = float(m.dir[6 * k + 2 * e + 1]);
            pairs |= (m.pair[6 * k + 2 * e] & 3) << (4 * e);
            pairs |= (m.pair[6 * k + 2 * e + 1] & 3) << (4 * e + 2);
        }
        st[12] = float(p->tvb_M * m.dk[k] * m.dk[k]);
        std::memcpy(&st[13], &pairs, 4);
    }
    // the kernels address nodal arrays with 32-bit byte offsets (4 fields)
    if (16.0 * double(h->K) * double(h->Np) >= 4294967296.0)
        return fail(DG_EINVAL, "too many nodes: 16 K Np must stay below 2^32 bytes");
    // multi-rate: one view spans both state buffers, another the half-step traces
    if (h->L > 1 && (32.0 * double(h->K) * double(h->Np) + 512.0 >= 4294967296.0 ||
                     12.0 * double(h->K) * double(h->nF) >= 4294967296.0))
        return fail(DG_EINVAL, "too many nodes for multi-rate: 32 K Np and 12 K 3(N+1) must stay below 2^32 bytes");
    compute_layout(h.get());
    *out = h.release();
    return DG_OK;
}

void dg_destroy(dg_solver* h) {
    if (!h) return;
    // graph replays may still be running on the solver's own stream and
    // writing into the caller's buffer: finish them before the caller can
    // free or reuse that memory (and before their executable goes away)
    if (h->exec) {
        int cur = -1;
        const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != h->device;
        if (switch_dev) (void)hipSetDevice(h->device);
        (void)hipStreamSynchronize(h->exec);
        if (switch_dev) (void)hipSetDevice(cur);
    }
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    for (auto* v : {&h->prof_events, &h->prof_tvb_events})
        for (auto& ev : *v) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    if (h->exec) (void)hipStreamDestroy(h->exec);
    delete h;
}

int32_t dg_query_sizes(const dg_solver* h, int64_t* total_elements, int32_t* Np, int32_t* Nfp,
                       int64_t* workspace_bytes) {
    if (!h) return fail(DG_EINVAL, "null handle");
    if (total_elements) *total_elements = h->K;
    if (Np) *Np = h->Np;
    if (Nfp) *Nfp = h->Nfp;
    if (workspace_bytes) *workspace_bytes = int64_t(h->lay.total);
    return DG_OK;
}

int32_t dg_instance_elements(const dg_solver* h, int32_t inst, int32_t* K) {
    if (!h || !K || inst < 0 || inst >= int(h->inst.size())) return fail(DG_EINVAL, "bad argument");
    *K = h->inst[inst].mesh.K;
    return DG_OK;
}

int32_t dg_node_coords(const dg_solver* h, int32_t inst, double* x, double* y) {
    if (!h || !x || !y || inst < 0 || inst >= int(h->inst.size())) return fail(DG_EINVAL, "bad argument");
    node_coords(h->inst[inst].mesh, h->re, x, y);
    return DG_OK;
}

int32_t dg_reference_nodes(const dg_solver* h, double* r, double* s) {
    if (!h || !r || !s) return fail(DG_EINVAL, "bad argument");
    std::copy(h->re.r.begin(), h->re.r.end(), r);
    std::copy(h->re.s.begin(), h->re.s.end(), s);
    return DG_OK;
}

int32_t dg_reference(const dg_solver* h, int32_t which, double* out) {
    if (!h || !out) return fail(DG_EINVAL, "bad argument");
    const RefElement& re = h->re;
    switch (which) {
        case 0: std::copy(re.Dr.a.begin(), re.Dr.a.end(), out); break;
        case 1: std::copy(re.Ds.a.begin(), re.Ds.a.end(), out); break;
        case 2: std::copy(re.LIFT.a.begin(), re.LIFT.a.end(), out); break;
        case 3: std::copy(re.M.a.begin(), re.M.a.end(), out); break;
        case 4: std::copy(re.w.begin(), re.w.end(), out); break;
        case 5:
            for (size_t t = 0; t < re.fmask.size(); ++t) out[t] = re.fmask[t];
            break;
        case 6: {
            const OverInt& oi = h->oi;
            for (int c = 0; c < oi.Ncub; ++c) {
                out[c] = oi.rc[c];
                out[oi.Ncub + c] = oi.sc[c];
                out[2 * oi.Ncub + c] = oi.wc[c];
            }
            break;
        }
        case 7: std::copy(h->oi.Ic.a.begin(), h->oi.Ic.a.end(), out); break;
        case 8: std::copy(h->oi.Pr.a.begin(), h->oi.Pr.a.end(), out); break;
        case 9: std::copy(h->oi.Ps.a.begin(), h->oi.Ps.a.end(), out); break;
        case 10: std::copy(h->oi.P.a.begin(), h->oi.P.a.end(), out); break;
        case 11:
            for (int g = 0; g < h->oi.NG; ++g) {
                out[g] = h->oi.xg[g];
                out[h->oi.NG + g] = h->oi.wg[g];
            }
            break;
        case 12: std::copy(h->oi.I1.a.begin(), h->oi.I1.a.end(), out); break;
        case 13: std::copy(h->oi.Lg.a.begin(), h->oi.Lg.a.end(), out); break;
        default: return fail(DG_EINVAL, "unknown operator id");
    }
    return DG_OK;
}

int32_t dg_get_connectivity(const dg_solver* h, int32_t inst, int32_t* etoe, int8_t* etof) {
    if (!h || !etoe || !etof || inst < 0 || inst >= int(h->inst.size()))
        return fail(DG_EINVAL, "bad argument");
    const HostMesh& m = h->inst[inst].mesh;
    std::copy(m.etoe.begin(), m.etoe.end(), etoe);
    std::copy(m.etof.begin(), m.etof.end(), etof);
    return DG_OK;
}

int32_t dg_get_levels(const dg_solver* h, int32_t inst, int8_t* level, double* dt_min) {
    if (!h || inst < 0 || inst >= int(h->inst.size())) return fail(DG_EINVAL, "bad argument");
    const HostMesh& m = h->inst[inst].mesh;
    if (level) std::copy(m.level.begin(), m.level.end(), level);
    if (dt_min) *dt_min = h->inst[inst].dt_min;
    return DG_OK;
}

int32_t dg_get_tvb_stencil(const dg_solver* h, int32_t inst, int8_t* pair, double* alpha) {
    if (!h || !pair || !alpha || inst < 0 || inst >= int(h->inst.size()))
        return fail(DG_EINVAL, "bad argument");
    const HostMesh& m = h->inst[inst].mesh;
    std::copy(m.pair.begin(), m.pair.end(), pair);
    std::copy(m.alpha.begin(), m.alpha.end(), alpha);
    return DG_OK;
}

int32_t dg_bind(dg_solver* h, void* device_workspace, int64_t bytes, void* stream) {
    if (!h || !device_workspace) return fail(DG_EINVAL, "null handle or workspace");
    if ((reinterpret_cast<uintptr_t>(device_workspace) & 255) != 0)
        return fail(DG_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < int64_t(h->lay.total))
        return fail(DG_ENOMEM, "workspace too small: need " + std::to_string(h->lay.total) + " bytes");
    HIPCHECK(hipGetDevice(&h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    h->ws = static_cast<char*>(device_workspace);
    const Layout& l = h->lay;
    const RefElement& re = h->re;
    const int Np = h->Np, nF = h->nF;
    std::vector<float> Dr(Np * Np), Ds(Np * Np), LIFT(Np * nF);
    for (int t = 0; t < Np * Np; ++t) { Dr[t] = float(re.Dr.a[t]); Ds[t] = float(re.Ds.a[t]); }
    for (int t = 0; t < Np * nF; ++t) LIFT[t] = float(re.LIFT.a[t]);
    std::vector<int> nodeface(2 * Np, -1);
    for (int f = 0; f < 3; ++f)
        for (int j = 0; j < h->Nfp; ++j) {
            const int n = re.fmask[f * h->Nfp + j];
            if (nodeface[2 * n] < 0) nodeface[2 * n] = f * h->Nfp + j;
            else nodeface[2 * n + 1] = f * h->Nfp + j;
        }
    std::vector<double> wh(Np), pmid(3 * Np), phi(3 * Np);
    for (int j = 0; j < Np; ++j) wh[j] = 0.5 * re.w[j];
    for (int e = 0; e < 3; ++e)
        for (int j = 0; j < Np; ++j) {
            pmid[e * Np + j] = re.p1_mid(e, j) - 0.5 * re.w[j];
            phi[e * Np + j] = re.phi_mid(e, j);
        }
    // MFMA B-operand of [Dr Ds LIFT]^T in lane order: step s, lane l holds
    // Op[node l % 16][K index 4 s + l / 16] (0 outside Np x (2Np + 3Nfp))
    // FP32 MFMA B operand: column tile t (nodes 16 t .. 16 t + 15), step st,
    // lane ln -> Op[16 t + ln % 16][4 st + ln / 16]
    std::vector<float> amfma, amfma_img;
    const int NT = mfma_tiles(h->p.N);
    if (h->p.N <= 5) {
        const int KV = mfma_kv(h->p.N), KS = mfma_steps(h->p.N);
        amfma.assign(size_t(NT) * KS * 64, 0.f);
        for (int t = 0; t < NT; ++t)
            for (int st = 0; st < KS; ++st)
                for (int ln = 0; ln < 64; ++ln) {
                    const int node = 16 * t + ln % 16, kk = 4 * st + ln / 16;
                    if (node >= Np) continue;
                    double v = 0.0;
                    if (kk < Np) v = re.Dr(node, kk);
                    else if (kk < 2 * Np) v = re.Ds(node, kk - Np);
                    else if (kk >= KV && kk < KV + nF) v = re.LIFT(node, kk - KV);
                    amfma[(size_t(t) * KS + st) * 64 + ln] = float(v);
                }
    }
    auto up = [&](size_t off, const void* src, size_t n) {
        return hipMemcpyAsync(h->ws + off, src, n, hipMemcpyHostToDevice, s);
    };
    HIPCHECK(up(l.Dr, Dr.data(), Dr.size() * 4));
    HIPCHECK(up(l.Ds, Ds.data(), Ds.size() * 4));
    HIPCHECK(up(l.LIFT, LIFT.data(), LIFT.size() * 4));
    if (!amfma.empty()) {
        HIPCHECK(up(l.Amfma, amfma.data(), amfma.size() * 4));
        // the block's LDS image of the same table (rows padded to mfma_lds_row)
        const int KS = mfma_steps(h->p.N), OPS = mfma_lds_row(h->p.N);
        amfma_img.assign(size_t(NT) * 64 * OPS, 0.f);
        for (int t = 0; t < NT; ++t)
            for (int ln = 0; ln < 64; ++ln)
                for (int st = 0; st < KS; ++st)
                    amfma_img[(size_t(t) * 64 + ln) * OPS + st] = amfma[(size_t(t) * KS + st) * 64 + ln];
        HIPCHECK(up(l.AmfmaL, amfma_img.data(), amfma_img.size() * 4));
    }
    // BF16 engines: the same operator with K steps of 32, split into hi, mid
    // and lo BF16 parts (op = hi + mid + lo to 2^-24 relative)
    if (h->p.N <= 5) {
        const int KV = mfma_kv(h->p.N), KS = (KV + nF + 31) / 32;
        std::vector<uint16_t> abf(size_t(NT) * KS * 64 * 24, 0);
        for (int t = 0; t < NT; ++t)
            for (int st = 0; st < KS; ++st)
                for (int ln = 0; ln < 64; ++ln)
                    for (int i = 0; i < 8; ++i) {
                        const int node = 16 * t + ln % 16, kk = 32 * st + 8 * (ln / 16) + i;
                        double v = 0.0;
                        if (node < Np) {
                            if (kk < Np) v = re.Dr(node, kk);
                            else if (kk < 2 * Np) v = re.Ds(node, kk - Np);
                            else if (kk >= KV && kk < KV + nF) v = re.LIFT(node, kk - KV);
                        }
                        float r = float(v);
                        for (int u = 0; u < 3; ++u) {
                            const uint16_t b = bf16_round(r);
                            abf[((size_t(t) * KS + st) * 64 + ln) * 24 + 8 * u + i] = b;
                            r -= bf16_value(b);
                        }
                    }
        HIPCHECK(up(l.Abf, abf.data(), abf.size() * 2));
    }
    // FP64 MFMA A-operand of the element reductions: step s, lane l holds
    // W[row l % 16][node 4 s + l / 16], rows 0: w/2, 1-3: P1 midpoint - mean
    // FP64 MFMA A operand of the element reductions: step st, lane ln ->
    // row ln % 16 (0: w/2, 1-3: P1 midpoint functionals) at node 4 st + ln / 16
    const int KR = (Np + 3) / 4;
    std::vector<double> wred(size_t(8) * 64, 0.0);
    if (Np <= 32)
        for (int st = 0; st < KR; ++st)
            for (int ln = 0; ln < 64; ++ln) {
                const int row = ln % 16, nd = 4 * st + ln / 16;
                if (row > 3 || nd >= Np) continue;
                wred[size_t(st) * 64 + ln] = row == 0 ? wh[nd] : pmid[(row - 1) * Np + nd];
            }
    HIPCHECK(up(l.Wred, wred.data(), wred.size() * 8));
    // the matrix-core kernel numbers face nodes by formula
    for (size_t t = 0; t < re.fmask.size(); ++t)
        if (re.fmask[t] != face_node_index(h->p.N, int(t)))
            return fail(DG_EINVAL, "reference face nodes do not follow the row-by-row numbering");
    HIPCHECK(up(l.fmask, re.fmask.data(), re.fmask.size() * 4));
    HIPCHECK(up(l.nodeface, nodeface.data(), nodeface.size() * 4));
    HIPCHECK(up(l.wh, wh.data(), wh.size() * 8));
    HIPCHECK(up(l.pmid, pmid.data(), pmid.size() * 8));
    HIPCHECK(up(l.phi, phi.data(), phi.size() * 8));
    HIPCHECK(up(l.wfull, re.w.data(), re.w.size() * 8));
    {
        auto f32 = [](const Mat& m) {
            std::vector<float> v(m.a.size());
            for (size_t t = 0; t < v.size(); ++t) v[t] = float(m.a[t]);
            return v;
        };
        const OverInt& oi = h->oi;
        const std::vector<float> ic = f32(oi.Ic), pr = f32(oi.Pr), ps = f32(oi.Ps), pp = f32(oi.P),
                                 lg = f32(oi.Lg), i1 = f32(oi.I1);
        HIPCHECK(up(l.oIc, ic.data(), ic.size() * 4));
        HIPCHECK(up(l.oPr, pr.data(), pr.size() * 4));
        HIPCHECK(up(l.oPs, ps.data(), ps.size() * 4));
        HIPCHECK(up(l.oP, pp.data(), pp.size() * 4));
        HIPCHECK(up(l.oLg, lg.data(), lg.size() * 4));
        HIPCHECK(up(l.oI1, i1.data(), i1.size() * 4));
        // matrix-core tables (B operands of v_mfma_f32_16x16x4f32 in lane order)
        const int N = h->p.N;
        if (N <= 5) {
            const int T1 = overint_mfma_t1(N), S1 = overint_mfma_s1(N), TN = overint_mfma_tn(N);
            const int SC = overint_mfma_sc(N), SG = overint_mfma_sg(N), ST3 = overint_mfma_t3_steps(N);
            const int NC = oi.Ncub, NGF = 3 * oi.NG;
            std::vector<float> t1(size_t(T1) * S1 * 64, 0.f), t3(size_t(TN) * ST3 * 64, 0.f);
            for (int t = 0; t < T1; ++t)
                for (int st = 0; st < S1; ++st)
                    for (int ln = 0; ln < 64; ++ln) {
                        const int cub = 16 * t + ln % 16, node = 4 * st + ln / 16;
                        if (cub < NC && node < Np) t1[(size_t(t) * S1 + st) * 64 + ln] = float(oi.Ic(cub, node));
                    }
            for (int tn = 0; tn < TN; ++tn)
                for (int st = 0; st < ST3; ++st)
                    for (int ln = 0; ln < 64; ++ln) {
                        const int node = 16 * tn + ln % 16;
                        if (node >= Np) continue;
                        double v = 0.0;
                        if (st < 3 * SC) {
                            const int ch = st / SC, kk = 4 * (st - ch * SC) + ln / 16;
                            if (kk < NC) v = (ch == 0 ? oi.Pr : (ch == 1 ? oi.Ps : oi.P))(node, kk);
                        } else {
                            const int kk = 4 * (st - 3 * SC) + ln / 16;
                            if (kk < NGF) v = -oi.Lg(node, kk);
                        }
                        (void)SG;
                        t3[(size_t(tn) * ST3 + st) * 64 + ln] = float(v);
                    }
            HIPCHECK(up(l.oT1, t1.data(), t1.size() * 4));
            HIPCHECK(up(l.oT3, t3.data(), t3.size() * 4));
        }
    }
    HIPCHECK(up(l.conn, h->conn.data(), h->conn.size() * 4));
    HIPCHECK(up(l.stencil, h->stencil.data(), h->stencil.size() * 4));
    HIPCHECK(hipMemsetAsync(h->ws + l.dyn_begin, 0, l.dyn_end - l.dyn_begin, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (!h->exec) HIPCHECK(hipStreamCreateWithFlags(&h->exec, hipStreamNonBlocking));
    h->bound = true;
    h->prepared = false;
    return DG_OK;
}

int32_t dg_set_bathymetry(dg_solver* h, int32_t inst, const double* B) {
    if (!h || !B || inst < 0 || inst >= int(h->inst.size())) return fail(DG_EINVAL, "bad argument");
    const int Np = h->Np;
    Inst& I = h->inst[inst];
    if (h->B64.empty()) h->B64.assign(size_t(h->K) * Np, 0.0);
    if (h->Bh.empty()) h->Bh.assign(size_t(h->K) * Np, 0.f);
    if (h->dBh.empty()) h->dBh.assign(2 * size_t(h->K) * Np, 0.f);
    for (size_t t = 0; t < size_t(I.mesh.K) * Np; ++t)
        if (!std::isfinite(B[t])) return fail(DG_ENUMERIC, "non-finite bathymetry");
    const size_t KNp = size_t(h->K) * Np;
    for (int k = 0; k < I.mesh.K; ++k) {
        const int s = h->inv[I.offset + k];
        const double* b = B + size_t(k) * Np;
        for (int j = 0; j < Np; ++j) h->B64[size_t(s) * Np + j] = b[j];
        // gradient of the nodal bed polynomial: (rx Dr + sx Ds) B, (ry Dr + sy Ds) B
        const HostMesh& m = I.mesh;
        for (int i = 0; i < Np; ++i) {
            double br = 0.0, bs = 0.0;
            for (int j = 0; j < Np; ++j) {
                br += h->re.Dr(i, j) * b[j];
                bs += h->re.Ds(i, j) * b[j];
            }
            h->dBh[size_t(s) * Np + i] = float(m.rx[k] * br + m.sx[k] * bs);
            h->dBh[KNp + size_t(s) * Np + i] = float(m.ry[k] * br + m.sy[k] * bs);
        }
    }
    I.has_state = false;
    I.has_B = true;
    h->prepared = false;
    return DG_OK;
}

int32_t dg_set_state(dg_solver* h, int32_t inst, const double* hh, const double* hu, const double* hv,
                     void* stream) {
    (void)stream;
    if (!h || !hh || !hu || !hv || inst < 0 || inst >= int(h->inst.size()))
        return fail(DG_EINVAL, "bad argument");
    if (!h->bound) return fail(DG_ENOTBOUND, "dg_bind must be called before dg_set_state");
    Inst& I = h->inst[inst];
    if (!I.has_B) return fail(DG_ESTATE, "set the bathymetry of the instance first");
    const int Np = h->Np;
    const size_t KNp = size_t(h->K) * Np;
    if (h->Qh.empty()) h->Qh.assign(3 * KNp, 0.f);
    if (h->Ql.empty()) h->Ql.assign(KNp, 0);
    if (h->Bl.empty()) h->Bl.assign(KNp, 0);
    double amax = 0.0, eta_sum = 0.0;
    long long n_wet = 0;
    for (int k = 0; k < I.mesh.K; ++k) {
        const int s = h->inv[I.offset + k];
        for (int j = 0; j < Np; ++j) {
            const size_t src = size_t(k) * Np + j, dst = size_t(s) * Np + j;
            const double d = hh[src], mu = hu[src], mv = hv[src];
            if (!std::isfinite(d) || !std::isfinite(mu) || !std::isfinite(mv))
                return fail(DG_ENUMERIC, "non-finite initial state");
            if (d < 0.0) return fail(DG_ENUMERIC, "negative initial depth");
            if (d > h->p.h0) {
                eta_sum += d + h->B64[dst];
                ++n_wet;
            }
            const double f = 2.0 * d / (d * d + std::fmax(d * d, h->p.hvel * h->p.hvel));
            const double u = mu * f, v = mv * f;
            amax = std::fmax(amax, std::sqrt(u * u + v * v) + std::sqrt(h->p.g * d));
        }
    }
    // datum: mean wet surface level, rounded to the 2^-22 grid (any value
    // serves: the bed and the level are both stored relative to it)
    I.datum = n_wet ? float(std::ldexp(std::nearbyint(std::ldexp(eta_sum / double(n_wet), 22)), -22)) : 0.f;
    const double datum = double(I.datum);
    shift_bed(h, I, datum);
    for (int k = 0; k < I.mesh.K; ++k) {
        const int s = h->inv[I.offset + k];
        for (int j = 0; j < Np; ++j) {
            const size_t src = size_t(k) * Np + j, dst = size_t(s) * Np + j;
            const double b = h->B64[dst];
            // eta = h + B is snapped to a 2^-40 grid so that FP64 noise of the
            // caller's data (still water given as h = eta0 - B) does not reach
            // the finely rounded eta - datum; the level is stored as an FP32
            // pair hi + lo (compensated sum).  A dry node stores its bed pair,
            // and no node stores a surface below its bed
            float es = h->Bh[dst];
            int16_t el16 = h->Bl[dst];
            if (hh[src] > 0.0) {
                const double eta = hh[src] + b;
                const double snapped = std::fabs(eta) < 4096.0 ? std::nearbyint(eta * 0x1p40) * 0x1p-40 : eta;
                const double v = snapped - datum;
                if (v > b - datum) {
                    es = float(v);
                    el16 = lo_encode(es, float(v - double(es)));
                }
            }
            h->Qh[dst] = es;
            h->Qh[KNp + dst] = float(hu[src]);
            h->Qh[2 * KNp + dst] = float(hv[src]);
            h->Ql[dst] = el16;
        }
    }
    double rmin = I.mesh.inradius[0];
    for (double r : I.mesh.inradius) rmin = std::fmin(rmin, r);
    I.a_max = amax;
    I.dt_min = h->p.cfl * rmin / (double((h->p.N + 1) * (h->p.N + 1)) * std::fmax(amax, 1e-12));
    I.staged_datum = I.datum;
    I.staged_dt_min = I.dt_min;
    I.staged_a_max = I.a_max;
    if (h->p.regroup_every > 0) element_speeds(I.mesh, Np, hh, hu, hv, h->p.g, h->p.hvel, I.speed0);
    I.has_state = true;
    h->prepared = false;
    return DG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// stepping helpers
// ---------------------------------------------------------------------------
static StepArgs base_step_args(dg_solver* h) {
    StepArgs a{};
    const Layout& l = h->lay;
    a.N = h->p.N;
    a.engine = engine_of(h->p.precision);
    a.K = h->K;
    a.KNp = (long long)h->K * h->Np;
    a.KnF = (long long)h->K * h->nF;
    a.nlev = h->L;
    for (int q = 0; q < 2; ++q) a.Q[q] = reinterpret_cast<float*>(h->ws + l.Q[q]);
    a.B = reinterpret_cast<const float*>(h->ws + l.B);
    a.Blo = reinterpret_cast<const short*>(h->ws + l.Blo);
    a.dB = reinterpret_cast<const float*>(h->ws + l.dB);
    for (int s = 0; s < 3; ++s) a.R[s] = reinterpret_cast<float*>(h->ws + l.R[s]);
    a.half = h->L > 1 ? reinterpret_cast<float*>(h->ws + l.half) : nullptr;
    a.geo = reinterpret_cast<const float*>(h->ws + l.geo);
    a.gm = reinterpret_cast<const float*>(h->ws + l.gm);
    a.idt = reinterpret_cast<const float*>(h->ws + l.idt);
    a.conn = reinterpret_cast<const int*>(h->ws + l.conn);
    a.mrec = reinterpret_cast<double*>(h->ws + l.mrec);
    a.devs = reinterpret_cast<float*>(h->ws + l.devs);
    a.flags = reinterpret_cast<uint8_t*>(h->ws + l.flags);
    a.counters = reinterpret_cast<unsigned long long*>(h->ws + l.counters);
    a.ops.Dr = reinterpret_cast<const float*>(h->ws + l.Dr);
    a.ops.Ds = reinterpret_cast<const float*>(h->ws + l.Ds);
    a.ops.LIFT = reinterpret_cast<const float*>(h->ws + l.LIFT);
    a.ops.Amfma = reinterpret_cast<const float*>(h->ws + l.Amfma);
    a.ops.AmfmaL = reinterpret_cast<const float*>(h->ws + l.AmfmaL);
    a.ops.Abf = h->ws + l.Abf;
    a.ops.fmask = reinterpret_cast<const int*>(h->ws + l.fmask);
    a.ops.nodeface = reinterpret_cast<const int*>(h->ws + l.nodeface);
    a.ops.wh = reinterpret_cast<const double*>(h->ws + l.wh);
    a.ops.pmid = reinterpret_cast<const double*>(h->ws + l.pmid);
    a.ops.phi = reinterpret_cast<const double*>(h->ws + l.phi);
    a.ops.Wred = reinterpret_cast<const double*>(h->ws + l.Wred);
    a.ops.oIc = reinterpret_cast<const float*>(h->ws + l.oIc);
    a.ops.oPr = reinterpret_cast<const float*>(h->ws + l.oPr);
    a.ops.oPs = reinterpret_cast<const float*>(h->ws + l.oPs);
    a.ops.oP = reinterpret_cast<const float*>(h->ws + l.oP);
    a.ops.oLg = reinterpret_cast<const float*>(h->ws + l.oLg);
    a.ops.oI1 = reinterpret_cast<const float*>(h->ws + l.oI1);
    a.ops.oT1 = reinterpret_cast<const float*>(h->ws + l.oT1);
    a.ops.oT3 = reinterpret_cast<const float*>(h->ws + l.oT3);
    a.g = float(h->p.g);
    a.h0 = float(h->p.h0);
    a.eps = float(h->p.eps);
    a.hvel = float(h->p.hvel);
    a.thin_cut = float(h->p.thin_cut);
    a.pp_on = (h->p.limiter_mask & DG_LIMIT_PP) ? 1 : 0;
    a.dry_literal = h->p.dry_literal;
    return a;
}

static void fill_levels(dg_solver* h, LevelArgs* lev, int n_active, bool limit_only) {
    for (int l = 0; l < h->L; ++l) {
        LevelArgs& la = lev[l];
        la = LevelArgs{};
        la.begin = h->lev_begin[l];
        la.end = h->lev_end[l];
        la.parity = h->parity[l];
        la.active = (l < n_active) ? 1 : 0;
        la.scale = float(1 << l);
        const int nh = std::min(h->nhist[l], 2);
        for (int c = 0; c < 3; ++c) {
            la.ab[c] = limit_only ? 0.f : kAB[nh][c];
            la.half[c] = kHalf[nh][c];
        }
        la.slot[0] = h->head[l];
        la.slot[1] = (h->head[l] + 2) % 3;
        la.slot[2] = (h->head[l] + 1) % 3;
        la.write_half = (l > 0 && h->L > 1) ? 1 : 0;
    }
}

static TvbArgs tvb_args(dg_solver* h, const StepArgs& sa) {
    TvbArgs t{};
    t.K = h->K;
    t.KNp = sa.KNp;
    t.Np = h->Np;
    t.nlev = h->L;
    for (int l = 0; l < kMaxLevels; ++l) t.lev[l] = sa.lev[l];
    t.Q[0] = sa.Q[0];
    t.Q[1] = sa.Q[1];
    t.B = sa.B;
    t.Blo = sa.Blo;
    t.geo = sa.geo;
    t.conn = sa.conn;
    t.stencil = reinterpret_cast<const float*>(h->ws + h->lay.stencil);
    t.mrec = sa.mrec;
    t.devs = sa.devs;
    t.flags = sa.flags;
    t.phi = sa.ops.phi;
    t.g = h->p.g;
    t.h0 = h->p.h0;
    t.nu = h->p.tvb_nu;
    t.thin_cut = h->p.thin_cut;
    return t;
}

// Enqueue one tick (single rate: one step) on stream s.
// single-rate buffers of level 0 resolved for the kernels
static void resolve_single_rate(dg_solver* h, StepArgs& a) {
    const LevelArgs& l0 = a.lev[0];
    a.q_in = a.Q[l0.parity];
    a.q_out = a.Q[1 - l0.parity];
    a.r_now = a.R[l0.slot[0]];
    a.r_prev1 = a.R[l0.slot[1]];
    a.r_prev2 = a.R[l0.slot[2]];
}

static int enqueue_tick(dg_solver* h, int tick, hipStream_t s, bool limit_only) {
    int m = 1;
    if (!limit_only)
        while (m < h->L && tick % (1 << m) == 0) ++m;
    else
        m = h->L;
    StepArgs a = base_step_args(h);
    fill_levels(h, a.lev, m, limit_only);
    resolve_single_rate(h, a);
    a.k_begin = 0;
    a.k_end = h->lev_end[m - 1];
    const bool prof = h->profiling && !limit_only;
    std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
    if (prof) {
        if (h->prof_used == h->prof_events.size()) {
            hipEvent_t e0, e1;
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
            h->prof_events.push_back({e0, e1});
        }
        ev = &h->prof_events[h->prof_used++];
        h->prof_elems += a.k_end - a.k_begin;
    }
    if (limit_only) {
        a.mode = MODE_LIMIT_ONLY;
        if (launch_step(a, s, h->p.elems_per_block)) return fail(DG_EDEVICE, device_error_string());
    } else if (h->p.overint) {
        // over-integrated weak form: its right-hand side into the ring, then
        // the update and positivity limiter of the vector-ALU step kernel
        if (launch_rhs_overint(a, s, prof ? ev->first : nullptr, prof ? ev->second : nullptr))
            return fail(DG_EDEVICE, device_error_string());
        a.mode = MODE_UPDATE_ONLY;
        if (launch_step(a, s, 0)) return fail(DG_EDEVICE, device_error_string());
    } else if (h->p.precision == DG_PLAIN_FP32) {
        a.mode = MODE_RHS_ONLY;
        if (launch_step(a, s, h->p.elems_per_block, prof ? ev->first : nullptr, prof ? ev->second : nullptr))
            return fail(DG_EDEVICE, device_error_string());
        a.mode = MODE_UPDATE_ONLY;
        if (launch_step(a, s, h->p.elems_per_block)) return fail(DG_EDEVICE, device_error_string());
    } else {
        a.mode = MODE_FUSED;
        if (launch_step(a, s, h->p.elems_per_block, prof ? ev->first : nullptr, prof ? ev->second : nullptr))
            return fail(DG_EDEVICE, device_error_string());
    }
    if (h->p.limiter_mask & DG_LIMIT_TVB) {
        TvbArgs t = tvb_args(h, a);
        t.k_begin = 0;
        t.k_end = a.k_end;
        std::pair<hipEvent_t, hipEvent_t>* tev = nullptr;
        if (prof) {
            if (h->prof_tvb_used == h->prof_tvb_events.size()) {
                hipEvent_t e0, e1;
                HIPCHECK(hipEventCreate(&e0));
                HIPCHECK(hipEventCreate(&e1));
                h->prof_tvb_events.push_back({e0, e1});
            }
            tev = &h->prof_tvb_events[h->prof_tvb_used++];
        }
        if (launch_tvb(t, s, tev ? tev->first : nullptr, tev ? tev->second : nullptr))
            return fail(DG_EDEVICE, device_error_string());
    }
    for (int l = 0; l < m; ++l) {
        h->parity[l] ^= 1;
        if (!limit_only) {
            h->head[l] = (h->head[l] + 1) % 3;
            h->nhist[l] = std::min(h->nhist[l] + 1, 2);
        }
    }
    if (!limit_only) ++h->ticks;
    return DG_OK;
}

static int enqueue_coarse_step(dg_solver* h, hipStream_t s) {
    const int ticks = 1 << (h->L - 1);
    for (int t = 0; t < ticks; ++t) {
        const int rc = enqueue_tick(h, t, s, false);
        if (rc) return rc;
    }
    h->steps += 1;
    return DG_OK;
}

static void state_key(const dg_solver* h, int* key) {
    for (int l = 0; l < kMaxLevels; ++l) {
        key[3 * l] = h->parity[l];
        key[3 * l + 1] = h->head[l];
        key[3 * l + 2] = h->nhist[l];
    }
}

static bool all_started(const dg_solver* h) {
    for (int l = 0; l < h->L; ++l)
        if (h->nhist[l] < 2) return false;
    return true;
}

// reduction arguments of instance `inst` over the current state buffers
static DiagArgs diag_args(dg_solver* h, int inst) {
    DiagArgs a{};
    const Layout& l = h->lay;
    a.K = h->K;
    a.Np = h->Np;
    a.k_begin = 0;
    a.k_end = h->K;
    a.inst = inst;
    a.KNp = (long long)h->K * h->Np;
    a.Q = reinterpret_cast<const float*>(h->ws + l.Q[0]);
    a.Q2 = reinterpret_cast<const float*>(h->ws + l.Q[1]);
    a.nlev = h->L;
    fill_levels(h, a.lev, h->L, true);
    a.B = reinterpret_cast<const float*>(h->ws + l.B);
    a.Blo = reinterpret_cast<const short*>(h->ws + l.Blo);
    a.geo = reinterpret_cast<const float*>(h->ws + l.geo);
    a.wfull = reinterpret_cast<const double*>(h->ws + l.wfull);
    a.flags = reinterpret_cast<const uint8_t*>(h->ws + l.flags);
    return a;
}

// Regroup the elements into levels from the current state (the option the
// paper names after Algorithm 4.1), at a coarse-step boundary where every
// level is at the same time t, all with a full Adams-Bashforth history.
// Each element's samples R(t - dt), R(t - 2 dt), R(t - 3 dt) at its old step
// are replaced by the quadratic through them at t - dt', t - 2 dt', t - 3 dt'
// (dt' its new step); the device arrays are rebuilt in the new element order
// with every level's state in buffer 0 and its ring normalised to head 0.
static int regroup_now(dg_solver* h, hipStream_t s) {
    HIPCHECK(hipStreamSynchronize(s));
    const int K = h->K, Np = h->Np;
    const size_t KNp = size_t(K) * Np;
    const Layout& l = h->lay;
    // current state (each level's parity) and history samples, old order
    std::vector<float> q(3 * KNp);
    std::vector<int16_t> ql(KNp);
    std::vector<float> S[3];
    for (int t = 0; t < 3; ++t) S[t].assign(3 * KNp, 0.f);
    for (int lv = 0; lv < h->L; ++lv) {
        const size_t b0 = size_t(h->lev_begin[lv]) * Np, n = size_t(h->lev_end[lv] - h->lev_begin[lv]) * Np;
        if (!n) continue;
        const char* Q = h->ws + l.Q[h->parity[lv]];
        for (int c = 0; c < 3; ++c)
            HIPCHECK(hipMemcpy(q.data() + c * KNp + b0, Q + (c * KNp + b0) * 4, n * 4, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(ql.data() + b0, Q + 12 * KNp + b0 * 2, n * 2, hipMemcpyDeviceToHost));
        // ring: R(t - dt) in (head + 2) % 3, R(t - 2 dt) in (head + 1) % 3, R(t - 3 dt) in head
        const int slot[3] = {(h->head[lv] + 2) % 3, (h->head[lv] + 1) % 3, h->head[lv]};
        for (int t = 0; t < 3; ++t)
            for (int c = 0; c < 3; ++c)
                HIPCHECK(hipMemcpy(S[t].data() + c * KNp + b0, h->ws + l.R[slot[t]] + (c * KNp + b0) * 4, n * 4,
                                   hipMemcpyDeviceToHost));
    }
    std::vector<uint8_t> flags(K);
    HIPCHECK(hipMemcpy(flags.data(), h->ws + l.flags, K, hipMemcpyDeviceToHost));
    // new levels per instance from the state's wave speeds (FP64 of the stored pairs)
    std::vector<double> old_dt(K);
    for (int sidx = 0; sidx < K; ++sidx) {
        const Inst& I = h->inst[h->inst_of[sidx]];
        old_dt[sidx] = std::ldexp(I.dt_min, I.mesh.level[h->perm[sidx] - I.offset] - 1);
    }
    for (Inst& I : h->inst) {
        std::vector<double> hh(size_t(I.mesh.K) * Np), hu(hh.size()), hv(hh.size());
        for (int k = 0; k < I.mesh.K; ++k)
            for (int j = 0; j < Np; ++j) {
                const size_t src = size_t(h->inv[I.offset + k]) * Np + j, dst = size_t(k) * Np + j;
                hh[dst] = (double(q[src]) - double(h->Bh[src])) +
                          (double(lo_decode(q[src], ql[src])) - double(lo_decode(h->Bh[src], h->Bl[src])));
                hu[dst] = q[KNp + src];
                hv[dst] = q[2 * KNp + src];
            }
        std::vector<double> a;
        element_speeds(I.mesh, Np, hh.data(), hu.data(), hv.data(), h->p.g, h->p.hvel, a);
        I.t_base += double(h->ticks - I.tick_base) * I.dt_min;
        I.tick_base = h->ticks;
        I.dt_min = speed_levels(I.mesh, h->p.N, h->p.cfl, a, h->L);
    }
    // re-sample each element's history at its new step (old order)
    for (int sidx = 0; sidx < K; ++sidx) {
        const Inst& I = h->inst[h->inst_of[sidx]];
        const double rho = std::ldexp(I.dt_min, I.mesh.level[h->perm[sidx] - I.offset] - 1) / old_dt[sidx];
        if (rho == 1.0) continue;
        double w[3][3];
        for (int t = 0; t < 3; ++t) {
            const double tau = -(t + 1) * rho;
            w[t][0] = (tau + 2.0) * (tau + 3.0) / 2.0;
            w[t][1] = -(tau + 1.0) * (tau + 3.0);
            w[t][2] = (tau + 1.0) * (tau + 2.0) / 2.0;
        }
        for (int c = 0; c < 3; ++c)
            for (int j = 0; j < Np; ++j) {
                const size_t idx = c * KNp + size_t(sidx) * Np + j;
                const double s0 = S[0][idx], s1 = S[1][idx], s2 = S[2][idx];
                for (int t = 0; t < 3; ++t) S[t][idx] = float(w[t][0] * s0 + w[t][1] * s1 + w[t][2] * s2);
            }
    }
    // new order; state, samples and flags move with it
    const std::vector<int> to = resort(h);
    move_rows(q, Np, 3, to);
    move_rows(ql, Np, 1, to);
    for (int t = 0; t < 3; ++t) move_rows(S[t], Np, 3, to);
    move_rows(flags, 1, 1, to);
    // every level: state in buffer 0, ring head 0 (slot 2: R(t - dt), slot 1:
    // R(t - 2 dt), slot 0: R(t - 3 dt), overwritten by the next right-hand side)
    for (int lv = 0; lv < kMaxLevels; ++lv) {
        h->parity[lv] = 0;
        h->head[lv] = 0;
        h->nhist[lv] = 2;
    }
    HIPCHECK(hipMemcpy(h->ws + l.Q[0], q.data(), q.size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.Q[0] + 12 * KNp, ql.data(), ql.size() * 2, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.R[2], S[0].data(), S[0].size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.R[1], S[1].data(), S[1].size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.R[0], S[2].data(), S[2].size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.flags, flags.data(), flags.size(), hipMemcpyHostToDevice));
    if (const int rc = upload_geometry(h, s, false); rc != DG_OK) return rc;
    HIPCHECK(hipMemcpy(h->ws + l.conn, h->conn.data(), h->conn.size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.stencil, h->stencil.data(), h->stencil.size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.B, h->Bh.data(), h->Bh.size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.Blo, h->Bl.data(), h->Bl.size() * 2, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.dB, h->dBh.data(), h->dBh.size() * 4, hipMemcpyHostToDevice));
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
        h->have_graph = false;
    }
    ++h->regroups;
    return DG_OK;
}

// Capture the next `period` coarse steps (the ring x ping-pong period) from
// the current schedule state into h->graph without running them.
static int capture_graph(dg_solver* h) {
    constexpr int period = 6;
    int key[3 * kMaxLevels];
    state_key(h, key);
    std::memcpy(h->graph_key, key, sizeof(key));
    const long long steps0 = h->steps;
    const int64_t ticks0 = h->ticks;
    int saved[3][kMaxLevels];
    for (int l = 0; l < kMaxLevels; ++l) {
        saved[0][l] = h->parity[l];
        saved[1][l] = h->head[l];
        saved[2][l] = h->nhist[l];
    }
    HIPCHECK(hipStreamBeginCapture(h->exec, hipStreamCaptureModeThreadLocal));
    int rc = DG_OK;
    for (int q = 0; q < period && rc == DG_OK; ++q) rc = enqueue_coarse_step(h, h->exec);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(h->exec, &g);
    // capture advanced the host-side schedule; the replays advance it
    for (int l = 0; l < kMaxLevels; ++l) {
        h->parity[l] = saved[0][l];
        h->head[l] = saved[1][l];
        h->nhist[l] = saved[2][l];
    }
    h->steps = steps0;
    h->ticks = ticks0;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ce != hipSuccess) return fail(DG_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    const hipError_t ie = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(DG_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    h->have_graph = true;
    return DG_OK;
}

extern "C" {

int32_t dg_capture_graph(dg_solver* h, void* stream) {
    if (!h) return fail(DG_EINVAL, "null handle");
    if (!h->prepared) {
        const int rc = dg_prepare(h, stream);
        if (rc) return rc;
    }
    if (!h->p.use_graph) return fail(DG_ESTATE, "graphs are off (use_graph = 0)");
    if (!all_started(h)) return fail(DG_ESTATE, "the Adams-Bashforth start-up (two steps) is not over");
    HIPCHECK(hipSetDevice(h->device));
    HIPCHECK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return capture_graph(h);
}

}  // extern "C"

extern "C" {

int32_t dg_prepare(dg_solver* h, void* stream) {
    if (!h) return fail(DG_EINVAL, "null handle");
    if (!h->bound) return fail(DG_ENOTBOUND, "no device buffer bound");
    for (size_t i = 0; i < h->inst.size(); ++i)
        if (!h->inst[i].has_state || !h->inst[i].has_B)
            return fail(DG_ENOTBOUND, "instance " + std::to_string(i) + " has no state/bathymetry");
    HIPCHECK(hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout& l = h->lay;
    // regrouping: the initial levels from the staged state's wave speeds
    if (h->p.regroup_every > 0) {
        for (Inst& I : h->inst) I.staged_dt_min = speed_levels(I.mesh, h->p.N, h->p.cfl, I.speed0, h->L);
        resort(h);
        HIPCHECK(hipMemcpyAsync(h->ws + l.conn, h->conn.data(), h->conn.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(h->ws + l.stencil, h->stencil.data(), h->stencil.size() * 4,
                                hipMemcpyHostToDevice, s));
        if (h->graph) {
            (void)hipGraphExecDestroy(h->graph);
            h->graph = nullptr;
            h->have_graph = false;
        }
    }
    // back to the staged state's datum and time step (a restored checkpoint
    // may have replaced them)
    for (Inst& I : h->inst) {
        if (I.datum != I.staged_datum) shift_bed(h, I, double(I.staged_datum));
        I.datum = I.staged_datum;
        I.dt_min = I.staged_dt_min;
        I.a_max = I.staged_a_max;
        I.t_base = 0.0;
        I.tick_base = 0;
    }
    if (const int rc = upload_geometry(h, s, true); rc != DG_OK) return rc;
    HIPCHECK(hipMemcpyAsync(h->ws + l.B, h->Bh.data(), h->Bh.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(h->ws + l.Blo, h->Bl.data(), h->Bl.size() * 2, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(h->ws + l.dB, h->dBh.data(), h->dBh.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemsetAsync(h->ws + l.dyn_begin, 0, l.dyn_end - l.dyn_begin, s));
    for (int q = 0; q < kMaxLevels; ++q) {
        h->parity[q] = 0;
        h->head[q] = 0;
        h->nhist[q] = 0;
    }
    HIPCHECK(hipMemcpyAsync(h->ws + l.Q[0], h->Qh.data(), h->Qh.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(h->ws + l.Q[0] + 12 * h->Ql.size(), h->Ql.data(), h->Ql.size() * 2,
                            hipMemcpyHostToDevice, s));
    h->steps = 0;
    h->ticks = 0;
    h->regroups = 0;
    // Q0 = TVB(PP(Pi_H Q0)), first line of Algorithm 5.1
    const int rc = enqueue_tick(h, 0, s, true);
    if (rc) return rc;
    HIPCHECK(hipStreamSynchronize(s));
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
        h->have_graph = false;
    }
    h->prepared = true;
    return DG_OK;
}

int32_t dg_advance(dg_solver* h, int32_t n_steps, void* stream) {
    if (!h) return fail(DG_EINVAL, "null handle");
    if (n_steps < 0) return fail(DG_EINVAL, "n_steps < 0");
    if (!h->prepared) {
        const int rc = dg_prepare(h, stream);
        if (rc) return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int period = 6;   // ring (3) and ping-pong (2) state repeats every 6 steps
    while (n_steps > 0) {
        const bool graph_ok = h->p.use_graph && !h->profiling && all_started(h) && n_steps >= period &&
                              h->p.regroup_every == 0;
        if (graph_ok) {
            int key[3 * kMaxLevels];
            state_key(h, key);
            if (h->have_graph && std::memcmp(key, h->graph_key, sizeof(key)) != 0) {
                // state not aligned with the captured sequence: one eager step
                const int rc = enqueue_coarse_step(h, s);
                if (rc) return rc;
                --n_steps;
                continue;
            }
            if (!h->have_graph) {
                const int rc = capture_graph(h);
                if (rc) return rc;
            }
            hipEvent_t e0, e1;
            HIPCHECK(hipEventCreateWithFlags(&e0, hipEventDisableTiming));
            HIPCHECK(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
            HIPCHECK(hipEventRecord(e0, s));
            HIPCHECK(hipStreamWaitEvent(h->exec, e0, 0));
            while (n_steps >= period) {
                HIPCHECK(hipGraphLaunch(h->graph, h->exec));
                n_steps -= period;
                h->steps += period;
                h->ticks += int64_t(period) << (h->L - 1);
            }
            HIPCHECK(hipEventRecord(e1, h->exec));
            HIPCHECK(hipStreamWaitEvent(s, e1, 0));
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            continue;
        }
        const int rc = enqueue_coarse_step(h, s);
        if (rc) return rc;
        --n_steps;
        if (h->p.regroup_every > 0 && h->steps % h->p.regroup_every == 0 && all_started(h)) {
            const int rr = regroup_now(h, s);
            if (rr) return rr;
        }
    }
    return DG_OK;
}

int32_t dg_autotune(dg_solver* h, int32_t reps, int32_t max_out, int32_t* n_out, int32_t* epb_out,
                    double* us_out, void* stream) {
    if (!h || !n_out || (max_out > 0 && (!epb_out || !us_out))) return fail(DG_EINVAL, "bad argument");
    if (!h->prepared) return fail(DG_ENOTBOUND, "prepare the state (dg_prepare) before tuning");
    if (reps < 1) reps = 10;
    HIPCHECK(hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int> cand;
    if (h->p.precision >= DG_FUSED_MFMA32) {
        const int epw = 64 / mfma_lanes(h->p.N);
        cand = {epw, 2 * epw, 4 * epw, 8 * epw};
    }
    else
        cand = {step_elems_per_block(h->p.N, engine_of(h->p.precision))};
    // The trial launches repeat the step kernel of the next tick (tick 0 of
    // the next coarse step, all levels active): they rewrite the buffers that
    // tick rewrites with the same values, except the flag bytes (which the TVB
    // pass has completed) and the negative-mean counter, saved and restored.
    HIPCHECK(hipStreamSynchronize(s));
    const Layout& l = h->lay;
    std::vector<uint8_t> flags(size_t(h->K));
    unsigned long long counter = 0;
    HIPCHECK(hipMemcpy(flags.data(), h->ws + l.flags, flags.size(), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(&counter, h->ws + l.counters, 8, hipMemcpyDeviceToHost));
    StepArgs a = base_step_args(h);
    fill_levels(h, a.lev, h->L, false);
    resolve_single_rate(h, a);
    a.k_begin = 0;
    a.k_end = h->lev_end[h->L - 1];
    a.mode = h->p.precision == DG_PLAIN_FP32 ? MODE_RHS_ONLY : MODE_FUSED;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    int best = cand[0];
    double best_us = 1e300;
    int n = 0;
    int rc = DG_OK;
    // over-integration: its right-hand-side kernel (one launch shape) is the
    // one timed; it rewrites ring slot 0 exactly as the next tick does
    const bool oi = h->p.overint != 0;
    if (oi) cand = {0};
    auto trial = [&](int c, hipEvent_t x, hipEvent_t y) {
        return oi ? launch_rhs_overint(a, s, x, y) : launch_step(a, s, c, x, y);
    };
    for (int c : cand) {
        double tot = 0.0;
        for (int w = 0; w < 2 && rc == DG_OK; ++w)
            if (trial(c, nullptr, nullptr)) rc = fail(DG_EDEVICE, device_error_string());
        for (int r = 0; r < reps && rc == DG_OK; ++r) {
            if (trial(c, e0, e1)) {
                rc = fail(DG_EDEVICE, device_error_string());
                break;
            }
            float ms = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = fail(DG_EDEVICE, "event timing failed");
                break;
            }
            tot += ms;
        }
        if (rc != DG_OK) break;
        const double us = 1000.0 * tot / reps;
        if (n < max_out) {
            epb_out[n] = c;
            us_out[n] = us;
        }
        ++n;
        if (us < best_us) {
            best_us = us;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DG_OK) return rc;
    HIPCHECK(hipStreamSynchronize(s));
    HIPCHECK(hipMemcpy(h->ws + l.flags, flags.data(), flags.size(), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + l.counters, &counter, 8, hipMemcpyHostToDevice));
    if (!oi) h->p.elems_per_block = best;
    if (h->graph) {   // captured launches carry the old block shape
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
        h->have_graph = false;
    }
    *n_out = n;
    return DG_OK;
}

int32_t dg_get_state(dg_solver* h, int32_t inst, double* hh, double* hu, double* hv, void* stream) {
    if (!h || !hh || !hu || !hv || inst < 0 || inst >= int(h->inst.size()))
        return fail(DG_EINVAL, "bad argument");
    if (!h->prepared) return fail(DG_ENOTBOUND, "no state on the device yet");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHECK(hipStreamSynchronize(s));
    const int Np = h->Np;
    const size_t KNp = size_t(h->K) * Np;
    const Inst& I = h->inst[inst];
    std::vector<float> q(3 * KNp), b(KNp);
    std::vector<int16_t> ql(KNp), bl(KNp);
    for (int l = 0; l < h->L; ++l) {
        const size_t b0 = size_t(h->lev_begin[l]) * Np, n = size_t(h->lev_end[l] - h->lev_begin[l]) * Np;
        if (!n) continue;
        const char* Q = h->ws + h->lay.Q[h->parity[l]];
        for (int c = 0; c < 3; ++c)
            HIPCHECK(hipMemcpy(q.data() + c * KNp + b0, Q + (c * KNp + b0) * 4, n * 4, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(ql.data() + b0, Q + 12 * KNp + b0 * 2, n * 2, hipMemcpyDeviceToHost));
    }
    HIPCHECK(hipMemcpy(b.data(), h->ws + h->lay.B, KNp * 4, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(bl.data(), h->ws + h->lay.Blo, KNp * 2, hipMemcpyDeviceToHost));
    for (int k = 0; k < I.mesh.K; ++k) {
        const size_t sidx = size_t(h->inv[I.offset + k]);
        for (int j = 0; j < Np; ++j) {
            const size_t src = sidx * Np + j, dst = size_t(k) * Np + j;
            hh[dst] = (double(q[src]) - double(b[src])) +
                      (double(lo_decode(q[src], ql[src])) - double(lo_decode(b[src], bl[src])));
            hu[dst] = double(q[KNp + src]);
            hv[dst] = double(q[2 * KNp + src]);
        }
    }
    return DG_OK;
}

int32_t dg_get_flags(dg_solver* h, int32_t inst, uint8_t* flags, void* stream) {
    if (!h || !flags || inst < 0 || inst >= int(h->inst.size())) return fail(DG_EINVAL, "bad argument");
    if (!h->prepared) return fail(DG_ENOTBOUND, "no state on the device yet");
    HIPCHECK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    std::vector<uint8_t> f(h->K);
    HIPCHECK(hipMemcpy(f.data(), h->ws + h->lay.flags, h->K, hipMemcpyDeviceToHost));
    const Inst& I = h->inst[inst];
    for (int k = 0; k < I.mesh.K; ++k) flags[k] = f[h->inv[I.offset + k]] & 0x0F;
    return DG_OK;
}

int32_t dg_get_diagnostics(dg_solver* h, int32_t inst, dg_diag* d, void* stream) {
    if (!h || !d || inst < 0 || inst >= int(h->inst.size())) return fail(DG_EINVAL, "bad argument");
    if (!h->prepared) return fail(DG_ENOTBOUND, "no state on the device yet");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout& l = h->lay;
    DiagArgs a = diag_args(h, inst);
    a.partial = reinterpret_cast<double*>(h->ws + l.diag_partial);
    a.out = reinterpret_cast<double*>(h->ws + l.diag_out);
    if (launch_diag(a, s)) return fail(DG_EDEVICE, device_error_string());
    double out[16];
    unsigned long long cnt[8];
    HIPCHECK(hipStreamSynchronize(s));
    HIPCHECK(hipMemcpy(out, h->ws + l.diag_out, 9 * 8, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(cnt, h->ws + l.counters, 8, hipMemcpyDeviceToHost));
    d->mass = out[0];
    d->min_depth = out[1];
    // simulated time from the tick count: independent of how the ticks were
    // grouped into launches, graph replays or checkpointed runs
    d->time = h->inst[inst].t_base + double(h->ticks - h->inst[inst].tick_base) * h->inst[inst].dt_min;
    d->steps = h->steps;
    d->negative_means = (int64_t)cnt[0];
    for (int q = 0; q < 3; ++q) d->pp_counts[q] = (int64_t)out[2 + q];
    for (int q = 0; q < 4; ++q) d->tvb_counts[q] = (int64_t)out[5 + q];
    return DG_OK;
}

int32_t dg_get_diagnostics_noalloc(dg_solver* h, int32_t inst, double* out_device, void* stream) {
    if (!h || !out_device || inst < 0 || inst >= int(h->inst.size())) return fail(DG_EINVAL, "bad argument");
    if (!h->prepared) return fail(DG_ENOTBOUND, "no state on the device yet");
    if ((reinterpret_cast<uintptr_t>(out_device) & 7) != 0) return fail(DG_EINVAL, "out_device must be 8-byte aligned");
    // the partial sums have a fixed count (the reduction's block count) that
    // the device array holds whatever the element count
    if (diag_scratch_doubles() < 256 * 16) return fail(DG_EINVAL, "reduction partials exceed the scratch array");
    const DiagArgs a = diag_args(h, inst);
    if (launch_diag_static(a, out_device, stream)) return fail(DG_EDEVICE, device_error_string());
    return DG_OK;
}

// checkpoint blob: a 256-byte header (solver shape, per-level schedule
// state, step and tick counts), one 32-byte record per instance (datum of the
// stored levels, time step, initial wave speed, hash of the FP64 bed), then
// the device state
struct CkptHeader {
    uint64_t magic, K, Np, L, n_inst;
    int32_t parity[kMaxLevels], head[kMaxLevels], nhist[kMaxLevels];
    int64_t steps, ticks;
};
static_assert(sizeof(CkptHeader) <= 256, "checkpoint header exceeds its slot");
struct CkptInst {
    double datum, dt_min, a_max;
    uint64_t bed_hash;
    double t_base;
    int64_t tick_base;
};
static constexpr uint64_t kCkptMagic = 0x4447535703ull;

// header, instance records, then every element's level (global order)
static size_t ckpt_levels_offset(const dg_solver* h) { return 256 + align256(h->inst.size() * sizeof(CkptInst)); }
static size_t ckpt_prefix_bytes(const dg_solver* h) { return ckpt_levels_offset(h) + align256(size_t(h->K)); }

// FNV-1a over the instance's FP64 bed values in the caller's element order
static uint64_t bed_hash(const dg_solver* h, int inst) {
    const Inst& I = h->inst[inst];
    uint64_t x = 1469598103934665603ull;
    for (int k = 0; k < I.mesh.K; ++k) {
        const unsigned char* p = reinterpret_cast<const unsigned char*>(&h->B64[size_t(h->inv[I.offset + k]) * h->Np]);
        for (size_t t = 0; t < size_t(h->Np) * 8; ++t) x = (x ^ p[t]) * 1099511628211ull;
    }
    return x;
}

int32_t dg_checkpoint_bytes(const dg_solver* h, int64_t* bytes) {
    if (!h || !bytes) return fail(DG_EINVAL, "bad argument");
    *bytes = int64_t(ckpt_prefix_bytes(h) + (h->lay.dyn_end - h->lay.dyn_begin));
    return DG_OK;
}

int32_t dg_get_checkpoint(dg_solver* h, void* blob, int64_t bytes, void* stream) {
    int64_t need = 0;
    if (dg_checkpoint_bytes(h, &need)) return DG_EINVAL;
    if (!blob || bytes < need) return fail(DG_EINVAL, "checkpoint buffer too small");
    if (!h->prepared) return fail(DG_ENOTBOUND, "no state on the device yet");
    HIPCHECK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    char* b = static_cast<char*>(blob);
    const size_t pb = ckpt_prefix_bytes(h);
    std::memset(b, 0, pb);
    CkptHeader* hd = reinterpret_cast<CkptHeader*>(b);
    hd->magic = kCkptMagic;
    hd->K = h->K;
    hd->Np = h->Np;
    hd->L = h->L;
    hd->n_inst = h->inst.size();
    for (int l = 0; l < kMaxLevels; ++l) {
        hd->parity[l] = h->parity[l];
        hd->head[l] = h->head[l];
        hd->nhist[l] = h->nhist[l];
    }
    hd->steps = h->steps;
    hd->ticks = h->ticks;
    CkptInst* ci = reinterpret_cast<CkptInst*>(b + 256);
    for (size_t i = 0; i < h->inst.size(); ++i) {
        ci[i].datum = double(h->inst[i].datum);
        ci[i].dt_min = h->inst[i].dt_min;
        ci[i].a_max = h->inst[i].a_max;
        ci[i].bed_hash = bed_hash(h, int(i));
        ci[i].t_base = h->inst[i].t_base;
        ci[i].tick_base = h->inst[i].tick_base;
        int8_t* lv = reinterpret_cast<int8_t*>(b + ckpt_levels_offset(h)) + h->inst[i].offset;
        std::copy(h->inst[i].mesh.level.begin(), h->inst[i].mesh.level.end(), lv);
    }
    HIPCHECK(hipMemcpy(b + pb, h->ws + h->lay.dyn_begin, h->lay.dyn_end - h->lay.dyn_begin,
                       hipMemcpyDeviceToHost));
    return DG_OK;
}

int32_t dg_set_checkpoint(dg_solver* h, const void* blob, int64_t bytes, void* stream) {
    int64_t need = 0;
    if (dg_checkpoint_bytes(h, &need)) return DG_EINVAL;
    if (!blob || bytes < need) return fail(DG_EINVAL, "checkpoint buffer too small");
    if (!h->prepared) return fail(DG_ESTATE, "call dg_prepare (or advance) before restoring");
    const char* b = static_cast<const char*>(blob);
    CkptHeader hd;
    std::memcpy(&hd, b, sizeof(hd));
    if (hd.magic != kCkptMagic || hd.K != uint64_t(h->K) || hd.Np != uint64_t(h->Np) ||
        hd.L != uint64_t(h->L) || hd.n_inst != uint64_t(h->inst.size()))
        return fail(DG_EINVAL, "checkpoint does not match this solver");
    // the schedule state indexes the state ping-pong and the RHS ring
    for (int l = 0; l < kMaxLevels; ++l)
        if (hd.parity[l] < 0 || hd.parity[l] > 1 || hd.head[l] < 0 || hd.head[l] > 2 || hd.nhist[l] < 0 ||
            hd.nhist[l] > 2)
            return fail(DG_EINVAL, "corrupt checkpoint: schedule state out of range");
    if (hd.steps < 0 || hd.ticks < 0) return fail(DG_EINVAL, "corrupt checkpoint: negative step or tick count");
    std::vector<CkptInst> ci(h->inst.size());
    std::memcpy(ci.data(), b + 256, ci.size() * sizeof(CkptInst));
    for (size_t i = 0; i < ci.size(); ++i) {
        if (!std::isfinite(ci[i].datum) || !(ci[i].dt_min > 0.0) || !std::isfinite(ci[i].dt_min) ||
            !std::isfinite(ci[i].a_max))
            return fail(DG_EINVAL, "corrupt checkpoint: instance " + std::to_string(i) + " record");
        if (ci[i].bed_hash != bed_hash(h, int(i)))
            return fail(DG_EINVAL, "checkpoint was taken over another bathymetry (instance " + std::to_string(i) + ")");
        if (ci[i].tick_base < 0 || ci[i].tick_base > hd.ticks || !std::isfinite(ci[i].t_base))
            return fail(DG_EINVAL, "corrupt checkpoint: instance " + std::to_string(i) + " time record");
    }
    const int8_t* blev = reinterpret_cast<const int8_t*>(b + ckpt_levels_offset(h));
    bool same_levels = true;
    for (size_t i = 0; i < ci.size(); ++i)
        for (int k = 0; k < h->inst[i].mesh.K; ++k) {
            const int8_t v = blev[h->inst[i].offset + k];
            if (v < 1 || v > h->L) return fail(DG_EINVAL, "corrupt checkpoint: element level out of range");
            if (v != h->inst[i].mesh.level[k]) same_levels = false;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHECK(hipStreamSynchronize(s));
    // the stored levels are relative to the checkpoint's datum and advance
    // with its time step: rebuild the shifted bed and the time-step slot of
    // the geometry records from them
    for (size_t i = 0; i < ci.size(); ++i) {
        Inst& I = h->inst[i];
        I.datum = float(ci[i].datum);
        I.dt_min = ci[i].dt_min;
        I.a_max = ci[i].a_max;
        I.t_base = ci[i].t_base;
        I.tick_base = ci[i].tick_base;
        shift_bed(h, I, double(I.datum));
    }
    // a regrouped run: the blob's element order is that of its levels
    if (!same_levels) {
        for (size_t i = 0; i < ci.size(); ++i)
            std::copy(blev + h->inst[i].offset, blev + h->inst[i].offset + h->inst[i].mesh.K,
                      h->inst[i].mesh.level.begin());
        resort(h);
        HIPCHECK(hipMemcpy(h->ws + h->lay.conn, h->conn.data(), h->conn.size() * 4, hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(h->ws + h->lay.stencil, h->stencil.data(), h->stencil.size() * 4, hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(h->ws + h->lay.dB, h->dBh.data(), h->dBh.size() * 4, hipMemcpyHostToDevice));
        if (h->graph) {
            (void)hipGraphExecDestroy(h->graph);
            h->graph = nullptr;
            h->have_graph = false;
        }
    }
    if (const int rc = upload_geometry(h, s, false); rc != DG_OK) return rc;
    HIPCHECK(hipMemcpy(h->ws + h->lay.B, h->Bh.data(), h->Bh.size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + h->lay.Blo, h->Bl.data(), h->Bl.size() * 2, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->ws + h->lay.dyn_begin, b + ckpt_prefix_bytes(h), h->lay.dyn_end - h->lay.dyn_begin,
                       hipMemcpyHostToDevice));
    for (int l = 0; l < kMaxLevels; ++l) {
        h->parity[l] = hd.parity[l];
        h->head[l] = hd.head[l];
        h->nhist[l] = hd.nhist[l];
    }
    h->steps = hd.steps;
    h->ticks = hd.ticks;
    return DG_OK;
}

int32_t dg_set_profiling(dg_solver* h, int32_t on) {
    if (!h) return fail(DG_EINVAL, "null handle");
    h->profiling = on != 0;
    h->prof_used = 0;
    h->prof_tvb_used = 0;
    h->prof_elems = 0;
    return DG_OK;
}

int32_t dg_kernel_timing(const dg_solver* hc, int32_t which, double* avg_us, int64_t* launches,
                         int64_t* elems) {
    if (!hc || (which != 0 && which != 1)) return fail(DG_EINVAL, "null handle or unknown kernel id");
    dg_solver* h = const_cast<dg_solver*>(hc);
    const auto& evs = which == 0 ? h->prof_events : h->prof_tvb_events;
    const size_t used = which == 0 ? h->prof_used : h->prof_tvb_used;
    double tot = 0.0;
    for (size_t i = 0; i < used; ++i) {
        HIPCHECK(hipEventSynchronize(evs[i].second));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, evs[i].first, evs[i].second));
        tot += ms;
    }
    if (avg_us) *avg_us = used ? tot * 1000.0 / used : 0.0;
    if (launches) *launches = (int64_t)used;
    // the TVB kernel of a tick covers the same element range as its step kernel
    if (elems) *elems = h->prof_used ? (h->prof_elems + (long long)h->prof_used / 2) / (long long)h->prof_used : 0;
    return DG_OK;
}

}  // extern "C"
