// Kernel argument blocks and launchers shared by the host solver and the HIP
// kernels.  Plain C++ types only; streams travel as void*.
#pragma once

#include <cstddef>
#include <cstdint>

namespace dgswe {

constexpr int kMaxLevels = 6;
// Connectivity record (int4 per element): the three neighbours (-1: wall),
// then the neighbours' face numbers in bits 0-5 (two bits per face) and the
// element's instance in bits kConnInstShift and up.
constexpr int kConnInstShift = 8;
constexpr int kMaxInstances = 1 << (31 - kConnInstShift);
// Face node fn = f (N+1) + p of the reference triangle (faces s = -1, r + s
// = 0, r = -1, each in counter-clockwise order) for nodes numbered row by row
// in s, row j holding N+1-j nodes in increasing r.  The host checks its face
// masks against this numbering when it binds.
constexpr int face_node_index(int N, int fn) {
    const int Nfp = N + 1, f = fn / Nfp, p = fn % Nfp;
    const int i = f == 0 ? p : (f == 1 ? N - p : 0);   // r index
    const int j = f == 0 ? 0 : (f == 1 ? p : N - p);   // s index
    return j * (N + 1) - j * (j - 1) / 2 + i;
}

// all 3(N+1) face nodes packed 4 bits each (N <= 4)
constexpr unsigned long long face_node_bits(int N) {
    unsigned long long b = 0;
    for (int fn = 0; fn < 3 * (N + 1); ++fn) b |= (unsigned long long)face_node_index(N, fn) << (4 * fn);
    return b;
}

// face nodes packed 5 bits each, twelve to a word (N = 5: two words)
constexpr unsigned long long face_node_bits5(int N, int part) {
    unsigned long long b = 0;
    for (int fn = 12 * part; fn < 3 * (N + 1) && fn < 12 * part + 12; ++fn)
        b |= (unsigned long long)face_node_index(N, fn) << (5 * (fn - 12 * part));
    return b;
}

// Kernel modes of the step kernel.
enum StepMode : int {
    MODE_FUSED = 0,        // RHS + AB update + positivity limiter + means/deviations
    MODE_RHS_ONLY = 1,     // RHS into ring slot 0 (unfused path, first kernel)
    MODE_UPDATE_ONLY = 2,  // AB update from ring slots + limiter (unfused path, second kernel)
    MODE_LIMIT_ONLY = 3,   // copy state + positivity limiter (initial Q0 = TVB(PP(Q0)))
};

// Contraction engine of the step kernel.
enum Engine : int { ENGINE_VALU = 0, ENGINE_MFMA_F32 = 1, ENGINE_MFMA_BF16X3 = 2, ENGINE_MFMA_BF16X6 = 3 };

struct LevelArgs {
    int begin, end;        // element range of the level (sorted order)
    int parity;            // ping-pong buffer holding the level's current state
    int active;            // level steps at this tick
    float scale;           // dt_l / dt_min = 2^(l-1)
    float ab[3];           // Adams-Bashforth weights (zeros beyond the history)
    int slot[3];           // ring slots of R^n, R^{n-1}, R^{n-2}
    float half[3];         // half-step weights when write_half
    int write_half;        // level writes its half-step face traces
};

struct DevOps {
    const float* Dr;       // Np x Np
    const float* Ds;       // Np x Np
    const float* LIFT;     // Np x 3Nfp
    const float* Amfma;    // FP32 MFMA B operand: step s, lane l -> Op[l % 16][4 s + l / 16]
    const float* AmfmaL;   // the same table as the block's LDS image: row 64 t + l holds the
                           // steps of lane l of tile t, row stride mfma_lds_row(N) floats
    const void* Abf;       // BF16 MFMA B operand: step s, lane l -> hi, mid, lo parts (8 bf16
                           // each) of Op[l % 16][32 s + 8 (l / 16) + i], i = 0..7
    const int* fmask;      // 3Nfp
    const int* nodeface;   // Np x 2 (face-node slot of each volume node, -1 none)
    const double* wh;      // Np: w / 2 (cell-mean weights)
    const double* pmid;    // 3 x Np: P1 midpoint value minus mean
    const double* phi;     // 3 x Np: midpoint-Lagrange P1 basis at the nodes
    const double* Wred;    // FP64 MFMA A-operand of [w/2; P1 midpoint - mean] (4 x 64)
    // over-integrated weak form (FP32): Ic [Ncub][Np], Pr, Ps, P [Np][Ncub],
    // Lg [Np][3 NG], I1 [NG][Nfp] (see overint_points)
    const float* oIc;
    const float* oPr;
    const float* oPs;
    const float* oP;
    const float* oLg;
    const float* oI1;
    // matrix-core tables of the over-integrated form, B operands of
    // v_mfma_f32_16x16x4f32 in lane order (see overint_mfma_* below)
    const float* oT1;      // Ic^T: [tile t][step st][lane l] = Ic[16 t + l % 16][4 st + l / 16]
    const float* oT3;      // [node tile][chunk][step][lane] = Op_chunk[node 16 tn + l % 16][4 st + l / 16],
                           // chunks Pr, Ps, P (K = Ncub), -L^g (K = 3 NG)
};

// points per direction of the over-integrated rules (exact to degree 3N):
// Ncub = q^2 cubature nodes, q Gauss points per face
constexpr int overint_points(int N) { return (3 * N + 2) / 2; }
// matrix-core form: steps of K = 4 over the nodes (stage 1), the cubature
// nodes and the Gauss points (stage 3), and the column tiles of 16
constexpr int overint_mfma_s1(int N) { return ((N + 1) * (N + 2) / 2 + 3) / 4; }
constexpr int overint_mfma_t1(int N) { return (overint_points(N) * overint_points(N) + 15) / 16; }
constexpr int overint_mfma_sc(int N) { return (overint_points(N) * overint_points(N) + 3) / 4; }
constexpr int overint_mfma_sg(int N) { return (3 * overint_points(N) + 3) / 4; }
constexpr int overint_mfma_tn(int N) { return ((N + 1) * (N + 2) / 2 + 15) / 16; }
constexpr int overint_mfma_t3_steps(int N) { return 3 * overint_mfma_sc(N) + overint_mfma_sg(N); }

struct StepArgs {
    int N, mode, engine;
    int K;                 // total elements
    long long KNp;         // K * Np (field stride)
    long long KnF;         // K * 3Nfp (half-trace field stride)
    int k_begin, k_end;    // element range of this launch
    int nlev;
    LevelArgs lev[kMaxLevels];
    float* Q[2];           // ping-pong state buffers: [3][K*Np] FP32 eta (hi), hu, hv, then
                           // [K*Np] 16-bit eta (lo) at float offset 3 K*Np
    const float* B;        // [K*Np] bed relative to the datum, FP32 high word
    const short* Blo;      // [K*Np] its low word, 16-bit (encoding of the level's low word)
    const float* dB;       // [2][K*Np] dB/dx, dB/dy at the nodes (static, from FP64 on the host)
    float* R[3];           // ring slots [3][K*Np]
    // single rate: the level's buffers resolved on the host (state in / out,
    // RHS slots of R^n, R^{n-1}, R^{n-2})
    const float* q_in;
    float* q_out;
    float* r_now;
    const float* r_prev1;
    const float* r_prev2;
    float* half;           // [3][K*3Nfp] half-step face traces (multi-rate) or null
    // multi-rate matrix-core kernel (filled by the launcher): the launch's
    // element range cut at level boundaries, each level's part taking whole
    // blocks so that a block belongs to one level
    int seg_begin[kMaxLevels], seg_end[kMaxLevels];
    int seg_block[kMaxLevels + 1];   // first block of each level's part; total last
    unsigned parity_bits;  // bit l: parity of level l
    unsigned active_bits;  // bit l: level l steps at this tick
    unsigned q_pair_bytes; // byte distance from Q[0] to Q[1]
    const float* geo;      // [K][16]
    const float* gm;       // [K][4] rx, ry, sx, sy (the geometry row's first four)
    const float* idt;      // [instances] FP32 time step dt_min of each instance
    const int* conn;       // [K][4]
    double* mrec;          // [K][4] post-positivity means h, hu, hv and the positivity code
    float* devs;           // [9][K] P1 edge-midpoint deviations (elements that are not dry)
    uint8_t* flags;        // [K]
    unsigned long long* counters;  // [0] negative-mean events
    DevOps ops;
    float g, h0, eps, hvel;
    float thin_cut;        // > 0: momentum zeroed at output nodes with depth below it
    int pp_on, dry_literal;
};

struct TvbArgs {
    int K;
    long long KNp;
    int Np;
    int k_begin, k_end;
    int nlev;
    LevelArgs lev[kMaxLevels];
    float* Q[2];
    const float* B;
    const short* Blo;
    const float* geo;
    const int* conn;
    const float* stencil;  // [K][16]
    const double* mrec;    // [K][4] as written by the step kernel
    const float* devs;     // [9][K]
    uint8_t* flags;
    const double* phi;     // 3 x Np
    double g, h0, nu;
    double thin_cut;       // as StepArgs::thin_cut
};

struct DiagArgs {
    int K, Np, k_begin, k_end, inst;
    long long KNp;
    const float* Q;        // state buffer, layout of StepArgs::Q (per element parity resolved by caller)
    const float* Q2;       // second buffer
    const int* parity_of;  // null: all from Q; else per-level parity via lev table
    int nlev;
    LevelArgs lev[kMaxLevels];
    const float* B;
    const short* Blo;
    const float* geo;
    const double* wfull;   // Np: w
    const uint8_t* flags;
    double* partial;       // [blocks][16]
    double* out;           // [16]
};

// ev_start / ev_stop (hipEvent_t, optional): timestamps of the kernel itself
int launch_step(const StepArgs& a, void* stream, int elems_per_block, void* ev_start = nullptr,
                void* ev_stop = nullptr);
int launch_tvb(const TvbArgs& a, void* stream, void* ev_start = nullptr, void* ev_stop = nullptr);
// right-hand side of the over-integrated weak form into a.r_now (multi-rate:
// the ring slot of each element's level), N <= 5
int launch_rhs_overint(const StepArgs& a, void* stream, void* ev_start = nullptr, void* ev_stop = nullptr);
int launch_diag(const DiagArgs& a, void* stream);
// the same reduction with its partial sums in a fixed device array (no
// workspace, no allocation), results (9 doubles) written to `out` on the device
int launch_diag_static(const DiagArgs& a, double* out, void* stream);
int diag_scratch_doubles();
// elements per block: matrix-core kernel 1, 2, 4 or 8 waves of 64 / lanes
// elements (N = 1, 2, 4: 4, 8, 16, 32; N = 3: 5, 10, 20, 40; N = 5: 3, 6, 12,
// 24), default 8 waves at N = 3 and 5 (the fastest shapes there: C5 1035
// against 966 us, C4 585 against 551 us), 4 waves otherwise; VALU kernel
// floor(256 / Np) (fixed)
constexpr int mfma_default_waves(int N) { return N == 3 || N == 5 ? 8 : 4; }
int step_elems_per_block(int N, int engine);

// Lane groups of the matrix-core kernel.  N = 1, 2, 4: 16 lanes per element
// (four elements per wave), lane j of the group is node j and the contraction
// result arrives in the lane that owns the node.  N = 3 and N = 5 are packed:
// max(Np, 3(N+1)) lanes per element (12 and 21: five and three elements per
// wave instead of four and two), the contraction result goes through a small
// LDS transpose, and the node columns span (Np + 15) / 16 tiles of 16.
constexpr bool mfma_compact(int N) { return N == 3 || N == 5; }
constexpr int mfma_lanes(int N) {
    return mfma_compact(N) ? ((N + 1) * (N + 2) / 2 > 3 * (N + 1) ? (N + 1) * (N + 2) / 2 : 3 * (N + 1)) : 16;
}
constexpr int mfma_tiles(int N) { return ((N + 1) * (N + 2) / 2 + 15) / 16; }

// K layout of the matrix-core contraction (N <= 5): Dr columns 0..Np-1, Ds
// columns Np..2Np-1, zero padding to mfma_kv(N) (a multiple of 4), LIFT
// columns from mfma_kv(N); mfma_steps(N) steps of K = 4 in total, the first
// mfma_kv(N) / 4 of them volume-only
constexpr int mfma_kv(int N) { return ((N + 1) * (N + 2) + 3) & ~3; }
constexpr int mfma_steps(int N) { return (mfma_kv(N) + 3 * (N + 1) + 3) / 4; }
// row stride (floats) of the FP32 operator table staged in LDS: the steps
// padded to a multiple of 4, plus 4 when that is a multiple of 8, so that the
// 128-bit reads of consecutive lanes fall in distinct banks
constexpr int mfma_lds_row(int N) {
    return ((mfma_steps(N) + 3) & ~3) % 8 == 0 ? ((mfma_steps(N) + 3) & ~3) + 4 : ((mfma_steps(N) + 3) & ~3);
}
const char* device_error_string();

}  // namespace dgswe
