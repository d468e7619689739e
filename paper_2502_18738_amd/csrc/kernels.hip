// kernels.hip -- gfx950 kernels of the wildfire cellular automaton.
//
// The hot path is `k_step`: one work-group advances one tile of one scenario
// by up to KM steps entirely in LDS (temporal blocking); step s of a K-step
// launch only tries the cells within K - s cells of the tile, the ones that
// can still reach it before the launch ends.  The state is two
// bit-planes (burning, burned); a 64-lane wavefront treats 64 words = 2048
// cells per bitwise instruction, so finding the cells that need a Bernoulli
// trial (burning cells, and burnable cells with fuel next to a burning cell,
// Sec. 2.2 transition rules) costs a handful of bit operations per 32 cells.
// The per-edge terms of Eq. 1-5 are evaluated once per run for every edge by
// `k_qtable` (parameters and fields do not change within a run); a step only
// gathers the 32-byte table row of each ignition-trial cell, so the step's
// memory traffic scales with the fire front, not with the grid.  Trials are
// compacted into an LDS list by a work-group prefix sum and dealt to the
// work-group's lanes, so one busy word does not serialise a wavefront.
//
// Compiled with -ffp-contract=off: every FP32 operation rounds as written, so
// every kernel that evaluates Eq. 2-5 and 9 produces the same bits, and the
// adjoint recompute takes exactly the forward's ignition decisions.
#include "internal.h"

#include <math.h>

#include <algorithm>
#include <climits>

namespace fs {

namespace {

constexpr float kRad2Deg = 57.295779513082320876798f;
constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kLn2 = 0.69314718055994530942f;
constexpr float kTwoM24 = 5.9604644775390625e-08f;  // 2^-24
constexpr float kTieEps = 1e-5f;

// Three-input XOR in one VALU instruction (gfx950 v_bitop3_b32, truth
// table 0x96 = a ^ b ^ c); the key operand may be a scalar register.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11): returns words 0 and 1.
__device__ __forceinline__ void philox_w01(uint32_t c0, uint32_t c1, uint32_t c2,
                                           uint32_t c3, uint32_t k0, uint32_t k1,
                                           uint32_t& w0, uint32_t& w1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        // one 32 x 32 -> 64-bit product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        if (i < 2) {
            // the callers' step and scenario words are uniform, so part of the
            // first two rounds stays in scalar registers: plain XORs there
            c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        } else {
            c0 = xor3((uint32_t)(p1 >> 32), c1, k0);
            c2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    w0 = c0;
    w1 = c1;
}

__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * kTwoM24; }

// Global-memory view of a pointer read from a descriptor.  The compiler cannot
// infer the address space of such pointers and would use generic (flat)
// accesses, which also count against the LDS wait counter: every LDS wait of
// the step loop would then wait for outstanding HBM reads as well.
#define FS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ FS_GLOBAL T* gmem(T* p) {
    return (FS_GLOBAL T*)p;
}

// 16-byte vector read through a global pointer (HIP's float4 cannot be copied
// out of a non-generic address space).
typedef float fs_f4 __attribute__((ext_vector_type(4)));
typedef int fs_i4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_f4(const void* base, int64_t i) {
    const fs_f4 v = ((const FS_GLOBAL fs_f4*)base)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

// Neighbour slot e = 0..7 walks the 3 x 3 block row by row, skipping the
// centre: (dr, dc) = (-1,-1), (-1,0), (-1,1), (0,-1), (0,1), (1,-1), (1,0), (1,1).
__device__ __forceinline__ void slot_dir(int e, int& dr, int& dc) {
    const int idx = e < 4 ? e : e + 1;
    dr = idx / 3 - 1;
    dc = idx - (idx / 3) * 3 - 1;
}

// Eq. 1: slope angle in degrees from neighbour i = (r + dr, c + dc) up to
// the receiving cell j (uphill spread is positive).
__device__ __forceinline__ float slope_deg(const DevScen& J, float Ej, float Ei, int dr, int dc) {
    const bool diag = (dr != 0) && (dc != 0);
    return atanf((Ej - Ei) * (diag ? J.inv_l_diag : J.inv_l)) * kRad2Deg;
}

// Per-edge terms of Eq. 2-5 for the edge from neighbour slot (dr, dc) into the
// receiving cell j.  rec = (F, V, V cos, V sin) of j, th = the Eq. 1 slope.
// The spread direction i -> j has east component -dc and north component
// +dr, so the projection of the wind on it is (-dc * Vc + dr * Vs) / |(dr, dc)|.
struct Edge {
    float q, ez, x, th, vterm;
};

// e^z as 2^(z log2 e) on the hardware exponential: relative error about
// |z| 2^-24 (the rounding of the product) plus one ulp, at a quarter of the
// library expf's instructions.  The per-edge tables and the adjoints use it
// alike, so the adjoints see the bits the tables were built from.
__device__ __forceinline__ float exp_hw(float z) { return __builtin_amdgcn_exp2f(z * kLog2e); }

// tanh, branch-free and odd: the Taylor series to y^9 below |y| = 0.25
// (truncation below 1e-8 relative), else 1 - 2 / (e^(2|y|) + 1) with the
// hardware reciprocal (relative error below 1e-6 there, where tanh > 0.24).
__device__ __forceinline__ float tanh_fast(float y) {
    const float a = fabsf(y), s = a * a;
    const float p = a * fmaf(s, fmaf(s, fmaf(s, fmaf(s, 62.f / 2835.f, -17.f / 315.f),
                                                2.f / 15.f), -1.f / 3.f), 1.f);
    const float e = exp_hw(2.f * a);
    const float r = fmaf(-2.f, __builtin_amdgcn_rcpf(e + 1.f), 1.f);
    return copysignf(a < 0.25f ? p : r, y);
}

__device__ __forceinline__ Edge edge_terms(const DevScen& J, float4 rec, float th, int dr,
                                           int dc) {
    const bool diag = (dr != 0) && (dc != 0);
    Edge e;
    e.th = th;
    float proj = (float)(-dc) * rec.z + (float)dr * rec.w;
    if (diag) proj = proj * kSqrtHalf;
    e.vterm = proj - rec.y;                               // V (cos(delta) - 1)
    const float z = J.c1 * rec.y + J.c2 * e.vterm + J.a * e.th;   // Eq. 3, 4 exponents
    e.ez = exp_hw(z);
    e.x = (J.p_h * rec.x) * e.ez;                         // Eq. 2
    e.q = tanh_fast(J.c * e.x);                           // Eq. 5
    return e;
}

// Eq. 9 for two disjoint sets of edges: 1 - (1 - a)(1 - b), written without
// cancellation.  por(a, 0) == a and por(0, b) == b exactly, so slots without a
// burning neighbour (q = 0) are neutral.
__device__ __forceinline__ float por(float a, float b) { return a + b * (1.f - a); }

// Eq. 9 over the 8 neighbour slots with a fixed pairing tree
// ((0,1),(2,3)),((4,5),(6,7)).  Every kernel that evaluates p_ignite uses this
// tree, so all of them produce bit-identical values.
__device__ __forceinline__ float combine8(const float q[8]) {
    return por(por(por(q[0], q[1]), por(q[2], q[3])), por(por(q[4], q[5]), por(q[6], q[7])));
}

// p_ignite of cell j from its 8 slots, one lane; nb(dr, dc) says whether that
// neighbour burns.
template <class NB>
__device__ __forceinline__ float cell_pignite(const DevScen& J, int64_t j, NB nb) {
    const float4 rec = J.rec[j];
    float q[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int dr, dc;
        slot_dir(e, dr, dc);
        q[e] = 0.f;
        if (nb(dr, dc)) q[e] = edge_terms(J, rec, J.th8[j * 8 + e], dr, dc).q;
    }
    return combine8(q);
}

// Step-ring attach test (Sec. 2.3, "update by step rings").
__device__ __forceinline__ bool attached(const Rings& rg, int t) {
    if (rg.first < 0) return true;
    if (t <= rg.first || t > rg.T - rg.last) return true;
    const int span = rg.T - rg.first - rg.last;
    for (int k = 1; k <= rg.between; ++k)
        if (t == rg.first + (int)(((long long)k * span + (rg.between + 1) / 2) / (rg.between + 1)))
            return true;
    return false;
}

// Value of lane - 1 / lane + 1 of the wavefront (0 at lane 0 / lane 63), by
// DPP whole-wavefront shifts.
__device__ __forceinline__ uint32_t lane_prev(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, true);  // wave_shr:1
}
__device__ __forceinline__ uint32_t lane_next(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, true);  // wave_shl:1
}

// Inclusive prefix sum over the 64 lanes of a wavefront with DPP lane moves
// (shifts inside 16-lane rows, then the row-15 and row-31 broadcasts), so the
// scan costs six register-to-register moves instead of LDS permutes.  Every
// lane of the wavefront must be active.
__device__ __forceinline__ int wave_incl_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// d p_ignite / d(p_h, a, c1, c2) of cell j: sm has bit m set for each burning
// neighbour slot, q[m] its Eq. 5 value (0 for other slots, as gathered from
// q8).  With dP/dq_m = prod over the other slots of (1 - q) (prefix x suffix
// products), dq/dx = c (1 - q^2), dx/dp_h = F e^z, x = p_h F e^z and
// dx/d(a, c1, c2) = x (theta_s, V, V (cos - 1)).  One exponential per burning
// slot; tanh is not re-evaluated (q comes from the table).  Both adjoints call
// this routine, so they agree cell by cell.
// The table rows of cell j (rec and th8 entries) are passed in, so that a
// caller can issue their reads early.
struct EdgeParams {
    float p_h, a, c1, c2, c;
};

__device__ __forceinline__ void pignite_grad_tab(const EdgeParams& J, float4 rec, fs_f4 ta,
                                                 fs_f4 tb, uint32_t sm, const float q[8],
                                                 float gl[4]) {
    const float th[8] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
    float pre[8], suf[8], acc = 1.f;
#pragma unroll
    for (int m = 0; m < 8; ++m) { pre[m] = acc; acc = acc * (1.f - q[m]); }
    acc = 1.f;
#pragma unroll
    for (int m = 7; m >= 0; --m) { suf[m] = acc; acc = acc * (1.f - q[m]); }
    gl[0] = gl[1] = gl[2] = gl[3] = 0.f;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        if (!((sm >> m) & 1u)) continue;
        int dr, dc;
        slot_dir(m, dr, dc);
        float proj = (float)(-dc) * rec.z + (float)dr * rec.w;
        if (dr != 0 && dc != 0) proj = proj * kSqrtHalf;
        const float vterm = proj - rec.y;
        // F e^z with the operations of edge_terms, so it has the bits the
        // table pass used for q
        const float gv = rec.x * exp_hw(J.c1 * rec.y + J.c2 * vterm + J.a * th[m]);
        const float x = J.p_h * gv;
        const float sc = pre[m] * suf[m] * (J.c * (1.f - q[m] * q[m]));
        gl[0] = gl[0] + sc * gv;
        gl[1] = gl[1] + sc * (x * th[m]);
        gl[2] = gl[2] + sc * (x * rec.y);
        gl[3] = gl[3] + sc * (x * vterm);
    }
}

template <int NWAVE>
__device__ __forceinline__ int block_exscan(int v, int* sWave, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = wave_incl_scan(v);
    if (lane == 63) sWave[wv] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NWAVE; ++k) {
        const int s = sWave[k];
        if (k < wv) pre += s;
        tot += s;
    }
    *total = tot;
    __syncthreads();
    return pre + x - v;
}

// XCD-aware tile order: consecutive workgroups are dealt round-robin to the 8
// XCDs, so give XCD x a contiguous run of tiles (neighbouring tiles share
// halo rows in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = bid & 7, local = bid >> 3;
    return x * q + min(x, r) + local;
}

}  // namespace

// --------------------------------------------------------------- main step

// Work items of a step launch: every tile (skip modes 0 and 2: all, or those
// whose neighbourhood's flags show fire), the tiles of the previous launch's
// worklist walked by a resident grid (mode 1), or every tile launched and
// tested against that worklist (mode 3: one read decides, before anything
// that depends on the tile's job).  Each is compiled separately.
constexpr int kAllTiles = 0, kWorklist = 1, kAllTilesListed = 2;

// 256-lane shapes serve many busy tiles at once (ensembles, calibration): they
// keep no per-word slot masks in LDS (see SN below), so that more work-groups
// fit a CU, and they aim at a register budget per wavefront: 64 registers (8
// wavefronts per SIMD) for launches over every tile (the adjoint recompute
// among them) with up to 2 words per lane, 72 (7) for those with more, 96 (5)
// for worklist launches, whose longer-lived state would spill below that
// (measured: the tighter targets gain 2-4 % on calibration and the ensemble).
// Where a shape cannot reach its target the compiler settles on the occupancy
// it can reach (its warning is silenced).
template <int TR, int TC, int KM, bool ADJ, int NT, int MODE>
constexpr int step_waves() {
    constexpr int wpt = ((TR + 2 * KM) * (TC + 2) + NT - 1) / NT;
    return NT >= 512 ? 1 : MODE == kWorklist ? 5 : (wpt <= 2 ? 8 : 7);
}
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wpass-failed"
template <int TR, int TC, int KM, bool ADJ, int NT, int MODE>
__global__ void __launch_bounds__(NT)
    __attribute__((amdgpu_waves_per_eu(step_waves<TR, TC, KM, ADJ, NT, MODE>())))
k_step(const DevScen* __restrict__ jobs, const int32_t* __restrict__ tile_job, int32_t ntiles,
       int32_t parity, int32_t t_off, int32_t ksteps, int32_t skip,
       const float* __restrict__ lam, Rings rings, Sched sched,
       unsigned long long* __restrict__ stats) {
    constexpr int RR = TR + 2 * KM, RC = TC + 2, NW = RR * RC;
    constexpr int WPT = (NW + NT - 1) / NT;
    constexpr bool LISTED = MODE == kWorklist;
    constexpr bool WLTEST = MODE == kAllTilesListed;
    constexpr int NWAVE = NT / 64;
    constexpr int LCAP = NW * 32;  // worst case: every cell of the region has a trial
    static_assert(LCAP <= 32768, "entries carry an ignition flag in bit 15");
    static_assert(NW * 32 < 65536, "trial list entries are 16-bit");
    static_assert(KM <= TR && KM <= 32, "halo deeper than a tile");

    // burning plane ping-pong: sB[cur] = S(t-1), sB[cur ^ 1] collects the
    // successful trials of step t, which are exactly the burning cells of S(t).
    // The burned plane of a word lives in its owner thread's registers.
    __shared__ uint32_t sB[2][NW];
    // The list holds LCH entries.  A step with more trials places and takes
    // them in chunks of LCH (a barrier between chunks).  256-lane shapes keep
    // 8 entries per lane, so that their LDS does not limit how many
    // work-groups share a compute unit; 512-lane shapes (one busy work-group
    // per compute unit) and one-step shapes (small regions, whose occupancy
    // the chunk loop's registers would lower) keep the worst case.
    constexpr int LCH = (NT >= 512 || KM == 1 || LCAP < 8 * NT) ? LCAP : 8 * NT;
    constexpr bool CHUNKED = LCH < LCAP;
    __shared__ uint16_t sL[LCH];
    // words holding a trial this step, one segment per wavefront (its lanes'
    // words in lane order): (word index, trial mask, ignition mask, offset of
    // the word's first list entry within the wavefront's trials)
    constexpr int SEG = 64 * WPT;
    __shared__ uint4 sWL[NWAVE * SEG];
    // per word, which of the 8 neighbour slots of each of its 32 cells burn
    // (one mask per slot), written for words with ignition trials by the
    // 512-lane shapes; the others rebuild an ignition trial's masks from the
    // state plane (nine LDS reads instead of two, a third less LDS)
    constexpr bool SN = NT >= 512;
    __shared__ uint4 sN[SN ? NW : 1][2];
    __shared__ int sWave[2 * NWAVE];
    __shared__ int sFlag;
    // all-tile launches find most regions without fire; a worklist's tiles
    // nearly always hold some, so they skip the test
    constexpr bool QUIET = !LISTED;
    __shared__ int sAny[QUIET ? NWAVE : 1];   // per wavefront: a loaded word holds a burning cell

    const int tid = threadIdx.x;

    // ---- work items: every tile (one per work-group), or the tiles the
    // previous launch marked (worklist: a fixed grid walks the set bits).
    // The modes are compiled separately, so that launches over every tile
    // carry none of the worklist walk's registers.
    __shared__ int sItems, sTile;
    constexpr bool listed = LISTED;
    const FS_GLOBAL unsigned long long* sin = gmem(sched.in);
    int my_pre = 0, my_cnt = 0, my_w0 = 0, my_w1 = 0;
    if (listed) {
        const int wpt = (sched.nwords + NT - 1) / NT;
        my_w0 = min(sched.nwords, tid * wpt);
        my_w1 = min(sched.nwords, my_w0 + wpt);
        for (int w = my_w0; w < my_w1; ++w) my_cnt += __popcll(sin[w]);
        int tot;
        my_pre = block_exscan<NWAVE>(my_cnt, sWave, &tot);
        if (tid == 0) sItems = tot;
        for (int w = blockIdx.x * NT + tid; w < sched.nwords; w += gridDim.x * NT)
            gmem(sched.clear)[w] = 0ull;
        __syncthreads();
    } else if (WLTEST) {
        // every tile launched, the worklist consulted: the same hand-over
        for (int w = blockIdx.x * NT + tid; w < sched.nwords; w += gridDim.x * NT)
            gmem(sched.clear)[w] = 0ull;
    }
    const int nitems = listed ? sItems : 1;
    for (int it = listed ? blockIdx.x : 0; it < nitems; it += listed ? gridDim.x : 1) {
    int g;
    if (listed) {
        __syncthreads();   // the previous item's use of LDS is over
        if (it >= my_pre && it < my_pre + my_cnt) {
            int k = it - my_pre;
            for (int w = my_w0; w < my_w1; ++w) {
                unsigned long long m = sin[w];
                const int c = __popcll(m);
                if (k < c) {
                    for (int q = 0; q < k; ++q) m &= m - 1;
                    sTile = w * 64 + (__ffsll((long long)m) - 1);
                    break;
                }
                k -= c;
            }
        }
        __syncthreads();
        g = sTile;
    } else {
        g = xcd_tile(blockIdx.x, gridDim.x);
        if (g >= ntiles) continue;
        // skip mode 3: a tile the previous launch did not list has no fire
        // within reach and two equal buffers; the test reads one word, before
        // anything that depends on the tile's job
        if (WLTEST && !((sin[g >> 6] >> (g & 63)) & 1ull)) continue;
    }
    // (launches over every tile of a single job pass no tile -> job table)
    const DevScen& J = jobs[(!LISTED && !tile_job) ? 0 : tile_job[g]];
    const int lt = g - J.tile0;
    const int trow = lt / J.tiles_c, tcol = lt - trow * J.tiles_c;
    const int H = J.H, pitch = J.pitch;
    const int64_t PW = (int64_t)H * pitch;
    const FS_GLOBAL uint8_t* fin = gmem(J.flags[parity]);
    FS_GLOBAL uint8_t* fout = gmem(J.flags[parity ^ 1]);
    const FS_GLOBAL uint32_t* pin = gmem(J.planes[parity]);
    FS_GLOBAL uint32_t* pout = gmem(J.planes[parity ^ 1]);
    const FS_GLOBAL uint32_t* fuel = gmem(J.fuel);
    const FS_GLOBAL float* q8g = gmem(J.q8);

    // steps of this launch for this job; never more than the halo covers
    const int kj = min(min(ksteps, KM), J.t_end - (J.t_base + t_off));
    if (kj <= 0) continue;

    // ---- skip a tile when no tile within reach holds a burning cell
    bool need = true;
    if (!WLTEST && skip) {
        need = false;
        for (int dr = -1; dr <= 1; ++dr)
            for (int dc = -1; dc <= 1; ++dc) {
                const int rr = trow + dr, cc = tcol + dc;
                if (rr >= 0 && rr < J.tiles_r && cc >= 0 && cc < J.tiles_c &&
                    (fin[rr * J.tiles_c + cc] & 1))
                    need = true;
            }
    }
    if (!need) {
        if (!(fin[lt] & 2)) {  // bring the other buffer up to date once
            for (int w = tid; w < TR * TC; w += NT) {
                const int gr = trow * TR + w / TC, gw = tcol * TC + w % TC;
                if (gr < H && gw < pitch) {
                    const int64_t o = (int64_t)gr * pitch + gw;
                    pout[o] = pin[o];
                    pout[PW + o] = pin[PW + o];
                }
            }
        }
        if (tid == 0) fout[lt] = 2;
        continue;
    }

    // ---- load the tile and a KM-row / 1-word halo into LDS
    const int r0 = trow * TR - KM;
    const int w0 = tcol * TC - 1;
    uint32_t origB[WPT], origD[WPT];
    uint32_t dreg[WPT], bprev[WPT];   // burned plane; burning plane one step back
    uint32_t ureg[WPT];               // fuel plane (constant)
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
        const int w = tid + i * NT;
        origB[i] = origD[i] = 0;
        dreg[i] = bprev[i] = 0;
        ureg[i] = 0;
        if (w < NW) {
            const int lr = w / RC, lc = w - (w / RC) * RC;
            const int gr = r0 + lr, gw = w0 + lc;
            uint32_t b = 0, d = 0, u = 0;
            if (gr >= 0 && gr < H && gw >= 0 && gw < pitch) {
                const int64_t o = (int64_t)gr * pitch + gw;
                b = pin[o];
                d = pin[PW + o];
                u = fuel[o];
            }
            sB[0][w] = b;
            ureg[i] = u;
            origB[i] = b;
            origD[i] = d;
        }
    }
    if (tid == 0) sFlag = 0;
    // whether the other buffer already equals this tile (read early: a tile
    // without fire in its region needs it right after the first barrier)
    const uint8_t fin_lt = QUIET ? fin[lt] : 0;
    bool myb = false;
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
        dreg[i] = origD[i];
        bprev[i] = origB[i];
        myb |= origB[i] != 0u;
    }
    // read after the first step's opening barrier
    bool quiet = false;
    if constexpr (QUIET) {
        const bool wave_b = __ballot(myb) != 0ull;
        if ((tid & 63) == 0) sAny[tid >> 6] = wave_b ? 1 : 0;
    }

    const uint32_t k0s = J.seed_lo, k1s = J.seed_hi, scen = J.scen_id;
    // fields every step reads, held in registers: after each work-group
    // barrier (an acquire fence) the compiler would reload them from memory
    // (the calibration and tie-log pointers, read only on some trials, are
    // left in the descriptor to keep scalar registers free; only whether
    // they are present is kept)
    const int Wg = J.W, t_base = J.t_base;
    const float p_cont = J.p_continue;
    // (adjoint recompute jobs never write the maps or the tie log)
    const bool has_yhat = !ADJ && J.yhat != nullptr, has_tign = !ADJ && J.tign != nullptr,
               has_tout = !ADJ && J.tout != nullptr, has_tlog = !ADJ && J.tielog != nullptr;
    const bool counting = stats != nullptr;   // trial and near-tie counters
    unsigned long long n_trials = 0, n_ties = 0;
    int cur = 0;

    for (int s = 1; s <= kj; ++s) {
        __syncthreads();
        if (QUIET && s == 1) {
            // no burning cell in the region: no trial in any step of this
            // launch (fire moves one cell per step and the halo is KM >= kj
            // deep), so the tile keeps its state
            int a = 0;
#pragma unroll
            for (int v = 0; v < NWAVE; ++v) a |= sAny[v];
            if (__builtin_amdgcn_readfirstlane(a) == 0) {
                quiet = true;
                break;
            }
        }
        const int t = t_base + t_off + s;
        // cells still needed: rows and halo-word bits within kj - s cells of
        // the tile (they are also the ones whose inputs are still valid; trials
        // farther out could not reach the tile before the launch ends)
        const int need_d = kj - s;
        const int lo = KM - need_d, hi = RR - lo;
        const uint32_t keepL = need_d == 0 ? 0u : ~0u << (32 - need_d);
        const uint32_t keepR = (1u << need_d) - 1u;
        const uint32_t* cB = sB[cur];
        uint32_t* nR = sB[cur ^ 1];

        // trial masks of this thread's words: continue trials (burning cells)
        // and ignition trials (burnable cells with fuel and a burning neighbour)
        uint32_t mc[WPT], mi[WPT];
        int cnt = 0;  // trials of this thread's words
        int nne = 0;  // words of this thread with a trial
#pragma unroll
        for (int i = 0; i < WPT; ++i) {
            const int w = tid + i * NT;
            mc[i] = mi[i] = 0;
            if (w < NW) {
                const int lr = w / RC, lc = w - (w / RC) * RC;
                uint32_t up = 0, mid = 0, dn = 0;
                uint32_t upL = 0, midL = 0, dnL = 0, upR = 0, midR = 0, dnR = 0;
                if constexpr (64 % RC == 0) {
                    // rows never straddle a wavefront: the left and right
                    // neighbour words are held by lanes -1 and +1 (every lane
                    // of the row's wavefront reads its words first)
                    if (lr > 0) up = cB[(lr - 1) * RC + lc];
                    mid = cB[lr * RC + lc];
                    if (lr < RR - 1) dn = cB[(lr + 1) * RC + lc];
                    const uint32_t uL = lane_prev(up), mL = lane_prev(mid), dL = lane_prev(dn);
                    const uint32_t uR = lane_next(up), mR = lane_next(mid), dR = lane_next(dn);
                    if (lc > 0) { upL = uL; midL = mL; dnL = dL; }
                    if (lc < RC - 1) { upR = uR; midR = mR; dnR = dR; }
                }
                if (lr >= lo && lr < hi) {
                    // burning-neighbour masks per slot (slot order of slot_dir):
                    // bit b of slot (dr, dc) = cell (lr + dr, 32 lc + b + dc) burns
                    if constexpr (64 % RC != 0) {
                        const int a = (lr - 1) * RC, b = lr * RC, c = (lr + 1) * RC;
                        up = cB[a + lc]; mid = cB[b + lc]; dn = cB[c + lc];
                        if (lc > 0) {
                            upL = cB[a + lc - 1];
                            midL = cB[b + lc - 1];
                            dnL = cB[c + lc - 1];
                        }
                        if (lc < RC - 1) {
                            upR = cB[a + lc + 1];
                            midR = cB[b + lc + 1];
                            dnR = cB[c + lc + 1];
                        }
                    }
                    const uint32_t n0 = (up << 1) | (upL >> 31), n1 = up,
                                   n2 = (up >> 1) | (upR << 31);
                    const uint32_t n3 = (mid << 1) | (midL >> 31), n4 = (mid >> 1) | (midR << 31);
                    const uint32_t n5 = (dn << 1) | (dnL >> 31), n6 = dn,
                                   n7 = (dn >> 1) | (dnR << 31);
                    const uint32_t nbm = n0 | n1 | n2 | n3 | n4 | n5 | n6 | n7;
                    // burned at t-1: burned before, or burning at t-2 and not at t-1
                    dreg[i] |= bprev[i] & ~mid;
                    bprev[i] = mid;
                    const uint32_t keep = lc == 0 ? keepL : (lc == RC - 1 ? keepR : ~0u);
                    mc[i] = mid & keep;
                    mi[i] = nbm & ~mid & ~dreg[i] & ureg[i] & keep;
                    cnt += __popc(mc[i] | mi[i]);
                    nne += (mc[i] | mi[i]) != 0u;
                    nR[w] = 0;
                    if constexpr (SN) {
                        if (mi[i]) {
                            sN[w][0] = make_uint4(n0, n1, n2, n3);
                            sN[w][1] = make_uint4(n4, n5, n6, n7);
                        }
                    }
                }
            }
        }
        // compacted trial list in thread order (the words of a thread in
        // index order), bit 15 of an entry marking an ignition trial (else a
        // continue trial).  Each wavefront lists its busy words in its own
        // segment of sWL before the work-group barrier, with offsets within
        // the wavefront (DPP scans); after the barrier the wavefronts' totals
        // give the work-group prefixes, and 8 lanes per listed word place its
        // set bits, 4 bits each (rank = popcount below the bit), so a busy
        // word costs little more than a quiet one
        // The two counts share one scan: trials in the low 16 bits, busy words
        // in the high 16 (a region has at most 32 768 cells, so neither half
        // overflows, per wavefront or per work-group).
        const int lane = tid & 63, wv = tid >> 6;
        {
            const int packed = cnt | (nne << 16);
            const int xp = wave_incl_scan(packed);
            int oc = (xp & 0xFFFF) - cnt, k = wv * SEG + (xp >> 16) - nne;
#pragma unroll
            for (int i = 0; i < WPT; ++i) {
                const uint32_t mm = mc[i] | mi[i];
                if (mm) {
                    sWL[k] = make_uint4((uint32_t)(tid + i * NT), mm, mi[i], (uint32_t)oc);
                    ++k;
                    oc += __popc(mm);
                }
            }
            if (lane == 63) sWave[wv] = xp;
        }
        __syncthreads();
        // work-group prefixes of the wavefronts' trials (tp) and busy words (bp)
        int tp[NWAVE], bp[NWAVE];
        int acc = 0;
#pragma unroll
        for (int v = 0; v < NWAVE; ++v) {
            tp[v] = acc & 0xFFFF;
            bp[v] = acc >> 16;
            acc += sWave[v];
        }
        const int tot = acc & 0xFFFF, tot_w = acc >> 16;
        // (a scalar: the branches on it below are uniform).  A step without
        // trials has no busy word either; testing both keeps every read of
        // the wavefront totals ahead of the branch (one LDS round trip).
        const int ntr = __builtin_amdgcn_readfirstlane(tot);
        if (ntr == 0 && __builtin_amdgcn_readfirstlane(tot_w) == 0) {
            // no trial within reach of the tile: no cell of the band burns or
            // can ignite, so the band stays as it is for the rest of the launch
            cur ^= 1;
            break;
        }

        for (int c0 = 0;; c0 += LCH) {
        const int cend = CHUNKED ? min(ntr, c0 + LCH) : ntr;
        for (int x = tid; x < tot_w * 8; x += NT) {
            // lane x & 7 of listed word k = x >> 3 places the trials among its
            // bits 4 (x & 7) .. 4 (x & 7) + 3; the word sits in the segment of
            // the last wavefront whose prefix does not exceed k
            const int k = x >> 3;
            int seg = 0, kb = 0, tb = 0;
#pragma unroll
            for (int v = 1; v < NWAVE; ++v) {
                if (k >= bp[v]) {
                    seg = v;
                    kb = bp[v];
                    tb = tp[v];
                }
            }
            const uint4 wl = sWL[seg * SEG + (k - kb)];
            const int b0 = (x & 7) * 4;
            const uint32_t m = (wl.y >> b0) & 15u;
            int pos = tb + (int)wl.w + __popc(wl.y & ((1u << b0) - 1u)) - c0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if ((m >> q) & 1u) {
                    const int b = b0 + q;
                    if (!CHUNKED || (unsigned)pos < (unsigned)LCH)
                        sL[pos] = (uint16_t)((wl.x * 32 + b) | (((wl.z >> b) & 1u) ? 0x8000u : 0u));
                    ++pos;
                }
            }
        }
        __syncthreads();

        {
            // p_ignite of an ignition trial is Eq. 9 over the q8 entries of its
            // burning neighbour slots (the Eq. 2-5 work was done for every edge
            // at the start of the run).  Each lane takes up to R trials per pass
            // and issues all of their gathers before deciding.  The adjoint
            // recompute takes the same decisions from the same values and, for
            // the cells that ignite inside the tile at an attached step,
            // records their burning slots (the gradient pass then adds
            // lambda_j * d p_ignite_j / d theta from them).
            // one trial per lane per pass: a busy tile rarely has more trials
            // than lanes, and fewer registers mean more resident wavefronts
            // (2 and 4 trials per lane measured slower on every workload)
            constexpr int R = 1;
            const bool att = ADJ && attached(rings, t);
            const FS_GLOBAL fs_f4* q8v = (const FS_GLOBAL fs_f4*)q8g;
            // flat index of the region's top-left cell (may be negative; every
            // listed cell lies inside the grid)
            const int64_t jbase = (int64_t)r0 * Wg + (int64_t)w0 * 32;
            for (int k0 = c0; k0 < cend; k0 += R * NT) {
                int ent[R], ign[R];
                fs_f4 qa[R], qb[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (k0 + r * NT >= cend) break;   // uniform: no lane has trial r
                    const int k = k0 + r * NT + tid;
                    ent[r] = k < cend ? (int)sL[k - c0] : 0;
                    ign[r] = (ent[r] >> 15) & 1;
                    ent[r] &= 0x7FFF;
                    qa[r] = qb[r] = (fs_f4)(0.f);
                    if (k < cend && ign[r]) {
                        const int w = ent[r] >> 5, bit = ent[r] & 31;
                        const int lr = w / RC, lc = w - (w / RC) * RC;
                        const int64_t j = jbase + (lr * Wg + lc * 32 + bit);
                        qa[r] = q8v[2 * j];
                        qb[r] = q8v[2 * j + 1];
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (k0 + r * NT >= cend) break;
                    const int k = k0 + r * NT + tid;
                    if (k >= cend) continue;
                    const int w = ent[r] >> 5, bit = ent[r] & 31;
                    const int lr = w / RC, lc = w - (w / RC) * RC;
                    const int64_t j = jbase + (lr * Wg + lc * 32 + bit);
                    const bool interior = lr >= KM && lr < KM + TR && lc >= 1 && lc <= TC;
                    uint32_t rw0, rw1;
                    // counter (cell, 0, step, scenario): a cell index fits 32 bits
                    // (H, W <= 65 536), so the second word is the constant 0 and
                    // the first two rounds each need one vector product only
                    philox_w01((uint32_t)j, 0u, (uint32_t)t, scen, k0s, k1s, rw0, rw1);
                    if (!ign[r]) {  // burning: continue trial
                        if (u24(rw1) < p_cont) {
                            atomicOr(&nR[w], 1u << bit);
                        } else if (interior && has_tout) {
                            gmem(J.tout)[j] = t;
                        }
                        if (counting && interior) ++n_trials;
                        continue;
                    }
                    const float qs[8] = {qa[r].x, qa[r].y, qa[r].z, qa[r].w,
                                         qb[r].x, qb[r].y, qb[r].z, qb[r].w};
                    uint32_t nm[8];
                    if constexpr (SN) {
                        const uint4 na = sN[w][0], nb = sN[w][1];
                        nm[0] = na.x; nm[1] = na.y; nm[2] = na.z; nm[3] = na.w;
                        nm[4] = nb.x; nm[5] = nb.y; nm[6] = nb.z; nm[7] = nb.w;
                    } else {
                        // the same masks as the mask phase, from S(t-1) (a
                        // trial cell lies in rows 1 .. RR-2 of the region)
                        const uint32_t* cB = sB[cur];
                        const int a = (lr - 1) * RC, bq = lr * RC, c = (lr + 1) * RC;
                        const uint32_t up = cB[a + lc], mid = cB[bq + lc], dn = cB[c + lc];
                        uint32_t upL = 0, midL = 0, dnL = 0, upR = 0, midR = 0, dnR = 0;
                        if (lc > 0) {
                            upL = cB[a + lc - 1];
                            midL = cB[bq + lc - 1];
                            dnL = cB[c + lc - 1];
                        }
                        if (lc < RC - 1) {
                            upR = cB[a + lc + 1];
                            midR = cB[bq + lc + 1];
                            dnR = cB[c + lc + 1];
                        }
                        nm[0] = (up << 1) | (upL >> 31);
                        nm[1] = up;
                        nm[2] = (up >> 1) | (upR << 31);
                        nm[3] = (mid << 1) | (midL >> 31);
                        nm[4] = (mid >> 1) | (midR << 31);
                        nm[5] = (dn << 1) | (dnL >> 31);
                        nm[6] = dn;
                        nm[7] = (dn >> 1) | (dnR << 31);
                    }
                    float q[8];
#pragma unroll
                    for (int m = 0; m < 8; ++m) q[m] = ((nm[m] >> bit) & 1u) ? qs[m] : 0.f;
                    const float P = combine8(q);
                    const float u = u24(rw0);
                    if (u < P) {
                        atomicOr(&nR[w], 1u << bit);
                        if (interior && has_yhat) gmem(J.yhat)[j] = P;
                        if (interior && has_tign) gmem(J.tign)[j] = t;
                        if constexpr (ADJ) {
                            if (interior && att) {
                                // the cell's burning slots at t - 1: all the
                                // gradient pass needs of the recomputed state
                                uint32_t sm = 0;
#pragma unroll
                                for (int m = 0; m < 8; ++m) sm |= ((nm[m] >> bit) & 1u) << m;
                                gmem(J.sm8)[j] = (uint8_t)sm;
                            }
                        }
                    }
                    if (interior) {
                        if (counting) {
                            ++n_trials;
                            if (fabsf(u - P) <= kTieEps) ++n_ties;
                        }
                        if (!ADJ && has_tlog && fabsf(u - P) <= kTieLogEps) {
                            const unsigned long long n = atomicAdd(J.tie_n, 1ull);
                            if (n < (unsigned long long)kTieLogCap) {
                                FS_GLOBAL TieRec* tr = gmem(reinterpret_cast<TieRec*>(J.tielog)) + n;
                                tr->scenario = J.sidx;
                                tr->step = t;
                                tr->cell = j;
                                tr->p = P;
                                tr->u = u;
                                tr->ignited = u < P ? 1 : 0;
                                tr->reserved = 0;
                            }
                        }
                    }
                }
            }
        }
        if (!CHUNKED || c0 + LCH >= ntr) break;   // uniform
        __syncthreads();   // the chunk's entries are taken
        // the prefixes again (read here so that they are not held through
        // the trials)
        acc = 0;
#pragma unroll
        for (int v = 0; v < NWAVE; ++v) {
            tp[v] = acc & 0xFFFF;
            bp[v] = acc >> 16;
            acc += sWave[v];
        }
        }  // chunks
        // the next step's opening barrier completes this step's trials
        cur ^= 1;
    }
    __syncthreads();

    if (QUIET && quiet) {
        // as a skipped tile: the other buffer is brought up to date once
        if (!(fin_lt & 2)) {
#pragma unroll
            for (int i = 0; i < WPT; ++i) {
                const int w = tid + i * NT;
                if (w < NW) {
                    const int lr = w / RC, lc = w - (w / RC) * RC;
                    if (lr >= KM && lr < KM + TR && lc >= 1 && lc <= TC) {
                        const int gr = r0 + lr, gw = w0 + lc;
                        if (gr < H && gw < pitch) {
                            const int64_t o = (int64_t)gr * pitch + gw;
                            pout[o] = origB[i];
                            pout[PW + o] = origD[i];
                        }
                    }
                }
            }
        }
        if (tid == 0) {
            fout[lt] = 2;
            if (stats) atomicAdd(&stats[0], 1ull);
        }
        continue;
    }

    // ---- write the tile interior back
    bool anyB = false, changed = false;
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
        const int w = tid + i * NT;
        if (w < NW) {
            const int lr = w / RC, lc = w - (w / RC) * RC;
            if (lr >= KM && lr < KM + TR && lc >= 1 && lc <= TC) {
                const int gr = r0 + lr, gw = w0 + lc;
                if (gr < H && gw < pitch) {
                    const int64_t o = (int64_t)gr * pitch + gw;
                    const uint32_t nb = sB[cur][w], nd = dreg[i] | (bprev[i] & ~nb);
                    pout[o] = nb;
                    pout[PW + o] = nd;
                    anyB |= nb != 0u;
                    changed |= (nb != origB[i]) || (nd != origD[i]);
                }
            }
        }
    }
    if (anyB) atomicOr(&sFlag, 1);
    if (changed) atomicOr(&sFlag, 2);

    __syncthreads();
    if (tid == 0) {
        const int f = sFlag;
        fout[lt] = (uint8_t)(((f & 1) ? 1 : 0) | ((f & 2) ? 0 : 2));
    }
    if (stats) {
        // per-wave reduction of the counters, one atomic per wave
        unsigned long long a = n_trials, b = n_ties;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            a += __shfl_down(a, d, 64);
            b += __shfl_down(b, d, 64);
        }
        if ((tid & 63) == 0) {
            if (a) atomicAdd(&stats[1], a);
            if (b) atomicAdd(&stats[2], b);
        }
        if (tid == 0) atomicAdd(&stats[0], 1ull);
    }
    if ((listed || WLTEST) && tid < 9) {
        // mark the next launch's work: the 3 x 3 tile neighbourhood while the
        // tile burns, the tile alone when it changed (its two buffers differ)
        const int f = sFlag;
        const int dr = tid / 3 - 1, dc = tid - (tid / 3) * 3 - 1;
        const int rr = trow + dr, cc = tcol + dc;
        if (((f & 1) || ((f & 2) && tid == 4)) && rr >= 0 && rr < J.tiles_r && cc >= 0 &&
            cc < J.tiles_c) {
            const int gn = J.tile0 + rr * J.tiles_c + cc;
            atomicOr(&sched.out[gn >> 6], 1ull << (gn & 63));
        }
    }
    }  // work items
}

#pragma clang diagnostic pop

// ------------------------------------------------- per-edge tables (Eq. 1-5)

// th8[j][m] = Eq. 1 slope from neighbour slot m up to cell j (0 where the
// neighbour is outside the grid; such slots never burn), or the matching
// entry of the paper-layout slope tensor slope9[j][dr+1][dc+1].
__global__ void __launch_bounds__(256)
k_slopes(DevScen J, float* __restrict__ th8, const float* __restrict__ slope9,
         int* __restrict__ err) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= J.W) return;
    const int64_t j = (int64_t)r * J.W + c;
    float th[8];
    if (slope9) {
        bool bad = false;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int dr, dc;
            slot_dir(m, dr, dc);
            th[m] = slope9[j * 9 + (dr + 1) * 3 + (dc + 1)];
            bad |= !isfinite(th[m]);
        }
        if (bad) atomicOr(err, 64);
    } else {
        const float Ej = J.elev[j];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int dr, dc;
            slot_dir(m, dr, dc);
            const int rr = r + dr, cc = c + dc;
            th[m] = 0.f;
            if (rr >= 0 && rr < J.H && cc >= 0 && cc < J.W)
                th[m] = slope_deg(J, Ej, J.elev[(int64_t)rr * J.W + cc], dr, dc);
        }
    }
    float4* o = reinterpret_cast<float4*>(th8 + j * 8);
    o[0] = make_float4(th[0], th[1], th[2], th[3]);
    o[1] = make_float4(th[4], th[5], th[6], th[7]);
}

// Bounding box (r0, r1, c0, c1) of the burning cells of every scenario in
// planes[parity] (r1 < r0 when nothing burns): the fire can only reach cells
// within t steps of it t steps later (one Moore neighbour per step).
__global__ void k_bbox_clear(int4* __restrict__ box, int32_t n, uint32_t* __restrict__ qburn,
                             int64_t qwords) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) box[i] = make_int4(INT_MAX, -1, INT_MAX, -1);
    for (int64_t w = i; w < qwords; w += (int64_t)gridDim.x * 256) qburn[w] = 0u;
}

__global__ void __launch_bounds__(256)
k_bbox(const DevScen* __restrict__ jobs, int32_t parity, int4* __restrict__ box) {
    const DevScen& J = jobs[blockIdx.y];
    const int64_t PW = (int64_t)J.H * J.pitch;
    const FS_GLOBAL uint32_t* B = gmem(J.planes[parity]);
    int r0 = INT_MAX, r1 = -1, c0 = INT_MAX, c1 = -1;
    FS_GLOBAL uint32_t* qb = gmem(J.qburn);
    const int nbw = (J.pitch + 31) >> 5;
    auto word = [&](int64_t o, uint32_t w) {
        if (w) {
            const int r = (int)(o / J.pitch), cw = (int)(o - (int64_t)r * J.pitch);
            r0 = min(r0, r);
            r1 = max(r1, r);
            c0 = min(c0, 32 * cw + __builtin_ctz(w));
            c1 = max(c1, 32 * cw + 31 - __builtin_clz(w));
            // block (r / 32, cw): set its bit unless already seen set
            const int64_t bw = (int64_t)(r >> 5) * nbw + (cw >> 5);
            const uint32_t bit = 1u << (cw & 31);
            if (!(qb[bw] & bit)) atomicOr(J.qburn + bw, bit);
        }
    };
    // 4 words (16 bytes) per lane; the plane starts 256-byte aligned
    const int64_t nq = PW >> 2;
    const FS_GLOBAL fs_i4* B4 = gmem(reinterpret_cast<const fs_i4*>(J.planes[parity]));
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * 256) {
        const fs_i4 v = B4[q];
        if ((v.x | v.y | v.z | v.w) != 0) {
            word(4 * q, (uint32_t)v.x);
            word(4 * q + 1, (uint32_t)v.y);
            word(4 * q + 2, (uint32_t)v.z);
            word(4 * q + 3, (uint32_t)v.w);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (int)(PW & 3)) word(4 * nq + threadIdx.x, B[4 * nq + threadIdx.x]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        r0 = min(r0, __shfl_down(r0, d, 64));
        r1 = max(r1, __shfl_down(r1, d, 64));
        c0 = min(c0, __shfl_down(c0, d, 64));
        c1 = max(c1, __shfl_down(c1, d, 64));
    }
    if ((threadIdx.x & 63) == 0 && r1 >= 0) {
        int* b = reinterpret_cast<int*>(box + blockIdx.y);
        atomicMin(&b[0], r0);
        atomicMax(&b[1], r1);
        atomicMin(&b[2], c0);
        atomicMax(&b[3], c1);
    }
}

// Blocks within R blocks (Chebyshev) of a qburn block, in two passes: ROWS
// writes qrow, each bit the OR of the qburn bits R blocks to either side in
// its row; the column pass writes qneed, the OR of the qrow bits R block rows
// above and below.  A cell within `reach` cells of a burning cell lies in a
// block within ceil(reach / 32) blocks of that cell's block.  One thread per
// output word; a grid row (blockIdx.y) per scenario.
template <bool ROWS>
__global__ void __launch_bounds__(256)
k_qdilate(const DevScen* __restrict__ jobs, int32_t R) {
    const DevScen& J = jobs[blockIdx.y];
    const int nbr = (J.H + 31) >> 5, nbw = (J.pitch + 31) >> 5;
    const int64_t words = (int64_t)nbr * nbw;
    const FS_GLOBAL uint32_t* in = gmem(ROWS ? J.qburn : J.qrow);
    FS_GLOBAL uint32_t* out = gmem(ROWS ? J.qrow : J.qneed);
    for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < words;
         o += (int64_t)gridDim.x * 256) {
        const int br = (int)(o / nbw), k = (int)(o - (int64_t)br * nbw);
        uint32_t acc = 0u;
        if constexpr (ROWS) {
            // bits 32 k + s .. 32 k + s + 31 of the row, zero outside it
            const FS_GLOBAL uint32_t* row = in + (int64_t)br * nbw;
            auto at = [&](int w) -> uint32_t { return (w >= 0 && w < nbw) ? row[w] : 0u; };
            for (int s = -R; s <= R; ++s) {
                const int p = 32 * k + s;
                const int w = p >> 5, sh = p & 31;   // (p >> 5 rounds down for p < 0)
                const uint32_t lo = at(w);
                acc |= sh ? (lo >> sh) | (at(w + 1) << (32 - sh)) : lo;
            }
        } else {
            for (int a = max(0, br - R); a <= min(nbr - 1, br + R); ++a)
                acc |= in[(int64_t)a * nbw + k];
        }
        out[o] = acc;
    }
}

// Region of the propagation table for the next steps: the burning box of
// each scenario grown by `reach` cells and clipped to the grid, as (r0, c0,
// width, height) with the prefix sums of the region sizes in cell0q[0..n]
// (one work-group; a thread takes a contiguous run of scenarios).
__global__ void __launch_bounds__(256)
k_qbox(const DevScen* __restrict__ jobs, const int4* __restrict__ box, int32_t n, int32_t reach,
       int4* __restrict__ qbox, int64_t* __restrict__ cell0q) {
    __shared__ long long sPart[256];
    const int per = (n + 255) / 256;
    const int a = min(n, (int)threadIdx.x * per), b = min(n, a + per);
    long long sum = 0;
    for (int i = a; i < b; ++i) {
        const int4 bb = box[i];
        const DevScen& J = jobs[i];
        int4 q = make_int4(0, 0, 0, 0);
        if (bb.y >= bb.x) {
            const int r0 = max(0, bb.x - reach), r1 = min(J.H - 1, bb.y + reach);
            const int c0 = max(0, bb.z - reach), c1 = min(J.W - 1, bb.w + reach);
            q = make_int4(r0, c0, c1 - c0 + 1, r1 - r0 + 1);
        }
        qbox[i] = q;
        sum += (long long)q.z * q.w;
    }
    sPart[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = 0;
        for (int k = 0; k < 256; ++k) {
            const long long v = sPart[k];
            sPart[k] = acc;
            acc += v;
        }
        cell0q[n] = acc;
    }
    __syncthreads();
    long long off = sPart[threadIdx.x];
    for (int i = a; i < b; ++i) {
        cell0q[i] = off;
        const int4 q = qbox[i];
        off += (long long)q.z * q.w;
    }
}

// q8[j][m] = f_p(p_propagate) of the edge from slot m into cell j (Eq. 2-5)
// for every cell of each scenario's table region; one flat index over the
// regions of all scenarios, mapped to scenarios through the prefix sums of
// the region sizes.  A fixed grid walks the 256-cell segments.
__global__ void __launch_bounds__(256)
k_qtable(const DevScen* __restrict__ jobs, const int4* __restrict__ qbox,
         const int64_t* __restrict__ cell0, int32_t n, int32_t masked) {
    // one cell: q8 of its 8 incoming edges
    auto cell = [&](const DevScen& J, int64_t j) {
        const float4 rec = load_f4(J.rec, j);
        const float4 ta = load_f4(J.th8, 2 * j), tb = load_f4(J.th8, 2 * j + 1);
        const float th[8] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
        float q[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int dr, dc;
            slot_dir(m, dr, dc);
            q[m] = edge_terms(J, rec, th[m], dr, dc).q;
        }
        FS_GLOBAL fs_f4* o = (FS_GLOBAL fs_f4*)gmem(J.q8) + 2 * j;
        o[0] = fs_f4{q[0], q[1], q[2], q[3]};
        o[1] = fs_f4{q[4], q[5], q[6], q[7]};
    };
    // region index i of scenario s -> its cell, if that cell's block is one
    // the table covers (a region holds at most 65 536^2 cells, so i fits 32
    // unsigned bits)
    auto at = [&](int s, int64_t i) {
        const int4 q = qbox[s];
        const uint32_t ii = (uint32_t)i, rr = ii / (uint32_t)q.z;
        const int r = q.x + (int)rr, c = q.y + (int)(ii - rr * (uint32_t)q.z);
        const DevScen& J = jobs[s];
        if (masked) {
            const int nbw = (J.pitch + 31) >> 5;
            const uint32_t w = gmem(J.qneed)[(int64_t)(r >> 5) * nbw + (c >> 10)];
            if (!((w >> ((c >> 5) & 31)) & 1u)) return (int64_t)-1;
        }
        return (int64_t)r * J.W + c;
    };
    const int64_t total = cell0[n];
    const int64_t nvb = (total + 255) / 256;
    int lo = 0;   // scenario s with cell0[s] <= g0 < cell0[s + 1]; g0 only grows
    {
        const int64_t g0 = (int64_t)blockIdx.x * 256;
        int hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cell0[mid] <= g0) lo = mid; else hi = mid;
        }
    }
    for (int64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t g0 = vb * 256;
        while (lo < n - 1 && g0 >= cell0[lo + 1]) ++lo;
        const int64_t gi = g0 + threadIdx.x;
        if (g0 + 256 <= cell0[lo + 1]) {
            // the whole segment lies in scenario lo: its descriptor is uniform
            const int su = __builtin_amdgcn_readfirstlane(lo);
            const int64_t j = at(su, gi - cell0[su]);
            if (j >= 0) cell(jobs[su], j);
        } else if (gi < total) {
            int s = lo;   // the segment straddles scenarios
            while (gi >= cell0[s + 1]) ++s;
            const int64_t j = at(s, gi - cell0[s]);
            if (j >= 0) cell(jobs[s], j);
        }
    }
}

// ------------------------------------------------ wind, spotting, metrics

// New wind for one scenario: (V, V cos(theta_w), V sin(theta_w)) of rec.
__global__ void __launch_bounds__(256)
k_set_wind(int32_t H, int32_t W, const float* __restrict__ ws, const float* __restrict__ wd,
           float ws0, float wd0, float4* __restrict__ rec, int* __restrict__ err) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= W) return;
    const int64_t j = (int64_t)r * W + c;
    const float V = ws ? ws[j] : ws0;
    const float th = wd ? wd[j] : wd0;
    if (!(V >= 0.f) || !isfinite(V) || !isfinite(th)) atomicOr(err, 8);
    float sn, cs;
    sincospif(th / 180.f, &sn, &cs);
    float4 v = rec[j];
    v.y = V;
    v.z = V * cs;
    v.w = V * sn;
    rec[j] = v;
}

// Spotting: listed cells become burning (unless burned) in both buffers.
__global__ void __launch_bounds__(256)
k_ignite(DevScen J, const int32_t* __restrict__ cells, int32_t count) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const int64_t j = cells[i];
    if (j < 0 || j >= (int64_t)J.H * J.W) return;
    const int r = (int)(j / J.W), c = (int)(j - (int64_t)r * J.W);
    const int64_t o = (int64_t)r * J.pitch + (c >> 5);
    const int64_t PW = (int64_t)J.H * J.pitch;
    const uint32_t bit = 1u << (c & 31);
    for (int b = 0; b < 2; ++b) {
        uint32_t* p = J.planes[b];
        if (!(p[PW + o] & bit)) atomicOr(&p[o], bit);
    }
}

// Burning / burned counts per job: popcount over the bit-planes.
__global__ void __launch_bounds__(256)
k_counts(const DevScen* __restrict__ jobs, int32_t parity, long long* __restrict__ out) {
    const DevScen& J = jobs[blockIdx.y];
    const int64_t PW = (int64_t)J.H * J.pitch;
    const uint32_t* B = J.planes[parity];
    long long nb = 0, nd = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < PW; i += (int64_t)gridDim.x * 256) {
        nb += __popc(B[i]);
        nd += __popc(B[PW + i]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        nb += __shfl_down(nb, d, 64);
        nd += __shfl_down(nd, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (nb) atomicAdd((unsigned long long*)&out[2 * blockIdx.y], (unsigned long long)nb);
        if (nd) atomicAdd((unsigned long long*)&out[2 * blockIdx.y + 1], (unsigned long long)nd);
    }
}

// |A & B| and |A | B| for affected cells A (burning or burned) and target B.
__global__ void __launch_bounds__(256)
k_overlap(DevScen J, int32_t parity, const uint8_t* __restrict__ target,
          long long* __restrict__ out) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    long long in = 0, un = 0;
    if (c < J.W) {
        const int64_t o = (int64_t)r * J.pitch + (c >> 5);
        const int64_t PW = (int64_t)J.H * J.pitch;
        const uint32_t* B = J.planes[parity];
        const bool a = ((B[o] | B[PW + o]) >> (c & 31)) & 1u;
        const bool b = target[(int64_t)r * J.W + c] != 0;
        in = a && b;
        un = a || b;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        in += __shfl_down(in, d, 64);
        un += __shfl_down(un, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (in) atomicAdd((unsigned long long*)&out[0], (unsigned long long)in);
        if (un) atomicAdd((unsigned long long*)&out[1], (unsigned long long)un);
    }
}

// Eq. 11 and Eq. 12 inputs of every scenario against its observed map, one
// launch: out[4 s .. 4 s + 3] += (|A & B|, |A | B|, |A|, |B|) with A the
// affected cells (burning or burned) of scenario s = blockIdx.y and B the
// non-zero cells of its target (concatenated grids, scenario s at cell0[s]).
__global__ void __launch_bounds__(256)
k_metrics(const DevScen* __restrict__ jobs, const int64_t* __restrict__ cell0,
          int32_t parity, const uint8_t* __restrict__ target, long long* __restrict__ out) {
    const DevScen& J = jobs[blockIdx.y];
    const int64_t HW = (int64_t)J.H * J.W, PW = (int64_t)J.H * J.pitch;
    const uint32_t* B = J.planes[parity];
    const uint8_t* y = target + cell0[blockIdx.y];
    long long in = 0, un = 0, na = 0, nb = 0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < HW;
         j += (int64_t)gridDim.x * 256) {
        const int r = (int)(j / J.W), c = (int)(j - (int64_t)r * J.W);
        const int64_t o = (int64_t)r * J.pitch + (c >> 5);
        const bool a = ((B[o] | B[PW + o]) >> (c & 31)) & 1u;
        const bool b = y[j] != 0;
        in += a && b;
        un += a || b;
        na += a;
        nb += b;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        in += __shfl_down(in, d, 64);
        un += __shfl_down(un, d, 64);
        na += __shfl_down(na, d, 64);
        nb += __shfl_down(nb, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        unsigned long long* o = (unsigned long long*)out + 4 * blockIdx.y;
        if (in) atomicAdd(&o[0], (unsigned long long)in);
        if (un) atomicAdd(&o[1], (unsigned long long)un);
        if (na) atomicAdd(&o[2], (unsigned long long)na);
        if (nb) atomicAdd(&o[3], (unsigned long long)nb);
    }
}

// Probability of arrival over an ensemble of runs (Sec. 1): per cell, the
// number of scenarios s0 .. s0+n-1 (one grid shape) in which the cell is
// affected, added to counts.
__global__ void __launch_bounds__(256)
k_arrival(const DevScen* __restrict__ jobs, int32_t s0, int32_t n, int32_t parity,
          uint32_t* __restrict__ counts) {
    const DevScen& J0 = jobs[s0];
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= J0.W) return;
    const int64_t o = (int64_t)r * J0.pitch + (c >> 5);
    const int64_t PW = (int64_t)J0.H * J0.pitch;
    uint32_t k = 0;
    for (int s = s0; s < s0 + n; ++s) {
        const uint32_t* B = jobs[s].planes[parity];
        k += ((B[o] | B[PW + o]) >> (c & 31)) & 1u;
    }
    counts[(int64_t)r * J0.W + c] += k;
}

// ------------------------------------------------------------- prologue

// One thread per cell of the padded grid (H rows x pitch*32 columns); a
// wavefront covers 64 aligned columns = 2 words and packs them by ballot.
__global__ void __launch_bounds__(256)
k_prologue(int32_t H, int32_t W, int32_t pitch, const float* __restrict__ p_veg,
           const float* __restrict__ p_den, const float* __restrict__ elev,
           const float* __restrict__ ws, const float* __restrict__ wd, float ws0, float wd0,
           const uint8_t* __restrict__ ign, float4* __restrict__ rec,
           uint32_t* __restrict__ fuel, uint32_t* __restrict__ planes,
           float* __restrict__ yhat, int* __restrict__ err) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool has_fuel = false, burning = false;
    if (c < W) {
        const int64_t j = (int64_t)r * W + c;
        const float pv = p_veg[j], pd = p_den[j], e = elev ? elev[j] : 0.f;
        const float V = ws ? ws[j] : ws0;
        const float th = wd ? wd[j] : wd0;
        int bad = 0;
        if (!(pv >= -1.f) || !isfinite(pv)) bad |= 1;
        if (!(pd >= -1.f) || !isfinite(pd)) bad |= 2;
        if (!isfinite(e)) bad |= 4;
        if (!(V >= 0.f) || !isfinite(V)) bad |= 8;
        if (!isfinite(th)) bad |= 16;
        if (bad) atomicOr(err, bad);
        const float F = (1.f + pv) * (1.f + pd);
        float sn, cs;
        sincospif(th / 180.f, &sn, &cs);
        rec[j] = make_float4(F, V, V * cs, V * sn);
        has_fuel = F > 0.f;
        burning = ign[j] != 0;
        if (yhat) yhat[j] = burning ? 1.f : 0.f;
    }
    const unsigned long long mf = __ballot(has_fuel);
    const unsigned long long mb = __ballot(burning);
    const int wbase = (blockIdx.x * 256 + (threadIdx.x & ~63)) >> 5;
    const int64_t PW = (int64_t)H * pitch;
    if (lane == 0 || lane == 32) {
        const int w = wbase + (lane >> 5);
        if (w < pitch) {
            const int64_t o = (int64_t)r * pitch + w;
            const int sh = lane;
            fuel[o] = (uint32_t)(mf >> sh);
            planes[o] = (uint32_t)(mb >> sh);
            planes[PW + o] = 0u;
        }
    }
}

__global__ void __launch_bounds__(256)
k_init_state(const DevScen* __restrict__ jobs, const int32_t* __restrict__ ib0, int32_t n,
             int32_t nblocks) {
    // 4 consecutive 32-cell words per thread (a block covers 1024): both
    // ping-pong buffers get the initial burning plane (packed once at set-up)
    // and an empty burned plane; 16-byte accesses where the burned plane
    // (offset PW words) is 16-byte aligned too
    int lo = 0;   // scenario s with ib0[s] <= b < ib0[s + 1]; b only grows
    {
        int hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ib0[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
        }
    }
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
        while (b >= ib0[lo + 1]) ++lo;
        const DevScen& J = jobs[lo];
        const int64_t PW = (int64_t)J.H * J.pitch;
        const int64_t o = 4 * ((int64_t)(b - ib0[lo]) * 256 + threadIdx.x);
        FS_GLOBAL uint32_t* p0 = gmem(J.planes[0]);
        FS_GLOBAL uint32_t* p1 = gmem(J.planes[1]);
        if ((PW & 3) == 0 && o < PW) {
            const fs_i4 w = *reinterpret_cast<const FS_GLOBAL fs_i4*>(gmem(J.init) + o);
            const fs_i4 z = {0, 0, 0, 0};
            *reinterpret_cast<FS_GLOBAL fs_i4*>(p0 + o) = w;
            *reinterpret_cast<FS_GLOBAL fs_i4*>(p1 + o) = w;
            *reinterpret_cast<FS_GLOBAL fs_i4*>(p0 + PW + o) = z;
            *reinterpret_cast<FS_GLOBAL fs_i4*>(p1 + PW + o) = z;
        } else {
            for (int64_t e = o; e < min(o + 4, PW); ++e) {
                const uint32_t w = gmem(J.init)[e];
                p0[e] = w;
                p1[e] = w;
                p0[PW + e] = 0u;
                p1[PW + e] = 0u;
            }
        }
    }
}

// Calibration maps at a reset: accumulator 1 on the initial burning cells (a
// constant) and 0 elsewhere, ignition step 0 or never, burn-out step never.
// One grid row per scenario (blockIdx.y).  A thread writes 4 consecutive
// cells with 16-byte stores (the maps of a scenario start 256-byte aligned);
// block 0 writes the last cells of a grid whose size is not a multiple of 4.
__global__ void __launch_bounds__(256)
k_init_maps(const DevScen* __restrict__ jobs) {
    const DevScen& J = jobs[blockIdx.y];
    const int W = J.W, pitch = J.pitch;
    const int64_t cells = (int64_t)J.H * W, nq = cells >> 2;
    const FS_GLOBAL uint32_t* init = gmem(J.init);
    auto burning = [&](int r, int c) -> bool {
        return (init[(int64_t)r * pitch + (c >> 5)] >> (c & 31)) & 1u;
    };
    FS_GLOBAL fs_f4* yh = gmem(reinterpret_cast<fs_f4*>(J.yhat));
    FS_GLOBAL fs_i4* tg = gmem(reinterpret_cast<fs_i4*>(J.tign));
    FS_GLOBAL fs_i4* to = gmem(reinterpret_cast<fs_i4*>(J.tout));
    // (row, column) of the quad's first cell, advanced by the stride without
    // a division per quad
    const int64_t q_first = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t step = 4 * (int64_t)gridDim.x * 256;
    const int dR = (int)(step / W), dC = (int)(step - (int64_t)dR * W);
    int qr = (int)((4 * q_first) / W), qc = (int)(4 * q_first - (int64_t)qr * W);
    for (int64_t q = q_first; q < nq; q += step / 4) {
        int r = qr, c = qc;
        qc += dC;
        qr += dR;
        if (qc >= W) {
            qc -= W;
            ++qr;
        }
        float y[4];
        int t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool b = burning(r, c);
            y[e] = b ? 1.f : 0.f;
            t[e] = b ? 0 : INT_MAX;
            if (++c == W) {
                c = 0;
                ++r;
            }
        }
        yh[q] = fs_f4{y[0], y[1], y[2], y[3]};
        tg[q] = fs_i4{t[0], t[1], t[2], t[3]};
        to[q] = fs_i4{INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    }
    if (blockIdx.x == 0 && threadIdx.x < (int)(cells & 3)) {
        const int64_t j = 4 * nq + threadIdx.x;
        const int r = (int)(j / W), c = (int)(j - (int64_t)r * W);
        const bool b = burning(r, c);
        gmem(J.yhat)[j] = b ? 1.f : 0.f;
        gmem(J.tign)[j] = b ? 0 : INT_MAX;
        gmem(J.tout)[j] = INT_MAX;
    }
}

// Gradient pass of both adjoints: for every cell j that ignited at an
// attached step, lambda_j * d p_ignite_j / d theta with the burning
// neighbours of j at its ignition step held constant (Eq. 2-5 and 9
// differentiated).  FROM_MAPS (time-map adjoint): j ignited at t_j >= 1 and
// neighbour i burned at t_j - 1 iff tign_i <= t_j - 1 < tout_i.  Otherwise
// (checkpoint adjoint) the recompute recorded the burning slots of each such
// cell in sm8 (0: no ignition at an attached step).
// A segment of 1024 cells lies in one scenario; gpart[segment] receives its
// FP64 sum in a fixed order.  A lane first tests 4 consecutive cells; the
// cells that ignited at an attached step are listed in cell order (a scan),
// and the lanes then take the list, so that the reads and the arithmetic of
// the gradient run on dense wavefronts.  Both adjoints list the same cells
// (an ignition needs a burning neighbour, and calibration handles take no
// ignitions or states from outside), so they add the same terms in the same
// order.
template <bool FROM_MAPS>
__global__ void __launch_bounds__(256)
k_adjoint_cells(const DevScen* __restrict__ jobs, const int32_t* __restrict__ bl0, int32_t n,
                const float* __restrict__ lam, Rings rings, double* __restrict__ gpart,
                int32_t nblocks) {
    __shared__ double sh[4][4];   // per wavefront, per parameter
    __shared__ int sWave[4];
    __shared__ uint16_t sOff[1024];   // listed cells: offset in the segment
    __shared__ uint32_t sVal[1024];   // and t_j (FROM_MAPS) or the burning slots
    // a fixed grid walks the nblocks segments of 1024 cells; each segment's
    // partial sums go to its own slot, and every sum runs in a fixed order
    int lo = 0;   // scenario s with bl0[s] <= b < bl0[s + 1]; b only grows
    {
        int hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bl0[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
        }
    }
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
    while (b >= bl0[lo + 1]) ++lo;
    const DevScen& J = jobs[lo];
    const int64_t cells = (int64_t)J.H * J.W;
    const int64_t j0 = (int64_t)(b - bl0[lo]) * 1024;
    const int64_t jq = j0 + 4 * threadIdx.x;   // this lane's 4 cells
    uint32_t v[4];   // per cell: t_j or its burning slots; 0 = not listed
    if constexpr (FROM_MAPS) {
        int t[4] = {0, 0, 0, 0};
        if (jq + 4 <= cells) {   // a scenario's maps start 256-byte aligned
            const fs_i4 x = *reinterpret_cast<const FS_GLOBAL fs_i4*>(gmem(J.tign) + jq);
            t[0] = x.x; t[1] = x.y; t[2] = x.z; t[3] = x.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (jq + e < cells) t[e] = gmem(J.tign)[jq + e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            v[e] = (t[e] >= 1 && t[e] <= rings.T && attached(rings, t[e])) ? (uint32_t)t[e] : 0u;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = jq + e < cells ? (uint32_t)gmem(J.sm8)[jq + e] : 0u;
    }
    int tot;
    int pos = block_exscan<4>((v[0] != 0u) + (v[1] != 0u) + (v[2] != 0u) + (v[3] != 0u), sWave,
                              &tot);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (v[e]) {
            sOff[pos] = (uint16_t)(4 * threadIdx.x + e);
            sVal[pos] = v[e];
            ++pos;
        }
    }
    if (__builtin_amdgcn_readfirstlane(tot) == 0) {   // uniform: nothing listed
        if (threadIdx.x < 4) gpart[(int64_t)b * 4 + threadIdx.x] = 0.0;
        continue;
    }
    __syncthreads();
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < tot; k += 256) {
        const int64_t j = j0 + sOff[k];
        const uint32_t val = sVal[k];
        uint32_t sm;
        if constexpr (FROM_MAPS) {
            // burning neighbours at t_j - 1: ignited by then and not yet out
            // (a grid holds at most 2^32 cells, so j fits 32 unsigned bits)
            const int tj1 = (int)val - 1;
            const uint32_t ju = (uint32_t)j, W = (uint32_t)J.W;
            const int r = (int)(ju / W), c = (int)(ju - (uint32_t)r * W);
            // (all 16 reads issued at once: a neighbour outside the grid
            // reads cell j and is masked out)
            const FS_GLOBAL int32_t* tg = gmem(J.tign);
            const FS_GLOBAL int32_t* to = gmem(J.tout);
            int ti[8], tu[8];
            bool in[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                int dr, dc;
                slot_dir(m, dr, dc);
                const int rr = r + dr, cc = c + dc;
                in[m] = rr >= 0 && rr < J.H && cc >= 0 && cc < J.W;
                const int64_t i = in[m] ? (int64_t)rr * J.W + cc : j;
                ti[m] = tg[i];
                tu[m] = to[i];
            }
            sm = 0u;
#pragma unroll
            for (int m = 0; m < 8; ++m)
                sm |= (uint32_t)(in[m] & (ti[m] <= tj1) & (tj1 < tu[m])) << m;
        } else {
            sm = val;
        }
        const float4 qa = load_f4(J.q8, 2 * j), qb = load_f4(J.q8, 2 * j + 1);
        const FS_GLOBAL fs_f4* t8v = (const FS_GLOBAL fs_f4*)gmem(J.th8);
        const fs_f4 ta = t8v[2 * j], tb = t8v[2 * j + 1];
        const float4 rec = load_f4(J.rec, j);
        const float lj = gmem(lam)[J.lam_off + j];
        // (keeps the compiler from moving the lambda read down to its use,
        // which would add a round trip after the arithmetic)
        asm volatile("" ::: "memory");
        const float qv[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
        float q[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) q[m] = ((sm >> m) & 1u) ? qv[m] : 0.f;
        float gl[4];
        pignite_grad_tab(EdgeParams{J.p_h, J.a, J.c1, J.c2, J.c}, rec, ta, tb, sm, q, gl);
#pragma unroll
        for (int m = 0; m < 4; ++m) g[m] += (double)(lj * gl[m]);
    }
    // wavefront sums by shuffles, then the 4 wavefronts in order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double x = g[m];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_down(x, d, 64);
        if (lane == 0) sh[wv][m] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4)
        gpart[(int64_t)b * 4 + threadIdx.x] =
            ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
    __syncthreads();   // sh and the list are reused by the next segment
    }
}

__global__ void __launch_bounds__(256)
k_set_state(int32_t H, int32_t W, int32_t pitch, const uint8_t* __restrict__ in,
            uint32_t* __restrict__ planes, uint32_t* __restrict__ planes2, int* __restrict__ err) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t HW = (int64_t)H * W;
    bool b = false, d = false;
    if (c < W) {
        const int64_t j = (int64_t)r * W + c;
        b = in[j] != 0;
        d = in[HW + j] != 0;
        if (b && d) atomicOr(err, 32);
    }
    const unsigned long long mb = __ballot(b);
    const unsigned long long md = __ballot(d);
    const int wbase = (blockIdx.x * 256 + (threadIdx.x & ~63)) >> 5;
    const int64_t PW = (int64_t)H * pitch;
    if (lane == 0 || lane == 32) {
        const int w = wbase + (lane >> 5);
        if (w < pitch) {
            const int64_t o = (int64_t)r * pitch + w;
            planes[o] = planes2[o] = (uint32_t)(mb >> lane);
            planes[PW + o] = planes2[PW + o] = (uint32_t)(md >> lane);
        }
    }
}

__global__ void __launch_bounds__(256)
k_get_state(int32_t H, int32_t W, int32_t pitch, const uint32_t* __restrict__ planes,
            uint8_t* __restrict__ out) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= W) return;
    const int64_t PW = (int64_t)H * pitch;
    const int64_t o = (int64_t)r * pitch + (c >> 5);
    const int64_t j = (int64_t)r * W + c;
    out[j] = (uint8_t)((planes[o] >> (c & 31)) & 1u);
    out[(int64_t)H * W + j] = (uint8_t)((planes[PW + o] >> (c & 31)) & 1u);
}

// One wavefront per tile: OR of the burning bit-plane over the tile.
__global__ void __launch_bounds__(256)
k_flags_init(const DevScen* __restrict__ jobs, const int32_t* __restrict__ tile_job,
             int32_t ntiles, int32_t parity, int32_t TR, int32_t TC) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= ntiles) return;
    const DevScen& J = jobs[tile_job[g]];
    const int lt = g - J.tile0;
    const int trow = lt / J.tiles_c, tcol = lt - trow * J.tiles_c;
    const uint32_t* p = J.planes[parity];
    bool any = false;
    for (int w = lane; w < TR * TC; w += 64) {
        const int r = trow * TR + w / TC, c = tcol * TC + w % TC;
        if (r < J.H && c < J.pitch) any |= p[(int64_t)r * J.pitch + c] != 0u;
    }
    any = __ballot(any) != 0ull;
    if (lane == 0) J.flags[parity][lt] = any ? 1 : 0;   // other buffer not known to match
}

__global__ void __launch_bounds__(256)
k_pignite(const DevScen* __restrict__ job, int32_t parity, float* __restrict__ out) {
    const DevScen& J = *job;
    const int r = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= J.W) return;
    const int64_t j = (int64_t)r * J.W + c;
    const int pitch = J.pitch;
    const uint32_t* B = J.planes[parity];
    const uint32_t* D = B + (int64_t)J.H * pitch;
    auto bit = [&](const uint32_t* p, int rr, int cc) -> bool {
        if (rr < 0 || rr >= J.H || cc < 0 || cc >= J.W) return false;
        return (p[(int64_t)rr * pitch + (cc >> 5)] >> (cc & 31)) & 1u;
    };
    float P = 0.f;
    const bool fuel = (J.fuel[(int64_t)r * pitch + (c >> 5)] >> (c & 31)) & 1u;
    if (fuel && !bit(B, r, c) && !bit(D, r, c)) {
        auto nb = [&](int dr, int dc) -> bool { return bit(B, r + dr, c + dc); };
        P = cell_pignite(J, j, nb);
    }
    out[j] = P;
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// Deterministic per-scenario sum of the per-block partials of the adjoint's
// gradient pass (ranges: the scenarios' block ranges): one work-group per
// scenario, fixed lane striding and a fixed tree.
__global__ void __launch_bounds__(256)
k_grad_reduce(const double* __restrict__ gpart, const int32_t* __restrict__ ranges,
              double* __restrict__ grad) {
    const int s = blockIdx.x;
    const int a = ranges[s], b = ranges[s + 1];
    __shared__ double sh[256 * 4];
    double v[4] = {0, 0, 0, 0};
    for (int g = a + threadIdx.x; g < b; g += 256)
        for (int m = 0; m < 4; ++m) v[m] += gpart[(int64_t)g * 4 + m];
    for (int m = 0; m < 4; ++m) sh[threadIdx.x * 4 + m] = v[m];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d)
            for (int m = 0; m < 4; ++m) sh[threadIdx.x * 4 + m] += sh[(threadIdx.x + d) * 4 + m];
        __syncthreads();
    }
    if (threadIdx.x < 4) grad[s * 4 + threadIdx.x] = sh[threadIdx.x];
}

// --------------------------------------------------------------- Eq. 10

// The loss kernels cover every scenario of a handle in one launch each:
// scenario i = blockIdx.y (blockIdx.x for k_loss_final) reads its accumulator
// from its descriptor and its target / writes its lambda at offset cell0[i] of
// the concatenated arrays; box holds 4 ints and part 2 * maxparts doubles per
// scenario.

// Bounding box of (yhat != 0) | (y != 0): box = {rmin, rmax, cmin, cmax}.  In
// a calibration handle the accumulator is non-zero exactly on the cells that
// burn or burned (1 on the initial burning cells, p_ignite > 0 at an
// ignition, and no outside states or ignitions), so the box reads the 2-bit
// state planes instead of the FP32 accumulator.  A block strides over its
// scenario, reduces its own box in LDS and merges it with four atomics, so
// the atomics do not contend per cell.  Rows of a multiple of 4 cells with a
// 4-byte aligned target are read 4 cells at a time (one 4-byte target load
// and the plane words holding the quad), other grids cell by cell.
__global__ void __launch_bounds__(256)
k_loss_box(const DevScen* __restrict__ jobs, const int64_t* __restrict__ cell0,
           const uint8_t* __restrict__ y_all, int32_t parity, int* __restrict__ box_all) {
    const DevScen& J = jobs[blockIdx.y];
    const uint8_t* y = y_all + cell0[blockIdx.y];
    const int W = J.W, pitch = J.pitch;
    const FS_GLOBAL uint32_t* burning = gmem(J.planes[parity]);
    const FS_GLOBAL uint32_t* burned = burning + (int64_t)J.H * pitch;
    int v[4] = {INT_MAX, -1, INT_MAX, -1};
    auto hit = [&](int r, int c) {
        v[0] = min(v[0], r);
        v[1] = max(v[1], r);
        v[2] = min(v[2], c);
        v[3] = max(v[3], c);
    };
    if ((W & 3) == 0 && ((uintptr_t)y & 3u) == 0) {
        const int64_t nq = (int64_t)J.H * W / 4;
        const FS_GLOBAL uint32_t* t4 = gmem(reinterpret_cast<const uint32_t*>(y));
        const int64_t q_first = (int64_t)blockIdx.x * 256 + threadIdx.x;
        const int64_t step = 4 * (int64_t)gridDim.x * 256;
        const int dR = (int)(step / W), dC = (int)(step - (int64_t)dR * W);
        int r = (int)((4 * q_first) / W), c = (int)(4 * q_first - (int64_t)r * W);
        for (int64_t q = q_first; q < nq; q += step / 4) {
            // the quad's 4 cells lie in one plane word (c is a multiple of 4)
            const int64_t o = (int64_t)r * pitch + (c >> 5);
            const uint32_t b = t4[q];
            const uint32_t st = ((burning[o] | burned[o]) >> (c & 31)) & 0xFu;
            // the quad's cells that count, one bit each: one update of the row
            // bounds, the columns from the first and last such cell
            const uint32_t nz = st | ((b & 0xFFu) ? 1u : 0u) | ((b & 0xFF00u) ? 2u : 0u) |
                                ((b & 0xFF0000u) ? 4u : 0u) | ((b & 0xFF000000u) ? 8u : 0u);
            if (nz) {
                v[0] = min(v[0], r);
                v[1] = max(v[1], r);
                v[2] = min(v[2], c + __builtin_ctz(nz));
                v[3] = max(v[3], c + 31 - __builtin_clz(nz));
            }
            c += dC;   // the next quad of this thread (a row holds a multiple of 4 cells)
            r += dR;
            if (c >= W) {
                c -= W;
                ++r;
            }
        }
    } else {
        for (int r = blockIdx.x; r < J.H; r += gridDim.x)
            for (int c = threadIdx.x; c < W; c += 256) {
                const int64_t o = (int64_t)r * pitch + (c >> 5);
                const bool st = (((burning[o] | burned[o]) >> (c & 31)) & 1u) != 0;
                if (st || y[(int64_t)r * W + c] != 0) hit(r, c);
            }
    }
    __shared__ int sh[4][256];
    for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] = v[m];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) {
            sh[0][threadIdx.x] = min(sh[0][threadIdx.x], sh[0][threadIdx.x + d]);
            sh[1][threadIdx.x] = max(sh[1][threadIdx.x], sh[1][threadIdx.x + d]);
            sh[2][threadIdx.x] = min(sh[2][threadIdx.x], sh[2][threadIdx.x + d]);
            sh[3][threadIdx.x] = max(sh[3][threadIdx.x], sh[3][threadIdx.x + d]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && sh[1][0] >= 0) {
        int* box = box_all + 4 * blockIdx.y;
        atomicMin(&box[0], sh[0][0]);
        atomicMax(&box[1], sh[1][0]);
        atomicMin(&box[2], sh[2][0]);
        atomicMax(&box[3], sh[3][0]);
    }
}

// BCE-with-logits over the crop (kind 0/1) and/or the 4x4 pool MSE (kind
// 1/2).  Writes lambda = dL/dyhat and per-block FP64 partial sums
// part[block] = (bce_sum, mse_sum); one block per 4 rows (a pool row).
__global__ void __launch_bounds__(256)
k_loss_terms(const DevScen* __restrict__ jobs, const int64_t* __restrict__ cell0,
             const uint8_t* __restrict__ y_all, int32_t kind, const int* __restrict__ box_all,
             float* __restrict__ lam_all, double* __restrict__ part_all, int32_t maxparts) {
    const DevScen& J = jobs[blockIdx.y];
    const int H = J.H, W = J.W;
    const int pr = blockIdx.x;  // rows 4 pr .. 4 pr + 3
    if (4 * pr >= H) return;    // whole block: this scenario has fewer rows
    const float* yhat = J.yhat;
    const uint8_t* y = y_all + cell0[blockIdx.y];
    float* lambda = lam_all + cell0[blockIdx.y];
    const int* box = box_all + 4 * blockIdx.y;
    double* part = part_all + 2 * (int64_t)blockIdx.y * maxparts;
    const int b0 = box[0], b1 = box[1], c0 = box[2], c1 = box[3];
    const bool has_box = b1 >= b0;
    const double N = has_box ? (double)(b1 - b0 + 1) * (double)(c1 - c0 + 1) : 1.0;
    const double invN = 1.0 / N;
    const int Hp = H / 4, Wp = W / 4;
    const double Np = (double)Hp * (double)Wp;
    double bce = 0.0, mse = 0.0;
    const bool use_bce = (kind == 0 || kind == 1) && has_box;
    // BCE with logits per cell in FP32, -(y log s + (1 - y) log(1 - s)) with
    // s = sigmoid(z), written as softplus(z) - y z; its derivative is s - y.
    // e = e^-|z| lies in (0, 1], so log(1 + e) loses nothing to the rounding
    // of 1 + e that matters next to max(z, 0); exponential, logarithm and
    // reciprocal are the hardware ones (a few 1e-7 relative per term, the
    // terms all positive).  The sums over cells are FP64.  Returns the cell's
    // lambda.
    auto cell = [&](int r, int c, float z, float yy) -> float {
        double lam = 0.0;
        if (use_bce && r >= b0 && r <= b1 && c >= c0 && c <= c1) {
            const float e = exp_hw(-fabsf(z));
            const float sp = fmaxf(z, 0.f) + __builtin_amdgcn_logf(1.f + e) * kLn2;
            const float sig = (z >= 0.f ? 1.f : e) * __builtin_amdgcn_rcpf(1.f + e);
            bce += (double)(sp - yy * z);
            lam += (double)(sig - yy) * invN;
        }
        return (float)lam;
    };
    const int r_end = min(H, 4 * pr + 4);
    if ((W & 3) == 0 && ((uintptr_t)y & 3u) == 0 && ((uintptr_t)lambda & 15u) == 0) {
        // 4 cells per thread: 16-byte yhat and lambda, 4-byte target accesses
        const int64_t q0 = (int64_t)pr * W, q1 = (int64_t)r_end * W / 4;
        const FS_GLOBAL fs_f4* y4 = gmem(reinterpret_cast<const fs_f4*>(yhat));
        const FS_GLOBAL uint32_t* t4 = gmem(reinterpret_cast<const uint32_t*>(y));
        FS_GLOBAL fs_f4* l4 = gmem(reinterpret_cast<fs_f4*>(lambda));
        const int dR = 1024 / W, dC = 1024 - dR * W;   // 256 quads on
        int r = 4 * pr + (4 * (int)threadIdx.x) / W, c = (4 * (int)threadIdx.x) % W;
        for (int64_t q = q0 + threadIdx.x; q < q1; q += 256) {
            const fs_f4 a = y4[q];
            const uint32_t b = t4[q];
            fs_f4 o;
            o.x = cell(r, c, a.x, (float)(b & 0xFFu));
            o.y = cell(r, c + 1, a.y, (float)((b >> 8) & 0xFFu));
            o.z = cell(r, c + 2, a.z, (float)((b >> 16) & 0xFFu));
            o.w = cell(r, c + 3, a.w, (float)(b >> 24));
            l4[q] = o;
            c += dC;
            r += dR;
            if (c >= W) {
                c -= W;
                ++r;
            }
        }
    } else {
        for (int r = 4 * pr; r < r_end; ++r)
            for (int c = threadIdx.x; c < W; c += 256) {
                const int64_t j = (int64_t)r * W + c;
                lambda[j] = cell(r, c, yhat[j], (float)y[j]);
            }
    }
    __syncthreads();
    if ((kind == 1 || kind == 2) && pr < Hp) {
        for (int pc = threadIdx.x; pc < Wp; pc += 256) {
            double a = 0.0, b = 0.0;
            for (int dr = 0; dr < 4; ++dr)
                for (int dc = 0; dc < 4; ++dc) {
                    const int64_t j = (int64_t)(4 * pr + dr) * W + 4 * pc + dc;
                    a += (double)yhat[j];
                    b += (double)y[j];
                }
            const double d = a / 16.0 - b / 16.0;
            mse += d * d;
            const float add = (float)(2.0 * d / (16.0 * Np));
            for (int dr = 0; dr < 4; ++dr)
                for (int dc = 0; dc < 4; ++dc) {
                    const int64_t j = (int64_t)(4 * pr + dr) * W + 4 * pc + dc;
                    lambda[j] = lambda[j] + add;
                }
        }
    }
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = bce;
    sh[1][threadIdx.x] = mse;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + d];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * pr] = sh[0][0];
        part[2 * pr + 1] = sh[1][0];
    }
}

__global__ void __launch_bounds__(256)
k_loss_final(const DevScen* __restrict__ jobs, int32_t kind, const int* __restrict__ box_all,
             const double* __restrict__ part_all, int32_t maxparts, double* __restrict__ loss_all) {
    const DevScen& J = jobs[blockIdx.x];
    const int H = J.H, W = J.W;
    const int nparts = (H + 3) / 4;
    const int* box = box_all + 4 * blockIdx.x;
    const double* part = part_all + 2 * (int64_t)blockIdx.x * maxparts;
    double* loss = loss_all + blockIdx.x;
    __shared__ double sh[2][256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + d];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double L = 0.0;
        if ((kind == 0 || kind == 1) && box[1] >= box[0])
            L += sh[0][0] / ((double)(box[1] - box[0] + 1) * (double)(box[3] - box[2] + 1));
        const double Np = (double)(H / 4) * (double)(W / 4);
        if ((kind == 1 || kind == 2) && Np > 0) L += sh[1][0] / Np;
        *loss = L;
    }
}

__global__ void __launch_bounds__(256)
k_box_init(const DevScen* __restrict__ jobs, int32_t n, int* __restrict__ box_all) {
    for (int i = threadIdx.x; i < n; i += 256) {
        box_all[4 * i] = jobs[i].H;
        box_all[4 * i + 1] = -1;
        box_all[4 * i + 2] = jobs[i].W;
        box_all[4 * i + 3] = -1;
    }
}

// ------------------------------------------------- checkpoints, parameters

// Copy of nw 32-bit words from src to d0 (and d1 unless null) by the
// blocks of one grid row: 16 bytes per lane where all pointers are 16-byte
// aligned, the remaining words one by one.
__device__ __forceinline__ void copy_words(uint32_t* d0, uint32_t* d1, const uint32_t* src,
                                           int64_t nw) {
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x, st = (int64_t)gridDim.x * 256;
    int64_t done = 0;
    if ((((uintptr_t)d0 | (uintptr_t)d1 | (uintptr_t)src) & 15u) == 0) {
        const int64_t nq = nw >> 2;
        const FS_GLOBAL fs_i4* s4 = gmem(reinterpret_cast<const fs_i4*>(src));
        FS_GLOBAL fs_i4* a4 = gmem(reinterpret_cast<fs_i4*>(d0));
        FS_GLOBAL fs_i4* b4 = gmem(reinterpret_cast<fs_i4*>(d1));
        for (int64_t i = t0; i < nq; i += st) {
            const fs_i4 v = s4[i];
            a4[i] = v;
            if (d1) b4[i] = v;
        }
        done = nq << 2;
    }
    for (int64_t i = done + t0; i < nw; i += st) {
        const uint32_t v = src[i];
        d0[i] = v;
        if (d1) d1[i] = v;
    }
}

__global__ void __launch_bounds__(256)
k_ckpt_save(const DevScen* __restrict__ jobs, int32_t parity, int32_t slot) {
    const DevScen& J = jobs[blockIdx.y];
    const int64_t nw = 2 * (int64_t)J.H * J.pitch;
    copy_words(J.ckpt + (int64_t)slot * nw, nullptr, J.planes[parity], nw);
}

__global__ void __launch_bounds__(256)
k_ckpt_load(const DevScen* __restrict__ jobs) {
    const DevScen& J = jobs[blockIdx.y];
    copy_words(J.planes[0], J.planes[1], J.ckpt, 2 * (int64_t)J.H * J.pitch);
}

__global__ void __launch_bounds__(256)
k_dup_planes(const DevScen* __restrict__ jobs, int32_t parity) {
    const DevScen& J = jobs[blockIdx.y];
    copy_words(J.planes[parity ^ 1], nullptr, J.planes[parity], 2 * (int64_t)J.H * J.pitch);
}

// Worklist of the first launch: tiles with a burning cell in their 3 x 3
// tile neighbourhood (flags of `parity`).
__global__ void __launch_bounds__(256)
k_mask_init(const DevScen* __restrict__ jobs, const int32_t* __restrict__ tile_job,
            int32_t ntiles, int32_t parity, unsigned long long* __restrict__ mask) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= ntiles) return;
    const DevScen& J = jobs[tile_job[g]];
    const int lt = g - J.tile0;
    const int trow = lt / J.tiles_c, tcol = lt - trow * J.tiles_c;
    bool need = false;
    for (int dr = -1; dr <= 1; ++dr)
        for (int dc = -1; dc <= 1; ++dc) {
            const int rr = trow + dr, cc = tcol + dc;
            if (rr >= 0 && rr < J.tiles_r && cc >= 0 && cc < J.tiles_c &&
                (J.flags[parity][rr * J.tiles_c + cc] & 1))
                need = true;
        }
    if (need) atomicOr(&mask[g >> 6], 1ull << (g & 63));
}

__global__ void k_set_params(DevScen* jobs, ParamBlock pb) {
    const int i = threadIdx.x;
    if (i < pb.count) {
        DevScen& J = jobs[pb.first + i];
        J.p_h = pb.v[i][0];
        J.a = pb.v[i][1];
        J.c1 = pb.v[i][2];
        J.c2 = pb.v[i][3];
        J.p_continue = pb.v[i][4];
    }
}

__global__ void k_set_seeds(DevScen* jobs, SeedBlock sb) {
    const int i = threadIdx.x;
    if (i < sb.count) {
        jobs[sb.first + i].seed_lo = sb.lo[i];
        jobs[sb.first + i].seed_hi = sb.hi[i];
    }
}

// theta (device, n rows of p_h, a, c1, c2): a row whose values are finite with
// p_h >= 0 replaces the scenario's parameters (p_continue is kept); any other
// row leaves them unchanged and is counted in *rejected.
__global__ void k_set_theta(DevScen* jobs, int32_t n, const float* __restrict__ theta,
                            int* __restrict__ rejected) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float p_h = theta[4 * i], a = theta[4 * i + 1], c1 = theta[4 * i + 2],
                c2 = theta[4 * i + 3];
    if (isfinite(p_h) && isfinite(a) && isfinite(c1) && isfinite(c2) && p_h >= 0.f) {
        DevScen& J = jobs[i];
        J.p_h = p_h;
        J.a = a;
        J.c1 = c1;
        J.c2 = c2;
    } else {
        atomicAdd(rejected, 1);
    }
}

// Segment k of the checkpoint adjoint belongs to scenario k / nseg: it takes
// that scenario's parameters and Philox keys (everything else in its
// descriptor is fixed by the run's length and the tiling).
__global__ void k_adj_params(DevScen* adj, int32_t nadj, int32_t nseg,
                             const DevScen* __restrict__ jobs) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nadj) {
        const DevScen& F = jobs[k / nseg];
        DevScen& J = adj[k];
        J.p_h = F.p_h;
        J.a = F.a;
        J.c1 = F.c1;
        J.c2 = F.c2;
        J.p_continue = F.p_continue;
        J.seed_lo = F.seed_lo;
        J.seed_hi = F.seed_hi;
    }
}

// --------------------------------------------------------------- launchers

hipError_t launch_ckpt_save(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                            int32_t slot, int64_t max_words) {
    if (n <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((2 * max_words + 1023) / 1024, 1024);
    hipLaunchKernelGGL(k_ckpt_save, dim3(gx, n), dim3(256), 0, st, d_jobs, parity, slot);
    return hipGetLastError();
}

hipError_t launch_ckpt_load(hipStream_t st, const DevScen* d_jobs, int32_t n, int64_t max_words) {
    if (n <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((2 * max_words + 1023) / 1024, 1024);
    hipLaunchKernelGGL(k_ckpt_load, dim3(gx, n), dim3(256), 0, st, d_jobs);
    return hipGetLastError();
}

hipError_t launch_set_params(hipStream_t st, DevScen* d_jobs, const ParamBlock& pb) {
    hipLaunchKernelGGL(k_set_params, dim3(1), dim3(64), 0, st, d_jobs, pb);
    return hipGetLastError();
}

hipError_t launch_set_seeds(hipStream_t st, DevScen* d_jobs, const SeedBlock& sb) {
    hipLaunchKernelGGL(k_set_seeds, dim3(1), dim3(64), 0, st, d_jobs, sb);
    return hipGetLastError();
}

hipError_t launch_set_theta(hipStream_t st, DevScen* d_jobs, int32_t n, const float* theta,
                            int* rejected) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_theta, dim3((n + 255) / 256), dim3(256), 0, st, d_jobs, n, theta,
                       rejected);
    return hipGetLastError();
}

hipError_t launch_adj_params(hipStream_t st, DevScen* d_adj, int32_t nadj, int32_t nseg,
                             const DevScen* d_jobs) {
    if (nadj <= 0 || nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_params, dim3((nadj + 255) / 256), dim3(256), 0, st, d_adj, nadj,
                       nseg, d_jobs);
    return hipGetLastError();
}

namespace {
inline dim3 cell_grid(int H, int cols) { return dim3((cols + 255) / 256, H); }
}  // namespace

hipError_t launch_prologue(hipStream_t st, const DevScen* /*d_job*/, const DevScen& J,
                           const float* p_veg, const float* p_den, const float* ws,
                           const float* wd, float ws0, float wd0, const uint8_t* ign,
                           float4* rec, uint32_t* fuel, float* yhat, int* d_err) {
    hipLaunchKernelGGL(k_prologue, cell_grid(J.H, J.pitch * 32), dim3(256), 0, st, J.H, J.W,
                       J.pitch, p_veg, p_den, J.elev, ws, wd, ws0, wd0, ign, rec, fuel,
                       J.planes[0], yhat, d_err);
    return hipGetLastError();
}

hipError_t launch_slopes(hipStream_t st, const DevScen& J, float* th8, const float* slope9,
                         int* d_err) {
    hipLaunchKernelGGL(k_slopes, cell_grid(J.H, J.W), dim3(256), 0, st, J, th8, slope9, d_err);
    return hipGetLastError();
}

hipError_t launch_set_wind(hipStream_t st, const DevScen& J, const float* ws, const float* wd,
                           float ws0, float wd0, float4* rec, int* d_err) {
    hipLaunchKernelGGL(k_set_wind, cell_grid(J.H, J.W), dim3(256), 0, st, J.H, J.W, ws, wd, ws0,
                       wd0, rec, d_err);
    return hipGetLastError();
}

hipError_t launch_ignite(hipStream_t st, const DevScen& J, const int32_t* cells, int32_t count) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ignite, dim3((count + 255) / 256), dim3(256), 0, st, J, cells, count);
    return hipGetLastError();
}

hipError_t launch_counts(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                         int64_t max_words, long long* out) {
    hipError_t e = launch_fill_u32(st, reinterpret_cast<uint32_t*>(out), (size_t)n * 4, 0u);
    if (e != hipSuccess || n <= 0) return e;
    const unsigned gx = (unsigned)std::min<int64_t>((max_words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_counts, dim3(gx, n), dim3(256), 0, st, d_jobs, parity, out);
    return hipGetLastError();
}

hipError_t launch_metrics(hipStream_t st, const DevScen* d_jobs, const int64_t* d_cell0, int32_t n,
                          int32_t parity, int64_t max_cells, const uint8_t* target,
                          long long* out) {
    hipError_t e = launch_fill_u32(st, reinterpret_cast<uint32_t*>(out), (size_t)n * 8, 0u);
    if (e != hipSuccess || n <= 0) return e;
    const unsigned gx = (unsigned)std::min<int64_t>((max_cells + 255) / 256, 512);
    hipLaunchKernelGGL(k_metrics, dim3(gx, n), dim3(256), 0, st, d_jobs, d_cell0, parity, target,
                       out);
    return hipGetLastError();
}
hipError_t launch_overlap(hipStream_t st, const DevScen& J, int32_t parity, const uint8_t* target,
                          long long* out) {
    hipError_t e = launch_fill_u32(st, reinterpret_cast<uint32_t*>(out), 4, 0u);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_overlap, cell_grid(J.H, J.W), dim3(256), 0, st, J, parity, target, out);
    return hipGetLastError();
}

hipError_t launch_arrival(hipStream_t st, const DevScen* d_jobs, const DevScen& J0, int32_t s0,
                          int32_t n, int32_t parity, uint32_t* counts) {
    hipLaunchKernelGGL(k_arrival, cell_grid(J0.H, J0.W), dim3(256), 0, st, d_jobs, s0, n, parity,
                       counts);
    return hipGetLastError();
}

hipError_t launch_bbox(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                       int64_t max_words, int4* box, uint32_t* qburn_all, int64_t qwords) {
    if (n <= 0) return hipSuccess;
    const int64_t gc = std::max<int64_t>((n + 255) / 256, std::min<int64_t>((qwords + 255) / 256, 1024));
    hipLaunchKernelGGL(k_bbox_clear, dim3((unsigned)gc), dim3(256), 0, st, box, n, qburn_all,
                       qwords);
    const unsigned gx = (unsigned)std::min<int64_t>((max_words + 1023) / 1024, 64);
    hipLaunchKernelGGL(k_bbox, dim3(gx, n), dim3(256), 0, st, d_jobs, parity, box);
    return hipGetLastError();
}

hipError_t launch_qtable(hipStream_t st, const DevScen* d_jobs, const int4* box, int32_t n,
                         int32_t reach, int64_t max_cells, int64_t max_qwords, int4* qbox,
                         int64_t* cell0q) {
    if (n <= 0) return hipSuccess;
    const int R = (reach + 31) / 32;
    const bool masked = R <= kMaxBlockReach;
    if (masked) {
        const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_qwords + 255) / 256, 64));
        hipLaunchKernelGGL(k_qdilate<true>, dim3(gx, n), dim3(256), 0, st, d_jobs, R);
        hipLaunchKernelGGL(k_qdilate<false>, dim3(gx, n), dim3(256), 0, st, d_jobs, R);
    }
    hipLaunchKernelGGL(k_qbox, dim3(1), dim3(256), 0, st, d_jobs, box, n, reach, qbox, cell0q);
    // the region sizes are known on the device only: a grid that covers the
    // largest possible total walks what is there
    const int64_t nvb = (max_cells + 255) / 256;
    hipLaunchKernelGGL(k_qtable, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(nvb, 8192))),
                       dim3(256), 0, st, d_jobs, qbox, cell0q, n, masked ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_init_state(hipStream_t st, const DevScen* d_jobs, const int32_t* d_ib0,
                             int32_t n, int32_t nblocks, const int64_t* d_cell0,
                             int64_t total_cells, bool maps) {
    if (nblocks > 0)
        hipLaunchKernelGGL(k_init_state, dim3(std::min(nblocks, 16384)), dim3(256), 0, st,
                           d_jobs, d_ib0, n, nblocks);
    if (maps && total_cells > 0 && n > 0) {
        // 4 cells per thread; a grid row per scenario, strided over its cells
        const int64_t per = (total_cells / n + 1023) / 1024;
        hipLaunchKernelGGL(k_init_maps, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(per, 512)),
                                             (unsigned)n), dim3(256), 0, st, d_jobs);
    }
    return hipGetLastError();
}

hipError_t launch_mask_init(hipStream_t st, const DevScen* d_jobs, const int32_t* d_tile_job,
                            int32_t ntiles, int32_t parity, unsigned long long* masks,
                            int32_t nwords) {
    hipError_t e = launch_fill_u32(st, reinterpret_cast<uint32_t*>(masks), (size_t)nwords * 6, 0u);
    if (e != hipSuccess || ntiles <= 0) return e;
    hipLaunchKernelGGL(k_mask_init, dim3((ntiles + 255) / 256), dim3(256), 0, st, d_jobs,
                       d_tile_job, ntiles, parity, masks);
    return hipGetLastError();
}

hipError_t launch_dup_planes(hipStream_t st, const DevScen* d_jobs, int32_t n, int32_t parity,
                             int64_t max_words) {
    if (n <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((2 * max_words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_dup_planes, dim3(gx, n), dim3(256), 0, st, d_jobs, parity);
    return hipGetLastError();
}

hipError_t launch_adjoint_cells(hipStream_t st, const DevScen* d_jobs, const int32_t* d_bl0,
                                int32_t n, int32_t nblocks, const float* lam, Rings rings,
                                double* gpart, bool from_maps) {
    if (nblocks <= 0) return hipSuccess;
    if (from_maps)
        hipLaunchKernelGGL(k_adjoint_cells<true>, dim3(std::min(nblocks, 16384)), dim3(256), 0,
                           st, d_jobs, d_bl0, n, lam, rings, gpart, nblocks);
    else
        hipLaunchKernelGGL(k_adjoint_cells<false>, dim3(std::min(nblocks, 16384)), dim3(256), 0,
                           st, d_jobs, d_bl0, n, lam, rings, gpart, nblocks);
    return hipGetLastError();
}

hipError_t launch_set_state(hipStream_t st, const DevScen& J, const uint8_t* in,
                            uint32_t* planes, int* d_err) {
    uint32_t* other = planes == J.planes[0] ? J.planes[1] : J.planes[0];
    hipLaunchKernelGGL(k_set_state, cell_grid(J.H, J.pitch * 32), dim3(256), 0, st, J.H, J.W,
                       J.pitch, in, planes, other, d_err);
    return hipGetLastError();
}

hipError_t launch_get_state(hipStream_t st, const DevScen& J, const uint32_t* planes,
                            uint8_t* out) {
    hipLaunchKernelGGL(k_get_state, cell_grid(J.H, J.W), dim3(256), 0, st, J.H, J.W, J.pitch,
                       planes, out);
    return hipGetLastError();
}

hipError_t launch_flags_init(hipStream_t st, const DevScen* d_jobs, const int32_t* d_tile_job,
                             int32_t ntiles, int32_t parity, TileShape sh) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flags_init, dim3((ntiles + 3) / 4), dim3(256), 0, st, d_jobs,
                       d_tile_job, ntiles, parity, sh.tr, sh.tc);
    return hipGetLastError();
}

hipError_t launch_pignite(hipStream_t st, const DevScen* d_job, const DevScen& J,
                          int32_t parity, float* out) {
    hipLaunchKernelGGL(k_pignite, cell_grid(J.H, J.W), dim3(256), 0, st, d_job, parity, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, size_t n, uint32_t v) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(hipStream_t st, const double* gpart, const int32_t* d_ranges,
                              int32_t n, double* grad) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_reduce, dim3(n), dim3(256), 0, st, gpart, d_ranges, grad);
    return hipGetLastError();
}

hipError_t launch_loss(hipStream_t st, const DevScen* d_jobs, const int64_t* d_cell0, int32_t n,
                       int32_t max_h, int32_t parity, const uint8_t* y, int32_t kind,
                       float* lambda, int* d_box, double* d_part, double* loss_out) {
    if (n <= 0) return hipSuccess;
    const int maxparts = (max_h + 3) / 4;
    hipLaunchKernelGGL(k_box_init, dim3(1), dim3(256), 0, st, d_jobs, n, d_box);
    hipLaunchKernelGGL(k_loss_box, dim3(128, n), dim3(256), 0, st, d_jobs, d_cell0, y, parity,
                       d_box);
    hipLaunchKernelGGL(k_loss_terms, dim3(maxparts, n), dim3(256), 0, st, d_jobs, d_cell0, y,
                       kind, d_box, lambda, d_part, maxparts);
    hipLaunchKernelGGL(k_loss_final, dim3(n), dim3(256), 0, st, d_jobs, kind, d_box, d_part,
                       maxparts, loss_out);
    return hipGetLastError();
}

// ------------------------------------------------- step shape dispatch table

namespace {
// Work-group size per shape: 256 lanes for tiles of up to 16 rows, 512 for
// 32-row tiles, whose taller regions hold more trials per step (measured on
// the 4096 x 4096 workload: 512 lanes are 5-30 % faster there and 10 %
// slower on 16-row tiles).
constexpr int kThreadsShort = 256;
constexpr int kThreadsTall = 512;
using StepFn = void (*)(const DevScen*, const int32_t*, int32_t, int32_t, int32_t, int32_t,
                        int32_t, const float*, Rings, Sched, unsigned long long*);

struct StepEntry {
    int tr, tc, km, nt;
    bool adj;
    StepFn fn;        // every tile (skip modes 0 and 2)
    StepFn fn_list;   // the tiles of a worklist (skip mode 1)
    StepFn fn_wl;     // every tile, tested against a worklist (skip mode 3)
    int resident;     // work-groups of fn_list resident at once (0: not queried yet)
};

#define FS_SHAPE_NT(TR, TC, KM, NT)                                                      \
    {TR, TC, KM, NT, false, &k_step<TR, TC, KM, false, NT, kAllTiles>,                     \
     &k_step<TR, TC, KM, false, NT, kWorklist>,                                            \
     &k_step<TR, TC, KM, false, NT, kAllTilesListed>, 0},                                  \
    {TR, TC, KM, NT, true, &k_step<TR, TC, KM, true, NT, kAllTiles>,                       \
     &k_step<TR, TC, KM, true, NT, kWorklist>,                                             \
     &k_step<TR, TC, KM, true, NT, kAllTilesListed>, 0},
// 32-row tiles come with both sizes (the default first): 512 lanes shorten
// the per-step latency of a few busy tiles, 256 lanes give more resident
// work-groups when many tiles are busy at once (large ensembles).
#define FS_SHAPE(TR, TC, KM) FS_SHAPE_NT(TR, TC, KM, (TR >= 32 ? kThreadsTall : kThreadsShort)) \
    FS_SHAPE_TALL256(TR, TC, KM)
#define FS_SHAPE_TALL256(TR, TC, KM) FS_SHAPE_TALL256_##TR(TC, KM)
#define FS_SHAPE_TALL256_8(TC, KM)
#define FS_SHAPE_TALL256_16(TC, KM)
#define FS_SHAPE_TALL256_32(TC, KM) FS_SHAPE_NT(32, TC, KM, kThreadsShort)

StepEntry kSteps[] = {
    FS_SHAPE(16, 4, 1) FS_SHAPE(16, 4, 4) FS_SHAPE(16, 4, 8) FS_SHAPE(16, 4, 16)
    FS_SHAPE(16, 8, 1) FS_SHAPE(16, 8, 4) FS_SHAPE(16, 8, 8) FS_SHAPE(16, 8, 16)
    FS_SHAPE(32, 4, 1) FS_SHAPE(32, 4, 8) FS_SHAPE(32, 4, 16)
    FS_SHAPE(32, 8, 1) FS_SHAPE(32, 8, 8) FS_SHAPE(32, 8, 16)
    FS_SHAPE(8, 16, 1) FS_SHAPE(8, 16, 4) FS_SHAPE(8, 16, 8)
    FS_SHAPE(8, 4, 1) FS_SHAPE(8, 4, 4) FS_SHAPE(8, 4, 8)
    FS_SHAPE(8, 8, 1) FS_SHAPE(8, 8, 4) FS_SHAPE(8, 8, 8)
    FS_SHAPE(16, 2, 1) FS_SHAPE(16, 2, 4) FS_SHAPE(16, 2, 8) FS_SHAPE(16, 2, 16)
    FS_SHAPE(16, 1, 8) FS_SHAPE(16, 1, 16)
    FS_SHAPE(32, 2, 16) FS_SHAPE(32, 1, 16)
    FS_SHAPE(32, 2, 32) FS_SHAPE(32, 1, 32) FS_SHAPE(32, 4, 32)
    FS_SHAPE(8, 2, 8) FS_SHAPE(8, 1, 8)
};
#undef FS_SHAPE
#undef FS_SHAPE_NT
#undef FS_SHAPE_TALL256
#undef FS_SHAPE_TALL256_8
#undef FS_SHAPE_TALL256_16
#undef FS_SHAPE_TALL256_32

const StepEntry* find_step(TileShape sh, bool adj) {
    for (const auto& e : kSteps)
        if (e.tr == sh.tr && e.tc == sh.tc && e.km == sh.km && e.adj == adj &&
            (sh.nt == 0 || sh.nt == e.nt))
            return &e;
    return nullptr;
}
}  // namespace

bool step_shape_supported(TileShape sh, bool adj) { return find_step(sh, adj) != nullptr; }

int step_shapes(TileShape* out, int max) {
    int n = 0;
    for (const auto& e : kSteps)
        if (!e.adj && n < max) out[n++] = TileShape{e.tr, e.tc, e.km, e.nt};
    return n;
}

hipError_t launch_step(hipStream_t st, TileShape sh, bool adj, const DevScen* d_jobs,
                       const int32_t* d_tile_job, int32_t ntiles, int32_t parity,
                       int32_t t_off, int32_t ksteps, int32_t skip, const float* lam,
                       Rings rings, Sched sched, int32_t grid, unsigned long long* d_stats) {
    const StepEntry* e = find_step(sh, adj);
    if (!e || ksteps > sh.km) return hipErrorInvalidValue;
    if (ntiles <= 0) return hipSuccess;
    int nb = ntiles;
    const bool listed = sched.in && skip == 1;
    if (listed) {
        // as many work-groups as can be resident at once (occupancy x CUs),
        // capped by the caller and by the tile count
        if (e->resident == 0) {
            int per_cu = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, e->fn_list, e->nt, 0) !=
                    hipSuccess || per_cu < 1)
                per_cu = 4;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                    hipSuccess || cus < 1)
                cus = 256;
            const_cast<StepEntry*>(e)->resident = per_cu * cus;
        }
        nb = std::max(1, std::min(std::min(grid, e->resident), ntiles));
    }
    hipLaunchKernelGGL(listed ? e->fn_list : (skip == 3 ? e->fn_wl : e->fn), dim3(nb),
                       dim3(e->nt), 0, st, d_jobs,
                       d_tile_job, ntiles, parity, t_off, ksteps, listed ? 0 : skip, lam,
                       rings, sched, d_stats);
    return hipGetLastError();
}

}  // namespace fs
