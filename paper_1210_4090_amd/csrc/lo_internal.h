// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lo.h"

namespace lo {

constexpr int kMaxDim = 3;
constexpr int kKinPad = 8;         // +inf entries on each side of a caller's kinetic table on the device
constexpr int kSlots = 3;          // rotating stats slots: read n%3, write (n+1)%3, clear (n+2)%3
constexpr int kSlotWords = 10;     // per slot: [a] max fwd diff, [3+a] max -fwd diff, [6] max|w|,
                                   // [7] max u, [8] max -u of the step result
constexpr int kSpread = 64;        // each word is spread over 64 sub-slots (block index mod 64) so
                                   // that thousands of blocks do not contend on one atomic address
constexpr int kSubStride = 16;     // a sub-slot holds its words in one 128-byte line: the blocks'
                                   // atomics on a word go to 64 lines (and L2 channels), not 5
constexpr int kSlotStride = kSpread * kSubStride;
static_assert(kSlotWords <= kSubStride, "a sub-slot's words fit its line");
// word w of sub-slot j of a statistics slot
__host__ __device__ constexpr int stat_index(int w, int j) { return j * kSubStride + w; }

// error bits latched in flags[0]
constexpr uint32_t kErrWindowCap = 1u;    // computed window exceeded the kinetic table
constexpr uint32_t kErrWindowEdge = 2u;   // fixed window: argmin on the edge
constexpr uint32_t kErrArgRange = 4u;     // argmin offset does not fit int16
constexpr uint32_t kErrFastPath = 8u;     // fast kernel left a target without a finite candidate
constexpr uint32_t kErrAdjointHalo = 16u; // reverse pass met an offset beyond its halo (internal error)
// flags layout: [0] error bits; the window used by axis a (max over blocks
// and steps) spread at [kFlagWin + a * kSpread + j]; the largest |argmin| of
// axis a (argmin sweeps) spread at [kFlagAmax + a * kSpread + j]
constexpr int kFlagWin = 8;
constexpr int kFlagAmax = kFlagWin + 3 * kSpread;
constexpr int kFlagWords = kFlagAmax + 3 * kSpread;

// Geometry of one axis sweep: a line is the set of points that differ only in
// coordinate a.  Point (line l, position p) lives at
//   inner(l) + stride * (p + n * outer(l)),  inner = l % stride, outer = l / stride.
struct AxisGeom {
    int64_t n;        // points on the line
    int64_t stride;   // distance between consecutive points of a line
    int64_t nlines;   // npts / n
};

// Kinetic cost table on the device: ktab[s] valid for s in [-kcap, kcap]
// (pointer already offset to s = 0).
struct KinTab {
    const double* k;
    int64_t kcap;
};

// What the last block of a time step needs to bound every axis' window for
// the next step (from the statistics the step's sweeps just recorded).
struct WinParams {
    const double* k[kMaxDim];      // kinetic tables, offset to s = 0
    int64_t kcap[kMaxDim];
    double dvf[kMaxDim];           // bound on tau*(V(x) - V(x+e_a))
    double dvb[kMaxDim];           // bound on tau*(V(x+e_a) - V(x))
    double osc_extra[kMaxDim];     // oscillation growth through the sweeps before axis a
    double cq[kMaxDim];            // mechanical cost c s^2 - p s: c and p / (2c), for guesses
    double pofs[kMaxDim];
    int quad[kMaxDim];
    int cap_err[kMaxDim];          // a window reaching the table end is an error
    int wfix[kMaxDim];
    double slack_extra;
    int ndim;
    // batched plans (one block per instance): instance b's tables, slot and
    // windows sit at b * bk[a], b * b_stats and b * b_win from instance 0's
    int64_t bk[kMaxDim];
    int64_t b_stats;
    int b_win;
    const double* pofs_b;          // [nb][kMaxDim] per-instance P tau / dx, nullptr: pofs[]
    // lag = 1: the statistics are those of u^n and the windows are for step
    // n + 1, one potential step later: forward differences grow by at most
    // dvf / dvb, the oscillation by at most hv_osc, |w| by slack_extra
    int lag;
    double hv_osc;
    // the mechanical cost evaluated in place by the search (quad axes)
    double dx[kMaxDim];
    double tau;
    double P[kMaxDim];
    const double* P_b;             // [nb][kMaxDim] per-instance P (nullptr: P[])
};

// Everything a sweep kernel needs besides the arrays.
struct SweepArgs {
    AxisGeom g;
    KinTab kin;
    int axis;
    int ndim;
    int32_t wfix;               // > 0: fixed window
    double slack_extra;         // added to max|w| in the rounding slack of the window test
    double dv_fwd;              // bound on tau*(V(x) - V(x+e_a)) over the grid and steps
    double dv_bwd;              // bound on tau*(V(x+e_a) - V(x))
    double osc_extra;           // growth of the oscillation through the sweeps before this one
    const uint64_t* stats_in;   // slot read for this step (nullptr: row-local window)
    uint64_t* stats_out;        // slot written (nullptr: none)
    uint64_t* stats_clear;      // slot cleared by block 0 (nullptr: none)
    uint32_t* flags;
    const double* hv;           // tau*V at this step (nullptr: no potential step)
    int16_t* argmin;            // nullptr or [npts] offsets for this axis
    int halo;                   // LDS halo rows of the tile kernels
    int tile_rows;              // targets per tile (tile kernels)
    int kind;                   // kKindRow or kKindTile
    int cap_is_error;           // 0 when the kinetic table is the cost's whole support
    int fast;                   // claim kernel (any convex cost)
    int quad;                   // the cost is the mechanical c s^2 - p s (window guesses, closed-form claim crossings)
    double cq;                  // c = dx^2 / (2 tau): k(s) = c s^2 - p s
    double inv2c;               // 1 / (2c)
    double pofs;                // p / (2c) = P tau / dx
    double kslack;              // 2^-40 (1 + max |k|): rounding slack of a table's crossings
    int kvert;                  // a caller table's minimising offset (the fast sweeps centre their cost band
                                // on the cost's vertex: this, or P tau / dx for the mechanical cost)
    const int* win_in;          // this step's windows: [2a] = W+, [2a+1] = W- of axis a
    // batched launches: blockIdx.y is the instance; its arrays, kinetic
    // table, stats slots and windows sit at these strides from instance 0's
    int grid_cap;               // persistent kernels: at most this many blocks along x
    int row_ch;                 // fast row kernel: points per thread (4 or 8)
    int nb;                     // instances (1: plain plan)
    int64_t b_u;
    int64_t b_k;
    int64_t b_stats;
    int b_win;
    const double* pofs_b;       // [nb][kMaxDim] per-instance P tau / dx (nullptr: pofs)
    // the next step's windows, computed by block 0 (of each instance) from
    // the statistics of this step's input (nullptr: not by this sweep)
    const WinParams* winp_dev;
    const uint64_t* win_slot;
    int* win_next;
    // host side only: when set, the sweep's kernel is launched with these
    // events recording its own start and end (lo_time_kernels)
    hipEvent_t ev_start;
    hipEvent_t ev_stop;
    uint32_t* amax_out;         // argmin sweeps: the step's largest |offset|, [axis][kSpread] (nullptr: the flags')
    int wt;                     // fast tiles of 16 lines: outputs written through the L2 (agent-scope stores)
    int16_t narrow;             // fast sweeps at one 512-thread block a CU (room for another stream's kernels)
    int16_t search_block;       // fast one-line tile sweeps: block 0 only computes the next step's windows,
                                // the sweep's tiles go to blocks 1, 2, ... (set by the launcher)
};

// Launch a sweep kernel K (parenthesised if it has template arguments) with
// the SweepArgs A's timing events when it has them.
#define LO_SWEEP_LAUNCH(K, G, B, SH, S, A, ...)                                              \
    do {                                                                                      \
        if ((A).ev_start)                                                                     \
            hipExtLaunchKernelGGL(K, G, B, SH, S, (A).ev_start, (A).ev_stop, 0u, __VA_ARGS__); \
        else                                                                                  \
            hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                                  \
    } while (0)

constexpr int kKindRow = 0;     // whole lines in LDS, unit stride
constexpr int kKindTile = 1;    // tile of lines x targets with a halo

// ---- kernel launchers (lo_kernels.hip) ----
hipError_t launch_clear_slots(uint64_t* stats, int nb, hipStream_t s);
hipError_t launch_windows(const WinParams& P, const uint64_t* slot, int* win_out, uint32_t* flags, int nb,
                          hipStream_t s);
hipError_t launch_stats(const double* u, int ndim, const int64_t* n, uint64_t* slot, int nb, int64_t b_u,
                        int64_t b_stats, hipStream_t s);
// t[s + cap] = the mechanical cost of s cells for s in [-cap, cap] (device-built, equal to the host's).
hipError_t launch_mech_table(double* t, int64_t cap, double dx, double tau, double P, hipStream_t s);
// w[0..n) = v (a kernel, so that no memset node enters a captured graph).
hipError_t launch_fill_u32(uint32_t* w, int64_t n, uint32_t v, hipStream_t s);
// per instance of a batch: [b][0] = enc max(u - snap), [b][1] = enc max(snap - u)
hipError_t launch_diff_range(const double* u, const double* snap, int64_t npts, int nb, uint64_t* out,
                             hipStream_t s);
hipError_t launch_synth_hv(const double* basis, const double* coef_dev, int nmodes, int64_t npts,
                           double tau, double* hv, hipStream_t s);
hipError_t launch_scale(const double* V, double tau, int64_t npts, double* hv, hipStream_t s);
// Q[i] = hv[0] + ... + hv[i-1] for i in [0, N] (device, one block).
hipError_t launch_prefix(const double* hv, int64_t N, double* Q, hipStream_t s);
// One step of the first discrete semigroup (1-D): u -> w, Q the prefix sums of hv ([N + 1]).
hipError_t launch_semigroup1(const double* u, double* w, int64_t N, int W, const double* kt_centre, const double* hv,
                             const double* Q, unsigned* sat, hipStream_t s);
// One step of the decomposition comparison path (1-D): u -> w (sweep) -> u_out = w - hv.
// tol: the slope tolerance on raw increments (eta dx); kabs: max |k| over the table.
hipError_t launch_decomp_step(const double* u, double* w, double* u_out, int N, int W, const double* kt_centre,
                              double tol, double kabs, const double* hv, unsigned long long* counts, hipStream_t s);
hipError_t launch_potential_diffs(const double* V, int ndim, const int64_t* n, double* out6,
                                  hipStream_t s);
hipError_t launch_sweep(int method, const double* in, double* out, const SweepArgs& a,
                        hipStream_t s);

hipError_t launch_fast(const double* in, double* out, const SweepArgs& a, double cq, double inv2c,
                       double pofs, hipStream_t s);
size_t fast_lds_for(int kind, int64_t N, int tile_rows, int H, int tile_lines);
int fast_tile_lines(int64_t nlines);   // lines side by side in a fast TILE sweep
void row_layout(int64_t N, int halo, int* nr, int* RS, int* H);
size_t row_lds_bytes(int64_t N, int halo);
size_t tile_lds_bytes(int halo);

// Reverse sweep (adjoint scatter) of one axis: tiles of C lines x R sources
// with a halo of h targets on each side (h >= max |argmin offset|).
struct ScatterArgs {
    AxisGeom g;
    int h;
    int R;
    int C;
    int span;   // R + 2h
    int wt;     // outputs written through the L2 (a small grid, stores of whole cache lines)
};

// ---- reverse pass (lo_adjoint.hip) ----
size_t scatter_lds_bytes(int C, int R, int h);
bool scatter_layout(const AxisGeom& g, int h, size_t lds_max, ScatterArgs* a);
hipError_t launch_scatter(const int16_t* E, const double* lam, double* out, double* Lam, const ScatterArgs& a,
                          uint32_t* flags, hipStream_t s);
int project_blocks(int64_t npts);
// Largest |argmin offset| of each axis over [steps][ndim][npts] int16 offsets (atomicMax into out[a]).
hipError_t launch_absmax16(const int16_t* E, int64_t steps, int ndim, int64_t npts, uint32_t* out, hipStream_t s);
hipError_t launch_project(const double* Lam, const double* basis, int M, int64_t npts, double* partial,
                          double* out, hipStream_t s);

}  // namespace lo
