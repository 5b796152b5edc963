// Device helpers shared by the sweep kernels: order-preserving encodings for
// atomic max/min of doubles, block reductions, and the rigorous window bound.
#pragma once

#include <math.h>

#include "lo_internal.h"

namespace lo {
namespace dev {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr uint64_t kSign = 0x8000000000000000ull;

// Monotone map double -> uint64 (x < y  <=>  enc(x) < enc(y)) so that
// unsigned integer atomics compute max / min of doubles.
__device__ __forceinline__ uint64_t enc(double x)
{
    uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b & kSign) ? ~b : (b | kSign);
}

__device__ __forceinline__ double dec(uint64_t k)
{
    uint64_t b = (k & kSign) ? (k & ~kSign) : ~k;
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ uint64_t enc_neg_inf() { return ~(uint64_t)0xFFF0000000000000ull; }

// One DPP move of a double (both halves with the same control); lanes without
// a source keep their own value.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = (int)b, hi = (int)(b >> 32);
    const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xf, false);
    const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)h2 << 32) | (unsigned)l2));
}

// Wave maximum through row shifts and row broadcasts; valid in lane 63 only.
__device__ __forceinline__ double wave_max_to63(double v)
{
    v = fmax(v, dpp_move<0x111, 0xf>(v));   // row_shr:1
    v = fmax(v, dpp_move<0x112, 0xf>(v));   // row_shr:2
    v = fmax(v, dpp_move<0x114, 0xf>(v));   // row_shr:4
    v = fmax(v, dpp_move<0x118, 0xf>(v));   // row_shr:8  -> lane 15 of each row: row max
    v = fmax(v, dpp_move<0x142, 0xa>(v));   // row_bcast:15 into rows 1, 3
    v = fmax(v, dpp_move<0x143, 0xc>(v));   // row_bcast:31 into rows 2, 3 -> lane 63: wave max
    return v;
}

// Wave maximum in every lane: the row shifts and broadcasts above, then lane
// 63 read out (register moves only; a butterfly of lane shuffles would take
// six LDS round trips).
__device__ __forceinline__ double wave_max(double v)
{
    const long long b = __double_as_longlong(wave_max_to63(v));
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, kWave - 1);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), kWave - 1);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Largest v >= 0 over the block into *dst with one global atomic (many
// blocks contending on one address cost far more than a block's barrier).
// Every thread of the block calls it.
__device__ inline void block_atomic_max(int v, uint32_t* dst)
{
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    v = (int)wave_max((double)v);
    if (threadIdx.x % kWave == 0 && v > 0) atomicMax(&s, v);
    __syncthreads();
    if (threadIdx.x == 0 && s > 0) atomicMax(dst, (uint32_t)s);
}

// The word of the sub-slots that an argmin sweep's block folds its largest
// |offset| into: the step's own words when given, else the flags' (spread
// over kSpread sub-slots, so that the blocks of a launch do not all contend
// on one address).
__device__ __forceinline__ uint32_t* amax_word(const SweepArgs& a)
{
    const int j = (int)(blockIdx.x % kSpread);
    return a.amax_out ? a.amax_out + a.axis * kSpread + j : a.flags + kFlagAmax + a.axis * kSpread + j;
}

// Block-wide max of three values (blockDim <= 512); result in every thread.
__device__ inline void block_max3(double& a, double& b, double& c, double* red)
{
    a = wave_max(a);
    b = wave_max(b);
    c = wave_max(c);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if (l == 0) {
        red[w] = a;
        red[8 + w] = b;
        red[16 + w] = c;
    }
    __syncthreads();
    a = red[0];
    b = red[8];
    c = red[16];
    for (int i = 1; i < nw; i++) {
        a = fmax(a, red[i]);
        b = fmax(b, red[8 + i]);
        c = fmax(c, red[16 + i]);
    }
    __syncthreads();
}

// Block-wide max of five values; result in every thread (red: 40 doubles).
__device__ inline void block_max5(double& a, double& b, double& c, double& d, double& e, double* red)
{
    a = wave_max(a);
    b = wave_max(b);
    c = wave_max(c);
    d = wave_max(d);
    e = wave_max(e);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if (l == 0) {
        red[w] = a;
        red[8 + w] = b;
        red[16 + w] = c;
        red[24 + w] = d;
        red[32 + w] = e;
    }
    __syncthreads();
    a = red[0];
    b = red[8];
    c = red[16];
    d = red[24];
    e = red[32];
    for (int i = 1; i < nw; i++) {
        a = fmax(a, red[i]);
        b = fmax(b, red[8 + i]);
        c = fmax(c, red[16 + i]);
        d = fmax(d, red[24 + i]);
        e = fmax(e, red[32 + i]);
    }
    __syncthreads();
}

// Block-wide max of five values, valid in thread 0 only (red: 40 doubles).
__device__ inline void block_max5_to0(double& a, double& b, double& c, double& d, double& e, double* red)
{
    a = wave_max_to63(a);
    b = wave_max_to63(b);
    c = wave_max_to63(c);
    d = wave_max_to63(d);
    e = wave_max_to63(e);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if (l == kWave - 1) {
        red[w] = a;
        red[8 + w] = b;
        red[16 + w] = c;
        red[24 + w] = d;
        red[32 + w] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = red[0];
        b = red[8];
        c = red[16];
        d = red[24];
        e = red[32];
        for (int i = 1; i < nw; i++) {
            a = fmax(a, red[i]);
            b = fmax(b, red[8 + i]);
            c = fmax(c, red[16 + i]);
            d = fmax(d, red[24 + i]);
            e = fmax(e, red[32 + i]);
        }
    }
}

__device__ __forceinline__ void clear_slot(uint64_t* slot)
{
    if (slot && blockIdx.x == 0)
        for (int i = threadIdx.x; i < kSlotStride; i += blockDim.x) slot[i] = enc_neg_inf();
}

// Fold a value into word `w` of a stats slot (sub-slot chosen by the block).
__device__ __forceinline__ void stat_put(uint64_t* slot, int w, double v)
{
    atomicMax((unsigned long long*)&slot[stat_index(w, (int)(blockIdx.x % kSpread))], (unsigned long long)enc(v));
}

// A wave-uniform 64-bit value moved to scalar registers, so that pointers
// offset by it still qualify for scalar loads.
__device__ __forceinline__ int64_t uniform64(int64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Batched launches: move a sweep's table, slots, windows and P to instance
// blockIdx.y; returns the offset of the instance's arrays (b * b_u) and sets
// *koff to that of its kinetic table.
__device__ __forceinline__ int64_t batch_shift(SweepArgs& a, int64_t* koff)
{
    const int64_t b = blockIdx.y;
    const int64_t ko = uniform64(b * a.b_k);
    *koff = ko;
    a.kin.k += ko;
    if (a.stats_in) a.stats_in += uniform64(b * a.b_stats);
    if (a.stats_out) a.stats_out += uniform64(b * a.b_stats);
    if (a.stats_clear) a.stats_clear += uniform64(b * a.b_stats);
    a.win_in += uniform64(b * a.b_win);
    if (a.pofs_b) a.pofs = a.pofs_b[b * kMaxDim + a.axis];
    return uniform64(b * a.b_u);
}

// Block 0 (of each instance) of the sweep that carries them computes the
// next step's windows; the sweeps of this step keep reading their own slot.
__device__ __forceinline__ void maybe_next_windows(const SweepArgs& a);

__device__ __forceinline__ int64_t remap_block(int64_t b, int64_t G)
{
    // consecutive tiles of the same lines go to one XCD (blocks are dealt to
    // the 8 XCDs round robin), so their shared halo rows hit in its L2
    if (G % 8 != 0) return b;
    return (b % 8) * (G / 8) + b / 8;
}

// Largest W in [0, kcap] such that every s = 1..W passes the test
//   level == false:  k(dir s) - k(dir (s-1)) <= D + slack   (neighbour bound)
//   level == true:   k(dir s) - k(0)         <= D + slack   (oscillation bound)
// with slack = 2^-40 (sbase + |k(dir s)| + |other|).  Both left sides are
// nondecreasing in s beyond the kernel's minimum (k is convex) and the level
// test passes below it, so the passing s form an interval 1..W.  One wave
// runs it, probing 64 values of s at a time starting below `est` (a
// closed-form guess for the mechanical cost; 0 when none): when the probe's
// first value passes, everything below it passes too.  *cap is set when the
// table ends before a failure.  kf(s) gives k(s): a table read, or the
// mechanical cost evaluated in place (the same operations as the table's,
// so the same values, without a memory round trip per probe).
template <class KF>
__device__ __forceinline__ int window_side(KF kf, int64_t kcap, int dir, double D, double sbase, bool level, int64_t est,
                                  bool* cap)
{
    const int lane = threadIdx.x % kWave;
    const double k0 = kf(0);
    auto fails = [&](int64_t s) {
        if (s > kcap) return true;
        const double a = kf(dir * s), b = level ? k0 : kf(dir * (s - 1));
        const double d = a - b;
        const double lim = D + (sbase + fabs(a) + fabs(b)) * 0x1p-40;
        return !(d <= lim);
    };
    int64_t base = est - kWave / 2;
    if (base < 1) base = 1;
    if (base > kcap) base = kcap;
    // probe s = base .. base+63; lane 0's value must pass for the shortcut
    {
        const uint64_t m = __ballot(fails(base + lane));
        if (m & 1ull) {
            base = 1;   // the guess was too high: scan from the start
        } else if (m) {
            const int64_t sf = base + __ffsll((unsigned long long)m) - 1;
            if (sf > kcap) {
                *cap = true;
                return (int)kcap;
            }
            return (int)(sf - 1);
        } else {
            base += kWave;
        }
    }
    for (; base <= kcap; base += kWave) {
        const uint64_t m = __ballot(fails(base + lane));
        if (m) {
            const int64_t sf = base + __ffsll((unsigned long long)m) - 1;
            if (sf > kcap) {
                *cap = true;
                return (int)kcap;
            }
            return (int)(sf - 1);
        }
    }
    *cap = true;
    return (int)kcap;
}

// The mechanical cost of s cells, tau K*(s dx / tau) for K(p) = (p + P)^2 / 2,
// in the evaluation order of the plans' tables (each operation rounded on its
// own, IEEE division).
__device__ __forceinline__ double mech_cost_dev(int64_t s, double dx, double tau, double P)
{
    const double d = (double)s * dx;
    const double a = 0.5 * d;
    const double b = a * d;
    const double c = b / tau;
    const double e = P * d;
    return c - e;
}

// Windows of every axis for the next step of instance `inst` (its kinetic
// tables at inst * bk[a]), from the statistics in `slot` (recorded by the
// step's sweep kernels, which have all completed).  All of its global loads
// go out at once: wave w reduces statistics words w, w + nwaves, ... (one
// sub-slot a lane) and wave 0 copies the parameters into LDS.  Then the four
// one-sided searches of each axis (the neighbour bound and the oscillation
// bound on each side) are dealt to the waves; the window is the smaller of
// the two bounds on each side.  Every thread of the block calls it.
__device__ inline void next_windows(const WinParams& Pg, int64_t inst, const uint64_t* slot, int* win_out,
                                    uint32_t* flags)
{
    constexpr int kWords = 9;   // [a] max fwd diff, [3 + a] max -fwd diff, [6] max|w|, [7] max u, [8] max -u
    constexpr int kParamWords = (int)(sizeof(WinParams) / 8);
    static_assert(sizeof(WinParams) % 8 == 0 && kParamWords <= kWave, "one wave copies the parameters");
    __shared__ double sw[kWords];
    __shared__ union {
        WinParams p;
        uint64_t w[kParamWords];
    } sp;
    __shared__ int part[kMaxDim][4];
    __shared__ int caps[kMaxDim][4];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, nwv = blockDim.x / kWave;
    {
        uint64_t v[3];   // every caller's blocks have 4 waves or more: at most 3 words a wave
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int k = w + i * nwv;
            v[i] = k < kWords ? slot[stat_index(k, lane)] : 0;
        }
        uint64_t pw = 0;
        if (w == 0 && lane < kParamWords) __builtin_memcpy(&pw, (const char*)&Pg + 8 * lane, 8);
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int k = w + i * nwv;
            if (k < kWords) {
                const double m = wave_max_to63(dec(v[i]));
                if (lane == kWave - 1) sw[k] = m;
            }
        }
        if (w == 0 && lane < kParamWords) sp.w[lane] = pw;
    }
    __syncthreads();
    const WinParams& P = sp.p;
    const double M = sw[6] + (P.lag ? P.slack_extra : 0.0);
    const double osc0 = sw[7] + sw[8] + (P.lag ? P.hv_osc : 0.0);
    for (int t = w; t < 4 * P.ndim; t += nwv) {
        const int ax = t >> 2, kind = t & 3;
        const int dir = kind < 2 ? 1 : -1;
        const bool level = (kind & 1) != 0;
        if (P.wfix[ax] > 0) continue;
        double D;
        if (level)
            D = osc0 + P.osc_extra[ax];
        else
            D = sw[dir > 0 ? ax : 3 + ax] + (dir > 0 ? P.dvf[ax] : P.dvb[ax]) * (P.lag ? 2.0 : 1.0);
        const double sbase = 1.0 + M + P.slack_extra;
        int64_t est = 0;
        if (P.quad[ax]) {
            const double po = P.pofs_b ? P.pofs_b[inst * kMaxDim + ax] : P.pofs[ax];
            const double c = P.cq[ax], p = 2.0 * P.cq[ax] * po * (double)dir;
            double e;
            if (level)
                e = (p + sqrt(fmax(p * p + 4.0 * c * fmax(D, 0.0), 0.0))) / (2.0 * c);
            else
                e = (D + p) / (2.0 * c) + 0.5;
            if (e > 0.0 && e < 1e9) est = (int64_t)e;
        }
        bool cap = false;
        int r;
        if (P.quad[ax]) {
            const double dx = P.dx[ax], tau = P.tau;
            const double Pa = P.P_b ? P.P_b[inst * kMaxDim + ax] : P.P[ax];
            r = window_side([=](int64_t s) { return mech_cost_dev(s, dx, tau, Pa); }, P.kcap[ax], dir, D, sbase,
                            level, est, &cap);
        } else {
            const double* __restrict__ kt = P.k[ax] + inst * P.bk[ax];
            r = window_side([=](int64_t s) { return kt[s]; }, P.kcap[ax], dir, D, sbase, level, est, &cap);
        }
        if (lane == 0) {
            part[ax][kind] = r;
            caps[ax][kind] = cap ? 1 : 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int ax = 0; ax < P.ndim; ax++) {
            int wp, wm;
            bool cap = false;
            if (P.wfix[ax] > 0) {
                wp = wm = P.wfix[ax];
            } else {
                wp = min(part[ax][0], part[ax][1]);
                wm = min(part[ax][2], part[ax][3]);
                cap = (caps[ax][0] && caps[ax][1]) || (caps[ax][2] && caps[ax][3]);
            }
            win_out[2 * ax] = wp;
            win_out[2 * ax + 1] = wm;
            if (cap && P.cap_err[ax]) atomicOr(&flags[0], kErrWindowCap);
            atomicMax(&flags[kFlagWin + ax * kSpread], (uint32_t)max(wp, wm));
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void maybe_next_windows(const SweepArgs& a)
{
    if (a.win_next && blockIdx.x == 0) {
        const int64_t b = blockIdx.y;
        next_windows(*a.winp_dev, b, a.win_slot + b * a.b_stats, a.win_next + b * a.b_win, a.flags);
    }
}

}  // namespace dev
}  // namespace lo
