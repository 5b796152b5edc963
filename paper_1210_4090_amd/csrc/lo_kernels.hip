// gfx950 kernels of the fully discrete Lax--Oleinik step: the 1-D min-plus
// sweeps of eq. eqconvol taken axis by axis (Remark rk28) on the periodic grid
// of Section 3.3, the potential step, and the device-side window bound.
//
// All floating point is IEEE binary64 with no contraction (the library is
// built with -ffp-contract=off): a candidate is fl(u[source] + k(s)), the
// potential step is fl(w - hv) with hv = fl(tau * V).
//
// Window.  For a minimiser at displacement s > 0 (source left of the
// target), comparing with the next source to the right gives
//     k(s) - k(s-1) <= u[j+1] - u[j] <= D+ = max forward difference,
// and for s < 0 symmetrically k(s) - k(s+1) <= D- = max backward difference
// (up to the rounding of the two sums, covered by a slack of 2^-40 of the
// magnitudes involved).  k is convex, so its differences grow and the set of
// admissible s is an interval [-W-, W+]: every minimiser, ties included,
// lies in it, and enumerating it gives the exact value and lowest offset.
// Row sweeps take D+- from the row itself; strided sweeps take it from the
// previous step's sweep along the same axis, which bounds it because a
// min-plus sweep along another axis never increases the differences along
// this one and the potential step adds at most tau * max(V(x) - V(x + e_a)).
#include "lo_internal.h"

#include <math.h>

namespace lo {

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr uint64_t kSign = 0x8000000000000000ull;

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

__device__ __forceinline__ uint64_t enc_neg_inf()
{
    return ~(uint64_t)0xFFF0000000000000ull;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Block-wide max of three values; result valid in every thread.
__device__ void block_max3(double& a, double& b, double& c, double* red)
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

// Largest W in [0, kcap] such that every s = 1..W passes the test
//   level == false:  k(dir s) - k(dir (s-1)) <= D + slack   (neighbour comparison)
//   level == true:   k(dir s) - k(0)         <= D + slack   (comparison with e = 0)
// with slack = 2^-40 (sbase + |k(dir s)| + |other|).  Executed by one full
// wave.  *cap is set when the table ends before a failure.
__device__ int window_side(const double* __restrict__ k, int64_t kcap, int dir, double D,
                           double sbase, bool level, bool* cap)
{
    const int lane = threadIdx.x % kWave;
    const double k0 = k[0];
    for (int64_t base = 0; base < kcap; base += kWave) {
        const int64_t s = base + lane + 1;
        bool fail = true;
        if (s <= kcap) {
            const double a = k[dir * s], b = level ? k0 : k[dir * (s - 1)];
            const double d = a - b;
            const double lim = D + (sbase + fabs(a) + fabs(b)) * 0x1p-40;
            fail = !(d <= lim);
        }
        const uint64_t m = __ballot(fail);
        if (m) {
            const int first = __ffsll((unsigned long long)m) - 1;
            const int64_t sf = base + first + 1;
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

// Computes (W+, W-) for this block and broadcasts them through shared memory:
// the smaller of the neighbour bound (max differences Dp, Dm) and the level
// bound (oscillation osc of the sweep input).
__device__ void block_window(const SweepArgs& a, double Dp, double Dm, double osc, double M, int* shw)
{
    if (threadIdx.x < kWave) {
        int wp, wm;
        bool cap = false;
        if (a.wfix > 0) {
            wp = wm = a.wfix;
        } else {
            const double sbase = 1.0 + M + a.slack_extra;
            bool c1 = false, c2 = false, c3 = false, c4 = false;
            const int lp = window_side(a.kin.k, a.kin.kcap, +1, Dp, sbase, false, &c1);
            const int op = window_side(a.kin.k, a.kin.kcap, +1, osc, sbase, true, &c2);
            const int lm = window_side(a.kin.k, a.kin.kcap, -1, Dm, sbase, false, &c3);
            const int om = window_side(a.kin.k, a.kin.kcap, -1, osc, sbase, true, &c4);
            wp = min(lp, op);
            wm = min(lm, om);
            cap = (c1 && c2) || (c3 && c4);
        }
        if (threadIdx.x == 0) {
            shw[0] = wp;
            shw[1] = wm;
            if (cap && a.cap_is_error) atomicOr(&a.flags[0], kErrWindowCap);
            atomicMax(&a.flags[1 + a.axis], (uint32_t)max(wp, wm));
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void clear_slot(uint64_t* slot)
{
    if (slot && blockIdx.x == 0 && threadIdx.x < kSlotWords) slot[threadIdx.x] = enc_neg_inf();
}

__device__ __forceinline__ void record_arg(const SweepArgs& a, int64_t idx, int e, int& amax)
{
    if (e > 32767 || e < -32767) {
        atomicOr(&a.flags[0], kErrArgRange);
        e = e > 0 ? 32767 : -32767;
    }
    a.argmin[idx] = (int16_t)e;
    amax = max(amax, abs(e));
}

// Minimum update: values only, or value and lowest candidate index (strict <
// keeps the first of equal values; candidates are visited in increasing e).
template <int ARG>
__device__ __forceinline__ void take(double& best, int& arg, double v, int q)
{
    if (ARG) {
        if (v < best) {
            best = v;
            arg = q;
        }
    } else {
        best = fmin(best, v);
    }
}

// Window loop over candidates q = 0 .. ne-1 (offset e = q - wp) for TB
// targets whose first candidate sits at src[k][0], consecutive candidates
// `step` doubles apart in LDS.  kr[-q] is the kinetic cost of candidate q;
// it is the same for every lane, so it comes through scalar loads.
template <int ARG, int TB>
__device__ __forceinline__ void window_loop(const double* const (&src)[TB], int step, int ne,
                                            const double* __restrict__ kr, double (&best)[TB],
                                            int (&arg)[TB])
{
    int q = 0;
    for (; q + 8 <= ne; q += 8) {
        double kv[8];
#pragma unroll
        for (int t = 0; t < 8; t++) kv[t] = kr[-(q + t)];
#pragma unroll
        for (int t = 0; t < 8; t++) {
#pragma unroll
            for (int k = 0; k < TB; k++) take<ARG>(best[k], arg[k], src[k][(q + t) * step] + kv[t], q + t);
        }
    }
    for (; q < ne; q++) {
        const double kv = kr[-q];
#pragma unroll
        for (int k = 0; k < TB; k++) take<ARG>(best[k], arg[k], src[k][q * step] + kv, q);
    }
}

// ---------------------------------------------------------------------------
// Row sweep (axis 0, unit stride): one block per row, the whole row plus a
// wrapped halo of H cells on each side in LDS.  The window comes from the row
// itself.  Threads own targets tid, tid+256, ...; the candidate offset e is
// the same in every lane, so the kinetic cost k(-e) is a scalar load.
// ---------------------------------------------------------------------------
template <int ARG, int EPI, int TB>
__global__ __launch_bounds__(kBlock) void k_row_brute(const double* __restrict__ in,
                                                      double* __restrict__ out,
                                                      const double* __restrict__ kc, SweepArgs a, int H)
{
    extern __shared__ double sm[];
    __shared__ double red[24];
    __shared__ int shw[2];
    const int64_t N = a.g.n;
    const int64_t row = blockIdx.x;
    const double* __restrict__ src = in + row * N;
    double* lrow = sm + H;

    clear_slot(a.stats_clear);
    for (int64_t p = (int64_t)threadIdx.x - H; p < N + H; p += blockDim.x) {
        int64_t q = p < 0 ? p + N : (p >= N ? p - N : p);
        lrow[p] = src[q];
    }
    __syncthreads();

    double dp = -INFINITY, dm = -INFINITY, am = 0.0, hi = -INFINITY, nlo = -INFINITY;
    if (a.wfix <= 0) {
        for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
            const double x = lrow[i], y = lrow[i + 1];
            dp = fmax(dp, y - x);
            dm = fmax(dm, x - y);
            am = fmax(am, fabs(x));
            hi = fmax(hi, x);
            nlo = fmax(nlo, -x);
        }
        block_max3(dp, dm, am, red);
        double t = 0.0;
        block_max3(hi, nlo, t, red);
    }
    block_window(a, dp, dm, hi + nlo, am, shw);
    const int wp = __builtin_amdgcn_readfirstlane(shw[0]);
    const int wm = __builtin_amdgcn_readfirstlane(shw[1]);
    const bool inlds = wp <= H && wm <= H;
    const double* __restrict__ kr = kc + wp;   // kr[-q] = k(-(q - wp))
    const int ne = wp + wm + 1;
    int amax = 0;

    for (int64_t i0 = 0; i0 < N; i0 += (int64_t)TB * blockDim.x) {
        int64_t it[TB];
        double best[TB];
        int arg[TB];
#pragma unroll
        for (int k = 0; k < TB; k++) {
            it[k] = i0 + threadIdx.x + (int64_t)k * blockDim.x;
            best[k] = INFINITY;
            arg[k] = 0;
        }
        if (inlds) {
            const double* sp[TB];
#pragma unroll
            for (int k = 0; k < TB; k++) sp[k] = lrow + (it[k] < N ? it[k] : N - 1) - wp;
            window_loop<ARG, TB>(sp, 1, ne, kr, best, arg);
        } else {
            // window wider than the halo: wrap source indices explicitly
#pragma unroll
            for (int k = 0; k < TB; k++) {
                if (it[k] >= N) continue;
                int64_t j = (it[k] - wp) % N;
                if (j < 0) j += N;
                for (int q = 0; q < ne; ++q) {
                    take<1>(best[k], arg[k], lrow[j] + kr[-q], q);
                    if (++j == N) j = 0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TB; k++) {
            if (it[k] >= N) continue;
            const int64_t idx = row * N + it[k];
            double w = best[k];
            if (EPI) w = w - a.hv[idx];
            out[idx] = w;
            const int e = arg[k] - wp;
            if (ARG && a.argmin) record_arg(a, idx, e, amax);
            if (ARG && a.wfix > 0 && (e == -wp || e == wm)) atomicOr(&a.flags[0], kErrWindowEdge);
        }
    }
    if (ARG && a.argmin) {
        amax = (int)wave_max((double)amax);
        if (threadIdx.x % kWave == 0) atomicMax(&a.flags[4 + a.axis], (uint32_t)amax);
    }
}

// ---------------------------------------------------------------------------
// Tile sweep (any axis, any stride): a block owns C consecutive lines and R
// consecutive targets; sources [r0 - H, r0 + R + H] are staged in LDS as
// [row][line] (consecutive lanes = consecutive lines = consecutive
// addresses).  Windows wider than H read sources straight from global memory.
// Each tile also evaluates one extra target (r0 + R) so that the forward
// differences of the output along the axis can be bounded for the next step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t remap_block(int64_t b, int64_t G)
{
    // consecutive tiles of the same lines go to one XCD (blocks are dealt to
    // the 8 XCDs round robin), so their shared halo rows hit in its L2
    if (G % 8 != 0) return b;
    return (b % 8) * (G / 8) + b / 8;
}

template <int ARG, int EPI, int C, int TB>
__global__ __launch_bounds__(kBlock) void k_tile_brute(const double* __restrict__ in,
                                                       double* __restrict__ out,
                                                       const double* __restrict__ kc, SweepArgs a)
{
    extern __shared__ double sm[];
    __shared__ double red[24];
    __shared__ int shw[2];
    constexpr int RP = kBlock / C;  // target rows per pass
    const int64_t N = a.g.n, S = a.g.stride;
    const int H = a.halo, R = a.tile_rows;
    const int64_t nTB = (N + R - 1) / R;
    const int64_t nLB = (a.g.nlines + C - 1) / C;
    const int64_t b = remap_block(blockIdx.x, nTB * nLB);
    const int64_t lb = b / nTB, tb = b % nTB;
    const int64_t r0 = tb * R;
    const int Rt = (int)min((int64_t)R, N - r0);    // real targets of this tile
    double* tile = sm;                               // (R + 2H + 1) * C
    double* wbuf = sm + (size_t)(R + 2 * H + 1) * C;  // (R + 1) * C

    const int c = threadIdx.x % C;
    const int rr = threadIdx.x / C;
    const int64_t line = lb * C + c;
    const bool lv = line < a.g.nlines;
    const int64_t inner = lv ? line % S : 0, outer = lv ? line / S : 0;
    const int64_t base = inner + S * N * outer;

    clear_slot(a.stats_clear);
    for (int p = rr; p <= Rt + 2 * H; p += RP) {
        int64_t q = r0 - H + p;
        q %= N;
        if (q < 0) q += N;
        tile[p * C + c] = lv ? in[base + S * q] : 0.0;
    }
    double dp = -INFINITY, dm = -INFINITY, mm = -INFINITY, osc = INFINITY;
    if (a.wfix <= 0) {
        dp = dec(a.stats_in[a.axis]) + a.dv_fwd;
        dm = dec(a.stats_in[3 + a.axis]) + a.dv_bwd;
        mm = dec(a.stats_in[6]);
        osc = (dec(a.stats_in[7]) + dec(a.stats_in[8])) + a.osc_extra;
    }
    block_window(a, dp, dm, osc, mm, shw);  // ends with __syncthreads: the tile is staged
    const int wp = __builtin_amdgcn_readfirstlane(shw[0]);
    const int wm = __builtin_amdgcn_readfirstlane(shw[1]);
    const bool inlds = wp <= H && wm <= H;
    const double* __restrict__ kr = kc + wp;
    const int ne = wp + wm + 1;
    int amax = 0;

    for (int rb = 0; rb <= Rt; rb += TB * RP) {
        int rk[TB];
        double best[TB];
        int arg[TB];
#pragma unroll
        for (int k = 0; k < TB; k++) {
            rk[k] = rb + rr + k * RP;
            best[k] = INFINITY;
            arg[k] = 0;
        }
        if (inlds) {
            const double* sp[TB];
#pragma unroll
            for (int k = 0; k < TB; k++) sp[k] = tile + (size_t)((rk[k] <= Rt ? rk[k] : Rt) + H - wp) * C + c;
            window_loop<ARG, TB>(sp, C, ne, kr, best, arg);
        } else if (lv) {
#pragma unroll
            for (int k = 0; k < TB; k++) {
                if (rk[k] > Rt) continue;
                int64_t j = (r0 + rk[k] - wp) % N;
                if (j < 0) j += N;
                for (int q = 0; q < ne; ++q) {
                    take<1>(best[k], arg[k], in[base + S * j] + kr[-q], q);
                    if (++j == N) j = 0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TB; k++) {
            const int r = rk[k];
            if (r > Rt) continue;
            wbuf[r * C + c] = best[k];
            if (r < Rt && lv) {
                const int64_t idx = base + S * (r0 + r);
                double w = best[k];
                if (EPI) w = w - a.hv[idx];
                out[idx] = w;
                const int e = arg[k] - wp;
                if (ARG && a.argmin) record_arg(a, idx, e, amax);
                if (ARG && a.wfix > 0 && (e == -wp || e == wm)) atomicOr(&a.flags[0], kErrWindowEdge);
            }
        }
    }
    if (ARG && a.argmin) {
        amax = (int)wave_max((double)amax);
        if (threadIdx.x % kWave == 0) atomicMax(&a.flags[4 + a.axis], (uint32_t)amax);
    }
    if (a.stats_out) {
        __syncthreads();
        double sp = -INFINITY, sn = -INFINITY, sa = 0.0, hi = -INFINITY, nlo = -INFINITY;
        if (lv) {
            for (int r = rr; r < Rt; r += RP) {
                const double x = wbuf[r * C + c], y = wbuf[(r + 1) * C + c];
                sp = fmax(sp, y - x);
                sn = fmax(sn, x - y);
                sa = fmax(sa, fabs(x));
                if (EPI) {
                    const double z = x - a.hv[base + S * (r0 + r)];
                    sa = fmax(sa, fabs(z));
                    hi = fmax(hi, z);
                    nlo = fmax(nlo, -z);
                }
            }
        }
        block_max3(sp, sn, sa, red);
        if (EPI) {
            double t = 0.0;
            block_max3(hi, nlo, t, red);
        }
        if (threadIdx.x == 0) {
            atomicMax((unsigned long long*)&a.stats_out[a.axis], (unsigned long long)enc(sp));
            atomicMax((unsigned long long*)&a.stats_out[3 + a.axis], (unsigned long long)enc(sn));
            atomicMax((unsigned long long*)&a.stats_out[6], (unsigned long long)enc(sa));
            if (EPI) {
                atomicMax((unsigned long long*)&a.stats_out[7], (unsigned long long)enc(hi));
                atomicMax((unsigned long long*)&a.stats_out[8], (unsigned long long)enc(nlo));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------
__global__ void k_clear_slots(uint64_t* stats)
{
    const int i = threadIdx.x;
    if (i < kSlots * kSlotWords) stats[i] = enc_neg_inf();
}

// Max forward / backward difference along every axis and max |u| of u.
__global__ __launch_bounds__(kBlock) void k_stats(const double* __restrict__ u, int ndim, int64_t n0,
                                                  int64_t n1, int64_t n2, uint64_t* slot)
{
    __shared__ double red[24];
    const int64_t npts = n0 * n1 * n2;
    double dp[3] = {-INFINITY, -INFINITY, -INFINITY};
    double dm[3] = {-INFINITY, -INFINITY, -INFINITY};
    double am = 0.0, hi = -INFINITY, nlo = -INFINITY;
    const int64_t nn[3] = {n0, n1, n2};
    const int64_t st[3] = {1, n0, n0 * n1};
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
         x += (int64_t)gridDim.x * blockDim.x) {
        const double v = u[x];
        am = fmax(am, fabs(v));
        hi = fmax(hi, v);
        nlo = fmax(nlo, -v);
        for (int ax = 0; ax < ndim; ax++) {
            const int64_t i = (x / st[ax]) % nn[ax];
            const int64_t y = (i == nn[ax] - 1) ? x - st[ax] * (nn[ax] - 1) : x + st[ax];
            const double d = u[y] - v;
            dp[ax] = fmax(dp[ax], d);
            dm[ax] = fmax(dm[ax], -d);
        }
    }
    for (int ax = 0; ax < 3; ax++) {
        double t = 0.0;
        block_max3(dp[ax], dm[ax], t, red);
    }
    block_max3(am, hi, nlo, red);
    if (threadIdx.x == 0) {
        for (int ax = 0; ax < ndim; ax++) {
            atomicMax((unsigned long long*)&slot[ax], (unsigned long long)enc(dp[ax]));
            atomicMax((unsigned long long*)&slot[3 + ax], (unsigned long long)enc(dm[ax]));
        }
        atomicMax((unsigned long long*)&slot[6], (unsigned long long)enc(am));
        atomicMax((unsigned long long*)&slot[7], (unsigned long long)enc(hi));
        atomicMax((unsigned long long*)&slot[8], (unsigned long long)enc(nlo));
    }
}

// hv = fl(tau * fl(sum_m fl(c_m * phi_m))), summed in m order.
__global__ __launch_bounds__(kBlock) void k_synth_hv(const double* __restrict__ basis,
                                                     const double* __restrict__ coef, int nmodes,
                                                     int64_t npts, double tau, double* __restrict__ hv)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
         x += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int m = 0; m < nmodes; m++) {
            const double t = coef[m] * basis[(int64_t)m * npts + x];
            v = v + t;
        }
        hv[x] = tau * v;
    }
}

__global__ __launch_bounds__(kBlock) void k_scale(const double* __restrict__ V, double tau, int64_t npts,
                                                  double* __restrict__ hv)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
         x += (int64_t)gridDim.x * blockDim.x)
        hv[x] = tau * V[x];
}

// out6[a] = max_x V(x) - V(x+e_a), out6[3+a] = max_x V(x+e_a) - V(x) (encoded).
__global__ __launch_bounds__(kBlock) void k_potential_diffs(const double* __restrict__ V, int ndim,
                                                            int64_t n0, int64_t n1, int64_t n2,
                                                            uint64_t* out6)
{
    __shared__ double red[24];
    const int64_t npts = n0 * n1 * n2;
    const int64_t nn[3] = {n0, n1, n2};
    const int64_t st[3] = {1, n0, n0 * n1};
    double f[3] = {-INFINITY, -INFINITY, -INFINITY}, g[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
         x += (int64_t)gridDim.x * blockDim.x) {
        for (int ax = 0; ax < ndim; ax++) {
            const int64_t i = (x / st[ax]) % nn[ax];
            const int64_t y = (i == nn[ax] - 1) ? x - st[ax] * (nn[ax] - 1) : x + st[ax];
            const double d = V[x] - V[y];
            f[ax] = fmax(f[ax], d);
            g[ax] = fmax(g[ax], -d);
        }
    }
    for (int ax = 0; ax < 3; ax++) {
        double t = 0.0;
        block_max3(f[ax], g[ax], t, red);
    }
    if (threadIdx.x == 0) {
        for (int ax = 0; ax < ndim; ax++) {
            atomicMax((unsigned long long*)&out6[ax], (unsigned long long)enc(f[ax]));
            atomicMax((unsigned long long*)&out6[3 + ax], (unsigned long long)enc(g[ax]));
        }
    }
}

int grid_for(int64_t npts)
{
    int64_t g = (npts + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

template <int ARG, int EPI>
hipError_t launch_row(const double* in, double* out, const SweepArgs& a, hipStream_t s)
{
    const int64_t N = a.g.n;
    const int H = (int)(N < (int64_t)a.halo ? N : (int64_t)a.halo);
    const size_t lds = sizeof(double) * (size_t)(N + 2 * H);
    hipLaunchKernelGGL((k_row_brute<ARG, EPI, 4>), dim3((unsigned)a.g.nlines), dim3(kBlock), lds, s, in,
                       out, a.kin.k, a, H);
    return hipGetLastError();
}

template <int ARG, int EPI>
hipError_t launch_tile(const double* in, double* out, const SweepArgs& a, hipStream_t s)
{
    constexpr int C = 16;
    const int64_t N = a.g.n;
    const int R = a.tile_rows, H = a.halo;
    const int64_t G = ((N + R - 1) / R) * ((a.g.nlines + C - 1) / C);
    const size_t lds = sizeof(double) * ((size_t)(R + 2 * H + 1) * C + (size_t)(R + 1) * C);
    hipLaunchKernelGGL((k_tile_brute<ARG, EPI, C, 4>), dim3((unsigned)G), dim3(kBlock), lds, s, in, out,
                       a.kin.k, a);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_clear_slots(uint64_t* stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_slots, dim3(1), dim3(64), 0, s, stats);
    return hipGetLastError();
}

hipError_t launch_stats(const double* u, int ndim, const int64_t* n, uint64_t* slot, hipStream_t s)
{
    const int64_t n0 = n[0], n1 = ndim > 1 ? n[1] : 1, n2 = ndim > 2 ? n[2] : 1;
    hipLaunchKernelGGL(k_stats, dim3(grid_for(n0 * n1 * n2)), dim3(kBlock), 0, s, u, ndim, n0, n1, n2, slot);
    return hipGetLastError();
}

hipError_t launch_synth_hv(const double* basis, const double* coef_dev, int nmodes, int64_t npts,
                           double tau, double* hv, hipStream_t s)
{
    hipLaunchKernelGGL(k_synth_hv, dim3(grid_for(npts)), dim3(kBlock), 0, s, basis, coef_dev, nmodes, npts,
                       tau, hv);
    return hipGetLastError();
}

hipError_t launch_scale(const double* V, double tau, int64_t npts, double* hv, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(grid_for(npts)), dim3(kBlock), 0, s, V, tau, npts, hv);
    return hipGetLastError();
}

hipError_t launch_potential_diffs(const double* V, int ndim, const int64_t* n, double* out6, hipStream_t s)
{
    const int64_t n0 = n[0], n1 = ndim > 1 ? n[1] : 1, n2 = ndim > 2 ? n[2] : 1;
    hipLaunchKernelGGL(k_potential_diffs, dim3(grid_for(n0 * n1 * n2)), dim3(kBlock), 0, s, V, ndim, n0, n1,
                       n2, (uint64_t*)out6);
    return hipGetLastError();
}

hipError_t launch_sweep(int method, const double* in, double* out, const SweepArgs& a, hipStream_t s)
{
    (void)method;
    const bool arg = a.argmin != nullptr || a.wfix > 0;
    const bool epi = a.hv != nullptr;
    const bool row = a.kind == kKindRow;
    if (row) {
        if (arg) return epi ? launch_row<1, 1>(in, out, a, s) : launch_row<1, 0>(in, out, a, s);
        return epi ? launch_row<0, 1>(in, out, a, s) : launch_row<0, 0>(in, out, a, s);
    }
    if (arg) return epi ? launch_tile<1, 1>(in, out, a, s) : launch_tile<1, 0>(in, out, a, s);
    return epi ? launch_tile<0, 1>(in, out, a, s) : launch_tile<0, 0>(in, out, a, s);
}

}  // namespace lo
