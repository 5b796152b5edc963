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
#include "lo_device.h"

#include <math.h>

#include <algorithm>

namespace lo {

namespace {

using namespace dev;

__device__ __forceinline__ void record_arg(const SweepArgs& a, int64_t idx, int e, int& amax)
{
    if (e > 32767 || e < -32767) {
        atomicOr(&a.flags[0], kErrArgRange);
        e = e > 0 ? 32767 : -32767;
    }
    a.argmin[idx] = (int16_t)e;
    amax = max(amax, abs(e));
}

// Minimum update: values only, or value and lowest candidate offset (strict <
// keeps the first of equal values; candidates arrive in increasing offset).
template <int ARG>
__device__ __forceinline__ void take(double& best, int& arg, double v, int e)
{
    if (ARG) {
        if (v < best) {
            best = v;
            arg = e;
        }
    } else {
        best = fmin(best, v);
    }
}

// Register-blocked window loop.  A thread owns TB consecutive targets
// base .. base+TB-1 of a line; source base+q (q = -wp .. TB-1+wm) is read
// from LDS once, at lds[lane + off(q)], and offered to all TB targets with
// the kinetic cost k(k - q) of target base+k.  Every target thereby sees a
// superset of its window [-wp, wm]: the extra candidates are genuine lifted
// sources, and none of them can tie the minimum (all minimisers lie inside
// the window), so values and lowest offsets are those of the window.  The
// costs depend only on (k, q), the same in every lane: scalar loads.  They
// are read for displacements -(TB-1+wm) .. TB-1+wp: a mechanical table spans
// two periods (beyond any window that fits the LDS halo) and a caller's table
// carries TB-1 entries of +inf past each end on the device.
template <int ARG, int TB, class Off>
__device__ __forceinline__ void blocked_loop(const double* lds, int lane, Off off, int wp, int wm,
                                             const double* __restrict__ kc, double (&best)[TB], int (&arg)[TB])
{
    const int qhi = TB - 1 + wm;
    int q = -wp;
    for (; q + 1 <= qhi; q += 2) {
        const double* __restrict__ kq = kc - q - 1;   // kq[i] = k(i - q - 1)
        double kv[TB + 1];
#pragma unroll
        for (int i = 0; i <= TB; i++) kv[i] = kq[i];
        const double v0 = lds[lane + off(q)];
        const double v1 = lds[lane + off(q + 1)];
#pragma unroll
        for (int k = 0; k < TB; k++) {
            take<ARG>(best[k], arg[k], v0 + kv[k + 1], q - k);
            take<ARG>(best[k], arg[k], v1 + kv[k], q + 1 - k);
        }
    }
    if (q <= qhi) {
        const double v0 = lds[lane + off(q)];
#pragma unroll
        for (int k = 0; k < TB; k++) take<ARG>(best[k], arg[k], v0 + kc[k - q], q - k);
    }
}

constexpr int kTB = 8;          // consecutive targets per thread
static_assert(kKinPad >= kTB - 1, "caller tables need TB - 1 entries of +inf past each end");
constexpr int kTileC = 16;      // lines per tile (16 doubles = one 128-byte line)
constexpr int kTileRP = kBlock / kTileC;
constexpr int kTileR = kTileRP * kTB;   // real targets per tile: 128

// ---------------------------------------------------------------------------
// Row sweep (axis 0, unit stride).  A block holds nr whole rows (nr * N =
// 256 * TB when N divides 2048, else one row in passes of 2048 targets) with
// a wrapped halo of H cells, in a skewed layout: element j of a row sits at
// (j + H) + (j + H) / TB, so the TB-strided reads of the blocked loop hit
// distinct banks.  The window is the widest over the block's rows, each from
// the row itself.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int skew(int x) { return x + x / kTB; }

template <int ARG, int EPI>
__global__ __launch_bounds__(kBlock) void k_row_brute(const double* __restrict__ in, double* __restrict__ out,
                                                      const double* __restrict__ kc, SweepArgs a, int H, int nr,
                                                      int RS)
{
    extern __shared__ double sm[];
    __shared__ double red[40];
    __shared__ int shw[2];
    {
        int64_t ko;
        const int64_t uo = batch_shift(a, &ko);
        in += uo;
        out += uo;
        kc += ko;
    }
    const int N = (int)a.g.n;
    const int lpr = nr > 1 ? N / kTB : kBlock;          // lanes per row
    const int rb = threadIdx.x / lpr, lr = threadIdx.x % lpr;
    const int64_t row0 = (int64_t)blockIdx.x * nr;
    const int nrow = (int)min((int64_t)nr, a.g.nlines - row0);
    const int span = N + 2 * H;

    clear_slot(a.stats_clear);
    for (int r = 0; r < nrow; r++) {
        const double* __restrict__ src = in + (row0 + r) * N;
        double* dst = sm + r * RS;
        int q = ((int)threadIdx.x - H) % N;   // source of jj = threadIdx.x, wrapped into [0, N)
        if (q < 0) q += N;
        for (int jj = threadIdx.x; jj < span; jj += kBlock) {
            dst[skew(jj)] = src[q];
            q += kBlock;
            while (q >= N) q -= N;
        }
    }
    __syncthreads();

    int wp = a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis];
    int wm = a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis + 1];
    wp = __builtin_amdgcn_readfirstlane(wp);
    wm = __builtin_amdgcn_readfirstlane(wm);
    const bool inlds = wp <= H && wm <= H;
    int amax = 0;
    double sp = -INFINITY, sn = -INFINITY, sa = 0.0, shi = -INFINITY, snlo = -INFINITY;

    const int per_pass = lpr * kTB;
    for (int i0 = 0; i0 < N; i0 += per_pass) {
        const int tbase = i0 + lr * kTB;
        double best[kTB];
        int arg[kTB];
#pragma unroll
        for (int k = 0; k < kTB; k++) {
            best[k] = INFINITY;
            arg[k] = 0;
        }
        const bool live = rb < nrow && tbase < N;
        if (inlds) {
            // lane part of the skewed address of element tbase + q
            const int lane = live ? rb * RS + (tbase / kTB) * (kTB + 1) : 0;
            blocked_loop<ARG, kTB>(sm, lane, [H](int q) { return skew(H + q); }, wp, wm, kc, best, arg);
        } else if (live) {
            const double* R = sm + rb * RS;
#pragma unroll
            for (int k = 0; k < kTB; k++) {
                int j = (tbase + k - wp) % N;
                if (j < 0) j += N;
                for (int e = -wp; e <= wm; ++e) {
                    take<1>(best[k], arg[k], R[skew(j + H)] + kc[-e], e);
                    if (++j == N) j = 0;
                }
            }
        }
        __syncthreads();   // all reads of this pass' sources done before outputs overwrite them
        // stage outputs in natural order, then store coalesced
        double* W = sm + rb * RS;
        int* A = (int*)(sm + (size_t)nr * RS) + rb * per_pass;
        if (live) {
#pragma unroll
            for (int k = 0; k < kTB; k++) {
                W[skew(lr * kTB + k)] = best[k];
                if (ARG) A[lr * kTB + k] = arg[k];
            }
        }
        __syncthreads();
        const int cnt = min(per_pass, N - i0);
        for (int t = lr; t < cnt && rb < nrow; t += lpr) {
            const int64_t idx = (row0 + rb) * N + i0 + t;
            const double x = W[skew(t)];
            double w = x;
            if (EPI) w = x - a.hv[idx];
            out[idx] = w;
            if (a.stats_out) {
                const double y = W[skew(t + 1 == N ? 0 : t + 1)];
                sp = fmax(sp, y - x);
                sn = fmax(sn, x - y);
                sa = fmax(sa, fabs(x));
                if (EPI) {
                    sa = fmax(sa, fabs(w));
                    shi = fmax(shi, w);
                    snlo = fmax(snlo, -w);
                }
            }
            if (ARG) {
                const int e = A[t];
                if (a.argmin) record_arg(a, idx, e, amax);
                // a fixed window is not a proven bound: a minimiser on or beyond its edge
                // (the blocked loop also offers offsets past it) leaves the result untrusted
                if (a.wfix > 0 && (e <= -wp || e >= wm)) atomicOr(&a.flags[0], kErrWindowEdge);
            }
        }
        if (i0 + per_pass < N) {
            // reload this row's sources for the next pass (outputs overwrote them)
            __syncthreads();
            int q = ((int)threadIdx.x - H) % N;
            if (q < 0) q += N;
            for (int jj = threadIdx.x; jj < span; jj += kBlock) {
                sm[skew(jj)] = in[row0 * N + q];
                q += kBlock;
                while (q >= N) q -= N;
            }
            __syncthreads();
        }
    }
    if (ARG && a.argmin) block_atomic_max(amax, amax_word(a));
    if (a.stats_out) {
        block_max5(sp, sn, sa, shi, snlo, red);
        if (threadIdx.x == 0) {
            stat_put(a.stats_out, a.axis, sp);
            stat_put(a.stats_out, 3 + a.axis, sn);
            stat_put(a.stats_out, 6, sa);
            if (EPI) {
                stat_put(a.stats_out, 7, shi);
                stat_put(a.stats_out, 8, snlo);
            }
        }
    }
    maybe_next_windows(a);   // after this block's own work: off the critical path
}

// ---------------------------------------------------------------------------
// Tile sweep (any axis, any stride): a block owns 16 consecutive lines and
// 128 consecutive targets; the window comes first (from the stats slot), then
// only the sources [r0 - W+, r0 + 128 + W-] are staged in LDS as [row][line]
// (16 lanes = 16 consecutive lines = one 128-byte segment).  Each thread owns
// 8 consecutive targets of one line.  Windows wider than the halo read
// sources straight from global memory.  Lanes of row group 0 also evaluate
// target r0 + Rt (the next tile's first), so the forward differences of the
// output along the axis -- the next step's window bound -- are complete.
// ---------------------------------------------------------------------------
template <int ARG, int EPI>
__global__ __launch_bounds__(kBlock) void k_tile_brute(const double* __restrict__ in, double* __restrict__ out,
                                                       const double* __restrict__ kc, SweepArgs a)
{
    extern __shared__ double sm[];
    __shared__ double red[40];
    __shared__ int shw[2];
    __shared__ double fv[kTileRP + 1][kTileC];
    {
        int64_t ko;
        const int64_t uo = batch_shift(a, &ko);
        in += uo;
        out += uo;
        kc += ko;
    }
    constexpr int C = kTileC;
    const int64_t N = a.g.n, S = a.g.stride;
    const int H = a.halo;
    const int64_t nTB = (N + kTileR - 1) / kTileR;
    const int64_t nLB = (a.g.nlines + C - 1) / C;
    const int64_t b = remap_block(blockIdx.x, nTB * nLB);
    const int64_t lb = b / nTB, tb = b % nTB;
    const int64_t r0 = tb * kTileR;
    const int Rt = (int)min((int64_t)kTileR, N - r0);   // real targets of this tile

    const int c = threadIdx.x % C;
    const int rr = threadIdx.x / C;
    const int64_t line = lb * C + c;
    const bool lv = line < a.g.nlines;
    const int64_t inner = lv ? line % S : 0, outer = lv ? line / S : 0;
    const int64_t base = inner + S * N * outer;

    clear_slot(a.stats_clear);
    const int wp = __builtin_amdgcn_readfirstlane(a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis]);
    const int wm = __builtin_amdgcn_readfirstlane(a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis + 1]);
    const bool inlds = wp <= H && wm <= H;
    if (inlds) {
        int q = (int)((r0 - wp + rr) % N);   // source of row p = H - wp + rr
        if (q < 0) q += (int)N;
        const double* __restrict__ src = in + base;
        const int Si = (int)S;
        for (int p = H - wp + rr; p <= H + kTileR + wm; p += kTileRP) {
            sm[p * C + c] = lv ? src[Si * q] : 0.0;
            q += kTileRP;
            while (q >= (int)N) q -= (int)N;
        }
        __syncthreads();
    }

    double best[kTB];
    int arg[kTB];
#pragma unroll
    for (int k = 0; k < kTB; k++) {
        best[k] = INFINITY;
        arg[k] = 0;
    }
    const int tbase = rr * kTB;
    double bnd = INFINITY;   // target r0 + Rt, evaluated by row group 0
    int bnd_arg = 0;
    if (inlds) {
        blocked_loop<ARG, kTB>(sm, tbase * C + c, [H](int q) { return (H + q) * C; }, wp, wm, kc, best, arg);
        if (rr == 0) {
            const double* col = sm + (size_t)(Rt + H) * C + c;
            for (int e = -wp; e <= wm; ++e) take<ARG>(bnd, bnd_arg, col[e * C] + kc[-e], e);
        }
    } else if (lv) {
        // window wider than the halo: every candidate from global memory
#pragma unroll
        for (int k = 0; k <= kTB; k++) {
            const int t = k < kTB ? tbase + k : Rt;
            const bool want = k < kTB ? t < Rt : rr == 0;
            double bb = INFINITY;
            int aa = 0;
            if (want) {
                int64_t j = (r0 + t - wp) % N;
                if (j < 0) j += N;
                for (int e = -wp; e <= wm; ++e) {
                    take<1>(bb, aa, in[base + S * j] + kc[-e], e);
                    if (++j == N) j = 0;
                }
            }
            // register arrays stay in registers only with compile-time indices
#pragma unroll
            for (int kk = 0; kk < kTB; kk++) {
                if (kk == k) {
                    best[kk] = bb;
                    arg[kk] = aa;
                }
            }
            if (k == kTB) bnd = bb;
        }
    }

    int amax = 0;
    if (lv) {
#pragma unroll
        for (int k = 0; k < kTB; k++) {
            const int t = tbase + k;
            if (t >= Rt) continue;
            const int64_t idx = base + S * (r0 + t);
            double w = best[k];
            if (EPI) w = w - a.hv[idx];
            out[idx] = w;
            if (ARG && a.argmin) record_arg(a, idx, arg[k], amax);
            if (ARG && a.wfix > 0 && (arg[k] <= -wp || arg[k] >= wm)) atomicOr(&a.flags[0], kErrWindowEdge);
        }
    }
    if (ARG && a.argmin) block_atomic_max(amax, amax_word(a));
    if (a.stats_out) {
        // forward differences of this sweep's output along the axis
        fv[rr][c] = best[0];
        if (rr == 0) fv[kTileRP][c] = bnd;
        __syncthreads();
        double sp = -INFINITY, sn = -INFINITY, sa = 0.0, hi = -INFINITY, nlo = -INFINITY;
        if (lv) {
            double nx[kTB];
#pragma unroll
            for (int k = 0; k + 1 < kTB; k++) nx[k] = best[k + 1];
            nx[kTB - 1] = fv[rr + 1 <= kTileRP ? rr + 1 : kTileRP][c];
#pragma unroll
            for (int k = 0; k < kTB; k++) {
                const int t = tbase + k;
                if (t >= Rt) continue;
                const double x = best[k];
                const double y = (t + 1 == Rt) ? fv[kTileRP][c] : nx[k];
                sp = fmax(sp, y - x);
                sn = fmax(sn, x - y);
                sa = fmax(sa, fabs(x));
                if (EPI) {
                    const double z = x - a.hv[base + S * (r0 + t)];
                    sa = fmax(sa, fabs(z));
                    hi = fmax(hi, z);
                    nlo = fmax(nlo, -z);
                }
            }
        }
        block_max5(sp, sn, sa, hi, nlo, red);
        if (threadIdx.x == 0) {
            stat_put(a.stats_out, a.axis, sp);
            stat_put(a.stats_out, 3 + a.axis, sn);
            stat_put(a.stats_out, 6, sa);
            if (EPI) {
                stat_put(a.stats_out, 7, hi);
                stat_put(a.stats_out, 8, nlo);
            }
        }
    }
    maybe_next_windows(a);   // after this block's own work: off the critical path
}

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------
// one block per instance
__global__ void k_clear_slots(uint64_t* stats)
{
    uint64_t* st = stats + (int64_t)blockIdx.x * kSlots * kSlotStride;
    for (int i = threadIdx.x; i < kSlots * kSlotStride; i += blockDim.x) st[i] = enc_neg_inf();
}

// The mechanical cost tau K*(s dx / tau) = ((0.5 d) d) / tau - P d, d = s dx,
// for s in [-cap, cap] at t[s + cap]: the host's evaluation order, every
// operation rounded on its own (IEEE division, no contraction), so the table
// equals the one a plan builds on the host bit for bit.
__global__ __launch_bounds__(kBlock) void k_mech_table(double* __restrict__ t, int64_t cap, double dx, double tau,
                                                       double P)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= 2 * cap;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)(i - cap) * dx;
        const double a = 0.5 * d;
        const double b = a * d;
        const double c = b / tau;
        const double e = P * d;
        t[i] = c - e;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ w, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = v;
}

// Max forward / backward difference along every axis and max |u| of u.
__global__ __launch_bounds__(kBlock) void k_stats(const double* __restrict__ u, int ndim, int64_t n0,
                                                  int64_t n1, int64_t n2, uint64_t* slot, int64_t b_u,
                                                  int64_t b_stats)
{
    __shared__ double red[40];
    u += (int64_t)blockIdx.y * b_u;      // instance blockIdx.y of a batch
    slot += (int64_t)blockIdx.y * b_stats;
    const int64_t npts = n0 * n1 * n2;
    double dp[3] = {-INFINITY, -INFINITY, -INFINITY};
    double dm[3] = {-INFINITY, -INFINITY, -INFINITY};
    double am = 0.0, hi = -INFINITY, nlo = -INFINITY;
    const int64_t nn[3] = {n0, n1, n2};
    const int64_t st[3] = {1, n0, n0 * n1};
    // grid-stride walk over the points with the coordinates (i0, i1, i2) of x
    // advanced by the stride's own coordinates (mixed-radix addition), so
    // that no point needs a division
    const int64_t G = (int64_t)gridDim.x * blockDim.x;
    const int64_t g0 = G % n0, g1 = (G / n0) % n1, g2 = G / (n0 * n1);
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t c[3] = {x % n0, (x / n0) % n1, x / (n0 * n1)};
    for (; x < npts; x += G) {
        const double v = u[x];
        am = fmax(am, fabs(v));
        hi = fmax(hi, v);
        nlo = fmax(nlo, -v);
        for (int ax = 0; ax < ndim; ax++) {
            const int64_t y = (c[ax] == nn[ax] - 1) ? x - st[ax] * (nn[ax] - 1) : x + st[ax];
            const double d = u[y] - v;
            dp[ax] = fmax(dp[ax], d);
            dm[ax] = fmax(dm[ax], -d);
        }
        c[0] += g0;
        const int64_t k0 = c[0] >= n0 ? 1 : 0;
        c[0] -= k0 * n0;
        c[1] += g1 + k0;
        const int64_t k1 = c[1] >= n1 ? 1 : 0;
        c[1] -= k1 * n1;
        c[2] += g2 + k1;
    }
    for (int ax = 0; ax < 3; ax++) {
        double t = 0.0;
        block_max3(dp[ax], dm[ax], t, red);
    }
    block_max3(am, hi, nlo, red);
    if (threadIdx.x == 0) {
        for (int ax = 0; ax < ndim; ax++) {
            stat_put(slot, ax, dp[ax]);
            stat_put(slot, 3 + ax, dm[ax]);
        }
        stat_put(slot, 6, am);
        stat_put(slot, 7, hi);
        stat_put(slot, 8, nlo);
    }
}

// The next step's windows of every axis (one block, after the step's sweeps).
// one block per instance
__global__ __launch_bounds__(kBlock) void k_windows(WinParams P, const uint64_t* slot, int* win_out, uint32_t* flags)
{
    const int64_t b = blockIdx.x;
    next_windows(P, b, slot + b * P.b_stats, win_out + b * P.b_win, flags);
}

// max(u - snap) and max(snap - u) of instance blockIdx.y
__global__ __launch_bounds__(kBlock) void k_diff_range(const double* __restrict__ u,
                                                       const double* __restrict__ snap, int64_t npts,
                                                       uint64_t* out)
{
    __shared__ double red[40];
    const int64_t b = blockIdx.y;
    u += b * npts;
    snap += b * npts;
    double hi = -INFINITY, lo = -INFINITY, t = 0.0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
         x += (int64_t)gridDim.x * blockDim.x) {
        const double d = u[x] - snap[x];
        hi = fmax(hi, d);
        lo = fmax(lo, -d);
    }
    block_max3(hi, lo, t, red);
    if (threadIdx.x == 0) {
        atomicMax((unsigned long long*)&out[2 * b], (unsigned long long)enc(hi));
        atomicMax((unsigned long long*)&out[2 * b + 1], (unsigned long long)enc(lo));
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
    __shared__ double red[40];
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
    int nr, RS, H;
    row_layout(a.g.n, a.halo, &nr, &RS, &H);
    const size_t lds = row_lds_bytes(a.g.n, a.halo);
    const int64_t G = (a.g.nlines + nr - 1) / nr;
    LO_SWEEP_LAUNCH((k_row_brute<ARG, EPI>), dim3((unsigned)G, a.nb), dim3(kBlock), lds, s, a, in, out, a.kin.k, a, H,
                    nr, RS);
    return hipGetLastError();
}

template <int ARG, int EPI>
hipError_t launch_tile(const double* in, double* out, const SweepArgs& a, hipStream_t s)
{
    const int64_t G = ((a.g.n + kTileR - 1) / kTileR) * ((a.g.nlines + kTileC - 1) / kTileC);
    LO_SWEEP_LAUNCH((k_tile_brute<ARG, EPI>), dim3((unsigned)G, a.nb), dim3(kBlock), tile_lds_bytes(a.halo), s, a, in,
                    out, a.kin.k, a);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
void row_layout(int64_t N, int halo, int* nr, int* RS, int* H)
{
    // halo rounded up to a multiple of TB, at most N
    int h = (int)std::min<int64_t>(N, (int64_t)halo);
    h = (h + kTB - 1) / kTB * kTB;
    *H = h;
    *nr = (N <= 2048 && 2048 % N == 0 && N % kTB == 0) ? (int)(2048 / N) : 1;
    const int span = (int)N + 2 * h;
    *RS = span + span / kTB + 1;
}

size_t row_lds_bytes(int64_t N, int halo)
{
    int nr, RS, H;
    row_layout(N, halo, &nr, &RS, &H);
    const int per_pass = (nr > 1 ? (int)N / kTB : kBlock) * kTB;
    return sizeof(double) * (size_t)nr * RS + sizeof(int) * (size_t)nr * per_pass;
}

size_t tile_lds_bytes(int halo) { return sizeof(double) * (size_t)(kTileR + 2 * halo + 1) * kTileC; }

hipError_t launch_windows(const WinParams& P, const uint64_t* slot, int* win_out, uint32_t* flags, int nb,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_windows, dim3(nb), dim3(kBlock), 0, s, P, slot, win_out, flags);
    return hipGetLastError();
}

hipError_t launch_clear_slots(uint64_t* stats, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_slots, dim3(nb), dim3(64), 0, s, stats);
    return hipGetLastError();
}

hipError_t launch_mech_table(double* t, int64_t cap, double dx, double tau, double P, hipStream_t s)
{
    hipLaunchKernelGGL(k_mech_table, dim3(grid_for(2 * cap + 1)), dim3(kBlock), 0, s, t, cap, dx, tau, P);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* w, int64_t n, uint32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, s, w, n, v);
    return hipGetLastError();
}

hipError_t launch_stats(const double* u, int ndim, const int64_t* n, uint64_t* slot, int nb, int64_t b_u,
                        int64_t b_stats, hipStream_t s)
{
    const int64_t n0 = n[0], n1 = ndim > 1 ? n[1] : 1, n2 = ndim > 2 ? n[2] : 1;
    // a few hundred blocks: each folds its maxima into the slot with atomics
    int g = std::min(grid_for(n0 * n1 * n2), 512);
    if (nb > 1) g = std::max(1, std::min(g, 8192 / nb));
    hipLaunchKernelGGL(k_stats, dim3(g, nb), dim3(kBlock), 0, s, u, ndim, n0, n1, n2, slot, b_u, b_stats);
    return hipGetLastError();
}

hipError_t launch_diff_range(const double* u, const double* snap, int64_t npts, int nb, uint64_t* out,
                             hipStream_t s)
{
    const int g = std::max(1, std::min(grid_for(npts), 16384 / nb));
    hipLaunchKernelGGL(k_diff_range, dim3(g, nb), dim3(kBlock), 0, s, u, snap, npts, out);
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
    if (a.fast && a.wfix <= 0) return launch_fast(in, out, a, a.cq, a.inv2c, a.pofs, s);
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
