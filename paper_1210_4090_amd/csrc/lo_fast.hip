// Fast axis sweep for the mechanical cost k(s) = c s^2 - p s
// (c = dx^2 / (2 tau), p = P dx): O(1) work per point instead of O(window).
//
// For a target t the candidate cost of source j is F_t(j) = u_j + k(t - j).
// Adjacent sources j, j+1 give equal costs at the real target
//     sigma_j = j + 1/2 + (u_{j+1} - u_j) / (2c) + p / (2c),
// j being cheaper below and j+1 above, because
//     F_t(j+1) - F_t(j) = 2c (sigma_j - t).
// The minimisers over all sources are the vertices of the lower convex hull
// of the points (j, u_j + c j^2 + p j) (the lower envelope of equal
// parabolas); a vertex owns the targets between its crossings with its two
// hull neighbours.  If a source j-1 lies above the hull edge ending at vertex
// j, its crossing with j comes no later than that edge's, and symmetrically
// on the right; so the interval (sigma_{j-1}, sigma_j] built from the grid
// neighbours alone always contains the targets a hull vertex owns.  Hence:
// every source claims the integer targets in (sigma_{j-1}, sigma_j], widened
// by 1e-6 against rounding, and each target keeps the smallest candidate
// fl(u_j + k(t - j)) among its claimants.  Sources that are not hull vertices
// only add genuine candidates (or claim nothing, where sigma decreases), so
// the minimum is the minimum over all sources -- no hull needs to be built.
// (The paper's own fast convolution, Section 4, splits u into convex and
// concave parts and merges slope sequences; this claim form is what turns
// the same convexity into independent per-source work for a wavefront.)
//
// The kept value is a genuine candidate of the definition and equals the
// exhaustive minimum except where two candidates differ by a few ulps.
// Ties are broken by a second pass that keeps the lowest claiming source
// among those attaining the minimum.  Windows beyond the staged halo fall back
// to the exhaustive window loop.
#include "lo_internal.h"
#include "lo_device.h"

#include <math.h>

namespace lo {

namespace {

using namespace dev;
constexpr int kKtPad = 4;   // staged kinetic costs cover |s| <= H + kKtPad

}  // namespace

// Layout of the dynamic LDS of the claim kernel.
struct ClaimLds {
    int arg;     // argmin array present
    int nr;      // lines per block along the sweep (row kernel: whole rows)
    int C;       // lines side by side (tile kernel: 16)
    int nt;      // targets per line (tile: R + 1, row: N)
    int H;       // halo
    int RS;      // stride of a staged line (row kernel) in doubles
};

__host__ __device__ inline size_t claim_lds_bytes(const ClaimLds& f)
{
    size_t b = 0;
    if (f.C == 1)
        b += sizeof(double) * (size_t)f.nr * f.RS;                     // sources
    else
        b += sizeof(double) * (size_t)(f.nt + 2 * f.H) * f.C;          // sources
    b += sizeof(unsigned long long) * (size_t)f.nr * f.nt * f.C;       // keys
    if (f.arg) b += sizeof(int) * (size_t)f.nr * f.nt * f.C;          // argmin sources
    b += sizeof(double) * (size_t)(2 * (f.H + kKtPad) + 1);            // staged costs
    return (b + 15) & ~(size_t)15;
}

namespace {

__device__ __forceinline__ unsigned long long kinf() { return enc(INFINITY); }

// ROW: nr whole rows of unit stride per block (window = widest of the rows'
// own bounds).  TILE: C lines x R targets (+1 extra target for the next
// step's bound), window from the stats slot, staged before the sources.
// Staged source p of line l: ROW -> U[l * RS + p], TILE -> U[p * C + l];
// key of target t of line l: ROW -> WK[l * nt + t], TILE -> WK[t * C + l].
template <int C, int ROW, int EPI, int ARG>
__global__ __launch_bounds__(kBlock) void k_claim(const double* __restrict__ in, double* __restrict__ out,
                                                  const double* __restrict__ kc, SweepArgs a, ClaimLds L,
                                                  double inv2c, double pofs)
{
    extern __shared__ double sm[];
    __shared__ double red[24];
    __shared__ int shw[4];
    constexpr double kEps = 1e-6;
    constexpr int RP = kBlock / C;     // TILE: target rows per pass
    const int H = L.H;
    const int64_t N = a.g.n, S = a.g.stride;

    int64_t r0 = 0, lb;
    int Rt, NT, nrow = 1;
    if (ROW) {
        lb = (int64_t)blockIdx.x * L.nr;
        nrow = (int)min((int64_t)L.nr, a.g.nlines - lb);
        Rt = (int)N;
        NT = (int)N;
    } else {
        const int R = a.tile_rows;
        const int64_t nTB = (N + R - 1) / R;
        const int64_t nLB = (a.g.nlines + C - 1) / C;
        const int64_t b = remap_block(blockIdx.x, nTB * nLB);
        lb = b / nTB;
        r0 = (b % nTB) * R;
        Rt = (int)min((int64_t)R, N - r0);
        NT = Rt + 1;
    }
    const int RS = L.RS;
    double* U = sm;
    unsigned long long* WK = (unsigned long long*)(sm + (ROW ? (size_t)L.nr * L.RS : (size_t)(L.nt + 2 * H) * C));
    int* AK = (int*)(WK + (size_t)L.nr * L.nt * C);
    double* KT = (double*)(AK + (ARG ? (size_t)L.nr * L.nt * C : 0));

    // TILE: every thread stays on line c = tid % C
    const int c = threadIdx.x % C, rr = threadIdx.x / C;
    int64_t tbase = 0;
    bool tok = true;
    if (!ROW) {
        const int64_t line = lb * C + c;
        tok = line < a.g.nlines;
        const int64_t ln = tok ? line : 0;
        tbase = (ln % S) + S * N * (ln / S);
    }

    clear_slot(a.stats_clear);
    const int ktn = 2 * (H + kKtPad) + 1;
    for (int i = threadIdx.x; i < ktn; i += kBlock) {
        const int s = i - (H + kKtPad);
        KT[i] = (s >= -a.kin.kcap && s <= a.kin.kcap) ? kc[s] : INFINITY;
    }
    if (ROW) {
        for (int l = 0; l < nrow; l++)
            for (int t = threadIdx.x; t < NT; t += kBlock) {
                WK[l * L.nt + t] = kinf();
                if (ARG) AK[l * L.nt + t] = 0x7fffffff;
            }
    } else {
        for (int t = rr; t < NT; t += RP) {
            WK[t * C + c] = kinf();
            if (ARG) AK[t * C + c] = 0x7fffffff;
        }
    }

    int wp, wm;
    if (ROW) {
        const int span = NT + 2 * H;
        for (int l = 0; l < nrow; l++) {
            const double* __restrict__ src = in + (lb + l) * N;
            int q = ((int)threadIdx.x - H) % (int)N;
            if (q < 0) q += (int)N;
            for (int p = threadIdx.x; p < span; p += kBlock) {
                U[l * RS + p] = src[q];
                q += kBlock;
                while (q >= N) q -= (int)N;
            }
        }
        __syncthreads();
        double dp = -INFINITY, dm = -INFINITY, am = 0.0, hi = -INFINITY, nlo = -INFINITY;
        if (a.wfix <= 0) {
            for (int l = 0; l < nrow; l++)
                for (int t = threadIdx.x; t < (int)N; t += kBlock) {
                    const double x = U[l * RS + H + t], y = U[l * RS + H + t + 1];
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
        block_window(a, nullptr, dp, dm, hi + nlo, am, shw);
        wp = __builtin_amdgcn_readfirstlane(shw[0]);
        wm = __builtin_amdgcn_readfirstlane(shw[1]);
    } else {
        block_window(a, a.stats_in, 0.0, 0.0, 0.0, 0.0, shw);
        wp = __builtin_amdgcn_readfirstlane(shw[0]);
        wm = __builtin_amdgcn_readfirstlane(shw[1]);
        if (wp <= H && wm <= H) {
            const int p0 = H - wp, p1 = H + NT - 1 + wm;
            int64_t q = (r0 - wp + rr) % N;
            if (q < 0) q += N;
            const double* __restrict__ src = in + tbase;
            for (int p = p0 + rr; p <= p1; p += RP) {
                U[p * C + c] = tok ? src[S * q] : 0.0;
                q += RP;
                while (q >= N) q -= N;
            }
        }
        __syncthreads();
    }
    const bool staged = wp <= H && wm <= H;
    const int pA = H - wp, pB = NT - 1 + H + wm;    // sources of all targets of a line
    const int kofs = H + kKtPad;

    // claim of source p of a line: targets (sigma_{p-1}, sigma_p], widened by kEps
    auto claim = [&](const double* Ul, int ustride, int p, int& tlo, int& thi) {
        const double up = Ul[p * ustride];
        const double jl = (double)(p - H);
        double slo = -INFINITY, shi = INFINITY;
        if (p > pA) slo = (jl - 0.5) + ((up - Ul[(p - 1) * ustride]) * inv2c + pofs);
        if (p < pB) shi = (jl + 0.5) + ((Ul[(p + 1) * ustride] - up) * inv2c + pofs);
        tlo = slo < -1.0 ? 0 : max(0, (int)ceil(slo - kEps));
        thi = shi > (double)NT ? NT - 1 : min(NT - 1, (int)floor(shi + kEps));
        return up;
    };

    if (staged) {
        for (int pass = 0; pass < (ARG ? 2 : 1); pass++) {
            const int nl = ROW ? nrow : 1;
            for (int l = 0; l < nl; l++) {
                const double* Ul = ROW ? U + l * RS : U + c;
                const int us = ROW ? 1 : C;
                unsigned long long* Wl = ROW ? WK + l * L.nt : WK + c;
                int* Al = ROW ? AK + l * L.nt : AK + c;
                const int ws = ROW ? 1 : C;
                const int step = ROW ? kBlock : RP;
                for (int p = pA + (ROW ? (int)threadIdx.x : rr); p <= pB; p += step) {
                    int tlo, thi;
                    const double up = claim(Ul, us, p, tlo, thi);
                    for (int t = tlo; t <= thi; t++) {
                        const int s = t - (p - H);
                        if (s < -(H + kKtPad) || s > H + kKtPad) continue;
                        const unsigned long long key = enc(up + KT[s + kofs]);
                        if (pass == 0)
                            atomicMin(&Wl[t * ws], key);
                        else if (key == Wl[t * ws])
                            atomicMin(&Al[t * ws], p);
                    }
                }
            }
            __syncthreads();
        }
    } else {
        // ---- fallback: exhaustive window ----
        const int nl = ROW ? nrow : 1;
        for (int l = 0; l < nl; l++) {
            const int step = ROW ? kBlock : RP;
            for (int t = ROW ? (int)threadIdx.x : rr; t < NT; t += step) {
                double best = INFINITY;
                int arg = 0;
                if (ROW || tok) {
                    int64_t j = (r0 + t - wp) % N;
                    if (j < 0) j += N;
                    for (int e = -wp; e <= wm; ++e) {
                        const double v = (ROW ? U[l * RS + H + (int)j] : in[tbase + S * j]) + kc[-e];
                        if (v < best) {
                            best = v;
                            arg = e;
                        }
                        if (++j == N) j = 0;
                    }
                }
                const int k = ROW ? l * L.nt + t : t * C + c;
                WK[k] = enc(best);
                if (ARG) AK[k] = t + arg + H;
            }
        }
        __syncthreads();
    }

    // ---- outputs, argmins, stats of this sweep's result ----
    double sp = -INFINITY, sn = -INFINITY, sa = 0.0, hi = -INFINITY, nlo = -INFINITY;
    int amax = 0;
    bool bad = false;
    const int nl = ROW ? nrow : 1;
    for (int l = 0; l < nl; l++) {
        if (!ROW && !tok) break;
        const int step = ROW ? kBlock : RP;
        const int64_t lbase = ROW ? (lb + l) * N : tbase;
        const int64_t sstride = ROW ? 1 : S;
        for (int t = ROW ? (int)threadIdx.x : rr; t < Rt; t += step) {
            const int k = ROW ? l * L.nt + t : t * C + c;
            const double x = dec(WK[k]);
            bad |= !(x < INFINITY);
            const int64_t idx = lbase + sstride * (r0 + t);
            double z = x;
            if (EPI) z = x - a.hv[idx];
            out[idx] = z;
            if (ARG && a.argmin) {
                const int e = AK[k] - H - t;
                a.argmin[idx] = (int16_t)e;
                amax = max(amax, abs(e));
            }
            if (!ROW && a.stats_out) {
                const double y = dec(WK[k + C]);
                sp = fmax(sp, y - x);
                sn = fmax(sn, x - y);
                sa = fmax(sa, fabs(x));
                if (EPI) {
                    sa = fmax(sa, fabs(z));
                    hi = fmax(hi, z);
                    nlo = fmax(nlo, -z);
                }
            }
        }
    }
    if (bad) atomicOr(&a.flags[0], kErrFastPath);
    if (ARG && a.argmin) {
        amax = (int)wave_max((double)amax);
        if (threadIdx.x % kWave == 0) atomicMax(&a.flags[4 + a.axis], (uint32_t)amax);
    }
    if (!ROW && a.stats_out) {
        block_max3(sp, sn, sa, red);
        if (EPI) {
            double t = 0.0;
            block_max3(hi, nlo, t, red);
        }
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
}

template <int C, int ROW>
hipError_t launch_claim_t(const double* in, double* out, const SweepArgs& a, const ClaimLds& L, double inv2c,
                          double pofs, int64_t grid, hipStream_t s)
{
    const size_t lds = claim_lds_bytes(L);
    const bool arg = a.argmin != nullptr;
    const bool epi = a.hv != nullptr;
#define LO_CLAIM_LAUNCH(E, A)                                                                              \
    hipLaunchKernelGGL((k_claim<C, ROW, E, A>), dim3((unsigned)grid), dim3(kBlock), lds, s, in, out,       \
                       a.kin.k, a, L, inv2c, pofs)
    if (epi) {
        if (arg) LO_CLAIM_LAUNCH(1, 1);
        else LO_CLAIM_LAUNCH(1, 0);
    } else {
        if (arg) LO_CLAIM_LAUNCH(0, 1);
        else LO_CLAIM_LAUNCH(0, 0);
    }
#undef LO_CLAIM_LAUNCH
    return hipGetLastError();
}

ClaimLds claim_layout(int kind, int64_t N, int tile_rows, int H, bool arg)
{
    ClaimLds L;
    L.arg = arg ? 1 : 0;
    L.H = H;
    if (kind == kKindRow) {
        L.C = 1;
        L.nt = (int)N;
        L.nr = (N <= 2048 && 2048 % N == 0) ? (int)(2048 / N) : 1;
        L.RS = (int)N + 2 * H + 1;
    } else {
        L.C = 16;
        L.nt = tile_rows + 1;
        L.nr = 1;
        L.RS = 0;
    }
    return L;
}

}  // namespace

size_t fast_lds_for(int kind, int64_t N, int tile_rows, int H)
{
    return claim_lds_bytes(claim_layout(kind, N, tile_rows, H, false));
}

hipError_t launch_fast(const double* in, double* out, const SweepArgs& a, double cq, double inv2c, double pofs,
                       hipStream_t s)
{
    (void)cq;
    const ClaimLds L = claim_layout(a.kind, a.g.n, a.tile_rows, a.halo, a.argmin != nullptr);
    if (a.kind == kKindRow)
        return launch_claim_t<1, 1>(in, out, a, L, inv2c, pofs, (a.g.nlines + L.nr - 1) / L.nr, s);
    const int64_t G = ((a.g.n + a.tile_rows - 1) / a.tile_rows) * ((a.g.nlines + 15) / 16);
    return launch_claim_t<16, 0>(in, out, a, L, inv2c, pofs, G, s);
}

}  // namespace lo
