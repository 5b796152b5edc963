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
    b += sizeof(double) * (size_t)f.nr * f.nt * f.C;                   // best candidate per target
    if (f.arg) b += sizeof(int) * (size_t)f.nr * f.nt * f.C;          // argmin sources
    b += sizeof(double) * (size_t)(2 * (f.H + kKtPad) + 1);            // staged costs
    return (b + 15) & ~(size_t)15;
}

namespace {

// ROW: nr whole rows of unit stride per block, 256/nr threads per row.
// TILE: C lines x R targets (+1 extra target for the next step's bound).
// Staged source p of line l: ROW -> U[l * RS + p], TILE -> U[p * C + l];
// key of target t of line l: ROW -> WK[l * nt + t], TILE -> WK[t * C + l].
// Each thread walks a contiguous run of sources of its line, so each u value
// is read once and each crossing sigma is computed once.
template <int C, int ROW, int EPI, int ARG>
__global__ __launch_bounds__(kBlock) void k_claim(const double* __restrict__ in, double* __restrict__ out,
                                                  const double* __restrict__ kc, SweepArgs a, ClaimLds L,
                                                  double inv2c, double pofs)
{
    extern __shared__ double sm[];
    __shared__ double red[40];
    constexpr double kEps = 1e-6;
    {
        int64_t ko;
        const int64_t uo = batch_shift(a, &ko);
        in += uo;
        out += uo;
        kc += ko;
        if (a.pofs_b) pofs = a.pofs;
    }
    const int H = L.H;
    const int N = (int)a.g.n;
    const int S = (int)a.g.stride;   // line offsets fit 32 bits (the plan caps the grid at 2^31 points)

    // ---- geometry ----
    int64_t r0 = 0, lb;
    int Rt, NT, nrow = 1;
    if (ROW) {
        lb = (int64_t)blockIdx.x * L.nr;
        nrow = (int)min((int64_t)L.nr, a.g.nlines - lb);
        Rt = N;
        NT = N;
    } else {
        const int R = a.tile_rows;
        const int64_t nTB = (N + R - 1) / R;
        const int64_t nLB = (a.g.nlines + C - 1) / C;
        const int64_t b = remap_block(blockIdx.x, nTB * nLB);
        lb = b / nTB;
        r0 = (b % nTB) * R;
        Rt = (int)min((int64_t)R, (int64_t)N - r0);
        NT = Rt + 1;
    }
    // a thread's line and its rank among the threads of that line
    const int tpl = ROW ? kBlock / L.nr : kBlock / C;         // threads per line
    const int l = ROW ? (int)threadIdx.x / tpl : (int)threadIdx.x % C;
    const int lt = ROW ? (int)threadIdx.x % tpl : (int)threadIdx.x / C;
    int64_t lbase;
    bool lok;
    if (ROW) {
        lok = l < nrow;
        lbase = (lb + (lok ? l : 0)) * (int64_t)N;
    } else {
        const int64_t line = lb * C + l;
        lok = line < a.g.nlines;
        const int64_t ln = lok ? line : 0;
        lbase = (ln % S) + S * N * (ln / S);
    }
    const int us = ROW ? 1 : C;                                 // stride of a line's sources in U
    double* U = sm;
    double* WK = sm + (ROW ? (size_t)L.nr * L.RS : (size_t)(L.nt + 2 * H) * C);
    int* AK = (int*)(WK + (size_t)L.nr * L.nt * C);
    double* KT = (double*)(AK + (ARG ? (size_t)L.nr * L.nt * C : 0));
    double* Ul = ROW ? U + (size_t)(lok ? l : 0) * L.RS : U + l;
    double* Wl = ROW ? WK + (size_t)(lok ? l : 0) * L.nt : WK + l;
    int* Al = ROW ? AK + (size_t)(lok ? l : 0) * L.nt : AK + l;

    clear_slot(a.stats_clear);
    int wp, wm;
    if (a.wfix > 0) {
        wp = wm = a.wfix;
    } else {
        wp = a.win_in[2 * a.axis];
        wm = a.win_in[2 * a.axis + 1];
    }
    wp = __builtin_amdgcn_readfirstlane(wp);
    wm = __builtin_amdgcn_readfirstlane(wm);
    const bool staged = wp <= H && wm <= H;
    const int pA = H - wp, pB = NT - 1 + H + wm;    // sources of all targets of a line

    // ---- stage costs, clear keys, stage sources ----
    const int ktn = 2 * (H + kKtPad) + 1;
    for (int i = threadIdx.x; i < ktn; i += kBlock) {
        const int s = i - (H + kKtPad);
        KT[i] = (s >= -a.kin.kcap && s <= a.kin.kcap) ? kc[s] : INFINITY;
    }
    for (int t = lt; t < NT; t += tpl) {
        Wl[t * us] = INFINITY;
        if (ARG) Al[t * us] = 0x7fffffff;
    }
    if (lok) {
        // ROW stages the whole wrapped line [-H, N + H); TILE only the window's sources
        const int p0 = ROW ? 0 : (staged ? pA : 0), p1 = ROW ? N + 2 * H - 1 : (staged ? pB : -1);
        int q = (int)((r0 - H + p0 + lt) % N);
        if (q < 0) q += N;
        const double* __restrict__ src = in + lbase;
        for (int p = p0 + lt; p <= p1; p += tpl) {
            Ul[p * us] = src[S * q];
            q += tpl;
            while (q >= N) q -= N;
        }
    }
    __syncthreads();

    const int kofs = H + kKtPad;
    if (staged) {
        // ---- claims: source p offers itself to the targets in (sigma_{p-1}, sigma_p] ----
        const int np = pB - pA + 1;
        int ch = (np + tpl - 1) / tpl;
        ch |= 1;   // odd run length: the runs' first sources fall on distinct LDS banks
        const int q0 = pA + lt * ch, q1 = min(q0 + ch, pB + 1);
        for (int pass = 0; pass < (ARG ? 2 : 1); pass++) {
            if (lok && q0 < q1) {
                double ucur = Ul[q0 * us];
                double jl = (double)(q0 - H);
                double slo = -INFINITY;
                if (q0 > pA) slo = (jl - 0.5) + ((ucur - Ul[(q0 - 1) * us]) * inv2c + pofs);
                for (int p = q0; p < q1; p++) {
                    double unext = 0.0, shi = INFINITY;
                    if (p < pB) {
                        unext = Ul[(p + 1) * us];
                        shi = (jl + 0.5) + ((unext - ucur) * inv2c + pofs);
                    }
                    const int tlo = slo < -1.0 ? 0 : max(0, (int)ceil(slo - kEps));
                    const int thi = shi > (double)NT ? NT - 1 : min(NT - 1, (int)floor(shi + kEps));
                    for (int t = tlo; t <= thi; t++) {
                        const int s = t - (p - H);
                        if ((unsigned)(s + kofs) > (unsigned)(2 * kofs)) continue;
                        const double v = ucur + KT[s + kofs];
                        if (pass == 0)
                            atomicMin(&Wl[t * us], v);
                        else if (v == Wl[t * us])
                            atomicMin(&Al[t * us], p);
                    }
                    slo = shi;
                    ucur = unext;
                    jl += 1.0;
                }
            }
            __syncthreads();
        }
    } else {
        // ---- fallback: exhaustive window (ROW: wrapped staged line, TILE: global) ----
        for (int t = lt; t < NT && lok; t += tpl) {
            double best = INFINITY;
            int arg = 0;
            int j = (int)((r0 + t - wp) % N);
            if (j < 0) j += N;
            for (int e = -wp; e <= wm; ++e) {
                const double v = (ROW ? Ul[H + j] : in[lbase + S * j]) + kc[-e];
                if (v < best) {
                    best = v;
                    arg = e;
                }
                if (++j == N) j = 0;
            }
            Wl[t * us] = best;
            if (ARG) Al[t * us] = t + arg + H;
        }
        __syncthreads();
    }

    // ---- outputs, argmins, stats of this sweep's result ----
    double sp = -INFINITY, sn = -INFINITY, sa = 0.0, hi = -INFINITY, nlo = -INFINITY;
    int amax = 0;
    bool bad = false;
    if (lok) {
        double* __restrict__ dst = out + lbase + S * r0;
        const double* __restrict__ hv = EPI ? a.hv + lbase + S * r0 : nullptr;
        int16_t* am = (ARG && a.argmin) ? a.argmin + lbase + S * r0 : nullptr;
        for (int t = lt; t < Rt; t += tpl) {
            const double x = Wl[t * us];
            bad |= !(x < INFINITY);
            double z = x;
            if (EPI) z = x - hv[S * t];
            dst[S * t] = z;
            if (ARG && am) {
                const int e = Al[t * us] - H - t;
                am[S * t] = (int16_t)e;
                amax = max(amax, abs(e));
            }
            if (a.stats_out) {
                // next target: TILE has the extra one, ROW wraps
                const double y = Wl[(ROW && t + 1 == N ? 0 : t + 1) * us];
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
    if (a.stats_out) {
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
}

template <int C, int ROW>
hipError_t launch_claim_t(const double* in, double* out, const SweepArgs& a, const ClaimLds& L, double inv2c,
                          double pofs, int64_t grid, hipStream_t s)
{
    const size_t lds = claim_lds_bytes(L);
    const bool arg = a.argmin != nullptr;
    const bool epi = a.hv != nullptr;
#define LO_CLAIM_LAUNCH(E, A)                                                                              \
    hipLaunchKernelGGL((k_claim<C, ROW, E, A>), dim3((unsigned)grid, a.nb), dim3(kBlock), lds, s, in, out, \
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
        // several short rows per block: a power of two (threads per row = 256 / nr)
        L.nr = 1;
        while (L.nr < 32 && (int64_t)L.nr * 2 * N <= 2048) L.nr *= 2;
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
