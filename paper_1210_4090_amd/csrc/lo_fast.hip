// Fast axis sweep: O(1) work per point for the mechanical cost
// k(s) = c s^2 - p s (c = dx^2 / (2 tau), p = P dx), O(log window) for any
// convex cost table.
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
// fl(u_j + k(t - j)) among its claimants (an LDS atomic minimum on doubles).
// Sources that are not hull vertices only add genuine candidates (or claim
// nothing, where sigma decreases), so the minimum is the minimum over all
// sources -- no hull needs to be built.  For a convex table the same holds
// with the crossing found by bisection: j is no worse than j + 1 at offset s
// exactly when k(s) - k(s-1) <= u_{j+1} - u_j, a condition monotone in s.
// (The paper's own fast convolution, Section 4, splits u into convex and
// concave parts and merges slope sequences; this claim form is what turns the
// same convexity into independent per-source work for a wavefront.)
//
// A minimiser lies within the step's window, so claims are clipped to it; a
// clipped candidate is never the minimum.  Costs come from a band of 2 KH + 1
// consecutive offsets of the table staged in LDS, centred on the cost's
// vertex (P tau / dx for the mechanical cost, a caller table's minimising
// offset), which is known before the window is read, so the band's loads go
// out first.  A large |P| shifts the minimisers, and the window with them,
// towards the vertex's side; KH (the plan's halo plus the vertex's distance
// from 0) then covers the window whenever its width fits.  A wider window is
// claimed band by band, restaging the table between bands (minima over the
// union of the candidates are the same), in chunks of two sources so that
// this rare path needs fewer registers than the main one.  The kept value is
// a genuine candidate of the definition and equals the exhaustive minimum
// except where two candidates differ by a few ulps (never, for a table: its
// comparisons are widened in value).  Ties are broken by a second pass that
// keeps the smallest offset (lowest lifted source) among the claimants
// attaining the minimum.  Row sweeps whose window reaches a whole row fall
// back to the exhaustive loop.
//
// Work layout: a thread takes chunks of kCh consecutive sources of one line,
// loads the kCh + 2 values around them once, and computes every crossing once.
//  - ROW kernel (axis 0, N a multiple of 8, N <= 2048): each thread owns 8
//    (or 4) consecutive points of a row (16-byte loads and stores), keys in
//    LDS in a skewed layout (x -> x + x/8, so chunk-strided lanes hit distinct
//    banks); claims wrap around the row, so no halo is read; persistent
//    blocks.
//  - TILE kernel (other axes): 16 lines side by side x R targets (one line x
//    4R targets for an axis with fewer than 16 lines); sources come straight
//    from global memory (16 adjacent lines = 128 contiguous bytes per
//    source), only the keys and the cost band live in LDS.
#include "lo_internal.h"
#include "lo_device.h"

#include <math.h>

#include <algorithm>
#include <type_traits>


namespace lo {

namespace {

using namespace dev;
constexpr int kCh = 8;           // sources per chunk (tile kernel)
constexpr int kRowPoints = 2048; // row kernel: points per tile (points per thread x threads)
constexpr int kTileLines = 16;   // TILE: lines side by side (1 for axes with fewer lines)
// TILE with the potential step: each thread prefetches tau V for its R / (BS / 16)
// outputs (16 or 8 in blocks of 256 threads, 4 or 8 in blocks of 512 threads)
constexpr double kEps = 1e-6;    // claim widening, in cells

// skewed LDS slot of key x >= 0 for chunks of CH points: one pad slot per
// chunk, so lanes that walk chunk-strided keys hit distinct banks
template <int CH>
__device__ __forceinline__ int skc(int x) { return x + (int)((unsigned)x / CH); }

// An output store, written through the L2 at agent scope when WT (a grid
// that fits the caches: the kernel's end then has little to write back).
// The tile kernels' stores cover whole cache lines (16 adjacent lines, or
// consecutive targets), which is what makes writing through cheap.
template <bool WT>
__device__ __forceinline__ void put(double* p, double v)
{
    if constexpr (WT)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

}  // namespace

// TILE key row stride in doubles: one pad slot per row of 16 lines (distinct
// banks for the lines), none for a single line.
__host__ __device__ constexpr int tile_key_stride(int C) { return C == 1 ? 1 : C + 1; }

// Layout of the dynamic LDS of the claim kernels.
struct ClaimLds {
    int arg;     // argmin array present
    int row;     // ROW (1) or TILE (0)
    int nr;      // ROW: rows per tile
    int RS;      // ROW: skewed key slots of a tile
    int NT;      // TILE: targets per line (R + 1)
    int C;       // TILE: lines side by side (kTileLines, or 1)
    int KH;      // staged cost table: a band of 2 KH + 1 offsets
};

__host__ __device__ inline size_t claim_lds_bytes(const ClaimLds& f)
{
    size_t b = sizeof(double) * (size_t)(2 * f.KH + 1);                    // costs
    if (f.row) {
        b += sizeof(double) * (size_t)f.RS;                                   // keys
        if (f.arg) b += sizeof(int) * (size_t)f.RS;                           // argmins
    } else {
        b += sizeof(double) * (size_t)f.NT * tile_key_stride(f.C);           // keys
        if (f.arg) b += sizeof(int) * (size_t)f.NT * tile_key_stride(f.C);
    }
    return (b + 15) & ~(size_t)15;
}

namespace {

// Largest s in [sl, sh] with K[s] - K[s - 1] <= D, or sl - 1 if there is none
// (K covers [sl - 1, sh]; its differences are nondecreasing: a convex cost).
__device__ __forceinline__ int table_cross(const double* K, int sl, int sh, double D)
{
    int lo = sl - 1, hi = sh;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (K[mid] - K[mid - 1] <= D)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Claims of one chunk: sources p0 .. min(p0 + kCh - 1, plast) (lifted) of one
// line with uu[k] = u(p0 - 1 + k), k = 0 .. kCh + 1.  Targets are clipped to
// [tmin, tmax] (lifted) and to t - p in [smin, smax], a range the staged cost
// table K (K[s] = k(s), in LDS) covers; key(t) gives the LDS slot of lifted
// target t.  PASS 0: atomic minimum of the candidate into W; PASS 1: among
// the candidates equal to W, atomic minimum of the offset (source - target)
// into A.
//
// Crossings.  Mechanical cost (GEN false): the parabolas of sources j and
// j + 1 cross at sigma = j + 1/2 + (u(j+1) - u(j)) / (2c) + P tau / dx, widened
// by kEps cells.  Any convex table (GEN true; K must also cover smin - 1):
// source j is no worse than j + 1 at offset s exactly when
// k(s) - k(s - 1) <= u(j+1) - u(j), a monotone condition found by bisection
// over the staged differences, with the comparison widened by
// gsl + 2^-40 (|u(j)| + |u(j+1)|), far above the rounding of the candidates,
// so that every minimiser (ties included) stays among the claimants.
template <int PASS, int CH, bool GEN, typename KeyOf, bool U2 = false>
__device__ __forceinline__ void claim_chunk(const double (&uu)[CH + 2], int p0, int plast, int tmin, int tmax,
                                            int smin, int smax, const double* K, double inv2c, double pofs,
                                            double gsl, double* W, int* A, KeyOf key)
{
    // crossing k lies between sources p0 - 1 + k and p0 + k
    int lo[CH + 1], hi[CH + 1];
    if (GEN) {
#pragma unroll
        for (int k = 0; k <= CH; k++) {
            const int j = p0 - 1 + k;
            const double D = uu[k + 1] - uu[k];
            const double dl = gsl + 0x1p-40 * (fabs(uu[k]) + fabs(uu[k + 1]));
            const int sp = table_cross(K, smin, smax, D + dl);
            const int sm = (sp >= smin && K[sp] - K[sp - 1] > D - dl) ? table_cross(K, smin, sp, D - dl) : sp;
            lo[k] = j + sm;   // source p0 + k claims from lo[k] + 1
            hi[k] = j + sp;   // source p0 - 1 + k claims up to hi[k]
        }
    } else {
        double jh = (double)p0 - 0.5;
#pragma unroll
        for (int k = 0; k <= CH; k++) {
            const double sg = jh + ((uu[k + 1] - uu[k]) * inv2c + pofs);
            lo[k] = (int)floor(sg - kEps);   // source p0 + k claims from lo[k] + 1
            hi[k] = (int)floor(sg + kEps);   // source p0 - 1 + k claims up to hi[k]
            jh += 1.0;
        }
    }
    auto claim = [&](int p, int t, double v) {
        const int s = key(t);
        if (PASS == 0)
            atomicMin(&W[s], v);
        else if (v == W[s])
            atomicMin(&A[s], p - t);
    };
#pragma unroll
    for (int k = 0; k < CH; k++) {
        const int p = p0 + k;
        if (p > plast) break;
        const int tlo = max(max(lo[k], p + smin - 1), tmin - 1) + 1;
        const int thi = min(min(hi[k + 1], p + smax), tmax);
        const double up = uu[k + 1];
        if (U2 && tlo <= thi) {
            // U2: a source claims one or two targets in the common case: both
            // costs are read at once (the second lies in the staged band, or
            // is the word just past it when tlo = thi), the rest in a loop
            const double k0 = K[tlo - p], k1 = K[tlo + 1 - p];
            claim(p, tlo, up + k0);
            if (tlo < thi) claim(p, tlo + 1, up + k1);
            for (int t = tlo + 2; t <= thi; t++) claim(p, t, up + K[t - p]);
        } else if (!U2) {
            for (int t = tlo; t <= thi; t++) claim(p, t, up + K[t - p]);
        }
    }
}

// Fold the forward differences of a run of outputs into the statistics.
struct SweepStats {
    double sp = -INFINITY, sn = -INFINITY, sa = 0.0, hi = -INFINITY, nlo = -INFINITY;
};

template <int EPI>
__device__ __forceinline__ void fold_stats(SweepStats& st, double x, double y, double z)
{
    const double d = y - x;
    st.sp = fmax(st.sp, d);
    st.sn = fmax(st.sn, -d);
    st.sa = fmax(st.sa, fabs(x));
    if (EPI) {
        st.sa = fmax(st.sa, fabs(z));
        st.hi = fmax(st.hi, z);
        st.nlo = fmax(st.nlo, -z);
    }
}

template <int EPI>
__device__ __forceinline__ void publish_stats(SweepStats& st, const SweepArgs& a, double* red)
{
    if (!a.stats_out) return;
    block_max5_to0(st.sp, st.sn, st.sa, st.hi, st.nlo, red);
    if (threadIdx.x == 0) {
        stat_put(a.stats_out, a.axis, st.sp);
        stat_put(a.stats_out, 3 + a.axis, st.sn);
        stat_put(a.stats_out, 6, st.sa);
        if (EPI) {
            stat_put(a.stats_out, 7, st.hi);
            stat_put(a.stats_out, 8, st.nlo);
        }
    }
}

// ---------------------------------------------------------------------------
// ROW kernel (axis 0, N a multiple of 8, N <= 2048): a tile is nr whole rows
// (nr N <= 2048 points); thread (r, j) owns points 8j .. 8j + 7 of row r of
// the tile: it loads them with 16-byte loads, claims for them as sources and
// writes them as targets.  Keys live in LDS in the skewed layout; claims wrap
// around the row.  Persistent: a block walks tiles blockIdx.x, + gridDim.x, ...
// The plain sweep (no epilogue, no argmins) is held to 128 registers (it fits
// without spilling): four waves a SIMD.
// ---------------------------------------------------------------------------
template <int EPI, int ARG, int CH, int BS, bool GEN>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(CH == 8 && !ARG && !EPI && !GEN ? 4 : 1))) void
k_claim_row(const double* __restrict__ in, double* __restrict__ out, const double* __restrict__ kc, SweepArgs a,
            ClaimLds L, double inv2c, double pofs)
{
    extern __shared__ double sm[];
    __shared__ double red[40];
    {
        int64_t ko;
        const int64_t uo = batch_shift(a, &ko);
        in += uo;
        out += uo;
        kc += ko;
        if (a.pofs_b) pofs = a.pofs;
    }
    const int N = (int)a.g.n;
    const int KH = L.KH, nr = L.nr;
    const int cpr = N / CH;                       // chunks per row
    const int r = (int)threadIdx.x / cpr;         // row of this thread within a tile
    const int p0 = ((int)threadIdx.x - r * cpr) * CH;
    const bool act = r < nr;
    const int g0 = r * N + p0;                    // first key of this thread (unskewed)
    const int gs = skc<CH>(g0);                   // its slot: g0 is a multiple of CH, so key g0 + k is at gs + k
    double* KT = sm;
    double* W = KT + (2 * KH + 1);
    int* A = (int*)(W + L.RS);

    // The cost band does not depend on the window (it is centred on the
    // cost's vertex): its loads are issued before the window is read, so that
    // the two latencies overlap.
    // KT[i] = k(sb + i), i < 2 KH + 1: offsets [vertex - KH - g, vertex + KH - g]
    // (a convex table's crossings also read k(smin - 1))
    const int kcap = (int)min((int64_t)a.kin.kcap, (int64_t)0x7fffffff);
    const int g = GEN ? 1 : 0;
    const int vtx = GEN ? a.kvert : (int)floor(pofs + 0.5);
    const int sb = vtx - KH - g;
    constexpr int kKtRegs = (2 * 512 + 1 + BS - 1) / BS;   // the band has at most 2 * 512 + 1 entries
    double ktv[kKtRegs];
#pragma unroll
    for (int j = 0; j < kKtRegs; j++) {
        const int i = (int)threadIdx.x + j * BS;
        const int s = sb + i;
        ktv[j] = (i < 2 * KH + 1 && s >= -kcap && s <= kcap) ? kc[s] : INFINITY;
    }
    const int64_t ntiles = (a.g.nlines + nr - 1) / nr;

    clear_slot(a.stats_clear);
    int wp = a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis];
    int wm = a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis + 1];
    wp = __builtin_amdgcn_readfirstlane(wp);
    wm = __builtin_amdgcn_readfirstlane(wm);
#pragma unroll
    for (int j = 0; j < kKtRegs; j++) {
        const int i = (int)threadIdx.x + j * BS;
        if (i < 2 * KH + 1) KT[i] = ktv[j];
    }
    // the minimisers of the step lie within its window: claims are clipped to
    // t - p in [-wm - 1, wp + 1] (offsets beyond the table's end cost +inf and
    // never win)
    const int smin = max(-wm - 1, -kcap), smax = min(wp + 1, kcap);
    // claims wrap once around the row (targets t of sources 0 .. N - 1 lie in
    // [smin, N - 1 + smax]); the main path needs the window inside the band
    const bool wraps = wp + 1 < N && wm + 1 < N;
    const bool fast = wraps && smin - g >= sb && smax <= sb + 2 * KH;
    const double* K = KT - sb;   // K[s] = k(s), s in [sb, sb + 2 KH]
    const double gsl = a.kslack;
    const int kbase = r * N;
    auto key = [N, kbase](int t) { return skc<CH>(kbase + (t < 0 ? t + N : (t >= N ? t - N : t))); };

    SweepStats st;
    int amax = 0;
    bool bad = false;
    // outputs, argmins and statistics of one tile row from the keys
    auto emit = [&](int64_t row, bool ok) {
        if (!ok) return;
        double x[CH + 1];
#pragma unroll
        for (int k = 0; k < CH; k++) x[k] = W[gs + k];
        x[CH] = W[skc<CH>(kbase + (p0 + CH == N ? 0 : p0 + CH))];
        double z[CH];
        if (EPI) {
            const double2* h2 = (const double2*)(a.hv + row * N + p0);
#pragma unroll
            for (int k = 0; k < CH / 2; k++) {
                const double2 v = h2[k];
                z[2 * k] = x[2 * k] - v.x;
                z[2 * k + 1] = x[2 * k + 1] - v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < CH; k++) z[k] = x[k];
        }
        double2* d2 = (double2*)(out + row * N + p0);
#pragma unroll
        for (int k = 0; k < CH / 2; k++) d2[k] = make_double2(z[2 * k], z[2 * k + 1]);
#pragma unroll
        for (int k = 0; k < CH; k++) {
            bad |= !(x[k] < INFINITY);
            if (a.stats_out) fold_stats<EPI>(st, x[k], x[k + 1], z[k]);
        }
        if (ARG && a.argmin) {
            int16_t* am = a.argmin + row * N + p0;
#pragma unroll
            for (int k = 0; k < CH; k++) {
                const int e = A[gs + k];
                am[k] = (int16_t)e;
                amax = max(amax, abs(e));
            }
        }
    };
    if (wraps && !fast) {
        // window wider than the band: band by band, chunks of two sources, in a
        // loop of its own (its registers stay apart from the main loop's)
        for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
            const int64_t row = tile * nr + r;
            const bool ok = act && row < a.g.nlines;
            const double* __restrict__ src = in + row * N;
            if (ok) {
#pragma unroll
                for (int k = 0; k < CH; k++) {
                    W[gs + k] = INFINITY;
                    if (ARG) A[gs + k] = 0x7fffffff;
                }
            }
            for (int pass = 0; pass < (ARG ? 2 : 1); pass++) {
                for (int blo = smin; blo <= smax; blo += max(2 * KH + 1 - g, 1)) {
                    const int bhi = min(blo + max(2 * KH - g, 0), smax);
                    __syncthreads();
                    for (int i = threadIdx.x; i < 2 * KH + 1; i += BS) {
                        const int s = blo - g + i;
                        KT[i] = (s >= -kcap && s <= kcap) ? kc[s] : INFINITY;
                    }
                    __syncthreads();
                    if (ok) {
#pragma unroll 1
                        for (int k = 0; k < CH; k += 2) {
                            // reloaded (not the registers above): keeps this path's registers low
                            double u4[4];
                            int j = p0 + k == 0 ? N - 1 : p0 + k - 1;
#pragma unroll
                            for (int i = 0; i < 4; i++) {
                                u4[i] = src[j];
                                j = j + 1 == N ? 0 : j + 1;
                            }
                            if (pass == 0)
                                claim_chunk<0, 2, GEN>(u4, p0 + k, N - 1, smin, N - 1 + smax, blo, bhi,
                                                       KT - (blo - g), inv2c, pofs, gsl, W, A, key);
                            else
                                claim_chunk<1, 2, GEN>(u4, p0 + k, N - 1, smin, N - 1 + smax, blo, bhi,
                                                       KT - (blo - g), inv2c, pofs, gsl, W, A, key);
                        }
                    }
                }
                __syncthreads();
            }
            emit(row, ok);
            __syncthreads();   // keys are reused by the next tile
        }
    } else {
        // this thread's sources of a tile: points p0 - 1 .. p0 + CH of its row
        auto load_src = [&](int64_t tile, double (&v)[CH + 2]) {
            const int64_t row = tile * nr + r;
            if (act && row < a.g.nlines) {
                const double* __restrict__ q = in + row * N;
                v[0] = q[p0 == 0 ? N - 1 : p0 - 1];
                const double2* q2 = (const double2*)(q + p0);
#pragma unroll
                for (int k = 0; k < CH / 2; k++) {
                    const double2 w = q2[k];
                    v[1 + 2 * k] = w.x;
                    v[2 + 2 * k] = w.y;
                }
                v[CH + 1] = q[p0 + CH == N ? 0 : p0 + CH];
            }
        };
        // 8 points a thread: a block's next tile's sources are loaded right
        // after the claims of its current one, so that their latency passes
        // during the emit (2048^2 row sweep 19.8 -> 19.3 us; with 4 points a
        // thread, twice the waves already hide it, and the 3-D and batched
        // row sweeps got 2-4% slower)
        constexpr bool kNextSrc = CH == 8;
        double uu[CH + 2];
        if (kNextSrc && blockIdx.x < ntiles) load_src(blockIdx.x, uu);
        for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
            const int64_t row = tile * nr + r;
            const bool ok = act && row < a.g.nlines;
            const double* __restrict__ src = in + row * N;
            if (!kNextSrc) load_src(tile, uu);
            if (ok) {
#pragma unroll
                for (int k = 0; k < CH; k++) {
                    W[gs + k] = INFINITY;
                    if (ARG) A[gs + k] = 0x7fffffff;
                }
            }
            __syncthreads();
            if (fast) {
                if (ok)
                    claim_chunk<0, CH, GEN, decltype(key), ARG>(uu, p0, N - 1, smin, N - 1 + smax, smin, smax, K,
                                                                inv2c, pofs, gsl, W, A, key);
                __syncthreads();
                if (ARG) {
                    if (ok)
                        claim_chunk<1, CH, GEN, decltype(key), ARG>(uu, p0, N - 1, smin, N - 1 + smax, smin, smax, K,
                                                                    inv2c, pofs, gsl, W, A, key);
                    __syncthreads();
                }
            } else {
                // exhaustive window over the wrapped row, sources from global memory
                if (ok) {
                    for (int k = 0; k < CH; k++) {
                        const int t = p0 + k;
                        double best = INFINITY;
                        int arg = 0;
                        int j = (t - wp) % N;
                        if (j < 0) j += N;
                        for (int e = -wp; e <= wm; ++e) {
                            const double v = src[j] + kc[-e];
                            if (v < best) {
                                best = v;
                                arg = e;
                            }
                            if (++j == N) j = 0;
                        }
                        W[gs + k] = best;
                        if (ARG) A[gs + k] = arg;
                    }
                }
                __syncthreads();
            }
            double un[CH + 2];
            if (kNextSrc && tile + gridDim.x < ntiles) load_src(tile + gridDim.x, un);
            if (ok) {
                double x[CH + 1];
#pragma unroll
                for (int k = 0; k < CH; k++) x[k] = W[gs + k];
                x[CH] = W[skc<CH>(kbase + (p0 + CH == N ? 0 : p0 + CH))];
                double z[CH];
                if (EPI) {
                    const double2* h2 = (const double2*)(a.hv + row * N + p0);
#pragma unroll
                    for (int k = 0; k < CH / 2; k++) {
                        const double2 v = h2[k];
                        z[2 * k] = x[2 * k] - v.x;
                        z[2 * k + 1] = x[2 * k + 1] - v.y;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < CH; k++) z[k] = x[k];
                }
                double2* d2 = (double2*)(out + row * N + p0);
#pragma unroll
                for (int k = 0; k < CH / 2; k++) d2[k] = make_double2(z[2 * k], z[2 * k + 1]);
#pragma unroll
                for (int k = 0; k < CH; k++) {
                    bad |= !(x[k] < INFINITY);
                    if (a.stats_out) fold_stats<EPI>(st, x[k], x[k + 1], z[k]);
                }
                if (ARG && a.argmin) {
                    int16_t* am = a.argmin + row * N + p0;
#pragma unroll
                    for (int k = 0; k < CH; k++) {
                        const int e = A[gs + k];
                        am[k] = (int16_t)e;
                        amax = max(amax, abs(e));
                    }
                }
            }
            __syncthreads();   // keys are reused by the next tile
            if (kNextSrc)
#pragma unroll
                for (int k = 0; k < CH + 2; k++) uu[k] = un[k];
        }
    }
    if (bad) atomicOr(&a.flags[0], kErrFastPath);
    if (ARG && a.argmin) {
        block_atomic_max(amax, amax_word(a));
        if (amax > 32767) atomicOr(&a.flags[0], kErrArgRange);   // stored offsets wrapped: unusable
    }
    publish_stats<EPI>(st, a, red);
    maybe_next_windows(a);   // after this block's own work: off the critical path
}

// ---------------------------------------------------------------------------
// TILE kernel: C lines side by side (16, or 1 for an axis with fewer lines:
// then the whole block works on one line) x R targets [r0, r0 + R) (+ target
// r0 + R for the forward differences of the output), lines of any stride.
// BS threads, BS / C per line.  PF > 0 (the potential step, R = PF BS / C):
// each thread loads the tau V values of its PF outputs before the claims.
// ---------------------------------------------------------------------------
template <int EPI, int ARG, int C, bool GEN, int BS, int PF>
__global__ __launch_bounds__(BS) void k_claim_tile(const double* __restrict__ in, double* __restrict__ out,
                                                       const double* __restrict__ kc, SweepArgs a, ClaimLds L,
                                                       double inv2c, double pofs)
{
    extern __shared__ double sm[];
    __shared__ double red[40];
    {
        int64_t ko;
        const int64_t uo = batch_shift(a, &ko);
        in += uo;
        out += uo;
        kc += ko;
        if (a.pofs_b) pofs = a.pofs;
    }
    // one-line tiles: a search block (block 0, dispatched first) only
    // computes the next step's windows, from statistics complete before the
    // launch, beside the tiles, which go to blocks 1, 2, ...  (In the row
    // sweeps, whose search block would have to share the start of the
    // launch with every tile's loads, it gained nothing.)
    const int sbk = C == 1 ? a.search_block : 0;
    if (sbk && blockIdx.x == 0) {
        clear_slot(a.stats_clear);
        maybe_next_windows(a);
        return;
    }
    constexpr int kKeyStride = tile_key_stride(C);
    // the first two claims of a source unrolled: faster in blocks of 512
    // threads of 16-line tiles (few tiles) and in argmin sweeps; slower in the
    // 3-D tile sweeps and in one-line tiles
    constexpr bool kU2 = (C == kTileLines && BS == 512) || ARG;
    const int N = (int)a.g.n;
    const int S = (int)a.g.stride;   // line offsets fit 32 bits (the plan caps the grid at 2^31 points)
    const int R = a.tile_rows;
    const int KH = L.KH;
    // block, tile and line indices fit 32 bits (the plan caps the grid at 2^31 points)
    const int nTB = (N + R - 1) / R;
    const int nLB = (int)((a.g.nlines + C - 1) / C);
    const int b = (int)remap_block(blockIdx.x - sbk, (int64_t)nTB * nLB);
    const int lb = b / nTB;
    const int r0 = (b - lb * nTB) * R;
    const int Rt = min(R, N - r0);
    const int NT = Rt + 1;

    const int c = (int)threadIdx.x % C;    // line of this thread
    const int q = (int)threadIdx.x / C;    // rank among the line's BS / C threads
    const int line = lb * C + c;
    const bool lok = line < a.g.nlines;
    const int ln = lok ? line : 0;
    const int64_t lbase = (ln % S) + (int64_t)S * N * (ln / S);

    double* KT = sm;
    double* W = KT + (2 * KH + 1);
    int* A = (int*)(W + (size_t)L.NT * kKeyStride);

    // The loads that the window does not decide are issued before the window
    // is read, so that their latencies overlap: the cost band (centred on the
    // cost's vertex) and the tau V values of this thread's outputs.
    // KT[i] = k(sb + i), i < 2 KH + 1: offsets [vertex - KH - g, vertex + KH - g]
    // (a convex table's crossings also read k(smin - 1))
    const int kcap = (int)min((int64_t)a.kin.kcap, (int64_t)0x7fffffff);
    const int g = GEN ? 1 : 0;
    const int vtx = GEN ? a.kvert : (int)floor(pofs + 0.5);
    const int sb = vtx - KH - g;
    constexpr int kKtRegs = (2 * 512 + 1 + BS - 1) / BS;   // the band has at most 2 * 512 + 1 entries
    double ktv[kKtRegs];
#pragma unroll
    for (int j = 0; j < kKtRegs; j++) {
        const int i = (int)threadIdx.x + j * BS;
        const int s = sb + i;
        ktv[j] = (i < 2 * KH + 1 && s >= -kcap && s <= kcap) ? kc[s] : INFINITY;
    }
    // PF > 0 (potential step, tiles of PF (BS / C) targets): the tau V values
    // of this thread's outputs, whose latency then passes during the claims
    double hvp[PF > 0 ? PF : 1];
    if (PF > 0 && lok) {
        const double* __restrict__ h = a.hv + lbase + (int64_t)S * r0;
#pragma unroll
        for (int i = 0; i < PF; i++) {
            const int t = q + i * (BS / C);
            hvp[i] = t < Rt ? h[(int64_t)S * t] : 0.0;
        }
    }
    const double* __restrict__ src = in + lbase;
    auto load_chunk = [&](int p0, double (&uu)[kCh + 2]) {
        int r = (p0 - 1) % N;
        if (r < 0) r += N;
#pragma unroll
        for (int k = 0; k < kCh + 2; k++) {
            uu[k] = src[S * r];
            r = r + 1 == N ? 0 : r + 1;
        }
    };

    clear_slot(a.stats_clear);
    int wp = a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis];
    int wm = a.wfix > 0 ? a.wfix : a.win_in[2 * a.axis + 1];
    wp = __builtin_amdgcn_readfirstlane(wp);
    wm = __builtin_amdgcn_readfirstlane(wm);
    for (int t = q; t < NT; t += BS / C) {
        W[t * kKeyStride + c] = INFINITY;
        if (ARG) A[t * kKeyStride + c] = 0x7fffffff;
    }
#pragma unroll
    for (int j = 0; j < kKtRegs; j++) {
        const int i = (int)threadIdx.x + j * BS;
        if (i < 2 * KH + 1) KT[i] = ktv[j];
    }
    // offsets beyond the table's end cost +inf and never win
    const int smin = max(-wm - 1, -kcap), smax = min(wp + 1, kcap);
    const bool fast = smin - g >= sb && smax <= sb + 2 * KH;
    const double* K = KT - sb;   // K[s] = k(s), s in [sb, sb + 2 KH]
    const double gsl = a.kslack;
    __syncthreads();

    // sources that can reach the targets: [r0 - wp, r0 + NT - 1 + wm]
    const int nch_fast = (NT - 1 + wm + wp + kCh) / kCh;
    if (ARG && fast && nch_fast <= BS / C) {
        // at most one chunk a thread: its sources stay in registers for the
        // second pass
        const int pA = r0 - wp, pB = r0 + NT - 1 + wm;
        const int p0 = pA + q * kCh;
        const bool has = q < nch_fast && lok;
        double uu[kCh + 2];
        auto key = [r0](int t) { return (t - r0) * kKeyStride; };
        if (has) {
            load_chunk(p0, uu);
            claim_chunk<0, kCh, GEN, decltype(key), true>(uu, p0, pB, r0, r0 + NT - 1, smin, smax, K, inv2c, pofs, gsl,
                                                          W + c, A + c, key);
        }
        __syncthreads();
        if (has)
            claim_chunk<1, kCh, GEN, decltype(key), true>(uu, p0, pB, r0, r0 + NT - 1, smin, smax, K, inv2c, pofs, gsl,
                                                          W + c, A + c, key);
        __syncthreads();
    } else if (fast) {
        const int pA = r0 - wp, pB = r0 + NT - 1 + wm;
        const int nch = nch_fast;
        for (int pass = 0; pass < (ARG ? 2 : 1); pass++) {
            for (int ch = q; ch < nch && lok; ch += BS / C) {
                const int p0 = pA + ch * kCh;
                double uu[kCh + 2];
                load_chunk(p0, uu);
                auto key = [r0](int t) { return (t - r0) * kKeyStride; };
                if (pass == 0)
                    claim_chunk<0, kCh, GEN, decltype(key), kU2>(uu, p0, pB, r0, r0 + NT - 1, smin, smax, K, inv2c,
                                                                 pofs, gsl, W + c, A + c, key);
                else
                    claim_chunk<1, kCh, GEN, decltype(key), kU2>(uu, p0, pB, r0, r0 + NT - 1, smin, smax, K, inv2c,
                                                                 pofs, gsl, W + c, A + c, key);
            }
            __syncthreads();
        }
    } else {
        // window wider than the band: band by band, chunks of two sources
        for (int pass = 0; pass < (ARG ? 2 : 1); pass++) {
            for (int blo = smin; blo <= smax; blo += max(2 * KH + 1 - g, 1)) {
                const int bhi = min(blo + max(2 * KH - g, 0), smax);
                __syncthreads();
                for (int i = threadIdx.x; i < 2 * KH + 1; i += BS) {
                    const int s = blo - g + i;
                    KT[i] = (s >= -kcap && s <= kcap) ? kc[s] : INFINITY;
                }
                __syncthreads();
                // sources that reach the targets with an offset of the window and of the band
                const int pA = max(r0 - wp, r0 - bhi), pB = min(r0 + NT - 1 + wm, r0 + NT - 1 - blo);
                const int nch = (pB - pA + 2) / 2;
                for (int ch = q; ch < nch && lok; ch += BS / C) {
                    const int p0 = pA + 2 * ch;
                    double u4[4];
                    int r = (p0 - 1) % N;
                    if (r < 0) r += N;
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        u4[k] = src[S * r];
                        r = r + 1 == N ? 0 : r + 1;
                    }
                    auto key = [r0](int t) { return (t - r0) * kKeyStride; };
                    if (pass == 0)
                        claim_chunk<0, 2, GEN>(u4, p0, pB, r0, r0 + NT - 1, blo, bhi, KT - (blo - g), inv2c, pofs,
                                               gsl, W + c, A + c, key);
                    else
                        claim_chunk<1, 2, GEN>(u4, p0, pB, r0, r0 + NT - 1, blo, bhi, KT - (blo - g), inv2c, pofs,
                                               gsl, W + c, A + c, key);
                }
            }
            __syncthreads();
        }
    }

    // ---- outputs, argmins, stats of this sweep's result ----
    SweepStats st;
    int amax = 0;
    bool bad = false;
    // the store kind is a compile-time choice inside the loops (one copy each)
    auto emit = [&](auto wt_tag) {
        constexpr bool kWt = decltype(wt_tag)::value;
        if (!lok) return;
        double* __restrict__ dst = out + lbase + (int64_t)S * r0;
        const double* __restrict__ hv = EPI ? a.hv + lbase + (int64_t)S * r0 : nullptr;
        int16_t* am = (ARG && a.argmin) ? a.argmin + lbase + (int64_t)S * r0 : nullptr;
        int off = S * q;
        if (PF > 0) {
#pragma unroll
            for (int i = 0; i < PF; i++) {
                const int t = q + i * (BS / C);
                if (t < Rt) {
                    const double x = W[t * kKeyStride + c];
                    bad |= !(x < INFINITY);
                    const double z = x - hvp[i];
                    put<kWt>(dst + off, z);
                    if (ARG && am) {
                        const int e = A[t * kKeyStride + c];
                        am[off] = (int16_t)e;
                        amax = max(amax, abs(e));
                    }
                    if (a.stats_out) fold_stats<EPI>(st, x, W[(t + 1) * kKeyStride + c], z);
                }
                off += S * (BS / C);
            }
        } else {
            for (int t = q; t < Rt; t += BS / C) {
                const double x = W[t * kKeyStride + c];
                bad |= !(x < INFINITY);
                const double z = EPI ? x - hv[off] : x;
                put<kWt>(dst + off, z);
                if (ARG && am) {
                    const int e = A[t * kKeyStride + c];
                    am[off] = (int16_t)e;
                    amax = max(amax, abs(e));
                }
                if (a.stats_out) fold_stats<EPI>(st, x, W[(t + 1) * kKeyStride + c], z);
                off += S * (BS / C);
            }
        }
    };
    if (C == kTileLines && a.wt)
        emit(std::true_type{});
    else
        emit(std::false_type{});
    if (bad) atomicOr(&a.flags[0], kErrFastPath);
    if (ARG && a.argmin) {
        block_atomic_max(amax, amax_word(a));
        if (amax > 32767) atomicOr(&a.flags[0], kErrArgRange);   // stored offsets wrapped: unusable
    }
    publish_stats<EPI>(st, a, red);
    // the next step's windows: one-line tiles (an axis of fewer than 16 lines,
    // 1-D grids) compute them here, after this block's own work; beside tiles
    // of 16 lines a kernel of their own does (the search would cost every
    // block of those registers)
    if constexpr (C == 1) maybe_next_windows(a);
}

ClaimLds claim_layout(int kind, int64_t N, int tile_rows, int H, bool arg, int row_ch, int tile_lines)
{
    ClaimLds L;
    L.C = 1;
    L.arg = arg ? 1 : 0;
    L.KH = H;
    if (kind == kKindRow) {
        L.row = 1;
        L.nr = (int)std::max<int64_t>(1, 2048 / N);   // whole rows, at most 2048 points per tile
        const int g = L.nr * (int)N;
        L.RS = g + g / row_ch + 1;                   // skewed keys
        L.NT = 0;
    } else {
        L.row = 0;
        L.nr = 1;
        L.RS = 0;
        L.NT = tile_rows + 1;
        L.C = tile_lines;
    }
    return L;
}

// Whether a launch of `grid` blocks (per instance) that computes the next
// step's windows can give them a block of its own: when one more block is
// resident at once, so that no tile waits for the search block's slot.
template <typename Kern>
bool search_block_fits(Kern k, int bs, size_t lds, int64_t grid, const SweepArgs& a)
{
    if (!a.win_next) return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, bs, lds) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const int64_t ncu = a.grid_cap / 4;   // plans size grid_cap at four blocks a compute unit
    return (grid + 1) * std::max(1, a.nb) <= (int64_t)per_cu * ncu;
}

template <int ROW>
hipError_t launch_claim_t(const double* in, double* out, const SweepArgs& a, const ClaimLds& L, double inv2c,
                          double pofs, int64_t grid, bool wide, hipStream_t s)
{
    const size_t lds = claim_lds_bytes(L);
    const bool arg = a.argmin != nullptr;
    const bool epi = a.hv != nullptr;
    // one-line tiles (with the potential step: tau V prefetched for tiles of
    // 2 or 4 targets a thread), with a search block when one fits
#define LO_LINE_LAUNCH(K, E, A, G, B, PF)                                                                      \
    do {                                                                                                        \
        SweepArgs c = a;                                                                                        \
        c.search_block = search_block_fits(K<E, A, 1, G, B, PF>, B, lds, grid, a) ? 1 : 0;                      \
        LO_SWEEP_LAUNCH((K<E, A, 1, G, B, PF>), dim3((unsigned)(grid + c.search_block), a.nb), dim3(B), lds, s, \
                        a, in, out, a.kin.k, c, L, inv2c, pofs);                                                \
    } while (0)
#define LO_CLAIM_LAUNCH_B(K, E, A, G, B)                                                                       \
    do {                                                                                                        \
        if (L.C == 1) {                                                                                         \
            if constexpr (E == 1) {                                                                             \
                if (a.tile_rows == 2 * B) LO_LINE_LAUNCH(K, E, A, G, B, 2);                                     \
                else if (a.tile_rows == 4 * B) LO_LINE_LAUNCH(K, E, A, G, B, 4);                                \
                else LO_LINE_LAUNCH(K, E, A, G, B, 0);                                                          \
            } else                                                                                              \
                LO_LINE_LAUNCH(K, E, A, G, B, 0);                                                               \
        } else if constexpr (E == 1) {                                                                            \
            constexpr int kPfA = B == kBlock ? 16 : 4, kPfB = 8;                                                \
            if (a.tile_rows == kPfA * (B / kTileLines))                                                         \
                LO_SWEEP_LAUNCH((K<E, A, kTileLines, G, B, kPfA>), dim3((unsigned)grid, a.nb), dim3(B), lds, s, \
                                a, in, out, a.kin.k, a, L, inv2c, pofs);                                        \
            else if (a.tile_rows == kPfB * (B / kTileLines))                                                    \
                LO_SWEEP_LAUNCH((K<E, A, kTileLines, G, B, kPfB>), dim3((unsigned)grid, a.nb), dim3(B), lds, s, \
                                a, in, out, a.kin.k, a, L, inv2c, pofs);                                        \
            else                                                                                                \
                LO_SWEEP_LAUNCH((K<E, A, kTileLines, G, B, 0>), dim3((unsigned)grid, a.nb), dim3(B), lds, s, a, \
                                in, out, a.kin.k, a, L, inv2c, pofs);                                           \
        } else                                                                                                  \
            LO_SWEEP_LAUNCH((K<E, A, kTileLines, G, B, 0>), dim3((unsigned)grid, a.nb), dim3(B), lds, s, a, in, \
                            out, a.kin.k, a, L, inv2c, pofs);                                                   \
    } while (0)
#define LO_CLAIM_LAUNCH_G(K, E, A, G)                                                                          \
    do {                                                                                                        \
        if (wide) LO_CLAIM_LAUNCH_B(K, E, A, G, 2 * kBlock);                                                    \
        else LO_CLAIM_LAUNCH_B(K, E, A, G, kBlock);                                                             \
    } while (0)
#define LO_CLAIM_LAUNCH(K, E, A)                                                                                \
    do {                                                                                                        \
        if (a.quad) LO_CLAIM_LAUNCH_G(K, E, A, false);                                                          \
        else LO_CLAIM_LAUNCH_G(K, E, A, true);                                                                  \
    } while (0)
#define LO_ROW_LAUNCH_G(E, A, CH, G)                                                                          \
    LO_SWEEP_LAUNCH((k_claim_row<E, A, CH, kRowPoints / CH, G>), dim3((unsigned)grid, a.nb),                  \
                    dim3(kRowPoints / CH), lds, s, a, in, out, a.kin.k, a, L, inv2c, pofs)
#define LO_ROW_LAUNCH_CH(E, A, CH)                                                                            \
    do {                                                                                                       \
        if (a.quad) LO_ROW_LAUNCH_G(E, A, CH, false);                                                          \
        else LO_ROW_LAUNCH_G(E, A, CH, true);                                                                  \
    } while (0)
#define LO_ROW_LAUNCH(E, A)                                                                                    \
    do {                                                                                                       \
        if (a.row_ch == 4) LO_ROW_LAUNCH_CH(E, A, 4);                                                          \
        else LO_ROW_LAUNCH_CH(E, A, 8);                                                                        \
    } while (0)
    if (ROW) {
        if (epi) {
            if (arg) LO_ROW_LAUNCH(1, 1);
            else LO_ROW_LAUNCH(1, 0);
        } else {
            if (arg) LO_ROW_LAUNCH(0, 1);
            else LO_ROW_LAUNCH(0, 0);
        }
    } else {
        if (epi) {
            if (arg) LO_CLAIM_LAUNCH(k_claim_tile, 1, 1);
            else LO_CLAIM_LAUNCH(k_claim_tile, 1, 0);
        } else {
            if (arg) LO_CLAIM_LAUNCH(k_claim_tile, 0, 1);
            else LO_CLAIM_LAUNCH(k_claim_tile, 0, 0);
        }
    }
#undef LO_CLAIM_LAUNCH
#undef LO_CLAIM_LAUNCH_G
#undef LO_CLAIM_LAUNCH_B
#undef LO_LINE_LAUNCH
#undef LO_ROW_LAUNCH
#undef LO_ROW_LAUNCH_CH
#undef LO_ROW_LAUNCH_G
    return hipGetLastError();
}

}  // namespace

int fast_tile_lines(int64_t nlines) { return nlines < kTileLines ? 1 : kTileLines; }

size_t fast_lds_for(int kind, int64_t N, int tile_rows, int H, int tile_lines)
{
    return claim_lds_bytes(claim_layout(kind, N, tile_rows, H, true, 4, tile_lines));   // the larger row layout
}

hipError_t launch_fast(const double* in, double* out, const SweepArgs& a, double cq, double inv2c, double pofs,
                       hipStream_t s)
{
    (void)cq;
    const int C = fast_tile_lines(a.g.nlines);
    const bool arg = a.argmin != nullptr;
    // A grid of few tiles (two blocks of 256 threads a CU or fewer) leaves the
    // SIMDs short of waves: its sweeps then take blocks of 512 threads (rows:
    // 4 points a thread), and tiles of 16 lines take 128 targets (twice the
    // blocks, for a few more halo sources).
    const int64_t nr = a.kind == kKindRow ? std::max<int64_t>(1, 2048 / a.g.n) : 1;
    int64_t tiles = a.kind == kKindRow
                        ? (a.g.nlines + nr - 1) / nr
                        : ((a.g.n + a.tile_rows - 1) / a.tile_rows) * ((a.g.nlines + C - 1) / C);
    // narrow: blocks of 512 threads, rows walked by one block a CU and tiles
    // of 16 lines x 256 targets, so that the sweep leaves room on every CU for
    // the blocks of a kernel on another stream
    const bool narrow = a.narrow != 0;
    const bool few = narrow || tiles * a.nb * 2 <= a.grid_cap;
    const int row_ch = a.row_ch == 4 || (few && a.kind == kKindRow) ? 4 : 8;
    SweepArgs b = a;
    b.row_ch = row_ch;
    if (narrow && a.kind == kKindTile && C == kTileLines) {
        b.tile_rows = 256;
        tiles = ((a.g.n + 255) / 256) * ((a.g.nlines + C - 1) / C);
    } else if (few && a.kind == kKindTile && C == kTileLines && a.tile_rows > 128) {
        b.tile_rows = 128;
        tiles = ((a.g.n + 127) / 128) * ((a.g.nlines + C - 1) / C);
    }
    const ClaimLds L = claim_layout(a.kind, a.g.n, b.tile_rows, a.halo, arg, row_ch, C);
    // ROW: persistent blocks, about grid_cap in all (instances included), each
    // walking several tiles so that its fixed costs are amortised
    const int64_t cap = std::max(1, (narrow ? a.grid_cap / 4 : a.grid_cap) / std::max(1, a.nb));
    if (a.kind == kKindRow) return launch_claim_t<1>(in, out, b, L, inv2c, pofs, std::min(tiles, cap), false, s);
    return launch_claim_t<0>(in, out, b, L, inv2c, pofs, tiles, few, s);
}

}  // namespace lo
