// Reverse pass of the N-step map of eq. uN.  Each axis sweep of eq. eqconvol
// is piecewise affine in its input: the derivative of w(x) is 1 at the
// argmin source of x and 0 elsewhere, so the adjoint of a sweep sends the
// upstream gradient of every target to its argmin source.  The potential
// step subtracts tau V pointwise, so it passes the gradient through and
// contributes -tau * sum_x lambda(x) phi_m(x) to the gradient of a basis
// coefficient.
//
// Scatter as a gather.  With a convex cost and the lowest-offset tie rule the
// lifted argmin source of target i is nondecreasing in i (the Monge property
// of k(i - j)), so the targets that choose a given source form one
// contiguous run.  A block stages the int16 offsets and the upstream
// gradients of the targets that can reach its tile of sources (a halo of max
// |offset| on each side) in LDS, marks the first and last target of every
// source's run, and each source sums its run in increasing target order.  No atomics, so the result is deterministic and
// the additions happen in the order of a sequential loop over the grid.  A
// line whose staged offsets are not monotone (possible only through rounding
// near exact ties) is summed by scanning every target within the halo.
#include <algorithm>
#include <type_traits>

#include "lo_device.h"

namespace lo {
namespace {

using namespace dev;

constexpr int kMaxLinesPerTile = 16;

__device__ __forceinline__ int floor_div(int x, int n) { return x >= 0 ? x / n : -((n - 1 - x) / n); }

__device__ __forceinline__ int64_t line_base(int ln, int S, int N)
{
    return (ln % S) + (int64_t)S * N * (ln / S);
}

// One tile: C lines x R sources [r0, r0 + R) of the axis, targets
// [r0 - h, r0 + R + h) staged (span = R + 2h positions, position p is the
// lifted target r0 - h + p) with their offsets and upstream gradients.
__global__ __launch_bounds__(kBlock) void k_scatter(const int16_t* __restrict__ E, const double* __restrict__ lam,
                                                    double* __restrict__ out, double* __restrict__ Lam,
                                                    ScatterArgs a, uint32_t* flags)
{
    extern __shared__ double smd[];
    __shared__ int nonmono[kMaxLinesPerTile];
    const int N = (int)a.g.n, S = (int)a.g.stride, C = a.C, R = a.R, h = a.h, span = a.span;
    const int nTB = (N + R - 1) / R;
    const int G = nTB * (int)((a.g.nlines + C - 1) / C);    // indices fit 32 bits (grids < 2^31 points)
    const int b = (int)remap_block(blockIdx.x, G);
    const int lb = b / nTB;
    const int r0 = (b - lb * nTB) * R;
    const int Rt = min(R, N - r0);
    double* ls = smd;                                // [C][span] upstream gradient of the staged targets
    int* first = (int*)(ls + (size_t)C * span);      // [C][R] first position of each source's run, -1: none
    int* last = first + C * R;                       // [C][R]
    int16_t* es = (int16_t*)(last + C * R);          // [C][span] offsets of the staged targets
    const bool unit = S == 1;
    // a thread's line (strided axes: fixed, lines are adjacent in memory) and its step along positions
    const int cq = unit ? 0 : (int)threadIdx.x % C;
    const int q0 = unit ? (int)threadIdx.x : (int)threadIdx.x / C;
    const int Q = unit ? kBlock : kBlock / C;
    const int c_lo = unit ? 0 : cq, c_hi = unit ? C : cq + 1;

    if (threadIdx.x < kMaxLinesPerTile) nonmono[threadIdx.x] = 0;
    for (int c = c_lo; c < c_hi; c++)
        for (int j = q0; j < R; j += Q) first[c * R + j] = -1;

    // stage offsets and gradients (lines beyond the grid read as offset 0 and
    // gradient 0; they are never written)
    const int T0 = r0 - h;                     // lifted target of position 0
    const int t0r = T0 - floor_div(T0, N) * N; // its residue
    const int qstep = Q % N;
    bool bad = false;
    for (int c = c_lo; c < c_hi; c++) {
        const int ln = lb * C + c;
        if (ln >= a.g.nlines) {
            for (int p = q0; p < span; p += Q) {
                es[c * span + p] = 0;
                ls[c * span + p] = 0.0;
            }
            continue;
        }
        const int64_t base = line_base(ln, S, N);
        int t = t0r + q0 % N;
        if (t >= N) t -= N;
        // kU positions per round with all their loads in flight at once
        constexpr int kU = 8;
        for (int p0 = q0; p0 < span; p0 += kU * Q) {
            int ev[kU];
            double lv[kU];
#pragma unroll
            for (int u = 0; u < kU; u++) {
                if (p0 + u * Q < span) {
                    const int64_t x = base + (int64_t)t * S;
                    ev[u] = E[x];
                    lv[u] = lam[x];
                }
                t += qstep;
                if (t >= N) t -= N;
            }
#pragma unroll
            for (int u = 0; u < kU; u++) {
                const int p = p0 + u * Q;
                if (p < span) {
                    bad |= ev[u] > h || ev[u] < -h;
                    es[c * span + p] = (int16_t)ev[u];
                    ls[c * span + p] = lv[u];
                }
            }
        }
    }
    // Lam (the running sum of gradients that the potential's coefficients
    // need) of this thread's sources, loaded now so that the latency passes
    // during the marking: when a thread serves one line and at most kLamPf
    // sources of it
    constexpr int kLamPf = 8;
    const bool lam_pf = Lam != nullptr && c_hi - c_lo == 1 && R <= kLamPf * Q;
    double lamv[kLamPf];
    if (lam_pf && lb * C + c_lo < a.g.nlines) {
        const int64_t base = line_base(lb * C + c_lo, S, N);
#pragma unroll
        for (int i = 0; i < kLamPf; i++) {
            const int j = q0 + i * Q;
            lamv[i] = j < Rt ? Lam[base + (int64_t)(r0 + j) * S] : 0.0;
        }
    }
    if (bad) atomicOr(&flags[0], kErrAdjointHalo);
    __syncthreads();

    // runs: a position heads (ends) its source's run when its predecessor
    // (successor) has another source; any decrease marks the line non-monotone
    for (int c = c_lo; c < c_hi; c++) {
        const int16_t* el = es + c * span;
        for (int p = q0; p < span; p += Q) {
            const int sr = p - h + el[p];   // source, relative to r0
            const int sp = p > 0 ? p - 1 - h + el[p - 1] : INT32_MIN;
            const int sn = p + 1 < span ? p + 1 - h + el[p + 1] : INT32_MAX;
            if (sp > sr) nonmono[c] = 1;
            if (sr >= 0 && sr < Rt) {
                if (sp != sr) first[c * R + sr] = p;
                if (sn != sr) last[c * R + sr] = p;
            }
        }
    }
    __syncthreads();

    // the sum of the run of targets of source j of line c of the tile
    auto run_sum = [&](int c, int j) -> double {
        const int16_t* el = es + c * span;
        const double* ll = ls + c * span;
        double acc = 0.0;
        if (nonmono[c] == 0) {
            const int f = first[c * R + j];
            if (f >= 0) {
                const int l = last[c * R + j];
                // targets in increasing residue order: when the run crosses a
                // multiple of N, the part at or above it comes first
                const int Tf = T0 + f;
                const int kN = (floor_div(Tf, N) + 1) * N;
                const int split = (kN <= T0 + l) ? kN - T0 : f;   // first position of the upper part
                for (int p = split; p <= l; p++) acc = acc + ll[p];
                for (int p = f; p < split; p++) acc = acc + ll[p];
            }
        } else {
            const int pe = min(j + 2 * h, span - 1);
            for (int p = j; p <= pe; p++)
                if (p - h + el[p] == j) acc = acc + ll[p];
        }
        return acc;
    };
    auto emit = [&](auto wt_tag) {
        constexpr bool kWt = decltype(wt_tag)::value;
        auto put = [](double* q, double v) {
            if constexpr (kWt)
                __hip_atomic_store(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                *q = v;
        };
        if (lam_pf) {
            const int c = c_lo, ln = lb * C + c;
            if (ln >= a.g.nlines) return;
            const int64_t base = line_base(ln, S, N);
            const double* ll = ls + c * span;
#pragma unroll
            for (int i = 0; i < kLamPf; i++) {
                const int j = q0 + i * Q;
                if (j < Rt) {
                    const int64_t x = base + (int64_t)(r0 + j) * S;
                    put(out + x, run_sum(c, j));
                    put(Lam + x, lamv[i] + ll[h + j]);
                }
            }
            return;
        }
        for (int c = c_lo; c < c_hi; c++) {
            const int ln = lb * C + c;
            if (ln >= a.g.nlines) continue;
            const int64_t base = line_base(ln, S, N);
            const double* ll = ls + c * span;
            for (int j = q0; j < Rt; j += Q) {
                const int64_t x = base + (int64_t)(r0 + j) * S;
                put(out + x, run_sum(c, j));
                if (Lam) put(Lam + x, Lam[x] + ll[h + j]);
            }
        }
    };
    if (a.wt)
        emit(std::true_type{});
    else
        emit(std::false_type{});
}

// Deterministic block sum (fixed shuffle pattern, waves combined in order).
__device__ double block_sum(double v, double* red)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v = v + __shfl_xor(v, o, kWave);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (threadIdx.x % kWave == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < (int)blockDim.x / kWave; i++) s = s + red[i];
    __syncthreads();
    return s;
}

// partial[m][b] = sum over block b's chunk of Lam(x) * basis_m(x)
__global__ __launch_bounds__(kBlock) void k_project(const double* __restrict__ Lam,
                                                    const double* __restrict__ basis, int M, int64_t npts,
                                                    int64_t chunk, double* __restrict__ partial)
{
    __shared__ double red[kBlock / kWave];
    const int64_t x0 = (int64_t)blockIdx.x * chunk;
    const int64_t x1 = min(npts, x0 + chunk);
    for (int m = 0; m < M; m++) {
        const double* ph = basis + (int64_t)m * npts;
        double acc = 0.0;
        for (int64_t x = x0 + threadIdx.x; x < x1; x += kBlock) acc = acc + Lam[x] * ph[x];
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) partial[(int64_t)m * gridDim.x + blockIdx.x] = acc;
    }
}

// out[m] = sum_b partial[m][b], one block per mode
__global__ __launch_bounds__(kBlock) void k_project_sum(const double* __restrict__ partial, int G,
                                                        double* __restrict__ out)
{
    __shared__ double red[kBlock / kWave];
    const double* row = partial + (int64_t)blockIdx.x * G;
    double acc = 0.0;
    for (int i = threadIdx.x; i < G; i += kBlock) acc = acc + row[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

}  // namespace

size_t scatter_lds_bytes(int C, int R, int h)
{
    const size_t span = R + 2 * (size_t)h;
    return sizeof(double) * (size_t)C * span + sizeof(int) * 2 * (size_t)C * R + sizeof(int16_t) * (size_t)C * span;
}

bool scatter_layout(const AxisGeom& g, int h, size_t lds_max, ScatterArgs* a)
{
    a->g = g;
    a->h = h;
    const int64_t N = g.n;
    int C, R;
    if (g.stride == 1) {
        R = (int)std::min<int64_t>(N, 1024);
        C = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxLinesPerTile, 1024 / R));
    } else {
        R = (int)std::min<int64_t>(N, 128);
        C = kMaxLinesPerTile;
    }
    // a wide halo (h large beside R) is staged for every line of a tile: give
    // up lines (down to 4, 32-byte rows) before shortening the tile, which
    // would stage the halo for fewer sources (measured on 1024^2 with
    // h ~ 100: 29 -> 18 us per strided scatter)
    const size_t budget = std::min<size_t>(lds_max, 40 * 1024);
    while (scatter_lds_bytes(C, R, h) > budget && C > 4) C /= 2;
    while (scatter_lds_bytes(C, R, h) > budget && R > 32) R /= 2;
    while (scatter_lds_bytes(C, R, h) > budget && C > 1) C /= 2;
    if (scatter_lds_bytes(C, R, h) > lds_max) return false;
    a->C = C;
    a->R = R;
    a->span = R + 2 * h;
    // a grid that fits the last-level caches is written through them when a
    // store instruction covers whole lines (unit stride, or 16 lines side by
    // side): the kernel's end then has little to write back
    a->wt = g.n * g.nlines <= ((int64_t)1 << 22) && (g.stride == 1 || C >= 16) ? 1 : 0;
    return true;
}

hipError_t launch_scatter(const int16_t* E, const double* lam, double* out, double* Lam, const ScatterArgs& a,
                          uint32_t* flags, hipStream_t s)
{
    const int64_t G = ((a.g.n + a.R - 1) / a.R) * ((a.g.nlines + a.C - 1) / a.C);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)G), dim3(kBlock), scatter_lds_bytes(a.C, a.R, a.h), s, E, lam,
                       out, Lam, a, flags);
    return hipGetLastError();
}

int project_blocks(int64_t npts) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (npts + 1023) / 1024)); }

hipError_t launch_project(const double* Lam, const double* basis, int M, int64_t npts, double* partial,
                          double* out, hipStream_t s)
{
    const int G = project_blocks(npts);
    const int64_t chunk = (npts + G - 1) / G;
    hipLaunchKernelGGL(k_project, dim3(G), dim3(kBlock), 0, s, Lam, basis, M, npts, chunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_project_sum, dim3(M), dim3(kBlock), 0, s, partial, G, out);
    return hipGetLastError();
}

namespace {

// Largest |offset| of every (step, axis) segment of a record of int16
// argmins laid out [step][axis][npts], into out[step * ndim + axis].  Block x
// takes part x % G of segment x / G; one global atomic a block.
// V8: npts a multiple of 8, 16-byte loads of 8 offsets.
template <bool V8>
__global__ __launch_bounds__(kBlock) void k_absmax16(const int16_t* __restrict__ E, int64_t npts, int G,
                                                     uint32_t* __restrict__ out)
{
    const int64_t seg = blockIdx.x / G;
    const int part = (int)(blockIdx.x - seg * G);
    const int16_t* base = E + seg * npts;
    uint32_t mx = 0;
    if (V8) {
        const int4* b4 = (const int4*)base;
        for (int64_t c = (int64_t)part * kBlock + threadIdx.x; c < npts / 8; c += (int64_t)G * kBlock) {
            const int4 v = b4[c];
            const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; k++) {
                mx = max(mx, (uint32_t)abs((int)(int16_t)(w[k] & 0xffff)));
                mx = max(mx, (uint32_t)abs((int)(int16_t)((uint32_t)w[k] >> 16)));
            }
        }
    } else {
        for (int64_t i = (int64_t)part * kBlock + threadIdx.x; i < npts; i += (int64_t)G * kBlock)
            mx = max(mx, (uint32_t)abs((int)base[i]));
    }
    block_atomic_max((int)mx, &out[seg]);
}

}  // namespace

hipError_t launch_absmax16(const int16_t* E, int64_t steps, int ndim, int64_t npts, uint32_t* out, hipStream_t s)
{
    const int64_t nseg = steps * ndim;
    if (nseg <= 0 || npts <= 0) return hipSuccess;
    // about 2048 blocks in all, a part of one segment each
    const int64_t per = (npts + 8 * kBlock - 1) / (8 * kBlock);   // blocks that a segment can keep busy
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(per, (2048 + nseg - 1) / nseg));
    if (nseg * G > 0x7fffffff) return hipErrorInvalidValue;
    if (npts % 8 == 0)
        hipLaunchKernelGGL(k_absmax16<true>, dim3((unsigned)(nseg * G)), dim3(kBlock), 0, s, E, npts, G, out);
    else
        hipLaunchKernelGGL(k_absmax16<false>, dim3((unsigned)(nseg * G)), dim3(kBlock), 0, s, E, npts, G, out);
    return hipGetLastError();
}

}  // namespace lo
