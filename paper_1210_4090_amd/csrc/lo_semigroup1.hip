// The first discrete semigroup (Section 2.2, eq. cost1) on 1-D grids: the
// cost of a move from lifted source y to target x in one step is the action
// of the straight path between them,
//     c(y, x) = k(x - y) - I(y, x),
// I the time integral of V along the path by the trapezoid rule over the grid
// points it crosses (hv = tau V on the grid, m = |x - y| crossings of tau/m):
//     I = hv(x)                                            if m = 0,
//     I = (hv(y)/2 + hv(y+d) + ... + hv(x-d) + hv(x)/2) / m   else.
// The cost depends on (y, x), not on x - y alone, so a step is a min-plus
// matrix-vector product, not a convolution: this kernel evaluates every
// candidate of the window (one thread per target), the path sums in O(1) from
// prefix sums of hv over the lifted line.  The potential is inside the cost:
// there is no separate potential step.
#include <hip/hip_runtime.h>

#include "lo_internal.h"

namespace lo {
namespace {

constexpr int kSgBlock = 256;
constexpr int kScanBlock = 1024;

// Q[i] = hv[0] + ... + hv[i-1], i in [0, N], in one block: each thread sums a
// contiguous run of hv, the run totals are scanned in order by thread 0, and
// each thread then writes the prefixes of its run.
__global__ __launch_bounds__(kScanBlock) void k_prefix(const double* __restrict__ hv, int64_t N,
                                                       double* __restrict__ Q)
{
    __shared__ double part[kScanBlock];
    const int t = (int)threadIdx.x;
    const int64_t per = (N + kScanBlock - 1) / kScanBlock;
    const int64_t b = min(N, (int64_t)t * per), e = min(N, b + per);
    double sum = 0.0;
    for (int64_t i = b; i < e; i++) sum += hv[i];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        double acc = 0.0;
        for (int i = 0; i < kScanBlock; i++) {
            const double v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    double acc = part[t];
    for (int64_t i = b; i < e; i++) {
        Q[i] = acc;
        acc += hv[i];
    }
    if (t == kScanBlock - 1) Q[N] = acc;   // the last run ends at N (it may be empty)
}

// Q[i] = hv[0] + ... + hv[i-1], i in [0, N]; lifted prefix P(i) = Q[i mod N] + floor(i / N) Q[N]
__device__ __forceinline__ double lifted_prefix(const double* __restrict__ Q, int64_t i, int64_t N)
{
    int64_t q = i / N, r = i - q * N;
    if (r < 0) {
        r += N;
        q -= 1;
    }
    return Q[r] + (double)q * Q[N];
}

__global__ __launch_bounds__(kSgBlock) void k_semigroup1(const double* __restrict__ u, double* __restrict__ w,
                                                         int64_t N, int W, const double* __restrict__ kt,
                                                         const double* __restrict__ hv,
                                                         const double* __restrict__ Q, unsigned* __restrict__ sat)
{
    const int64_t x = (int64_t)blockIdx.x * kSgBlock + threadIdx.x;
    if (x >= N) return;
    auto wrap = [N](int64_t i) {
        int64_t r = i % N;
        return r < 0 ? r + N : r;
    };
    double best = INFINITY;
    int arg = 0;
    for (int e = -W; e <= W; e++) {
        const int64_t y = x + e;   // lifted source; s = x - y = -e
        double I = 0.0;
        if (hv) {
            if (e == 0) {
                I = hv[x];
            } else {
                const int64_t lo = e < 0 ? y : x, hi = e < 0 ? x : y;
                const double inner = lifted_prefix(Q, hi, N) - lifted_prefix(Q, lo + 1, N);
                I = (inner + 0.5 * hv[wrap(lo)] + 0.5 * hv[wrap(hi)]) / (double)(e < 0 ? -e : e);
            }
        }
        const double v = (u[wrap(y)] + kt[-e]) - I;
        if (v < best) {
            best = v;
            arg = e;
        }
    }
    w[x] = best;
    if (arg == W || arg == -W) atomicOr(sat, 1u);
}

}  // namespace

hipError_t launch_prefix(const double* hv, int64_t N, double* Q, hipStream_t s)
{
    hipLaunchKernelGGL(k_prefix, dim3(1), dim3(kScanBlock), 0, s, hv, N, Q);
    return hipGetLastError();
}

hipError_t launch_semigroup1(const double* u, double* w, int64_t N, int W, const double* kt_centre, const double* hv,
                             const double* Q, unsigned* sat, hipStream_t s)
{
    hipLaunchKernelGGL(k_semigroup1, dim3((unsigned)((N + kSgBlock - 1) / kSgBlock)), dim3(kSgBlock), 0, s, u, w, N,
                       W, kt_centre, hv, Q, sat);
    return hipGetLastError();
}

}  // namespace lo
