// The paper's own fast algorithm (Section 4), as a comparison kernel for 1-D
// grids: the line is split into convex and concave pieces, each piece is
// convolved with the convex kinetic cost in linear time, and the result is the
// minimum over the pieces (distributivity of the min-plus convolution over the
// minimum, Section 4.1).
//
//  * Pieces (Section 4.2, "decompose u into convex and concave parts"): grown
//    greedily from their first point; the first second difference fixes the
//    type; a convex piece continues while its slopes do not drop by more than
//    eta (second differences >= -eta dx), a concave one while they do not rise
//    by more than eta.  eta = 0 is the exact decomposition, eta > 0 the
//    tolerant variant of Section 4.3.  Consecutive pieces share their junction
//    point.
//  * Convex piece (Theorem th:convex): the convolution walks the two slope
//    sequences in increasing order, one target a step; each target's value is
//    the candidate of the current (source, offset) pair.
//  * Concave piece (Theorem th:ccc): a first convex part from the piece's first
//    source, then for each further source only the offset where the kernel's
//    slope crosses the piece's slope (a pointer that only moves back,
//    Lemma lm:simplif), then a last convex part from the piece's last source.
//
// Every value written is a genuine candidate fl(u(p) + k(t - p)); with eta = 0
// and a window that holds the minimisers the result is the definition's
// minimum.  GPU mapping: one thread per segment of kSeg lifted sources (a
// segment border is an extra junction, which changes no minimum); candidates
// are combined with atomic minima in global memory.
#include <hip/hip_runtime.h>

#include "lo_internal.h"

namespace lo {
namespace {

constexpr int kSeg = 64;    // lifted sources per thread
constexpr int kDecompBlock = 256;

__global__ __launch_bounds__(kDecompBlock) void k_fill(double* w, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * kDecompBlock + threadIdx.x;
    if (i < n) w[i] = v;
}

// u[N] periodic -> w[N]: candidates of the lifted sources q - W, q in [0, L),
// L = N + 2W, with offsets s = target - source in [-W, W] (f[s] = k(s)).
__global__ __launch_bounds__(kDecompBlock) void k_decomp(const double* __restrict__ u, double* __restrict__ w,
                                                         int N, int W, const double* __restrict__ f, double tol,
                                                         unsigned long long* __restrict__ counts)
{
    const int L = N + 2 * W;
    const int s0 = (blockIdx.x * kDecompBlock + threadIdx.x) * kSeg;
    if (s0 >= L - 1) return;
    const int s1 = min(s0 + kSeg, L - 1);   // this thread's pieces cover lifted [s0, s1]
    auto g = [&](int q) {
        int p = (q - W) % N;
        if (p < 0) p += N;
        return u[p];
    };
    // candidate of lifted source q (piece index) and offset index j (s = j - W)
    auto emit = [&](int q, int j) {
        const int x = q - W + j - W;
        if (x >= 0 && x < N) atomicMin(&w[x], g(q) + f[j - W]);
    };
    const int n = 2 * W;
    unsigned long long pieces = 0, breaks = 0;
    int a = s0;
    while (a < s1) {
        int b = a + 1, typ = 0;
        while (b < s1) {
            const double d2 = g(b + 1) - 2.0 * g(b) + g(b - 1);
            if (typ == 0) typ = d2 >= 0.0 ? 1 : -1;
            else if (typ == 1 ? d2 < -tol : d2 > tol) {
                breaks++;
                break;
            }
            b++;
        }
        const int m = b - a;
        if (typ >= 0) {
            // convex (or two points): merge the slopes of the piece and of the kernel
            int i = 0, j = 0;
            emit(a, 0);
            while (i + j < m + n) {
                if (i < m && (j == n || g(a + i + 1) - g(a + i) < f[j + 1 - W] - f[j - W]))
                    i++;
                else
                    j++;
                emit(a + i, j);
            }
        } else {
            // concave: first source, crossing offsets of the middle sources, last source
            int i = 0;
            emit(a, 0);
            const double g1 = g(a + 1) - g(a);
            while (i < n && f[i + 1 - W] - f[i - W] <= g1) emit(a, ++i);
            for (int jj = 1; jj <= m; jj++) {
                const double gs = g(a + jj) - g(a + jj - 1);
                while (i > 0 && gs < f[i - W] - f[i - 1 - W]) i--;
                emit(a + jj - 1, i);
                emit(a + jj, i);
            }
            while (i < n) emit(b, ++i);
        }
        pieces++;
        a = b;
    }
    atomicAdd(&counts[0], pieces);
    atomicAdd(&counts[1], breaks);
}

__global__ __launch_bounds__(kDecompBlock) void k_potential(const double* __restrict__ w, const double* __restrict__ hv,
                                                            double* __restrict__ u, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kDecompBlock + threadIdx.x;
    if (i < n) u[i] = hv ? w[i] - hv[i] : w[i];
}

}  // namespace

hipError_t launch_decomp_step(const double* u, double* w, double* u_out, int N, int W, const double* kt_centre,
                              double tol, const double* hv, unsigned long long* counts, hipStream_t s)
{
    const unsigned gb = (unsigned)((N + kDecompBlock - 1) / kDecompBlock);
    hipLaunchKernelGGL(k_fill, dim3(gb), dim3(kDecompBlock), 0, s, w, (int64_t)N, (double)INFINITY);
    const int L = N + 2 * W;
    const int nseg = (L - 1 + kSeg - 1) / kSeg;
    hipLaunchKernelGGL(k_decomp, dim3((unsigned)((nseg + kDecompBlock - 1) / kDecompBlock)), dim3(kDecompBlock), 0,
                       s, u, w, N, W, kt_centre, tol, counts);
    hipLaunchKernelGGL(k_potential, dim3(gb), dim3(kDecompBlock), 0, s, w, hv, u_out, (int64_t)N);
    return hipGetLastError();
}

}  // namespace lo
