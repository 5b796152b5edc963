// The paper's own fast algorithm (Section 4), as a comparison kernel for 1-D
// grids: the lifted line is cut into convex and concave pieces, each piece is
// convolved with the convex kinetic cost, and the result is the minimum over
// the pieces (the min-plus convolution distributes over a minimum,
// Section 4.1).
//
// Pieces (Section 4.2, step 1 of its application): a piece starts at a point,
// the sign of its first second difference gives its type, and it grows while
// the type holds.  With a tolerance eta (Section 4.3) a convex piece accepts a
// slope that drops by at most eta and a concave one a slope that rises by at
// most eta; eta = 0 is the exact split.  Consecutive pieces share their
// junction point.
//
// Convolution of one piece, per source rather than by a walk over merged slope
// lists.  Let the piece have sources 0..m with slopes rho_i = g(i) - g(i - 1)
// and let the cost f on offsets 0..n have slopes r_j = f(j) - f(j - 1), a
// nondecreasing sequence (f is convex).  The pair (source i, offset j) can give
// the minimum at target i + j only if neither neighbouring pair on the same
// target does better:
//     (i + 1, j - 1) is not better  <=>  r_j <= rho_{i+1},
//     (i - 1, j + 1) is not better  <=>  r_{j+1} >= rho_i,
// with rho_0 = -inf and rho_{m+1} = +inf at the piece's ends.  A minimum over
// the piece is such a pair, so source i needs only the offsets
//     j in [ #{r < rho_i}, #{r <= rho_{i+1}} ],
// two binary searches over the cost's slopes.  On a convex piece these ranges
// cover the offsets end to end in slope order (Theorem th:convex); on a
// concave piece the first source keeps the offsets below the first crossing,
// the last one those above the last crossing, and each interior source at most
// its crossing offset (Lemma lm:simplif, Theorem th:ccc's convex / concave /
// convex parts).  A piece accepted under the tolerance is convolved as if it
// had the type it was given: its slopes are replaced by their running maximum
// (convex) or running minimum (concave) before the searches, so that every
// target of the piece is still covered.  The value written for a pair is
// always the genuine candidate fl(u(p) + k(t - p)).
//
// Rounding: both conditions are evaluated on rounded slopes, so they are
// widened by 2^-40 (1 + max|k| + |g| at the two sources compared), far above the rounding of
// the candidate sums; with eta = 0 the pair that attains the rounded minimum is
// then among those written, and the result is the definition's minimum.
//
// GPU mapping: one thread per segment of kSeg lifted sources (a segment border
// is an extra junction, which changes no minimum); candidates are combined
// with atomic minima in global memory.
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

// Number of cost slopes r_1..r_n that are <= s (strict: < s).  f is the cost
// at offsets 0..n (f[0] = k(-W)).
__device__ int slopes_upto(const double* __restrict__ f, int n, double s, bool strict)
{
    int lo = 0, hi = n;   // the answer lies in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const double r = f[mid] - f[mid - 1];
        if (strict ? r < s : r <= s) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// u[N] periodic -> w[N]: candidates of the lifted sources q - W, q in [0, L),
// L = N + 2W, with offsets s = target - source in [-W, W] (f[j] = k(j - W)).
__global__ __launch_bounds__(kDecompBlock) void k_decomp(const double* __restrict__ u, double* __restrict__ w,
                                                         int N, int W, const double* __restrict__ f, double tol,
                                                         double kabs, unsigned long long* __restrict__ counts)
{
    const int L = N + 2 * W;
    const int n = 2 * W;
    const int s0 = (blockIdx.x * kDecompBlock + threadIdx.x) * kSeg;
    if (s0 >= L - 1) return;
    const int s1 = min(s0 + kSeg, L - 1);   // this thread's pieces cover lifted [s0, s1]
    auto g = [&](int q) {
        int p = (q - W) % N;
        if (p < 0) p += N;
        return u[p];
    };
    unsigned long long pieces = 0, breaks = 0;
    int a = s0;
    while (a < s1) {
        // the piece [a, b] and its type (+1 convex, -1 concave)
        int b = a + 1, typ = 1;
        bool typed = false;
        double last = g(a + 1) - g(a);
        while (b < s1) {
            const double next = g(b + 1) - g(b);
            const double d2 = next - last;
            if (!typed) {
                typ = d2 >= 0.0 ? 1 : -1;
                typed = true;
            } else if (typ == 1 ? d2 < -tol : d2 > tol) {
                breaks++;
                break;
            }
            last = next;
            b++;
        }
        // per-source offset ranges from the (monotone-projected) slopes
        double gp = 0.0, gi = g(a);
        double rho_in = -INFINITY;            // projected slope into source i (none at the first)
        double run = 0.0;                     // running max / min of the piece's slopes
        for (int i = a; i <= b; i++) {
            const double gn = i < b ? g(i + 1) : 0.0;
            double rho_out = INFINITY;        // projected slope out of source i (none at the last)
            if (i < b) {
                const double r = gn - gi;
                run = i == a ? r : (typ == 1 ? fmax(run, r) : fmin(run, r));
                rho_out = run;
            }
            const double wlo = 0x1p-40 * (1.0 + kabs + fabs(gp) + fabs(gi));
            const double whi = 0x1p-40 * (1.0 + kabs + fabs(gi) + fabs(gn));
            const int jlo = i == a ? 0 : slopes_upto(f, n, rho_in - wlo, true);
            const int jhi = i == b ? n : slopes_upto(f, n, rho_out + whi, false);
            // targets x = (i - W) + (j - W), kept when inside [0, N)
            const int x0 = i - 2 * W;
            const int jb = max(jlo, -x0), je = min(jhi, N - 1 - x0);
            for (int j = jb; j <= je; j++) atomicMin(&w[x0 + j], gi + f[j]);
            rho_in = rho_out;
            gp = gi;
            gi = gn;
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
                              double tol, double kabs, const double* hv, unsigned long long* counts, hipStream_t s)
{
    const unsigned gb = (unsigned)((N + kDecompBlock - 1) / kDecompBlock);
    hipLaunchKernelGGL(k_fill, dim3(gb), dim3(kDecompBlock), 0, s, w, (int64_t)N, (double)INFINITY);
    const int L = N + 2 * W;
    const int nseg = (L - 1 + kSeg - 1) / kSeg;
    hipLaunchKernelGGL(k_decomp, dim3((unsigned)((nseg + kDecompBlock - 1) / kDecompBlock)), dim3(kDecompBlock), 0,
                       s, u, w, N, W, kt_centre - W, tol, kabs, counts);
    hipLaunchKernelGGL(k_potential, dim3(gb), dim3(kDecompBlock), 0, s, w, hv, u_out, (int64_t)N);
    return hipGetLastError();
}

}  // namespace lo
