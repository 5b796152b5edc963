/*
 * lo_oracle.c -- plain, slow, FP64 CPU oracle of the fully discrete
 * Lax--Oleinik scheme of Bouillard, Faou and Zavidovique, "Fast weak-KAM
 * integrators for separable Hamiltonian systems".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP path.
 *
 * What it computes (all IEEE binary64, round to nearest, no contraction:
 * build with -ffp-contract=off and without -ffast-math):
 *
 *  - Kinetic cost of a displacement of s cells along axis a (Section 2.3,
 *    eq. cost2, with the mechanical Lagrangian L = |v|^2/2 - P.v - V of
 *    Section 2.1):  k_a(s) = tau * K*_a(s dx_a / tau), evaluated as
 *        d = s * dx;  k = ((0.5 * d) * d) / tau - P * d
 *    or read from a caller table of tau*K*_a for a general convex K*.
 *
 *  - One axis sweep (the 1-D min-plus convolution of eq. eqconvol, taken
 *    along one axis as in Remark rk28) on the periodic grid, over lifted
 *    sources (Remark rk282: the torus scheme is the scheme on periodic lifts):
 *        w[i] = min over e in Z of  fl( u[(i+e) mod N] + k(-e) ),
 *    e = source - target.  Reported argmin: the smallest e attaining the min.
 *    The enumeration of e is restricted to the displacements s = -e with
 *    k(s) <= k(0) + osc(u) + slack: a source outside that set costs more
 *    than staying put (e = 0) and can never attain the min, so the
 *    restriction is exact, not an approximation.
 *
 *  - One time step (eq. eqconvol + Remark rk28): sweep axis 0, then 1, ...,
 *    then the potential step  u+[x] = fl( w[x] - fl(tau * V(t_n, x)) ).
 *
 *  - N steps (eq. uN) with V either static or V(t_n) = sum_m c_m(t_n) phi_m.
 *
 *  - The joint n-D minimum over displacement vectors (the left side of
 *    Remark rk28), for checking the axis splitting on tiny grids.
 *
 *  - The adjoint of the N-step map (piecewise affine in u0 and in the
 *    Fourier coefficients of V): scatter of the upstream gradient onto the
 *    argmin sources, axis by axis in reverse, and the projection of the
 *    accumulated potential gradient onto the basis.
 *
 * Every entry point returns 0 on success, a negative number on bad input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double dx, tau, P;
    const double* tab;  /* optional table of tau*K*(s dx/tau), s in [-half, half] */
    int64_t half;
} orc_kin;

/* Kinetic cost k(s); *ok = 0 when s lies outside a caller table (cost +inf). */
static double kin_eval(const orc_kin* K, int64_t s, int* ok)
{
    if (K->tab) {
        if (s < -K->half || s > K->half) { *ok = 0; return INFINITY; }
        *ok = 1;
        return K->tab[s + K->half];
    }
    *ok = 1;
    double d = (double)s * K->dx;
    double a = 0.5 * d;
    double b = a * d;
    double c = b / K->tau;
    double e = K->P * d;
    return c - e;
}

static int64_t imod(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/* Largest and smallest displacement s with k(s) <= k(0) + osc + slack. */
static int kin_interval(const orc_kin* K, double osc, double umax, int64_t* lo, int64_t* hi)
{
    int ok;
    double k0 = kin_eval(K, 0, &ok);
    if (!ok) return -1;
    double slack = ldexp(1.0 + umax + fabs(k0) + osc, -40);
    double lim = k0 + osc + slack;
    int64_t s = 0;
    for (;;) {
        double v = kin_eval(K, s + 1, &ok);
        if (!ok || !(v <= lim)) break;
        s++;
        if (s > ((int64_t)1 << 40)) return -2;
    }
    *hi = s;
    s = 0;
    for (;;) {
        double v = kin_eval(K, s - 1, &ok);
        if (!ok || !(v <= lim)) break;
        s--;
        if (s < -((int64_t)1 << 40)) return -2;
    }
    *lo = s;
    return 0;
}

static void array_stats(const double* u, int64_t npts, double* osc, double* umax)
{
    double mx = -INFINITY, mn = INFINITY, am = 0.0;
    for (int64_t i = 0; i < npts; i++) {
        double v = u[i];
        if (v > mx) mx = v;
        if (v < mn) mn = v;
        double a = fabs(v);
        if (a > am) am = a;
    }
    *osc = mx - mn;
    *umax = am;
}

static int64_t prod(const int64_t* n, int lo, int hi)
{
    int64_t p = 1;
    for (int a = lo; a < hi; a++) p *= n[a];
    return p;
}

/*
 * One sweep along `axis`.  u and w may not alias.  argmin (nullable) gets the
 * offset e = source - target of the smallest-e minimiser (lifted index).
 */
int orc_sweep(int ndim, const int64_t* n, int axis, double dx, double tau, double P,
              const double* ktab, int64_t khalf,
              const double* u, double* w, int32_t* argmin)
{
    if (ndim < 1 || ndim > 3 || axis < 0 || axis >= ndim || !(tau > 0)) return -1;
    orc_kin K = {dx, tau, P, ktab, khalf};
    int64_t npts = prod(n, 0, ndim);
    int64_t L = n[axis];
    int64_t S = prod(n, 0, axis);
    int64_t nlines = npts / L;
    double osc, umax;
    array_stats(u, npts, &osc, &umax);
    int64_t slo, shi;
    if (kin_interval(&K, osc, umax, &slo, &shi) != 0) return -2;
    int64_t ne = shi - slo + 1;
    /* cost per offset e = -s, e from -shi (lowest source) up to -slo */
    double* kt = (double*)malloc(sizeof(double) * (size_t)ne);
    if (!kt) return -3;
    for (int64_t q = 0; q < ne; q++) {
        int ok;
        int64_t e = -shi + q;
        kt[q] = kin_eval(&K, -e, &ok);
    }
#pragma omp parallel for schedule(static)
    for (int64_t ln = 0; ln < nlines; ln++) {
        int64_t inner = ln % S, outer = ln / S;
        int64_t base = inner + outer * S * L;
        for (int64_t i = 0; i < L; i++) {
            double best = INFINITY;
            int64_t arg = 0;
            for (int64_t q = 0; q < ne; q++) {
                int64_t e = -shi + q;
                int64_t j = imod(i + e, L);
                double v = u[base + S * j] + kt[q];
                if (v < best) { best = v; arg = e; }
            }
            w[base + S * i] = best;
            if (argmin) argmin[base + S * i] = (int32_t)arg;
        }
    }
    free(kt);
    return 0;
}

/*
 * One step of the first discrete semigroup (Section 2.2, eq. cost1) on a 1-D
 * periodic grid of N points with a static potential: the cost of moving from
 * lifted source y to target x in one step is the action of the straight path
 * between them, tau K*((x - y) dx / tau) minus the time integral of V along
 * the path.  The integral is taken by the trapezoid rule over the grid points
 * the path crosses, each crossed after tau / m of time (m = |x - y|), on the
 * table hv = fl(tau V):
 *     I(y, x) = hv[x]                                                m = 0,
 *     I(y, x) = (hv[y]/2 + hv[y+d] + ... + hv[x-d] + hv[x]/2) / m      m > 0,
 * d = sign(x - y), summed in path order from y.  Then
 *     w[x] = min over lifted y of fl( fl(u[y] + k(x - y)) - I(y, x) ),
 * with argmin the lowest lifted source (smallest e = y - x).  A source whose
 * kinetic cost exceeds k(0) + osc(u) + osc(hv) cannot beat staying put, so
 * that interval is enumerated.  hv may be NULL (V = 0).
 */
int orc_semigroup1_step(int64_t N, double dx, double tau, double P, const double* ktab, int64_t khalf,
                        const double* hv, const double* u, double* w, int32_t* argmin)
{
    if (N < 1 || !(tau > 0)) return -1;
    orc_kin K = {dx, tau, P, ktab, khalf};
    double osc, umax, hosc = 0.0, hmax = 0.0;
    array_stats(u, N, &osc, &umax);
    if (hv) array_stats(hv, N, &hosc, &hmax);
    int64_t slo, shi;
    if (kin_interval(&K, osc + hosc, umax + hmax, &slo, &shi) != 0) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) {
        double best = INFINITY;
        int64_t arg = 0;
        for (int64_t e = -shi; e <= -slo; e++) {
            const int64_t y = x + e;   /* lifted source */
            int ok;
            const double k = kin_eval(&K, -e, &ok);
            if (!ok) continue;
            double I = 0.0;
            if (hv) {
                const int64_t m = e < 0 ? -e : e;
                if (m == 0) {
                    I = hv[x];
                } else {
                    const int64_t d = y < x ? 1 : -1;
                    double sum = 0.5 * hv[imod(y, N)];
                    for (int64_t i = 1; i < m; i++) sum = sum + hv[imod(y + i * d, N)];
                    sum = sum + 0.5 * hv[x];
                    I = sum / (double)m;
                }
            }
            const double v = (u[imod(y, N)] + k) - I;
            if (v < best) { best = v; arg = e; }
        }
        w[x] = best;
        if (argmin) argmin[x] = (int32_t)arg;
    }
    return 0;
}

/* Potential synthesis  V[x] = sum_m fl(c_m * phi_m[x]), summed in m order. */
int orc_potential(int64_t npts, int nmodes, const double* basis, const double* coef, double* V)
{
    if (nmodes < 0) return -1;
    for (int64_t x = 0; x < npts; x++) {
        double v = 0.0;
        for (int m = 0; m < nmodes; m++) {
            double t = coef[m] * basis[(int64_t)m * npts + x];
            v = v + t;
        }
        V[x] = v;
    }
    return 0;
}

/* Potential step  u[x] = fl(w[x] - fl(tau * V[x])). */
static void potential_step(int64_t npts, double tau, const double* V, const double* w, double* u)
{
    for (int64_t x = 0; x < npts; x++) {
        double hv = V ? tau * V[x] : 0.0;
        u[x] = w[x] - hv;
    }
}

/*
 * One time step in place on u.  dx, P: per axis.  ktabs/khalf: per axis
 * caller tables (entries may be NULL: mechanical cost).  V: potential at
 * t_n on the grid (NULL: V = 0).  argmin: NULL or [ndim][npts].
 */
int orc_step(int ndim, const int64_t* n, const double* dx, double tau, const double* P,
             const double* const* ktabs, const int64_t* khalf,
             const double* V, double* u, int32_t* argmin)
{
    int64_t npts = prod(n, 0, ndim);
    double* a = (double*)malloc(sizeof(double) * (size_t)npts);
    double* b = (double*)malloc(sizeof(double) * (size_t)npts);
    if (!a || !b) { free(a); free(b); return -3; }
    memcpy(a, u, sizeof(double) * (size_t)npts);
    for (int ax = 0; ax < ndim; ax++) {
        int rc = orc_sweep(ndim, n, ax, dx[ax], tau, P[ax],
                           ktabs ? ktabs[ax] : NULL, khalf ? khalf[ax] : 0,
                           a, b, argmin ? argmin + (int64_t)ax * npts : NULL);
        if (rc) { free(a); free(b); return rc; }
        double* t = a; a = b; b = t;
    }
    potential_step(npts, tau, V, a, u);
    free(a);
    free(b);
    return 0;
}

/*
 * nsteps steps in place on u.  Potential: if tcoef != NULL, V(t_n) =
 * sum_m tcoef[n*nmodes + m] phi_m (basis [nmodes][npts]); else the static
 * table V (NULL: V = 0).  Step n uses the potential at t_n = t_0 + n tau,
 * i.e. row n0 + n of tcoef.
 */
int orc_run(int ndim, const int64_t* n, const double* dx, double tau, const double* P,
            const double* const* ktabs, const int64_t* khalf,
            const double* V, int nmodes, const double* basis, const double* tcoef,
            int64_t n0, int64_t nsteps, double* u)
{
    int64_t npts = prod(n, 0, ndim);
    double* Vn = NULL;
    if (tcoef) {
        Vn = (double*)malloc(sizeof(double) * (size_t)npts);
        if (!Vn) return -3;
    }
    for (int64_t s = 0; s < nsteps; s++) {
        const double* Vs = V;
        if (tcoef) {
            orc_potential(npts, nmodes, basis, tcoef + (n0 + s) * nmodes, Vn);
            Vs = Vn;
        }
        int rc = orc_step(ndim, n, dx, tau, P, ktabs, khalf, Vs, u, NULL);
        if (rc) { free(Vn); return rc; }
    }
    free(Vn);
    return 0;
}

/*
 * Joint n-D step: min over displacement vectors (s_0, ..., s_{d-1}) of
 * fl(...fl(fl(u(x - s) + k_0(s_0)) + k_1(s_1))... ), then the potential
 * step.  Each s_a ranges over the same rigorous interval as the sweeps
 * (k_a(s_a) <= k_a(0) + osc + slack, with osc of u; since all k_a terms are
 * added to a single source value, a source outside the product of the
 * intervals loses to x itself).  Exponential cost: tiny grids only.
 */
int orc_joint_step(int ndim, const int64_t* n, const double* dx, double tau, const double* P,
                   const double* V, double* u)
{
    if (ndim < 1 || ndim > 3) return -1;
    int64_t npts = prod(n, 0, ndim);
    double osc, umax;
    array_stats(u, npts, &osc, &umax);
    orc_kin K[3];
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < ndim; a++) {
        K[a].dx = dx[a]; K[a].tau = tau; K[a].P = P[a]; K[a].tab = NULL; K[a].half = 0;
        /* the sum of the other axes' costs is at least their minima, which are
           <= their k(0); widen each interval by the other axes' k(0)-min drop */
        if (kin_interval(&K[a], osc, umax, &lo[a], &hi[a])) return -2;
    }
    /* widen: k_b(s_b) may be below k_b(0) by up to drop_b */
    for (int a = 0; a < ndim; a++) {
        double extra = 0.0;
        for (int b = 0; b < ndim; b++) {
            if (b == a) continue;
            int ok;
            double k0 = kin_eval(&K[b], 0, &ok), mn = k0;
            for (int64_t s = lo[b]; s <= hi[b]; s++) {
                double v = kin_eval(&K[b], s, &ok);
                if (v < mn) mn = v;
            }
            extra += k0 - mn;
        }
        if (kin_interval(&K[a], osc + extra, umax, &lo[a], &hi[a])) return -2;
    }
    double* out = (double*)malloc(sizeof(double) * (size_t)npts);
    if (!out) return -3;
    int64_t n0 = n[0], n1 = ndim > 1 ? n[1] : 1, n2 = ndim > 2 ? n[2] : 1;
    for (int64_t i2 = 0; i2 < n2; i2++)
        for (int64_t i1 = 0; i1 < n1; i1++)
            for (int64_t i0 = 0; i0 < n0; i0++) {
                double best = INFINITY;
                int64_t l2 = ndim > 2 ? lo[2] : 0, h2 = ndim > 2 ? hi[2] : 0;
                int64_t l1 = ndim > 1 ? lo[1] : 0, h1 = ndim > 1 ? hi[1] : 0;
                for (int64_t s2 = l2; s2 <= h2; s2++)
                    for (int64_t s1 = l1; s1 <= h1; s1++)
                        for (int64_t s0 = lo[0]; s0 <= hi[0]; s0++) {
                            int ok;
                            int64_t j0 = imod(i0 - s0, n0), j1 = imod(i1 - s1, n1), j2 = imod(i2 - s2, n2);
                            double v = u[j0 + n0 * (j1 + n1 * j2)];
                            v = v + kin_eval(&K[0], s0, &ok);
                            if (ndim > 1) v = v + kin_eval(&K[1], s1, &ok);
                            if (ndim > 2) v = v + kin_eval(&K[2], s2, &ok);
                            if (v < best) best = v;
                        }
                out[i0 + n0 * (i1 + n1 * i2)] = best;
            }
    potential_step(npts, tau, V, out, u);
    free(out);
    return 0;
}

/*
 * Adjoint of  u0 -> u^N  and  c -> u^N  for V = sum_m c_m phi_m (static).
 * Forward: N steps from u0 (written to uT), storing every argmin.
 * Backward, from lambda = grad_uT, for n = N-1 down to 0:
 *   Lambda += lambda                         (u^{n+1} = w - tau V)
 *   for axis a = d-1 down to 0:
 *     lambda'[src(x)] += lambda[x]  for every target x, in increasing x
 * Then grad_u0 = lambda and grad_coef[m] = -tau * sum_x Lambda[x] phi_m[x].
 */
int orc_adjoint(int ndim, const int64_t* n, const double* dx, double tau, const double* P,
                int64_t nsteps, const double* u0, int nmodes, const double* basis,
                const double* coef, const double* grad_uT,
                double* uT, double* grad_u0, double* grad_coef)
{
    int64_t npts = prod(n, 0, ndim);
    double* V = (double*)malloc(sizeof(double) * (size_t)npts);
    int32_t* arg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(npts * ndim) * (size_t)(nsteps > 0 ? nsteps : 1));
    double* lam = (double*)malloc(sizeof(double) * (size_t)npts);
    double* nl = (double*)malloc(sizeof(double) * (size_t)npts);
    double* Lam = (double*)calloc((size_t)npts, sizeof(double));
    if (!V || !arg || !lam || !nl || !Lam) {
        free(V); free(arg); free(lam); free(nl); free(Lam);
        return -3;
    }
    orc_potential(npts, nmodes, basis, coef, V);
    memcpy(uT, u0, sizeof(double) * (size_t)npts);
    for (int64_t s = 0; s < nsteps; s++) {
        int rc = orc_step(ndim, n, dx, tau, P, NULL, NULL, V, uT, arg + s * ndim * npts);
        if (rc) { free(V); free(arg); free(lam); free(nl); free(Lam); return rc; }
    }
    memcpy(lam, grad_uT, sizeof(double) * (size_t)npts);
    for (int64_t s = nsteps - 1; s >= 0; s--) {
        for (int64_t x = 0; x < npts; x++) Lam[x] = Lam[x] + lam[x];
        for (int ax = ndim - 1; ax >= 0; ax--) {
            const int32_t* A = arg + (s * ndim + ax) * npts;
            int64_t L = n[ax], S = prod(n, 0, ax);
            memset(nl, 0, sizeof(double) * (size_t)npts);
            for (int64_t x = 0; x < npts; x++) {
                int64_t i = (x / S) % L;
                int64_t j = imod(i + A[x], L);
                int64_t src = x + (j - i) * S;
                nl[src] = nl[src] + lam[x];
            }
            double* t = lam; lam = nl; nl = t;
        }
    }
    memcpy(grad_u0, lam, sizeof(double) * (size_t)npts);
    for (int m = 0; m < nmodes; m++) {
        double acc = 0.0;
        for (int64_t x = 0; x < npts; x++) acc = acc + Lam[x] * basis[(int64_t)m * npts + x];
        grad_coef[m] = -tau * acc;
    }
    free(V); free(arg); free(lam); free(nl); free(Lam);
    return 0;
}

/* Threads the oracle's parallel loops use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
