// Host side of the C ABI declared in include/lo.h: plan construction (kinetic
// tables of Section 2.3's cost, tau*V, window margins), the time loop of
// eq. uN, HIP graphs for it, diagnostics.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lo_internal.h"

using namespace lo;

struct lo_plan_s {
    lo_desc d;
    int nb = 1;                  // instances advanced together (batched effective Hamiltonians)
    int grid_cap = 1024;         // blocks of a persistent sweep launch (4 per compute unit)
    std::vector<double> Pb;      // [nb][kMaxDim] rotation vector of each instance
    double* dpofs = nullptr;     // device [nb][kMaxDim] P tau / dx per instance (nb > 1)
    double* dPb = nullptr;       // device [nb][kMaxDim] P per instance (nb > 1)
    int ndim = 0;
    int64_t n[kMaxDim] = {1, 1, 1};
    int64_t npts = 0;
    double dx[kMaxDim] = {0, 0, 0};
    int64_t kcap[kMaxDim] = {0, 0, 0};
    std::vector<double> hkt[kMaxDim];   // host kinetic tables, index s + kcap
    double* dkt[kMaxDim] = {nullptr, nullptr, nullptr};        // kinetic table, entry s = -kcap at dkt[a]
    double* dkt_alloc[kMaxDim] = {nullptr, nullptr, nullptr};  // its allocation (+inf pads around a caller table)
    double kmaxabs[kMaxDim] = {0, 0, 0};
    double kzero_drop[kMaxDim] = {0, 0, 0};   // k(0) - min_s k(s), rounded up
    int kvert[kMaxDim] = {0, 0, 0};           // minimising offset of the table (instance 0)
    int vabs[kMaxDim] = {0, 0, 0};            // largest |vertex| of the cost over the instances
    bool user_table[kMaxDim] = {false, false, false};
    int kind[kMaxDim] = {kKindRow, kKindTile, kKindTile};
    int halo[kMaxDim] = {0, 0, 0};       // halo of the next launches (adapted by lo_run)
    int wseg[kMaxDim] = {0, 0, 0};       // widest window of the last segment (or the first step)
    int halo_max[kMaxDim] = {0, 0, 0};   // largest halo the LDS budget allows
    int tile_rows[kMaxDim] = {0, 0, 0};
    int tile_fix[kMaxDim] = {0, 0, 0};    // fast tiles: length chosen by the tuner (0: from the halo)
    int row_ch[kMaxDim] = {8, 8, 8};      // fast rows: points per thread
    bool tuned = false;
    double* tune_u = nullptr;             // the tuner's copy of the input (while it runs)
    bool fast[kMaxDim] = {false, false, false};
    // potential
    int nmodes = 0;
    const double* basis = nullptr;
    std::vector<double> coef;
    std::vector<double> tcoef;
    int64_t ntcoef = 0;
    double* dcoef = nullptr;     // [nmodes] static coefficients
    double* dtcoef = nullptr;    // [ntcoef][nmodes]
    double* dhv = nullptr;       // tau*V (static) or the current step's tau*V(t_n)
    double* dc_w = nullptr;      // lo_run_decomp: sweep output [npts]
    unsigned long long* dc_cnt = nullptr;   // lo_run_decomp: pieces, breaks
    double* sg_q = nullptr;      // lo_run_semigroup1: prefix sums of hv [npts + 1]
    unsigned* sg_sat = nullptr;  // lo_run_semigroup1: an argmin reached the window's edge
    bool has_v = false;
    bool time_dep = false;
    double dvf[kMaxDim] = {0, 0, 0}, dvb[kMaxDim] = {0, 0, 0};
    double hvmax = 0.0;
    // work
    double* scratch = nullptr;
    uint64_t* stats = nullptr;   // kSlots * kSlotStride
    int* win = nullptr;          // windows of the current and next step: [2][2 * kMaxDim]
    WinParams winp;
    WinParams* dwinp = nullptr;  // device copy read by the sweeps that compute the next windows
    bool next_win = true;        // the axis-0 sweep computes the next step's windows
    uint32_t* flags = nullptr;   // kFlagWords
    uint32_t hflags[8] = {0};    // folded: [0] errors, [1+a] window used, [4+a] max |argmin|
    bool have_diag = false;
    bool had_argmin = false;
    // graph cache for lo_run: one executable graph of kGraphSteps steps per
    // (u, stats phase, halo) configuration
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        double* u = nullptr;
        int64_t phase = -1;
        int halo[kMaxDim] = {0, 0, 0};
        uint64_t stamp = 0;
    };
    GraphEntry graphs[4];
    uint64_t graph_clock = 0;
    hipStream_t cap_stream = nullptr;
    // reverse pass work buffers, grown on demand
    double* bw_u = nullptr;          // recomputed state
    double* bw_lam[2] = {nullptr, nullptr};
    double* bw_Lam = nullptr;        // sum over steps of the adjoint of u^{n+1}
    int16_t* bw_arg = nullptr;       // argmins of two segments [2][steps][ndim][npts]
    int64_t bw_arg_steps = 0;        // steps of one of them
    uint32_t* bw_err = nullptr;      // error bits of the reverse sweeps
    uint32_t* bw_amax = nullptr;     // largest |offset| of every (step, axis) whose scatter follows
    int64_t bw_amax_words = 0;
    // pinned host words for the read-backs of flags and offsets during a run:
    // a copy into pageable memory is staged by the runtime, which held back
    // the reverse pass's recompute stream until the other stream had drained
    uint32_t* hpin = nullptr;
    size_t hpin_words = 0;
    bool narrow = false;             // sweeps at one block a CU (the reverse pass's recompute)
    // lo_run in the steady state: each segment's window maxima read back
    // behind it (two pinned buffers of 3 kSpread words, their events)
    uint32_t* seg_pin = nullptr;
    hipEvent_t seg_ev[2] = {nullptr, nullptr};
    hipStream_t bw_stream = nullptr; // lo_backward: segment recomputes, beside the reverse sweeps
    hipEvent_t bw_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // start, recomputed[2], reversed[2]
    double* bw_part = nullptr;       // projection partial sums [nmodes][blocks] + [nmodes]
};

namespace {

uint64_t host_enc_neg_inf() { return ~(uint64_t)0xFFF0000000000000ull; }

double host_dec(uint64_t k)
{
    const uint64_t sign = 0x8000000000000000ull;
    uint64_t b = (k & sign) ? (k & ~sign) : ~k;
    double x;
    memcpy(&x, &b, 8);
    return x;
}

// max over the sub-slots of every word of a host copy of a slot
void fold_slot(const uint64_t* raw, double* out)
{
    for (int w = 0; w < kSlotWords; w++) {
        double m = -INFINITY;
        for (int j = 0; j < kSpread; j++) m = std::max(m, host_dec(raw[stat_index(w, j)]));
        out[w] = m;
    }
}

uint32_t fold_window(const uint32_t* f, int a)
{
    uint32_t m = 0;
    for (int j = 0; j < kSpread; j++) m = std::max(m, f[kFlagWin + a * kSpread + j]);
    return m;
}

// Largest of kSpread sub-slot words.
uint32_t fold_spread(const uint32_t* w)
{
    uint32_t m = 0;
    for (int j = 0; j < kSpread; j++) m = std::max(m, w[j]);
    return m;
}

// tau K*(s dx / tau) for K(p) = (p + P)^2 / 2, evaluated in a fixed order.
double mech_cost(int64_t s, double dx, double tau, double P)
{
    const double d = (double)s * dx;
    const double a = 0.5 * d;
    const double b = a * d;
    const double c = b / tau;
    const double e = P * d;
    return c - e;
}

#define HIPCHK(x)                                 \
    do {                                          \
        hipError_t _e = (x);                      \
        if (_e != hipSuccess) return LO_ERR_HIP;  \
    } while (0)

lo_status alloc(void** p, size_t bytes)
{
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return LO_ERR_OOM;
    }
    return LO_OK;
}

void free_plan(lo_plan_t p)
{
    if (!p) return;
    for (int a = 0; a < kMaxDim; a++)
        if (p->dkt_alloc[a]) (void)hipFree(p->dkt_alloc[a]);
    if (p->dcoef) (void)hipFree(p->dcoef);
    if (p->dtcoef) (void)hipFree(p->dtcoef);
    if (p->dhv) (void)hipFree(p->dhv);
    if (p->scratch) (void)hipFree(p->scratch);
    if (p->stats) (void)hipFree(p->stats);
    if (p->flags) (void)hipFree(p->flags);
    if (p->win) (void)hipFree(p->win);
    for (auto& g : p->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->bw_u) (void)hipFree(p->bw_u);
    for (double* l : p->bw_lam)
        if (l) (void)hipFree(l);
    if (p->bw_Lam) (void)hipFree(p->bw_Lam);
    if (p->bw_arg) (void)hipFree(p->bw_arg);
    if (p->bw_err) (void)hipFree(p->bw_err);
    if (p->bw_amax) (void)hipFree(p->bw_amax);
    if (p->hpin) (void)hipHostFree(p->hpin);
    if (p->seg_pin) (void)hipHostFree(p->seg_pin);
    for (auto& e : p->seg_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : p->bw_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->bw_stream) (void)hipStreamDestroy(p->bw_stream);
    if (p->bw_part) (void)hipFree(p->bw_part);
    if (p->dpofs) (void)hipFree(p->dpofs);
    if (p->dPb) (void)hipFree(p->dPb);
    if (p->dwinp) (void)hipFree(p->dwinp);
    if (p->tune_u) (void)hipFree(p->tune_u);
    if (p->dc_w) (void)hipFree(p->dc_w);
    if (p->dc_cnt) (void)hipFree(p->dc_cnt);
    if (p->sg_q) (void)hipFree(p->sg_q);
    if (p->sg_sat) (void)hipFree(p->sg_sat);
    delete p;
}

// Waits for the stream when an entry point returns, on every path: nothing a
// call launched is still running when it reports an error (its caller may
// free the buffers at once).  On success the stream is already idle.
struct StreamDrain {
    hipStream_t s;
    ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

lo_status build_tables(lo_plan_t p)
{
    for (int a = 0; a < p->ndim; a++) {
        std::vector<double>& t = p->hkt[a];
        if (p->d.kstar_tab[a]) {
            const int64_t half = p->d.kstar_half[a];
            if (half < 1 || half > (1 << 20)) return LO_ERR_INVALID;
            p->kcap[a] = half;
            p->user_table[a] = true;
            t.assign(p->d.kstar_tab[a], p->d.kstar_tab[a] + 2 * half + 1);
        } else {
            // every displacement the window can reach on the lifted line: two periods;
            // instance b of a batch at b * (2 cap + 1)
            const int64_t cap = std::min<int64_t>(32767, std::max<int64_t>(64, 2 * p->n[a]));
            p->kcap[a] = cap;
            t.resize((size_t)p->nb * (2 * cap + 1));
            for (int b = 0; b < p->nb; b++)
                for (int64_t s = -cap; s <= cap; s++)
                    t[(size_t)b * (2 * cap + 1) + s + cap] =
                        mech_cost(s, p->dx[a], p->d.tau, p->Pb[(size_t)b * kMaxDim + a]);
        }
        // hypothesis (i): discretely convex (differences nondecreasing), finite
        const size_t len = 2 * (size_t)p->kcap[a] + 1;
        double mx = 0.0, drop = 0.0;
        for (size_t i = 0; i < t.size(); i++) {
            if (!std::isfinite(t[i])) return LO_ERR_INVALID;
            mx = std::max(mx, fabs(t[i]));
        }
        int vabs = 0;
        for (size_t b0 = 0; b0 < t.size(); b0 += len) {
            for (size_t i = b0 + 2; i < b0 + len; i++)
                if (!((t[i] - t[i - 1]) >= (t[i - 1] - t[i - 2]))) return LO_ERR_INVALID;
            const double k0 = t[b0 + p->kcap[a]];
            const auto mit = std::min_element(t.begin() + b0, t.begin() + b0 + len);
            drop = std::max(drop, k0 - *mit);
            const int v = (int)((mit - (t.begin() + b0)) - p->kcap[a]);
            if (b0 == 0) p->kvert[a] = v;
            vabs = std::max(vabs, std::abs(v));
        }
        p->vabs[a] = vabs;
        p->kmaxabs[a] = mx;
        p->kzero_drop[a] = drop * (1.0 + 0x1p-40) + 0x1p-60;
        // A caller table is the cost's whole support (+inf beyond it), and a
        // window may reach its end; the brute kernels' register-blocked loop
        // reads up to kKinPad offsets past either side of the window, so the
        // device copy carries kKinPad entries of +inf on each side.  (A
        // mechanical table spans two periods, beyond every window and halo.)
        const size_t pad = p->user_table[a] ? (size_t)kKinPad : 0;
        std::vector<double> dev(t.size() + 2 * pad, INFINITY);
        std::copy(t.begin(), t.end(), dev.begin() + pad);
        lo_status st = alloc((void**)&p->dkt_alloc[a], sizeof(double) * dev.size());
        if (st) return st;
        p->dkt[a] = p->dkt_alloc[a] + pad;
        HIPCHK(hipMemcpy(p->dkt_alloc[a], dev.data(), sizeof(double) * dev.size(), hipMemcpyHostToDevice));
    }
    return LO_OK;
}

// Bound of tau*(V(x) - V(x + e_a)) and tau*(V(x + e_a) - V(x)) from the hv table.
lo_status add_potential_margins(lo_plan_t p, const double* hv, bool first)
{
    double* d6 = nullptr;
    const size_t words = 16 + kSlotStride;
    lo_status st = alloc((void**)&d6, sizeof(uint64_t) * words);
    if (st) return st;
    std::vector<uint64_t> init(words, host_enc_neg_inf());
    HIPCHK(hipMemcpy(d6, init.data(), sizeof(uint64_t) * words, hipMemcpyHostToDevice));
    if (launch_potential_diffs(hv, p->ndim, p->n, d6, nullptr) != hipSuccess) {
        (void)hipFree(d6);
        return LO_ERR_HIP;
    }
    if (launch_stats(hv, p->ndim, p->n, (uint64_t*)d6 + 16, 1, 0, 0, nullptr) != hipSuccess) {
        (void)hipFree(d6);
        return LO_ERR_HIP;
    }
    std::vector<uint64_t> h(words);
    hipError_t e = hipMemcpy(h.data(), d6, sizeof(uint64_t) * words, hipMemcpyDeviceToHost);
    (void)hipFree(d6);
    if (e != hipSuccess) return LO_ERR_HIP;
    for (int a = 0; a < p->ndim; a++) {
        double f = host_dec(h[a]), b = host_dec(h[3 + a]);
        f = f * (1.0 + 0x1p-40) + 0x1p-60;
        b = b * (1.0 + 0x1p-40) + 0x1p-60;
        if (first) {
            p->dvf[a] = f;
            p->dvb[a] = b;
        } else {
            p->dvf[a] = std::max(p->dvf[a], f);
            p->dvb[a] = std::max(p->dvb[a], b);
        }
    }
    double folded[kSlotWords];
    fold_slot(h.data() + 16, folded);
    double m = folded[6];
    p->hvmax = first ? m : std::max(p->hvmax, m);
    return LO_OK;
}

lo_status setup_potential(lo_plan_t p, const lo_potential* V)
{
    if (!V) return LO_OK;
    const size_t bytes = sizeof(double) * (size_t)p->npts;
    if (V->table) {
        lo_status st = alloc((void**)&p->dhv, bytes);
        if (st) return st;
        HIPCHK(launch_scale(V->table, p->d.tau, p->npts, p->dhv, nullptr));
        p->has_v = true;
    } else if (V->nmodes > 0) {
        if (!V->basis) return LO_ERR_INVALID;
        p->nmodes = V->nmodes;
        p->basis = V->basis;
        lo_status st = alloc((void**)&p->dhv, bytes);
        if (st) return st;
        if (V->tcoef) {
            if (V->ntcoef < 1) return LO_ERR_INVALID;
            p->time_dep = true;
            p->ntcoef = V->ntcoef;
            p->tcoef.assign(V->tcoef, V->tcoef + V->ntcoef * V->nmodes);
            st = alloc((void**)&p->dtcoef, sizeof(double) * p->tcoef.size());
            if (st) return st;
            HIPCHK(hipMemcpy(p->dtcoef, p->tcoef.data(), sizeof(double) * p->tcoef.size(),
                             hipMemcpyHostToDevice));
        } else {
            if (!V->coef) return LO_ERR_INVALID;
            p->coef.assign(V->coef, V->coef + V->nmodes);
            st = alloc((void**)&p->dcoef, sizeof(double) * p->nmodes);
            if (st) return st;
            HIPCHK(hipMemcpy(p->dcoef, p->coef.data(), sizeof(double) * p->nmodes, hipMemcpyHostToDevice));
            HIPCHK(launch_synth_hv(p->basis, p->dcoef, p->nmodes, p->npts, p->d.tau, p->dhv, nullptr));
        }
        p->has_v = true;
    }
    if (!p->has_v) return LO_OK;
    if (p->time_dep) {
        for (int64_t k = 0; k < p->ntcoef; k++) {
            HIPCHK(launch_synth_hv(p->basis, p->dtcoef + k * p->nmodes, p->nmodes, p->npts, p->d.tau, p->dhv,
                                   nullptr));
            lo_status st = add_potential_margins(p, p->dhv, k == 0);
            if (st) return st;
        }
    } else {
        lo_status st = add_potential_margins(p, p->dhv, true);
        if (st) return st;
    }
    HIPCHK(hipDeviceSynchronize());
    return LO_OK;
}

// Lines side by side in axis a's fast tiles, and the tile length: a tile of one
// line (an axis with fewer than 16 lines) is 4x longer, so that a block still
// has as many targets.
int tile_lines_of(lo_plan_t p, int a) { return fast_tile_lines(p->npts / p->n[a]); }
int tile_len(lo_plan_t p, int a, bool wide) { return (wide ? 256 : 128) * (tile_lines_of(p, a) == 1 ? 4 : 1); }

void choose_kernels(lo_plan_t p)
{
    int dev = 0, lds_max = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds_max = 65536;
    (void)hipGetLastError();
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        p->grid_cap = 4 * ncu;
    (void)hipGetLastError();
    const size_t budget = std::min<size_t>((size_t)lds_max, 64 * 1024);
    const size_t fbudget = std::min<size_t>((size_t)lds_max, 96 * 1024);
    const bool fast = p->d.method == LO_FAST;
    for (int a = 0; a < p->ndim; a++) {
        const int64_t N = p->n[a];
        p->fast[a] = fast;
        // fast: whole rows of a multiple of 8 points for axis 0, tiles otherwise
        const bool row_ok = a == 0 && N <= 2048 &&
                            (p->fast[a] ? N % 8 == 0 && fast_lds_for(kKindRow, N, 0, 1, 1) <= fbudget
                                        : row_lds_bytes(N, 8) <= budget);
        if (row_ok) {
            p->kind[a] = kKindRow;
            // the fast row kernel wraps claims once around the row: its cost table stays below N
            int64_t H = p->fast[a] ? std::min<int64_t>(N - 1, 512) : std::min<int64_t>(N, 1024);
            if (p->fast[a])
                while (H > 1 && fast_lds_for(kKindRow, N, 0, (int)H, 1) > fbudget) H = H * 7 / 8;
            else
                while (H > 8 && row_lds_bytes(N, (int)H) > budget) H = H * 7 / 8;
            p->halo[a] = (int)std::max<int64_t>(H, 1);
            p->halo_max[a] = p->halo[a];
            p->tile_rows[a] = 0;
            // rows of at most 1024 points in sweeps of 2^24 points or more take
            // 4 points a thread (blocks of 512): the faster shape on every such
            // grid timed (256^3; batches of 512^2, 768^2 and 1024^2 grids)
            p->row_ch[a] = N <= 1024 && p->npts * p->nb >= ((int64_t)1 << 24) ? 4 : 8;
        } else {
            p->kind[a] = kKindTile;
            int R = p->fast[a] ? tile_len(p, a, true) : (int)std::min<int64_t>(N, 128);
            int H = (int)std::min<int64_t>(N, p->fast[a] ? 512 : 256);
            if (p->fast[a])
                while (H > 8 && fast_lds_for(kKindTile, N, R, H, tile_lines_of(p, a)) > fbudget) H -= 4;
            else
                while (H > 8 && tile_lds_bytes(H) > budget) H -= 8;
            p->tile_rows[a] = R;
            p->halo[a] = H;
            p->halo_max[a] = H;
        }
    }
}

double slack_extra(lo_plan_t p)
{
    double s = p->hvmax;
    for (int a = 0; a < p->ndim; a++) s += p->kmaxabs[a];
    return s;
}

uint64_t* slot(lo_plan_t p, int64_t n) { return p->stats + (size_t)(((n % kSlots) + kSlots) % kSlots) * kSlotStride; }



// Buffers of the sweeps of one step: in/out per axis so that the result lands in u.
void sweep_buffers(lo_plan_t p, double* u, double* in[kMaxDim], double* out[kMaxDim])
{
    int tiles = 0;
    for (int a = 0; a < p->ndim; a++) tiles += p->kind[a] == kKindTile;
    bool flip_row = (tiles % 2) == 1;  // one row sweep goes out of place to keep the parity
    double* cur = u;
    for (int a = 0; a < p->ndim; a++) {
        in[a] = cur;
        bool oop = p->kind[a] == kKindTile || (flip_row && p->kind[a] == kKindRow);
        if (p->kind[a] == kKindRow && flip_row) flip_row = false;
        double* nxt = oop ? (cur == u ? p->scratch : u) : cur;
        out[a] = nxt;
        cur = nxt;
    }
}

void fill_winparams(lo_plan_t p)
{
    WinParams& W = p->winp;
    memset(&W, 0, sizeof(W));
    W.ndim = p->ndim;
    W.slack_extra = slack_extra(p);
    double drop = 0.0;   // a sweep raises the max by at most k(0) and lowers the min by at most -min k
    for (int a = 0; a < p->ndim; a++) {
        W.k[a] = p->dkt[a] + p->kcap[a];
        W.kcap[a] = p->kcap[a];
        W.dvf[a] = p->dvf[a];
        W.dvb[a] = p->dvb[a];
        W.osc_extra[a] = drop;
        drop += p->kzero_drop[a];
        W.cq[a] = p->dx[a] * p->dx[a] / (2.0 * p->d.tau);
        W.pofs[a] = p->d.P[a] * p->d.tau / p->dx[a];
        W.quad[a] = p->user_table[a] ? 0 : 1;
        W.cap_err[a] = p->user_table[a] ? 0 : 1;
        W.wfix[a] = p->d.window[a];
        W.bk[a] = 2 * p->kcap[a] + 1;
        W.dx[a] = p->dx[a];
        W.P[a] = p->d.P[a];
    }
    W.tau = p->d.tau;
    W.P_b = p->nb > 1 ? p->dPb : nullptr;
    W.b_stats = (int64_t)kSlots * kSlotStride;
    W.b_win = 4 * kMaxDim;
    W.pofs_b = p->nb > 1 ? p->dpofs : nullptr;
    W.lag = 1;
    W.hv_osc = 2.0 * p->hvmax;   // tau * (max V - min V) <= 2 max |tau V|
}

lo_status upload_winparams(lo_plan_t p)
{
    if (!p->dwinp) {
        lo_status st = alloc((void**)&p->dwinp, sizeof(WinParams));
        if (st) return st;
    }
    HIPCHK(hipMemcpy(p->dwinp, &p->winp, sizeof(WinParams), hipMemcpyHostToDevice));
    return LO_OK;
}

int choose_halo(lo_plan_t p, int a, int W)
{
    if (p->d.window[a] > 0) W = p->d.window[a];
    int H = W + std::max(16, W / 8);
    H = (H + 7) / 8 * 8;
    H = std::max(8, std::min(H, p->halo_max[a]));
    // fast tiles: longer tiles when the window's halo is wide (fewer halo
    // sources per target), shorter ones keep more blocks resident otherwise;
    // the last axis (potential step) always takes the longer tiles, whose
    // blocks load their tau V values before the claims
    if (p->fast[a] && p->kind[a] == kKindTile)
        p->tile_rows[a] = p->tile_fix[a] > 0 ? p->tile_fix[a] : tile_len(p, a, H >= 40 || a == p->ndim - 1);
    // the fast sweeps stage a band of offsets centred on the cost's vertex
    // (so that its loads need not wait for the window); the window lies
    // within |vertex| + W of it
    if (p->fast[a] && p->d.window[a] <= 0)
        H = std::max(8, std::min((H + p->vabs[a] + 7) / 8 * 8, p->halo_max[a]));
    return H;
}

// Halos from the widest window the kernels used since the last call.
// At least `words` pinned host words (nullptr if they cannot be had).
uint32_t* host_words(lo_plan_t p, size_t words)
{
    if (words > p->hpin_words) {
        if (p->hpin) (void)hipHostFree(p->hpin);
        p->hpin = nullptr;
        p->hpin_words = 0;
        if (hipHostMalloc((void**)&p->hpin, sizeof(uint32_t) * words, hipHostMallocDefault) != hipSuccess) {
            p->hpin = nullptr;
            return nullptr;
        }
        p->hpin_words = words;
    }
    return p->hpin;
}

lo_status adapt_from_flags(lo_plan_t p, hipStream_t s)
{
    uint32_t* f = host_words(p, kFlagWords);
    if (!f) return LO_ERR_HIP;
    HIPCHK(hipMemcpyAsync(f, p->flags, sizeof(uint32_t) * kFlagWords, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int a = 0; a < p->ndim; a++) {
        const uint32_t wu = fold_window(f, a);
        p->hflags[1 + a] = std::max(p->hflags[1 + a], wu);
        p->halo[a] = choose_halo(p, a, (int)wu);
        p->wseg[a] = (int)wu;
    }
    // restart the per-segment window maxima (error bits and argmin maxima stay)
    HIPCHK(hipMemsetAsync(p->flags + kFlagWin, 0, sizeof(uint32_t) * 3 * kSpread, s));
    return LO_OK;
}

lo_status enqueue_step(lo_plan_t p, double* u, int64_t n, int16_t* argmin, hipStream_t s,
                       hipEvent_t* ev = nullptr, uint32_t* amax_out = nullptr)
{
    const double* hv = p->has_v ? p->dhv : nullptr;
    if (p->time_dep) {
        if (n < 0 || n >= p->ntcoef) return LO_ERR_INVALID;
        HIPCHK(launch_synth_hv(p->basis, p->dtcoef + n * p->nmodes, p->nmodes, p->npts, p->d.tau, p->dhv, s));
    }
    double* in[kMaxDim];
    double* out[kMaxDim];
    sweep_buffers(p, u, in, out);
    const double sx = slack_extra(p);
    for (int a = 0; a < p->ndim; a++) {
        SweepArgs A;
        memset(&A, 0, sizeof(A));
        A.g.n = p->n[a];
        A.g.stride = 1;
        for (int b = 0; b < a; b++) A.g.stride *= p->n[b];
        A.g.nlines = p->npts / p->n[a];
        A.kin.k = p->dkt[a] + p->kcap[a];
        A.kin.kcap = p->kcap[a];
        A.axis = a;
        A.ndim = p->ndim;
        A.wfix = p->d.window[a];
        A.slack_extra = sx;
        A.dv_fwd = p->dvf[a];
        A.dv_bwd = p->dvb[a];
        A.osc_extra = p->winp.osc_extra[a];
        A.kind = p->kind[a];
        A.cap_is_error = p->user_table[a] ? 0 : 1;
        A.stats_in = slot(p, n);
        A.stats_out = slot(p, n + 1);
        A.stats_clear = a == 0 ? slot(p, n + 2) : nullptr;
        A.win_in = p->win + (size_t)(((n % 2) + 2) % 2) * 2 * kMaxDim;
        A.grid_cap = p->grid_cap;
        A.row_ch = p->row_ch[a];
        A.nb = p->nb;
        A.b_u = p->npts;
        A.b_k = 2 * p->kcap[a] + 1;
        A.b_stats = (int64_t)kSlots * kSlotStride;
        A.b_win = 4 * kMaxDim;
        A.pofs_b = p->nb > 1 ? p->dpofs : nullptr;
        A.flags = p->flags;
        A.hv = a == p->ndim - 1 ? hv : nullptr;
        A.argmin = argmin ? argmin + (size_t)a * p->npts : nullptr;
        A.amax_out = argmin ? amax_out : nullptr;
        A.halo = p->halo[a];
        A.tile_rows = p->tile_rows[a];
        if (argmin && p->fast[a]) {
            // argmin sweeps keep the default shapes (the tuner times the plain sweeps)
            A.row_ch = 8;
            if (p->kind[a] == kKindTile) A.tile_rows = p->halo[a] >= 40 ? 256 : 128;
        }
        A.fast = p->fast[a] ? 1 : 0;
        // a grid whose u fits the last-level caches of the XCDs (2^22 points, 32 MB)
        // is written through them by the tile sweeps: the kernel's end then has
        // little to write back (a larger grid's dirty lines leave the caches
        // during the sweep anyway, and writing through costs it time)
        A.wt = p->npts * p->nb <= ((int64_t)1 << 22) ? 1 : 0;
        A.narrow = p->narrow ? 1 : 0;
        A.quad = p->user_table[a] ? 0 : 1;
        A.cq = p->dx[a] * p->dx[a] / (2.0 * p->d.tau);
        A.inv2c = 1.0 / (2.0 * A.cq);
        A.pofs = p->d.P[a] * p->d.tau / p->dx[a];
        A.kslack = 0x1p-40 * (1.0 + p->kmaxabs[a]);
        A.kvert = p->kvert[a];
        if (a == 0 && p->next_win) {
            // windows of step n + 1 from the statistics of u^n (slot n), one step
            // early: block 0 of the row, one-line tile and brute sweeps computes
            // them after its own work; beside a fast sweep of 16-line tiles
            // (which keeps its registers for the claims) a small kernel does
            int* next = p->win + (size_t)((((n + 1) % 2) + 2) % 2) * 2 * kMaxDim;
            if (p->fast[0] && p->kind[0] == kKindTile && p->d.window[0] <= 0 && tile_lines_of(p, 0) > 1) {
                HIPCHK(launch_windows(p->winp, slot(p, n), next, p->flags, p->nb, s));
            } else {
                A.winp_dev = p->dwinp;
                A.win_slot = slot(p, n);
                A.win_next = next;
            }
        }
        if (ev) {
            A.ev_start = ev[2 * a];
            A.ev_stop = ev[2 * a + 1];
        }
        HIPCHK(launch_sweep(p->d.method, in[a], out[a], A, s));
    }
    if (out[p->ndim - 1] != u)
        HIPCHK(hipMemcpyAsync(u, out[p->ndim - 1], sizeof(double) * p->npts * p->nb, hipMemcpyDeviceToDevice, s));
    return LO_OK;
}

// wait: read the first windows back and size the halos from them (a host
// wait); otherwise the halos stay as they are (they choose kernel paths,
// never values) and the first windows are left in the flags' maxima
lo_status prologue(lo_plan_t p, const double* u, int64_t n0, hipStream_t s, bool wait = true)
{
    HIPCHK(hipMemsetAsync(p->flags, 0, sizeof(uint32_t) * kFlagWords, s));
    HIPCHK(launch_clear_slots(p->stats, p->nb, s));
    HIPCHK(launch_stats(u, p->ndim, p->n, slot(p, n0), p->nb, p->npts, (int64_t)kSlots * kSlotStride, s));
    for (int i = 0; i < 8; i++) p->hflags[i] = 0;
    // every instance's first windows on the device (the bounds the sweeps
    // compute for the following steps), halos from their maximum
    HIPCHK(launch_windows(p->winp, slot(p, n0), p->win + (size_t)(((n0 % 2) + 2) % 2) * 2 * kMaxDim, p->flags, p->nb,
                          s));
    return wait ? adapt_from_flags(p, s) : LO_OK;
}

lo_status finish(lo_plan_t p, hipStream_t s, bool argmin)
{
    HIPCHK(hipStreamSynchronize(s));
    uint32_t f[kFlagWords];
    HIPCHK(hipMemcpy(f, p->flags, sizeof(uint32_t) * kFlagWords, hipMemcpyDeviceToHost));
    p->hflags[0] = f[0];
    for (int a = 0; a < kMaxDim; a++) {
        p->hflags[1 + a] = std::max(p->hflags[1 + a], a < p->ndim ? fold_window(f, a) : 0u);
        p->hflags[4 + a] = a < p->ndim ? fold_spread(f + kFlagAmax + a * kSpread) : 0u;
    }
    p->have_diag = true;
    p->had_argmin = argmin;
    if (p->hflags[0] & (kErrWindowCap | kErrWindowEdge | kErrFastPath)) return LO_ERR_WINDOW;
    if (p->hflags[0] & kErrArgRange) return LO_ERR_UNSUPPORTED;
    return LO_OK;
}

bool graphable(lo_plan_t p) { return !(p->d.flags & LO_FLAG_NO_GRAPH) && !p->time_dep; }

constexpr int kGraphSteps = 30;   // multiple of the 3 stats slots

// Work buffers of lo_backward for segments of `steps` steps.
lo_status backward_buffers(lo_plan_t p, int64_t steps, bool coef)
{
    const size_t bytes = sizeof(double) * (size_t)p->npts;
    lo_status st = LO_OK;
    if (!p->bw_u) st = alloc((void**)&p->bw_u, bytes);
    for (int i = 0; i < 2 && !st; i++)
        if (!p->bw_lam[i]) st = alloc((void**)&p->bw_lam[i], bytes);
    if (!st && coef && !p->bw_Lam) st = alloc((void**)&p->bw_Lam, bytes);
    if (!st && coef && !p->bw_part)
        st = alloc((void**)&p->bw_part, sizeof(double) * (size_t)p->nmodes * (project_blocks(p->npts) + 1));
    if (!st && !p->bw_err) st = alloc((void**)&p->bw_err, sizeof(uint32_t));
    if (!st && steps > p->bw_arg_steps) {
        if (p->bw_arg) (void)hipFree(p->bw_arg);
        p->bw_arg = nullptr;
        p->bw_arg_steps = 0;
        st = alloc((void**)&p->bw_arg, sizeof(int16_t) * 2 * (size_t)steps * p->ndim * p->npts);
        if (!st) p->bw_arg_steps = steps;
    }
    return st;
}

// At least `words` words for the per-(step, axis) largest offsets.
lo_status amax_buffer(lo_plan_t p, int64_t words)
{
    if (words <= p->bw_amax_words) return LO_OK;
    if (p->bw_amax) (void)hipFree(p->bw_amax);
    p->bw_amax = nullptr;
    p->bw_amax_words = 0;
    lo_status st = alloc((void**)&p->bw_amax, sizeof(uint32_t) * (size_t)std::max<int64_t>(words, 1));
    if (!st) p->bw_amax_words = words;
    return st;
}

// Launch-shape tuner (LO_FLAG_AUTOTUNE).  The shapes: points per thread of a
// row sweep (8, or 4 with blocks of twice the threads) and targets per tile of
// the last axis's tile sweep (256 or 128; other tile axes keep their default,
// which follows the window during the run).  Every shape computes the same values (the
// minimum over a target's claimants does not depend on how sources are
// grouped), so the choice only affects speed.
//  - Steady state: the windows of the first steps of a run from smooth data
//    are several times wider than later on, so the tuner first advances a copy
//    of u by kTuneWarm steps with the default shapes, and times from there.
//  - Both shapes of every axis are timed over kTuneSteps steps from that same
//    state, each sweep's kernel between its own start and stop events, twice
//    and alternately (the faster of the two counts); an axis leaves its
//    default only for a gain of more than 3%.
//  - Choices are kept per (grid, instances, method, sweep kinds, cost kinds)
//    for the life of the process, and in the file named by LO_TUNE_CACHE when
//    that is set (one choice a line, read once, appended); a plan whose key is
//    known takes the choice without timing anything.
constexpr int kTuneWarm = 60;
constexpr int kTuneSteps = 8;

lo_status run_steps(lo_plan_t p, double* u, int64_t n0, int64_t nsteps, int64_t ckpt_every, double* ckpt,
                    hipStream_t s);

struct TuneChoice {
    int row_ch[kMaxDim];
    int tile_fix[kMaxDim];
};

std::mutex g_tune_mutex;
std::vector<std::pair<std::string, TuneChoice>> g_tune_cache;
bool g_tune_file_read = false;

std::string tune_key(lo_plan_t p)
{
    char buf[256];
    int k = snprintf(buf, sizeof(buf), "d%d nb%d m%d", p->ndim, p->nb, p->d.method);
    for (int a = 0; a < p->ndim && k < (int)sizeof(buf); a++)
        k += snprintf(buf + k, sizeof(buf) - k, " n%lld k%d q%d", (long long)p->n[a], p->kind[a],
                      p->user_table[a] ? 0 : 1);
    return std::string(buf);
}

// the cache file: lines "<key> | row_ch0 row_ch1 row_ch2 tile0 tile1 tile2"
void tune_file_read()
{
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = getenv("LO_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        char* bar = strchr(line, '|');
        if (!bar) continue;
        std::string key(line, bar - line);
        while (!key.empty() && key.back() == ' ') key.pop_back();
        TuneChoice c;
        if (sscanf(bar + 1, "%d %d %d %d %d %d", &c.row_ch[0], &c.row_ch[1], &c.row_ch[2], &c.tile_fix[0],
                   &c.tile_fix[1], &c.tile_fix[2]) == 6)
            g_tune_cache.emplace_back(key, c);
    }
    fclose(f);
}

void tune_file_append(const std::string& key, const TuneChoice& c)
{
    const char* path = getenv("LO_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s | %d %d %d %d %d %d\n", key.c_str(), c.row_ch[0], c.row_ch[1], c.row_ch[2], c.tile_fix[0],
            c.tile_fix[1], c.tile_fix[2]);
    fclose(f);
}

void apply_choice(lo_plan_t p, const TuneChoice& c)
{
    for (int a = 0; a < p->ndim; a++) {
        p->row_ch[a] = c.row_ch[a];
        p->tile_fix[a] = c.tile_fix[a];
        if (p->kind[a] == kKindTile && c.tile_fix[a] > 0) p->tile_rows[a] = c.tile_fix[a];
    }
}

// Time kTuneSteps steps of the current shapes from `from` (copied into tune_u
// first); ms[a] receives each axis' summed kernel time.
lo_status time_shapes(lo_plan_t p, const double* from, int64_t n0, double* ms, hipStream_t s)
{
    const size_t bytes = sizeof(double) * (size_t)p->npts * p->nb;
    HIPCHK(hipMemcpyAsync(p->tune_u, from, bytes, hipMemcpyDeviceToDevice, s));
    lo_status st = prologue(p, p->tune_u, n0, s);
    if (st) return st;
    std::vector<hipEvent_t> ev((size_t)kTuneSteps * 2 * p->ndim, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) st = LO_ERR_HIP;
    for (int k = 0; k < kTuneSteps && !st; k++)
        st = enqueue_step(p, p->tune_u, n0 + k, nullptr, s, &ev[(size_t)k * 2 * p->ndim]);
    if (!st && hipStreamSynchronize(s) != hipSuccess) st = LO_ERR_HIP;
    for (int a = 0; a < p->ndim; a++) ms[a] = 0.0;
    for (int k = 1; k < kTuneSteps && !st; k++)   // the first step warms the shape up
        for (int a = 0; a < p->ndim; a++) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[(size_t)k * 2 * p->ndim + 2 * a], ev[(size_t)k * 2 * p->ndim + 2 * a + 1]) !=
                hipSuccess)
                st = LO_ERR_HIP;
            ms[a] += t;
        }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

lo_status autotune(lo_plan_t p, const double* u, int64_t n0, hipStream_t s)
{
    p->tuned = true;
    bool any = false;
    for (int a = 0; a < p->ndim; a++) any |= p->fast[a];
    if (!any) return LO_OK;
    const std::string key = tune_key(p);
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        tune_file_read();
        for (auto& e : g_tune_cache)
            if (e.first == key) {
                apply_choice(p, e.second);
                return LO_OK;
            }
    }
    const size_t bytes = sizeof(double) * (size_t)p->npts * p->nb;
    double* adv = nullptr;   // the steady state the shapes are timed from
    lo_status st = alloc((void**)&adv, bytes);
    if (!st && !p->tune_u) st = alloc((void**)&p->tune_u, bytes);
    if (st) {
        if (adv) (void)hipFree(adv);
        return st;
    }
    // both buffers are the tuner's own: freed when it returns (after its
    // final synchronisation), so that a tuned plan holds what a default one does
    struct Free {
        double* q;
        double** t;
        ~Free()
        {
            (void)hipFree(q);
            (void)hipFree(*t);
            *t = nullptr;
        }
    } free_adv{adv, &p->tune_u};
    HIPCHK(hipMemcpyAsync(adv, u, bytes, hipMemcpyDeviceToDevice, s));
    st = prologue(p, adv, n0, s);
    if (!st) st = run_steps(p, adv, n0, kTuneWarm, 0, nullptr, s);
    if (!st) st = adapt_from_flags(p, s);
    if (st) return st;
    const int64_t t0 = n0 + kTuneWarm;
    TuneChoice def, alt, best;
    for (int a = 0; a < kMaxDim; a++) {
        def.row_ch[a] = a < p->ndim ? p->row_ch[a] : 8;
        alt.row_ch[a] = 12 - def.row_ch[a];
        // tile lengths: the last axis (fixed at the longer tiles by default)
        // is tuned; the others keep their default, which follows the window
        // (long tiles while it is wide, short ones after), a better schedule
        // over a run than any one length timed from one state
        const bool last = a == p->ndim - 1;
        def.tile_fix[a] = last && p->kind[a] == kKindTile ? tile_len(p, a, true) : 0;
        alt.tile_fix[a] = last && p->kind[a] == kKindTile ? tile_len(p, a, false) : 0;
    }
    {
        // two rounds, alternating the shapes; the faster round of each counts
        double ms_def[kMaxDim], ms_alt[kMaxDim], m[kMaxDim];
        for (int a = 0; a < kMaxDim; a++) ms_def[a] = ms_alt[a] = INFINITY;
        for (int round = 0; round < 2 && !st; round++) {
            apply_choice(p, def);
            st = time_shapes(p, adv, t0, m, s);
            for (int a = 0; a < p->ndim && !st; a++) ms_def[a] = std::min(ms_def[a], m[a]);
            if (st) break;
            apply_choice(p, alt);
            st = time_shapes(p, adv, t0, m, s);
            for (int a = 0; a < p->ndim && !st; a++) ms_alt[a] = std::min(ms_alt[a], m[a]);
        }
        if (st) return st;
        best = def;
        for (int a = 0; a < p->ndim; a++)
            if (p->fast[a] && ms_alt[a] < 0.97 * ms_def[a]) {
                best.row_ch[a] = alt.row_ch[a];
                best.tile_fix[a] = alt.tile_fix[a];
            }
        if (getenv("LO_TUNE_LOG"))
            for (int a = 0; a < p->ndim; a++)
                fprintf(stderr, "lo tune %s axis %d: default (%d pts/thread, %d targets) %.4f ms, "
                        "other (%d, %d) %.4f ms over %d steps -> %s\n", key.c_str(), a, def.row_ch[a],
                        def.tile_fix[a], ms_def[a], alt.row_ch[a], alt.tile_fix[a], ms_alt[a], kTuneSteps - 1,
                        best.row_ch[a] == def.row_ch[a] && best.tile_fix[a] == def.tile_fix[a] ? "default" : "other");
        apply_choice(p, best);
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        g_tune_cache.emplace_back(key, best);
        tune_file_append(key, best);
    }
    // the run proper starts from its own prologue; captured steps used other shapes
    for (auto& g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = lo_plan_s::GraphEntry();
    }
    return hipStreamSynchronize(s) == hipSuccess ? LO_OK : LO_ERR_HIP;
}

// A plan for nb instances that share the grid, time step and potential and
// differ in the rotation vector (Pb: [nb][kMaxDim]); nb > 1 is the batched
// path of lo_effective_H (mechanical costs only).
lo_status plan_create(const lo_desc* desc, const lo_potential* V, int nb, const double* Pb, lo_plan_t* out)
{
    if (!desc || !out || !Pb || nb < 1) return LO_ERR_INVALID;
    *out = nullptr;
    if (desc->ndim < 1 || desc->ndim > kMaxDim) return LO_ERR_INVALID;
    if (!(desc->tau > 0) || !std::isfinite(desc->tau)) return LO_ERR_INVALID;
    if (desc->method != LO_BRUTE && desc->method != LO_FAST) return LO_ERR_INVALID;
    if (nb > 1)
        for (int a = 0; a < desc->ndim; a++)
            if (desc->kstar_tab[a]) return LO_ERR_UNSUPPORTED;
    lo_plan_t p = new (std::nothrow) lo_plan_s();
    if (!p) return LO_ERR_OOM;
    p->d = *desc;
    p->nb = nb;
    p->Pb.assign((size_t)nb * kMaxDim, 0.0);
    for (int a = 0; a < desc->ndim; a++) p->d.P[a] = Pb[a];
    p->ndim = desc->ndim;
    p->npts = 1;
    for (int a = 0; a < p->ndim; a++) {
        if (desc->n[a] < 3 || desc->n[a] > (1ll << 31)) {
            free_plan(p);
            return LO_ERR_INVALID;
        }
        if (!(desc->period[a] > 0) || !std::isfinite(desc->period[a]) || !std::isfinite(Pb[a]) ||
            desc->window[a] < 0) {
            free_plan(p);
            return LO_ERR_INVALID;
        }
        p->n[a] = desc->n[a];
        p->npts *= desc->n[a];
        p->dx[a] = desc->period[a] / (double)desc->n[a];
    }
    for (int b = 0; b < nb; b++)
        for (int a = 0; a < p->ndim; a++) {
            if (!std::isfinite(Pb[(size_t)b * kMaxDim + a])) {
                free_plan(p);
                return LO_ERR_INVALID;
            }
            p->Pb[(size_t)b * kMaxDim + a] = Pb[(size_t)b * kMaxDim + a];
        }
    if (p->npts >= (1ll << 31)) {   // kernels address a line with 32-bit offsets
        free_plan(p);
        return LO_ERR_UNSUPPORTED;
    }
    lo_status st = build_tables(p);
    if (!st) {
        for (int a = 0; a < p->ndim; a++)
            if (desc->window[a] > 0 && desc->window[a] > p->kcap[a]) st = LO_ERR_INVALID;
    }
    if (!st) st = alloc((void**)&p->scratch, sizeof(double) * (size_t)p->npts * nb);
    if (!st) st = alloc((void**)&p->stats, sizeof(uint64_t) * kSlots * kSlotStride * nb);
    if (!st) st = alloc((void**)&p->flags, sizeof(uint32_t) * kFlagWords);
    if (!st) st = alloc((void**)&p->win, sizeof(int) * 4 * kMaxDim * nb);
    if (!st && hipMemset(p->win, 0, sizeof(int) * 4 * kMaxDim * nb) != hipSuccess) st = LO_ERR_HIP;
    if (!st && nb > 1) {
        std::vector<double> po((size_t)nb * kMaxDim, 0.0);
        for (int b = 0; b < nb; b++)
            for (int a = 0; a < p->ndim; a++)
                po[(size_t)b * kMaxDim + a] = p->Pb[(size_t)b * kMaxDim + a] * p->d.tau / p->dx[a];
        st = alloc((void**)&p->dpofs, sizeof(double) * po.size());
        if (!st && hipMemcpy(p->dpofs, po.data(), sizeof(double) * po.size(), hipMemcpyHostToDevice) != hipSuccess)
            st = LO_ERR_HIP;
        if (!st) st = alloc((void**)&p->dPb, sizeof(double) * p->Pb.size());
        if (!st && hipMemcpy(p->dPb, p->Pb.data(), sizeof(double) * p->Pb.size(), hipMemcpyHostToDevice) != hipSuccess)
            st = LO_ERR_HIP;
    }
    if (!st) st = setup_potential(p, V);
    if (st) {
        free_plan(p);
        return st;
    }
    choose_kernels(p);
    fill_winparams(p);
    st = upload_winparams(p);
    if (st) {
        free_plan(p);
        return st;
    }
    *out = p;
    return LO_OK;
}


}  // namespace

extern "C" {

const char* lo_status_string(lo_status s)
{
    switch (s) {
    case LO_OK: return "ok";
    case LO_ERR_INVALID: return "invalid argument";
    case LO_ERR_UNSUPPORTED: return "unsupported";
    case LO_ERR_OOM: return "out of device memory";
    case LO_ERR_HIP: return "HIP runtime error";
    case LO_ERR_WINDOW: return "window saturated or beyond capacity";
    }
    return "unknown status";
}

lo_status lo_plan(const lo_desc* desc, const lo_potential* V, lo_plan_t* out)
{
    if (!desc) return LO_ERR_INVALID;
    return plan_create(desc, V, 1, desc->P, out);
}

lo_status lo_plan_destroy(lo_plan_t p)
{
    if (!p) return LO_ERR_INVALID;
    free_plan(p);
    return LO_OK;
}

lo_status lo_set_coef(lo_plan_t p, const double* coef)
{
    if (!p || !coef || p->nmodes <= 0 || p->time_dep || !p->dcoef) return LO_ERR_INVALID;
    p->coef.assign(coef, coef + p->nmodes);
    HIPCHK(hipMemcpy(p->dcoef, coef, sizeof(double) * p->nmodes, hipMemcpyHostToDevice));
    HIPCHK(launch_synth_hv(p->basis, p->dcoef, p->nmodes, p->npts, p->d.tau, p->dhv, nullptr));
    lo_status st = add_potential_margins(p, p->dhv, true);
    if (st) return st;
    HIPCHK(hipDeviceSynchronize());
    fill_winparams(p);
    st = upload_winparams(p);
    if (st) return st;
    // captured steps hold the old margins by value
    for (auto& g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = lo_plan_s::GraphEntry();
    }
    return LO_OK;
}

lo_status lo_step(lo_plan_t p, double* u, int64_t n, int16_t* argmin, void* stream)
{
    if (!p || !u) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    lo_status st = prologue(p, u, n, s);
    if (st) return st;
    st = enqueue_step(p, u, n, argmin, s);
    if (st) return st;
    return finish(p, s, argmin != nullptr);
}

}  // extern "C"

namespace {

// An executable graph of kGraphSteps steps from phase n0 % 3 at the current halos.
lo_status get_graph(lo_plan_t p, double* u, int64_t n0, hipGraphExec_t* out)
{
    const int64_t phase = ((n0 % kSlots) + kSlots) % kSlots;
    lo_plan_s::GraphEntry* hit = nullptr;
    lo_plan_s::GraphEntry* victim = &p->graphs[0];
    for (auto& g : p->graphs) {
        if (g.exec && g.u == u && g.phase == phase && !memcmp(g.halo, p->halo, sizeof(g.halo))) hit = &g;
        if (!g.exec || g.stamp < victim->stamp) victim = &g;
    }
    if (!hit) {
        if (victim->exec) (void)hipGraphExecDestroy(victim->exec);
        victim->exec = nullptr;
        if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        lo_status cst = LO_OK;
        for (int k = 0; k < kGraphSteps && !cst; k++) cst = enqueue_step(p, u, n0 + k, nullptr, p->cap_stream);
        hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
        if (cst) {
            if (g) (void)hipGraphDestroy(g);
            return cst;
        }
        HIPCHK(ce);
        hipError_t ie = hipGraphInstantiate(&victim->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(ie);
        victim->u = u;
        victim->phase = phase;
        memcpy(victim->halo, p->halo, sizeof(victim->halo));
        hit = victim;
    }
    hit->stamp = ++p->graph_clock;
    *out = hit->exec;
    return LO_OK;
}

// The step loop of lo_run after its prologue.  It may return with segments
// still running on s (the caller drains the stream on error).
// The halo update of a step loop without a host wait: behind each segment
// its window maxima are copied into pinned memory (an event marks the copy)
// and the window words cleared; the copy of the segment before is folded in
// meanwhile, so a segment's halos come from the windows two segments back
// (halos choose kernel paths, never values).
struct LaggedAdapt {
    lo_plan_t p;
    hipStream_t s;
    int pend = -1;   // read-back buffer not yet folded
    static constexpr size_t kWords = (size_t)kMaxDim * kSpread;

    void fold(int b, bool halos)
    {
        const uint32_t* w = p->seg_pin + (size_t)b * kWords;
        for (int a = 0; a < p->ndim; a++) {
            const uint32_t wu = fold_spread(w + (size_t)a * kSpread);
            p->hflags[1 + a] = std::max(p->hflags[1 + a], wu);
            if (halos) {
                p->halo[a] = choose_halo(p, a, (int)wu);
                p->wseg[a] = (int)wu;
            }
        }
    }
    // after a segment that another one follows
    lo_status segment_done()
    {
        if (!p->seg_pin &&
            hipHostMalloc((void**)&p->seg_pin, sizeof(uint32_t) * 2 * kWords, hipHostMallocDefault) != hipSuccess) {
            p->seg_pin = nullptr;
            return LO_ERR_HIP;
        }
        for (auto& e : p->seg_ev)
            if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        const int b = pend == 0 ? 1 : 0;
        HIPCHK(hipMemcpyAsync(p->seg_pin + (size_t)b * kWords, p->flags + kFlagWin, sizeof(uint32_t) * kWords,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(p->seg_ev[b], s));
        HIPCHK(launch_fill_u32(p->flags + kFlagWin, (int64_t)kWords, 0u, s));
        if (pend >= 0) {
            HIPCHK(hipEventSynchronize(p->seg_ev[pend]));
            fold(pend, true);
        }
        pend = b;
        return LO_OK;
    }
    // at the loop's end: the last segment's maxima stay in the flags (finish
    // reads them); a copy still pending joins the run's maxima
    lo_status end()
    {
        if (pend >= 0) {
            HIPCHK(hipEventSynchronize(p->seg_ev[pend]));
            fold(pend, false);
            pend = -1;
        }
        return LO_OK;
    }
};

lo_status run_steps(lo_plan_t p, double* u, int64_t n0, int64_t nsteps, int64_t ckpt_every, double* ckpt,
                    hipStream_t s)
{
    lo_status st = LO_OK;
    const bool use_graph = graphable(p) && !ckpt;
    // From smooth data (u0 = 0, say) the windows first widen by several points
    // a step, more than the halos' slack covers over a whole segment.  While
    // they grow, segments stay short (2, 4, 8, 16 steps), and the halos are
    // sized for the growth the last segment predicts for the next.
    int64_t warm = 2;
    int wl[kMaxDim];
    for (int a = 0; a < kMaxDim; a++) wl[a] = p->wseg[a];
    // past the warm-up the halo update does not wait for the stream
    LaggedAdapt lag{p, s};
    int64_t done = 0;
    while (done < nsteps) {
        const int64_t seg = std::min<int64_t>(warm > 0 ? warm : kGraphSteps, nsteps - done);
        if (use_graph && seg == kGraphSteps) {
            hipGraphExec_t ge = nullptr;
            st = get_graph(p, u, n0 + done, &ge);
            if (st) return st;
            HIPCHK(hipGraphLaunch(ge, s));
        } else {
            for (int64_t k = 0; k < seg; k++) {
                const int64_t i = done + k;
                if (ckpt && i % ckpt_every == 0)
                    HIPCHK(hipMemcpyAsync(ckpt + (size_t)(i / ckpt_every) * p->npts, u, sizeof(double) * p->npts,
                                          hipMemcpyDeviceToDevice, s));
                st = enqueue_step(p, u, n0 + i, nullptr, s);
                if (st) return st;
            }
        }
        done += seg;
        if (done < nsteps && warm == 0) {
            st = lag.segment_done();
            if (st) return st;
        } else if (done < nsteps) {
            st = adapt_from_flags(p, s);
            if (st) return st;
            const int64_t next = std::min<int64_t>(2 * warm, 16);
            bool grows = false;
            for (int a = 0; a < p->ndim; a++) {
                const int64_t d = (int64_t)p->wseg[a] - wl[a];
                if (d * kGraphSteps > 8 * seg) grows = true;   // would outgrow half the slack in a segment
                if (d > 0) p->halo[a] = choose_halo(p, a, (int)std::min<int64_t>(p->wseg[a] + d * next / seg, 1 << 30));
                wl[a] = p->wseg[a];
            }
            warm = grows ? next : 0;
        }
    }
    return lag.end();
}

}  // namespace

extern "C" {

lo_status lo_run(lo_plan_t p, double* u, int64_t n0, int64_t nsteps, int64_t ckpt_every, double* ckpt,
                 void* stream)
{
    if (!p || !u || nsteps < 0) return LO_ERR_INVALID;
    if (ckpt && ckpt_every <= 0) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    lo_status st = LO_OK;
    if ((p->d.flags & LO_FLAG_AUTOTUNE) && !p->tuned) {
        st = autotune(p, u, n0, s);
        if (st) return st;
    }
    st = prologue(p, u, n0, s);
    if (!st) st = run_steps(p, u, n0, nsteps, ckpt_every, ckpt, s);
    if (st) {
        (void)hipStreamSynchronize(s);   // nothing of this call stays in flight
        return st;
    }
    return finish(p, s, false);
}

lo_status lo_run_decomp(lo_plan_t p, double* u, int64_t n0, int64_t nsteps, double eta, int32_t window,
                        int64_t* pieces, int64_t* breaks, void* stream)
{
    if (!p || !u || nsteps < 0 || !(eta >= 0.0) || window < 0) return LO_ERR_INVALID;
    if (p->ndim != 1 || p->nb != 1) return LO_ERR_UNSUPPORTED;
    const int64_t N = p->n[0];
    const int64_t W = window > 0 ? window : p->kcap[0];
    if (W > p->kcap[0] || N + 2 * W > (int64_t)1 << 30) return LO_ERR_INVALID;
    if (p->time_dep && n0 + nsteps > p->ntcoef) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    if (!p->dc_w) {
        lo_status st = alloc((void**)&p->dc_w, sizeof(double) * (size_t)N);
        if (!st) st = alloc((void**)&p->dc_cnt, sizeof(unsigned long long) * 2);
        if (st) return st;
    }
    HIPCHK(hipMemsetAsync(p->dc_cnt, 0, sizeof(unsigned long long) * 2, s));
    for (int64_t k = 0; k < nsteps; k++) {
        const int64_t n = n0 + k;
        if (p->time_dep)
            HIPCHK(launch_synth_hv(p->basis, p->dtcoef + n * p->nmodes, p->nmodes, p->npts, p->d.tau, p->dhv, s));
        HIPCHK(launch_decomp_step(u, p->dc_w, u, (int)N, (int)W, p->dkt[0] + p->kcap[0], eta * p->dx[0],
                                  p->kmaxabs[0], p->has_v ? p->dhv : nullptr, p->dc_cnt, s));
    }
    unsigned long long c[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(c, p->dc_cnt, sizeof(c), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (pieces) *pieces = (int64_t)c[0];
    if (breaks) *breaks = (int64_t)c[1];
    return LO_OK;
}

lo_status lo_run_semigroup1(lo_plan_t p, double* u, int64_t nsteps, int32_t window, void* stream)
{
    if (!p || !u || nsteps < 0 || window < 0) return LO_ERR_INVALID;
    if (p->ndim != 1 || p->nb != 1 || p->time_dep) return LO_ERR_UNSUPPORTED;
    const int64_t N = p->n[0];
    const int64_t W = window > 0 ? window : p->kcap[0];
    if (W > p->kcap[0]) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    if (!p->dc_w) {
        lo_status st = alloc((void**)&p->dc_w, sizeof(double) * (size_t)N);
        if (!st) st = alloc((void**)&p->dc_cnt, sizeof(unsigned long long) * 2);
        if (st) return st;
    }
    if (!p->sg_q) {
        lo_status st = alloc((void**)&p->sg_q, sizeof(double) * (size_t)(N + 1));
        if (!st) st = alloc((void**)&p->sg_sat, sizeof(unsigned));
        if (st) return st;
    }
    const double* hv = p->has_v ? p->dhv : nullptr;
    if (hv) HIPCHK(launch_prefix(hv, N, p->sg_q, s));   // prefix sums of the static tau V table
    HIPCHK(hipMemsetAsync(p->sg_sat, 0, sizeof(unsigned), s));
    for (int64_t k = 0; k < nsteps; k++) {
        HIPCHK(launch_semigroup1(u, p->dc_w, N, (int)W, p->dkt[0] + p->kcap[0], hv, p->sg_q, p->sg_sat, s));
        HIPCHK(hipMemcpyAsync(u, p->dc_w, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, s));
    }
    unsigned sat = 0;
    HIPCHK(hipMemcpyAsync(&sat, p->sg_sat, sizeof(sat), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return sat ? LO_ERR_WINDOW : LO_OK;
}

lo_status lo_last_diag(lo_plan_t p, int32_t* max_abs_offset, int32_t* window_used)
{
    if (!p || !p->have_diag) return LO_ERR_INVALID;
    for (int a = 0; a < p->ndim; a++) {
        if (window_used) window_used[a] = (int32_t)p->hflags[1 + a];
        if (max_abs_offset) max_abs_offset[a] = p->had_argmin ? (int32_t)p->hflags[4 + a] : -1;
    }
    if (p->hflags[0] & (kErrWindowCap | kErrWindowEdge)) return LO_ERR_WINDOW;
    return LO_OK;
}

lo_status lo_kinetic_table(lo_plan_t p, int32_t axis, int64_t s0, int64_t count, double* out)
{
    if (!p || !out || axis < 0 || axis >= p->ndim || count < 0) return LO_ERR_INVALID;
    for (int64_t i = 0; i < count; i++) {
        const int64_t s = s0 + i;
        out[i] = (s < -p->kcap[axis] || s > p->kcap[axis]) ? INFINITY : p->hkt[axis][s + p->kcap[axis]];
    }
    return LO_OK;
}

lo_status lo_time_kernels(lo_plan_t p, double* u, int64_t n0, int64_t nsteps, double* ms, void* stream)
{
    if (!p || !u || !ms || nsteps <= 0) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    lo_status st = prologue(p, u, n0, s);
    if (st) return st;
    // a pair of events around every sweep of a segment of steps; the stream
    // runs the segment's steps back to back and the host reads the intervals
    // at the segment's end (where lo_run adapts its halos too)
    constexpr int kSeg = kGraphSteps;
    const int per = 2 * p->ndim;
    std::vector<hipEvent_t> ev((size_t)kSeg * per, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) st = LO_ERR_HIP;
    double acc[kMaxDim] = {0, 0, 0};
    for (int64_t k0 = 0; k0 < nsteps && !st; k0 += kSeg) {
        if (k0 > 0) st = adapt_from_flags(p, s);
        const int64_t seg = std::min<int64_t>(kSeg, nsteps - k0);
        for (int64_t k = 0; k < seg && !st; k++) st = enqueue_step(p, u, n0 + k0 + k, nullptr, s, &ev[k * per]);
        if (!st && hipStreamSynchronize(s) != hipSuccess) st = LO_ERR_HIP;
        for (int64_t k = 0; k < seg && !st; k++)
            for (int a = 0; a < p->ndim; a++) {
                float t = 0.f;
                if (hipEventElapsedTime(&t, ev[k * per + 2 * a], ev[k * per + 2 * a + 1]) != hipSuccess)
                    st = LO_ERR_HIP;
                acc[a] += t;
            }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st) return st;
    for (int a = 0; a < p->ndim; a++) ms[a] = acc[a] / (double)nsteps;
    return finish(p, s, false);
}

lo_status lo_effective_H(int32_t ninst, const lo_desc* descs, const lo_potential* V, double T, double* hbar_out,
                         void* stream)
{
    if (ninst < 0 || (ninst > 0 && (!descs || !V || !hbar_out))) return LO_ERR_INVALID;
    if (!(T > 0) || !std::isfinite(T)) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    // instances sharing everything but P run as one batch: the same grid, time
    // step, method, windows and potential table
    struct Group {
        std::vector<int> idx;
        int64_t steps = 0, per_unit = 0;
    };
    std::vector<std::pair<std::vector<uint8_t>, Group>> groups;
    for (int i = 0; i < ninst; i++) {
        const lo_desc& d = descs[i];
        if (d.ndim < 1 || d.ndim > kMaxDim || !(d.tau > 0) || !std::isfinite(d.tau)) return LO_ERR_INVALID;
        for (int a = 0; a < d.ndim; a++)
            if (d.kstar_tab[a]) return LO_ERR_UNSUPPORTED;
        if (V[i].nmodes != 0 || V[i].tcoef) return LO_ERR_UNSUPPORTED;
        // (dx, tau) rational with 1/tau an integer: whole time units are whole step counts
        const double inv = 1.0 / d.tau;
        const int64_t m = llround(inv);
        if (m < 1 || fabs((double)m - inv) > 1e-9 * inv) return LO_ERR_INVALID;
        const int64_t K = llround(T * (double)m);
        if (K < m || fabs((double)K - T * (double)m) > 1e-9 * T * (double)m) return LO_ERR_INVALID;
        std::vector<uint8_t> key;
        auto put = [&](const void* v, size_t nbytes) {
            const uint8_t* c = (const uint8_t*)v;
            key.insert(key.end(), c, c + nbytes);
        };
        put(&d.ndim, sizeof(d.ndim));
        put(d.n, sizeof(int64_t) * d.ndim);
        put(d.period, sizeof(double) * d.ndim);
        put(&d.tau, sizeof(d.tau));
        put(d.window, sizeof(int32_t) * d.ndim);
        put(&d.method, sizeof(d.method));
        put(&d.flags, sizeof(d.flags));
        put(&V[i].table, sizeof(V[i].table));
        put(&K, sizeof(K));
        Group* g = nullptr;
        for (auto& e : groups)
            if (e.first == key) g = &e.second;
        if (!g) {
            groups.emplace_back(key, Group());
            g = &groups.back().second;
            g->steps = K;
            g->per_unit = m;
        }
        g->idx.push_back(i);
    }
    for (auto& e : groups) {
        Group& g = e.second;
        const lo_desc& d0 = descs[g.idx[0]];
        int64_t npts = 1;
        for (int a = 0; a < d0.ndim; a++) npts *= d0.n[a];
        // batches of at most ~12 GiB of state (u, the step's scratch, the snapshot)
        const int64_t cap = std::max<int64_t>(1, ((int64_t)12 << 30) / (24 * std::max<int64_t>(npts, 1)));
        for (size_t c0 = 0; c0 < g.idx.size(); c0 += (size_t)cap) {
            const int nb = (int)std::min<size_t>((size_t)cap, g.idx.size() - c0);
            std::vector<double> Pb((size_t)nb * kMaxDim, 0.0);
            for (int b = 0; b < nb; b++)
                for (int a = 0; a < d0.ndim; a++) Pb[(size_t)b * kMaxDim + a] = descs[g.idx[c0 + b]].P[a];
            lo_plan_t p = nullptr;
            lo_status st = plan_create(&d0, &V[g.idx[c0]], nb, Pb.data(), &p);
            if (st) return st;
            double* u = nullptr;
            double* snap = nullptr;
            uint64_t* rng = nullptr;
            st = alloc((void**)&u, sizeof(double) * (size_t)npts * nb);
            if (!st) st = alloc((void**)&snap, sizeof(double) * (size_t)npts * nb);
            if (!st) st = alloc((void**)&rng, sizeof(uint64_t) * 2 * nb);
            std::vector<uint64_t> h(2 * (size_t)nb, host_enc_neg_inf());
            if (!st && (hipMemsetAsync(u, 0, sizeof(double) * (size_t)npts * nb, s) != hipSuccess ||
                        hipMemcpyAsync(rng, h.data(), sizeof(uint64_t) * h.size(), hipMemcpyHostToDevice, s) !=
                            hipSuccess))
                st = LO_ERR_HIP;
            // u0 = 0; u(T - 1) kept, then one more time unit to u(T)
            if (!st) st = lo_run(p, u, 0, g.steps - g.per_unit, 0, nullptr, s);
            if (!st && hipMemcpyAsync(snap, u, sizeof(double) * (size_t)npts * nb, hipMemcpyDeviceToDevice, s) !=
                           hipSuccess)
                st = LO_ERR_HIP;
            if (!st) st = lo_run(p, u, g.steps - g.per_unit, g.per_unit, 0, nullptr, s);
            if (!st && launch_diff_range(u, snap, npts, nb, rng, s) != hipSuccess) st = LO_ERR_HIP;
            if (!st && (hipMemcpyAsync(h.data(), rng, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost, s) !=
                            hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
                st = LO_ERR_HIP;
            if (!st) {
                for (int b = 0; b < nb; b++) {
                    const double dmax = host_dec(h[2 * b]), dmin = -host_dec(h[2 * b + 1]);
                    double* o = hbar_out + (size_t)g.idx[c0 + b] * 3;
                    o[0] = -dmax;
                    o[1] = -(dmax + dmin) * 0.5;
                    o[2] = -dmin;
                }
            }
            if (u) (void)hipFree(u);
            if (snap) (void)hipFree(snap);
            if (rng) (void)hipFree(rng);
            free_plan(p);
            if (st) return st;
        }
    }
    return LO_OK;
}

}  // extern "C"

namespace {

// Scatter layouts of `steps` steps, every axis of step k for offsets up to
// amax[k * ndim + a] (each step's own largest offsets: the first steps of a
// run from smooth data reach several times further than the later ones).
lo_status scatter_layouts(lo_plan_t p, const uint32_t* amax, int64_t steps, ScatterArgs* sa)
{
    int dev = 0, lds_max = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return LO_ERR_HIP;
    for (int64_t i = 0; i < steps * p->ndim; i++) {
        const int a = (int)(i % p->ndim);
        AxisGeom g;
        g.n = p->n[a];
        g.stride = 1;
        for (int b = 0; b < a; b++) g.stride *= p->n[b];
        g.nlines = p->npts / p->n[a];
        if (!scatter_layout(g, (int)amax[i], (size_t)lds_max, &sa[i])) return LO_ERR_UNSUPPORTED;
    }
    return LO_OK;
}

// Reverse of steps n1-1 .. n0 whose argmins are E[(n - n0)][a][npts] and
// scatter layouts sa[(n - n0) * ndim + a]: axes d-1 .. 0, the adjoint of
// u^{n+1} entering the potential's gradient before the sweeps are undone.
// lam ping-pongs between the plan's two buffers.
lo_status reverse_steps(lo_plan_t p, const int16_t* E, int64_t n0, int64_t n1, const ScatterArgs* sa, int* cur,
                        bool coef, hipStream_t s)
{
    for (int64_t n = n1 - 1; n >= n0; n--) {
        for (int a = p->ndim - 1; a >= 0; a--) {
            const int16_t* Ea = E + ((size_t)(n - n0) * p->ndim + a) * p->npts;
            double* Lam = (coef && a == p->ndim - 1) ? p->bw_Lam : nullptr;
            HIPCHK(launch_scatter(Ea, p->bw_lam[*cur], p->bw_lam[*cur ^ 1], Lam, sa[(n - n0) * p->ndim + a],
                                  p->bw_err, s));
            *cur ^= 1;
        }
    }
    return LO_OK;
}

// Gradient outputs and the error report of a reverse pass.
lo_status finish_backward(lo_plan_t p, int cur, double* grad_u0, double* grad_coef, uint32_t errs, uint32_t* hf,
                          lo_status st, hipStream_t s)
{
    const size_t bytes = sizeof(double) * (size_t)p->npts;
    if (!st && grad_u0) HIPCHK(hipMemcpyAsync(grad_u0, p->bw_lam[cur], bytes, hipMemcpyDeviceToDevice, s));
    if (!st && grad_coef) {
        const int G = project_blocks(p->npts);
        double* out = p->bw_part + (size_t)p->nmodes * G;
        HIPCHK(launch_project(p->bw_Lam, p->basis, p->nmodes, p->npts, p->bw_part, out, s));
        std::vector<double> acc(p->nmodes);
        HIPCHK(hipMemcpyAsync(acc.data(), out, sizeof(double) * p->nmodes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int m = 0; m < p->nmodes; m++) grad_coef[m] = -p->d.tau * acc[m];
    }
    HIPCHK(hipStreamSynchronize(s));
    uint32_t f0 = 0, e0 = 0;
    HIPCHK(hipMemcpy(&f0, p->flags, sizeof(f0), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&e0, p->bw_err, sizeof(e0), hipMemcpyDeviceToHost));
    errs |= f0 | e0;
    hf[0] = errs;
    for (int i = 0; i < 8; i++) p->hflags[i] = hf[i];
    p->have_diag = true;
    p->had_argmin = true;
    if (st) return st;
    if (errs & (kErrWindowCap | kErrWindowEdge | kErrFastPath | kErrAdjointHalo)) return LO_ERR_WINDOW;
    if (errs & kErrArgRange) return LO_ERR_UNSUPPORTED;
    return LO_OK;
}

lo_status check_backward_args(lo_plan_t p, int64_t nsteps, const double* grad_uT, const double* grad_coef)
{
    if (!p || !grad_uT || nsteps < 0) return LO_ERR_INVALID;
    if (grad_coef && (p->nmodes <= 0 || !p->basis)) return LO_ERR_INVALID;
    if (grad_coef && p->time_dep) return LO_ERR_UNSUPPORTED;
    return LO_OK;
}

}  // namespace

extern "C" {

lo_status lo_backward(lo_plan_t p, const double* ckpt, int64_t nsteps, int64_t ckpt_every,
                      const double* grad_uT, double* grad_u0, double* grad_coef, void* stream)
{
    lo_status st = check_backward_args(p, nsteps, grad_uT, grad_coef);
    if (st) return st;
    if ((!ckpt && nsteps > 0) || ckpt_every <= 0) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    const int64_t seg = std::min<int64_t>(ckpt_every, std::max<int64_t>(nsteps, 1));
    st = backward_buffers(p, seg, grad_coef != nullptr);
    if (!st) st = amax_buffer(p, 2 * seg * p->ndim * kSpread);
    if (st) return st;
    if (!p->bw_stream) HIPCHK(hipStreamCreateWithFlags(&p->bw_stream, hipStreamNonBlocking));
    for (auto& e : p->bw_ev)
        if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipStream_t s2 = p->bw_stream;
    StreamDrain drain2{s2};
    const size_t bytes = sizeof(double) * (size_t)p->npts;
    const size_t seg_arg = (size_t)seg * p->ndim * p->npts;
    int cur = 0;
    HIPCHK(hipMemcpyAsync(p->bw_lam[cur], grad_uT, bytes, hipMemcpyDeviceToDevice, s));
    if (grad_coef) HIPCHK(hipMemsetAsync(p->bw_Lam, 0, bytes, s));
    HIPCHK(hipMemsetAsync(p->bw_err, 0, sizeof(uint32_t), s));
    // the recomputes run on s2, after everything the caller queued on s (the checkpoints)
    HIPCHK(hipEventRecord(p->bw_ev[0], s));
    HIPCHK(hipStreamWaitEvent(s2, p->bw_ev[0], 0));
    uint32_t hf[8] = {0};
    uint32_t errs = 0;
    std::vector<ScatterArgs> sa[2];
    std::vector<uint32_t> am((size_t)seg * p->ndim);
    // Segment k recomputed from its checkpoint (on s2) with every sweep's
    // argmins in buffer k % 2; each step's largest offsets size its scatter
    // tiles.  Enqueued in two parts: the checkpoint, the prologue and the
    // first kGraphSteps steps go ahead of the reverse sweeps of the segment
    // after it (so that s2, the longer chain, starts at once), the rest behind
    // them; no part waits on the host before the read-back at its end (the
    // halos carry over from the segment before, sized by its windows).
    auto seg_of = [&](int64_t k, int64_t* n0, int64_t* n1) {
        *n0 = k * ckpt_every;
        *n1 = std::min(nsteps, *n0 + ckpt_every);
    };
    auto seg_steps = [&](int64_t k, int64_t from, int64_t to) -> lo_status {
        int64_t n0, n1;
        seg_of(k, &n0, &n1);
        int16_t* E = p->bw_arg + (size_t)(k % 2) * seg_arg;
        uint32_t* AM = p->bw_amax + (size_t)(k % 2) * seg * p->ndim * kSpread;
        // every recompute but the first runs beside the scatters of the segment
        // after it: its sweeps leave room for them on every CU
        p->narrow = n1 < nsteps;
        lo_status r = LO_OK;
        for (int64_t n = from; n < to && !r; n++)
            r = enqueue_step(p, p->bw_u, n, E + (size_t)(n - n0) * p->ndim * p->npts, s2, nullptr,
                             AM + (n - n0) * p->ndim * kSpread);
        p->narrow = false;
        return r;
    };
    auto recompute_start = [&](int64_t k) -> lo_status {
        int64_t n0, n1;
        seg_of(k, &n0, &n1);
        uint32_t* AM = p->bw_amax + (size_t)(k % 2) * seg * p->ndim * kSpread;
        HIPCHK(hipMemcpyAsync(p->bw_u, ckpt + (size_t)k * p->npts, bytes, hipMemcpyDeviceToDevice, s2));
        HIPCHK(launch_fill_u32(AM, (int64_t)((n1 - n0) * p->ndim * kSpread), 0u, s2));
        lo_status r = prologue(p, p->bw_u, n0, s2, false);
        return r ? r : seg_steps(k, n0, std::min(n1, n0 + kGraphSteps));
    };
    // The rest of segment k and its read-back (flags and offset maxima into
    // the pinned slot k % 2), then the event that marks it recomputed.
    const size_t rb_words = kFlagWords + (size_t)seg * p->ndim * kSpread;
    uint32_t* rb = host_words(p, 2 * rb_words);
    if (!rb) return LO_ERR_HIP;
    auto recompute_rest = [&](int64_t k) -> lo_status {
        int64_t n0, n1;
        seg_of(k, &n0, &n1);
        uint32_t* AM = p->bw_amax + (size_t)(k % 2) * seg * p->ndim * kSpread;
        const size_t am_words = (size_t)(n1 - n0) * p->ndim;
        lo_status r = seg_steps(k, std::min(n1, n0 + kGraphSteps), n1);
        if (r) return r;
        uint32_t* f = rb + (size_t)(k % 2) * rb_words;
        HIPCHK(hipMemcpyAsync(f, p->flags, sizeof(uint32_t) * kFlagWords, hipMemcpyDeviceToHost, s2));
        HIPCHK(hipMemcpyAsync(f + kFlagWords, AM, sizeof(uint32_t) * am_words * kSpread, hipMemcpyDeviceToHost,
                              s2));
        HIPCHK(hipEventRecord(p->bw_ev[1 + k % 2], s2));
        return LO_OK;
    };
    // The host's part of segment k once its read-back has landed: errors,
    // window and offset maxima, halos for the segments recomputed later, and
    // the scatter layouts.
    auto recompute_wait = [&](int64_t k) -> lo_status {
        int64_t n0, n1;
        seg_of(k, &n0, &n1);
        const size_t am_words = (size_t)(n1 - n0) * p->ndim;
        HIPCHK(hipEventSynchronize(p->bw_ev[1 + k % 2]));
        const uint32_t* f = rb + (size_t)(k % 2) * rb_words;
        for (size_t i = 0; i < am_words; i++) am[i] = fold_spread(f + kFlagWords + i * kSpread);
        errs |= f[0];
        if (f[0] & (kErrWindowCap | kErrWindowEdge | kErrFastPath | kErrArgRange)) return LO_ERR_WINDOW;
        for (int a = 0; a < p->ndim; a++) {
            const uint32_t wu = fold_window(f, a);
            hf[1 + a] = std::max(hf[1 + a], std::max(p->hflags[1 + a], wu));
            p->halo[a] = choose_halo(p, a, (int)wu);
            p->wseg[a] = (int)wu;
        }
        for (size_t i = 0; i < am_words; i++) hf[4 + i % p->ndim] = std::max(hf[4 + i % p->ndim], am[i]);
        sa[k % 2].resize(am_words);
        return scatter_layouts(p, am.data(), n1 - n0, sa[k % 2].data());
    };
    // Segments are undone from the last.  The reverse sweeps of segment k (on
    // s) run while segment k - 1 is recomputed (on s2) into the other buffer,
    // which the reverse sweeps of segment k + 1 have released.  Segment k - 2's
    // first part is enqueued behind segment k - 1's read-back, before the host
    // waits for it, so that s2 does not idle between segments.
    const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
    if (nseg > 0) st = recompute_start(nseg - 1);
    if (nseg > 0 && !st) st = recompute_rest(nseg - 1);
    if (nseg > 0 && !st) st = recompute_wait(nseg - 1);
    bool started = false;   // segment k - 1's first part already enqueued
    for (int64_t k = nseg - 1; k >= 0 && !st; k--) {
        const int64_t n0 = k * ckpt_every, n1 = std::min(nsteps, n0 + ckpt_every);
        if (k > 0 && !started) {
            if (k + 1 < nseg) HIPCHK(hipStreamWaitEvent(s2, p->bw_ev[3 + (k + 1) % 2], 0));
            st = recompute_start(k - 1);
            if (st) break;
        }
        started = false;
        HIPCHK(hipStreamWaitEvent(s, p->bw_ev[1 + k % 2], 0));
        st = reverse_steps(p, p->bw_arg + (size_t)(k % 2) * seg_arg, n0, n1, sa[k % 2].data(), &cur,
                           grad_coef != nullptr, s);
        if (st) break;
        HIPCHK(hipEventRecord(p->bw_ev[3 + k % 2], s));
        if (k > 0) {
            st = recompute_rest(k - 1);
            if (!st && k > 1) {
                // segment k - 2 overwrites buffer k % 2 once the reverse sweeps of k are done
                HIPCHK(hipStreamWaitEvent(s2, p->bw_ev[3 + k % 2], 0));
                st = recompute_start(k - 2);
                started = true;
            }
            if (!st) st = recompute_wait(k - 1);
        }
    }
    // a window or argmin error of a recompute is reported through errs
    if (st == LO_ERR_WINDOW && (errs & (kErrWindowCap | kErrWindowEdge | kErrFastPath | kErrArgRange))) st = LO_OK;
    return finish_backward(p, cur, grad_u0, grad_coef, errs, hf, st, s);
}

lo_status lo_run_record(lo_plan_t p, double* u, int64_t n0, int64_t nsteps, int16_t* argmins, void* stream)
{
    if (!p || !u || nsteps < 0 || (!argmins && nsteps > 0)) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    lo_status st = prologue(p, u, n0, s);
    LaggedAdapt lag{p, s};
    for (int64_t k = 0; k < nsteps && !st; k++) {
        if (k > 0 && k % kGraphSteps == 0) st = lag.segment_done();
        if (!st) st = enqueue_step(p, u, n0 + k, argmins + (size_t)k * p->ndim * p->npts, s);
    }
    if (!st) st = lag.end();
    if (st) return st;
    return finish(p, s, true);
}

lo_status lo_backward_recorded(lo_plan_t p, const int16_t* argmins, int64_t nsteps, const double* grad_uT,
                               double* grad_u0, double* grad_coef, void* stream)
{
    lo_status st = check_backward_args(p, nsteps, grad_uT, grad_coef);
    if (st) return st;
    if (!argmins && nsteps > 0) return LO_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    st = backward_buffers(p, 1, grad_coef != nullptr);
    if (!st) st = amax_buffer(p, nsteps * p->ndim);
    if (st) return st;
    const size_t bytes = sizeof(double) * (size_t)p->npts;
    int cur = 0;
    HIPCHK(hipMemcpyAsync(p->bw_lam[cur], grad_uT, bytes, hipMemcpyDeviceToDevice, s));
    if (grad_coef) HIPCHK(hipMemsetAsync(p->bw_Lam, 0, bytes, s));
    HIPCHK(hipMemsetAsync(p->flags, 0, sizeof(uint32_t) * kFlagWords, s));
    HIPCHK(hipMemsetAsync(p->bw_err, 0, sizeof(uint32_t), s));
    // each step's largest offsets size its scatter tiles' halos
    const size_t am_words = (size_t)nsteps * p->ndim;
    std::vector<uint32_t> am(am_words);
    if (nsteps > 0) {
        HIPCHK(launch_fill_u32(p->bw_amax, (int64_t)am_words, 0u, s));
        HIPCHK(launch_absmax16(argmins, nsteps, p->ndim, p->npts, p->bw_amax, s));
        HIPCHK(hipMemcpyAsync(am.data(), p->bw_amax, sizeof(uint32_t) * am_words, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    uint32_t hf[8] = {0};
    for (size_t i = 0; i < am_words; i++) hf[4 + i % p->ndim] = std::max(hf[4 + i % p->ndim], am[i]);
    std::vector<ScatterArgs> sa(am_words);
    st = scatter_layouts(p, am.data(), nsteps, sa.data());
    if (!st) st = reverse_steps(p, argmins, 0, nsteps, sa.data(), &cur, grad_coef != nullptr, s);
    return finish_backward(p, cur, grad_u0, grad_coef, 0, hf, st, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// lo_step_noalloc: one step for callers that cannot allocate device memory.
// Its work memory (kinetic tables, the second grid array the sweeps ping-pong
// with, statistics slots, flags, windows) is one static device array, which
// every GPU the library runs on holds until the process ends.  Host code never
// passes the array's name to a kernel or a copy: on each device the array's
// address comes from hipGetSymbolAddress, taken once with that device current.
namespace {

constexpr int64_t kNaTab = 65536 + 64;                 // doubles per axis table: 2 * 32767 + 1 costs
constexpr int64_t kNaTabPad = 32;                      // and 32 unused doubles on either side
constexpr int64_t kNaGrid = LO_NOALLOC_MAX_POINTS;     // the second grid array
constexpr int64_t kNaStats = (int64_t)kSlots * kSlotStride;   // 64-bit words
constexpr int64_t kNaFlags = 256;                      // doubles: 512 flag words >= kFlagWords
constexpr int64_t kNaWin = 32;                         // doubles: 64 window ints >= 4 kMaxDim
constexpr int64_t kNaOffGrid = kMaxDim * kNaTab;
constexpr int64_t kNaOffStats = kNaOffGrid + kNaGrid;
constexpr int64_t kNaOffFlags = kNaOffStats + kNaStats;
constexpr int64_t kNaOffWin = kNaOffFlags + kNaFlags;
constexpr int64_t kNaWords = kNaOffWin + kNaWin;
static_assert(kNaOffGrid % 32 == 0 && kNaOffStats % 32 == 0 && kNaOffFlags % 32 == 0 && kNaOffWin % 32 == 0,
              "every region starts on a 256-byte boundary");
static_assert(2 * kNaFlags >= kFlagWords && 2 * kNaWin >= 4 * kMaxDim, "flag and window regions fit");

static __device__ __align__(256) double scratch[kNaWords];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
double* g_na_base[kNaMaxDevices] = {};

// The address of the current device's copy of `scratch`.
lo_status noalloc_base(double** out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return LO_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_base[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return LO_ERR_HIP;
        }
        g_na_base[dev] = (double*)ptr;
    }
    *out = g_na_base[dev];
    return LO_OK;
}

// max |k| and k(0) - min k of the mechanical cost over [-cap, cap] without the
// table: k is a convex quadratic, so its extremes lie at the ends and next to
// the vertex P tau / dx.
void mech_extremes(int64_t cap, double dx, double tau, double P, double* maxabs, double* zero_drop)
{
    const double v = P * tau / dx;
    double kmin = INFINITY, mx = 0.0;
    auto visit = [&](int64_t s) {
        if (s < -cap || s > cap) return;
        const double k = mech_cost(s, dx, tau, P);
        kmin = std::min(kmin, k);
        mx = std::max(mx, fabs(k));
    };
    visit(-cap);
    visit(cap);
    if (std::isfinite(v) && fabs(v) < 4.0 * (double)cap) {
        const int64_t c = (int64_t)floor(v);
        for (int64_t s = c - 3; s <= c + 4; s++) visit(s);
    }
    if (kmin > mech_cost(0, dx, tau, P)) kmin = mech_cost(0, dx, tau, P);
    *maxabs = mx;
    *zero_drop = (mech_cost(0, dx, tau, P) - kmin) * (1.0 + 0x1p-40) + 0x1p-60;
}

}  // namespace

extern "C" lo_status lo_step_noalloc(const lo_desc* desc, const double* tau_v, double* u, int64_t n,
                                     int16_t* argmin, void* stream)
{
    // checks that need no device come first
    if (!desc || !u) return LO_ERR_INVALID;
    if (desc->ndim < 1 || desc->ndim > kMaxDim) return LO_ERR_INVALID;
    if (!(desc->tau > 0) || !std::isfinite(desc->tau)) return LO_ERR_INVALID;
    if (desc->method != LO_BRUTE && desc->method != LO_FAST) return LO_ERR_INVALID;
    int64_t npts = 1;
    for (int a = 0; a < desc->ndim; a++) {
        if (desc->n[a] < 3 || desc->n[a] > kNaGrid) return LO_ERR_INVALID;
        if (!(desc->period[a] > 0) || !std::isfinite(desc->period[a]) || !std::isfinite(desc->P[a]) ||
            desc->window[a] < 0)
            return LO_ERR_INVALID;
        if (desc->kstar_tab[a]) return LO_ERR_UNSUPPORTED;
        npts *= desc->n[a];
        if (npts > kNaGrid) return LO_ERR_UNSUPPORTED;
    }
    double* base = nullptr;
    lo_status st = noalloc_base(&base);
    if (st) return st;

    // a plan description on the host stack whose device pointers lie in the
    // static array (its vectors stay empty: nothing is allocated)
    lo_plan_s q;
    lo_plan_t p = &q;
    p->d = *desc;
    p->ndim = desc->ndim;
    p->npts = npts;
    for (int a = 0; a < p->ndim; a++) {
        p->n[a] = desc->n[a];
        p->dx[a] = desc->period[a] / (double)desc->n[a];
        p->kcap[a] = std::min<int64_t>(32767, std::max<int64_t>(64, 2 * p->n[a]));
        if (desc->window[a] > p->kcap[a]) return LO_ERR_INVALID;
        p->dkt[a] = base + a * kNaTab + kNaTabPad;
        mech_extremes(p->kcap[a], p->dx[a], desc->tau, desc->P[a], &p->kmaxabs[a], &p->kzero_drop[a]);
        const double v = fabs(desc->P[a] * desc->tau / p->dx[a]);
        p->vabs[a] = (int)std::min(v + 1.0, (double)p->kcap[a]);
    }
    p->scratch = base + kNaOffGrid;
    p->stats = (uint64_t*)(base + kNaOffStats);
    p->flags = (uint32_t*)(base + kNaOffFlags);
    p->win = (int*)(base + kNaOffWin);
    p->has_v = tau_v != nullptr;
    p->dhv = const_cast<double*>(tau_v);   // read only
    p->next_win = false;
    choose_kernels(p);
    fill_winparams(p);
    // windows from the statistics of this step's own input: no potential step
    // lies between them, so no potential margins
    p->winp.lag = 0;
    p->winp.hv_osc = 0.0;

    hipStream_t s = (hipStream_t)stream;
    StreamDrain drain{s};
    for (int a = 0; a < p->ndim; a++)
        HIPCHK(launch_mech_table(p->dkt[a], p->kcap[a], p->dx[a], desc->tau, desc->P[a], s));
    HIPCHK(launch_fill_u32(p->flags, kFlagWords, 0u, s));
    HIPCHK(launch_clear_slots(p->stats, 1, s));
    HIPCHK(launch_stats(u, p->ndim, p->n, slot(p, n), 1, p->npts, kNaStats, s));
    HIPCHK(launch_windows(p->winp, slot(p, n), p->win + (size_t)(((n % 2) + 2) % 2) * 2 * kMaxDim, p->flags, 1, s));
    uint32_t f[kFlagWords];
    HIPCHK(hipMemcpyAsync(f, p->flags, sizeof(f), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int a = 0; a < p->ndim; a++) p->halo[a] = choose_halo(p, a, (int)fold_window(f, a));
    st = enqueue_step(p, u, n, argmin, s);
    if (st) return st;
    return finish(p, s, argmin != nullptr);
}
