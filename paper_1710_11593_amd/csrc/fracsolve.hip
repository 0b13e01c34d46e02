// Host runtime of the fracsolve library: handle, planner, the recursive
// (divide-and-conquer in time) driver and the C ABI of include/fracsolve.h.
//
// The block lower-triangular Toeplitz system (time-major form of eq. e21)
//   (a_0 I + K) U^n + sum_{j<n} a_{n-j} U^j = R^n
// is solved by recursive halving of [0, Np), Np = 2^k >= N:
//   solve(lo, 2s): solve(lo, s); Y[lo+s, lo+2s) -= T_s X[lo, lo+s); solve(lo+s, s)
// with T_s[p][q] = a_{s+p-q}; leaves of L rows are solved by k_leaf.  Run in
// depth-first order, leaf k is followed by exactly one level product of
// half-size s = L * lowbit(k+1).  Rows at or beyond N are never touched
// (the system is causal, so padding N up to Np is exact).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fracsolve.h"
#include "common.hpp"
#include "plan.hpp"

using namespace fs;

namespace {

std::string g_create_error;

struct Inst {
    fracsolve_problem p;
    int regime = 0;  // 0 diffusion, 1 diffusion-wave
    double tau = 0, h = 0, e = 0, coef = 0, dcoef = 0, pexp = 0;
    int64_t M = 0, N = 0, Np = 0;
    LeafCfg lc{};
    bool scan = true;  // leaf solver: closed-form scan (true) or block Thomas + PCR
    int adv = 0;       // advection equations: 2 = Scheme 2 (gamma < 1), 3 = Scheme 3; 0 = diffusion
    bool cn = false;   // diffusion-wave with the spatial term averaged over t_n and t_{n-1}
    ColPerm perm{0, 0};  // internal column order of the solve's fields
    double *b = nullptr, *a = nullptr, *rho = nullptr, *psi = nullptr;
    double *da = nullptr, *drho = nullptr, *dpsi = nullptr;
    double *fac = nullptr;
    // spectra of a and of da for every FFT level, indexed by log2(s)
    std::vector<int64_t> spec_off;
    cplx<double> *spec64 = nullptr, *dspec64 = nullptr;
    cplx<float> *spec32 = nullptr;
    // workspaces (allocated on first use)
    double *R = nullptr;      // saved right-hand side (refinement)
    double *W = nullptr;      // residual / correction / reversed field
    double *V = nullptr;      // operator apply output
    float *hist32 = nullptr;  // float32 history accumulator
    float *x32 = nullptr;     // float32 shadow of solved rows
    double *kry = nullptr;    // GMRES: Krylov basis, kry_cap vectors of M N
    int kry_cap = 0;
};

double digamma_host(double x)
{
    // psi(x) for x > 0: recurrence psi(x) = psi(x+1) - 1/x up to x >= 12,
    // then the asymptotic expansion ln x - 1/(2x) - sum B_2k/(2k x^2k)
    // (Abramowitz & Stegun 6.3.5 and 6.3.18).
    double r = 0.0;
    while (x < 12.0) {
        r -= 1.0 / x;
        x += 1.0;
    }
    const double B[] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730, 7.0 / 6};
    double x2 = 1.0 / (x * x), pw = x2, s = 0.0;
    for (int k = 1; k <= 7; ++k) {
        s += B[k - 1] / (2.0 * k) * pw;
        pw *= x2;
    }
    return r + std::log(x) - 0.5 / x - s;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int64_t next_pow2(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}
int ilog2i(int64_t v)
{
    int r = 0;
    while ((1LL << r) < v) ++r;
    return r;
}

}  // namespace

struct fracsolve_ctx {
    std::vector<Inst> inst;
    fracsolve_options opts{};
    hipStream_t st = nullptr;
    int device = 0;
    int L = 8;
    int crossover = 64;
    int64_t nmax = 0;
    cplx<double> *tw64 = nullptr;
    cplx<float> *tw32 = nullptr;
    // descriptor staging: pinned host copy and device copy
    void *h_desc = nullptr, *d_desc = nullptr;
    size_t desc_cap = 0, desc_used = 0;
    hipEvent_t desc_ready = nullptr;
    // multi-pass FFT scratch
    void *zs = nullptr;
    size_t zs_bytes = 0;
    double *partial = nullptr;  // reduction partials
    std::string err;
    int timing = 0;
    int check = 0;  // scan outputs for non-finite values (fracsolve_set_check)
    fracsolve_stats stats{};
    std::vector<hipEvent_t> evpool;
    struct Rec {
        int kind, s, ntasks;
        double bytes;
        size_t ev;
    };
    std::vector<Rec> recs;
    std::vector<fracsolve_kernel_stat> kstats;
    // replay of recorded launch sequences (hipGraph) on an internal stream
    bool use_graph = false;
    bool capturing = false;  // a launch sequence is being recorded into a graph
    hipStream_t gst = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    struct GraphEntry {
        uint64_t key;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    int kernels = 0;
    std::vector<double *> allocs;
    // batches: every instance uses the leaf configuration of the widest one,
    // so that one launch per step covers all leaves (0: single instance)
    int64_t batch_M = 0;
    // leaves in pairs with the level product of half-size L inside the leaf
    // kernel (dense levels at s = L, scan or advection leaves, L <= 8)
    bool pair = false;
    // GMRES: zero history weights (block-diagonal solves through the leaf
    // kernels), multi-dot partials and results
    double *zeros = nullptr;
    double *gpart = nullptr, *gdots = nullptr;
    int gcap = 0;
    int plan_source = 0;  // where L and the crossover came from (FRACSOLVE_PLAN_*)
};

namespace {

int fail(fracsolve_ctx *h, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define HIPCHK(h, expr)                                                                           \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess)                                                                     \
            return fail((h), FRACSOLVE_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

template <typename T>
int dalloc(fracsolve_ctx *h, T **p, size_t count)
{
    void *q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 16;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        hipGetLastError();
        return fail(h, FRACSOLVE_E_NOMEM, "device allocation of %zu bytes failed", bytes);
    }
    h->allocs.push_back((double *)q);
    *p = (T *)q;
    return FRACSOLVE_OK;
}

// ---- descriptor staging: all task descriptors of one call go to the device
// in one copy; kernels receive pointers into the device copy.
struct DescBuilder {
    fracsolve_ctx *h;
    std::vector<char> host;
    size_t add(const void *p, size_t bytes)
    {
        size_t off = (host.size() + 15) & ~(size_t)15;
        host.resize(off + bytes);
        memcpy(host.data() + off, p, bytes);
        return off;
    }
};

int desc_upload(fracsolve_ctx *h, const DescBuilder &db)
{
    size_t need = db.host.size();
    if (need == 0) return FRACSOLVE_OK;
    if (h->desc_ready) HIPCHK(h, hipEventSynchronize(h->desc_ready));
    if (need > h->desc_cap) {
        HIPCHK(h, hipStreamSynchronize(h->st));
        if (h->gst) HIPCHK(h, hipStreamSynchronize(h->gst));
        for (auto &g : h->graphs) hipGraphExecDestroy(g.exec);
        h->graphs.clear();
        if (h->h_desc) hipHostFree(h->h_desc);
        if (h->d_desc) hipFree(h->d_desc);
        h->h_desc = h->d_desc = nullptr;
        size_t cap = std::max(need, (size_t)1 << 20);
        HIPCHK(h, hipHostMalloc(&h->h_desc, cap, hipHostMallocDefault));
        HIPCHK(h, hipMalloc(&h->d_desc, cap));
        h->desc_cap = cap;
    }
    memcpy(h->h_desc, db.host.data(), need);
    HIPCHK(h, hipMemcpyAsync(h->d_desc, h->h_desc, need, hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipEventRecord(h->desc_ready, h->st));
    return FRACSOLVE_OK;
}

template <typename T>
const T *dptr(fracsolve_ctx *h, size_t off)
{
    return (const T *)((const char *)h->d_desc + off);
}

// ---- one call = a list of launch records built on the host, then replayed.
enum OpKind { OP_LEAF, OP_LEAF_SCAN, OP_GEMM64, OP_GEMM32, OP_FFT64, OP_FFT32, OP_LEAF_ADV, OP_LAG1 };
struct Op {
    OpKind kind;
    size_t off;   // descriptor offset
    int ntasks;
    int s;        // level half-size (updates) or leaf config index
    int64_t maxM;
    LeafCfg lc;
    bool mixed;
    double bytes = 0.0;  // algorithmic HBM bytes of the launch
    bool even = false;   // FFT levels: every task has M even and aligned rows
    size_t goff = 0;     // single-pass FFT levels: descriptor offset of the group offsets
    int lead = 0;        // dense levels of a solve: rows the next leaf reads first
    bool wsum = false;   // advection leaves: Scheme 2 (X = B U, U to its own field)
    bool cn = false;     // scan leaves: the lag-1 spatial term of the averaged variant
    bool pair = false;   // scan leaves: two leaves and the level of half-size L between them
};

// Flat column-group offsets of the tasks of a single-pass FFT level (see
// launch_fft_update_ex), added to the descriptors; returns their offset.
template <typename T>
size_t add_group_offsets(DescBuilder &db, const std::vector<UpdTask<T>> &tv, int s)
{
    const int cc = fft_update_cc(2 * s, sizeof(T) == 4);
    std::vector<int64_t> gb(tv.size() + 1, 0);
    for (size_t k = 0; k < tv.size(); ++k) gb[k + 1] = gb[k] + ((tv[k].M + 1) / 2 + cc - 1) / cc;
    return db.add(gb.data(), gb.size() * sizeof(int64_t));
}

// Column pairs of every row are whole, aligned vector elements.
template <typename T>
bool pairs_aligned(const UpdTask<T> &t)
{
    const uintptr_t a = 2 * sizeof(T);
    return (t.M % 2) == 0 && ((uintptr_t)t.x % a) == 0 && ((uintptr_t)t.y % a) == 0;
}

// Single-task launches carry their descriptor inline, except while a graph is
// being recorded (a replay must read the descriptors uploaded for it).
template <typename TASK>
TaskRef<TASK> task_ref(fracsolve_ctx *h, const Op &op)
{
    TaskRef<TASK> r{dptr<TASK>(h, op.off), TASK{}, 0};
    if (op.ntasks == 1 && !h->capturing) {
        memcpy(&r.one, (const char *)h->h_desc + op.off, sizeof(TASK));
        r.one_valid = 1;
    }
    return r;
}

int get_event(fracsolve_ctx *h, size_t idx, hipEvent_t *ev)
{
    while (h->evpool.size() <= idx) {
        hipEvent_t e;
        HIPCHK(h, hipEventCreate(&e));
        h->evpool.push_back(e);
    }
    *ev = h->evpool[idx];
    return FRACSOLVE_OK;
}

int run_ops(fracsolve_ctx *h, const std::vector<Op> &ops)
{
    for (const Op &op : ops) {
        hipError_t e = hipSuccess;
        size_t evi = 0;
        if (h->timing >= 2) {
            evi = 2 * h->recs.size();
            hipEvent_t e0;
            int rc = get_event(h, evi, &e0);
            if (rc) return rc;
            rc = get_event(h, evi + 1, &e0);
            if (rc) return rc;
            HIPCHK(h, hipEventRecord(h->evpool[evi], h->st));
        }
        switch (op.kind) {
            case OP_LEAF:
                e = launch_leaf(h->st, op.lc, h->L, dptr<LeafTask>(h, op.off), op.ntasks, op.mixed);
                break;
            case OP_LEAF_SCAN:
                e = launch_leaf_scan(h->st, op.lc, h->L, task_ref<LeafTask>(h, op), op.ntasks, op.mixed, op.lc.vec,
                                     op.cn, op.pair);
                break;
            case OP_LAG1:
                e = launch_halfK_tasks(h->st, dptr<Lag1Task>(h, op.off), op.ntasks, op.maxM);
                break;
            case OP_LEAF_ADV:
                e = launch_leaf_adv(h->st, op.lc, h->L, task_ref<AdvTask>(h, op), op.ntasks, op.wsum, op.pair);
                break;
            case OP_GEMM64:
                e = launch_gemm_update<double>(h->st, task_ref<UpdTask<double>>(h, op), op.ntasks, op.s, op.maxM,
                                               op.lead);
                break;
            case OP_GEMM32:
                e = launch_gemm_update<float>(h->st, task_ref<UpdTask<float>>(h, op), op.ntasks, op.s, op.maxM);
                break;
            case OP_FFT64:
                e = launch_fft_update_ex<double>(h->st, dptr<UpdTask<double>>(h, op.off), dptr<int64_t>(h, op.goff),
                                                 op.ntasks, op.s, op.maxM,
                                                 h->tw64, h->nmax, (cplx<double> *)h->zs,
                                                 h->zs_bytes / sizeof(cplx<double>), op.even, h->timing < 2);
                break;
            case OP_FFT32:
                e = launch_fft_update_ex<float>(h->st, dptr<UpdTask<float>>(h, op.off), dptr<int64_t>(h, op.goff),
                                                op.ntasks, op.s, op.maxM,
                                                h->tw32, h->nmax, (cplx<float> *)h->zs,
                                                h->zs_bytes / sizeof(cplx<float>), op.even, h->timing < 2);
                break;
        }
        if (e != hipSuccess) return fail(h, FRACSOLVE_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        h->kernels++;
        if (h->timing >= 2) {
            HIPCHK(h, hipEventRecord(h->evpool[evi + 1], h->st));
            const bool lf = op.kind == OP_LEAF || op.kind == OP_LEAF_SCAN || op.kind == OP_LEAF_ADV;
            int kind = lf                       ? 0
                       : op.kind == OP_GEMM64   ? 1
                       : op.kind == OP_GEMM32   ? 2
                       : op.kind == OP_FFT64    ? 3
                       : op.kind == OP_LAG1     ? 5
                                                : 4;
            h->recs.push_back({kind, lf ? h->L * (op.pair ? 2 : 1) : op.s, op.ntasks, op.bytes, evi});
            // the near-corner band of an FFT level as a group of its own:
            // X rows s-31..s-1, Y rows 0..30 read and written
            const bool fft = op.kind == OP_FFT64 || op.kind == OP_FFT32;
            if (fft && 2 * op.s <= fft_max_single_pass(op.kind == OP_FFT32) && corner_width(op.s) >= 2 &&
                !fft_band_in_update(op.s, op.kind == OP_FFT32)) {
                const size_t evj = 2 * h->recs.size();
                hipEvent_t e1;
                int rc = get_event(h, evj + 1, &e1);
                if (rc) return rc;
                HIPCHK(h, hipEventRecord(h->evpool[evj], h->st));
                e = op.kind == OP_FFT64
                        ? launch_fft_corner<double>(h->st, dptr<UpdTask<double>>(h, op.off), op.ntasks, op.s, op.maxM)
                        : launch_fft_corner<float>(h->st, dptr<UpdTask<float>>(h, op.off), op.ntasks, op.s, op.maxM);
                if (e != hipSuccess)
                    return fail(h, FRACSOLVE_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
                h->kernels++;
                HIPCHK(h, hipEventRecord(h->evpool[evj + 1], h->st));
                const double band = 3.0 * (double)(corner_width(op.s) - 1) * (double)op.maxM * 8.0 * op.ntasks;
                h->recs.push_back({5, op.s, op.ntasks, band, evj});
            }
        }
    }
    return FRACSOLVE_OK;
}

// Algorithmic HBM bytes of one level product: read the s rows of X, read and
// write the ny rows of Y (M columns each).
template <typename T>
double upd_bytes(const UpdTask<T> &t, double elem)
{
    return ((double)t.s + 2.0 * (double)t.ny) * (double)t.M * elem;
}

// Launch-sequence signature: equal signatures replay the same recorded graph
// (kernel arguments point into the descriptor buffer, whose contents are
// re-uploaded before every replay).
uint64_t ops_key(const std::vector<Op> &ops, const void *d_desc)
{
    uint64_t hsh = 1469598103934665603ULL ^ (uint64_t)(uintptr_t)d_desc;
    auto mix = [&](uint64_t v) {
        hsh ^= v;
        hsh *= 1099511628211ULL;
    };
    for (const Op &op : ops) {
        mix((uint64_t)op.kind);
        mix((uint64_t)op.off);
        mix((uint64_t)op.ntasks);
        mix((uint64_t)op.s);
        mix((uint64_t)op.maxM);
        mix((uint64_t)(op.lc.nt * 100 + op.lc.pt));
        mix((uint64_t)op.mixed);
        mix((uint64_t)op.even);
        mix((uint64_t)op.goff);
        mix((uint64_t)op.lead);
        mix((uint64_t)op.lc.vec);
        mix((uint64_t)op.wsum);
        mix((uint64_t)op.cn);
        mix((uint64_t)op.pair);
    }
    mix((uint64_t)ops.size());
    return hsh;
}

// Run a launch sequence through a cached graph on the internal stream,
// ordered after and before the caller's stream by events.
int run_ops_graph(fracsolve_ctx *h, const std::vector<Op> &ops)
{
    uint64_t key = ops_key(ops, h->d_desc);
    hipGraphExec_t exec = nullptr;
    for (auto &g : h->graphs)
        if (g.key == key) exec = g.exec;
    HIPCHK(h, hipEventRecord(h->ev_in, h->st));
    HIPCHK(h, hipStreamWaitEvent(h->gst, h->ev_in, 0));
    if (!exec) {
        hipStream_t user = h->st;
        h->st = h->gst;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(h->gst, hipStreamCaptureModeThreadLocal);
        h->capturing = true;
        int rc = (e == hipSuccess) ? run_ops(h, ops) : FRACSOLVE_E_DEVICE;
        h->capturing = false;
        hipError_t e2 = hipStreamEndCapture(h->gst, &graph);
        h->st = user;
        if (rc) return rc;
        if (e != hipSuccess || e2 != hipSuccess)
            return fail(h, FRACSOLVE_E_DEVICE, "graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(h, FRACSOLVE_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        if (h->graphs.size() >= 16) {
            hipGraphExecDestroy(h->graphs.front().exec);
            h->graphs.erase(h->graphs.begin());
        }
        h->graphs.push_back({key, exec});
    }
    HIPCHK(h, hipGraphLaunch(exec, h->gst));
    HIPCHK(h, hipEventRecord(h->ev_out, h->gst));
    HIPCHK(h, hipStreamWaitEvent(h->st, h->ev_out, 0));
    return FRACSOLVE_OK;
}

int run_ops_any(fracsolve_ctx *h, const std::vector<Op> &ops)
{
    if (h->use_graph && h->timing < 2) return run_ops_graph(h, ops);
    return run_ops(h, ops);
}

// Field views of one recursive solve.
struct Field {
    double *u;        // right-hand side in / solution out [N][M]
    float *hist32;    // mixed: history accumulator (zeroed by caller)
    float *x32;       // mixed: float32 shadow of solved rows
    double *out = nullptr;  // advection, Scheme 2: solution U (u then holds W = B U)
};

// Build the launch list of the recursive solve of every instance in `sel`
// (lockstep over leaf index).  prec: FRACSOLVE_FP64 or FRACSOLVE_FP32.
void build_solve(fracsolve_ctx *h, const std::vector<int> &sel, const std::vector<Field> &fld, int prec,
                 DescBuilder &db, std::vector<Op> &ops)
{
    const int L = h->L;
    const bool mixed = (prec != FRACSOLVE_FP64);
    int64_t K = 0;
    for (int i : sel) K = std::max(K, h->inst[i].Np / L);
    for (int64_t k = 0; k < K; ++k) {
        // leaves, one launch per leaf configuration; in pair mode leaf k + 1
        // (k even) runs in the launch of leaf k
        const bool pair_first = h->pair && (k % 2 == 0);
        const bool pair_second = h->pair && (k % 2 == 1);
        std::vector<std::pair<int, LeafTask>> lt;
        std::vector<std::pair<int, AdvTask>> at;
        for (size_t q = 0; q < sel.size() && !pair_second; ++q) {
            const Inst &in = h->inst[sel[q]];
            int64_t lo = k * L;
            if (lo >= in.N) continue;
            if (in.adv) {
                AdvTask t{};
                t.x = fld[q].u;
                t.u = (in.adv == 2) ? fld[q].out : nullptr;
                t.a = in.a;
                t.fac = in.fac;
                t.M = in.M;
                t.lo = lo;
                t.nrows = (int)std::min<int64_t>(pair_first ? 2 * L : L, in.N - lo);
                at.push_back({(in.adv == 2 ? 100000 : 0) + in.lc.nt * 100 + in.lc.pt, t});
                continue;
            }
            LeafTask t{};
            t.u = fld[q].u;
            t.a = in.a;
            t.fac = in.fac;
            t.hist = mixed ? fld[q].hist32 : nullptr;
            t.x32 = mixed ? fld[q].x32 : nullptr;
            t.M = in.M;
            t.lo = lo;
            t.nrows = (int)std::min<int64_t>(pair_first ? 2 * L : L, in.N - lo);
            t.flags = (in.perm.pt > 2 && in.perm.mfull > 0) ? LEAF_PERM : 0;
            // whole 16-byte row units for the scan leaf
            if (in.scan && (in.M % in.lc.pt) == 0 && ((uintptr_t)t.u & 15) == 0) t.flags |= LEAF_VEC;
            lt.push_back({(in.scan ? 1000000 : 0) + in.lc.nt * 100 + in.lc.pt, t});
        }
        std::stable_sort(at.begin(), at.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
        for (size_t b = 0; b < at.size();) {
            size_t e = b;
            while (e < at.size() && at[e].first == at[b].first) ++e;
            std::vector<AdvTask> v;
            for (size_t j = b; j < e; ++j) v.push_back(at[j].second);
            size_t off = db.add(v.data(), v.size() * sizeof(AdvTask));
            const int key = at[b].first % 100000;
            LeafCfg lc{key / 100, key % 100, 0};
            Op op{OP_LEAF_ADV, off, (int)v.size(), 0, 0, lc, false};
            op.wsum = at[b].first >= 100000;
            op.pair = pair_first;
            for (auto &t : v) op.bytes += (double)t.nrows * (double)t.M * (op.wsum ? 24.0 : 16.0);
            ops.push_back(op);
            b = e;
        }
        // stable: with one leaf configuration, leaf task t is level task t
        // (the dense levels place task t's tiles on leaf t's XCD)
        std::stable_sort(lt.begin(), lt.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
        for (size_t b = 0; b < lt.size();) {
            size_t e = b;
            while (e < lt.size() && lt[e].first == lt[b].first) ++e;
            std::vector<LeafTask> v;
            int nvec = 0;
            for (size_t j = b; j < e; ++j) {
                v.push_back(lt[j].second);
                nvec += (lt[j].second.flags & LEAF_VEC) ? 1 : 0;
            }
            size_t off = db.add(v.data(), v.size() * sizeof(LeafTask));
            const int key = lt[b].first % 1000000;
            LeafCfg lc{key / 100, key % 100, 0};
            lc.S = ilog2i(2 * lc.nt);
            // one launch per configuration: vector rows for all, for none, or per task
            lc.vec = nvec == (int)v.size() ? 1 : (nvec == 0 ? 0 : 2);
            Op op{lt[b].first >= 1000000 ? OP_LEAF_SCAN : OP_LEAF, off, (int)v.size(), 0, 0, lc, mixed};
            op.cn = (h->opts.equation == FRACSOLVE_DIFFUSION_CN);
            op.pair = pair_first;
            for (auto &t : v) op.bytes += (double)t.nrows * (double)t.M * (mixed ? 24.0 : 16.0);
            ops.push_back(op);
            b = e;
        }
        // level product after leaf k (of half-size L after an even leaf:
        // inside the pair's launch in pair mode)
        if (k + 1 >= K) break;
        if (pair_first) continue;
        int64_t kk = k + 1;
        int64_t s = (int64_t)L * (kk & -kk);
        int64_t mid = kk * L, lo = mid - s;
        // Dense levels carry the largest weights and stay float64 in every
        // mode; FFT levels use float32 products in the mixed modes (their
        // near-corner band is added in float64 through xc/yc).
        const bool fft = s > h->crossover;
        const bool f32 = mixed && fft;
        std::vector<UpdTask<double>> t64;
        std::vector<UpdTask<float>> t32;
        int64_t maxM = 0;
        for (size_t q = 0; q < sel.size(); ++q) {
            const Inst &in = h->inst[sel[q]];
            if (mid >= in.N) continue;
            const int lev = ilog2i(s);
            if (!f32) {
                UpdTask<double> t{};
                t.x = fld[q].u;
                t.y = fld[q].u;
                t.w = in.a;
                t.spec = fft ? in.spec64 + in.spec_off[lev] : nullptr;
                t.xc = fld[q].u;
                t.yc = fld[q].u;
                t.M = in.M;
                t.xlo = lo;
                t.ylo = mid;
                t.s = (int)s;
                t.ny = (int)std::min<int64_t>(s, in.N - mid);
                t.alpha = -1.0;
                t64.push_back(t);
            } else {
                UpdTask<float> t{};
                t.x = fld[q].x32;
                t.y = fld[q].hist32;
                t.w = in.a;
                t.spec = in.spec32 + in.spec_off[lev];
                t.xc = fld[q].u;
                t.yc = fld[q].u;
                t.M = in.M;
                t.xlo = lo;
                t.ylo = mid;
                t.s = (int)s;
                t.ny = (int)std::min<int64_t>(s, in.N - mid);
                t.alpha = -1.0;
                t32.push_back(t);
            }
            maxM = std::max(maxM, in.M);
        }
        const bool multipass = 2 * s > fft_max_single_pass(f32);
        if (!t64.empty()) {
            if (fft && multipass) {
                for (auto &t : t64) {
                    Op op{OP_FFT64, db.add(&t, sizeof t), 1, (int)s, t.M, {}, false};
                    op.bytes = upd_bytes(t, 8);
                    ops.push_back(op);
                }
            } else {
                size_t off = db.add(t64.data(), t64.size() * sizeof(t64[0]));
                Op op{fft ? OP_FFT64 : OP_GEMM64, off, (int)t64.size(), (int)s, maxM, {}, false};
                if (fft)
                    op.goff = add_group_offsets(db, t64, (int)s);
                else
                    op.lead = L;
                op.even = true;
                for (auto &t : t64) {
                    op.bytes += upd_bytes(t, 8);
                    op.even = op.even && pairs_aligned(t);
                }
                ops.push_back(op);
            }
        }
        if (h->opts.equation == FRACSOLVE_DIFFUSION_CN) {
            // lag-1 block a_1 I + K/2: its K/2 part from the last row of the
            // block to the first row of the next leaf
            std::vector<Lag1Task> lg;
            int64_t lm = 0;
            for (size_t q = 0; q < sel.size(); ++q) {
                const Inst &in = h->inst[sel[q]];
                if (mid >= in.N) continue;
                lg.push_back(Lag1Task{fld[q].u + (mid - 1) * in.M, fld[q].u + mid * in.M, in.M, -0.5 * in.e, in.perm});
                lm = std::max(lm, in.M);
            }
            if (!lg.empty()) {
                Op op{OP_LAG1, db.add(lg.data(), lg.size() * sizeof(Lag1Task)), (int)lg.size(), (int)s, lm, {}, false};
                op.bytes = 0.0;
                for (auto &g : lg) op.bytes += 3.0 * (double)g.M * 8.0;
                ops.push_back(op);
            }
        }
        if (!t32.empty()) {
            if (multipass) {
                for (auto &t : t32) {
                    Op op{OP_FFT32, db.add(&t, sizeof t), 1, (int)s, t.M, {}, true};
                    op.bytes = upd_bytes(t, 4);
                    ops.push_back(op);
                }
            } else {
                size_t off = db.add(t32.data(), t32.size() * sizeof(t32[0]));
                Op op{OP_FFT32, off, (int)t32.size(), (int)s, maxM, {}, true};
                op.goff = add_group_offsets(db, t32, (int)s);
                op.even = true;
                for (auto &t : t32) {
                    op.bytes += upd_bytes(t, 4);
                    op.even = op.even && pairs_aligned(t);
                }
                ops.push_back(op);
            }
        }
    }
}

// Build the launch list of the off-diagonal part of an operator apply
// y += alpha * (sum over level tiles) for one instance and weights (a or da).
void build_apply_levels(fracsolve_ctx *h, const Inst &in, const double *x, double *y, bool deriv, DescBuilder &db,
                        std::vector<Op> &ops)
{
    const int L = h->L;
    for (int64_t s = L; s < in.Np; s *= 2) {
        int lev = ilog2i(s);
        bool fft = s > h->crossover;
        bool multipass = 2 * s > fft_max_single_pass(false);
        std::vector<UpdTask<double>> tv;
        for (int64_t lo = 0; lo + s < in.N; lo += 2 * s) {
            UpdTask<double> t{};
            t.x = x;
            t.y = y;
            t.w = deriv ? in.da : in.a;
            t.spec = fft ? (deriv ? in.dspec64 : in.spec64) + in.spec_off[lev] : nullptr;
            t.M = in.M;
            t.xlo = lo;
            t.ylo = lo + s;
            t.s = (int)s;
            t.ny = (int)std::min<int64_t>(s, in.N - (lo + s));
            t.alpha = 1.0;
            t.xc = x;
            t.yc = y;
            tv.push_back(t);
        }
        if (tv.empty()) continue;
        if (fft && multipass) {
            for (auto &t : tv) {
                Op op{OP_FFT64, db.add(&t, sizeof t), 1, (int)s, in.M, {}, false};
                op.bytes = upd_bytes(t, 8);
                ops.push_back(op);
            }
        } else {
            size_t off = db.add(tv.data(), tv.size() * sizeof(tv[0]));
            Op op{fft ? OP_FFT64 : OP_GEMM64, off, (int)tv.size(), (int)s, in.M, {}, false};
            if (fft) op.goff = add_group_offsets(db, tv, (int)s);
            op.even = true;
            for (auto &t : tv) {
                op.bytes += upd_bytes(t, 8);
                op.even = op.even && pairs_aligned(t);
            }
            ops.push_back(op);
        }
    }
}

int ensure(fracsolve_ctx *h, double **p, int64_t n)
{
    if (*p) return FRACSOLVE_OK;
    return dalloc(h, p, (size_t)n);
}
int ensuref(fracsolve_ctx *h, float **p, int64_t n)
{
    if (*p) return FRACSOLVE_OK;
    return dalloc(h, p, (size_t)n);
}

// Recursive solve of the assembled right-hand sides in fld (u in place).
int dc_solve(fracsolve_ctx *h, const std::vector<int> &sel, const std::vector<Field> &fld, int prec)
{
    if (prec != FRACSOLVE_FP64) {
        for (size_t q = 0; q < sel.size(); ++q) {
            const Inst &in = h->inst[sel[q]];
            HIPCHK(h, launch_zero(h->st, fld[q].hist32, sizeof(float) * (size_t)(in.M * in.N)));
            h->kernels++;
        }
    }
    DescBuilder db{h, {}};
    std::vector<Op> ops;
    build_solve(h, sel, fld, prec, db, ops);
    int rc = desc_upload(h, db);
    if (rc) return rc;
    return run_ops_any(h, ops);
}

// y = A x in float64 (deriv: y = (dA/dgamma) x, i.e. weights a' and no K).
// x and y are distinct [N][M] device arrays of instance i.
// x and y are in the column order perm (natural order: {0, 0}).
int apply_op(fracsolve_ctx *h, int i, const double *x, double *y, bool deriv, ColPerm perm)
{
    Inst &in = h->inst[i];
    const double eb = in.cn ? 0.5 * in.e : in.e;  // K's coefficient in the diagonal block
    HIPCHK(h, launch_diag_apply(h->st, x, y, deriv ? in.da : in.a, deriv ? 0.0 : eb, in.M, in.N, h->L, perm));
    h->kernels++;
    DescBuilder db{h, {}};
    std::vector<Op> ops;
    build_apply_levels(h, in, x, y, deriv, db, ops);
    int rc = desc_upload(h, db);
    if (rc) return rc;
    if ((rc = run_ops_any(h, ops))) return rc;
    if (in.cn && !deriv && in.N > 1) {
        // (K/2) U^{n-1} in row n
        HIPCHK(h, launch_halfK_rows(h->st, x, y + in.M, in.M, in.N - 1, 0.5 * in.e, perm));
        h->kernels++;
    }
    return FRACSOLVE_OK;
}

// sum of a device reduction written as per-block partials
int finish_sum(fracsolve_ctx *h, int nb, double *out)
{
    std::vector<double> hp(nb);
    HIPCHK(h, hipMemcpyAsync(hp.data(), h->partial, sizeof(double) * nb, hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    double s = 0.0;
    for (double v : hp) s += v;
    *out = s;
    return FRACSOLVE_OK;
}

int finish_max(fracsolve_ctx *h, int nb, double *out)
{
    std::vector<double> hp(nb);
    HIPCHK(h, hipMemcpyAsync(hp.data(), h->partial, sizeof(double) * nb, hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    double s = 0.0;
    for (double v : hp) s = std::max(s, v);
    *out = s;
    return FRACSOLVE_OK;
}

constexpr int kRedBlocks = 1024;

// Leaf size and crossover of a handle: options, plan cache or built-in table
// (plan.hip).  A looked-up leaf size the leaf kernels cannot take for some
// instance (L = 16 needs at most two rows per leaf thread, and the advection
// leaf at most 8) falls back to 8.
Plan plan_for(const fracsolve_problem *probs, int32_t count, const fracsolve_options &o)
{
    int64_t mmax = 0;
    for (int k = 0; k < count; ++k) mmax = std::max<int64_t>(mmax, probs[k].M);
    Plan pl = resolve_plan(o.precision, o.equation, mmax, o.leaf, o.crossover);
    if (o.leaf == 0 && pl.leaf > 8) {
        bool ok = o.equation != FRACSOLVE_ADVECTION;
        for (int k = 0; k < count && ok; ++k) {
            const bool scan = o.leaf_solver == 0;
            const LeafCfg lc = scan ? scan_config(count > 1 ? mmax : probs[k].M, count > 1,
                                                  o.equation == FRACSOLVE_DIFFUSION_CN)
                                    : leaf_config(probs[k].M);
            if ((scan && lc.pt > 2) || (!scan && lc.pt == 16)) ok = false;
        }
        if (!ok) pl.leaf = 8;
    }
    // Batches in float64: a batch's FFT level is one persistent launch over
    // the column groups of every instance, while a dense level's grid is
    // sized by the widest one, so the looked-up crossover (tuned on single
    // instances) is capped at 128.  Measured on five batches (8 to 256
    // instances, uniform and uneven widths): 2 to 15% faster than the
    // single-instance plan.
    if (o.crossover == 0 && count > 1 && o.precision == FRACSOLVE_FP64 && pl.crossover > 128) pl.crossover = 128;
    return pl;
}

int validate_problem(const fracsolve_problem &p, int k)
{
    char what[64];
    snprintf(what, sizeof what, "instance %d", k);
    if (!(p.gamma > 0.0 && p.gamma < 2.0) || p.gamma == 1.0 || !std::isfinite(p.gamma))
        return fail(nullptr, FRACSOLVE_E_ARG, "%s: gamma must lie in (0,1) or (1,2), got %g", what, p.gamma);
    if (!(p.T > 0.0) || !std::isfinite(p.T))
        return fail(nullptr, FRACSOLVE_E_ARG, "%s: T must be positive, got %g", what, p.T);
    if (!(p.x1 > p.x0) || !std::isfinite(p.x0) || !std::isfinite(p.x1))
        return fail(nullptr, FRACSOLVE_E_ARG, "%s: need x1 > x0, got [%g, %g]", what, p.x0, p.x1);
    if (p.M < 1 || p.M > 4096)
        return fail(nullptr, FRACSOLVE_E_ARG, "%s: M must lie in [1, 4096], got %lld", what, (long long)p.M);
    // the largest level product is an FFT of 2 Np / 2 = Np points: one
    // single-pass transform of at most 8192 points times an outer digit of
    // at most 16 (multi-pass route), so Np <= 2^17
    if (p.N < 1 || p.N > (1LL << 17))
        return fail(nullptr, FRACSOLVE_E_ARG, "%s: N must lie in [1, 2^17], got %lld", what, (long long)p.N);
    return FRACSOLVE_OK;
}

void free_all(fracsolve_ctx *h)
{
    for (auto &g : h->graphs) hipGraphExecDestroy(g.exec);
    h->graphs.clear();
    if (h->gst) hipStreamDestroy(h->gst);
    if (h->ev_in) hipEventDestroy(h->ev_in);
    if (h->ev_out) hipEventDestroy(h->ev_out);
    h->gst = nullptr;
    h->ev_in = h->ev_out = nullptr;
    for (double *p : h->allocs) hipFree(p);
    h->allocs.clear();
    if (h->h_desc) hipHostFree(h->h_desc);
    if (h->d_desc) hipFree(h->d_desc);
    if (h->zs) hipFree(h->zs);
    if (h->desc_ready) hipEventDestroy(h->desc_ready);
    h->h_desc = h->d_desc = h->zs = nullptr;
    h->desc_ready = nullptr;
}

int setup_instance(fracsolve_ctx *h, Inst &in)
{
    const fracsolve_problem &p = in.p;
    in.regime = (p.gamma < 1.0) ? 0 : 1;
    in.M = p.M;
    in.N = p.N;
    in.Np = std::max<int64_t>(next_pow2(p.N), h->L);
    in.tau = p.T / (double)p.N;
    in.h = (p.x1 - p.x0) / (double)(p.M + 1);
    in.e = 1.0 / (in.h * in.h);
    in.pexp = (in.regime == 0) ? 1.0 - p.gamma : 2.0 - p.gamma;
    double garg = (in.regime == 0) ? 2.0 - p.gamma : 3.0 - p.gamma;
    in.coef = std::pow(in.tau, -p.gamma) / std::tgamma(garg);
    in.dcoef = in.coef * (-std::log(in.tau) + digamma_host(garg));
    in.adv = (h->opts.equation == FRACSOLVE_ADVECTION) ? (in.regime == 0 ? 2 : 3) : 0;
    in.cn = (h->opts.equation == FRACSOLVE_DIFFUSION_CN);
    in.scan = (h->opts.leaf_solver == 0) || in.adv;
    in.lc = in.scan ? scan_config(h->batch_M > 0 ? h->batch_M : in.M, h->batch_M > 0, in.cn) : leaf_config(in.M);
    if (!in.adv && in.scan && in.lc.pt > 2 && in.M % in.lc.pt == 0)
        in.perm = ColPerm{in.lc.pt, (in.M / (64 * (int64_t)in.lc.pt)) * 64 * (int64_t)in.lc.pt};
    if (h->L > 8 && ((in.scan && in.lc.pt > 2) || (!in.scan && in.lc.pt == 16)))
        return fail(h, FRACSOLVE_E_ARG, "leaf size %d is not available for M = %lld (use 4 or 8)", h->L,
                    (long long)in.M);

    // weights: length Np plus slack for the dense kernel's window reads
    const int64_t WL = in.Np + 2048;
    int rc;
    if ((rc = dalloc(h, &in.b, WL)) || (rc = dalloc(h, &in.a, WL)) || (rc = dalloc(h, &in.rho, WL)) ||
        (rc = dalloc(h, &in.psi, WL)) || (rc = dalloc(h, &in.da, WL)) || (rc = dalloc(h, &in.drho, WL)) ||
        (rc = dalloc(h, &in.dpsi, WL)))
        return rc;
    for (double *q : {in.b, in.a, in.rho, in.psi, in.da, in.drho, in.dpsi})
        HIPCHK(h, launch_zero(h->st, q, sizeof(double) * (size_t)WL));
    HIPCHK(h, launch_weights(h->st, in.regime, in.pexp, in.coef, in.dcoef, in.tau, in.Np, in.b, in.a, in.rho,
                             in.psi, in.da, in.drho, in.dpsi));

    // factor table of a_0 I + K (advection: of the bidiagonal block)
    if (in.adv) {
        if ((rc = dalloc(h, &in.fac, adv_table_doubles()))) return rc;
        HIPCHK(h, launch_adv_factor(h->st, in.lc, in.coef, in.h, in.adv == 2, in.fac));
    } else if (in.scan) {
        if ((rc = dalloc(h, &in.fac, scan_table_doubles(in.lc)))) return rc;
        // averaged variant: diagonal block a_0 I + K/2
        HIPCHK(h, launch_scan_factor(h->st, in.lc, in.M, in.coef, in.cn ? 0.5 * in.e : in.e, in.fac));
    } else {
        if ((rc = dalloc(h, &in.fac, leaf_table_doubles(in.lc)))) return rc;
        HIPCHK(h, launch_leaf_factor(h->st, in.lc, in.M, in.coef, in.e, in.fac));
    }

    // spectra of a and a' for every level s in [L, Np/2] (all levels, so that
    // the crossover can be changed and the apply can use the FFT route)
    int nlev = ilog2i(in.Np) + 1;
    in.spec_off.assign(nlev, -1);
    int64_t total = 0;
    for (int64_t s = h->L; s < in.Np; s *= 2) {
        in.spec_off[ilog2i(s)] = total;
        total += 2 * s;
    }
    if ((rc = dalloc(h, &in.spec64, total)) || (rc = dalloc(h, &in.dspec64, total)) ||
        (rc = dalloc(h, &in.spec32, total)))
        return rc;
    cplx<double> *scr = nullptr;
    if ((rc = dalloc(h, &scr, 2 * in.Np))) return rc;
    for (int64_t s = h->L; s < in.Np; s *= 2) {
        int64_t off = in.spec_off[ilog2i(s)];
        HIPCHK(h, launch_spectrum(h->st, in.a, (int)s, in.spec64 + off, in.spec32 + off, h->tw64, h->nmax, scr));
        HIPCHK(h, launch_spectrum(h->st, in.da, (int)s, in.dspec64 + off, nullptr, h->tw64, h->nmax, scr));
    }
    return FRACSOLVE_OK;
}

int check_fields(fracsolve_ctx *h, const void *const *arr, const char *name, bool required)
{
    if (!arr) {
        if (required) return fail(h, FRACSOLVE_E_ARG, "%s is NULL", name);
        return FRACSOLVE_OK;
    }
    if (required)
        for (size_t k = 0; k < h->inst.size(); ++k)
            if (!arr[k]) return fail(h, FRACSOLVE_E_ARG, "%s[%zu] is NULL", name, k);
    return FRACSOLVE_OK;
}

const double *opt_ptr(const double *const *arr, size_t k) { return arr ? arr[k] : nullptr; }

// Refinement and solve driver for all instances.
int solve_all(fracsolve_ctx *h, const double *const *f, const double *const *u0, const double *const *phi,
              double *const *u)
{
    const size_t cnt = h->inst.size();
    const int prec = h->opts.precision;
    std::vector<int> sel(cnt);
    for (size_t k = 0; k < cnt; ++k) sel[k] = (int)k;
    int rc;
    // right-hand sides R = F - rho u0 + psi phi, written into u
    std::vector<Field> fld(cnt);
    for (size_t k = 0; k < cnt; ++k) {
        Inst &in = h->inst[k];
        fld[k] = {u[k], nullptr, nullptr};
        if (in.adv == 2) {
            // Scheme 2: the recursion runs on W = B U; twice the scheme's
            // right-hand sides go to the workspace, U to u
            int rc2 = ensure(h, &in.W, in.M * in.N);
            if (rc2) return rc2;
            HIPCHK(h, launch_rhs_adv2(h->st, f[k], opt_ptr(u0, k), in.rho, in.W, in.M, in.N));
            h->kernels++;
            fld[k] = {in.W, nullptr, nullptr, u[k]};
            continue;
        }
        const double *ph = (in.regime == 1) ? opt_ptr(phi, k) : nullptr;
        if (in.perm.mfull > 0 && !in.cn) {
            // right-hand sides written straight into the internal column order
            HIPCHK(h, launch_rhs_perm(h->st, f[k], opt_ptr(u0, k), ph, in.rho, in.psi, u[k], in.M, in.N, in.perm));
            h->kernels++;
            continue;
        }
        HIPCHK(h, launch_rhs(h->st, f[k], opt_ptr(u0, k), ph, in.rho, in.psi, u[k], in.M, in.N));
        h->kernels++;
        if (in.cn && opt_ptr(u0, k)) {
            // step 1 of the averaged variant carries -(K/2) u0
            HIPCHK(h, launch_halfK_rows(h->st, opt_ptr(u0, k), u[k], in.M, 1, -0.5 * in.e, ColPerm{0, 0}));
            h->kernels++;
        }
        // to the internal column order (in place)
        if (in.perm.mfull > 0) {
            HIPCHK(h, launch_permute(h->st, u[k], u[k], in.M, in.N, in.perm, true, false));
            h->kernels++;
        }
    }
    // back to the natural column order (in place)
    auto restore = [&]() -> int {
        for (size_t k = 0; k < cnt; ++k) {
            Inst &in = h->inst[k];
            if (in.perm.mfull > 0) {
                HIPCHK(h, launch_permute(h->st, u[k], u[k], in.M, in.N, in.perm, false, false));
                h->kernels++;
            }
        }
        return FRACSOLVE_OK;
    };
    if (prec == FRACSOLVE_FP64) {
        if ((rc = dc_solve(h, sel, fld, FRACSOLVE_FP64))) return rc;
        return restore();
    }
    // mixed: float32 products, float64 leaves; then refinement steps
    for (size_t k = 0; k < cnt; ++k) {
        Inst &in = h->inst[k];
        int64_t n = in.M * in.N;
        if ((rc = ensuref(h, &in.hist32, n)) || (rc = ensuref(h, &in.x32, n))) return rc;
        if (h->opts.refine_steps > 0) {
            if ((rc = ensure(h, &in.R, n)) || (rc = ensure(h, &in.W, n)) || (rc = ensure(h, &in.V, n))) return rc;
            HIPCHK(h, hipMemcpyAsync(in.R, u[k], sizeof(double) * n, hipMemcpyDeviceToDevice, h->st));
        }
        fld[k] = {u[k], in.hist32, in.x32};
    }
    if ((rc = dc_solve(h, sel, fld, FRACSOLVE_FP32))) return rc;
    for (int step = 0; step < h->opts.refine_steps; ++step) {
        // W = R - A U ; solve A D = W (mixed) ; U += D
        for (size_t k = 0; k < cnt; ++k) {
            Inst &in = h->inst[k];
            if ((rc = apply_op(h, (int)k, u[k], in.V, false, in.perm))) return rc;
            HIPCHK(h, launch_sub(h->st, in.W, in.R, in.V, in.M * in.N));
            h->kernels++;
            fld[k] = {in.W, in.hist32, in.x32};
        }
        if (h->timing) {
            Inst &in0 = h->inst[0];
            HIPCHK(h, launch_absmax_partial(h->st, in0.W, in0.M * in0.N, h->partial, kRedBlocks));
            if ((rc = finish_max(h, kRedBlocks, &h->stats.residual_norm))) return rc;
        }
        if ((rc = dc_solve(h, sel, fld, FRACSOLVE_FP32))) return rc;
        for (size_t k = 0; k < cnt; ++k) {
            Inst &in = h->inst[k];
            HIPCHK(h, launch_axpy(h->st, u[k], in.W, 1.0, in.M * in.N));
            h->kernels++;
        }
    }
    return restore();
}

// ---- restarted GMRES(m) on the same system (section 3.1) ----

void dfree(fracsolve_ctx *h, double *p)
{
    if (!p) return;
    hipFree(p);
    h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), p), h->allocs.end());
}

// z <- diag(a_0 I + K)^-1 z, every time row on its own: the leaf kernels with
// zero history weights, all blocks of rows in one launch.
int block_diag_solve(fracsolve_ctx *h, const Inst &in, double *z)
{
    const int L = h->L;
    std::vector<LeafTask> v;
    for (int64_t lo = 0; lo < in.N; lo += L) {
        LeafTask t{};
        t.u = z;
        t.a = h->zeros;
        t.fac = in.fac;
        t.M = in.M;
        t.lo = lo;
        t.nrows = (int)std::min<int64_t>(L, in.N - lo);
        t.flags = (in.scan && (in.M % in.lc.pt) == 0 && ((uintptr_t)z & 15) == 0) ? LEAF_VEC : 0;
        v.push_back(t);
    }
    DescBuilder db{h, {}};
    const size_t off = db.add(v.data(), v.size() * sizeof(LeafTask));
    LeafCfg lc = in.lc;
    lc.S = ilog2i(2 * lc.nt);
    lc.vec = (v[0].flags & LEAF_VEC) ? 1 : 0;
    Op op{in.scan ? OP_LEAF_SCAN : OP_LEAF, off, (int)v.size(), 0, 0, lc, false};
    op.bytes = 16.0 * (double)in.M * (double)in.N;
    int rc = desc_upload(h, db);
    if (rc) return rc;
    return run_ops_any(h, std::vector<Op>{op});
}

int dev_norm2(fracsolve_ctx *h, const double *x, int64_t n, double *out)
{
    HIPCHK(h, launch_dot_partial(h->st, x, x, n, h->partial, kRedBlocks));
    h->kernels++;
    double s = 0.0;
    int rc = finish_sum(h, kRedBlocks, &s);
    *out = std::sqrt(s);
    return rc;
}

constexpr int kDotBlocks = 512;

// out[i] = <V_i, w>, i < nv, on the host
int basis_dots(fracsolve_ctx *h, const double *V, int64_t n, int nv, const double *w, double *out)
{
    const int nb = (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (n + 1023) / 1024));
    HIPCHK(h, launch_multidot(h->st, V, n, nv, w, n, h->gpart, nb, h->gdots));
    h->kernels += 2;
    HIPCHK(h, hipMemcpyAsync(out, h->gdots, sizeof(double) * (size_t)nv, hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return FRACSOLVE_OK;
}

int lincomb(fracsolve_ctx *h, double *y, double beta, const double *V, int64_t n, int nv, const double *c)
{
    HIPCHK(h, launch_lincomb(h->st, y, beta, V, n, nv, c, n));
    h->kernels += (nv + LINCOMB_MAX - 1) / LINCOMB_MAX;
    return FRACSOLVE_OK;
}

struct GmresResult {
    int iters = 0, cycles = 0, converged = 0;
    double relres = 0.0, est = 0.0;
};

// One instance.  Arnoldi with classical Gram-Schmidt applied twice (two
// multi-dot / multi-update passes per step instead of the j sequential dot
// products of modified Gram-Schmidt), Givens rotations on the Hessenberg
// column as it arrives, restart after m steps; the control flow (early stop
// on the least-squares residual, recomputed residual after every cycle)
// matches the oracle's.
int gmres_one(fracsolve_ctx *h, int k, const double *f, const double *u0, const double *phi, double *u,
              const fracsolve_gmres_options &o, GmresResult &res, double *hist, int hist_cap)
{
    Inst &in = h->inst[k];
    const int64_t n = in.M * in.N;
    const int m = o.restart;
    int rc;
    if ((rc = ensure(h, &in.R, n)) || (rc = ensure(h, &in.W, n)) || (rc = ensure(h, &in.V, n))) return rc;
    if (in.kry_cap < m + 1) {
        dfree(h, in.kry);
        in.kry = nullptr;
        in.kry_cap = 0;
        if ((rc = dalloc(h, &in.kry, (size_t)(m + 1) * (size_t)n))) return rc;
        in.kry_cap = m + 1;
    }
    double *b = in.R, *w = in.W, *z = in.V, *B = in.kry;
    const double *ph = (in.regime == 1) ? phi : nullptr;
    HIPCHK(h, launch_rhs(h->st, f, u0, ph, in.rho, in.psi, b, in.M, in.N));
    h->kernels++;
    if (in.cn && u0) {
        HIPCHK(h, launch_halfK_rows(h->st, u0, b, in.M, 1, -0.5 * in.e, ColPerm{0, 0}));
        h->kernels++;
    }
    double bnorm = 0.0;
    if ((rc = dev_norm2(h, b, n, &bnorm))) return rc;
    if (!o.use_guess || bnorm == 0.0) {
        HIPCHK(h, launch_zero(h->st, u, sizeof(double) * (size_t)n));
        h->kernels++;
    }
    auto put_hist = [&](int i, double v) {
        if (hist && i < hist_cap) hist[i] = v;
    };
    if (bnorm == 0.0) {
        res.converged = 1;
        put_hist(0, 0.0);
        return FRACSOLVE_OK;
    }
    // w = b - A u
    auto residual = [&](double *beta) -> int {
        int r = apply_op(h, k, u, w, false, ColPerm{0, 0});
        if (r) return r;
        HIPCHK(h, launch_sub(h->st, w, b, w, n));
        h->kernels++;
        return dev_norm2(h, w, n, beta);
    };
    double beta = 0.0;
    if ((rc = residual(&beta))) return rc;
    put_hist(0, beta / bnorm);
    res.est = beta / bnorm;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m), c1(m + 1), c2(m + 1);
    auto HH = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    int it = 0;
    while (beta > o.rtol * bnorm && it < o.max_iters) {
        res.cycles++;
        const double sc0 = 1.0 / beta;
        if ((rc = lincomb(h, B, 0.0, w, n, 1, &sc0))) return rc;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int kk = 0;
        for (int j = 0; j < m && it < o.max_iters; ++j) {
            const double *vj = B + (int64_t)j * n;
            const double *x = vj;
            if (o.precond) {
                HIPCHK(h, hipMemcpyAsync(z, vj, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, h->st));
                if ((rc = block_diag_solve(h, in, z))) return rc;
                x = z;
            }
            if ((rc = apply_op(h, k, x, w, false, ColPerm{0, 0}))) return rc;
            // w -= V h twice (classical Gram-Schmidt with reorthogonalisation)
            if ((rc = basis_dots(h, B, n, j + 1, w, c1.data()))) return rc;
            for (int i = 0; i <= j; ++i) c2[i] = -c1[i];
            if ((rc = lincomb(h, w, 1.0, B, n, j + 1, c2.data()))) return rc;
            for (int i = 0; i <= j; ++i) HH(i, j) = c1[i];
            if ((rc = basis_dots(h, B, n, j + 1, w, c1.data()))) return rc;
            for (int i = 0; i <= j; ++i) c2[i] = -c1[i];
            if ((rc = lincomb(h, w, 1.0, B, n, j + 1, c2.data()))) return rc;
            for (int i = 0; i <= j; ++i) HH(i, j) += c1[i];
            double hn = 0.0;
            if ((rc = dev_norm2(h, w, n, &hn))) return rc;
            if (!std::isfinite(hn)) return fail(h, FRACSOLVE_E_NUMERIC, "GMRES: non-finite basis norm at step %d", it);
            // previous rotations on column j, then the one that removes hn
            for (int i = 0; i < j; ++i) {
                const double t0 = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
                const double t1 = -sn[i] * HH(i, j) + cs[i] * HH(i + 1, j);
                HH(i, j) = t0;
                HH(i + 1, j) = t1;
            }
            const double rr = std::hypot(HH(j, j), hn);
            cs[j] = HH(j, j) / rr;
            sn[j] = hn / rr;
            HH(j, j) = rr;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            kk = j + 1;
            res.est = std::fabs(g[j + 1]) / bnorm;
            put_hist(it, res.est);
            if (hn == 0.0 || std::fabs(g[j + 1]) <= o.rtol * bnorm) break;
            const double sc = 1.0 / hn;
            if ((rc = lincomb(h, B + (int64_t)(j + 1) * n, 0.0, w, n, 1, &sc))) return rc;
        }
        // u += P^-1 V y with R y = g
        for (int i = kk - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < kk; ++q) s -= HH(i, q) * y[q];
            y[i] = s / HH(i, i);
        }
        if ((rc = lincomb(h, z, 0.0, B, n, kk, y.data()))) return rc;
        if (o.precond && (rc = block_diag_solve(h, in, z))) return rc;
        HIPCHK(h, launch_axpy(h->st, u, z, 1.0, n));
        h->kernels++;
        if ((rc = residual(&beta))) return rc;
    }
    res.iters = it;
    res.converged = beta <= o.rtol * bnorm;
    res.relres = beta / bnorm;
    return FRACSOLVE_OK;
}

// ---- Scheme 1 (eq. e7): conjugate gradients with the FFT operator ----
//
// The two-sided ODE's matrix is A = I + T + T^T with T the lower-triangular
// Toeplitz matrix of the diffusion weights a (a_0 on the diagonal), so A is
// symmetric Toeplitz with column c_0 = 1 + 2 a_0, c_m = a_m (Theorem 1).  The
// weights come from the diffusion path's weight kernel on tau = 1/N; the
// product A x goes through the circulant embedding of length L >= 2n - 1
// (eq. e10): one forward and one inverse FFT of L points per product.  The
// handle (one point, one step) only provides the stream, the allocations and
// the error state.

struct OdeWork {
    double *r, *p, *Ap;
    double *S;       // real spectrum of the embedded column, divided by L
    double *za, *zb;  // two complex work arrays of L points
    double *pap;      // partial sums of <p, A p> from the product's last pass
    int64_t L;
};

int ode_matvec(fracsolve_ctx *h, const OdeWork &w, int64_t n, const double *x, double *y)
{
    HIPCHK(h, launch_circ_apply(h->st, x, y, n, w.L, w.S, w.za, w.zb));
    h->kernels += circ_launches(w.L);
    return FRACSOLVE_OK;
}

// Device buffers of one Scheme 1 CG call (n = N - 1 unknowns, L = circ_length(n)).
struct OdeBuffers {
    OdeWork w;
    double *a;     // [n]  Toeplitz column before the embedding
    CgState *ds;   // the device-side CG scalars
    double *dh;    // [hist_cap] residual history, or NULL
};

int ode_cg_core(fracsolve_ctx *h, double gamma, int64_t N, const double *f, double *u, const fracsolve_cg_options &o,
                fracsolve_cg_info *info, double *hist, int hist_cap, const OdeBuffers &bufs, bool allow_graph);

int ode_cg_run(fracsolve_ctx *h, double gamma, int64_t N, const double *f, double *u, const fracsolve_cg_options &o,
               fracsolve_cg_info *info, double *hist, int hist_cap)
{
    const int64_t n = N - 1;
    OdeBuffers b{};
    OdeWork &w = b.w;
    int rc;
    w.L = circ_length(n);
    for (double **q : {&w.r, &w.p, &w.Ap, &b.a})
        if ((rc = dalloc(h, q, (size_t)n))) return rc;
    if ((rc = dalloc(h, &w.S, (size_t)w.L)) || (rc = dalloc(h, &w.za, 2 * (size_t)w.L)) ||
        (rc = dalloc(h, &w.zb, 2 * (size_t)w.L)) || (rc = dalloc(h, &w.pap, (size_t)circ_dot_parts(w.L))))
        return rc;
    if ((rc = dalloc(h, &b.ds, 1))) return rc;
    if (hist_cap > 1 && (rc = dalloc(h, &b.dh, (size_t)hist_cap))) return rc;
    const char *genv = getenv("FRACSOLVE_ODE_GRAPH");
    return ode_cg_core(h, gamma, N, f, u, o, info, hist, hist_cap, b, !(genv && genv[0] == '0'));
}

int ode_cg_core(fracsolve_ctx *h, double gamma, int64_t N, const double *f, double *u, const fracsolve_cg_options &o,
                fracsolve_cg_info *info, double *hist, int hist_cap, const OdeBuffers &bufs, bool allow_graph)
{
    const int64_t n = N - 1;
    const OdeWork &w = bufs.w;
    double *a = bufs.a;
    int rc;
    // the L1 weights a_m of the left derivative (Lemma 2) on tau = 1/N,
    // scaled by mu = tau^-gamma / Gamma(2 - gamma)
    const double tau = 1.0 / (double)N;
    const double mu = std::pow(tau, -gamma) / std::tgamma(2.0 - gamma);
    HIPCHK(h, launch_weights(h->st, 0, 1.0 - gamma, mu, 0.0, tau, n, nullptr, a, nullptr, nullptr, nullptr, nullptr,
                             nullptr));
    // the embedded column is staged in S before its transform replaces it
    HIPCHK(h, launch_circ_spectrum(h->st, a, n, w.L, w.S, w.S, w.za, w.zb));
    auto put_hist = [&](int i, double v) {
        if (hist && i < hist_cap) hist[i] = v;
    };
    double fn = 0.0;
    if ((rc = dev_norm2(h, f, n, &fn))) return rc;
    if (!o.use_guess || fn == 0.0) HIPCHK(h, launch_zero(h->st, u, sizeof(double) * (size_t)n));
    fracsolve_cg_info res{0, 0, 0.0, 0.0};
    if (fn == 0.0) {
        res.converged = 1;
        put_hist(0, 0.0);
        if (info) *info = res;
        return FRACSOLVE_OK;
    }
    // r = f - A u, p = r
    if ((rc = ode_matvec(h, w, n, u, w.Ap))) return rc;
    HIPCHK(h, launch_sub(h->st, w.r, f, w.Ap, n));
    HIPCHK(h, hipMemcpyAsync(w.p, w.r, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, h->st));
    double rr = 0.0;
    if ((rc = dev_norm2(h, w.r, n, &rr))) return rc;
    rr *= rr;
    put_hist(0, std::sqrt(rr) / fn);
    // The scalars live on the device; the host enqueues a batch of steps and
    // reads the state back once per batch.  Steps past the stop are no-ops.
    CgState hs{};
    hs.rr = rr;
    hs.rtol_fn = o.rtol * fn;
    hs.fn = fn;
    hs.maxit = o.max_iters;
    hs.done = (o.max_iters <= 0 || std::sqrt(rr) <= o.rtol * fn) ? 1 : 0;
    CgState *ds = bufs.ds;
    double *dh = hist_cap > 1 ? bufs.dh : nullptr;
    HIPCHK(h, hipMemcpyAsync(ds, &hs, sizeof hs, hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    const int32_t *skip = &ds->done;
    const int batch = 8;
    // <p, A p> from the product's last pass saves a launch per step; above
    // L = 2^19 its partials (one per 8 butterflies) and the gathered reads of
    // p cost more than the separate reduction
    const bool fused_dot = w.L <= (int64_t(1) << 19);
    auto enqueue_batch = [&](hipStream_t st) -> hipError_t {
        for (int b = 0; b < batch; ++b) {
            int64_t npap = 0;
            double *pap = fused_dot ? w.pap : nullptr;
            hipError_t e = launch_circ_apply(st, w.p, w.Ap, n, w.L, w.S, w.za, w.zb, skip, pap, &npap);
            if (e == hipSuccess)
                e = launch_cg_step_tail(st, ds, u, w.r, w.p, w.Ap, n, pap, npap, h->partial, dh, hist_cap);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const int per_batch = batch * (circ_launches(w.L) + (fused_dot ? 4 : 5));
    // Up to L = 2^19 a step is launch-bound: one batch is captured once and
    // replayed as a graph on a stream of this call (default priority).  The
    // caller's stream is idle here (synchronised above) and every batch ends
    // with a host synchronisation, so no events are needed.
    struct OdeGraph {
        hipStream_t st = nullptr;
        hipGraphExec_t exec = nullptr;
        ~OdeGraph()
        {
            if (exec) hipGraphExecDestroy(exec);
            if (st) hipStreamDestroy(st);
        }
    } og;
    if (!hs.done && w.L <= (int64_t(1) << 19) && allow_graph) {
        HIPCHK(h, hipStreamCreateWithFlags(&og.st, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIPCHK(h, hipStreamBeginCapture(og.st, hipStreamCaptureModeThreadLocal));
        const hipError_t e1 = enqueue_batch(og.st);
        const hipError_t e2 = hipStreamEndCapture(og.st, &graph);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return fail(h, FRACSOLVE_E_DEVICE, "CG graph capture failed: %s",
                        hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        }
        const hipError_t e3 = hipGraphInstantiate(&og.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e3 != hipSuccess)
            return fail(h, FRACSOLVE_E_DEVICE, "CG graph instantiate failed: %s", hipGetErrorString(e3));
    }
    hipStream_t bst = og.exec ? og.st : h->st;
    while (!hs.done) {
        if (og.exec)
            HIPCHK(h, hipGraphLaunch(og.exec, bst));
        else
            HIPCHK(h, enqueue_batch(bst));
        h->kernels += per_batch;
        HIPCHK(h, hipMemcpyAsync(&hs, ds, sizeof hs, hipMemcpyDeviceToHost, bst));
        HIPCHK(h, hipStreamSynchronize(bst));
    }
    if (hs.bad) return fail(h, FRACSOLVE_E_NUMERIC, "CG: <p, A p> = %g at step %d", hs.pAp, (int)hs.it);
    const int it = hs.it;
    rr = hs.rr;
    if (dh && hist) {
        const int nh = std::min(hist_cap, it + 1);
        if (nh > 1) {
            HIPCHK(h, hipMemcpyAsync(hist + 1, dh + 1, sizeof(double) * (size_t)(nh - 1), hipMemcpyDeviceToHost,
                                     h->st));
            HIPCHK(h, hipStreamSynchronize(h->st));
        }
    }
    // the residual from its definition
    if ((rc = ode_matvec(h, w, n, u, w.Ap))) return rc;
    HIPCHK(h, launch_sub(h->st, w.r, f, w.Ap, n));
    double tr = 0.0;
    if ((rc = dev_norm2(h, w.r, n, &tr))) return rc;
    res.iterations = it;
    res.relres = tr / fn;
    res.relres_est = std::sqrt(rr) / fn;
    res.converged = (std::sqrt(rr) <= o.rtol * fn) ? 1 : 0;
    if (info) *info = res;
    return FRACSOLVE_OK;
}

// Argument checks shared by the two Scheme 1 entry points (before any
// device work); *o receives the options with their defaults.
int ode_check_args(double gamma, int64_t N, const double *f, const double *u, const fracsolve_cg_options *opts,
                   const double *hist, int32_t hist_cap, fracsolve_cg_options *o)
{
    if (!(gamma > 0.0 && gamma < 1.0))
        return fail(nullptr, FRACSOLVE_E_ARG, "gamma must lie in (0,1) for the two-sided ODE, got %g", gamma);
    if (N < 3 || N - 1 > (1LL << 22))
        return fail(nullptr, FRACSOLVE_E_ARG, "N must lie in [3, 2^22 + 1], got %lld", (long long)N);
    if (!f || !u) return fail(nullptr, FRACSOLVE_E_ARG, "f and u must not be NULL");
    *o = fracsolve_cg_options{10000, 1e-10, 0};
    if (opts) *o = *opts;
    if (o->max_iters < 0) return fail(nullptr, FRACSOLVE_E_ARG, "max_iters must be >= 0, got %d", (int)o->max_iters);
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol))
        return fail(nullptr, FRACSOLVE_E_ARG, "rtol must be finite and >= 0, got %g", o->rtol);
    if (o->use_guess < 0 || o->use_guess > 1)
        return fail(nullptr, FRACSOLVE_E_ARG, "use_guess must be 0 or 1, got %d", (int)o->use_guess);
    if (hist_cap < 0 || (hist_cap > 0 && !hist))
        return fail(nullptr, FRACSOLVE_E_ARG, "hist is NULL with hist_cap %d", (int)hist_cap);
    return FRACSOLVE_OK;
}

// Fixed workspace of fracsolve_ode_cg_noalloc: one copy per device, held for
// the life of the process.  Its host-side name is not a device address; the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and is the only way host code refers to the array.
constexpr size_t kOdeScratchBytes = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kOdeScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

int ode_scratch(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, FRACSOLVE_E_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, FRACSOLVE_E_DEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, FRACSOLVE_E_DEVICE, "hipGetSymbolAddress of the fixed workspace failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return FRACSOLVE_OK;
}

}  // namespace

extern "C" {

int fracsolve_ode_cg(double gamma, int64_t N, const double *f, double *u, const fracsolve_cg_options *opts,
                     fracsolve_cg_info *info, double *hist, int32_t hist_cap, void *stream)
{
    fracsolve_cg_options o{};
    int rc = ode_check_args(gamma, N, f, u, opts, hist, hist_cap, &o);
    if (rc) return rc;
    fracsolve_problem p{gamma, 1.0, 0.0, 1.0, 1, 1};
    fracsolve_options ho{};
    ho.stream = stream;
    fracsolve_t h = nullptr;
    rc = fracsolve_create(&p, 1, &ho, &h);
    if (rc) return rc;
    rc = ode_cg_run(h, gamma, N, f, u, o, info, hist, hist_cap);
    if (rc) g_create_error = h->err;
    fracsolve_destroy(h);
    return rc;
}

int fracsolve_ode_cg_noalloc(double gamma, int64_t N, const double *f, double *u, const fracsolve_cg_options *opts,
                             fracsolve_cg_info *info, double *hist, int32_t hist_cap, void *stream)
{
    fracsolve_cg_options o{};
    int rc = ode_check_args(gamma, N, f, u, opts, hist, hist_cap, &o);
    if (rc) return rc;
    if (N > FRACSOLVE_ODE_NOALLOC_MAX_N)
        return fail(nullptr, FRACSOLVE_E_ARG, "N = %lld exceeds the fixed workspace of the no-allocation entry point "
                    "(N <= %lld)", (long long)N, (long long)FRACSOLVE_ODE_NOALLOC_MAX_N);
    if (hist_cap > FRACSOLVE_ODE_NOALLOC_MAX_HIST)
        return fail(nullptr, FRACSOLVE_E_ARG, "hist_cap %d exceeds the fixed history of the no-allocation entry point "
                    "(%d)", (int)hist_cap, (int)FRACSOLVE_ODE_NOALLOC_MAX_HIST);
    char *base = nullptr;
    if ((rc = ode_scratch(&base))) return rc;
    const int64_t n = N - 1;
    OdeBuffers b{};
    b.w.L = circ_length(n);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *q = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return q;
    };
    b.w.r = (double *)take(sizeof(double) * (size_t)n);
    b.w.p = (double *)take(sizeof(double) * (size_t)n);
    b.w.Ap = (double *)take(sizeof(double) * (size_t)n);
    b.a = (double *)take(sizeof(double) * (size_t)n);
    b.w.S = (double *)take(sizeof(double) * (size_t)b.w.L);
    b.w.za = (double *)take(2 * sizeof(double) * (size_t)b.w.L);
    b.w.zb = (double *)take(2 * sizeof(double) * (size_t)b.w.L);
    b.w.pap = (double *)take(sizeof(double) * (size_t)circ_dot_parts(b.w.L));
    b.ds = (CgState *)take(sizeof(CgState));
    b.dh = (double *)take(sizeof(double) * (size_t)FRACSOLVE_ODE_NOALLOC_MAX_HIST);
    double *partial = (double *)take(sizeof(double) * kRedBlocks);
    if (off > kOdeScratchBytes)
        return fail(nullptr, FRACSOLVE_E_ARG, "workspace of %zu bytes exceeds the fixed array (%zu bytes)", off,
                    (size_t)kOdeScratchBytes);
    // a context without allocations: the stream, the reduction partials in
    // the fixed array and the error text; every buffer comes from the array
    // and the steps are launched directly (no captured graph)
    fracsolve_ctx ctx;
    ctx.st = (hipStream_t)stream;
    ctx.partial = partial;
    rc = ode_cg_core(&ctx, gamma, N, f, u, o, info, hist, hist_cap, b, false);
    if (rc) g_create_error = ctx.err;
    return rc;
}
int fracsolve_create(const fracsolve_problem *probs, int32_t count, const fracsolve_options *opts, fracsolve_t *out)
{
    if (!out) return fail(nullptr, FRACSOLVE_E_ARG, "out is NULL");
    *out = nullptr;
    if (!probs) return fail(nullptr, FRACSOLVE_E_ARG, "probs is NULL");
    if (count < 1) return fail(nullptr, FRACSOLVE_E_ARG, "count must be >= 1, got %d", (int)count);
    for (int k = 0; k < count; ++k) {
        int rc = validate_problem(probs[k], k);
        if (rc) return rc;
    }
    fracsolve_options o{};
    if (opts) o = *opts;
    if (o.precision < FRACSOLVE_FP64 || o.precision > FRACSOLVE_BF16X3)
        return fail(nullptr, FRACSOLVE_E_ARG, "unknown precision %d", (int)o.precision);
    if (o.precision == FRACSOLVE_BF16X3)
        return fail(nullptr, FRACSOLVE_E_ARG,
                    "precision 2 (split bf16 products) is not available in this version; use 0 (float64) or 1 "
                    "(float32 products with float64 refinement)");
    if (o.refine_steps < 0 || o.refine_steps > 8)
        return fail(nullptr, FRACSOLVE_E_ARG, "refine_steps must lie in [0, 8], got %d", (int)o.refine_steps);
    if (o.leaf_solver < 0 || o.leaf_solver > 1)
        return fail(nullptr, FRACSOLVE_E_ARG, "leaf_solver must be 0 or 1, got %d", (int)o.leaf_solver);
    if (o.leaf != 0 && o.leaf != 4 && o.leaf != 8 && o.leaf != 16)
        return fail(nullptr, FRACSOLVE_E_ARG, "leaf must be 0, 4, 8 or 16, got %d", (int)o.leaf);
    if (o.equation != FRACSOLVE_DIFFUSION && o.equation != FRACSOLVE_ADVECTION &&
        o.equation != FRACSOLVE_DIFFUSION_CN)
        return fail(nullptr, FRACSOLVE_E_ARG,
                    "equation must be 0 (diffusion), 1 (advection) or 2 (diffusion, averaged spatial term), got %d",
                    (int)o.equation);
    if (o.equation == FRACSOLVE_DIFFUSION_CN) {
        for (int k = 0; k < count; ++k)
            if (!(probs[k].gamma > 1.0))
                return fail(nullptr, FRACSOLVE_E_ARG,
                            "instance %d: the averaged spatial term is for 1 < gamma < 2, got gamma %g", k,
                            probs[k].gamma);
        if (o.precision != FRACSOLVE_FP64)
            return fail(nullptr, FRACSOLVE_E_ARG, "the averaged spatial term is solved in float64 only (precision 0)");
        if (o.leaf_solver != 0)
            return fail(nullptr, FRACSOLVE_E_ARG, "the averaged spatial term needs the scan leaf (leaf_solver 0)");
    }
    if (o.equation == FRACSOLVE_ADVECTION) {
        if (o.precision != FRACSOLVE_FP64)
            return fail(nullptr, FRACSOLVE_E_ARG, "the advection equations are solved in float64 only (precision 0)");
        if (o.leaf_solver != 0)
            return fail(nullptr, FRACSOLVE_E_ARG, "the advection equations have their own leaf (leaf_solver 0)");
        if (o.leaf == 16) return fail(nullptr, FRACSOLVE_E_ARG, "leaf must be 0, 4 or 8 for the advection equations");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        hipGetLastError();
        return fail(nullptr, FRACSOLVE_E_DEVICE, "no HIP device available");
    }
    fracsolve_ctx *h = new fracsolve_ctx();
    h->opts = o;
    h->st = (hipStream_t)o.stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(nullptr, FRACSOLVE_E_DEVICE, "hipGetDevice failed");
    }
    {
        const Plan pl = plan_for(probs, count, o);
        h->L = pl.leaf;
        // dense products are limited to s <= 1024 (k_gemm.hip)
        h->crossover = (pl.crossover > 0) ? std::min(pl.crossover, 1024) : 0;
        h->plan_source = pl.source;
    }
    {
        const char *pv = getenv("FRACSOLVE_PAIR");
        h->pair = !(pv && pv[0] == '0') && o.leaf_solver == 0 && h->L <= 8 && h->L <= h->crossover;
        // the advection leaf reads its rows element by element: past M = 1024
        // re-reading the first leaf's rows on one CU costs more than the
        // separate level product (measured)
        if (o.equation == FRACSOLVE_ADVECTION)
            for (int k = 0; k < count; ++k)
                if (probs[k].M > 1024) h->pair = false;
    }
    int64_t npmax = 0;
    for (int k = 0; k < count; ++k) npmax = std::max(npmax, std::max<int64_t>(next_pow2(probs[k].N), h->L));
    h->nmax = std::max<int64_t>(npmax, 16384);
    int rc = FRACSOLVE_OK;
    if (hipEventCreateWithFlags(&h->desc_ready, hipEventDisableTiming) != hipSuccess) rc = FRACSOLVE_E_DEVICE;
    {
        const char *g = getenv("FRACSOLVE_GRAPH");
        h->use_graph = g && g[0] == '1';
    }
    if (!rc && h->use_graph) {
        // internal stream at the default priority
        if (hipStreamCreateWithFlags(&h->gst, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming) != hipSuccess)
            rc = fail(h, FRACSOLVE_E_DEVICE, "stream/event creation failed");
    }
    if (!rc) rc = dalloc(h, &h->tw64, h->nmax);
    if (!rc) rc = dalloc(h, &h->tw32, h->nmax);
    if (!rc) rc = dalloc(h, &h->partial, kRedBlocks);
    if (!rc && launch_twiddles(h->st, h->nmax, h->tw64, h->tw32) != hipSuccess)
        rc = fail(h, FRACSOLVE_E_DEVICE, "twiddle kernel launch failed");
    h->inst.resize(count);
    if (count > 1)
        for (int k = 0; k < count; ++k) h->batch_M = std::max<int64_t>(h->batch_M, probs[k].M);
    for (int k = 0; k < count && !rc; ++k) {
        h->inst[k].p = probs[k];
        rc = setup_instance(h, h->inst[k]);
    }
    // multi-pass scratch: only when some FFT level exceeds the single-pass size
    if (!rc) {
        bool need = false;
        for (auto &in : h->inst)
            if (in.Np > fft_max_single_pass(false)) need = true;
        if (need) {
            // FRACSOLVE_MP_SCRATCH_MB: scratch size in MiB (16 to 4096)
            size_t mb = 256;
            if (const char *e = getenv("FRACSOLVE_MP_SCRATCH_MB")) {
                const long v = strtol(e, nullptr, 10);
                if (v >= 16 && v <= 4096) mb = (size_t)v;
            }
            h->zs_bytes = mb << 20;
            if (hipMalloc(&h->zs, h->zs_bytes) != hipSuccess) {
                hipGetLastError();
                rc = fail(h, FRACSOLVE_E_NOMEM, "multi-pass scratch allocation failed");
            }
        }
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) rc = fail(h, FRACSOLVE_E_DEVICE, "setup failed: %s", hipGetErrorString(e));
    }
    if (rc) {
        g_create_error = h->err.empty() ? g_create_error : h->err;
        free_all(h);
        delete h;
        return rc;
    }
    h->stats.leaf = h->L;
    h->stats.crossover = h->crossover;
    h->stats.levels = ilog2i(h->inst[0].Np / h->L);
    *out = h;
    return FRACSOLVE_OK;
}

int fracsolve_plan(const fracsolve_problem *probs, int32_t count, const fracsolve_options *opts, int32_t *leaf,
                   int32_t *crossover, int32_t *source)
{
    if (!probs) return fail(nullptr, FRACSOLVE_E_ARG, "probs is NULL");
    if (count < 1) return fail(nullptr, FRACSOLVE_E_ARG, "count must be >= 1, got %d", (int)count);
    for (int k = 0; k < count; ++k) {
        int rc = validate_problem(probs[k], k);
        if (rc) return rc;
    }
    fracsolve_options o{};
    if (opts) o = *opts;
    if (o.leaf != 0 && o.leaf != 4 && o.leaf != 8 && o.leaf != 16)
        return fail(nullptr, FRACSOLVE_E_ARG, "leaf must be 0, 4, 8 or 16, got %d", (int)o.leaf);
    const Plan pl = plan_for(probs, count, o);
    if (leaf) *leaf = pl.leaf;
    if (crossover) *crossover = pl.crossover > 0 ? std::min(pl.crossover, 1024) : -1;
    if (source) *source = pl.source;
    return FRACSOLVE_OK;
}

int fracsolve_weights(fracsolve_t h, int32_t inst, double *b, double *a, double *rho, double *psi, double *da,
                      double *drho, double *dpsi)
{
    if (!h) return fail(nullptr, FRACSOLVE_E_ARG, "handle is NULL");
    if (inst < 0 || inst >= (int32_t)h->inst.size())
        return fail(h, FRACSOLVE_E_ARG, "instance %d out of range [0, %zu)", (int)inst, h->inst.size());
    Inst &in = h->inst[inst];
    size_t bytes = sizeof(double) * (size_t)in.N;
    std::pair<double *, double *> pr[] = {{b, in.b},   {a, in.a},   {rho, in.rho}, {psi, in.psi},
                                          {da, in.da}, {drho, in.drho}, {dpsi, in.dpsi}};
    for (auto &x : pr)
        if (x.first) HIPCHK(h, hipMemcpyAsync(x.first, x.second, bytes, hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return FRACSOLVE_OK;
}

// With checking on (fracsolve_set_check): E_NUMERIC if a field of the call's
// output holds a NaN or an infinity.
static int check_outputs(fracsolve_ctx *h, const double *const *x, const char *name, int rc)
{
    if (rc || !h->check) return rc;
    for (size_t k = 0; k < h->inst.size(); ++k) {
        const Inst &in = h->inst[k];
        double cnt = 0.0;
        HIPCHK(h, launch_nonfinite_partial(h->st, x[k], in.M * in.N, h->partial, kRedBlocks));
        if ((rc = finish_sum(h, kRedBlocks, &cnt))) return rc;
        if (cnt > 0.0)
            return fail(h, FRACSOLVE_E_NUMERIC, "%s[%zu] holds %.0f non-finite values (of %lld)", name, k, cnt,
                        (long long)(in.M * in.N));
    }
    return FRACSOLVE_OK;
}

static int timed_begin(fracsolve_ctx *h, hipEvent_t *ev)
{
    h->kernels = 0;
    h->recs.clear();
    h->kstats.clear();
    if (!h->timing) return FRACSOLVE_OK;
    HIPCHK(h, hipEventCreate(&ev[0]));
    HIPCHK(h, hipEventCreate(&ev[1]));
    HIPCHK(h, hipEventRecord(ev[0], h->st));
    return FRACSOLVE_OK;
}

static int timed_end(fracsolve_ctx *h, hipEvent_t *ev, int rc)
{
    h->stats.kernels = h->kernels;
    if (!h->timing) return rc;
    if (!rc) {
        float ms = 0.0f;
        if (hipEventRecord(ev[1], h->st) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
            hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess)
            h->stats.ms_total = ms;
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (!rc && h->timing >= 2) {
        for (const auto &r : h->recs) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, h->evpool[r.ev], h->evpool[r.ev + 1]) != hipSuccess) continue;
            fracsolve_kernel_stat *ks = nullptr;
            for (auto &k : h->kstats)
                if (k.kind == r.kind && k.s == r.s) ks = &k;
            if (!ks) {
                h->kstats.push_back({r.kind, r.s, 0, 0, 0.0, 0.0});
                ks = &h->kstats.back();
            }
            ks->launches += 1;
            ks->tasks += r.ntasks;
            ks->ms += ms;
            ks->bytes += r.bytes;
        }
    }
    return rc;
}

int fracsolve_solve(fracsolve_t h, const double *const *f, const double *const *u0, const double *const *phi,
                    double *const *u)
{
    if (!h) return fail(nullptr, FRACSOLVE_E_ARG, "handle is NULL");
    int rc;
    if ((rc = check_fields(h, (const void *const *)f, "f", true))) return rc;
    if ((rc = check_fields(h, (const void *const *)u, "u", true))) return rc;
    hipEvent_t ev[2];
    if ((rc = timed_begin(h, ev))) return rc;
    rc = solve_all(h, f, u0, phi, u);
    rc = check_outputs(h, (const double *const *)u, "u", rc);
    return timed_end(h, ev, rc);
}

int fracsolve_apply(fracsolve_t h, const double *const *u, double *const *y)
{
    if (!h) return fail(nullptr, FRACSOLVE_E_ARG, "handle is NULL");
    if (h->opts.equation == FRACSOLVE_ADVECTION)
        return fail(h, FRACSOLVE_E_ARG, "not available for the advection equations");
    int rc;
    if ((rc = check_fields(h, (const void *const *)u, "u", true))) return rc;
    if ((rc = check_fields(h, (const void *const *)y, "y", true))) return rc;
    for (size_t k = 0; k < h->inst.size(); ++k)
        if ((const void *)u[k] == (const void *)y[k]) return fail(h, FRACSOLVE_E_ARG, "u[%zu] and y[%zu] alias", k, k);
    hipEvent_t ev[2];
    if ((rc = timed_begin(h, ev))) return rc;
    for (size_t k = 0; k < h->inst.size() && !rc; ++k) rc = apply_op(h, (int)k, u[k], y[k], false, ColPerm{0, 0});
    rc = check_outputs(h, (const double *const *)y, "y", rc);
    return timed_end(h, ev, rc);
}

int fracsolve_adjoint(fracsolve_t h, const double *const *g, const double *const *u, const double *const *u0,
                      const double *const *phi, double *const *dL_df, double *dL_dgamma)
{
    if (!h) return fail(nullptr, FRACSOLVE_E_ARG, "handle is NULL");
    if (h->opts.equation == FRACSOLVE_ADVECTION)
        return fail(h, FRACSOLVE_E_ARG, "not available for the advection equations");
    int rc;
    if ((rc = check_fields(h, (const void *const *)g, "g", true))) return rc;
    if ((rc = check_fields(h, (const void *const *)dL_df, "dL_df", true))) return rc;
    if (dL_dgamma && (rc = check_fields(h, (const void *const *)u, "u", true))) return rc;
    hipEvent_t ev[2];
    if ((rc = timed_begin(h, ev))) return rc;
    const size_t cnt = h->inst.size();
    std::vector<int> sel(cnt);
    std::vector<Field> fld(cnt);
    for (size_t k = 0; k < cnt && !rc; ++k) {
        Inst &in = h->inst[k];
        sel[k] = (int)k;
        if ((rc = ensure(h, &in.W, in.M * in.N))) break;
        // reversed time: lambda~^m = lambda^{N-1-m} solves the same lower-triangular system
        // (and the internal column order of the solve)
        if (launch_permute(h->st, g[k], in.W, in.M, in.N, in.perm, true, true) != hipSuccess) {
            rc = fail(h, FRACSOLVE_E_DEVICE, "launch failed");
            break;
        }
        fld[k] = {in.W, nullptr, nullptr};
    }
    if (!rc) rc = dc_solve(h, sel, fld, FRACSOLVE_FP64);
    for (size_t k = 0; k < cnt && !rc; ++k) {
        Inst &in = h->inst[k];
        if (launch_permute(h->st, in.W, dL_df[k], in.M, in.N, in.perm, false, true) != hipSuccess)
            rc = fail(h, FRACSOLVE_E_DEVICE, "launch failed");
    }
    if (!rc && dL_dgamma) {
        for (size_t k = 0; k < cnt && !rc; ++k) {
            Inst &in = h->inst[k];
            if ((rc = ensure(h, &in.V, in.M * in.N))) break;
            // V = (dA/dgamma) U
            if ((rc = apply_op(h, (int)k, u[k], in.V, true, ColPerm{0, 0}))) break;
            double t1 = 0.0, t2 = 0.0;
            HIPCHK(h, launch_dot_partial(h->st, dL_df[k], in.V, in.M * in.N, h->partial, kRedBlocks));
            if ((rc = finish_sum(h, kRedBlocks, &t1))) break;
            const double *ph = (in.regime == 1) ? opt_ptr(phi, k) : nullptr;
            HIPCHK(h, launch_gamma_rhs_terms(h->st, dL_df[k], opt_ptr(u0, k), ph, in.drho, in.dpsi, in.M, in.N,
                                             h->partial, kRedBlocks));
            if ((rc = finish_sum(h, kRedBlocks, &t2))) break;
            dL_dgamma[k] = t2 - t1;
            if (h->check && !std::isfinite(dL_dgamma[k]))
                rc = fail(h, FRACSOLVE_E_NUMERIC, "dL_dgamma[%zu] is not finite", k);
        }
    }
    rc = check_outputs(h, (const double *const *)dL_df, "dL_df", rc);
    return timed_end(h, ev, rc);
}

int fracsolve_gmres(fracsolve_t h, const double *const *f, const double *const *u0, const double *const *phi,
                    double *const *u, const fracsolve_gmres_options *opts, fracsolve_gmres_info *info,
                    double *hist, int32_t hist_cap)
{
    if (!h) return fail(nullptr, FRACSOLVE_E_ARG, "handle is NULL");
    if (h->opts.equation == FRACSOLVE_ADVECTION)
        return fail(h, FRACSOLVE_E_ARG, "not available for the advection equations");
    int rc;
    if ((rc = check_fields(h, (const void *const *)f, "f", true))) return rc;
    if ((rc = check_fields(h, (const void *const *)u, "u", true))) return rc;
    fracsolve_gmres_options o{30, 1000, 1e-10, 0, 0};
    if (opts) o = *opts;
    if (o.restart < 1 || o.restart > 512)
        return fail(h, FRACSOLVE_E_ARG, "restart must lie in [1, 512], got %d", (int)o.restart);
    if (o.max_iters < 0) return fail(h, FRACSOLVE_E_ARG, "max_iters must be >= 0, got %d", (int)o.max_iters);
    if (!(o.rtol >= 0.0) || !std::isfinite(o.rtol))
        return fail(h, FRACSOLVE_E_ARG, "rtol must be finite and >= 0, got %g", o.rtol);
    if (o.precond < 0 || o.precond > 1)
        return fail(h, FRACSOLVE_E_ARG, "precond must be 0 or 1, got %d", (int)o.precond);
    if (o.use_guess < 0 || o.use_guess > 1)
        return fail(h, FRACSOLVE_E_ARG, "use_guess must be 0 or 1, got %d", (int)o.use_guess);
    if (hist_cap < 0 || (hist_cap > 0 && !hist))
        return fail(h, FRACSOLVE_E_ARG, "hist is NULL with hist_cap %d", (int)hist_cap);
    hipEvent_t ev[2];
    if ((rc = timed_begin(h, ev))) return rc;
    if (!h->zeros) {
        if ((rc = dalloc(h, &h->zeros, 64))) return timed_end(h, ev, rc);
        if (launch_zero(h->st, h->zeros, 64 * sizeof(double)) != hipSuccess)
            return timed_end(h, ev, fail(h, FRACSOLVE_E_DEVICE, "launch failed"));
    }
    if (h->gcap < o.restart + 1) {
        dfree(h, h->gpart);
        dfree(h, h->gdots);
        h->gpart = h->gdots = nullptr;
        h->gcap = 0;
        if ((rc = dalloc(h, &h->gpart, (size_t)(o.restart + 1) * kDotBlocks)) ||
            (rc = dalloc(h, &h->gdots, (size_t)(o.restart + 1))))
            return timed_end(h, ev, rc);
        h->gcap = o.restart + 1;
    }
    for (size_t k = 0; k < h->inst.size() && !rc; ++k) {
        GmresResult r;
        rc = gmres_one(h, (int)k, f[k], opt_ptr(u0, k), opt_ptr(phi, k), u[k], o, r, k == 0 ? hist : nullptr,
                       k == 0 ? hist_cap : 0);
        if (!rc && info) info[k] = fracsolve_gmres_info{r.iters, r.cycles, r.converged, 0, r.relres, r.est};
    }
    return timed_end(h, ev, rc);
}

int fracsolve_set_timing(fracsolve_t h, int32_t on)
{
    if (!h) return fail(nullptr, FRACSOLVE_E_ARG, "handle is NULL");
    h->timing = on;
    return FRACSOLVE_OK;
}

int fracsolve_set_check(fracsolve_t h, int32_t on)
{
    if (!h) return fail(nullptr, FRACSOLVE_E_ARG, "handle is NULL");
    h->check = on ? 1 : 0;
    return FRACSOLVE_OK;
}

int fracsolve_get_stats(fracsolve_t h, fracsolve_stats *out)
{
    if (!h || !out) return fail(h, FRACSOLVE_E_ARG, "NULL argument");
    *out = h->stats;
    return FRACSOLVE_OK;
}

int fracsolve_kernel_stats(fracsolve_t h, fracsolve_kernel_stat *out, int32_t cap, int32_t *count)
{
    if (!h || !count || (cap > 0 && !out)) return fail(h, FRACSOLVE_E_ARG, "NULL argument");
    int32_t n = (int32_t)h->kstats.size();
    for (int32_t k = 0; k < n && k < cap; ++k) out[k] = h->kstats[k];
    *count = n;
    return FRACSOLVE_OK;
}

void fracsolve_destroy(fracsolve_t h)
{
    if (!h) return;
    hipStreamSynchronize(h->st);
    if (h->gst) hipStreamSynchronize(h->gst);
    for (hipEvent_t e : h->evpool) hipEventDestroy(e);
    h->evpool.clear();
    free_all(h);
    delete h;
}

const char *fracsolve_last_error(fracsolve_t h)
{
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
