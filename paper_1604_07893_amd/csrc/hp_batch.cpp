// Batched and served forms of the hyperpower iteration.
//
// A group holds problems of uneven shapes, each with its own workspace and
// its own host-side loop state. One group loop runs, for every product of the
// loop of (PM) (Section 2) -- and of (PM-modified) (Section 7) for problems
// past the switch -- a single persistent grouped MFMA launch over all
// unfinished problems, then one fixed-order reduction per problem, one copy of
// all stopping sums to the host and each problem's own stop/switch/stage
// decision. Per-tile arithmetic never depends on the other entries of a
// table, so a problem's result is the same alone or in any mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "hp_host.h"
#include "hp_sched.h"

namespace hp {

// fixed-order per-problem sum of partial pairs (hp_kernels.hip)
struct ReduceEntry {
    const double* partials;
    int npairs;
    int pad;
};
// grid >= *count blocks; blocks past *count exit at once
hipError_t reduce_pairs_grouped(const int* count, const ReduceEntry* ents, int grid, double* out,
                                hipStream_t s);
// Adds one to *counter (device memory) and writes the new value to *flag
// (pinned host memory, device address) after everything before it on the
// stream: the host polls it for the end of a grouped loop (hp_kernels.hip).
hipError_t signal_host(unsigned long long* counter, double* flag, hipStream_t s);

}  // namespace hp

namespace {

using namespace hp;
using Clock = std::chrono::steady_clock;

inline double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kSlots = 9;  // products per loop at most (7 plain + 2 stabilising)

struct Problem {
    hp_problem pr{};
    hp_params prm{};      // the group's parameters (FP64 only on a retry)
    bool retried = false;
    Plan pl;
    Buffers bf;
    char* ws = nullptr;
    size_t ws_off = 0, ws_bytes = 0;  // arena placement (server)
    LoopState st;
    hp_result res{};
    int last_tiles = 0;
    bool finished = false;
    Clock::time_point t_submit, t_admit, t_finish;
};

// Device tables of a group: for every product slot and precision a header
// and up to `cap` entries, then the reduction table and its output; mirrored
// by a pinned host staging area that is copied over once per loop.
struct Tables {
    int cap = 0;
    size_t bytes = 0;
    size_t off_hdr[2][kSlots] = {};
    size_t off_ent[2][kSlots] = {};
    size_t off_cnt = 0, off_red = 0, off_out = 0, off_sig = 0;
    char* dev = nullptr;
    char* host = nullptr;

    static size_t layout(int cap, Tables* t) {
        size_t off = 0;
        for (int prec = 0; prec < 2; ++prec) {
            const size_t esz = prec == 0 ? sizeof(GroupEntry<double>) : sizeof(GroupEntry<float>);
            for (int j = 0; j < kSlots; ++j) {
                if (t) t->off_hdr[prec][j] = off;
                off = align_up(off + sizeof(GroupHeader));
                if (t) t->off_ent[prec][j] = off;
                off = align_up(off + esz * (size_t)cap);
            }
        }
        if (t) t->off_cnt = off;
        off = align_up(off + sizeof(int));
        if (t) t->off_red = off;
        off = align_up(off + sizeof(ReduceEntry) * (size_t)cap);
        if (t) t->off_out = off;
        off = align_up(off + 2 * sizeof(double) * (size_t)cap);
        if (t) t->off_sig = off;  // loops signalled so far (device counter)
        off = align_up(off + sizeof(unsigned long long));
        return off;
    }
};

// One captured loop: the launches of the non-empty (precision, slot) tables
// named by `mask` (bit prec * kSlots + slot).
struct LoopGraph {
    uint32_t mask = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};

struct Group {
    hp_handle* h = nullptr;
    hp_params prm{};
    hipStream_t s = nullptr;
    Tables tb;
    int grid = 1024;  // persistent grid of the grouped launches
    int tile_cfg[2] = {GTILE_64, GTILE_64};  // grouped tile per precision (FP64, FP32)
    // One loop's device work -- table upload, a grouped launch per non-empty
    // (precision, product slot) table, the per-problem reduction and the
    // download of the sums -- captured as a hipGraph per set of non-empty
    // tables and replayed (every launch has a fixed grid and reads its sizes
    // from the uploaded tables). No memset nodes.
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;  // capture needs a stream other than the null stream
    static constexpr int kGraphs = 6;  // cached sets; the least recently used goes first
    LoopGraph graphs[kGraphs];
    uint64_t clock = 0;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;  // order the replay against stream s
    // The per-problem sums land in fine-grained pinned host memory (2 per
    // problem, then the loop number): the reduction writes them and a signal
    // kernel the number, which the host polls instead of a copy and a stream
    // wait. Null when that memory is unavailable (copy and wait instead).
    double* sums = nullptr;
    double* sums_dev = nullptr;
    uint64_t signals = 0;
};

// Enqueue one loop's device work on stream s (used eagerly or under capture).
int enqueue_loop(Group& g, uint32_t mask, hipStream_t s) {
    Tables& tb = g.tb;
    HIPCHK(hipMemcpyAsync(tb.dev, tb.host, tb.off_out, hipMemcpyHostToDevice, s));
    for (int j = 0; j < kSlots; ++j) {
        if (mask >> j & 1u)
            HIPCHK(gemm_grouped(reinterpret_cast<const GroupHeader*>(tb.dev + tb.off_hdr[0][j]),
                                reinterpret_cast<const GroupEntry<double>*>(tb.dev + tb.off_ent[0][j]),
                                g.grid, g.tile_cfg[0], s));
        if (mask >> (kSlots + j) & 1u)
            HIPCHK(gemm_grouped(reinterpret_cast<const GroupHeader*>(tb.dev + tb.off_hdr[1][j]),
                                reinterpret_cast<const GroupEntry<float>*>(tb.dev + tb.off_ent[1][j]),
                                g.grid, g.tile_cfg[1], s));
    }
    if (g.sums_dev) {
        HIPCHK(reduce_pairs_grouped(reinterpret_cast<const int*>(tb.dev + tb.off_cnt),
                                    reinterpret_cast<const ReduceEntry*>(tb.dev + tb.off_red),
                                    tb.cap, g.sums_dev, s));
        HIPCHK(signal_host(reinterpret_cast<unsigned long long*>(tb.dev + tb.off_sig),
                           g.sums_dev + 2 * tb.cap, s));
        return HP_OK;
    }
    HIPCHK(reduce_pairs_grouped(reinterpret_cast<const int*>(tb.dev + tb.off_cnt),
                                reinterpret_cast<const ReduceEntry*>(tb.dev + tb.off_red), tb.cap,
                                reinterpret_cast<double*>(tb.dev + tb.off_out), s));
    HIPCHK(hipMemcpyAsync(tb.host + tb.off_out, tb.dev + tb.off_out, 2 * sizeof(double) * (size_t)tb.cap,
                          hipMemcpyDeviceToHost, s));
    return HP_OK;
}

void drop_graph(LoopGraph& lg) {
    if (lg.exec) (void)hipGraphExecDestroy(lg.exec);
    if (lg.graph) (void)hipGraphDestroy(lg.graph);
    lg = LoopGraph{};
}

int run_loop_device(Group& g, uint32_t mask) {
    if (!g.use_graph) return enqueue_loop(g, mask, g.s);
    LoopGraph* lg = nullptr;
    for (LoopGraph& c : g.graphs)
        if (c.exec && c.mask == mask) lg = &c;
    if (!lg) {
        if (!g.cap_stream) HIPCHK(hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking));
        if (!g.ev_in) HIPCHK(hipEventCreateWithFlags(&g.ev_in, hipEventDisableTiming));
        if (!g.ev_out) HIPCHK(hipEventCreateWithFlags(&g.ev_out, hipEventDisableTiming));
        lg = &g.graphs[0];
        for (LoopGraph& c : g.graphs)
            if (!c.exec || c.used < lg->used) lg = &c;
        if (lg->exec) {
            // a replay of the evicted graph may still be running
            HIPCHK(hipStreamSynchronize(g.cap_stream));
            drop_graph(*lg);
        }
        HIPCHK(hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_loop(g, mask, g.cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(g.cap_stream, &graph);
        if (rc != HP_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc != HP_OK ? rc : HP_EHIP;
        }
        lg->graph = graph;
        if (hipGraphInstantiate(&lg->exec, lg->graph, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(*lg);
            return HP_EHIP;
        }
        lg->mask = mask;
    }
    lg->used = ++g.clock;
    // the graph runs on the capture stream, ordered after the group stream's work
    HIPCHK(hipEventRecord(g.ev_in, g.s));
    HIPCHK(hipStreamWaitEvent(g.cap_stream, g.ev_in, 0));
    HIPCHK(hipGraphLaunch(lg->exec, g.cap_stream));
    HIPCHK(hipEventRecord(g.ev_out, g.cap_stream));
    HIPCHK(hipStreamWaitEvent(g.s, g.ev_out, 0));
    return HP_OK;
}

void group_release(Group& g) {
    if (g.cap_stream) (void)hipStreamSynchronize(g.cap_stream);
    if (g.s) (void)hipStreamSynchronize(g.s);
    if (g.sums) (void)hipHostFree(g.sums);
    g.sums = g.sums_dev = nullptr;
    if (g.ev_in) (void)hipEventDestroy(g.ev_in);
    if (g.ev_out) (void)hipEventDestroy(g.ev_out);
    g.ev_in = g.ev_out = nullptr;
    for (LoopGraph& c : g.graphs) drop_graph(c);
    if (g.cap_stream) (void)hipStreamDestroy(g.cap_stream);
    g.cap_stream = nullptr;
}

void group_init(Group& g, hp_handle* h, const hp_params* p, void* stream) {
    g.h = h;
    g.prm = *p;
    g.s = reinterpret_cast<hipStream_t>(stream);
    g.use_graph = (p->flags & HP_FLAG_NO_GRAPH) == 0;
    for (int i = 0; i < 2; ++i) g.tile_cfg[i] = h->grouped_cfg[i];
}

// Once the tables exist: the host area for the sums and a zero loop counter
// (a plain memset: no graph is being captured yet).
int group_sums_init(Group& g) {
    const size_t bytes = sizeof(double) * (2 * (size_t)g.tb.cap + 1);
    if (hipHostMalloc(reinterpret_cast<void**>(&g.sums), bytes,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        g.sums = nullptr;
        return HP_OK;  // copy and wait instead
    }
    std::memset(g.sums, 0, bytes);
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&g.sums_dev), g.sums, 0) != hipSuccess) {
        (void)hipHostFree(g.sums);
        g.sums = g.sums_dev = nullptr;
        return HP_OK;
    }
    g.signals = 0;
    HIPCHK(hipMemsetAsync(g.tb.dev + g.tb.off_sig, 0, sizeof(unsigned long long), g.s));
    return HP_OK;
}

// Products outside the loop (Drazin set-up, projection) run as single
// launches on the problem's own shapes.
auto single_gemm(Group& g, Problem& P) {
    return [&g, &P](const GemmCall<double>& c) {
        if (!c.A || !c.B || !c.ep.out[0]) return HP_EINVAL;
        const GemmTile t = choose_tile(g.h, HP_DTYPE_F64, c.M, c.N, c.K);
        if (hp::gemm(t, c.M, c.N, c.K, c.A, c.lda, c.B, c.ldb, c.ep, g.s) != hipSuccess) return HP_EHIP;
        const double gf = 2.0 * (double)c.M * (double)c.N * (double)c.K * 1e-9;
        P.res.gflop += gf;
        P.res.gflop_stage[2] += gf;
        P.res.gemms += 1;
        return HP_OK;
    };
}

int admit_setup(Group& g, Problem& P) {
    P.bf = carve(P.pl, P.ws);
    std::memset(&P.res, 0, sizeof(P.res));
    P.res.switch_iter = -1;
    P.res.side_used = P.pl.left ? HP_SIDE_LEFT : HP_SIDE_RIGHT;
    double alpha = 0.0;
    CHK(setup_x0(&P.prm, P.pl, P.bf, P.pr.A, P.pr.lda, P.pr.X0, P.pr.ldx0, g.h->host_scal, g.s,
                 single_gemm(g, P), &alpha));
    P.res.alpha = alpha;
    P.st.init(&P.prm, &P.res, alpha);
    if (P.st.stage < 2) {
        HIPCHK(convert(P.bf.b64.A, P.bf.b64.ldA, P.pl.m, P.pl.n, P.bf.b32.A, P.bf.b32.ldA, g.s));
        HIPCHK(convert(P.bf.b64.X[0], P.bf.b64.ldX, P.pl.n, P.pl.m, P.bf.b32.X[0], P.bf.b32.ldX, g.s));
    }
    return HP_OK;
}

// Set a problem up from its X0. On failure it is finished with that error
// (so neither a loop nor a poll sees a half-initialised state).
int admit(Group& g, Problem& P) {
    const int rc = admit_setup(g, P);
    if (rc != HP_OK) {
        P.res.status = rc;
        P.finished = true;
        return rc;
    }
    P.finished = false;
    return HP_OK;
}

template <typename T>
void append(Tables& tb, int prec, int slot, int cfg, const GemmCall<T>& c, int* tiles_out) {
    GroupHeader* hdr = reinterpret_cast<GroupHeader*>(tb.host + tb.off_hdr[prec][slot]);
    GroupEntry<T>* ents = reinterpret_cast<GroupEntry<T>*>(tb.host + tb.off_ent[prec][slot]);
    const int dim = grouped_tile_dim(cfg);
    const int tn = (int)cdiv(c.N, dim), tm = (int)cdiv(c.M, dim);
    GroupEntry<T>& e = ents[hdr->count];
    e.M = (int)c.M;
    e.N = (int)c.N;
    e.K = (int)c.K;
    e.tiles_n = tn;
    e.tile_start = hdr->total_tiles;
    e.pad = 0;
    e.A = c.A;
    e.lda = c.lda;
    e.B = c.B;
    e.ldb = c.ldb;
    e.ep = c.ep;
    hdr->count += 1;
    hdr->total_tiles += tm * tn;
    *tiles_out = tm * tn;
}

// Retire a finished problem: write X (FP64) and stamp it.
int retire(Group& g, Problem& P) {
    LoopState& st = P.st;
    st.finish_maxiter();
    const int64_t m = P.pl.m, n = P.pl.n;
    if (st.stage == 2) {
        HIPCHK(hipMemcpy2DAsync(P.pr.X, P.pr.ldx * sizeof(double), P.bf.b64.X[st.result_idx],
                                P.bf.b64.ldX * sizeof(double), m * sizeof(double), n,
                                hipMemcpyDeviceToDevice, g.s));
    } else {
        HIPCHK(convert(P.bf.b32.X[st.result_idx], P.bf.b32.ldX, n, m, P.pr.X, P.pr.ldx, g.s));
    }
    P.res.status = st.status;
    P.finished = true;
    return HP_OK;
}

// One loop of every problem in `act` (all admitted, none finished). Problems
// that finish are retired (X written, stream synchronised before return).
int group_loop(Group& g, std::vector<Problem*>& act) {
    Range range("grouped loop, %d problems", (int)act.size());
    Tables& tb = g.tb;
    std::memset(tb.host, 0, tb.off_red);
    const int np = (int)act.size();
    *reinterpret_cast<int*>(tb.host + tb.off_cnt) = np;
    ReduceEntry* red = reinterpret_cast<ReduceEntry*>(tb.host + tb.off_red);
    uint32_t mask = 0;  // the non-empty (precision, slot) tables
    for (int i = 0; i < np; ++i) {
        Problem& P = *act[i];
        LoopState& st = P.st;
        int tiles = 0;
        if (st.stage == 2) {
            GemmCall<double> calls[kMaxLoopGemms];
            const int nc = describe_loop<double>(HP_METHOD_PM, P.pl, P.bf.b64, P.bf.b64.X[st.ik],
                                                    P.bf.b64.X[st.in_], P.bf.b64.X[2],
                                                    st.stabilising, P.bf.small, calls);
            if (nc > kSlots) return HP_EUNSUPPORTED;
            for (int j = 0; j < nc; ++j) {
                if (!calls[j].A || !calls[j].B || !calls[j].ep.out[0]) return HP_EINVAL;
                append(tb, 0, j, g.tile_cfg[0], calls[j], &tiles);
                mask |= 1u << j;
                const double gf = 2.0 * (double)calls[j].M * calls[j].N * calls[j].K * 1e-9;
                P.res.gflop += gf;
                P.res.gflop_stage[2] += gf;
            }
            P.res.gemms += nc;
        } else {
            if (st.engine() != ENG_F32) return HP_EUNSUPPORTED;
            GemmCall<float> calls[kMaxLoopGemms];
            const int nc = describe_loop<float>(HP_METHOD_PM, P.pl, P.bf.b32, P.bf.b32.X[st.ik],
                                                   P.bf.b32.X[st.in_], P.bf.b32.X[2],
                                                   st.stabilising, P.bf.small, calls);
            if (nc > kSlots) return HP_EUNSUPPORTED;
            for (int j = 0; j < nc; ++j) {
                if (!calls[j].A || !calls[j].B || !calls[j].ep.out[0]) return HP_EINVAL;
                append(tb, 1, j, g.tile_cfg[1], calls[j], &tiles);
                mask |= 1u << (kSlots + j);
                const double gf = 2.0 * (double)calls[j].M * calls[j].N * calls[j].K * 1e-9;
                P.res.gflop += gf;
                P.res.gflop_stage[st.stage] += gf;
            }
            P.res.gemms += nc;
        }
        P.last_tiles = tiles;
        red[i] = ReduceEntry{P.bf.small, tiles, 0};
    }
    CHK(run_loop_device(g, mask));
    const double* hout = reinterpret_cast<const double*>(tb.host + tb.off_out);
    if (g.sums) {
        // a grouped loop takes from tens of microseconds to tens of
        // milliseconds: poll for its signal, then wait for the stream
        const double want = (double)++g.signals;
        if (!poll_host(g.sums + 2 * tb.cap, want, 20000.0)) HIPCHK(hipStreamSynchronize(g.s));
        hout = g.sums;
    } else {
        HIPCHK(hipStreamSynchronize(g.s));
    }

    bool any_done = false;
    for (int i = 0; i < np; ++i) {
        Problem& P = *act[i];
        LoopState& st = P.st;
        const LoopState::Action a = st.step(hout[2 * i], hout[2 * i + 1], 0.0, false);
        if (a == LoopState::CONTINUE && st.projection_due() && P.pl.has_proj) {
            CHK(project_mp(P.pl, P.bf, st.ik, g.s, single_gemm(g, P)));
            st.projected();
        }
        if (a == LoopState::NEXT_STAGE) {
            const int next = st.stage + 1;
            if (next == 2) {
                HIPCHK(convert(P.bf.b32.X[st.from_idx], P.bf.b32.ldX, P.pl.n, P.pl.m,
                               P.bf.b64.X[0], P.bf.b64.ldX, g.s));
                bool proj = false;
                CHK(needs_projection(P.pl, P.bf, g.h->host_scal, g.s, &proj));
                if (proj && st.exit_converged) CHK(project_mp(P.pl, P.bf, 0, g.s, single_gemm(g, P)));
                else if (proj) st.proj_pending = true;
            }
            st.enter_stage(next);
        }
        if (a == LoopState::DONE || st.k >= P.prm.max_iter) {
            CHK(retire(g, P));
            any_done = true;
        }
    }
    if (any_done) HIPCHK(hipStreamSynchronize(g.s));
    const Clock::time_point now = Clock::now();
    for (Problem* P : act)
        if (P->finished) P->t_finish = now;
    return HP_OK;
}

int validate_group_params(const hp_params* p) {
    if (p->precision != HP_PREC_FP64 && p->precision != HP_PREC_FP32 &&
        p->precision != HP_PREC_FP32_FP64)
        return HP_EUNSUPPORTED;
    if (p->stop_rule == HP_STOP_ABS_INF || (p->flags & HP_FLAG_INF_NORM)) return HP_EUNSUPPORTED;
    if (p->method != HP_METHOD_PM || p->stop_rule == HP_STOP_REL_FRO_BOUND) return HP_EUNSUPPORTED;
    if (p->chop > 0.0 || p->alpha_rule == HP_ALPHA_DIAG) return HP_EUNSUPPORTED;
    return HP_OK;
}

int validate_problem(const hp_params* p, const hp_problem& pr) {
    CHK(validate(p, pr.m, pr.n));
    if (!pr.A || !pr.X) return HP_EINVAL;
    if (pr.lda < pr.n || pr.ldx < pr.m || (pr.X0 && pr.ldx0 < pr.m)) return HP_EINVAL;
    return HP_OK;
}

int tables_alloc(Tables& tb, int cap) {
    tb.cap = cap;
    tb.bytes = Tables::layout(cap, &tb);
    if (hipMalloc(reinterpret_cast<void**>(&tb.dev), tb.bytes) != hipSuccess) return HP_EHIP;
    if (hipHostMalloc(reinterpret_cast<void**>(&tb.host), tb.bytes, hipHostMallocDefault) != hipSuccess)
        return HP_EHIP;
    return HP_OK;
}

void tables_free(Tables& tb) {
    if (tb.dev) (void)hipFree(tb.dev);
    if (tb.host) (void)hipHostFree(tb.host);
    tb.dev = tb.host = nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
// Server
// ---------------------------------------------------------------------------

struct hp_server {
    Group g;
    char* arena = nullptr;
    size_t budget = 0;
    Admission adm;
    uint64_t next_ticket = 1;
    std::map<uint64_t, Problem> reqs;
};

extern "C" {

int hp_batched_workspace_bytes(const hp_params* p, int count, const hp_problem* probs, size_t* bytes) {
    if (!p || !bytes || count < 1 || !probs) return HP_EINVAL;
    CHK(validate_group_params(p));
    size_t total = Tables::layout(count, nullptr);
    for (int i = 0; i < count; ++i) {
        CHK(validate(p, probs[i].m, probs[i].n));
        total += align_up(make_plan(p, probs[i].m, probs[i].n, false).total);
    }
    *bytes = total;
    return HP_OK;
}

int hp_solve_batched(hp_handle* h, const hp_params* p, int count, const hp_problem* probs,
                     void* workspace, size_t ws_bytes, void* stream, hp_result* outs) {
    const Clock::time_point t0 = Clock::now();
    if (!h || !p || count < 1 || !probs) return HP_EINVAL;
    CHK(validate_group_params(p));
    for (int i = 0; i < count; ++i) CHK(validate_problem(p, probs[i]));
    Range range("hp_solve_batched %d problems", count);
    size_t need = 0;
    CHK(hp_batched_workspace_bytes(p, count, probs, &need));
    if (!workspace || ws_bytes < need) return HP_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return HP_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;

    Group g;
    group_init(g, h, p, stream);
    char* ws = static_cast<char*>(workspace);
    // the tables live at the start of the workspace; staging is pinned host memory
    g.tb.cap = count;
    g.tb.bytes = Tables::layout(count, &g.tb);
    g.tb.dev = ws;
    if (hipHostMalloc(reinterpret_cast<void**>(&g.tb.host), g.tb.bytes, hipHostMallocDefault) != hipSuccess)
        return HP_EHIP;
    if (group_sums_init(g) != HP_OK) {
        (void)hipHostFree(g.tb.host);
        return HP_EHIP;
    }
    std::vector<Problem> P(count);
    size_t off = align_up(g.tb.bytes);
    int rc = HP_OK;
    for (int i = 0; i < count && rc == HP_OK; ++i) {
        P[i].pr = probs[i];
        P[i].prm = *p;
        P[i].pl = make_plan(p, probs[i].m, probs[i].n, false);
        P[i].ws = ws + off;
        off += align_up(P[i].pl.total);
        rc = admit(g, P[i]);
    }
    std::vector<Problem*> act;
    for (auto& q : P) act.push_back(&q);
    while (rc == HP_OK && !act.empty()) {
        rc = group_loop(g, act);
        act.erase(std::remove_if(act.begin(), act.end(), [](Problem* q) { return q->finished; }),
                  act.end());
    }
    group_release(g);
    (void)hipHostFree(g.tb.host);
    if (rc != HP_OK) return rc;
    const double wall = ms_between(t0, Clock::now());
    if (outs) {
        for (int i = 0; i < count; ++i) {
            P[i].res.time_ms = wall;
            outs[i] = P[i].res;
        }
    }
    return HP_OK;
}

int hp_serve_create(hp_handle* h, const hp_params* p, size_t hbm_budget, int max_slots,
                    void* stream, hp_server** out) {
    if (!h || !p || !out || max_slots < 1 || hbm_budget < kAlign) return HP_EINVAL;
    *out = nullptr;
    CHK(validate_group_params(p));
    CHK(validate(p, 1, 1));
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
    hp_server* sv = new hp_server();
    group_init(sv->g, h, p, stream);
    sv->budget = hbm_budget / kAlign * kAlign;
    sv->adm = Admission(sv->budget, max_slots);
    if (hipMalloc(reinterpret_cast<void**>(&sv->arena), sv->budget) != hipSuccess) {
        delete sv;
        return HP_EHIP;
    }
    if (tables_alloc(sv->g.tb, max_slots) != HP_OK || group_sums_init(sv->g) != HP_OK) {
        group_release(sv->g);
        (void)hipFree(sv->arena);
        tables_free(sv->g.tb);
        delete sv;
        return HP_EHIP;
    }
    *out = sv;
    return HP_OK;
}

int hp_serve_submit(hp_server* sv, const hp_problem* prob, uint64_t* ticket) {
    if (!sv || !prob || !ticket) return HP_EINVAL;
    CHK(validate_problem(&sv->g.prm, *prob));
    const Plan pl = make_plan(&sv->g.prm, prob->m, prob->n, false);
    if (align_up(pl.total) > sv->budget) return HP_EBUDGET;
    const uint64_t t = sv->next_ticket++;
    Problem& P = sv->reqs[t];
    P.pr = *prob;
    P.prm = sv->g.prm;
    P.pl = pl;
    P.ws_bytes = align_up(pl.total);
    P.t_submit = Clock::now();
    sv->adm.submit(t, P.ws_bytes);
    *ticket = t;
    return HP_OK;
}

int hp_serve_step(hp_server* sv, int* active, int* waiting) {
    if (!sv) return HP_EINVAL;
    Range range("hp_serve_step");
    if (hipSetDevice(sv->g.h->device) != hipSuccess) return HP_EHIP;
    // the GPU side of serve_step (hp_sched.h, which holds the bookkeeping)
    struct Exec {
        hp_server* sv;
        Problem& req(uint64_t t) { return sv->reqs[t]; }
        int enter(uint64_t t, size_t off) {
            Problem& P = req(t);
            P.ws_off = off;
            P.ws = sv->arena + off;
            P.t_admit = Clock::now();
            return admit(sv->g, P);
        }
        int run(const std::vector<uint64_t>& ts) {
            std::vector<Problem*> act;
            for (uint64_t t : ts) act.push_back(&req(t));
            return group_loop(sv->g, act);
        }
        bool finished(uint64_t t) { return req(t).finished; }
        // the lower precisions failed: once more from X0, FP64 only, in the
        // same arena space (the FP64 plan needs less of it)
        bool wants_retry(uint64_t t) {
            Problem& P = req(t);
            if (P.res.status == HP_OK || P.retried || P.prm.precision == HP_PREC_FP64 ||
                (sv->g.prm.flags & HP_FLAG_NO_RETRY))
                return false;
            hp_params q = P.prm;
            q.precision = HP_PREC_FP64;
            return align_up(make_plan(&q, P.pr.m, P.pr.n, false).total) <= P.ws_bytes;
        }
        int reenter(uint64_t t) {
            Problem& P = req(t);
            P.retried = true;
            P.prm.precision = HP_PREC_FP64;
            P.pl = make_plan(&P.prm, P.pr.m, P.pr.n, false);
            return admit(sv->g, P);
        }
        void fail(uint64_t t, int rc) {
            Problem& P = req(t);
            P.res.status = rc;
            P.finished = true;
            P.t_finish = Clock::now();
        }
        void settle(uint64_t t) {
            Problem& P = req(t);
            P.res.queue_ms = ms_between(P.t_submit, P.t_admit);
            P.res.run_ms = ms_between(P.t_admit, P.t_finish);
            P.res.time_ms = ms_between(P.t_submit, P.t_finish);
            P.ws = nullptr;
        }
    } ex{sv};
    const int rc = serve_step(sv->adm, ex);
    if (active) *active = (int)sv->adm.active_count();
    if (waiting) *waiting = (int)sv->adm.waiting();
    return rc;
}

int hp_serve_poll(hp_server* sv, uint64_t ticket, hp_result* out) {
    if (!sv) return HP_EINVAL;
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return HP_EINVAL;
    if (!it->second.finished) return HP_PENDING;
    const int st = it->second.res.status;
    if (out) *out = it->second.res;
    sv->reqs.erase(it);
    return st;
}

int hp_serve_destroy(hp_server* sv) {
    if (!sv) return HP_EINVAL;
    (void)hipSetDevice(sv->g.h->device);
    (void)hipStreamSynchronize(sv->g.s);
    group_release(sv->g);
    if (sv->arena) (void)hipFree(sv->arena);
    tables_free(sv->g.tb);
    delete sv;
    return HP_OK;
}

}  // extern "C"
