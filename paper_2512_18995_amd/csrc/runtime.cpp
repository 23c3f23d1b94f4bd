// runtime.cpp -- host side of libdq: argument validation, the planner that
// turns a gate list into register-tile passes, matrix slots, lazy device
// upload of the plan tables, and the C ABI of include/dq.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <optional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dq.h"
#include "dq_internal.h"

// Device scratch of dq_apply_circuit_noalloc: the per-sample gate-matrix
// blocks live here instead of in a caller's workspace.  Each device that the
// library runs on holds one copy until the process ends.  Host code never
// uses this name as an address: it takes the device address from
// hipGetSymbolAddress once per device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[DQ_NOALLOC_SCRATCH_BYTES];

using namespace dq;

// ================================================================ errors
namespace {
thread_local std::string g_err;

dq_status fail(dq_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
dq_status ok() {
    g_err.clear();
    return DQ_OK;
}
// No C++ exception crosses the C ABI: every entry point is a function-try-
// block whose handler turns a host-side failure (std::bad_alloc from a plan's
// tables, a missing map entry, ...) into DQ_ERR_INTERNAL and dq_last_error().
dq_status fail_nothrow(const char *what) noexcept {
    try {
        g_err.assign(what);
    } catch (...) {
        g_err.clear();
    }
    return DQ_ERR_INTERNAL;
}
#define DQ_CATCH                                                                            \
    catch (const std::bad_alloc &) {                                                        \
        return fail_nothrow("host memory allocation failed");                               \
    }                                                                                       \
    catch (const std::exception &e_) {                                                      \
        return fail_nothrow(e_.what());                                                     \
    }                                                                                       \
    catch (...) {                                                                           \
        return fail_nothrow("unexpected C++ exception");                                    \
    }
#define DQ_CATCH_VOID \
    catch (...) {     \
    }
#define DQ_HIP(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(DQ_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool is_rotation(int op) {
    return op == OP_RX || op == OP_RY || op == OP_RZ || op == OP_CP || op == OP_RZZ || op == OP_RXX || op == OP_RYY ||
           op == OP_U3 || op == OP_CRX || op == OP_CRY || op == OP_CRZ || op == OP_PHASE;
}
int arity(int op) {
    switch (op) {
    case OP_CNOT: case OP_CZ: case OP_SWAP: case OP_CP: case OP_RZZ: case OP_RXX: case OP_RYY:
    case OP_CRX: case OP_CRY: case OP_CRZ: return 2;
    case OP_UNITARY: return -1;
    default: return 1;
    }
}
bool is_diag1(int op) { return op == OP_RZ || op == OP_Z || op == OP_PHASE; }
int gen_of(int op) {
    switch (op) {
    case OP_RX: return GEN_X;
    case OP_RY: return GEN_Y;
    // diag(1, e^{it}) = e^{it/2} RZ(t): dE/dt = Im<l|Z|p> - Im<l|p>, and <l|p> =
    // sum_o w_o <psi|H_o|psi> is real, so the phase gate takes RZ's generator
    case OP_RZ: case OP_PHASE: return GEN_Z;
    case OP_RZZ: return GEN_ZZ;
    case OP_CP: return GEN_P11;
    default: return GEN_NONE;
    }
}
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
struct dq_plan_s;
namespace {
hipEvent_t prof_event(dq_plan_s &p);
void prof_push(dq_plan_s &p, int kind, int nl, hipEvent_t a, hipEvent_t b, double bytes, double flops);
bool prof_on(const dq_plan_s &p);

// Brackets one or more launches with a pair of events when profiling is on.
struct ProfScope {
    dq_plan_s &p;
    int kind, nl;
    double bytes;
    hipStream_t s;
    hipEvent_t a = nullptr;
    double flops = 0;
    // timed = false: no events (the allocation-free entry point creates none)
    ProfScope(dq_plan_s &pl, int k, int nlaunch, double b, hipStream_t st, bool timed = true)
        : p(pl), kind(k), nl(nlaunch), bytes(b), s(st) {
        if (timed && prof_on(p)) {
            a = prof_event(p);
            (void)hipEventRecord(a, s);
        }
    }
    void done() {
        if (a) {
            hipEvent_t b = prof_event(p);
            (void)hipEventRecord(b, s);
            prof_push(p, kind, nl, a, b, bytes, flops);
            a = nullptr;
        }
    }
};

// ================================================================ plan
enum StepKind { ST_TILE = 0, ST_G1, ST_CNOT, ST_CZ, ST_GK, ST_GRAD, ST_DENSE };

struct Step {
    int kind = 0;
    int R = 0;
    int32_t rbits[MAX_TILE_R] = {0};
    int32_t lbits[3] = {0};
    int32_t tbits[MAX_TILE_R + 3] = {0};
    int64_t op0 = 0, nops = 0;      // into plan.ops
    int64_t ls0 = 0, nls = 0;       // into plan.lsg
    int k = 0;
    int32_t bits[5] = {0};          // per-gate: physical bits, bits[0] = matrix MSB / control
    int64_t slot = 0;
    int gen = 0, gslot = -1;
    double flops_per_amp = 0;       // algorithmic flops per amplitude of one state
};

struct Program {
    std::vector<Step> steps;
    // compiled passes (option jit): per step, the index of its kernel in the
    // plan's kernel list (-1: interpreted) and the pass's first matrix slot
    std::vector<int> jk;
    std::vector<int64_t> js0;
    int64_t slot_lo = 0, slot_hi = 0;  // slot index range used (for prepare)
    int64_t blk_lo = 0, blk_hi = 0;    // fused dense block range used
    int64_t tile_passes = 0, dense_steps = 0;
};

struct DevData {
    std::vector<hipFunction_t> jfn;   // compiled passes, in the plan's kernel-list order
    int jit_adj_cap = 0;              // resident waves of the slowest-filling compiled adjoint pass
    void *blob = nullptr;
    DGate *gates = nullptr;
    double2 *fixed = nullptr;
    DSlot *slots = nullptr;
    DBlock *blocks = nullptr;
    int32_t *factors = nullptr;
    TOp *ops = nullptr;
    int32_t *lsg = nullptr;
    int64_t *fold = nullptr;
    int64_t *poff = nullptr, *doff = nullptr;
    int32_t *pg = nullptr, *dg = nullptr;
    double *pf = nullptr, *df = nullptr;
    int32_t *occ_param = nullptr, *hocc = nullptr;   // Hessian: angle occurrences of parameters
    double *occ_scale = nullptr;
    int64_t *hoff = nullptr;
};

}  // namespace

struct dq_plan_s {
    int n = 0;
    int dbl = 0;                        // states in complex128
    int mdbl = 0;                       // gate matrices and tile-pass arithmetic in float64
    dq_options opt{};
    int64_t nparams = 0, ndata = 0;
    std::vector<DGate> gates;
    std::vector<double2> fixed;
    std::vector<DSlot> slots;
    std::vector<DBlock> blocks;         // fused dense blocks (dense_fuse)
    std::vector<int32_t> factors;       // their factor gate lists
    int64_t block = 0;                  // complex elements per sample's matrix block
    std::vector<TOp> ops;
    std::vector<int32_t> lsg;
    Program fwd_full, fwd_fold, adj;
    bool has_fold = false;
    std::vector<std::string> jnames, jsrcs;   // compiled passes: kernel names and sources
    int64_t user_gates = 0;                    // gates given by the caller (the layout may append swaps)
    int64_t entry_gates = 0;                   // last gates of the list: run first, by the forward from a given state only
    int32_t layout_swaps = 0;
    std::vector<int64_t> fold_off;      // per physical bit: slot offset of the folded column, -1 none
    int64_t folded_gates = 0;
    int R_fwd = 0, R_adj = 0;
    int32_t ngrad = 0;
    // the adjoint's gate order and gradient slots, and the sizes of what its
    // planner appends to (slots, ops, lsg, factors, blocks, block), so that
    // it can be planned again
    std::vector<int> adj_rev, adj_gslot;
    std::vector<size_t> adj_mark;
    std::vector<int64_t> poff, doff;
    std::vector<int32_t> pg, dg;
    std::vector<double> pf, df;
    // Hessian (dq_hessian): the expanded gate list in canonical bit order,
    // the gate angles that read a parameter ("occurrences", in gate order:
    // parameter index and chain factor), parameter -> occurrences (CSR), and
    // the derived plan in which occurrence k reads its own parameter k with
    // scale 1, built on the first dq_hessian call
    std::vector<DGate> canon;
    std::vector<int32_t> occ_param, hocc;
    std::vector<double> occ_scale;
    std::vector<int64_t> hoff;
    std::mutex hmu;
    std::unique_ptr<dq_plan_s> hess;
    std::mutex mu;
    std::map<int, DevData> dev;
    // kernel timing (dq_profile_enable / dq_profile_read)
    bool prof = false;
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    struct PRec {
        int kind;
        int nl;
        hipEvent_t a, b;
        double bytes, flops;
    };
    std::vector<PRec> precs;
    dq_profile acc{};
};

struct dq_obs_s {
    int n = 0;
    int nobs = 0;
    std::vector<DGroup> groups;
    std::vector<DTerm> terms;
    // groups [0, npair) go through the pair kernels; the one-bit-X groups
    // after them also through register tiles (complex64 states, n >= 11)
    int npair = 0;
    std::vector<XSet> xsets;
    std::vector<XTerm> xterms;
    size_t og = 0, ot = 0, ox = 0;   // byte offsets of groups / terms / tile terms in the device copy
    std::mutex mu;
    std::map<int, void *> dev;   // device -> [groups][terms]
};

namespace {

bool prof_on(const dq_plan_s &p) { return p.prof; }
hipEvent_t prof_event(dq_plan_s &p) {
    if (p.evused < p.evpool.size()) return p.evpool[p.evused++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p.evpool.push_back(e);
    p.evused++;
    return e;
}
void prof_push(dq_plan_s &p, int kind, int nl, hipEvent_t a, hipEvent_t b, double bytes, double flops) {
    if (a && b) p.precs.push_back({kind, nl, a, b, bytes, flops});
}
double state_bytes(const dq_plan_s &p, int64_t batch) { return (double)batch * std::ldexp(1.0, p.n) * (p.dbl ? 16 : 8); }

// ---------------------------------------------------------------- slots
int64_t add_slot(dq_plan_s &p, int dim, const std::vector<int> &factors, int dagger) {
    DSlot s{};
    s.dim = dim;
    s.nf = (int32_t)factors.size();
    for (size_t i = 0; i < factors.size(); ++i) s.f[i] = factors[i];
    s.dagger = dagger;
    s.off = p.block;
    p.block += (int64_t)dim * dim;
    p.slots.push_back(s);
    return (int64_t)p.slots.size() - 1;
}

// ---------------------------------------------------------------- planner
// operations x amplitudes per lane (per state) of the longest pass that is
// compiled; a 32-qubit HEA pass (about 23 operations on 64 amplitudes per
// lane) compiles in about 10 s, an 84-operation one in about a minute
constexpr int64_t kJitMaxWork = 2048;
// working sets beyond the 256 MB last-level cache are swept with
// non-temporal loads and stores (smaller ones keep their cache reuse)
constexpr double kStreamBytes = 256.0 * 1024 * 1024;

struct Planner {
    dq_plan_s &p;
    bool adjoint;
    int R;
    // Physical bits 3 and 4 in every tile of a large state: each group of 16
    // lanes then reads 128 contiguous bytes and each register pair 256.
    // Tiles whose bits are all high physical bits scatter every wave's
    // accesses over the whole state in 64-byte pieces, which halves the
    // bandwidth the memory system sustains once the state no longer fits the
    // last-level cache.
    uint64_t pinned = 0;
    // operations per pass in compiled plans: a longer pass would exceed the
    // compiled-kernel size limit and run interpreted, and the interpreted
    // kernel with 64 registers per lane keeps its tile in scratch memory
    int max_ops = 0;        // 0: no limit
    bool fusing = false;    // one-qubit gates on a wire fold into one operation (forward)
    explicit Planner(dq_plan_s &pl, bool adj, int r) : p(pl), adjoint(adj), R(r) {
        if (p.opt.jit && R > 0) max_ops = (int)(kJitMaxWork >> R);
        const int64_t state_bytes = (int64_t)(p.dbl ? 16 : 8) << p.n;
        // auto: bits 3 and 4 in both directions.  Pinning bit 3 alone frees
        // one more bit for gates (fewer adjoint passes), but its 128-byte
        // pieces made the adjoint passes' speed depend on where the state's
        // pages landed (27 to 37 ms per 32-qubit pass between runs of one
        // plan, against 25 ms with 256-byte pieces)
        const int want = p.opt.low_bits > 0 ? p.opt.low_bits - 1 : 2;   // physical bits 3.. to pin
        if (want > 0 && R >= 2 && p.n >= R + 8 && state_bytes >= (int64_t(128) << 20))
            pinned = want >= 2 ? (1ull << 3) | (1ull << 4) : (1ull << 3);
    }

    void gbits(int g, int *q, int &nq) const {
        nq = p.gates[g].nq;
        for (int i = 0; i < nq; ++i) q[i] = p.gates[g].bits[i];
    }
    bool tile_ok(int g) const {
        if (R <= 0) return false;
        const DGate &G = p.gates[g];
        if (G.op == OP_UNITARY && G.nq != 1) return false;
        int hi = 0;
        for (int i = 0; i < G.nq; ++i) hi += G.bits[i] >= 3;
        return hi <= R + 3;
    }
    bool diff(int g) const { return adjoint && p.gates[g].src != SRC_NONE && is_rotation(p.gates[g].op); }
    // With float64 arithmetic in compiled passes a diagonal one-qubit gate
    // does not fold into a non-diagonal slot, nor the reverse: the pass then
    // applies RY as a real matrix and takes the RZs of its bits as one
    // diagonal run (one complex product per amplitude for all of them)
    // instead of a dense matrix per bit (32-qubit, 20-layer forward: 1588 ->
    // 1496 ms).
    bool diag_apart() const { return p.opt.jit && p.opt.arith64; }

    // Greedy in-order selection of the gates one tile pass can execute when
    // the free tile bits are S (grown up to R + 3 bits while scanning; bits
    // 0..2 are in every tile).  Returns the executed gate positions (indices
    // into `rem`).
    std::vector<int> select(const std::vector<int> &rem, uint64_t &S, int seed) const {
        uint64_t blocked = 0;
        std::vector<int> out;
        int lslots = 0;
        int ops = 0;                // operations after folding, as plan() will fold
        uint64_t last_1q = 0;       // bits whose last selected gate is a one-qubit gate
        uint64_t diag_1q = 0;       // bits whose current one-qubit slot is diagonal
        int scount[64];             // per bit: gates folded into its current one-qubit slot
        auto popc = [](uint64_t x) { return __builtin_popcountll(x); };
        if (seed >= 0) {
            int q[5], nq;
            gbits(rem[seed], q, nq);
            for (int i = 0; i < nq; ++i)
                if (q[i] >= 3) S |= 1ull << q[i];
            if (popc(S) > R + 3) return out;
        }
        for (size_t r = 0; r < rem.size(); ++r) {
            const int g = rem[r];
            int q[5], nq;
            gbits(g, q, nq);
            uint64_t Q = 0, need = 0;
            for (int i = 0; i < nq; ++i) {
                Q |= 1ull << q[i];
                if (q[i] >= 3) need |= 1ull << q[i];
            }
            if ((Q & blocked) || !tile_ok(g) || (diff(g) && lslots >= 32) || popc(S | need) > R + 3) {
                blocked |= Q;
                continue;
            }
            const bool dg = nq == 1 && is_diag1(p.gates[g].op);
            const bool folds = fusing && nq == 1 && ((last_1q >> q[0]) & 1) && scount[q[0]] < SLOT_MAXF &&
                               (!diag_apart() || dg == (((diag_1q >> q[0]) & 1) != 0));
            if (max_ops && !folds && ops >= max_ops) break;
            S |= need;
            out.push_back((int)r);
            if (diff(g)) ++lslots;
            if (!folds) ++ops;
            if (nq == 1) {
                scount[q[0]] = folds ? scount[q[0]] + 1 : 1;
                last_1q |= 1ull << q[0];
                if (dg && !folds) diag_1q |= 1ull << q[0];
                else if (!dg) diag_1q &= ~(1ull << q[0]);
            } else {
                last_1q &= ~Q;
            }
        }
        return out;
    }

    void emit_pergate(Program &prog, int g) {
        const DGate &G = p.gates[g];
        if (adjoint && diff(g)) {
            Step gs;
            gs.kind = ST_GRAD;
            gs.gen = gen_of(G.op);
            gs.bits[0] = G.bits[0];
            gs.bits[1] = G.nq > 1 ? G.bits[1] : 0;
            gs.gslot = grad_slot(g);
            prog.steps.push_back(gs);
        }
        Step s;
        s.k = G.nq;
        for (int i = 0; i < G.nq; ++i) s.bits[i] = G.bits[i];
        if (G.op == OP_CNOT) {
            s.kind = ST_CNOT;
        } else if (G.op == OP_CZ) {
            s.kind = ST_CZ;
        } else if (G.op == OP_UNITARY && G.nq >= 4 && p.opt.fusion && p.n >= G.nq + (p.dbl ? 4 : 5)) {
            s.kind = ST_DENSE;           // matrix cores
            s.slot = p.slots[add_slot(p, 1 << G.nq, {g}, adjoint ? 1 : 0)].off;
            ++prog.dense_steps;
        } else {
            s.kind = G.nq == 1 ? ST_G1 : ST_GK;
            s.slot = p.slots[add_slot(p, 1 << G.nq, {g}, adjoint ? 1 : 0)].off;
        }
        s.flops_per_amp = G.op == OP_CNOT || G.op == OP_CZ || G.op == OP_SWAP ? 0.0 : (G.nq == 1 ? 14.0 : 8.0 * (1 << G.nq) - 2.0);
        prog.steps.push_back(s);
    }

    std::vector<int> gslot_of;   // gate -> gradient slot
    int grad_slot(int g) const { return gslot_of[g]; }

    // Greedy in-order selection for a fused dense block on at most K bits.
    std::vector<int> select_dense(const std::vector<int> &rem, uint64_t &W, int seed, int K) const {
        uint64_t blocked = 0;
        std::vector<int> out;
        auto popc = [](uint64_t x) { return __builtin_popcountll(x); };
        auto ok = [&](const DGate &G) { return G.nq <= 2; };
        if (seed >= 0) {
            const DGate &G = p.gates[rem[seed]];
            for (int i = 0; i < G.nq; ++i) W |= 1ull << G.bits[i];
            if (popc(W) > K) return out;
        }
        for (size_t r = 0; r < rem.size(); ++r) {
            const DGate &G = p.gates[rem[r]];
            uint64_t Q = 0;
            for (int i = 0; i < G.nq; ++i) Q |= 1ull << G.bits[i];
            if ((Q & blocked) || !ok(G) || popc(W | Q) > K) {
                blocked |= Q;
                continue;
            }
            W |= Q;
            out.push_back((int)r);
        }
        return out;
    }

    // Forward plan of fused K-qubit dense blocks applied on the matrix cores.
    void plan_dense(Program &prog, std::vector<int> order, int K) {
        prog.slot_lo = (int64_t)p.slots.size();
        prog.blk_lo = (int64_t)p.blocks.size();
        std::vector<int> rem = order;
        while (!rem.empty()) {
            const int g0 = rem[0];
            uint64_t bestW = 0;
            std::vector<int> best;
            if (p.gates[g0].nq <= 2) {
                int tried = 0;
                for (size_t r = 0; r < rem.size() && tried < 48; ++r) {
                    if (p.gates[rem[r]].nq > 2) continue;
                    ++tried;
                    uint64_t W = 0;
                    std::vector<int> sel = select_dense(rem, W, (int)r, K);
                    if (sel.size() > best.size()) {
                        best = sel;
                        bestW = W;
                    }
                }
            }
            if (best.empty()) {
                emit_pergate(prog, g0);
                rem.erase(rem.begin());
                continue;
            }
            for (int b = 0; b < p.n && __builtin_popcountll(bestW) < K; ++b) bestW |= 1ull << b;
            DBlock bl{};
            bl.k = K;
            bl.nf = (int32_t)best.size();
            bl.foff = (int32_t)p.factors.size();
            int t = 0;
            for (int b = p.n - 1; b >= 0; --b)            // most significant block bit first
                if (bestW >> b & 1) bl.bb[t++] = b;
            for (int r : best) p.factors.push_back(rem[r]);
            bl.off = p.block;
            p.block += (int64_t)(1 << K) * (1 << K);
            p.blocks.push_back(bl);
            Step st;
            st.kind = ST_DENSE;
            st.k = K;
            for (int i = 0; i < K; ++i) st.bits[i] = bl.bb[i];
            st.slot = bl.off;
            st.flops_per_amp = 8.0 * (1 << K) - 2.0;
            prog.steps.push_back(st);
            ++prog.dense_steps;
            std::vector<char> done(rem.size(), 0);
            for (int r : best) done[r] = 1;
            std::vector<int> nrem;
            for (size_t r = 0; r < rem.size(); ++r)
                if (!done[r]) nrem.push_back(rem[r]);
            rem.swap(nrem);
        }
        prog.slot_hi = (int64_t)p.slots.size();
        prog.blk_hi = (int64_t)p.blocks.size();
    }

    // A tile whose register bits all sit at byte offsets of 1 GiB or more,
    // with lane bits other than 3, 4, 5, has each wave issue its loads to
    // pieces of a few hundred bytes scattered over every 1 GiB region of the
    // state: on MI355X such sweeps of two states ran at less than half the
    // bandwidth of any other split of the same tile bits between lanes and
    // registers.  Then the highest register bit becomes a lane bit, in place
    // of the free lane bit with the most data-moving operations.
    void far_register_rule(std::vector<int> &lanes, std::vector<int> &regs, const int *moves) const {
        const int amp_log2 = p.dbl ? 4 : 3;
        for (int b : regs)
            if (b + amp_log2 < 30) return;
        std::vector<int> sl(lanes);
        std::sort(sl.begin(), sl.end());
        if (sl[0] == 3 && sl[1] == 4 && sl[2] == 5) return;
        int out = -1;   // lane to give up: never the pinned bit 3
        for (int k = 0; k < 3; ++k) {
            if (((pinned >> lanes[k]) & 1) != 0) continue;
            if (out < 0 || moves[lanes[k]] > moves[lanes[out]] ||
                (moves[lanes[k]] == moves[lanes[out]] && lanes[k] < lanes[out]))
                out = k;
        }
        if (out < 0) return;
        auto hi = std::max_element(regs.begin(), regs.end());
        std::swap(lanes[out], *hi);
    }

    static bool real1(int op) { return op == OP_RY || op == OP_H || op == OP_X || op == OP_Z; }

    void plan(Program &prog, std::vector<int> order, bool fuse_1q) {
        fusing = fuse_1q;
        prog.slot_lo = (int64_t)p.slots.size();
        std::vector<int> rem = order;
        while (!rem.empty()) {
            const int g0 = rem[0];
            if (!tile_ok(g0)) {
                emit_pergate(prog, g0);
                rem.erase(rem.begin());
                continue;
            }
            // candidate register sets: unseeded, and seeded by each of the
            // first few gates that need non-lane bits
            uint64_t bestS = pinned;
            std::vector<int> best;
            {
                uint64_t S = pinned;
                best = select(rem, S, -1);
                bestS = S;
            }
            int tried = 0;
            for (size_t r = 0; r < rem.size() && tried < 48; ++r) {
                const DGate &G = p.gates[rem[r]];
                bool hi = false;
                for (int i = 0; i < G.nq; ++i) hi |= G.bits[i] >= 3;
                if (!hi || !tile_ok(rem[r])) continue;
                ++tried;
                uint64_t S = pinned;
                std::vector<int> sel = select(rem, S, (int)r);
                if (sel.size() > best.size()) {
                    best = sel;
                    bestS = S;
                }
            }
            if (best.empty()) {            // nothing fits a tile: keep making progress
                emit_pergate(prog, g0);
                rem.erase(rem.begin());
                continue;
            }
            // pad the free set to exactly R + 3 bits
            for (int b = 3; b < p.n && __builtin_popcountll(bestS) < R + 3; ++b) bestS |= 1ull << b;
            // lane bits 3..5: the three free bits that see the fewest
            // data-moving ops (those need cross-lane shuffles); the rest are
            // register bits
            int moves[64] = {0};
            for (int r : best) {
                const DGate &G = p.gates[rem[r]];
                const bool diag = is_diag1(G.op) || G.op == OP_CZ || G.op == OP_CP || G.op == OP_RZZ;
                if (diag) continue;
                if (G.op == OP_CNOT) moves[G.bits[1]] += 1;
                else
                    for (int i = 0; i < G.nq; ++i) moves[G.bits[i]] += 1;
            }
            std::vector<int> freeb;
            for (int b = 3; b < p.n; ++b)
                if (bestS >> b & 1) freeb.push_back(b);
            std::stable_sort(freeb.begin(), freeb.end(), [&](int x, int y) { return moves[x] < moves[y]; });
            if (pinned) {   // lane bit 3 = physical bit 3, physical bit 4 (if pinned) a register bit
                const bool p4 = (pinned >> 4) & 1;
                std::vector<int> rest;
                for (int b : freeb)
                    if (b != 3 && !(p4 && b == 4)) rest.push_back(b);
                freeb.assign({3});
                freeb.insert(freeb.end(), rest.begin(), rest.begin() + 2);
                if (p4) freeb.push_back(4);
                freeb.insert(freeb.end(), rest.begin() + 2, rest.end());
            }
            Step st;
            st.kind = ST_TILE;
            st.R = R;
            int local[64];
            for (int b = 0; b < 64; ++b) local[b] = -1;
            for (int b = 0; b < 3; ++b) local[b] = b;
            std::vector<int> lanes(freeb.begin(), freeb.begin() + 3), regs(freeb.begin() + 3, freeb.end());
            far_register_rule(lanes, regs, moves);
            std::sort(lanes.begin(), lanes.end());
            std::sort(regs.begin(), regs.end());
            for (int k = 0; k < 3; ++k) {
                st.lbits[k] = lanes[k];
                local[lanes[k]] = 3 + k;
            }
            for (int k = 0; k < R; ++k) {
                st.rbits[k] = regs[k];
                local[regs[k]] = 6 + k;
            }
            std::vector<int> all(freeb);
            std::sort(all.begin(), all.end());
            for (int k = 0; k < R + 3; ++k) st.tbits[k] = all[k];
            st.op0 = (int64_t)p.ops.size();
            st.ls0 = (int64_t)p.lsg.size();
            std::vector<int> last_op(64, -1);     // per physical bit: index (in p.ops) of the last op touching it
            std::vector<int64_t> op_slot;         // per op of this pass: its slot index, -1 none
            for (int r : best) {
                const int g = rem[r];
                const DGate &G = p.gates[g];
                TOp op{};
                int64_t slot_idx = -1;
                op.q0 = local[G.bits[0]];
                op.q1 = G.nq > 1 ? local[G.bits[1]] : 0;
                op.gen = GEN_NONE;
                op.lslot = -1;
                if (G.nq == 1) {
                    const int prev = last_op[G.bits[0]];
                    // (as select() predicts: diagonal and non-diagonal gates
                    // stay in separate slots where diag_apart())
                    if (fuse_1q && prev >= st.op0 && (p.ops[prev].kind == TK_1Q || p.ops[prev].kind == TK_1QDIAG) &&
                        (!diag_apart() || is_diag1(G.op) == (p.ops[prev].kind == TK_1QDIAG))) {
                        DSlot &sl = p.slots[op_slot[prev - st.op0]];
                        if (sl.nf < SLOT_MAXF) {   // fold into the previous one-qubit slot of this bit
                            sl.f[sl.nf++] = g;
                            if (!is_diag1(G.op)) p.ops[prev].kind = TK_1Q;
                            continue;
                        }
                    }
                    op.kind = is_diag1(G.op) ? TK_1QDIAG : TK_1Q;
                    slot_idx = add_slot(p, 2, {g}, adjoint ? 1 : 0);
                    op.slot = (int32_t)p.slots[slot_idx].off;
                } else {
                    switch (G.op) {
                    case OP_CNOT: op.kind = TK_CNOT; break;
                    case OP_CZ: op.kind = TK_CZ; break;
                    case OP_SWAP: op.kind = TK_SWAP; break;
                    default:
                        op.kind = TK_2QDIAG;
                        slot_idx = add_slot(p, 4, {g}, adjoint ? 1 : 0);
                        op.slot = (int32_t)p.slots[slot_idx].off;
                        break;
                    }
                }
                if (diff(g)) {
                    op.gen = gen_of(G.op);
                    op.lslot = (int32_t)((int64_t)p.lsg.size() - st.ls0);
                    p.lsg.push_back(grad_slot(g));
                }
                for (int i = 0; i < G.nq; ++i) last_op[G.bits[i]] = (int)p.ops.size();
                p.ops.push_back(op);
                op_slot.push_back(slot_idx);
            }
            // cheapest kernel form of each one-qubit slot: diagonal (RZ, Z),
            // real (RY, H, X, Z and their products), RX form, or dense
            for (int64_t k = st.op0; k < (int64_t)p.ops.size(); ++k) {
                TOp &o = p.ops[k];
                if (o.kind != TK_1Q && o.kind != TK_1QDIAG) continue;
                const DSlot &sl = p.slots[op_slot[k - st.op0]];
                bool diag = true, real = true;
                for (int f = 0; f < sl.nf; ++f) {
                    const int op = p.gates[sl.f[f]].op;
                    diag = diag && is_diag1(op);
                    real = real && real1(op);
                }
                if (diag) o.kind = TK_1QDIAG;
                else if (real) o.kind = TK_1QREAL;
                else if (sl.nf == 1 && p.gates[sl.f[0]].op == OP_RX) o.kind = TK_1QRX;
                else o.kind = TK_1Q;
            }
            st.nops = (int64_t)p.ops.size() - st.op0;
            for (int64_t k = st.op0; k < (int64_t)p.ops.size(); ++k) {
                const TOp &o = p.ops[k];
                double f = 0;
                switch (o.kind) {
                case TK_1Q: f = 14; break;
                case TK_1QREAL: case TK_1QRX: case TK_1QDIAG: case TK_2QDIAG: f = 6; break;
                default: f = 0; break;
                }
                st.flops_per_amp += f;
                if (o.lslot >= 0) st.flops_per_amp += 3.0 / (adjoint ? 2 : 1);   // per state (the adjoint sweeps two)
            }
            st.nls = (int64_t)p.lsg.size() - st.ls0;
            prog.steps.push_back(st);
            ++prog.tile_passes;
            std::vector<char> done(rem.size(), 0);
            for (int r : best) done[r] = 1;
            std::vector<int> nrem;
            for (size_t r = 0; r < rem.size(); ++r)
                if (!done[r]) nrem.push_back(rem[r]);
            rem.swap(nrem);
        }
        prog.slot_hi = (int64_t)p.slots.size();
        prog.blk_lo = prog.blk_hi = (int64_t)p.blocks.size();
    }
};

int default_R(const dq_plan_s &p) {
    // defaults keep two resident waves per SIMD: interpreted passes hold 32
    // complex64 (16 complex128) amplitudes per lane; compiled passes, which
    // need no registers for dispatch, hold twice that
    const int base = p.opt.jit ? (p.mdbl ? 5 : 6) : (p.mdbl ? 4 : 5);
    int R = p.opt.tile_bits > 0 ? p.opt.tile_bits : base;
    // 64 amplitudes per lane only in compiled passes: the interpreted kernel
    // cannot keep that many in registers (its tile went to scratch memory);
    // the same holds for 32 complex128 amplitudes per lane, interpreted
    if ((p.mdbl || !p.opt.jit) && R > 5) R = 5;
    if (!p.opt.jit && p.dbl && R > 4) R = 4;
    if (R > p.n - 6) R = p.n - 6;
    return R < 0 ? 0 : R;
}

// (Re)plan the adjoint program, at most `cap` operations per tile pass when
// cap > 0; returns its number of steps.
size_t plan_adjoint(dq_plan_s &p, int cap) {
    const auto &m = p.adj_mark;
    p.slots.resize(m[0]);
    p.ops.resize(m[1]);
    p.lsg.resize(m[2]);
    p.factors.resize(m[3]);
    p.blocks.resize(m[4]);
    p.block = (int64_t)m[5];
    p.adj = Program();
    Planner pl(p, true, p.R_adj);
    if (cap > 0) pl.max_ops = pl.max_ops > 0 ? std::min(pl.max_ops, cap) : cap;
    pl.gslot_of = p.adj_gslot;
    pl.plan(p.adj, p.adj_rev, false);
    return p.adj.steps.size();
}

// Compiled adjoint passes: the greedy packing leaves some passes much fuller
// than the rest (the 32-qubit ring workload, float64 arithmetic: one pass
// per layer with 21 operations beside passes of 15, running 47-54 ms
// against 25-29 ms; two waves per SIMD cannot hide its arithmetic behind its
// memory traffic).  The operations per pass are capped at the smallest value
// that needs no more passes than the fewest any cap down to half the fullest
// pass reaches (that workload: 121 passes, at most 18 operations; adjoint
// 3.93 -> 3.55 s per step).  Run once, on the plan's final layout, for
// float64 arithmetic only: with float32 arithmetic the passes are not
// arithmetic-bound (the same workload unchanged, a 20-qubit Hessian 2.8 %
// slower).
void balance_adjoint(dq_plan_s &p) {
    if (!p.opt.jit || !p.mdbl || p.R_adj <= 0 || p.adj_mark.empty()) return;
    size_t best = p.adj.steps.size();
    int most = 0;
    for (const Step &S : p.adj.steps)
        if (S.kind == ST_TILE) most = std::max(most, (int)S.nops);
    int cap_best = 0;
    for (int cap = most - 1; cap >= std::max(2, most / 2); --cap) {
        const size_t n = plan_adjoint(p, cap);
        if (n <= best) {
            best = n;
            cap_best = cap;
        } else if (n > best + std::max<size_t>(2, best / 20)) {
            break;   // well past the point where passes start to multiply
        }
    }
    plan_adjoint(p, cap_best);
}

dq_status build_plan(dq_plan_s &p) {
    const int G_all = (int)p.gates.size();
    const int G = G_all - (int)p.entry_gates;   // the circuit proper; entry gates follow it in the list
    const bool fused = p.opt.fusion != 0;
    p.R_fwd = fused ? default_R(p) : 0;
    // two states per tile in the adjoint: fewer register bits by default
    const int abase = p.opt.jit ? (p.mdbl ? 4 : 5) : (p.mdbl ? 3 : 4);
    int ra = p.opt.adj_tile_bits > 0 ? p.opt.adj_tile_bits : std::min(p.R_fwd, abase);
    // interpreted adjoint kernels exist up to 16 complex64 / 8 complex128
    // amplitudes per lane and state: wider ones kept their tiles in scratch
    if (!p.opt.jit && ra > (p.dbl ? 3 : 4)) ra = p.dbl ? 3 : 4;
    if (ra > p.n - 6) ra = p.n - 6;
    p.R_adj = fused && ra > 0 ? ra : 0;
    // gradient slots: every differentiable gate occurrence, in gate order
    std::vector<int> gslot(G_all, -1);
    p.ngrad = 0;
    for (int g = 0; g < G; ++g)
        if (p.gates[g].src != SRC_NONE && is_rotation(p.gates[g].op)) gslot[g] = p.ngrad++;
    // CSR: parameter / data -> gradient slots with chain factors
    auto csr = [&](int src, int64_t count, std::vector<int64_t> &off, std::vector<int32_t> &gi,
                   std::vector<double> &f) {
        std::vector<std::vector<std::pair<int, double>>> lists((size_t)count);
        for (int g = 0; g < G; ++g)
            if (gslot[g] >= 0 && p.gates[g].src == src)
                lists[(size_t)p.gates[g].idx].push_back(
                    {gslot[g], p.gates[g].scale * (p.gates[g].op == OP_CP ? -2.0 : 1.0)});
        off.assign((size_t)count + 1, 0);
        for (int64_t i = 0; i < count; ++i) {
            off[i + 1] = off[i] + (int64_t)lists[i].size();
            for (auto &e : lists[i]) {
                gi.push_back(e.first);
                f.push_back(e.second);
            }
        }
    };
    csr(SRC_PARAM, p.nparams, p.poff, p.pg, p.pf);
    csr(SRC_DATA, p.ndata, p.doff, p.dg, p.df);

    std::vector<int> order(G);
    for (int g = 0; g < G; ++g) order[g] = g;
    const int dense_k = fused ? p.opt.dense_fuse : 0;
    const bool dense = dense_k >= 4 && p.n >= dense_k + (p.dbl ? 4 : 5);
    // forward from a given state: the entry gates, then the circuit
    {
        std::vector<int> full;
        for (int g = G; g < G_all; ++g) full.push_back(g);
        full.insert(full.end(), order.begin(), order.end());
        Planner pl(p, false, p.R_fwd);
        pl.gslot_of = gslot;
        if (dense) pl.plan_dense(p.fwd_full, full, dense_k);
        else pl.plan(p.fwd_full, full, true);
    }
    // forward from |0..0> with the leading one-qubit gates of every wire folded
    p.fold_off.assign(p.n, -1);
    p.has_fold = false;
    p.folded_gates = 0;
    if (fused && p.opt.fold_init) {
        std::vector<std::vector<int>> lead(p.n);
        std::vector<char> closed(p.n, 0), folded(G, 0);
        for (int g = 0; g < G; ++g) {
            const DGate &D = p.gates[g];
            if (D.nq == 1) {
                const int b = D.bits[0];
                if (!closed[b] && (int)lead[b].size() < SLOT_MAXF) {
                    lead[b].push_back(g);
                    folded[g] = 1;
                } else {
                    closed[b] = 1;
                }
            } else {
                for (int i = 0; i < D.nq; ++i) closed[D.bits[i]] = 1;
            }
        }
        for (int b = 0; b < p.n; ++b)
            if (!lead[b].empty()) {
                p.fold_off[b] = p.slots[add_slot(p, 2, lead[b], 0)].off;
                p.folded_gates += (int64_t)lead[b].size();
            }
        if (p.folded_gates > 0) {
            p.has_fold = true;
            std::vector<int> rest;
            for (int g = 0; g < G; ++g)
                if (!folded[g]) rest.push_back(g);
            Planner pl(p, false, p.R_fwd);
            pl.gslot_of = gslot;
            const int64_t lo = (int64_t)p.slots.size() - (int64_t)std::count_if(p.fold_off.begin(), p.fold_off.end(),
                                                                                [](int64_t o) { return o >= 0; });
            if (dense) pl.plan_dense(p.fwd_fold, rest, dense_k);
            else pl.plan(p.fwd_fold, rest, true);
            p.fwd_fold.slot_lo = lo;
        }
    }
    // adjoint: the reversed gate list, daggers, no fusion of one-qubit gates;
    // what it needs to be planned again is kept (balance_adjoint)
    p.adj_rev.assign(order.rbegin(), order.rend());
    p.adj_gslot = gslot;
    p.adj_mark = {p.slots.size(), p.ops.size(), p.lsg.size(), p.factors.size(), p.blocks.size(), (size_t)p.block};
    plan_adjoint(p, 0);
    return DQ_OK;
}

// ---------------------------------------------------------------- device upload
template <typename T>
size_t put(std::vector<char> &blob, const std::vector<T> &v) {
    const size_t off = align256(blob.size());
    blob.resize(off + std::max<size_t>(v.size() * sizeof(T), 1));
    if (!v.empty()) memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

// ---------------------------------------------------------------- compiled passes
// Source of the kernel that runs one tile pass as straight-line code: every
// operation becomes a call with compile-time operand positions (tile-local
// bits; matrix slots relative to the pass's first matrix, whose address the
// launch passes in).  Passes with equal operation lists share one kernel.
bool has_matrix(int kind) {
    return kind == TK_1Q || kind == TK_1QDIAG || kind == TK_2QDIAG || kind == TK_1QREAL || kind == TK_1QRX;
}

std::string pass_body(const dq_plan_s &p, const Step &S, bool adj, int64_t &s0) {
    s0 = -1;
    for (int64_t i = 0; i < S.nops; ++i) {
        const TOp &o = p.ops[(size_t)(S.op0 + i)];
        if (has_matrix(o.kind) && (s0 < 0 || o.slot < s0)) s0 = o.slot;
    }
    if (s0 < 0) s0 = 0;
    const char *T = p.mdbl ? "double" : "float";              // arithmetic
    const char *SS = p.dbl ? "double" : "float";              // storage
    const int R = S.R, NR = 1 << R, NS = adj ? 2 : 1;
    // compiled per plan: the streaming choice follows one sample's working set
    const char *nt = std::ldexp((double)NS * (p.dbl ? 16 : 8), p.n) > kStreamBytes ? "true" : "false";
    // occupancy target (waves per SIMD): two while a lane holds up to 64
    // complex64 amplitudes of one state (32 of each of two in the adjoint)
    const int rb = NR * (p.mdbl ? 8 : 4);
    const int W = adj ? (rb >= 256 ? 1 : (rb >= 64 ? 2 : 4)) : (rb >= 512 ? 1 : (rb >= 128 ? 2 : 3));
    char line[256];
    std::string b;
    snprintf(line, sizeof line, "__launch_bounds__(64, %d) void @NAME@(dq::TileArgs a) {\n", W);
    b += line;
    if (adj) {
        snprintf(line, sizeof line,
                 "    extern __shared__ double acc[];\n"
                 "    dq::jit_adj<%s, %d, %s, %s>(a, acc, [&](auto &v, auto m, int lane, double *ac) {\n", T, R, nt, SS);
    } else {
        snprintf(line, sizeof line, "    dq::jit_fwd<%s, %d, %s, %s>(a, [&](auto &v, auto m, int lane) {\n", T, R, nt, SS);
    }
    b += line;
    const TOp *ops = p.ops.data() + S.op0;
    for (int64_t i = 0; i < S.nops;) {
        // a run of one-qubit diagonal gates (the RZ of a layer and the like)
        // becomes one product diagonal; diagonal gates commute, so their
        // gradient terms are all taken at the start of the run
        int64_t e = i;
        while (e < S.nops && ops[e].kind == TK_1QDIAG) ++e;
        if (e - i >= 2) {
            b += "        {\n";
            bool anyg = false;
            for (int64_t j = i; j < e; ++j) anyg |= adj && ops[j].lslot >= 0;
            std::vector<int> regk;   // distinct register bits of the run, in first-use order
            for (int64_t j = i; j < e; ++j)
                if (ops[j].q0 >= 6 && std::find(regk.begin(), regk.end(), ops[j].q0 - 6) == regk.end()) regk.push_back(ops[j].q0 - 6);
            if (anyg) {
                snprintf(line, sizeof line, "            %s sa_, sk_[%d];\n            dq::run_sums<%s, dq::cx<%s>, %d", T,
                         regk.empty() ? 1 : (int)regk.size(), T, T, NR);
                b += line;
                for (int k : regk) b += ", " + std::to_string(k);
                b += ">(v[0], v[1], sa_, sk_);\n";
            }
            for (int64_t j = i; j < e; ++j) {
                const TOp &o = ops[j];
                if (!adj || o.lslot < 0) continue;
                if (o.q0 < 6) {
                    snprintf(line, sizeof line, "            ac[%d * 64 + lane] += (double)(((lane >> %d) & 1) ? -sa_ : sa_);\n", o.lslot, o.q0);
                } else {
                    const size_t ri = (size_t)(std::find(regk.begin(), regk.end(), o.q0 - 6) - regk.begin());
                    snprintf(line, sizeof line, "            ac[%d * 64 + lane] += (double)sk_[%zu];\n", o.lslot, ri);
                }
                b += line;
            }
            // the lane factor fl_ and the ratios r_ are formed in double and
            // rounded once inside diag_run
            snprintf(line, sizeof line, "            dq::C128 fl_{1.0, 0.0}, r_[%d];\n", regk.empty() ? 1 : (int)regk.size());
            b += line;
            std::vector<char> started(regk.size(), 0);
            for (int64_t j = i; j < e; ++j) {
                const TOp &o = ops[j];
                const long long sl = (long long)(o.slot - s0);
                if (o.q0 < 6) {
                    snprintf(line, sizeof line, "            fl_ = dq::cmul(fl_, dq::widen(dq::csel(((lane >> %d) & 1) != 0, dq::ldc(m, %lld), dq::ldc(m, %lld))));\n",
                             o.q0, sl + 3, sl);
                } else {
                    const size_t ri = (size_t)(std::find(regk.begin(), regk.end(), o.q0 - 6) - regk.begin());
                    // a second gate on the same bit multiplies into that bit's ratio
                    const std::string rv = "r_[" + std::to_string(ri) + "]";
                    const std::string ratio = "dq::cmul(d1, dq::cconj(d0))";
                    snprintf(line, sizeof line,
                             "            { const auto d0 = dq::widen(dq::ldc(m, %lld)), d1 = dq::widen(dq::ldc(m, %lld)); fl_ = dq::cmul(fl_, d0); "
                             "%s = %s; }\n", sl, sl + 3, rv.c_str(),
                             (started[ri] ? "dq::cmul(" + rv + ", " + ratio + ")" : ratio).c_str());
                    started[ri] = 1;
                }
                b += line;
            }
            snprintf(line, sizeof line, "            dq::diag_run<%s, %d, %d", T, NS, NR);
            b += line;
            for (int k : regk) b += ", " + std::to_string(k);
            b += ">(v, fl_, r_);\n        }\n";
            i = e;
            continue;
        }
        const TOp &o = ops[i];
        if (adj && o.lslot >= 0) {
            snprintf(line, sizeof line, "        ac[%d * 64 + lane] += (double)dq::gen_s<%s, %d, %d, %d, %d>(v[0], v[1], lane);\n",
                     o.lslot, T, NR, o.gen, o.q0, o.q1);
            b += line;
        }
        snprintf(line, sizeof line, "        dq::op_s<%s, %d, %d, %d, %d, %d, %lld>(v, m, lane);\n", T, NS, NR, o.kind, o.q0,
                 o.q1, has_matrix(o.kind) ? (long long)(o.slot - s0) : 0ll);
        b += line;
        ++i;
    }
    b += "    });\n}\n";
    return b;
}


void jit_generate(dq_plan_s &p) {
    std::map<std::string, int> index;
    auto gen = [&](Program &prog, bool adj) {
        prog.jk.assign(prog.steps.size(), -1);
        prog.js0.assign(prog.steps.size(), 0);
        for (size_t k = 0; k < prog.steps.size(); ++k) {
            const Step &S = prog.steps[k];
            if (S.kind != ST_TILE) continue;
            // compile time grows faster than linearly with the length of the
            // straight-line code: longer passes stay interpreted, except
            // 64-amplitude tiles, which have no interpreted kernel (the
            // planner keeps them within the limit in any case)
            if (S.R < 6 && S.nops * (int64_t(1) << S.R) > kJitMaxWork) continue;
            int64_t s0 = 0;
            const std::string body = pass_body(p, S, adj, s0);
            auto it = index.find(body);
            if (it == index.end()) {
                const std::string name = jit_key(body);
                std::string src = "#include \"tile_dev.h\"\nextern \"C\" __global__ " + body;
                src.replace(src.find("@NAME@"), 6, name);
                it = index.emplace(body, (int)p.jnames.size()).first;
                p.jnames.push_back(name);
                p.jsrcs.push_back(src);
            }
            prog.jk[k] = it->second;
            prog.js0[k] = s0;
        }
    };
    gen(p.fwd_full, false);
    if (p.has_fold) gen(p.fwd_fold, false);
    gen(p.adj, true);
}

// every step of every program is a compiled tile pass (the float64
// arithmetic of arith64 plans exists only in compiled passes)
bool all_compiled(const dq_plan_s &p) {
    for (const Program *pr : {&p.fwd_full, &p.fwd_fold, &p.adj}) {
        if (pr == &p.fwd_fold && !p.has_fold) continue;
        for (size_t k = 0; k < pr->steps.size(); ++k)
            if (pr->steps[k].kind != ST_TILE || pr->jk.size() <= k || pr->jk[k] < 0) return false;
    }
    return true;
}

// ---------------------------------------------------------------- qubit layout
// Physical bits 0..2 (and, in large states, 3 and 4) are in every tile, so
// the wires that sit there cost nothing to include in a pass.  When those
// wires are adjacent in the circuit's entangling structure (the ring's last
// five wires in wire order), every pass must re-include a linking wire; the
// search below relabels physical bits 1..4 with four wires spread evenly over
// the register (a set of transpositions), plans each candidate, and keeps the
// one with the fewest state sweeps (forward steps x 2 + adjoint steps x 4).
// The same transpositions are appended as SWAP gates, so the state handed back
// keeps the canonical order; the adjoint undoes them first.
double plan_cost(const dq_plan_s &p) {
    const Program &f = p.has_fold ? p.fwd_fold : p.fwd_full;
    return 2.0 * (double)f.steps.size() + 4.0 * (double)p.adj.steps.size();
}

dq_plan_s *plan_clone_base(const dq_plan_s &p) {
    auto *q = new dq_plan_s();
    q->n = p.n;
    q->dbl = p.dbl;
    q->mdbl = p.mdbl;
    q->opt = p.opt;
    q->nparams = p.nparams;
    q->ndata = p.ndata;
    q->fixed = p.fixed;
    q->user_gates = p.user_gates;
    q->entry_gates = 0;
    q->canon = p.canon;
    q->occ_param = p.occ_param;
    q->occ_scale = p.occ_scale;
    q->hoff = p.hoff;
    q->hocc = p.hocc;
    return q;
}

dq_plan_s *search_layout(dq_plan_s *p_in) {
    std::unique_ptr<dq_plan_s> canon(p_in), chosen;   // the canonical plan; the best relabelled one
    const dq_plan_s *const p = canon.get();
    const int64_t state_bytes = (int64_t)(p->dbl ? 16 : 8) << p->n;
    if (!p->opt.fusion || p->R_fwd < 2 || p->n < 16 || state_bytes < (int64_t(128) << 20)) return canon.release();
    const std::vector<DGate> base(p->gates.begin(), p->gates.begin() + p->user_gates);
    double best = plan_cost(*p);
    // k of the low bits 4, 3, .. (those pinned last first) move to k wires
    // spaced d apart from offset o
    for (int k : {3, 4})
    for (int d : {p->n / 3, p->n / 4, p->n / 5}) {
        if (d < 2) continue;
        for (int o = 0; o < d; ++o) {
            int tgt[4], lows[4];
            bool ok = true;
            for (int j = 0; j < k; ++j) {
                tgt[j] = o + j * d;
                lows[j] = 1 + j;
                ok &= tgt[j] >= 5 && tgt[j] < p->n;
            }
            if (!ok) continue;
            int perm[64];
            for (int b = 0; b < p->n; ++b) perm[b] = b;
            for (int j = 0; j < k; ++j) {
                perm[lows[j]] = tgt[k - 1 - j];
                perm[tgt[k - 1 - j]] = lows[j];
            }
            std::unique_ptr<dq_plan_s> q(plan_clone_base(*p));
            q->gates = base;
            for (DGate &g : q->gates)
                for (int i = 0; i < g.nq; ++i) g.bits[i] = perm[g.bits[i]];
            // back to the canonical order at the end; and, for a forward from a
            // given state (not |0..0>, which the relabelling leaves alone),
            // into the relabelled order at the start: the same transpositions,
            // kept at the end of the list as entry gates
            for (int rep = 0; rep < 2; ++rep)
                for (int j = 0; j < k; ++j) {
                    DGate sw{};
                    sw.op = OP_SWAP;
                    sw.nq = 2;
                    sw.bits[0] = tgt[k - 1 - j];
                    sw.bits[1] = lows[j];
                    sw.src = SRC_NONE;
                    q->gates.push_back(sw);
                }
            q->entry_gates = k;
            q->layout_swaps = k;
            if (build_plan(*q) == DQ_OK && plan_cost(*q) < best) {
                best = plan_cost(*q);
                chosen = std::move(q);
            }
        }
    }
    return chosen ? chosen.release() : canon.release();
}

dq_status ensure_device(dq_plan_s &p, DevData **out) {
    int dev = 0;
    DQ_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(p.mu);
    auto it = p.dev.find(dev);
    if (it != p.dev.end()) {
        *out = &it->second;
        return DQ_OK;
    }
    std::vector<char> blob;
    const size_t o_b = put(blob, p.blocks), o_fa = put(blob, p.factors);
    const size_t o_g = put(blob, p.gates), o_f = put(blob, p.fixed), o_s = put(blob, p.slots),
                 o_o = put(blob, p.ops), o_l = put(blob, p.lsg), o_fo = put(blob, p.fold_off),
                 o_po = put(blob, p.poff), o_pg = put(blob, p.pg), o_pf = put(blob, p.pf),
                 o_do = put(blob, p.doff), o_dg = put(blob, p.dg), o_df = put(blob, p.df),
                 o_op = put(blob, p.occ_param), o_os = put(blob, p.occ_scale), o_ho = put(blob, p.hoff),
                 o_hc = put(blob, p.hocc);
    void *d = nullptr;
    DQ_HIP(hipMalloc(&d, blob.size()));
    hipError_t e = hipMemcpy(d, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(DQ_ERR_HIP, "plan upload: %s", hipGetErrorString(e));
    }
    DevData dd;
    char *b = (char *)d;
    dd.blob = d;
    dd.gates = (DGate *)(b + o_g);
    dd.fixed = (double2 *)(b + o_f);
    dd.slots = (DSlot *)(b + o_s);
    dd.blocks = (DBlock *)(b + o_b);
    dd.factors = (int32_t *)(b + o_fa);
    dd.ops = (TOp *)(b + o_o);
    dd.lsg = (int32_t *)(b + o_l);
    dd.fold = (int64_t *)(b + o_fo);
    dd.poff = (int64_t *)(b + o_po);
    dd.pg = (int32_t *)(b + o_pg);
    dd.pf = (double *)(b + o_pf);
    dd.doff = (int64_t *)(b + o_do);
    dd.dg = (int32_t *)(b + o_dg);
    dd.df = (double *)(b + o_df);
    dd.occ_param = (int32_t *)(b + o_op);
    dd.occ_scale = (double *)(b + o_os);
    dd.hoff = (int64_t *)(b + o_ho);
    dd.hocc = (int32_t *)(b + o_hc);
    if (!p.jnames.empty()) {
        std::string err;
        if (!jit_load(p.jnames, p.jsrcs, dd.jfn, err)) {
            (void)hipFree(dd.blob);
            return fail(DQ_ERR_INTERNAL, "%s", err.c_str());
        }
        // the adjoint's work units per sample follow the compiled kernels'
        // occupancy (with their accumulator LDS), not the interpreter's
        for (size_t k = 0; k < p.adj.steps.size(); ++k) {
            if (p.adj.jk.empty() || p.adj.jk[k] < 0) continue;
            const size_t lds = sizeof(double) * 64 * (size_t)std::max<int64_t>(p.adj.steps[k].nls, 1);
            const int cap = jit_resident(dd.jfn[(size_t)p.adj.jk[k]], lds);
            if (cap > 0 && (dd.jit_adj_cap == 0 || cap < dd.jit_adj_cap)) dd.jit_adj_cap = cap;
        }
    }
    *out = &(p.dev[dev] = dd);
    return DQ_OK;
}

// One-bit-X groups (X_h times a Z string: the transverse-field terms of an
// Ising Hamiltonian, for one) in register tiles of 2048 amplitudes, lanes on
// physical bits 0..5: the first set takes registers on bits 6..10 and so
// every such term with h < 11, later sets the remaining X bits five at a
// time.  One read of the state per set instead of one per group.  The groups
// move to the end of the group list, after the ones the pair kernels take.
void plan_xtiles(dq_obs_s &o) {
    o.npair = (int)o.groups.size();
    if (o.n < 11) return;
    std::vector<DGroup> pair, single;
    for (const DGroup &g : o.groups) (__builtin_popcountll(g.xmask) == 1 ? single : pair).push_back(g);
    if (single.empty()) return;
    // register bits of each set; the set and tile place of every X bit
    std::vector<std::vector<int>> regsets;
    int set_of[64], pos_of[64];
    bool low = false;
    std::vector<int> high;
    for (const DGroup &g : single) {
        const int h = __builtin_ctzll(g.xmask);
        if (h < 11) low = true;
        else high.push_back(h);   // ascending: groups are sorted by X mask
    }
    if (low) {
        regsets.push_back({6, 7, 8, 9, 10});
        for (int h = 0; h < 11; ++h) {
            set_of[h] = 0;
            pos_of[h] = h;   // lane bit h, or register h - 6 at place 6 + (h - 6)
        }
    }
    for (size_t i = 0; i < high.size(); i += 5) {
        std::vector<int> rb(high.begin() + i, high.begin() + std::min(high.size(), i + 5));
        for (int b = 6; (int)rb.size() < 5; ++b)   // pad with bits below 11 (n >= 11)
            if (std::find(rb.begin(), rb.end(), b) == rb.end()) rb.push_back(b);
        std::sort(rb.begin(), rb.end());
        for (int r = 0; r < 5; ++r)
            if (rb[r] >= 11) {
                set_of[rb[r]] = (int)regsets.size();
                pos_of[rb[r]] = 6 + r;
            }
        regsets.push_back(rb);
    }
    for (size_t k = 0; k < regsets.size(); ++k) {
        std::vector<XTerm> ts;
        for (const DGroup &g : single) {
            const int h = __builtin_ctzll(g.xmask);
            if (set_of[h] != (int)k) continue;
            for (int t = g.t0; t < g.t1; ++t) ts.push_back(XTerm{t, pos_of[h]});
        }
        for (size_t i = 0; i < ts.size(); i += XT_MAX) {
            XSet S{};
            for (int r = 0; r < 5; ++r) S.rb[r] = regsets[k][r];
            S.x0 = (int32_t)o.xterms.size();
            for (size_t q = i; q < std::min(ts.size(), i + (size_t)XT_MAX); ++q) o.xterms.push_back(ts[q]);
            S.x1 = (int32_t)o.xterms.size();
            o.xsets.push_back(S);
        }
    }
    o.groups = pair;
    o.groups.insert(o.groups.end(), single.begin(), single.end());
    o.npair = (int)pair.size();
}

dq_status ensure_obs(dq_obs_s &o, const DGroup **groups, const DTerm **terms) {
    int dev = 0;
    DQ_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(o.mu);
    auto it = o.dev.find(dev);
    if (it == o.dev.end()) {
        std::vector<char> blob;
        o.og = put(blob, o.groups);
        o.ot = put(blob, o.terms);
        o.ox = put(blob, o.xterms);
        void *d = nullptr;
        DQ_HIP(hipMalloc(&d, blob.size()));
        hipError_t e = hipMemcpy(d, blob.data(), blob.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return fail(DQ_ERR_HIP, "observable upload: %s", hipGetErrorString(e));
        }
        it = o.dev.emplace(dev, d).first;
    }
    char *b = (char *)it->second;
    *groups = (const DGroup *)(b + o.og);
    *terms = (const DTerm *)(b + o.ot);
    return DQ_OK;
}

// The pair-kernel groups and tile sets of an expectation or adjoint seed on
// a plan's state: the tile kernels take complex64 states only.
struct ObsRun {
    int32_t ngroups = 0, nxs = 0;
    const XSet *xs = nullptr;
    const XTerm *xt = nullptr;
};
ObsRun obs_run(const dq_plan_s &p, const dq_obs_s &o, const DTerm *terms) {
    ObsRun r;
    const bool tiles = !p.dbl && p.n >= 11 && !o.xsets.empty();
    r.ngroups = tiles ? o.npair : (int32_t)o.groups.size();
    if (tiles) {
        r.nxs = (int32_t)o.xsets.size();
        r.xs = o.xsets.data();
        r.xt = (const XTerm *)((const char *)terms - o.ot + o.ox);
    }
    return r;
}

// ---------------------------------------------------------------- sizes
int64_t expval_blocks(int n, int64_t batch) {
    const int64_t N = int64_t(1) << n;
    int64_t eb = N / (256 * 64);
    const int64_t cap = std::max<int64_t>(1, 2048 / batch);
    eb = std::min(eb, cap);
    return std::max<int64_t>(eb, 1);
}

int64_t grad_waves(const dq_plan_s &p, int64_t batch) {
    int64_t units;
    if (p.R_adj > 0) units = int64_t(1) << (p.n - 6 - p.R_adj);      // tiles per sample
    else units = std::max<int64_t>(1, (int64_t(1) << p.n) / (256 * 16));
    const int64_t cap = std::max<int64_t>(1, 4096 / batch);
    return std::max<int64_t>(1, std::min(units, cap));
}

struct WsLayout {
    size_t mats = 0, expv = 0, zdp = 0, lam = 0, keep = 0, part = 0, total = 0;
};

// terms [t0, t1) of the X-free group when the diagonal kernel takes it
// (group 0 has xmask 0 and the state is at least one 2048-amplitude tile)
bool zdiag_range(const dq_plan_s &p, const dq_obs_s &o, int32_t &t0, int32_t &t1) {
    t0 = t1 = 0;
    if (p.n < 11 || o.groups.empty() || o.groups[0].xmask != 0) return false;
    t0 = o.groups[0].t0;
    t1 = o.groups[0].t1;
    return t0 < t1;
}

WsLayout layout(const dq_plan_s &p, const dq_obs_s *o, int64_t batch, int per_sample, int grad) {
    WsLayout L;
    const size_t amp = p.dbl ? 16 : 8;
    const int64_t bm = per_sample ? batch : 1;
    size_t off = 0;
    L.mats = off;
    off = align256(off + (size_t)bm * (size_t)std::max<int64_t>(p.block, 1) * (p.mdbl ? 16 : 8));
    L.expv = off;
    if (o) off = align256(off + (size_t)batch * expval_blocks(p.n, batch) * std::max<size_t>(o->terms.size(), 1) * 16);
    L.zdp = off;
    if (o) off = align256(off + (size_t)batch * zdiag_blocks(p.n) * o->nobs * 8);
    // lambda starts 256 bytes past a 256-byte boundary: the adjoint reads psi
    // and lambda at the same offsets, and this shift puts the two pieces of
    // each pair on different memory channels (two-state sweeps of a 32-qubit
    // state: about 3 % faster than with both at the same offset modulo 512)
    L.lam = off + (grad ? 256 : 0);
    const size_t sbytes = (size_t)batch * ((size_t)1 << p.n) * amp;
    if (grad) off = align256(L.lam + sbytes);
    L.keep = off;
    if (grad == 2) off = align256(off + sbytes);
    L.part = off;
    if (grad) off = align256(off + (size_t)batch * grad_waves(p, batch) * std::max<int32_t>(p.ngrad, 1) * 8);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- execution
dq_status run_program(dq_plan_s &p, DevData &d, const Program &prog, void *st, void *lam, int64_t batch,
                      const void *mats, int64_t mstride, double *partial, int wps, hipStream_t s, bool timed = true) {
    const double SB = state_bytes(p, batch);
    // consecutive launches of one kind share one pair of timing events, so
    // that profiling adds no work between them
    std::optional<ProfScope> ps;
    for (const Step &S : prog.steps) {
        hipError_t e = hipSuccess;
        const int nst = lam ? 2 : 1;   // states a per-gate sweep touches
        double bytes = 0;
        int kind = DQ_PROF_GATE, nl = nst;
        switch (S.kind) {
        case ST_TILE: kind = lam ? DQ_PROF_ADJ_TILE : DQ_PROF_FWD_TILE; nl = 1; bytes = (lam ? 4 : 2) * SB; break;
        case ST_GRAD: kind = DQ_PROF_GRAD_GATE; nl = 1; bytes = 2 * SB; break;
        case ST_DENSE: kind = DQ_PROF_DENSE; bytes = nst * 2 * SB; break;
        case ST_CNOT: bytes = nst * SB; break;
        case ST_CZ: bytes = nst * SB / 2; break;
        default: bytes = nst * 2 * SB; break;
        }
        if (!ps || ps->kind != kind) {
            if (ps) ps->done();
            ps.emplace(p, kind, 0, 0.0, s, timed);
        }
        ps->nl += nl;
        ps->bytes += bytes;
        ps->flops += S.kind == ST_GRAD ? 3.0 * (double)batch * std::ldexp(1.0, p.n)
                                       : S.flops_per_amp * (double)batch * std::ldexp(1.0, p.n) * (lam ? 2 : 1);
        switch (S.kind) {
        case ST_TILE: {
            TileArgs a{};
            a.st = st;
            a.lam = lam;
            a.n = p.n;
            a.R = S.R;
            for (int i = 0; i < MAX_TILE_R; ++i) a.rbits[i] = S.rbits[i];
            for (int i = 0; i < 3; ++i) a.lbits[i] = S.lbits[i];
            for (int i = 0; i < MAX_TILE_R + 3; ++i) a.tbits[i] = S.tbits[i];
            a.batch = batch;
            a.ops = d.ops + S.op0;
            a.nops = (int32_t)S.nops;
            a.nlslots = (int32_t)S.nls;
            a.mats = mats;
            a.mstride = mstride;
            a.partial = partial;
            a.lslot_gslot = d.lsg + S.ls0;
            a.wps = wps;
            a.ngrad = p.ngrad;
            a.nt = std::ldexp((double)batch * (lam ? 2 : 1) * (p.dbl ? 16 : 8), p.n) > kStreamBytes ? 1 : 0;
            const size_t si = (size_t)(&S - prog.steps.data());
            if (!prog.jk.empty() && prog.jk[si] >= 0 && (size_t)prog.jk[si] < d.jfn.size()) {
                a.mats = (const char *)mats + prog.js0[si] * (p.mdbl ? 16 : 8);
                e = jit_launch(d.jfn[prog.jk[si]], p.jnames[prog.jk[si]], a, lam != nullptr, s);
            } else {
                e = lam ? launch_tile_adj(p.dbl, a, s) : launch_tile_fwd(p.dbl, a, s);
            }
            break;
        }
        case ST_GRAD:
            e = launch_grad_gate(p.dbl, st, lam, p.n, batch, S.gen, S.bits[0], S.bits[1], partial, wps, p.ngrad,
                                 S.gslot, s);
            break;
        default:
            for (int which = 0; which < (lam ? 2 : 1) && e == hipSuccess; ++which) {
                void *x = which ? lam : st;
                switch (S.kind) {
                case ST_G1: e = launch_gate1(p.dbl, x, p.n, batch, S.bits[0], mats, mstride, S.slot, s); break;
                case ST_CNOT: e = launch_cnot(p.dbl, x, p.n, batch, S.bits[0], S.bits[1], s); break;
                case ST_CZ: e = launch_cz(p.dbl, x, p.n, batch, S.bits[0], S.bits[1], s); break;
                case ST_DENSE: e = launch_dense(p.dbl, x, p.n, batch, S.k, S.bits, mats, mstride, S.slot, s); break;
                default: e = launch_gatek(p.dbl, x, p.n, batch, S.k, S.bits, mats, mstride, S.slot, s); break;
                }
            }
            break;
        }
        if (e != hipSuccess) {
            ps->done();
            return fail(DQ_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
        }
    }
    if (ps) ps->done();
    return DQ_OK;
}

dq_status check_batch(const dq_plan_s &p, int64_t batch) {
    if (batch < 1) return fail(DQ_ERR_INVALID_ARG, "batch must be >= 1 (got %lld)", (long long)batch);
    if (batch > 65535) return fail(DQ_ERR_OUT_OF_RANGE, "batch %lld exceeds 65535", (long long)batch);
    const double bytes = (double)batch * std::ldexp(1.0, p.n) * (p.dbl ? 16 : 8);
    if (bytes > 512e9) return fail(DQ_ERR_OUT_OF_RANGE, "batch x 2^n state of %.3g bytes exceeds device memory", bytes);
    return DQ_OK;
}

dq_status check_sources(const dq_plan_s &p, const double *params, int64_t pstride, const double *data, int64_t dstride) {
    if (p.nparams > 0 && !params) return fail(DQ_ERR_INVALID_ARG, "params is NULL but the circuit reads %lld parameters", (long long)p.nparams);
    if (p.ndata > 0 && !data) return fail(DQ_ERR_INVALID_ARG, "data is NULL but the circuit reads %lld data columns", (long long)p.ndata);
    if (pstride != 0 && pstride < p.nparams) return fail(DQ_ERR_INVALID_ARG, "params_bstride %lld < nparams %lld", (long long)pstride, (long long)p.nparams);
    if (dstride != 0 && dstride < p.ndata) return fail(DQ_ERR_INVALID_ARG, "data_bstride %lld < ndata %lld", (long long)dstride, (long long)p.ndata);
    if (pstride < 0 || dstride < 0) return fail(DQ_ERR_INVALID_ARG, "negative batch stride");
    return DQ_OK;
}

// argument checks shared by the two apply entry points (host only)
dq_status check_apply(const dq_plan_s *plan, const void *state, int64_t batch, const double *params,
                      int64_t params_bstride, const double *data, int64_t data_bstride) {
    if (!plan || !state) return fail(DQ_ERR_INVALID_ARG, "NULL plan or state");
    dq_status st = check_batch(*plan, batch);
    if (st != DQ_OK) return st;
    return check_sources(*plan, params, params_bstride, data, data_bstride);
}

// Forward sweep of dq_apply_circuit with the gate-matrix blocks at `mats`:
// prepare the matrices, write the start state, run the tile passes.
dq_status apply_on_device(dq_plan_s &p, DevData &d, void *state, int64_t batch, const double *params,
                          int64_t params_bstride, const double *data, int64_t data_bstride, int32_t from_zero,
                          void *mats, int per_sample, hipStream_t s, bool timed) {
    const bool fold = from_zero && p.has_fold;
    const Program &prog = fold ? p.fwd_fold : p.fwd_full;
    const int64_t bm = per_sample ? batch : 1;
    const int64_t mstride = per_sample ? p.block : 0;
    ProfScope pp(p, DQ_PROF_OTHER, 1, 0.0, s, timed);
    hipError_t e = launch_prepare(p.mdbl, d.gates, d.fixed, d.slots + prog.slot_lo, (int32_t)(prog.slot_hi - prog.slot_lo),
                                  params, params_bstride, data, data_bstride, mats, p.block, bm, s);
    if (e == hipSuccess)
        e = launch_prepare_blocks(p.dbl, d.gates, d.fixed, d.blocks + prog.blk_lo, (int32_t)(prog.blk_hi - prog.blk_lo),
                                  d.factors, params, params_bstride, data, data_bstride, mats, p.block, bm, s);
    pp.done();
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "prepare: %s", hipGetErrorString(e));
    if (from_zero) {
        ProfScope pi(p, DQ_PROF_INIT, 1, state_bytes(p, batch), s, timed);
        if (fold) e = launch_init_product(p.dbl, p.mdbl, state, p.n, batch, mats, mstride, d.fold, s);
        else e = launch_init_zero(p.dbl, state, p.n, batch, s);
        pi.done();
    }
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "init: %s", hipGetErrorString(e));
    return run_program(p, d, prog, state, nullptr, batch, mats, mstride, nullptr, 0, s, timed);
}

// The adjoint sweep of dq_adjoint_grad on a validated call (workspace laid
// out by L at w): seed lambda = sum_o w_o H_o psi, un-apply every gate from
// psi and lambda while summing the gradient terms, then reduce them in a
// fixed order into grad_params / grad_data.
dq_status adjoint_core(dq_plan_s &plan, DevData &d, const dq_obs_s &obs, const DGroup *g, const DTerm *t, void *state,
                       int64_t batch, const double *params, int64_t params_bstride, const double *data,
                       int64_t data_bstride, const double *grad_out, double *grad_params, double *grad_data,
                       int32_t preserve_state, char *w, const WsLayout &L, hipStream_t s) {
    const int per_sample = (params_bstride != 0 || data_bstride != 0) ? 1 : 0;
    void *mats = w + L.mats;
    void *lam = w + L.lam;
    double *partial = (double *)(w + L.part);
    const int64_t bm = per_sample ? batch : 1;
    const int64_t mstride = per_sample ? plan.block : 0;
    // partial sums per sample: at most grad_waves (the workspace size), and
    // no more than the adjoint tile kernel keeps resident, so that one
    // round of waves covers every tile
    int wps = (int)grad_waves(plan, batch);
    if (plan.R_adj > 0) {
        const int resident = d.jit_adj_cap > 0 ? d.jit_adj_cap : tile_adj_capacity(plan.dbl, plan.R_adj);
        const int cap = std::max<int64_t>(1, resident / batch);
        wps = std::min(wps, cap);
    }
    void *psi = state;
    hipError_t e;
    const double SB = state_bytes(plan, batch);
    if (preserve_state) {
        psi = w + L.keep;
        ProfScope pc(plan, DQ_PROF_OTHER, 1, 2 * SB, s);
        e = launch_copy(plan.dbl, psi, state, batch << plan.n, s);
        pc.done();
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "copy: %s", hipGetErrorString(e));
    }
    ProfScope pp(plan, DQ_PROF_OTHER, 1, 0.0, s);
    e = launch_prepare(plan.mdbl, d.gates, d.fixed, d.slots + plan.adj.slot_lo,
                       (int32_t)(plan.adj.slot_hi - plan.adj.slot_lo), params, params_bstride, data, data_bstride,
                       mats, plan.block, bm, s);
    pp.done();
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "prepare: %s", hipGetErrorString(e));
    int32_t dt0, dt1;
    zdiag_range(plan, obs, dt0, dt1);
    const ObsRun orun = obs_run(plan, obs, t);
    ProfScope pl(plan, DQ_PROF_LAMBDA, 1, 2 * SB, s);
    e = launch_lambda(plan.dbl, psi, lam, plan.n, batch, g, orun.ngroups, t, grad_out, obs.nobs, dt0, dt1, orun.xs,
                      orun.nxs, orun.xt, s);
    pl.done();
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "lambda: %s", hipGetErrorString(e));
    dq_status st = run_program(plan, d, plan.adj, psi, lam, batch, mats, mstride, partial, wps, s);
    if (st != DQ_OK) return st;
    ProfScope pf(plan, DQ_PROF_OTHER, 1, 0.0, s);
    if (plan.nparams > 0) {
        e = launch_grad_final(partial, batch, wps, plan.ngrad, d.poff, d.pg, d.pf, plan.nparams,
                              params_bstride != 0 ? 1 : 0, grad_params, s);
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "grad reduce: %s", hipGetErrorString(e));
    }
    if (grad_data && plan.ndata > 0) {
        e = launch_grad_final(partial, batch, wps, plan.ngrad, d.doff, d.dg, d.df, plan.ndata,
                              data_bstride != 0 ? 1 : 0, grad_data, s);
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "grad reduce: %s", hipGetErrorString(e));
    }
    pf.done();
    return DQ_OK;
}

// ---------------------------------------------------------------- Hessian
// The derived plan of dq_hessian: the same expanded gates, occurrence k
// (the k-th gate angle that reads a parameter) reading parameter k with
// scale 1, so that a batch row of angles can shift one occurrence alone and
// the adjoint returns the gradient with respect to every occurrence's angle.
dq_status ensure_hess_plan(dq_plan_s &p, dq_plan_s **out) {
    std::lock_guard<std::mutex> lk(p.hmu);
    if (!p.hess) {
        std::unique_ptr<dq_plan_s> q(new dq_plan_s());
        q->n = p.n;
        q->dbl = p.dbl;
        q->mdbl = p.mdbl;
        q->opt = p.opt;
        q->nparams = (int64_t)p.occ_param.size();
        q->ndata = p.ndata;
        q->fixed = p.fixed;
        q->gates = p.canon;
        int64_t k = 0;
        for (DGate &g : q->gates)
            if (g.src == SRC_PARAM) {
                g.idx = k++;
                g.scale = 1.0;
            }
        q->user_gates = (int64_t)q->gates.size();
        q->canon = q->gates;
        dq_status st = build_plan(*q);
        if (st != DQ_OK) return st;
        if (q->opt.layout == 0) q.reset(search_layout(q.release()));
        balance_adjoint(*q);
        if (q->opt.jit) jit_generate(*q);
        if (q->opt.arith64 && !all_compiled(*q))
            return fail(DQ_ERR_UNSUPPORTED, "arith64: a step of the derived plan is not a compiled tile pass");
        p.hess = std::move(q);
    }
    *out = p.hess.get();
    return DQ_OK;
}

// occurrences shifted per batch: all (max_shifts = 0) or max_shifts, within
// the batch limit (two shifted circuits per occurrence)
dq_status hess_shifts(const dq_plan_s &p, int32_t max_shifts, int64_t &m) {
    if (max_shifts < 0) return fail(DQ_ERR_INVALID_ARG, "max_shifts %d is negative", max_shifts);
    const int64_t K = std::max<int64_t>((int64_t)p.occ_param.size(), 1);
    m = max_shifts == 0 ? K : std::min<int64_t>(max_shifts, K);
    if (2 * m > 65535) return fail(DQ_ERR_OUT_OF_RANGE, "%lld shifts per batch exceed 32767", (long long)m);
    return check_batch(p, 2 * m);
}

struct HessLayout {
    size_t rows = 0, grads = 0, wts = 0, states = 0, sub = 0, total = 0;
};

HessLayout hess_layout(const dq_plan_s &p, const dq_plan_s &h, const dq_obs_s *o, int64_t m) {
    HessLayout L;
    const int64_t K = std::max<int64_t>((int64_t)p.occ_param.size(), 1), B = 2 * m;
    size_t off = 0;
    L.rows = off;
    off = align256(off + (size_t)(B * K) * 8);
    L.grads = off;
    off = align256(off + (size_t)(B * K) * 8);
    L.wts = off;
    off = align256(off + (size_t)(B * std::max(o->nobs, 1)) * 8);
    L.states = off;
    off = align256(off + (size_t)B * ((size_t)1 << p.n) * (p.dbl ? 16 : 8));
    L.sub = off;
    off += layout(h, o, B, 1, 1).total;
    L.total = off;
    return L;
}

// Device address of `scratch` on the current device, looked up with
// hipGetSymbolAddress on the first call per device (with that device
// current) and kept in a fixed table, so later calls allocate nothing.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

dq_status noalloc_scratch(void **out) {
    int dev = 0;
    DQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DQ_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DQ_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DQ_OK;
}

// the plan's device tables and compiled passes on the current device, if
// an earlier call has put them there (nothing is uploaded or compiled here)
dq_status resident_device(dq_plan_s &p, DevData **out) {
    int dev = 0;
    DQ_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(p.mu);
    const auto it = p.dev.find(dev);
    if (it == p.dev.end())
        return fail(DQ_ERR_INVALID_ARG, "plan not yet resident on device %d: call dq_apply_circuit with it once first", dev);
    *out = &it->second;
    return DQ_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char *dq_last_error(void) { return g_err.c_str(); }
int32_t dq_version(void) { return DQ_VERSION; }

dq_status dq_plan_create(dq_plan *out, int32_t nqubits, const dq_gate *gates, int64_t ngates, int64_t nparams,
                         int64_t ndata, dq_dtype dtype, const dq_options *opt) try {
    if (!out) return fail(DQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nqubits < 1 || nqubits > DQ_MAX_QUBITS)
        return fail(DQ_ERR_OUT_OF_RANGE, "nqubits %d outside 1..%d", nqubits, DQ_MAX_QUBITS);
    if (ngates < 0 || (ngates > 0 && !gates)) return fail(DQ_ERR_INVALID_ARG, "bad gate list");
    if (ngates > (1 << 24)) return fail(DQ_ERR_OUT_OF_RANGE, "too many gates (%lld)", (long long)ngates);
    if (nparams < 0 || ndata < 0) return fail(DQ_ERR_INVALID_ARG, "negative nparams / ndata");
    if (dtype != DQ_C64 && dtype != DQ_C128) return fail(DQ_ERR_UNSUPPORTED, "dtype %d", (int)dtype);
    dq_options o{1, 0, 1, 0, 0, 0, 0, 0, 0};
    if (opt) o = *opt;
    if (o.arith64 != 0 && o.arith64 != 1) return fail(DQ_ERR_INVALID_ARG, "arith64 must be 0 or 1 (got %d)", o.arith64);
    if (o.arith64 && (dtype != DQ_C64 || !o.jit || !o.fusion || o.dense_fuse))
        return fail(DQ_ERR_UNSUPPORTED, "arith64 needs a complex64 plan with jit = 1, fusion = 1 and dense_fuse = 0");
    if (o.low_bits < 0 || o.low_bits > 3) return fail(DQ_ERR_INVALID_ARG, "low_bits %d outside 0..3", o.low_bits);
    if (o.layout != 0 && o.layout != 1) return fail(DQ_ERR_INVALID_ARG, "layout must be 0 or 1 (got %d)", o.layout);
    if (o.adj_tile_bits < 0 || o.adj_tile_bits > (dtype == DQ_C128 ? 4 : 5))
        return fail(DQ_ERR_INVALID_ARG, "adj_tile_bits %d outside 0..%d", o.adj_tile_bits, dtype == DQ_C128 ? 4 : 5);
    if (o.jit != 0 && o.jit != 1) return fail(DQ_ERR_INVALID_ARG, "jit must be 0 or 1 (got %d)", o.jit);
    if (o.tile_bits < 0 || o.tile_bits > 6) return fail(DQ_ERR_INVALID_ARG, "tile_bits %d outside 0..6", o.tile_bits);
    if (o.dense_fuse != 0 && o.dense_fuse != 4 && o.dense_fuse != 5)
        return fail(DQ_ERR_INVALID_ARG, "dense_fuse must be 0, 4 or 5 (got %d)", o.dense_fuse);
    std::unique_ptr<dq_plan_s> p(new dq_plan_s());
    p->n = nqubits;
    p->dbl = dtype == DQ_C128;
    p->mdbl = p->dbl || o.arith64;
    p->opt = o;
    p->nparams = nparams;
    p->ndata = ndata;
    for (int64_t g = 0; g < ngates; ++g) {
        const dq_gate &G = gates[g];
        if (G.op < DQ_OP_H || G.op > DQ_OP_CRZ) {
            return fail(DQ_ERR_INVALID_ARG, "gate %lld: unknown op %d", (long long)g, G.op);
        }
        const int a = arity(G.op);
        if ((a > 0 && G.nq != a) || (a < 0 && (G.nq < 1 || G.nq > DQ_MAX_GATE_QUBITS))) {
            return fail(DQ_ERR_INVALID_ARG, "gate %lld: op %d with %d wires", (long long)g, G.op, G.nq);
        }
        for (int i = 0; i < G.nq; ++i) {
            if (G.wires[i] < 0 || G.wires[i] >= nqubits) {
                return fail(DQ_ERR_INVALID_ARG, "gate %lld: wire %d outside 0..%d", (long long)g, G.wires[i], nqubits - 1);
            }
            for (int j = 0; j < i; ++j)
                if (G.wires[j] == G.wires[i]) {
                    return fail(DQ_ERR_INVALID_ARG, "gate %lld: wire %d repeated", (long long)g, G.wires[i]);
                }
        }
        if (G.src < DQ_SRC_NONE || G.src > DQ_SRC_DATA) {
            return fail(DQ_ERR_INVALID_ARG, "gate %lld: bad angle source %d", (long long)g, G.src);
        }
        if (G.src != DQ_SRC_NONE && !is_rotation(G.op)) {
            return fail(DQ_ERR_INVALID_ARG, "gate %lld: op %d takes no angle", (long long)g, G.op);
        }
        const int64_t nang = G.op == DQ_OP_U3 ? 3 : 1;   // U3 reads idx, idx+1, idx+2
        if ((G.src == DQ_SRC_PARAM && (G.idx < 0 || G.idx > nparams - nang)) ||
            (G.src == DQ_SRC_DATA && (G.idx < 0 || G.idx > ndata - nang))) {
            return fail(DQ_ERR_INVALID_ARG, "gate %lld: source index %lld out of range", (long long)g, (long long)G.idx);
        }
        if (!std::isfinite(G.scale)) {
            return fail(DQ_ERR_INVALID_ARG, "gate %lld: non-finite scale", (long long)g);
        }
        DGate D{};
        D.op = G.op;
        D.nq = G.nq;
        for (int i = 0; i < G.nq; ++i) D.bits[i] = nqubits - 1 - G.wires[i];
        D.src = G.src;
        D.idx = G.idx;
        D.scale = G.scale;
        D.mat_off = -1;
        if (G.op == DQ_OP_RXX || G.op == DQ_OP_RYY) {
            // exp(-i t P(x)P / 2) = (V(x)V)^dagger exp(-i t Z(x)Z / 2) (V(x)V) with
            // V Z-diagonalising P: H for X (H Z H = X), RX(pi/2) for Y
            // (RX(pi/2)^dagger Z RX(pi/2) = Y); the RZZ carries the angle and
            // its gradient, the basis changes are fixed
            auto basis = [&](double sign) {
                for (int i = 0; i < 2; ++i) {
                    DGate B{};
                    B.op = G.op == DQ_OP_RXX ? OP_H : OP_RX;
                    B.nq = 1;
                    B.bits[0] = D.bits[i];
                    B.src = SRC_NONE;
                    B.scale = G.op == DQ_OP_RXX ? 0.0 : sign * M_PI / 2;
                    B.mat_off = -1;
                    p->gates.push_back(B);
                }
            };
            basis(1.0);
            D.op = OP_RZZ;
            p->gates.push_back(D);
            basis(-1.0);
            continue;
        }
        if (G.op == DQ_OP_U3) {
            // U3(theta, phi, lambda) = P(phi) RY(theta) P(lambda) with the phase
            // gate P(t) = diag(1, e^{it}): the product's entries are those of U3
            // exactly (no global phase), and each factor carries one angle and
            // its gradient slot (theta at idx, phi at idx+1, lambda at idx+2)
            const int64_t k_of[3] = {2, 0, 1};
            const int op_of[3] = {OP_PHASE, OP_RY, OP_PHASE};
            for (int i = 0; i < 3; ++i) {
                DGate F = D;
                F.op = op_of[i];
                F.idx = G.src == DQ_SRC_NONE ? G.idx : G.idx + k_of[i];
                p->gates.push_back(F);
            }
            continue;
        }
        if (G.op == DQ_OP_CRX || G.op == DQ_OP_CRY || G.op == DQ_OP_CRZ) {
            // controlled R(t) on (c, t) = E R(-t/2) E R(t/2) with E = CNOT(c, t)
            // for RY and RZ (X R(a) X = R(-a)) and E = CZ(c, t) for RX
            // (Z RX(a) Z = RX(-a)): where the control is 0 the two halves
            // cancel, where it is 1 they add.  Both halves read the gate's
            // angle source with half its scale, so its gradient is the sum of
            // theirs (chain factors +1/2 and -1/2)
            const int rop = G.op == DQ_OP_CRX ? OP_RX : (G.op == DQ_OP_CRY ? OP_RY : OP_RZ);
            DGate E{};
            E.op = G.op == DQ_OP_CRX ? OP_CZ : OP_CNOT;
            E.nq = 2;
            E.bits[0] = D.bits[0];
            E.bits[1] = D.bits[1];
            E.src = SRC_NONE;
            E.mat_off = -1;
            for (int h = 0; h < 2; ++h) {
                DGate R = D;
                R.op = rop;
                R.nq = 1;
                R.bits[0] = D.bits[1];
                R.bits[1] = 0;
                R.scale = (h ? -0.5 : 0.5) * G.scale;
                p->gates.push_back(R);
                p->gates.push_back(E);
            }
            continue;
        }
        if (G.op == DQ_OP_UNITARY) {
            if (!G.matrix) {
                return fail(DQ_ERR_INVALID_ARG, "gate %lld: UNITARY without a matrix", (long long)g);
            }
            const int dim = 1 << G.nq;
            D.mat_off = (int64_t)p->fixed.size();
            for (int i = 0; i < dim * dim; ++i) p->fixed.push_back(double2{G.matrix[2 * i], G.matrix[2 * i + 1]});
        }
        p->gates.push_back(D);
    }
    p->user_gates = (int64_t)p->gates.size();
    p->canon = p->gates;
    {
        std::vector<std::vector<int32_t>> by_param((size_t)nparams);
        for (const DGate &D : p->canon)
            if (D.src == SRC_PARAM) {
                by_param[(size_t)D.idx].push_back((int32_t)p->occ_param.size());
                p->occ_param.push_back((int32_t)D.idx);
                p->occ_scale.push_back(D.scale);
            }
        p->hoff.assign((size_t)nparams + 1, 0);
        for (int64_t i = 0; i < nparams; ++i) {
            p->hoff[(size_t)i + 1] = p->hoff[(size_t)i] + (int64_t)by_param[(size_t)i].size();
            p->hocc.insert(p->hocc.end(), by_param[(size_t)i].begin(), by_param[(size_t)i].end());
        }
    }
    dq_status st = build_plan(*p);
    if (st != DQ_OK) {
        return st;
    }
    if (o.layout == 0) p.reset(search_layout(p.release()));
    balance_adjoint(*p);
    if (o.jit) jit_generate(*p);
    if (o.arith64 && !all_compiled(*p))
        return fail(DQ_ERR_UNSUPPORTED, "arith64: a step of this plan is not a compiled tile pass");
    *out = p.release();
    return ok();
} DQ_CATCH

void dq_plan_destroy(dq_plan plan) try {
    if (!plan) return;
    for (dq_plan_s *q : {plan->hess.get(), plan}) {   // the Hessian's derived plan, then the plan
        if (!q) continue;
        for (hipEvent_t e : q->evpool) (void)hipEventDestroy(e);
        for (auto &kv : q->dev) {
            int cur = 0;
            if (hipGetDevice(&cur) == hipSuccess) {
                (void)hipSetDevice(kv.first);
                (void)hipFree(kv.second.blob);
                (void)hipSetDevice(cur);
            }
        }
    }
    delete plan;
} DQ_CATCH_VOID

dq_status dq_plan_get_stats(dq_plan plan, dq_plan_stats *out) try {
    if (!plan || !out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    dq_plan_stats s{};
    s.nqubits = plan->n;
    s.dtype = plan->dbl ? DQ_C128 : DQ_C64;
    s.ngates = plan->user_gates;
    const Program &f = plan->has_fold ? plan->fwd_fold : plan->fwd_full;
    s.fwd_steps = (int64_t)f.steps.size() + (plan->has_fold ? 1 : 0);
    s.fwd_tile_passes = f.tile_passes;
    s.fwd_dense_blocks = f.dense_steps;
    s.adj_steps = (int64_t)plan->adj.steps.size();
    s.folded_gates = plan->folded_gates;
    s.grad_gates = plan->ngrad;
    s.tile_bits = plan->R_fwd;
    s.adj_tile_bits = plan->R_adj;
    s.layout_swaps = plan->layout_swaps;
    for (int which = 0; which < 2; ++which) {
        const Program &prog = which ? plan->adj : f;
        for (const Step &S : prog.steps) {
            if (S.kind != ST_TILE) continue;
            for (int64_t k = 0; k < S.nops; ++k) {
                const TOp &o = plan->ops[(size_t)(S.op0 + k)];
                if (o.kind < 0 || o.kind > 7) continue;
                // the bit the operation exchanges amplitudes over (none for diagonals)
                int tq = o.q0;
                if (o.kind == TK_CNOT) tq = o.q1;
                if (o.kind == TK_SWAP) tq = std::min(o.q0, o.q1);
                const bool diag = o.kind == TK_1QDIAG || o.kind == TK_CZ || o.kind == TK_2QDIAG;
                s.tile_ops[which][(!diag && tq < 6) ? 0 : 1][o.kind] += 1;
            }
        }
    }
    *out = s;
    return ok();
} DQ_CATCH

dq_status dq_plan_describe(dq_plan plan, char *buf, size_t cap, size_t *needed) try {
    if (!plan) return fail(DQ_ERR_INVALID_ARG, "NULL plan");
    std::string t;
    char line[256];
    const Program &f = plan->has_fold ? plan->fwd_fold : plan->fwd_full;
    for (int which = 0; which < 2; ++which) {
        const Program &prog = which ? plan->adj : f;
        for (size_t k = 0; k < prog.steps.size(); ++k) {
            const Step &S = prog.steps[k];
            if (S.kind == ST_TILE) {
                snprintf(line, sizeof line, "%s %zu tile R=%d lbits=%d,%d,%d rbits=", which ? "adj" : "fwd", k, S.R,
                         S.lbits[0], S.lbits[1], S.lbits[2]);
                t += line;
                for (int i = 0; i < S.R; ++i) t += std::to_string(S.rbits[i]) + (i + 1 < S.R ? "," : "");
                if (k < prog.jk.size() && prog.jk[k] >= 0) t += " kernel=" + plan->jnames[(size_t)prog.jk[k]];
                t += " ops=";
                for (int64_t i = 0; i < S.nops; ++i) {
                    const TOp &o = plan->ops[(size_t)(S.op0 + i)];
                    snprintf(line, sizeof line, "%s%d:%d:%d:%d:%d:%d", i ? ";" : "", o.kind, o.q0, o.q1, o.gen, o.slot,
                             o.lslot);
                    t += line;
                }
                t += "\n";
            } else {
                snprintf(line, sizeof line, "%s %zu sweep kind=%d k=%d bits=%d,%d,%d,%d,%d slot=%lld gen=%d gslot=%d\n",
                         which ? "adj" : "fwd", k, S.kind, S.k, S.bits[0], S.bits[1], S.bits[2], S.bits[3], S.bits[4],
                         (long long)S.slot, S.gen, S.gslot);
                t += line;
            }
        }
    }
    if (needed) *needed = t.size() + 1;
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, t.size());
        memcpy(buf, t.data(), n);
        buf[n] = 0;
    }
    return ok();
} DQ_CATCH

dq_status dq_plan_jit_source(dq_plan plan, int32_t index, char *buf, size_t cap, size_t *needed, int32_t *count) try {
    if (!plan) return fail(DQ_ERR_INVALID_ARG, "NULL plan");
    if (count) *count = (int32_t)plan->jsrcs.size();
    if (index < 0) return ok();
    if ((size_t)index >= plan->jsrcs.size())
        return fail(DQ_ERR_OUT_OF_RANGE, "pass kernel %d of %zu", index, plan->jsrcs.size());
    const std::string &t = plan->jsrcs[(size_t)index];
    if (needed) *needed = t.size() + 1;
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, t.size());
        memcpy(buf, t.data(), n);
        buf[n] = 0;
    }
    return ok();
} DQ_CATCH

dq_status dq_obs_create(dq_obs *out, int32_t nqubits, const dq_pauli_term *terms, const int64_t *obs_offsets,
                        int32_t nobs) try {
    if (!out) return fail(DQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nqubits < 1 || nqubits > DQ_MAX_QUBITS) return fail(DQ_ERR_OUT_OF_RANGE, "nqubits %d", nqubits);
    if (nobs < 1 || !obs_offsets) return fail(DQ_ERR_INVALID_ARG, "need nobs >= 1 and obs_offsets");
    if (obs_offsets[0] != 0) return fail(DQ_ERR_INVALID_ARG, "obs_offsets[0] must be 0");
    for (int o = 0; o < nobs; ++o)
        if (obs_offsets[o + 1] < obs_offsets[o]) return fail(DQ_ERR_INVALID_ARG, "obs_offsets not ascending");
    const int64_t nterms = obs_offsets[nobs];
    if (nterms > 0 && !terms) return fail(DQ_ERR_INVALID_ARG, "terms is NULL");
    if (nterms > (1 << 20)) return fail(DQ_ERR_OUT_OF_RANGE, "too many terms");
    const uint64_t valid = nqubits >= 64 ? ~0ull : ((1ull << nqubits) - 1);
    std::unique_ptr<dq_obs_s> o(new dq_obs_s());
    o->n = nqubits;
    o->nobs = nobs;
    struct Tm { uint64_t x, z; double c; int obs; };
    std::vector<Tm> all;
    for (int ob = 0; ob < nobs; ++ob)
        for (int64_t t = obs_offsets[ob]; t < obs_offsets[ob + 1]; ++t) {
            const dq_pauli_term &T = terms[t];
            if ((T.xmask | T.zmask) & ~valid) {
                return fail(DQ_ERR_INVALID_ARG, "term %lld touches a wire >= %d", (long long)t, nqubits);
            }
            if (!std::isfinite(T.coef)) {
                return fail(DQ_ERR_INVALID_ARG, "term %lld: non-finite coefficient", (long long)t);
            }
            uint64_t px = 0, pz = 0;   // wire w -> physical bit n-1-w
            for (int w = 0; w < nqubits; ++w) {
                if (T.xmask >> w & 1) px |= 1ull << (nqubits - 1 - w);
                if (T.zmask >> w & 1) pz |= 1ull << (nqubits - 1 - w);
            }
            all.push_back({px, pz, T.coef, ob});
        }
    // grouped by X mask (one pass over the state per group), and within a
    // group by observable (the diagonal kernel sums one observable's run)
    std::stable_sort(all.begin(), all.end(),
                     [](const Tm &a, const Tm &b) { return a.x != b.x ? a.x < b.x : a.obs < b.obs; });
    for (size_t i = 0; i < all.size(); ++i) {
        if (o->groups.empty() || o->groups.back().xmask != all[i].x)
            o->groups.push_back(DGroup{all[i].x, (int32_t)i, (int32_t)i});
        o->groups.back().t1 = (int32_t)i + 1;
        const int ny = __builtin_popcountll(all[i].x & all[i].z) & 3;   // i^{nY}
        const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
        o->terms.push_back(DTerm{all[i].z, all[i].c * re[ny], all[i].c * im[ny], all[i].obs, 0});
    }
    plan_xtiles(*o);
    *out = o.release();
    return ok();
} DQ_CATCH

void dq_obs_destroy(dq_obs obs) try {
    if (!obs) return;
    for (auto &kv : obs->dev) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess) {
            (void)hipSetDevice(kv.first);
            (void)hipFree(kv.second);
            (void)hipSetDevice(cur);
        }
    }
    delete obs;
} DQ_CATCH_VOID

dq_status dq_workspace_size(dq_plan plan, dq_obs obs, int64_t batch, int32_t per_sample, int32_t grad, size_t *bytes) try {
    if (!plan || !bytes) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (grad < 0 || grad > 2) return fail(DQ_ERR_INVALID_ARG, "grad must be 0, 1 or 2");
    if (grad && !obs) return fail(DQ_ERR_INVALID_ARG, "the adjoint needs an observable");
    dq_status st = check_batch(*plan, batch);
    if (st != DQ_OK) return st;
    *bytes = layout(*plan, obs, batch, per_sample ? 1 : 0, grad).total;
    return ok();
} DQ_CATCH

dq_status dq_state_init(dq_plan plan, void *state, int64_t batch, const void *init, void *stream) try {
    if (!plan || !state) return fail(DQ_ERR_INVALID_ARG, "NULL plan or state");
    dq_status st = check_batch(*plan, batch);
    if (st != DQ_OK) return st;
    hipError_t e = init ? launch_init_copy(plan->dbl, state, init, plan->n, batch, (hipStream_t)stream)
                        : launch_init_zero(plan->dbl, state, plan->n, batch, (hipStream_t)stream);
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "state init: %s", hipGetErrorString(e));
    return ok();
} DQ_CATCH

dq_status dq_apply_circuit(dq_plan plan, void *state, int64_t batch, const double *params, int64_t params_bstride,
                           const double *data, int64_t data_bstride, int32_t from_zero, void *ws, size_t ws_bytes,
                           void *stream) try {
    dq_status st = check_apply(plan, state, batch, params, params_bstride, data, data_bstride);
    if (st != DQ_OK) return st;
    const int per_sample = (params_bstride != 0 || data_bstride != 0) ? 1 : 0;
    const WsLayout L = layout(*plan, nullptr, batch, per_sample, 0);
    if (!ws || ws_bytes < L.total)
        return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws ? ws_bytes : 0);
    DevData *d = nullptr;
    if ((st = ensure_device(*plan, &d)) != DQ_OK) return st;
    if ((st = apply_on_device(*plan, *d, state, batch, params, params_bstride, data, data_bstride, from_zero,
                              (char *)ws + L.mats, per_sample, (hipStream_t)stream, true)) != DQ_OK)
        return st;
    return ok();
} DQ_CATCH

dq_status dq_apply_circuit_noalloc(dq_plan plan, void *state, int64_t batch, const double *params,
                                   int64_t params_bstride, const double *data, int64_t data_bstride, int32_t from_zero,
                                   void *stream) try {
    dq_status st = check_apply(plan, state, batch, params, params_bstride, data, data_bstride);
    if (st != DQ_OK) return st;
    const int per_sample = (params_bstride != 0 || data_bstride != 0) ? 1 : 0;
    const WsLayout L = layout(*plan, nullptr, batch, per_sample, 0);
    if (L.total > (size_t)DQ_NOALLOC_SCRATCH_BYTES)
        return fail(DQ_ERR_OUT_OF_RANGE, "gate matrices of %zu bytes exceed the %zu-byte scratch; use dq_apply_circuit",
                    L.total, (size_t)DQ_NOALLOC_SCRATCH_BYTES);
    DevData *d = nullptr;
    if ((st = resident_device(*plan, &d)) != DQ_OK) return st;
    void *scr = nullptr;
    if ((st = noalloc_scratch(&scr)) != DQ_OK) return st;
    // every matrix slot the passes read is written by the prepare kernel
    // first, so the scratch needs no clearing; no timing events are made
    if ((st = apply_on_device(*plan, *d, state, batch, params, params_bstride, data, data_bstride, from_zero,
                              (char *)scr + L.mats, per_sample, (hipStream_t)stream, false)) != DQ_OK)
        return st;
    return ok();
} DQ_CATCH

dq_status dq_expval(dq_plan plan, dq_obs obs, const void *state, int64_t batch, double *out, void *ws,
                    size_t ws_bytes, void *stream) try {
    if (!plan || !obs || !state || !out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (obs->n != plan->n) return fail(DQ_ERR_INVALID_ARG, "observable is for %d qubits, plan for %d", obs->n, plan->n);
    dq_status st = check_batch(*plan, batch);
    if (st != DQ_OK) return st;
    const WsLayout L = layout(*plan, obs, batch, 0, 0);
    if (!ws || ws_bytes < L.total)
        return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws ? ws_bytes : 0);
    const DGroup *g = nullptr;
    const DTerm *t = nullptr;
    if ((st = ensure_obs(*obs, &g, &t)) != DQ_OK) return st;
    const int eb = (int)expval_blocks(plan->n, batch);
    int32_t dt0, dt1;
    if (!zdiag_range(*plan, *obs, dt0, dt1) || obs->nobs > ZD_MAXOBS) dt0 = dt1 = 0;
    const ObsRun orun = obs_run(*plan, *obs, t);
    ProfScope pe(*plan, DQ_PROF_EXPVAL, 2, state_bytes(*plan, batch) * (double)(orun.ngroups + orun.nxs),
                 (hipStream_t)stream);
    hipError_t e = launch_expval(plan->dbl, state, plan->n, batch, g, orun.ngroups, t, (int32_t)obs->terms.size(),
                                 obs->nobs, (double *)((char *)ws + L.expv), eb, out, dt0, dt1,
                                 (double *)((char *)ws + L.zdp), orun.xs, orun.nxs, orun.xt, (hipStream_t)stream);
    pe.done();
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "expval: %s", hipGetErrorString(e));
    return ok();
} DQ_CATCH

namespace {
// blocks per outcome of the probability reduction
int64_t probs_blocks(const dq_plan_s &p, int32_t nwires) {
    const int64_t per = int64_t(1) << (p.n - nwires);
    return (per + PROB_CHUNK - 1) / PROB_CHUNK;
}
}  // namespace

dq_status dq_probs_workspace_size(dq_plan plan, int64_t batch, int32_t nwires, size_t *bytes) try {
    if (!plan || !bytes) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    dq_status st = check_batch(*plan, batch);
    if (st != DQ_OK) return st;
    if (nwires < 1 || nwires > PROB_MAXW || nwires > plan->n)
        return fail(DQ_ERR_INVALID_ARG, "nwires %d outside 1..%d", nwires, std::min(PROB_MAXW, (int)plan->n));
    *bytes = align256((size_t)batch * ((size_t)1 << nwires) * (size_t)probs_blocks(*plan, nwires) * sizeof(double));
    return ok();
} DQ_CATCH

dq_status dq_probs(dq_plan plan, const void *state, int64_t batch, const int32_t *wires, int32_t nwires, double *out,
                   void *ws, size_t ws_bytes, void *stream) try {
    if (!plan || !state || !wires || !out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    size_t need = 0;
    dq_status st = dq_probs_workspace_size(plan, batch, nwires, &need);
    if (st != DQ_OK) return st;
    ProbArgs a{};
    a.n = plan->n;
    a.k = nwires;
    uint64_t seen = 0;
    for (int i = 0; i < nwires; ++i) {
        if (wires[i] < 0 || wires[i] >= plan->n)
            return fail(DQ_ERR_INVALID_ARG, "wire %d outside 0..%d", wires[i], plan->n - 1);
        if ((seen >> wires[i]) & 1) return fail(DQ_ERR_INVALID_ARG, "wire %d listed twice", wires[i]);
        seen |= 1ull << wires[i];
        a.pb[i] = plan->n - 1 - wires[i];   // wire w -> physical bit n-1-w
        a.asc[i] = a.pb[i];
    }
    std::sort(a.asc, a.asc + nwires);
    if (!ws || ws_bytes < need)
        return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
    ProfScope pr(*plan, DQ_PROF_OTHER, 2, state_bytes(*plan, batch), (hipStream_t)stream);
    const hipError_t e = launch_probs(plan->dbl, state, batch, a, (double *)ws, probs_blocks(*plan, nwires), out,
                                      (hipStream_t)stream);
    pr.done();
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "probs: %s", hipGetErrorString(e));
    return ok();
} DQ_CATCH

dq_status dq_sample(const double *p, int64_t batch, int32_t nout, const double *u, int32_t shots, int64_t *out,
                    void *stream) try {
    if (!p || !u || !out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (batch < 1 || batch > 65535) return fail(DQ_ERR_OUT_OF_RANGE, "batch %lld outside 1..65535", (long long)batch);
    if (nout < 1 || nout > (1 << 20)) return fail(DQ_ERR_INVALID_ARG, "nout %d outside 1..2^20", nout);
    if (shots < 0) return fail(DQ_ERR_INVALID_ARG, "shots %d is negative", shots);
    if (shots == 0) return ok();
    const hipError_t e = launch_sample(p, batch, nout, u, shots, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "sample: %s", hipGetErrorString(e));
    return ok();
} DQ_CATCH

dq_status dq_adjoint_grad(dq_plan plan, dq_obs obs, void *state, int64_t batch, const double *params,
                          int64_t params_bstride, const double *data, int64_t data_bstride, const double *grad_out,
                          double *grad_params, double *grad_data, int32_t preserve_state, void *ws, size_t ws_bytes,
                          void *stream) try {
    if (!plan || !obs || !state || !grad_out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (obs->n != plan->n) return fail(DQ_ERR_INVALID_ARG, "observable is for %d qubits, plan for %d", obs->n, plan->n);
    if (plan->nparams > 0 && !grad_params) return fail(DQ_ERR_INVALID_ARG, "grad_params is NULL");
    dq_status st = check_batch(*plan, batch);
    if (st != DQ_OK) return st;
    if ((st = check_sources(*plan, params, params_bstride, data, data_bstride)) != DQ_OK) return st;
    const int per_sample = (params_bstride != 0 || data_bstride != 0) ? 1 : 0;
    const int grad = preserve_state ? 2 : 1;
    const WsLayout L = layout(*plan, obs, batch, per_sample, grad);
    if (!ws || ws_bytes < L.total)
        return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws ? ws_bytes : 0);
    DevData *d = nullptr;
    if ((st = ensure_device(*plan, &d)) != DQ_OK) return st;
    const DGroup *g = nullptr;
    const DTerm *t = nullptr;
    if ((st = ensure_obs(*obs, &g, &t)) != DQ_OK) return st;
    if ((st = adjoint_core(*plan, *d, *obs, g, t, state, batch, params, params_bstride, data, data_bstride, grad_out,
                           grad_params, grad_data, preserve_state, (char *)ws, L, (hipStream_t)stream)) != DQ_OK)
        return st;
    return ok();
} DQ_CATCH

dq_status dq_hessian_workspace_size(dq_plan plan, dq_obs obs, int32_t max_shifts, size_t *bytes) try {
    if (!plan || !obs || !bytes) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (obs->n != plan->n) return fail(DQ_ERR_INVALID_ARG, "observable is for %d qubits, plan for %d", obs->n, plan->n);
    dq_plan_s *h = nullptr;
    dq_status st = ensure_hess_plan(*plan, &h);
    if (st != DQ_OK) return st;
    int64_t m = 0;
    if ((st = hess_shifts(*plan, max_shifts, m)) != DQ_OK) return st;
    *bytes = hess_layout(*plan, *h, obs, m).total;
    return ok();
} DQ_CATCH

dq_status dq_hessian(dq_plan plan, dq_obs obs, const double *params, const double *data, const double *weights,
                     double *hess, int32_t max_shifts, void *ws, size_t ws_bytes, void *stream) try {
    if (!plan || !obs || !weights || !hess) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (obs->n != plan->n) return fail(DQ_ERR_INVALID_ARG, "observable is for %d qubits, plan for %d", obs->n, plan->n);
    if (plan->nparams < 1) return fail(DQ_ERR_INVALID_ARG, "the circuit reads no parameters");
    dq_status st = check_sources(*plan, params, 0, data, 0);
    if (st != DQ_OK) return st;
    dq_plan_s *h = nullptr;
    if ((st = ensure_hess_plan(*plan, &h)) != DQ_OK) return st;
    int64_t m = 0;
    if ((st = hess_shifts(*plan, max_shifts, m)) != DQ_OK) return st;
    const HessLayout HL = hess_layout(*plan, *h, obs, m);
    if (!ws || ws_bytes < HL.total)
        return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", HL.total, ws ? ws_bytes : 0);
    DevData *d = nullptr, *dh = nullptr;
    if ((st = ensure_device(*plan, &d)) != DQ_OK) return st;
    if ((st = ensure_device(*h, &dh)) != DQ_OK) return st;
    const DGroup *g = nullptr;
    const DTerm *t = nullptr;
    if ((st = ensure_obs(*obs, &g, &t)) != DQ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    const int64_t K = (int64_t)plan->occ_param.size(), P = plan->nparams;
    double *rows = (double *)(w + HL.rows), *G = (double *)(w + HL.grads), *go = (double *)(w + HL.wts);
    if (K == 0) {   // no angle reads a parameter: H = 0
        const hipError_t e = launch_hess_accum(G, 0, 0, 0, d->hoff, d->hocc, d->occ_scale, P, hess, s);
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "hessian: %s", hipGetErrorString(e));
        return ok();
    }
    for (int64_t c0 = 0; c0 < K; c0 += m) {
        const int64_t mc = std::min<int64_t>(m, K - c0), B = 2 * mc;
        const WsLayout L = layout(*h, obs, B, 1, 1);
        char *wd = w + HL.sub;
        void *states = w + HL.states;
        hipError_t e = launch_hess_rows(params, d->occ_param, d->occ_scale, K, c0, mc, rows, s);
        if (e == hipSuccess) e = launch_bcast_rows(weights, obs->nobs, B, go, s);
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "hessian rows: %s", hipGetErrorString(e));
        if ((st = apply_on_device(*h, *dh, states, B, rows, K, data, 0, 1, wd + L.mats, 1, s, true)) != DQ_OK) return st;
        if ((st = adjoint_core(*h, *dh, *obs, g, t, states, B, rows, K, data, 0, go, G, nullptr, 0, wd, L, s)) != DQ_OK)
            return st;
        e = launch_hess_accum(G, K, c0, mc, d->hoff, d->hocc, d->occ_scale, P, hess, s);
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "hessian accumulate: %s", hipGetErrorString(e));
    }
    return ok();
} DQ_CATCH

dq_status dq_profile_enable(dq_plan plan, int32_t on) try {
    if (!plan) return fail(DQ_ERR_INVALID_ARG, "NULL plan");
    plan->prof = on != 0;
    return ok();
} DQ_CATCH

dq_status dq_profile_read(dq_plan plan, dq_profile *out, int32_t reset) try {
    if (!plan || !out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    for (const auto &r : plan->precs) {
        DQ_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        DQ_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        plan->acc.launches[r.kind] += r.nl;
        plan->acc.ms[r.kind] += ms;
        plan->acc.bytes[r.kind] += r.bytes;
        plan->acc.flops[r.kind] += r.flops;
    }
    plan->precs.clear();
    plan->evused = 0;
    *out = plan->acc;
    if (reset) plan->acc = dq_profile{};
    return ok();
} DQ_CATCH

// ================================================================ uneven batches
}  // extern "C"

namespace {
constexpr int64_t kMultiWps = 256;   // adjoint waves per circuit in an uneven batch (at most)
}

struct dq_multi_s {
    int dbl = 0;
    int R_fwd = 0, R_adj = 0;
    std::vector<dq_plan> plans;
    std::vector<dq_obs> obs;
    std::vector<int64_t> st_off, par_off, out_off;
    int64_t st_total = 0, par_total = 0, out_total = 0;
    std::vector<size_t> ws_off;
    std::vector<WsLayout> lay;
    size_t ws_total = 0;
    std::vector<char> batched;
    // host entries: depth-major, circuits in order; ops / lsg hold the
    // element index into the plan tables until the device upload resolves them
    std::vector<std::vector<MultiEntry>> fwd, adj;
    std::vector<std::vector<int>> fwd_c, adj_c;       // circuit of each entry
    std::vector<int64_t> fwd_units, adj_units;
    std::vector<int32_t> adj_maxnls;
    std::vector<int32_t> wps;                          // adjoint waves per circuit
    std::vector<int> bc;                               // the batched circuits, in order
    std::mutex mu;
    struct Dev {
        void *blob = nullptr;
        std::vector<MultiEntry *> fwd, adj;
        // the per-circuit steps around the tile passes, one launch each
        MPrep *prep_fwd = nullptr, *prep_adj = nullptr;
        MInit *init = nullptr;
        MExp *exp = nullptr;
        MGrad *grad = nullptr;
        int32_t max_slots_fwd = 0, max_slots_adj = 0, max_n = 0;
        int64_t exp_units = 0, lam_total = 0, grad_total = 0;
        int32_t exp_max_group = 0;   // the most terms of one X-mask group over the batched circuits
    };
    std::map<int, Dev> dev;
};

namespace {

bool tile_only(const Program &p, int R) {
    for (const Step &s : p.steps)
        if (s.kind != ST_TILE || s.R != R) return false;
    return true;
}

MultiEntry make_entry(const Step &S, int n) {
    MultiEntry E{};
    E.n = n;
    E.nops = (int32_t)S.nops;
    E.nls = (int32_t)S.nls;
    E.ops = reinterpret_cast<const TOp *>((intptr_t)S.op0);
    E.lsg = reinterpret_cast<const int32_t *>((intptr_t)S.ls0);
    for (int k = 0; k < MAX_TILE_R; ++k) E.rbits[k] = S.rbits[k];
    for (int k = 0; k < 3; ++k) E.lbits[k] = S.lbits[k];
    for (int k = 0; k < MAX_TILE_R + 3; ++k) E.tbits[k] = S.tbits[k];
    return E;
}

dq_status ensure_multi(dq_multi_s &m, dq_multi_s::Dev **out) {
    int dev = 0;
    DQ_HIP(hipGetDevice(&dev));
    for (dq_plan p : m.plans) {
        DevData *d = nullptr;
        dq_status st = ensure_device(*p, &d);
        if (st != DQ_OK) return st;
    }
    std::lock_guard<std::mutex> lk(m.mu);
    auto it = m.dev.find(dev);
    if (it != m.dev.end()) {
        *out = &it->second;
        return DQ_OK;
    }
    std::vector<MultiEntry> all;
    std::vector<size_t> fstart, astart;
    auto resolve = [&](const std::vector<MultiEntry> &v, const std::vector<int> &cs) {
        for (size_t i = 0; i < v.size(); ++i) {
            MultiEntry E = v[i];
            DevData &d = m.plans[cs[i]]->dev[dev];
            E.ops = d.ops + (intptr_t)E.ops;
            E.lsg = d.lsg + (intptr_t)E.lsg;
            all.push_back(E);
        }
    };
    for (size_t k = 0; k < m.fwd.size(); ++k) {
        fstart.push_back(all.size());
        resolve(m.fwd[k], m.fwd_c[k]);
    }
    for (size_t k = 0; k < m.adj.size(); ++k) {
        astart.push_back(all.size());
        resolve(m.adj[k], m.adj_c[k]);
    }
    // the batched circuits' per-circuit steps, resolved for this device
    dq_multi_s::Dev D;
    std::vector<MPrep> pf, pa;
    std::vector<MInit> in;
    std::vector<MExp> ex;
    std::vector<MGrad> gr;
    for (int c : m.bc) {
        dq_plan p = m.plans[c];
        DevData &d = p->dev[dev];
        const WsLayout &L = m.lay[c];
        const size_t wo = m.ws_off[c];
        const Program &f = p->has_fold ? p->fwd_fold : p->fwd_full;
        MPrep P{};
        P.gates = d.gates;
        P.fixed = d.fixed;
        P.par_off = m.par_off[c];
        P.mats_off = (int64_t)(wo + L.mats);
        P.slots = d.slots + f.slot_lo;
        P.nslots = (int32_t)(f.slot_hi - f.slot_lo);
        pf.push_back(P);
        D.max_slots_fwd = std::max(D.max_slots_fwd, P.nslots);
        P.slots = d.slots + p->adj.slot_lo;
        P.nslots = (int32_t)(p->adj.slot_hi - p->adj.slot_lo);
        pa.push_back(P);
        D.max_slots_adj = std::max(D.max_slots_adj, P.nslots);
        MInit I{};
        I.st_off = m.st_off[c];
        I.mats_off = (int64_t)(wo + L.mats);
        I.fold = d.fold;
        I.n = p->n;
        I.has_fold = p->has_fold ? 1 : 0;
        in.push_back(I);
        D.max_n = std::max(D.max_n, p->n);
        const DGroup *g = nullptr;
        const DTerm *t = nullptr;
        dq_status st = ensure_obs(*m.obs[c], &g, &t);
        if (st != DQ_OK) return st;
        // the adjoint-seed kernel takes a wave's 64 amplitudes from one circuit
        if (p->n < 6) return fail(DQ_ERR_INTERNAL, "multi-plan circuit %d: batched with %d qubits", c, p->n);
        MExp X{};
        X.st_off = m.st_off[c];
        X.lam_off = (int64_t)(wo + L.lam);
        X.part_off = (int64_t)(wo + L.expv);
        X.unit_begin = D.exp_units;
        X.amp_begin = D.lam_total;
        X.out_off = m.out_off[c];
        X.groups = g;
        X.terms = t;
        X.n = p->n;
        X.ngroups = (int32_t)m.obs[c]->groups.size();
        X.nterms = (int32_t)m.obs[c]->terms.size();
        X.nobs = m.obs[c]->nobs;
        X.eb = (int32_t)expval_blocks(p->n, 1);
        for (const auto &gr_ : m.obs[c]->groups) D.exp_max_group = std::max(D.exp_max_group, gr_.t1 - gr_.t0);
        ex.push_back(X);
        D.exp_units += X.eb;
        D.lam_total += int64_t(1) << p->n;
        MGrad G{};
        G.part_off = (int64_t)(wo + L.part);
        G.par_off = m.par_off[c];
        G.unit_begin = D.grad_total;
        G.poff = d.poff;
        G.pg = d.pg;
        G.pf = d.pf;
        G.wps = m.wps[c];
        G.ngrad = p->ngrad;
        gr.push_back(G);
        D.grad_total += p->nparams;
    }
    std::vector<char> blob;
    const size_t o_all = put(blob, all), o_pf = put(blob, pf), o_pa = put(blob, pa), o_in = put(blob, in),
                 o_ex = put(blob, ex), o_gr = put(blob, gr);
    DQ_HIP(hipMalloc(&D.blob, std::max<size_t>(blob.size(), 1)));
    hipError_t e = hipMemcpy(D.blob, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(D.blob);
        return fail(DQ_ERR_HIP, "multi upload: %s", hipGetErrorString(e));
    }
    char *bb = (char *)D.blob;
    for (size_t k : fstart) D.fwd.push_back((MultiEntry *)(bb + o_all) + k);
    for (size_t k : astart) D.adj.push_back((MultiEntry *)(bb + o_all) + k);
    D.prep_fwd = (MPrep *)(bb + o_pf);
    D.prep_adj = (MPrep *)(bb + o_pa);
    D.init = (MInit *)(bb + o_in);
    D.exp = (MExp *)(bb + o_ex);
    D.grad = (MGrad *)(bb + o_gr);
    *out = &(m.dev[dev] = D);
    return DQ_OK;
}

}  // namespace

extern "C" {

dq_status dq_multi_create(dq_multi *out, const dq_plan *plans, const dq_obs *obs, int32_t nplans) try {
    if (!out || !plans || !obs || nplans < 1) return fail(DQ_ERR_INVALID_ARG, "need plans, observables and nplans >= 1");
    *out = nullptr;
    std::unique_ptr<dq_multi_s> m(new dq_multi_s());
    m->dbl = plans[0] ? plans[0]->dbl : 0;
    for (int c = 0; c < nplans; ++c) {
        if (!plans[c] || !obs[c]) {
            return fail(DQ_ERR_INVALID_ARG, "circuit %d: NULL plan or observable", c);
        }
        if (plans[c]->dbl != m->dbl) {
            return fail(DQ_ERR_INVALID_ARG, "circuit %d: dtype differs from circuit 0", c);
        }
        if (plans[c]->ndata > 0) {
            return fail(DQ_ERR_UNSUPPORTED, "circuit %d: data-encoded gates are not supported in a multi-plan", c);
        }
        if (obs[c]->n != plans[c]->n) {
            return fail(DQ_ERR_INVALID_ARG, "circuit %d: observable for %d qubits, plan for %d", c, obs[c]->n, plans[c]->n);
        }
        m->plans.push_back(plans[c]);
        m->obs.push_back(obs[c]);
    }
    // common tile shape: that of the first fused plan the shared kernels can run
    for (dq_plan p : m->plans)
        if (p->R_fwd > 0 && !p->opt.arith64) {
            m->R_fwd = p->R_fwd;
            m->R_adj = p->R_adj;
            break;
        }
    const size_t amp = m->dbl ? 16 : 8;
    for (int c = 0; c < nplans; ++c) {
        dq_plan p = m->plans[c];
        m->st_off.push_back(m->st_total);
        m->st_total += (int64_t)(align256(((size_t)1 << p->n) * amp) / amp);
        m->par_off.push_back(m->par_total);
        m->par_total += p->nparams;
        m->out_off.push_back(m->out_total);
        m->out_total += m->obs[c]->nobs;
        const WsLayout L = layout(*p, m->obs[c], 1, 0, 1);
        m->ws_off.push_back(m->ws_total);
        m->lay.push_back(L);
        m->ws_total += align256(L.total);
        const Program &f = p->has_fold ? p->fwd_fold : p->fwd_full;
        // batched: pure tile programs of the common shape, for which the
        // multi-circuit kernels exist; the rest take the single-plan path
        m->batched.push_back(!p->opt.arith64 && p->R_fwd > 0 && p->R_fwd == m->R_fwd && p->R_adj == m->R_adj &&
                             tile_only(f, m->R_fwd) &&
                             tile_only(p->adj, m->R_adj) && multi_fwd_has(m->dbl, m->R_fwd) &&
                             multi_adj_has(m->dbl, m->R_adj));
    }
    // adjoint waves per circuit: each wave walks tiles w, w + wps, ... and
    // leaves one row of partial gradient sums, which the final reduction
    // adds; capped, so that the rows stay few while the waves of all
    // circuits together still fill the device
    for (int c = 0; c < nplans; ++c) {
        m->wps.push_back((int32_t)std::min<int64_t>(grad_waves(*m->plans[c], 1), kMultiWps));
        if (m->batched[c]) m->bc.push_back(c);
    }
    // depth tables
    const double tot_bytes = (double)m->st_total * (double)amp;   // all circuits' states
    for (int pass = 0; pass < 2; ++pass) {
        auto &tab = pass ? m->adj : m->fwd;
        auto &tabc = pass ? m->adj_c : m->fwd_c;
        auto &units = pass ? m->adj_units : m->fwd_units;
        for (int c = 0; c < nplans; ++c) {
            if (!m->batched[c]) continue;
            dq_plan p = m->plans[c];
            const Program &prog = pass ? p->adj : (p->has_fold ? p->fwd_fold : p->fwd_full);
            for (size_t d = 0; d < prog.steps.size(); ++d) {
                if (tab.size() <= d) {
                    tab.resize(d + 1);
                    tabc.resize(d + 1);
                    units.resize(d + 1, 0);
                    if (pass) m->adj_maxnls.resize(d + 1, 0);
                }
                MultiEntry E = make_entry(prog.steps[d], p->n);
                const WsLayout &L = m->lay[c];
                E.st_off = m->st_off[c];
                E.mats_off = (int64_t)(m->ws_off[c] + L.mats);
                E.lam_off = (int64_t)(m->ws_off[c] + L.lam);
                E.part_off = (int64_t)(m->ws_off[c] + L.part);
                E.ngrad = p->ngrad;
                E.nt = tot_bytes * (pass ? 2 : 1) > kStreamBytes ? 1 : 0;
                const int64_t tiles = int64_t(1) << (p->n - 6 - (pass ? m->R_adj : m->R_fwd));
                E.wps = pass ? m->wps[c] : 1;
                E.unit_begin = units[d];
                units[d] += pass ? E.wps : tiles;
                if (pass) m->adj_maxnls[d] = std::max<int32_t>(m->adj_maxnls[d], E.nls);
                tab[d].push_back(E);
                tabc[d].push_back(c);
            }
        }
    }
    *out = m.release();
    return ok();
} DQ_CATCH

void dq_multi_destroy(dq_multi m) try {
    if (!m) return;
    for (auto &kv : m->dev) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess) {
            (void)hipSetDevice(kv.first);
            (void)hipFree(kv.second.blob);
            (void)hipSetDevice(cur);
        }
    }
    delete m;
} DQ_CATCH_VOID

dq_status dq_multi_layout(dq_multi m, int64_t *state_amps, int64_t *param_count, int64_t *nout, int64_t *state_off,
                          int64_t *param_off, int64_t *out_off) try {
    if (!m) return fail(DQ_ERR_INVALID_ARG, "NULL multi-plan");
    if (state_amps) *state_amps = m->st_total;
    if (param_count) *param_count = m->par_total;
    if (nout) *nout = m->out_total;
    for (size_t c = 0; c < m->plans.size(); ++c) {
        if (state_off) state_off[c] = m->st_off[c];
        if (param_off) param_off[c] = m->par_off[c];
        if (out_off) out_off[c] = m->out_off[c];
    }
    return ok();
} DQ_CATCH

dq_status dq_multi_workspace_size(dq_multi m, size_t *bytes) try {
    if (!m || !bytes) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    *bytes = m->ws_total;
    return ok();
} DQ_CATCH

dq_status dq_multi_batched(dq_multi m, int32_t *batched, int32_t *count) try {
    if (!m) return fail(DQ_ERR_INVALID_ARG, "NULL multi-plan");
    int32_t k = 0;
    for (size_t c = 0; c < m->plans.size(); ++c) {
        if (batched) batched[c] = m->batched[c] ? 1 : 0;
        k += m->batched[c] ? 1 : 0;
    }
    if (count) *count = k;
    return ok();
} DQ_CATCH

dq_status dq_multi_apply(dq_multi m, void *states, const double *params, void *ws, size_t ws_bytes, void *stream) try {
    if (!m || !states) return fail(DQ_ERR_INVALID_ARG, "NULL multi-plan or states");
    if (m->par_total > 0 && !params) return fail(DQ_ERR_INVALID_ARG, "params is NULL");
    if (!ws || ws_bytes < m->ws_total) return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed", m->ws_total);
    dq_multi_s::Dev *D = nullptr;
    dq_status st = ensure_multi(*m, &D);
    if (st != DQ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t amp = m->dbl ? 16 : 8;
    char *w = (char *)ws;
    for (size_t c = 0; c < m->plans.size(); ++c) {
        if (m->batched[c]) continue;
        void *sc = (char *)states + m->st_off[c] * amp;
        const double *pc = params ? params + m->par_off[c] : nullptr;
        if ((st = dq_apply_circuit(m->plans[c], sc, 1, pc, 0, nullptr, 0, 1, w + m->ws_off[c], m->lay[c].total,
                                   stream)) != DQ_OK)
            return st;
    }
    // the batched circuits: matrices, start states, then one tile launch per depth
    const int32_t nb = (int32_t)m->bc.size();
    hipError_t e = launch_prepare_multi(m->dbl, D->prep_fwd, nb, D->max_slots_fwd, params, ws, s);
    if (e == hipSuccess) e = launch_init_multi(m->dbl, states, ws, D->init, nb, D->max_n, s);
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "multi init: %s", hipGetErrorString(e));
    for (size_t k = 0; k < m->fwd.size(); ++k) {
        e = launch_tile_fwd_multi(m->dbl, m->R_fwd, states, ws, D->fwd[k], (int32_t)m->fwd[k].size(), m->fwd_units[k], s);
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "multi tile pass: %s", hipGetErrorString(e));
    }
    return ok();
} DQ_CATCH

dq_status dq_multi_expval(dq_multi m, const void *states, double *out, void *ws, size_t ws_bytes, void *stream) try {
    if (!m || !states || !out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (!ws || ws_bytes < m->ws_total) return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed", m->ws_total);
    dq_multi_s::Dev *D = nullptr;
    dq_status st = ensure_multi(*m, &D);
    if (st != DQ_OK) return st;
    const size_t amp = m->dbl ? 16 : 8;
    for (size_t c = 0; c < m->plans.size(); ++c) {
        if (m->batched[c]) continue;
        if ((st = dq_expval(m->plans[c], m->obs[c], (const char *)states + m->st_off[c] * amp, 1, out + m->out_off[c],
                            (char *)ws + m->ws_off[c], m->lay[c].total, stream)) != DQ_OK)
            return st;
    }
    const hipError_t e = launch_expval_multi(m->dbl, states, ws, D->exp, (int32_t)m->bc.size(), D->exp_units, D->exp_max_group, out,
                                             (hipStream_t)stream);
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "multi expval: %s", hipGetErrorString(e));
    return ok();
} DQ_CATCH

dq_status dq_multi_adjoint_grad(dq_multi m, void *states, const double *params, const double *grad_out,
                                double *grad_params, void *ws, size_t ws_bytes, void *stream) try {
    if (!m || !states || !grad_out) return fail(DQ_ERR_INVALID_ARG, "NULL argument");
    if (m->par_total > 0 && (!params || !grad_params)) return fail(DQ_ERR_INVALID_ARG, "params / grad_params is NULL");
    if (!ws || ws_bytes < m->ws_total) return fail(DQ_ERR_WORKSPACE, "workspace of %zu bytes needed", m->ws_total);
    dq_multi_s::Dev *D = nullptr;
    dq_status st = ensure_multi(*m, &D);
    if (st != DQ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t amp = m->dbl ? 16 : 8;
    char *w = (char *)ws;
    for (size_t c = 0; c < m->plans.size(); ++c) {
        if (m->batched[c]) continue;
        dq_plan p = m->plans[c];
        void *sc = (char *)states + m->st_off[c] * amp;
        const double *pc = params ? params + m->par_off[c] : nullptr;
        double *gc = grad_params ? grad_params + m->par_off[c] : nullptr;
        if ((st = dq_adjoint_grad(p, m->obs[c], sc, 1, pc, 0, nullptr, 0, grad_out + m->out_off[c], gc, nullptr, 0,
                                  w + m->ws_off[c], m->lay[c].total, stream)) != DQ_OK)
            return st;
    }
    const int32_t nb = (int32_t)m->bc.size();
    hipError_t e = launch_prepare_multi(m->dbl, D->prep_adj, nb, D->max_slots_adj, params, ws, s);
    if (e == hipSuccess) e = launch_lambda_multi(m->dbl, states, ws, D->exp, nb, D->lam_total, grad_out, s);
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "multi adjoint seed: %s", hipGetErrorString(e));
    for (size_t k = 0; k < m->adj.size(); ++k) {
        e = launch_tile_adj_multi(m->dbl, m->R_adj, states, ws, D->adj[k], (int32_t)m->adj[k].size(), m->adj_units[k],
                                  m->adj_maxnls[k], s);
        if (e != hipSuccess) return fail(DQ_ERR_HIP, "multi adjoint pass: %s", hipGetErrorString(e));
    }
    e = launch_grad_final_multi(ws, D->grad, nb, D->grad_total, grad_params, s);
    if (e != hipSuccess) return fail(DQ_ERR_HIP, "multi grad reduce: %s", hipGetErrorString(e));
    return ok();
} DQ_CATCH

}  // extern "C"
