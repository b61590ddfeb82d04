// C ABI of libqc (declared in include/qc.h): argument validation, the
// per-device workspace and staging ring, kernel timing, the host-side gate
// fuser and the circuit executor.  Device work is delegated to the
// launchers in qc_gates.hip, qc_fused_mfma.hip, qc_reduce.hip and
// qc_adjoint.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qc.h"
#include "qc_internal.h"

using cd = std::complex<double>;

namespace {

thread_local std::string t_err;

int fail(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(QC_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- workspace

constexpr size_t kWorkElems = size_t(8) << 20;     // 64 MiB of FP64 partials
constexpr size_t kRingBytes = size_t(64) << 20;    // staging ring
constexpr int kMaxDevices = 64;

struct DevCtx {
    bool ready = false;
    double *work = nullptr;
    char *ring_dev = nullptr;
    char *ring_host = nullptr;
    size_t ring_head = 0;
    // ring bytes [prot_lo, prot_hi) hold slots staged while a stream was
    // being captured into a HIP graph: every replay copies them again, so
    // later calls skip them until the next qc_reserve
    size_t prot_lo = 0, prot_hi = 0;
};

DevCtx g_dev[kMaxDevices];
std::mutex g_mu;

// true while `s` is being captured into a HIP graph
bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

int get_ctx(DevCtx **out) {
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (d < 0 || d >= kMaxDevices) return fail(QC_ERR_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx &c = g_dev[d];
    if (!c.ready) {
        // first use on this device (qc_reserve does it before a graph capture)
        if (hipMalloc(&c.work, kWorkElems * sizeof(double)) != hipSuccess)
            return fail(QC_ERR_NOMEM, "workspace allocation failed");
        if (hipMalloc(&c.ring_dev, kRingBytes) != hipSuccess)
            return fail(QC_ERR_NOMEM, "staging ring allocation failed");
        if (hipHostMalloc(&c.ring_host, kRingBytes, hipHostMallocDefault) != hipSuccess)
            return fail(QC_ERR_NOMEM, "pinned staging allocation failed");
        c.ring_head = 0;
        c.ready = true;
    }
    *out = &c;
    return QC_OK;
}

// Copy a small host array into device memory owned by the ring.  The copy
// is ordered on `s` before any kernel the caller enqueues afterwards.  When
// the ring wraps, the device is drained first so no slot still in use by an
// earlier copy or kernel is overwritten.  While `s` is being captured into
// a HIP graph there is no drain: a slot that does not fit before the end of
// the ring is refused (QC_ERR_UNSUPPORTED; qc_reserve makes room before a
// capture), and the slots taken are protected from later calls.
int stage(DevCtx *c, const void *src, size_t bytes, hipStream_t s, void **dev) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (need > kRingBytes) return fail(QC_ERR_ARG, "staged array too large");
    const bool cap = capturing(s);
    auto overlaps_prot = [&](size_t h) {
        return c->prot_hi > c->prot_lo && h < c->prot_hi && h + need > c->prot_lo;
    };
    if (!cap && overlaps_prot(c->ring_head)) c->ring_head = c->prot_hi;
    if (c->ring_head + need > kRingBytes) {
        if (cap)
            return fail(QC_ERR_UNSUPPORTED,
                        "staging ring full during graph capture (call qc_reserve before capturing)");
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        c->ring_head = 0;
        if (overlaps_prot(c->ring_head)) c->ring_head = c->prot_hi;
        if (c->ring_head + need > kRingBytes)
            return fail(QC_ERR_NOMEM, "staging ring held by captured graphs (call qc_reserve)");
    }
    if (cap) {
        if (c->prot_hi <= c->prot_lo) c->prot_lo = c->ring_head;
        if (c->ring_head < c->prot_lo) c->prot_lo = c->ring_head;
        c->prot_hi = std::max(c->prot_hi, c->ring_head + need);
    }
    std::memcpy(c->ring_host + c->ring_head, src, bytes);
    hipError_t e = hipMemcpyAsync(c->ring_dev + c->ring_head, c->ring_host + c->ring_head, bytes,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    *dev = c->ring_dev + c->ring_head;
    c->ring_head += need;
    return QC_OK;
}

// ---------------------------------------------------------------- timing

std::atomic<bool> g_timing{false};
struct TimerRec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};
std::vector<TimerRec> g_trecs;
std::map<std::string, std::pair<int64_t, double>> g_tsum;
std::mutex g_tmu;

// launch-shape knobs (QC_KNOB_*)
std::atomic<int> g_knob_mfma{4};
std::atomic<int> g_knob_tile{8};
std::atomic<int> g_knob_look{16};
std::atomic<int> g_knob_tbits{13};
std::atomic<int> g_knob_tile_bits{13};
std::atomic<int> g_knob_tile_engine{1};
std::atomic<int> g_knob_wide{12};

// ---------------------------------------------------------------- validation

int check_state(const qc_state_t &s) {
    if (!s.amp) return fail(QC_ERR_ARG, "state amplitude pointer is NULL");
    if (s.n < 1 || s.n > QC_MAX_QUBITS) return fail(QC_ERR_ARG, "qubit count out of range");
    if (s.dtype != QC_C64 && s.dtype != QC_C128) return fail(QC_ERR_DTYPE, "unknown dtype");
    return QC_OK;
}

// labels must be in [0, n) and pairwise distinct
int check_qubits(int n, const int *q, int m, const char *what) {
    if (m > 0 && !q) return fail(QC_ERR_ARG, std::string(what) + " pointer is NULL");
    uint64_t seen = 0;
    for (int i = 0; i < m; ++i) {
        if (q[i] < 0 || q[i] >= n)
            return fail(QC_ERR_QUBIT, std::string(what) + " label out of range");
        const uint64_t bit = uint64_t(1) << q[i];
        if (seen & bit) return fail(QC_ERR_QUBIT, std::string(what) + " labels repeat");
        seen |= bit;
    }
    return QC_OK;
}

inline int bitpos(int n, int q) { return n - 1 - q; }

// ---------------------------------------------------------------- host math

// Apply a gate (targets/controls given as block-local bit positions, MSB
// first for targets) to a small dense vector of 2^k amplitudes.
void host_apply(std::vector<cd> &v, int k, int nt, const int *tbit, int nc, const int *cbit,
                const int *cval, const cd *u) {
    const int d = 1 << nt;
    uint64_t fixed = 0, want = 0;
    for (int j = 0; j < nt; ++j) fixed |= uint64_t(1) << tbit[j];
    for (int j = 0; j < nc; ++j) {
        fixed |= uint64_t(1) << cbit[j];
        if (cval[j]) want |= uint64_t(1) << cbit[j];
    }
    std::vector<uint64_t> off(d);
    for (int r = 0; r < d; ++r) {
        uint64_t o = 0;
        for (int j = 0; j < nt; ++j)
            if ((r >> (nt - 1 - j)) & 1) o |= uint64_t(1) << tbit[j];
        off[r] = o;
    }
    std::vector<cd> in(d);
    const uint64_t dim = uint64_t(1) << k;
    for (uint64_t i = 0; i < dim; ++i) {
        if ((i & fixed) != want) continue;   // not a group base
        for (int c = 0; c < d; ++c) in[c] = v[i | off[c]];
        for (int r = 0; r < d; ++r) {
            cd acc = 0.0;
            for (int c = 0; c < d; ++c) acc += u[r * d + c] * in[c];
            v[i | off[r]] = acc;
        }
    }
}

std::vector<cd> to_cd(const double *u, int d) {
    std::vector<cd> m(size_t(d) * d);
    for (size_t i = 0; i < m.size(); ++i) m[i] = cd(u[2 * i], u[2 * i + 1]);
    return m;
}

// A gate as it acts inside one block: targets and controls are labels of
// block qubits; nt == 0 is a (controlled) scalar phase u[0].
struct LocalGate {
    int nt = 0, nc = 0;
    int tq[QC_MAX_FUSED];
    int cq[QC_MAX_CTRLS];
    int cv[QC_MAX_CTRLS];
    std::vector<cd> u;
};

bool matrix_is_diagonal(const double *u, int nt) {
    const int d = 1 << nt;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && (u[2 * (r * d + c)] != 0.0 || u[2 * (r * d + c) + 1] != 0.0))
                return false;
    return true;
}

// Qubits on which the gate acts non-diagonally: its targets unless the
// target matrix is diagonal.  On every other qubit of the gate (controls,
// targets of a diagonal matrix) the gate is block diagonal, so it commutes
// with any other gate that is also diagonal on each qubit they share.
uint64_t gate_nd_mask(const qc_gate_t &g) {
    if (matrix_is_diagonal(g.matrix, g.n_targets)) return 0;
    uint64_t m = 0;
    for (int j = 0; j < g.n_targets; ++j) m |= uint64_t(1) << g.targets[j];
    return m;
}

// The gate restricted to the selector assignment `sv` of the selector
// qubits `sq` (sq[0] = most significant bit of sv).  Returns false when the
// gate is the identity there (a control on a selector qubit not met).  A
// selector qubit is never a target of a non-diagonal matrix (the fuser and
// the multiplexed-gate path guarantee this).
bool restrict_gate(const qc_gate_t &g, int ns, const int *sq, int sv, LocalGate &out) {
    auto sel_bit = [&](int label) {
        for (int j = 0; j < ns; ++j)
            if (sq[j] == label) return (sv >> (ns - 1 - j)) & 1;
        return -1;
    };
    out.nc = 0;
    for (int j = 0; j < g.n_ctrls; ++j) {
        const int b = sel_bit(g.ctrls[j]);
        if (b < 0) {
            out.cq[out.nc] = g.ctrls[j];
            out.cv[out.nc++] = g.ctrl_vals[j];
        } else if (b != g.ctrl_vals[j]) {
            return false;
        }
    }
    const int d = 1 << g.n_targets;
    int fixed_idx = 0, keep = 0, kept_pos[QC_MAX_FUSED];
    out.nt = 0;
    for (int j = 0; j < g.n_targets; ++j) {
        const int b = sel_bit(g.targets[j]);
        const int shift = g.n_targets - 1 - j;
        if (b < 0) {
            out.tq[out.nt++] = g.targets[j];
            kept_pos[keep++] = shift;
        } else if (b) {
            fixed_idx |= 1 << shift;
        }
    }
    if (out.nt == g.n_targets) {
        out.u = to_cd(g.matrix, d);
        return true;
    }
    // diagonal matrix with some targets fixed by the selector
    const int dk = 1 << out.nt;
    out.u.assign(size_t(dk) * dk, cd(0.0, 0.0));
    for (int r = 0; r < dk; ++r) {
        int full = fixed_idx;
        for (int j = 0; j < out.nt; ++j)
            if ((r >> (out.nt - 1 - j)) & 1) full |= 1 << kept_pos[j];
        out.u[size_t(r) * dk + r] = cd(g.matrix[2 * (full * d + full)], g.matrix[2 * (full * d + full) + 1]);
    }
    return true;
}

// Dense matrix (2^k, row-major) of a list of gates acting inside the block
// whose qubits (labels, qubits[0] = MSB) are `bq`.
std::vector<cd> block_matrix_local(int k, const int *bq, const std::vector<LocalGate> &gs) {
    const int dim = 1 << k;
    auto local = [&](int label) {
        for (int j = 0; j < k; ++j)
            if (bq[j] == label) return k - 1 - j;
        return -1;
    };
    // columns of the product, evolved as 2^k small states
    std::vector<std::vector<cd>> cols(dim, std::vector<cd>(dim, 0.0));
    for (int c = 0; c < dim; ++c) cols[c][c] = 1.0;
    for (const LocalGate &g : gs) {
        int tb[QC_MAX_FUSED], cb[QC_MAX_CTRLS];
        for (int j = 0; j < g.nt; ++j) tb[j] = local(g.tq[j]);
        for (int j = 0; j < g.nc; ++j) cb[j] = local(g.cq[j]);
        for (int c = 0; c < dim; ++c) host_apply(cols[c], k, g.nt, tb, g.nc, cb, g.cv, g.u.data());
    }
    std::vector<cd> m(size_t(dim) * dim);
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) m[size_t(r) * dim + c] = cols[c][r];
    return m;
}

// Matrices U_s of a multiplexed block: for every assignment s of the
// selector qubits `sq`, the product of the gates restricted to s.  The
// result holds the 2^ns matrices one after the other.
std::vector<cd> block_matrices(int k, const int *bq, int ns, const int *sq,
                               const std::vector<const qc_gate_t *> &gs) {
    std::vector<cd> all;
    std::vector<LocalGate> loc;
    for (int sv = 0; sv < (1 << ns); ++sv) {
        loc.clear();
        for (const qc_gate_t *g : gs) {
            LocalGate lg;
            if (restrict_gate(*g, ns, sq, sv, lg)) loc.push_back(std::move(lg));
        }
        const std::vector<cd> m = block_matrix_local(k, bq, loc);
        all.insert(all.end(), m.begin(), m.end());
    }
    return all;
}

std::vector<cd> block_matrix(int k, const int *bq, const std::vector<const qc_gate_t *> &gs) {
    return block_matrices(k, bq, 0, nullptr, gs);
}

uint64_t gate_mask(const qc_gate_t &g) {
    uint64_t m = 0;
    for (int j = 0; j < g.n_targets; ++j) m |= uint64_t(1) << g.targets[j];
    for (int j = 0; j < g.n_ctrls; ++j) m |= uint64_t(1) << g.ctrls[j];
    return m;
}

int check_gate(int n, const qc_gate_t &g) {
    if (g.n_targets < 1 || g.n_targets > QC_MAX_FUSED)
        return fail(QC_ERR_ARG, "gate target count out of range");
    if (g.n_ctrls < 0 || g.n_ctrls > QC_MAX_CTRLS)
        return fail(QC_ERR_ARG, "gate control count out of range");
    if (!g.matrix) return fail(QC_ERR_ARG, "gate matrix is NULL");
    int all[QC_MAX_FUSED + QC_MAX_CTRLS];
    for (int j = 0; j < g.n_targets; ++j) all[j] = g.targets[j];
    for (int j = 0; j < g.n_ctrls; ++j) {
        all[g.n_targets + j] = g.ctrls[j];
        if (g.ctrl_vals[j] != 0 && g.ctrl_vals[j] != 1)
            return fail(QC_ERR_ARG, "control value must be 0 or 1");
    }
    return check_qubits(n, all, g.n_targets + g.n_ctrls, "gate qubit");
}

// Qubit masks of one gate for the fuser: every qubit, and the qubits it
// acts on non-diagonally.
struct GateMasks {
    uint64_t all, nd;
};

// Members (positions in `pending`) of a block seeded by pending[seed].
// The pending list is scanned in order.  A gate may move ahead of the
// earlier pending gates left out of the block only if it commutes with
// them: on a qubit where it acts non-diagonally no gate may have been left
// out ("blocked_any"), and on a qubit where it acts diagonally no gate
// acting non-diagonally there may have been left out ("blocked_nd").  It
// must also fit: its non-diagonal qubits inside the block qubits (the label
// set `window` when one is given, else at most k qubits grown so far); its
// diagonal qubits either inside the block or among at most `smax` selector
// qubits outside it.  On a selector qubit every member acts diagonally, so
// the block is a multiplexed gate: one k-qubit matrix per selector value.
// The seed has no pending predecessor on its qubits, so the block can be
// applied before every gate left out.
void grow_block(const std::vector<int> &pending, const std::vector<GateMasks> &gm, int seed,
                uint64_t window, int k, int smax, uint64_t all, std::vector<int> &members) {
    members.clear();
    const GateMasks sm = gm[pending[seed]];
    uint64_t held = window ? window : sm.all, sel = 0, blocked_any = 0, blocked_nd = 0;
    const bool oversize = __builtin_popcountll(sm.all) > k;
    for (int i = 0; i < int(pending.size()); ++i) {
        if (i == seed) {
            members.push_back(i);
            continue;
        }
        const GateMasks g = gm[pending[i]];
        const uint64_t diag = g.all & ~g.nd;
        bool fits = !oversize && !(g.nd & blocked_any) && !(diag & blocked_nd) && !(g.nd & sel);
        uint64_t new_held = held, new_sel = sel;
        if (fits) {
            if (window) {
                fits = (g.nd & ~window) == 0;
                new_sel = sel | (g.all & ~window);
            } else {
                new_held = held | g.nd;
                const uint64_t free_diag = diag & ~new_held & ~sel;
                if (__builtin_popcountll(new_held | free_diag) <= k) new_held |= free_diag;
                else new_sel = sel | free_diag;
                fits = __builtin_popcountll(new_held) <= k;
            }
            fits = fits && __builtin_popcountll(new_sel) <= smax;
        }
        if (fits) {
            held = new_held;
            sel = new_sel;
            members.push_back(i);
        } else {
            blocked_any |= g.all;
            blocked_nd |= g.nd;
            if ((blocked_nd & all) == all) break;   // nothing can join any more
        }
    }
}

// Candidate blocks for the current pending list: for each of the first
// gates that have no pending predecessor ("front" gates), the block grown
// greedily from it and the blocks confined to each window of k consecutive
// qubit labels that holds it.
void block_candidates(int n, const std::vector<int> &pending, const std::vector<GateMasks> &gm,
                      int k, int smax, uint64_t all, std::vector<std::vector<int>> &out) {
    constexpr int kMaxFront = 32;
    out.clear();
    std::vector<int> front, cand;
    uint64_t seen = 0;
    for (int i = 0; i < int(pending.size()) && int(front.size()) < kMaxFront; ++i) {
        const uint64_t m = gm[pending[i]].all;
        if (!(m & seen)) front.push_back(i);
        seen |= m;
        if ((seen & all) == all) break;
    }
    for (int f : front) {
        const uint64_t sm = gm[pending[f]].all;
        grow_block(pending, gm, f, 0, k, smax, all, cand);
        out.push_back(cand);
        if (__builtin_popcountll(sm) > k || k >= n) continue;
        const int lo = __builtin_ctzll(sm), hi = 63 - __builtin_clzll(sm);
        for (int a = std::max(0, hi - k + 1); a <= std::min(lo, n - k); ++a) {
            const uint64_t w = ((uint64_t(1) << k) - 1) << a;
            grow_block(pending, gm, f, w, k, smax, all, cand);
            out.push_back(cand);
        }
    }
}

void remove_members(const std::vector<int> &pending, const std::vector<int> &members,
                    std::vector<int> &rest) {
    std::vector<char> taken(pending.size(), 0);
    for (int i : members) taken[i] = 1;
    rest.clear();
    for (int i = 0; i < int(pending.size()); ++i)
        if (!taken[i]) rest.push_back(pending[i]);
}

// Partition into dependency-respecting blocks of <= k qubits (plus at most
// smax selector qubits), handing each block to `emit` (its gate indices in
// order) as soon as it is chosen, so a caller can launch block b while
// block b + 1 is planned.  Each step takes the candidate block (see
// block_candidates) that absorbs the most gates together with the best
// candidate of the step after it, a one-step lookahead over the `look`
// largest candidates (look <= 1: plain greedy); ties go to the larger
// block now.
template <typename Emit>
void fuse_plan_each(int n, int ng, const qc_gate_t *gs, int k, int smax, int look, Emit &&emit) {
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    std::vector<GateMasks> gm(ng);
    for (int i = 0; i < ng; ++i) gm[i] = {gate_mask(gs[i]), gate_nd_mask(gs[i])};
    std::vector<int> pending(ng), rest, members;
    for (int i = 0; i < ng; ++i) pending[i] = i;
    std::vector<std::vector<int>> cands, next;
    while (!pending.empty()) {
        block_candidates(n, pending, gm, k, smax, all, cands);
        std::stable_sort(cands.begin(), cands.end(),
                         [](const std::vector<int> &a, const std::vector<int> &b) {
                             return a.size() > b.size();
                         });
        int pick = 0;
        if (look > 1) {
            size_t best_score = 0;
            for (int c = 0; c < std::min<int>(look, int(cands.size())); ++c) {
                remove_members(pending, cands[c], rest);
                size_t nx = 0;
                if (!rest.empty()) {
                    block_candidates(n, rest, gm, k, smax, all, next);
                    for (auto &v : next) nx = std::max(nx, v.size());
                }
                const size_t score = cands[c].size() + nx;
                if (score > best_score) {
                    best_score = score;
                    pick = c;
                }
            }
        }
        members.clear();
        for (int i : cands[pick]) members.push_back(pending[i]);
        remove_members(pending, cands[pick], rest);
        pending.swap(rest);
        if (!emit(members)) return;
    }
}

void fuse_plan(int n, int ng, const qc_gate_t *gs, int k, int smax, int look,
               std::vector<int> &block_of, int &n_blocks) {
    block_of.assign(ng, -1);
    n_blocks = 0;
    fuse_plan_each(n, ng, gs, k, smax, look, [&](const std::vector<int> &m) {
        for (int i : m) block_of[i] = n_blocks;
        ++n_blocks;
        return true;
    });
}

double sweep_bytes(int n, int dtype) {
    return 2.0 * double(uint64_t(1) << n) * (dtype == QC_C64 ? 8.0 : 16.0);
}

}  // namespace

// ======================================================================
// services used by the launchers
// ======================================================================
namespace qcx {

int knob(int which) {
    switch (which) {
    case QC_KNOB_MFMA_WG_PER_CU: return g_knob_mfma.load();
    case QC_KNOB_TILE_WG_PER_CU: return g_knob_tile.load();
    case QC_KNOB_MFMA_TILE_BITS: return g_knob_tbits.load();
    case QC_KNOB_TILE_BITS: return g_knob_tile_bits.load();
    case QC_KNOB_TILE_ENGINE: return g_knob_tile_engine.load();
    case QC_KNOB_WIDE_MIN_TILES: return g_knob_wide.load();
    default: return g_knob_look.load();
    }
}

int timer_begin(const char *name, hipStream_t s) {
    if (!g_timing.load(std::memory_order_relaxed) || capturing(s)) return -1;
    TimerRec r;
    r.name = name;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    (void)hipEventRecord(r.a, s);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_trecs.push_back(r);
    return int(g_trecs.size()) - 1;
}

void timer_end(int token, hipStream_t s) {
    if (token < 0) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    if (size_t(token) < g_trecs.size()) (void)hipEventRecord(g_trecs[token].b, s);
}

}  // namespace qcx

// ======================================================================
// C ABI
// ======================================================================
extern "C" {

const char *qc_status_string(int status) {
    switch (status) {
    case QC_OK: return "ok";
    case QC_ERR_ARG: return "invalid argument";
    case QC_ERR_QUBIT: return "invalid qubit";
    case QC_ERR_DTYPE: return "invalid dtype";
    case QC_ERR_UNSUPPORTED: return "unsupported";
    case QC_ERR_HIP: return "HIP error";
    case QC_ERR_NOMEM: return "out of memory";
    default: return "unknown status";
    }
}

const char *qc_last_error(void) { return t_err.c_str(); }

int qc_version(void) { return 10100; }

int qc_reserve(void *stream) {
    const hipStream_t hs = (hipStream_t)stream;
    if (capturing(hs)) return fail(QC_ERR_UNSUPPORTED, "qc_reserve inside a graph capture");
    DevCtx *c;
    int rc = get_ctx(&c);
    if (rc) return rc;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    c->ring_head = 0;
    c->prot_lo = c->prot_hi = 0;
    return QC_OK;
}

int qc_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (on) {
        for (auto &r : g_trecs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        g_trecs.clear();
        g_tsum.clear();
    }
    g_timing.store(on != 0);
    return QC_OK;
}

int qc_timing_query(const char *name, int64_t *count, double *total_ms) {
    if (!name || !count || !total_ms) return fail(QC_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &r : g_trecs) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        auto &acc = g_tsum[r.name];
        acc.first += 1;
        acc.second += double(ms);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_trecs.clear();
    auto it = g_tsum.find(name);
    *count = it == g_tsum.end() ? 0 : it->second.first;
    *total_ms = it == g_tsum.end() ? 0.0 : it->second.second;
    return QC_OK;
}

int qc_set_knob(int knob, int value) {
    if (knob == QC_KNOB_MFMA_WG_PER_CU) {
        if (value < 1 || value > 5) return fail(QC_ERR_ARG, "MFMA workgroups per CU must be 1..5");
        g_knob_mfma.store(value);
        return QC_OK;
    }
    if (knob == QC_KNOB_TILE_WG_PER_CU) {
        if (value < 1 || value > 16) return fail(QC_ERR_ARG, "tile workgroups per CU must be 1..16");
        g_knob_tile.store(value);
        return QC_OK;
    }
    if (knob == QC_KNOB_FUSE_LOOKAHEAD) {
        if (value < 0 || value > 256) return fail(QC_ERR_ARG, "fuse lookahead must be 0..256");
        g_knob_look.store(value);
        return QC_OK;
    }
    if (knob == QC_KNOB_MFMA_TILE_BITS) {
        if (value != 12 && value != 13) return fail(QC_ERR_ARG, "MFMA tile bits must be 12 or 13");
        g_knob_tbits.store(value);
        return QC_OK;
    }
    if (knob == QC_KNOB_TILE_BITS) {
        if (value < 6 || value > 13) return fail(QC_ERR_ARG, "tile bits must be 6..13");
        g_knob_tile_bits.store(value);
        return QC_OK;
    }
    if (knob == QC_KNOB_TILE_ENGINE) {
        if (value != 0 && value != 1) return fail(QC_ERR_ARG, "tile engine must be 0 or 1");
        g_knob_tile_engine.store(value);
        return QC_OK;
    }
    if (knob == QC_KNOB_WIDE_MIN_TILES) {
        if (value < 8 || value > 30) return fail(QC_ERR_ARG, "wide-tile minimum must be 8..30");
        g_knob_wide.store(value);
        return QC_OK;
    }
    return fail(QC_ERR_ARG, "unknown knob");
}

int qc_get_knob(int knob, int *value) {
    if (!value) return fail(QC_ERR_ARG, "NULL argument");
    if (knob != QC_KNOB_MFMA_WG_PER_CU && knob != QC_KNOB_TILE_WG_PER_CU &&
        knob != QC_KNOB_FUSE_LOOKAHEAD && knob != QC_KNOB_MFMA_TILE_BITS &&
        knob != QC_KNOB_TILE_BITS && knob != QC_KNOB_TILE_ENGINE && knob != QC_KNOB_WIDE_MIN_TILES)
        return fail(QC_ERR_ARG, "unknown knob");
    *value = qcx::knob(knob);
    return QC_OK;
}

int qc_state_init(qc_state_t s, uint64_t basis_index, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (basis_index >= (uint64_t(1) << s.n)) return fail(QC_ERR_ARG, "basis index out of range");
    hipError_t e = qcx::launch_init(s.amp, s.dtype, s.n, basis_index, (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "init");
}

int qc_state_copy(qc_state_t dst, qc_state_t src, void *stream) {
    int rc = check_state(dst);
    if (rc) return rc;
    if ((rc = check_state(src))) return rc;
    if (dst.n != src.n) return fail(QC_ERR_ARG, "states differ in qubit count");
    const uint64_t count = uint64_t(1) << dst.n;
    const char *a = (const char *)dst.amp, *b = (const char *)src.amp;
    const size_t la = count * (dst.dtype == QC_C64 ? 8 : 16), lb = count * (src.dtype == QC_C64 ? 8 : 16);
    if (a < b + lb && b < a + la) return fail(QC_ERR_ARG, "states overlap");
    hipError_t e = qcx::launch_copy(dst.amp, dst.dtype, src.amp, src.dtype, count,
                                    (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "copy");
}

int qc_state_diff(qc_state_t a, qc_state_t b, double *out_dev, void *stream) {
    int rc = check_state(a);
    if (rc) return rc;
    if ((rc = check_state(b))) return rc;
    if (a.n != b.n) return fail(QC_ERR_ARG, "states differ in qubit count");
    if (!out_dev) return fail(QC_ERR_ARG, "output pointer is NULL");
    DevCtx *c;
    if ((rc = get_ctx(&c))) return rc;
    hipError_t e = qcx::launch_diff(a.amp, a.dtype, b.amp, b.dtype, uint64_t(1) << a.n, out_dev,
                                    c->work, (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "diff");
}

int qc_apply_1q(qc_state_t s, int q, const double *u, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!u) return fail(QC_ERR_ARG, "matrix is NULL");
    if ((rc = check_qubits(s.n, &q, 1, "target"))) return rc;
    const int tp = bitpos(s.n, q);
    hipError_t e = qcx::launch_small_gate(s.amp, s.dtype, s.n, 1, &tp, 0, nullptr, nullptr, u,
                                          (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "apply_1q");
}

int qc_apply_2q(qc_state_t s, int qa, int qb, const double *u, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!u) return fail(QC_ERR_ARG, "matrix is NULL");
    if (s.n < 2) return fail(QC_ERR_QUBIT, "two-qubit gate on a one-qubit register");
    const int q[2] = {qa, qb};
    if ((rc = check_qubits(s.n, q, 2, "target"))) return rc;
    const int tp[2] = {bitpos(s.n, qa), bitpos(s.n, qb)};
    hipError_t e = qcx::launch_small_gate(s.amp, s.dtype, s.n, 2, tp, 0, nullptr, nullptr, u,
                                          (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "apply_2q");
}

int qc_apply_controlled(qc_state_t s, int n_ctrl, const int *ctrl, const int *ctrl_val,
                        int target, const double *u, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!u) return fail(QC_ERR_ARG, "matrix is NULL");
    if (n_ctrl < 0 || n_ctrl > QC_MAX_CTRLS || n_ctrl + 1 > s.n)
        return fail(QC_ERR_ARG, "control count out of range");
    if (n_ctrl > 0 && (!ctrl || !ctrl_val)) return fail(QC_ERR_ARG, "control arrays are NULL");
    int all[QC_MAX_CTRLS + 1];
    all[0] = target;
    for (int j = 0; j < n_ctrl; ++j) {
        all[1 + j] = ctrl[j];
        if (ctrl_val[j] != 0 && ctrl_val[j] != 1)
            return fail(QC_ERR_ARG, "control value must be 0 or 1");
    }
    if ((rc = check_qubits(s.n, all, n_ctrl + 1, "qubit"))) return rc;
    int cp[QC_MAX_CTRLS + 1], cv[QC_MAX_CTRLS + 1];
    for (int j = 0; j < n_ctrl; ++j) {
        cp[j] = bitpos(s.n, ctrl[j]);
        cv[j] = ctrl_val[j];
    }
    hipError_t e;
    const bool diag_one = u[2] == 0.0 && u[3] == 0.0 && u[4] == 0.0 && u[5] == 0.0 &&
                          u[0] == 1.0 && u[1] == 0.0;
    if (diag_one) {
        // only the target-1 part of the control subspace changes
        cp[n_ctrl] = bitpos(s.n, target);
        cv[n_ctrl] = 1;
        e = qcx::launch_phase(s.amp, s.dtype, s.n, n_ctrl + 1, cp, cv, u[6], u[7],
                              (hipStream_t)stream);
    } else {
        const int tp = bitpos(s.n, target);
        e = qcx::launch_small_gate(s.amp, s.dtype, s.n, 1, &tp, n_ctrl, cp, cv, u,
                                   (hipStream_t)stream);
    }
    return e == hipSuccess ? QC_OK : hip_fail(e, "apply_controlled");
}

}  // extern "C"

namespace {

// FP32 matrix-core operand layout of a 32x32 complex U (see qc_fused_mfma.hip).
void mfma_operand_c64(const std::vector<cd> &u, std::vector<float> &out);

// Apply a k-qubit block, multiplexed over `ns` selector qubits `sq` when
// ns > 0: `u` holds the 2^ns matrices U_s one after the other (s = the
// values of the selector qubits, sq[0] = most significant bit).
int fused_apply(qc_state_t s, int k, const int *qubits, int ns, const int *sq,
                const std::vector<cd> &u, hipStream_t stream) {
    DevCtx *c;
    int rc = get_ctx(&c);
    if (rc) return rc;
    qcx::FusedGeom g{};
    g.k = k;
    int pos[QC_MAX_FUSED];
    for (int j = 0; j < k; ++j) pos[j] = bitpos(s.n, qubits[j]);
    int srt[QC_MAX_FUSED];
    std::copy(pos, pos + k, srt);
    std::sort(srt, srt + k);
    g.n_pos = k;
    for (int j = 0; j < k; ++j) g.pos[j] = uint32_t(srt[j]);
    for (int r = 0; r < (1 << k); ++r) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((r >> (k - 1 - j)) & 1) o |= uint64_t(1) << pos[j];
        g.tgt_off[r] = o;
    }
    g.n_sel = ns;
    for (int j = 0; j < ns; ++j) g.sel_pos[j] = uint32_t(bitpos(s.n, sq[j]));
    const size_t dd = size_t(1) << (2 * k);
    void *dev = nullptr;
    hipError_t e;
    // the matrix-core kernel moves 16-byte pairs of amplitudes
    const bool aligned16 = (reinterpret_cast<uintptr_t>(s.amp) & 15) == 0;
    if (s.dtype == QC_C64 && k == 5 && s.n >= 12 + ns && aligned16) {
        std::vector<float> op, all;
        for (int v = 0; v < (1 << ns); ++v) {
            mfma_operand_c64(std::vector<cd>(u.begin() + v * dd, u.begin() + (v + 1) * dd), op);
            all.insert(all.end(), op.begin(), op.end());
        }
        // the kernel's tile counters follow the operands, zeroed by the same upload
        const size_t op_floats = all.size();
        all.resize(op_floats + qcx::kMfmaTicketBytes / sizeof(float), 0.0f);
        if ((rc = stage(c, all.data(), all.size() * sizeof(float), stream, &dev))) return rc;
        e = qcx::launch_fused_mfma_c64(
            s.amp, s.n, g, static_cast<const float *>(dev),
            reinterpret_cast<unsigned *>(static_cast<float *>(dev) + op_floats), stream);
    } else if (s.dtype == QC_C128 && k == 5 && aligned16 && qcx::fused_mfma_c128_fits(s.n, g)) {
        // FP64 matrix cores: per selector value Ur, Ui, Ur + Ui, then the
        // kernel's tile counters, zeroed by the same upload
        std::vector<double> all(size_t(3 * 1024) << ns);
        for (int v = 0; v < (1 << ns); ++v)
            for (int r = 0; r < 32; ++r)
                for (int c = 0; c < 32; ++c) {
                    const cd x = u[size_t(v) * dd + size_t(r) * 32 + c];
                    double *m = all.data() + size_t(v) * 3072;
                    m[r * 32 + c] = x.real();
                    m[1024 + r * 32 + c] = x.imag();
                    m[2048 + r * 32 + c] = x.real() + x.imag();
                }
        const size_t op_doubles = all.size();
        all.resize(op_doubles + qcx::kMfmaTicketBytes / sizeof(double), 0.0);
        if ((rc = stage(c, all.data(), all.size() * sizeof(double), stream, &dev))) return rc;
        e = qcx::launch_fused_mfma_c128(
            s.amp, s.n, g, static_cast<const double *>(dev),
            reinterpret_cast<unsigned *>(static_cast<double *>(dev) + op_doubles), stream);
    } else if (s.dtype == QC_C64) {
        std::vector<float> f(u.size() * 2);
        for (size_t i = 0; i < u.size(); ++i) {
            f[2 * i] = float(u[i].real());
            f[2 * i + 1] = float(u[i].imag());
        }
        if ((rc = stage(c, f.data(), f.size() * sizeof(float), stream, &dev))) return rc;
        e = qcx::launch_fused_valu(s.amp, s.dtype, s.n, g, dev, stream);
    } else {
        if ((rc = stage(c, u.data(), u.size() * sizeof(cd), stream, &dev))) return rc;
        e = qcx::launch_fused_valu(s.amp, s.dtype, s.n, g, dev, stream);
    }
    return e == hipSuccess ? QC_OK : hip_fail(e, "apply_fused_k");
}

// One gate, one launch (the plain per-gate path).
int apply_gate_unfused(qc_state_t s, const qc_gate_t &g, qc_exec_stats_t &st, void *stream) {
    const double sweep = sweep_bytes(s.n, s.dtype);
    const int nq = g.n_targets + g.n_ctrls;
    int rc;
    if (g.n_targets == 1) {
        rc = g.n_ctrls ? qc_apply_controlled(s, g.n_ctrls, g.ctrls, g.ctrl_vals, g.targets[0],
                                             g.matrix, stream)
                       : qc_apply_1q(s, g.targets[0], g.matrix, stream);
        const double *u = g.matrix;
        const bool phase_only = g.n_ctrls && u[2] == 0 && u[3] == 0 && u[4] == 0 && u[5] == 0 &&
                                u[0] == 1.0 && u[1] == 0;
        st.state_bytes += sweep / double(uint64_t(1) << (g.n_ctrls + (phase_only ? 1 : 0)));
    } else if (g.n_targets == 2 && g.n_ctrls == 0) {
        rc = qc_apply_2q(s, g.targets[0], g.targets[1], g.matrix, stream);
        st.state_bytes += sweep;
    } else if (nq <= QC_MAX_FUSED) {
        int bq[QC_MAX_FUSED];
        for (int j = 0; j < g.n_targets; ++j) bq[j] = g.targets[j];
        for (int j = 0; j < g.n_ctrls; ++j) bq[g.n_targets + j] = g.ctrls[j];
        std::vector<const qc_gate_t *> one{&g};
        rc = fused_apply(s, nq, bq, 0, nullptr, block_matrix(nq, bq, one), (hipStream_t)stream);
        st.state_bytes += sweep;
    } else {
        rc = fail(QC_ERR_UNSUPPORTED, "gate with more than 5 qubits and targets > 1");
    }
    if (rc == QC_OK) {
        st.launches += 1;
        st.sweeps += 1;
    }
    return rc;
}

// ---- LDS tile runs -----------------------------------------------------------

struct TileClass {
    bool tileable;      // one- or two-target gate
    uint64_t tbits;     // bit positions that must be tile bits
    uint64_t touch;     // qubit labels the gate involves
};

bool is_diag_1q(const double *u) { return u[2] == 0 && u[3] == 0 && u[4] == 0 && u[5] == 0; }
bool is_x_1q(const double *u) {
    return u[0] == 0 && u[1] == 0 && u[2] == 1 && u[3] == 0 && u[4] == 1 && u[5] == 0 && u[6] == 0 &&
           u[7] == 0;
}

TileClass tile_class(int n, const qc_gate_t &g) {
    TileClass c{};
    c.touch = gate_mask(g);
    if (g.n_targets == 1) {
        c.tileable = true;
        c.tbits = is_diag_1q(g.matrix) ? 0 : uint64_t(1) << bitpos(n, g.targets[0]);
    } else if (g.n_targets == 2) {
        c.tileable = true;
        c.tbits = (uint64_t(1) << bitpos(n, g.targets[0])) | (uint64_t(1) << bitpos(n, g.targets[1]));
    }
    return c;
}

// Op list of one tile run for the tile bit set P (bit-position mask), with
// two peephole rewrites that keep the product unchanged:
//  * an unconditioned one-qubit gate on a tile bit is held back and
//    multiplied into the gates that follow on the same bit, until an op
//    touches that bit (it commutes with every op on other bits);
//  * diagonal phase terms (CZ, CP, diagonal gates, controlled phases) are
//    collected into one multi-term TILE_PHASES op; a term first flushes the
//    held gates on its bits, and a later gate on one of its bits first
//    emits the collected terms (diagonal terms commute with each other and
//    with every op on other bits).
// Ops that touch held bits flush them first; reductions (TILE_GRAD) are
// added as ops that touch their bit (the reduction is invariant under
// unitaries on other bits applied to both vectors).
struct TileOpBuilder {
    int n;
    uint64_t P;
    std::vector<qcx::TileOp> &out;
    cd held[qcx::kTileMaxBits][4];
    uint32_t held_bits = 0;
    int kron_max = qcx::kKronMax;   // 1: held bits are flushed one op per bit
    bool fans = true;                // false: no TILE_FAN ops (kernels without them)
    struct Term {
        uint32_t mlo, vlo;
        uint64_t mhi, vhi;
        cd phase;
    };
    std::vector<Term> terms;   // diagonal terms collected since the last emission
    uint32_t ph_bits = 0;      // the tile bits they test
    // controlled-X gates collected for one TILE_XPERM op: no target is
    // another's target or control, so they commute and their product is
    // its own inverse.  (Pending phase terms never test a collected target,
    // and collected gates never target a bit a pending term tests: the two
    // collections commute.)
    qcx::TileOp xp{};
    uint32_t xp_bits = 0, xp_tgt = 0;   // the tile bits the gates touch / target
    bool xperms = true;                 // false: no TILE_XPERM ops (kernels without them)

    TileOpBuilder(int n_, uint64_t P_, std::vector<qcx::TileOp> &o) : n(n_), P(P_), out(o) {}

    int cidx(int p) const { return __builtin_popcountll(P & ((uint64_t(1) << p) - 1)); }
    bool in_tile(int p) const { return (P >> p) & 1; }

    void flush_bit(int b) {
        if (!((held_bits >> b) & 1)) return;
        const cd *m = held[b];
        qcx::TileOp op{};
        const bool diag = m[1] == 0.0 && m[2] == 0.0;
        op.kind = diag ? qcx::TILE_DIAG1 : qcx::TILE_DENSE1;
        op.b0 = b;
        if (diag) {
            op.u[0] = m[0].real(); op.u[1] = m[0].imag();
            op.u[2] = m[3].real(); op.u[3] = m[3].imag();
        } else {
            for (int i = 0; i < 4; ++i) {
                op.u[2 * i] = m[i].real();
                op.u[2 * i + 1] = m[i].imag();
            }
        }
        out.push_back(op);
        held_bits &= ~(1u << b);
    }
    // Two held gates on bits a and b: one two-qubit op with the Kronecker
    // product U_a (x) U_b (local index 2 bit(a) + bit(b)), one pass over
    // the tile instead of two at the same flops per amplitude.
    // one-qubit matrices held on 2..kKronMax bits: one op, applied to each
    // group of amplitudes in registers
    void flush_group(const int *bits, int g) {
        if (g < 2) {   // a single bit is a plain one-qubit op
            for (int j = 0; j < g; ++j) flush_bit(bits[j]);
            return;
        }
        qcx::TileOp op{};
        op.kind = qcx::TILE_KRON;
        op.b0 = g;
        op.b1 = 0;
        for (int j = 0; j < g; ++j) {
            op.b1 |= bits[j] << (5 * j);
            for (int e = 0; e < 4; ++e) {
                op.u[8 * j + 2 * e] = held[bits[j]][e].real();
                op.u[8 * j + 2 * e + 1] = held[bits[j]][e].imag();
            }
            held_bits &= ~(1u << bits[j]);
        }
        out.push_back(op);
    }
    void flush_bits(uint32_t bits) {
        bits &= held_bits;
        int group[qcx::kKronMax], g = 0;
        for (int b = 0; bits >> b; ++b) {
            if (!((bits >> b) & 1)) continue;
            group[g++] = b;
            if (g == kron_max) {
                if (g == 1) flush_bit(group[0]);
                else flush_group(group, g);
                g = 0;
            }
        }
        if (g == 1) flush_bit(group[0]);
        else if (g > 1) flush_group(group, g);
    }
    // The collected terms as ops: one TILE_FAN op when they are the phases
    // of controlled-phase gates sharing an in-tile target (conditions all
    // "= 1", each term testing the target and at most one other bit), else
    // TILE_PHASES ops of at most kTilePhaseTerms terms testing at most
    // kPhaseTableBits tile bits, in order (the terms commute), a lone term
    // or one testing more bits as a TILE_PHASE op.
    void emit_phases() {
        // a lone term joins the fan form only behind a one-qubit gate on one
        // of its bits (the pair becomes one dense-then-fan op)
        const bool behind_dense = !out.empty() && out.back().kind == qcx::TILE_DENSE1 &&
                                  out.back().cmask_lo == 0 && out.back().cmask_hi == 0;
        if (!terms.empty() &&
            !(fans && (terms.size() > 1 || behind_dense) && emit_fan())) {
            qcx::TileOp op{};
            int nt = 0;
            uint32_t bits = 0;
            auto flush = [&]() {
                if (nt == 1) {
                    qcx::TileOp one{};
                    one.kind = qcx::TILE_PHASE;
                    one.cmask_lo = op.pm_lo[0];
                    one.cval_lo = op.pv_lo[0];
                    one.cmask_hi = op.pm_hi[0];
                    one.cval_hi = op.pv_hi[0];
                    one.u[0] = op.u[0];
                    one.u[1] = op.u[1];
                    out.push_back(one);
                } else if (nt > 1) {
                    op.kind = qcx::TILE_PHASES;
                    op.b0 = nt;
                    op.b1 = int32_t(bits);
                    out.push_back(op);
                }
                op = qcx::TileOp{};
                nt = 0;
                bits = 0;
            };
            for (const Term &tm : terms) {
                if (nt == qcx::kTilePhaseTerms ||
                    __builtin_popcount(bits | tm.mlo) > qcx::kPhaseTableBits)
                    flush();
                op.pm_lo[nt] = tm.mlo;
                op.pv_lo[nt] = tm.vlo;
                op.pm_hi[nt] = tm.mhi;
                op.pv_hi[nt] = tm.vhi;
                op.u[2 * nt] = tm.phase.real();
                op.u[2 * nt + 1] = tm.phase.imag();
                ++nt;
                bits |= tm.mlo;
                if (__builtin_popcount(tm.mlo) > qcx::kPhaseTableBits) flush();
            }
            flush();
        }
        terms.clear();
        ph_bits = 0;
    }
    // TILE_FAN op(s) for the collected terms if they have the fan form;
    // false (nothing emitted) otherwise.  Out-of-tile controls beyond
    // kTilePhaseTerms go to further TILE_FAN ops on the same target.
    bool emit_fan() {
        // the kernels keep one group entry per kBlock amplitudes for at most
        // 2^13-amplitude tiles (64 KiB of complex64, the LDS tile limit)
        if (__builtin_popcountll(P) > 13) return false;
        uint32_t common = ~0u;
        for (const Term &tm : terms) {
            const int lo = __builtin_popcount(tm.mlo), hi = __builtin_popcountll(tm.mhi);
            if (tm.vlo != tm.mlo || tm.vhi != tm.mhi || lo < 1 || hi > 1 || lo + hi > 2) return false;
            common &= tm.mlo;
        }
        if (!common) return false;
        // the target: the bit of the one-qubit gate just before, if the terms
        // share it (the two then merge into one op), else the lowest shared bit
        int t = __builtin_ctz(common);
        if (!out.empty() && out.back().kind == qcx::TILE_DENSE1 && ((common >> out.back().b0) & 1))
            t = out.back().b0;
        else if (terms.size() == 1)
            return false;
        cd bitph[qcx::kTileMaxBits];
        for (auto &v : bitph) v = 1.0;
        uint32_t ctl = 0;
        std::vector<std::pair<uint64_t, cd>> hi;   // out-of-tile control bit, phase
        for (const Term &tm : terms) {
            if (tm.mhi) {
                auto it = std::find_if(hi.begin(), hi.end(),
                                       [&](const std::pair<uint64_t, cd> &h) { return h.first == tm.mhi; });
                if (it == hi.end()) hi.push_back({tm.mhi, tm.phase});
                else it->second *= tm.phase;
                continue;
            }
            const uint32_t c = tm.mlo & ~(1u << t);   // the control bit, or none
            const int b = c ? __builtin_ctz(c) : t;
            bitph[b] *= tm.phase;
            ctl |= c;
        }
        size_t h0 = 0;
        do {
            qcx::TileOp op{};
            op.kind = qcx::TILE_FAN;
            op.b0 = t;
            if (h0 == 0) {   // the in-tile controls and target-only terms go with the first op
                op.b1 = int32_t(ctl);
                for (int b = 0; b < qcx::kTileMaxBits; ++b) {
                    op.u[2 * b] = (b == t || ((ctl >> b) & 1)) ? bitph[b].real() : 1.0;
                    op.u[2 * b + 1] = (b == t || ((ctl >> b) & 1)) ? bitph[b].imag() : 0.0;
                }
            } else {
                op.u[2 * t] = 1.0;
            }
            int k = 0;
            for (; h0 < hi.size() && k < qcx::kTilePhaseTerms; ++h0, ++k) {
                op.fan_mask[k] = hi[h0].first;
                op.fan_ph[2 * k] = hi[h0].second.real();
                op.fan_ph[2 * k + 1] = hi[h0].second.imag();
            }
            op.pad = k;
            out.push_back(op);
        } while (h0 < hi.size());
        return true;
    }
    // one diagonal term: multiply by `phase` where the conditions hold
    void add_phase(uint32_t mlo, uint32_t vlo, uint64_t mhi, uint64_t vhi, cd phase) {
        // all held gates go out now, in groups of kron_max bits (a ladder of
        // diagonal gates would otherwise flush them one bit at a time)
        if (mlo & held_bits) flush_bits(held_bits);
        if (mlo & xp_tgt) emit_xperm();
        terms.push_back({mlo, vlo, mhi, vhi, phase});
        ph_bits |= mlo;
    }
    void emit_xperm() {
        if (xp.b0 > 0) {
            xp.kind = qcx::TILE_XPERM;
            out.push_back(xp);
        }
        xp = qcx::TileOp{};
        xp_bits = xp_tgt = 0;
    }
    // X on tile bit t where the controls hold (clo/cvlo in the tile, chi/cvhi
    // outside)
    void add_xgate(int t, uint32_t clo, uint32_t cvlo, uint64_t chi, uint64_t cvhi) {
        const uint32_t tb = 1u << t;
        flush_bits(clo | tb);
        if (ph_bits & tb) emit_phases();
        if ((xp_bits & tb) || (clo & xp_tgt) || xp.b0 == qcx::kXpermTerms) emit_xperm();
        const int k = xp.b0++;
        xp.x_cm[k] = clo;
        xp.x_cv[k] = cvlo;
        xp.x_t[k] = uint32_t(t);
        xp.x_hm[k] = chi;
        xp.x_hv[k] = cvhi;
        xp_bits |= clo | tb;
        xp_tgt |= tb;
    }
    void add_op(const qcx::TileOp &op, uint32_t touched) {
        flush_bits(touched);
        if (ph_bits & touched) emit_phases();
        if (xp_bits & touched) emit_xperm();
        out.push_back(op);
    }
    void add_1q(int b, const double *u) {
        if ((ph_bits >> b) & 1) emit_phases();
        if ((xp_bits >> b) & 1) emit_xperm();
        const cd m[4] = {cd(u[0], u[1]), cd(u[2], u[3]), cd(u[4], u[5]), cd(u[6], u[7])};
        if (!((held_bits >> b) & 1)) {
            for (int i = 0; i < 4; ++i) held[b][i] = m[i];
            held_bits |= 1u << b;
            return;
        }
        const cd *h = held[b];   // new = m * h (m applied after h)
        const cd r[4] = {m[0] * h[0] + m[1] * h[2], m[0] * h[1] + m[1] * h[3],
                         m[2] * h[0] + m[3] * h[2], m[2] * h[1] + m[3] * h[3]};
        for (int i = 0; i < 4; ++i) held[b][i] = r[i];
    }
    void add_gate(const qc_gate_t &g) {
        uint32_t clo = 0, cvlo = 0;
        uint64_t chi = 0, cvhi = 0;
        for (int j = 0; j < g.n_ctrls; ++j) {
            const int p = bitpos(n, g.ctrls[j]);
            if (in_tile(p)) {
                clo |= 1u << cidx(p);
                if (g.ctrl_vals[j]) cvlo |= 1u << cidx(p);
            } else {
                chi |= uint64_t(1) << p;
                if (g.ctrl_vals[j]) cvhi |= uint64_t(1) << p;
            }
        }
        const double *u = g.matrix;
        if (g.n_targets == 1) {
            const int tp = bitpos(n, g.targets[0]);
            const bool t_in = in_tile(tp);
            const uint32_t tb = t_in ? 1u << cidx(tp) : 0u;
            const uint64_t th = t_in ? 0 : uint64_t(1) << tp;
            if (is_diag_1q(u)) {
                if (g.n_ctrls == 0 && t_in) {
                    add_1q(cidx(tp), u);
                    return;
                }
                // diagonal: a term for target 1 and, unless U00 == 1, for target 0
                add_phase(clo | tb, cvlo | tb, chi | th, cvhi | th, cd(u[6], u[7]));
                if (!(u[0] == 1.0 && u[1] == 0.0))
                    add_phase(clo | tb, cvlo, chi | th, cvhi, cd(u[0], u[1]));
                return;
            }
            if (g.n_ctrls == 0) {
                add_1q(cidx(tp), u);
                return;
            }
            if (xperms && t_in && is_x_1q(u)) {
                add_xgate(cidx(tp), clo, cvlo, chi, cvhi);
                return;
            }
            qcx::TileOp op{};
            op.kind = qcx::TILE_DENSE1;
            op.b0 = cidx(tp);
            op.cmask_lo = clo;
            op.cval_lo = cvlo;
            op.cmask_hi = chi;
            op.cval_hi = cvhi;
            for (int i = 0; i < 8; ++i) op.u[i] = u[i];
            add_op(op, clo | tb);
        } else {
            qcx::TileOp op{};
            op.kind = qcx::TILE_DENSE2;
            op.b0 = cidx(bitpos(n, g.targets[0]));
            op.b1 = cidx(bitpos(n, g.targets[1]));
            op.cmask_lo = clo;
            op.cval_lo = cvlo;
            op.cmask_hi = chi;
            op.cval_hi = cvhi;
            for (int i = 0; i < 32; ++i) op.u[i] = u[i];
            add_op(op, clo | (1u << op.b0) | (1u << op.b1));
        }
    }
    void finish() {
        emit_phases();
        emit_xperm();
        flush_bits(held_bits);
    }
};

// An unconditioned one-qubit op followed by a phase op becomes one
// TILE_DENSE1_PHASES op: one pass over the tile instead of two.  Only the
// ops from index `begin` on (one run's list) are merged.
void merge_dense_phases(std::vector<qcx::TileOp> &ops, size_t begin) {
    std::vector<qcx::TileOp> out;   // the run's merged list (the ops before begin stay put)
    out.reserve(ops.size() - begin);
    for (size_t k = begin; k < ops.size(); ++k) {
        const qcx::TileOp &d = ops[k];
        if (k + 1 < ops.size() && d.kind == qcx::TILE_DENSE1 && d.cmask_lo == 0 && d.cmask_hi == 0) {
            const qcx::TileOp &p = ops[k + 1];
            qcx::TileOp mo{};
            bool ok = false;
            if (p.kind == qcx::TILE_PHASES && p.cmask_lo == 0 && p.cmask_hi == 0) {
                mo = p;          // terms and their bit set b1
                mo.pad = p.b0;   // term count
                ok = true;
            } else if (p.kind == qcx::TILE_PHASE &&
                       __builtin_popcount(p.cmask_lo) <= qcx::kPhaseTableBits) {
                mo.pm_lo[0] = p.cmask_lo;   // the op's conditions become the term's
                mo.pv_lo[0] = p.cval_lo;
                mo.pm_hi[0] = p.cmask_hi;
                mo.pv_hi[0] = p.cval_hi;
                mo.u[0] = p.u[0];
                mo.u[1] = p.u[1];
                mo.pad = 1;
                mo.b1 = int32_t(p.cmask_lo);
                ok = true;
            }
            if (!ok && p.kind == qcx::TILE_FAN && p.b0 == d.b0) {
                mo = p;
                mo.kind = qcx::TILE_DENSE1_FAN;
                for (int i = 0; i < 8; ++i) mo.u1[i] = d.u[i];
                out.push_back(mo);
                ++k;
                continue;
            }
            if (ok) {
                mo.kind = qcx::TILE_DENSE1_PHASES;
                mo.b0 = d.b0;
                mo.cmask_lo = mo.cval_lo = 0;
                mo.cmask_hi = mo.cval_hi = 0;
                for (int i = 0; i < 8; ++i) mo.u1[i] = d.u[i];
                out.push_back(mo);
                ++k;
                continue;
            }
        }
        out.push_back(d);
    }
    ops.resize(begin);
    ops.insert(ops.end(), out.begin(), out.end());
}

// Convert a list of gates into the op list of one tile run.
void tile_ops_for(int n, const qc_gate_t *gs, const std::vector<int> &idx, uint64_t P,
                  std::vector<qcx::TileOp> &out) {
    const size_t begin = out.size();
    TileOpBuilder B(n, P, out);
    for (int i : idx) B.add_gate(gs[i]);
    B.finish();
    merge_dense_phases(out, begin);
}

// LDS tile of the tile-run kernel: at most 64 KiB (2^13 complex64 or 2^12
// complex128 amplitudes), capped by QC_KNOB_TILE_BITS and by n.
constexpr int kRtMinTileBits = 8;           // register tiles need >= 2^8 tiles in the register

// complex128 takes the wide register tiles (2^13 amplitudes) when the
// register engine runs them and there are 2^QC_KNOB_WIDE_MIN_TILES of them:
// one workgroup per CU needs more tiles per workgroup to hide its latency
// (at 24 qubits the 2^12 tiles are faster, at 28 the wide ones)
int tile_bits_for(const qc_state_t &s) {
    const bool wide = g_knob_tile_engine.load() == 1 &&
                      s.n - qcx::kRtWideBits >= std::max(kRtMinTileBits, g_knob_wide.load());
    return std::min({s.n, s.dtype == QC_C64 || wide ? 13 : 12, g_knob_tile_bits.load()});
}

// Greedy run formation: starting from the earliest pending gate, a gate
// joins the run when none of its qubits is held by an earlier gate left out
// and its non-diagonal targets still fit in the m tile bits.
struct TileRun {
    uint64_t P;              // tile bits (bit-position mask); 0 for a standalone gate
    std::vector<int> gates;  // gate indices in order
};

// Greedy run formation: starting from the earliest pending gate, a gate
// joins the run when none of its qubits is held by an earlier gate left out
// and its non-diagonal targets (plus extra_tbits[i], if given) still fit in
// the m tile bits.  Gates that cannot be tiled become standalone runs.
void form_runs(int n, int m, int ng, const qc_gate_t *gs, const uint64_t *extra_tbits,
               std::vector<TileRun> &runs) {
    const int low = std::min(m, 5);      // always-resident low bits: runs of >= 32 amplitudes
    const uint64_t low_mask = (uint64_t(1) << low) - 1;
    const uint64_t all = (uint64_t(1) << n) - 1;
    std::vector<int> pending(ng);
    for (int i = 0; i < ng; ++i) pending[i] = i;
    runs.clear();
    while (!pending.empty()) {
        if (!tile_class(n, gs[pending[0]]).tileable) {
            runs.push_back({0, {pending[0]}});
            pending.erase(pending.begin());
            continue;
        }
        uint64_t P = low_mask, blocked = 0;
        std::vector<int> run, rest;
        for (int idx : pending) {
            const TileClass tc = tile_class(n, gs[idx]);
            const uint64_t tb = tc.tbits | (extra_tbits ? extra_tbits[idx] : 0);
            if (!(tc.touch & blocked) && tc.tileable && __builtin_popcountll(P | tb) <= m &&
                blocked != all) {
                P |= tb;
                run.push_back(idx);
            } else {
                blocked |= tc.touch;
                rest.push_back(idx);
            }
        }
        for (int p = 0; __builtin_popcountll(P) < m && p < n; ++p) P |= uint64_t(1) << p;
        runs.push_back({P, run});
        pending.swap(rest);
    }
}

qcx::TileArgs tile_args(int n, int m, uint64_t P, int n_ops) {
    qcx::TileArgs a{};
    a.m = m;
    a.n_ops = n_ops;
    a.n_tiles = uint64_t(1) << (n - m);
    for (int p = 0, j = 0; p < n; ++p)
        if ((P >> p) & 1) a.pos[j++] = uint32_t(p);
    return a;
}

// ---------------------------------------------------------------------------
// Register-resident tile programs: the op list of a run (TileOpBuilder) is
// lowered to RtOps for a layout that changes as the run proceeds (see RtOp
// in qc_internal.h).  Slots 0..rb-1 are the register (element index) bits,
// slot rb + k is bit k of the thread index.  Before an op whose
// non-diagonal targets are not all register slots, an RT_REMAP brings them
// in; the register set chosen then holds the targets plus the bits whose
// next use comes soonest (farthest next use leaves first), so one exchange
// serves as many later ops as possible.
constexpr uint32_t kRtLdsTabMax = 16384;   // LDS bytes for the lane tables of one program
struct RtLayout {
    int m = 0, rb = 0;
    int bit_of[32];    // slot -> compressed tile bit
    int slot_of[32];   // compressed tile bit -> slot
};

struct RtLowering {
    int n, m, rb, dtype;
    uint64_t P;
    const qcx::TileOp *ops;
    int n_ops;
    std::vector<uint32_t> need;   // per op: compressed bits that must be register slots
    RtLayout L;
    std::vector<qcx::RtOp> out;
    double scale = 1.0;           // deferred factor of the unscaled Hadamards
    // table blob: lane tables (copied to LDS) and wave / window tables
    std::vector<unsigned char> lblob, gblob;
    bool too_wide = false;        // an op needs more out-of-tile windows than kRtWindows
    bool adjoint = false;         // backward program: gradient ops, no deferred scale
    bool defer_scale = false;     // leave the Hadamard factor to the caller (no RT_SCALE)
    bool had_remap = false;       // an RT_REMAP was emitted before

    static uint32_t add_tab(std::vector<unsigned char> &b, const void *p, size_t bytes) {
        while (b.size() % 16) b.push_back(0);
        const uint32_t off = uint32_t(b.size());
        const unsigned char *c = static_cast<const unsigned char *>(p);
        b.insert(b.end(), c, c + bytes);
        return off;
    }
    // complex table in the program's precision
    uint32_t add_ctab(std::vector<unsigned char> &b, const std::vector<cd> &t) {
        if (is64()) {
            std::vector<float> f(2 * t.size());
            for (size_t i = 0; i < t.size(); ++i) {
                f[2 * i] = float(t[i].real());
                f[2 * i + 1] = float(t[i].imag());
            }
            return add_tab(b, f.data(), f.size() * sizeof(float));
        }
        std::vector<double> d(2 * t.size());
        for (size_t i = 0; i < t.size(); ++i) {
            d[2 * i] = t[i].real();
            d[2 * i + 1] = t[i].imag();
        }
        return add_tab(b, d.data(), d.size() * sizeof(double));
    }
    // windows of 3 consecutive global positions covering the bits of `hi`
    static std::vector<int> windows_of(uint64_t hi) {
        std::vector<int> lo;
        for (int p = 0; p < 64; ++p)
            if ((hi >> p) & 1) {
                lo.push_back(p);
                p += 2;
            }
        return lo;
    }

    int E() const { return 1 << rb; }
    bool is64() const { return dtype == QC_C64; }
    void put(double *arr, int i, double v) {
        if (is64()) qcx::rt_vals<float>(arr)[i] = float(v);
        else arr[i] = v;
    }
    void put_c(double *arr, int i, cd v) {
        put(arr, 2 * i, v.real());
        put(arr, 2 * i + 1, v.imag());
    }
    uint32_t swz(uint32_t j) const {
        return is64() ? qcx::rt_swizzle<4>(j) : qcx::rt_swizzle<3>(j);
    }
    // element part of the tile index of element e under layout l
    uint32_t dep_reg(const RtLayout &l, int e) const {
        uint32_t j = 0;
        for (int i = 0; i < rb; ++i)
            if ((e >> i) & 1) j |= 1u << l.bit_of[i];
        return j;
    }

    // ops here are the expanded ones of rt_expand (at most two targets)
    static uint32_t need_of(const qcx::TileOp &op) {
        switch (op.kind) {
        case qcx::TILE_DENSE1: return 1u << op.b0;
        case qcx::TILE_DENSE2: return (1u << op.b0) | (1u << op.b1);
        case qcx::TILE_XPERM: {
            uint32_t b = 0;
            for (int k = 0; k < op.b0; ++k) b |= 1u << op.x_t[k];
            return b;
        }
        case qcx::TILE_GRAD:
        case qcx::TILE_GRAD_APPLY:
        case qcx::TILE_GRAD_APPLY_REAL:
        case qcx::TILE_GRAD_APPLY_DIAG:
        case qcx::TILE_GRAD_APPLY2_DIAG_REAL: return 1u << op.b0;
        default: return 0;   // diagonal ops: any slot
        }
    }

    // initial layout: lanes on the lowest compressed bits (coalesced loads),
    // registers on the earliest-needed other bits, wavefronts on the rest
    void initial_layout() {
        L.m = m;
        L.rb = rb;
        const int tb = m - rb;
        const int lanes = std::min(tb, 6);
        std::vector<int> order;   // candidate register bits by first use
        std::vector<int> first(m, INT32_MAX);
        for (int i = n_ops - 1; i >= 0; --i)
            for (int b = 0; b < m; ++b)
                if ((need[i] >> b) & 1) first[b] = i;
        std::vector<int> rest;
        for (int b = lanes; b < m; ++b) rest.push_back(b);
        std::stable_sort(rest.begin(), rest.end(), [&](int a, int b) { return first[a] < first[b]; });
        int slot = 0;
        std::vector<bool> used(m, false);
        for (int k = 0; k < rb; ++k) {   // register slots
            L.bit_of[slot++] = rest[k];
            used[rest[k]] = true;
        }
        for (int b = 0; b < lanes; ++b) {   // lane slots
            L.bit_of[slot++] = b;
            used[b] = true;
        }
        for (int b = 0; b < m; ++b)          // wavefront slots
            if (!used[b]) L.bit_of[slot++] = b;
        for (int sl = 0; sl < m; ++sl) L.slot_of[L.bit_of[sl]] = sl;
    }

    int next_use(int b, int from) const {
        for (int i = from; i < n_ops; ++i)
            if ((need[i] >> b) & 1) return i;
        return INT32_MAX;
    }

    void emit_remap(const RtLayout &nl) {
        qcx::RtOp r{};
        r.kind = qcx::rt_code(qcx::RT_REMAP, 0);
        // b = 1: every wavefront keeps its wavefront bits, so it reads back
        // only the LDS slots it wrote, which are those it read in the
        // previous exchange of the same tile: no workgroup barrier (the
        // first exchange of a program keeps them, since the previous
        // tile's last exchange may have had other wavefronts on its slots)
        bool same_waves = true;
        for (int k = 6; k < m - rb; ++k) same_waves = same_waves && L.bit_of[rb + k] == nl.bit_of[rb + k];
        r.b = same_waves && had_remap ? 1 : 0;
        had_remap = true;
        for (int e = 0; e < E(); ++e) {
            r.w[e] = swz(dep_reg(nl, e));
            r.w[16 + e] = swz(dep_reg(L, e));
        }
        for (int k = 0; k < m - rb; ++k) {
            r.w[32 + k] = uint32_t(L.bit_of[rb + k]);
            r.w[48 + k] = uint32_t(nl.bit_of[rb + k]);
        }
        out.push_back(r);
        L = nl;
    }

    // make every bit of `req` a register slot (op index i for the lookahead)
    void ensure(uint32_t req, int i) {
        uint32_t missing = 0;
        for (int b = 0; b < m; ++b)
            if (((req >> b) & 1) && L.slot_of[b] >= rb) missing |= 1u << b;
        if (!missing) return;
        // the new register set: req plus the soonest-needed other bits
        std::vector<int> cand;
        for (int b = 0; b < m; ++b)
            if (!((req >> b) & 1)) cand.push_back(b);
        std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
            const int na = next_use(a, i), nb = next_use(b, i);
            if (na != nb) return na < nb;
            return L.slot_of[a] < rb && L.slot_of[b] >= rb;   // ties: keep residents
        });
        uint32_t keep = req;
        for (size_t k = 0; __builtin_popcount(keep) < rb && k < cand.size(); ++k) {
            const int b = cand[k];
            if (next_use(b, i) == INT32_MAX && L.slot_of[b] >= rb) continue;   // no gain
            keep |= 1u << b;
        }
        // bits already in registers stay in their slots; the others swap with
        // register bits that leave, the sooner needed into the lower slot
        RtLayout nl = L;
        std::vector<int> leaving, arriving;
        for (int sl = 0; sl < rb; ++sl)
            if (!((keep >> L.bit_of[sl]) & 1)) leaving.push_back(sl);
        for (int b = 0; b < m; ++b)
            if (((keep >> b) & 1) && L.slot_of[b] >= rb) arriving.push_back(b);
        std::stable_sort(arriving.begin(), arriving.end(),
                         [&](int a, int b) { return next_use(a, i) < next_use(b, i); });
        // fewer arrivals than free slots: keep the rest of the leavers
        for (size_t k = 0; k < arriving.size(); ++k) {
            const int rs = leaving[k], ts = L.slot_of[arriving[k]];
            nl.bit_of[rs] = arriving[k];
            nl.bit_of[ts] = L.bit_of[rs];
        }
        for (int sl = 0; sl < m; ++sl) nl.slot_of[nl.bit_of[sl]] = sl;
        emit_remap(nl);
    }

    // conditions on compressed tile bits -> thread (tm/tv) and element (rm/rv) parts
    void split(uint32_t cm, uint32_t cv, uint32_t &tm, uint32_t &tv, uint32_t &rm, uint32_t &rv) const {
        tm = tv = rm = rv = 0;
        for (int b = 0; b < m; ++b) {
            if (!((cm >> b) & 1)) continue;
            const int sl = L.slot_of[b];
            const uint32_t v = (cv >> b) & 1;
            if (sl < rb) {
                rm |= 1u << sl;
                rv |= v << sl;
            } else {
                tm |= 1u << (sl - rb);
                tv |= v << (sl - rb);
            }
        }
    }

    static bool is_hadamard(const double *u) {
        const double s = 0.70710678118654752440;
        auto near = [](double a, double b) { return std::fabs(a - b) < 1e-15; };
        return near(u[0], s) && near(u[2], s) && near(u[4], s) && near(u[6], -s) && u[1] == 0 &&
               u[3] == 0 && u[5] == 0 && u[7] == 0;
    }

    void u1(int b, const double *u, uint32_t cm, uint32_t cv, uint64_t hm, uint64_t hv) {
        qcx::RtOp r{};
        r.a = L.slot_of[b];
        r.hm = hm;
        r.hv = hv;
        split(cm, cv, r.tm, r.tv, r.rm, r.rv);
        const bool uncond = cm == 0 && hm == 0;
        if (uncond && !adjoint && is_hadamard(u)) {   // gradients need the true scale
            r.kind = qcx::rt_code(qcx::RT_H, r.a);
            scale *= 0.70710678118654752440;
            out.push_back(r);
            return;
        }
        const bool real = u[1] == 0 && u[3] == 0 && u[5] == 0 && u[7] == 0;
        const bool cond = (r.tm | r.rm) != 0 || r.hm != 0;
        r.kind = qcx::rt_code(real ? (cond ? qcx::RT_U1RC : qcx::RT_U1R) : (cond ? qcx::RT_U1C : qcx::RT_U1),
                              r.a);
        for (int i = 0; i < 8; ++i) put(r.u, i, u[i]);
        out.push_back(r);
    }

    // diagonal terms (the TILE_PHASES term arrays, or one TILE_PHASE term):
    // the terms whose thread and tile conditions hold come from a lane table,
    // a wave table and window tables of bit masks
    void diag_terms(int nt, const uint32_t *pm, const uint32_t *pv, const uint64_t *hm,
                    const uint64_t *hv, const double *ph) {
        bool all_neg = true;
        for (int k = 0; k < nt; ++k)
            if (!(ph[2 * k] == -1.0 && ph[2 * k + 1] == 0.0)) all_neg = false;
        qcx::RtOp r{};
        r.kind = qcx::rt_code(all_neg ? qcx::RT_SIGN : qcx::RT_TERMS, 0);
        r.nt = nt;
        uint32_t lane[64], wave[8];
        for (auto &x : lane) x = 0;
        for (auto &x : wave) x = 0;
        uint64_t hi_all = 0;
        for (int k = 0; k < nt; ++k) hi_all |= hm[k];
        const std::vector<int> win = windows_of(hi_all);
        if (win.size() > size_t(qcx::kRtWindows)) too_wide = true;
        std::vector<std::vector<uint32_t>> wt(win.size(), std::vector<uint32_t>(8, 0));
        for (int k = 0; k < nt; ++k) {
            uint32_t tm, tv, rm, rv;
            split(pm[k], pv[k], tm, tv, rm, rv);
            for (uint32_t l = 0; l < 64; ++l)
                if ((l & tm & 63u) == (tv & 63u)) lane[l] |= 1u << k;
            for (uint32_t w8 = 0; w8 < 8; ++w8)
                if ((w8 & (tm >> 6)) == (tv >> 6)) wave[w8] |= 1u << k;
            for (size_t j = 0; j < win.size(); ++j) {
                const uint64_t wm = uint64_t(7) << win[j];
                for (uint64_t x = 0; x < 8; ++x)
                    if (((x << win[j]) & hm[k] & wm) == (hv[k] & wm)) wt[j][x] |= 1u << k;
            }
            for (int e = 0; e < E(); ++e)
                if ((uint32_t(e) & rm) == rv) r.w[32 + e] |= 1u << k;
            if (!all_neg) put_c(r.u, k, cd(ph[2 * k], ph[2 * k + 1]));
        }
        r.w[0] = add_tab(lblob, lane, sizeof(lane));
        for (int w8 = 0; w8 < 8; ++w8) r.w[8 + w8] = wave[w8];
        r.b = int(std::min(win.size(), size_t(qcx::kRtWindows)));
        for (int j = 0; j < qcx::kRtWindows; ++j)   // unused windows: all terms pass
            for (int x = 0; x < 8; ++x) r.wt[8 * j + x] = j < r.b ? wt[j][x] : ~0u;
        for (int j = 0; j < r.b; ++j) r.hw[j] = uint64_t(win[j]);
        out.push_back(r);
    }

    void fan(const qcx::TileOp &op) {
        const int t = op.b0;
        const uint32_t ctl = uint32_t(op.b1);
        qcx::RtOp r{};
        r.a = L.slot_of[t];
        if (r.a < rb) {
            r.kind = qcx::rt_code(qcx::RT_FAN, r.a);
        } else {
            r.kind = qcx::rt_code(qcx::RT_FAN, qcx::kRtThreadSlot);
            r.a -= rb;   // the target's thread bit
        }
        const cd tphase(op.u[2 * t], op.u[2 * t + 1]);
        for (int e = 0; e < E(); ++e) {
            cd g = tphase;
            for (int c = 0; c < m; ++c)
                if (((ctl >> c) & 1) && L.slot_of[c] < rb && ((e >> L.slot_of[c]) & 1))
                    g *= cd(op.u[2 * c], op.u[2 * c + 1]);
            put_c(r.u, e, g);
        }
        // thread-bit controls: lane and wave tables of their phase products
        std::vector<cd> lane(64, cd(1.0)), wave(8, cd(1.0));
        for (int c = 0; c < m; ++c) {
            if (!((ctl >> c) & 1) || L.slot_of[c] < rb) continue;
            const int tbit = L.slot_of[c] - rb;
            const cd p(op.u[2 * c], op.u[2 * c + 1]);
            if (tbit < 6) {
                for (int l = 0; l < 64; ++l)
                    if ((l >> tbit) & 1) lane[l] *= p;
            } else {
                for (int w8 = 0; w8 < 8; ++w8)
                    if ((w8 >> (tbit - 6)) & 1) wave[w8] *= p;
            }
        }
        // out-of-tile controls: window tables in the op
        uint64_t hi_all = 0;
        for (int h = 0; h < op.pad; ++h) hi_all |= op.fan_mask[h];
        const std::vector<int> win = windows_of(hi_all);
        if (win.size() > size_t(qcx::kRtWindows)) too_wide = true;
        r.w[0] = add_ctab(lblob, lane);
        for (int w8 = 0; w8 < 8; ++w8) put_c(r.ph, w8, wave[w8]);
        r.b = int(std::min(win.size(), size_t(qcx::kRtWindows)));
        for (int j = r.b; j < qcx::kRtWindows; ++j)   // unused windows: factor 1
            for (int x = 0; x < 8; ++x) put_c(r.ph, 8 + 8 * j + x, cd(1.0));
        for (int j = 0; j < r.b; ++j) {
            for (int x = 0; x < 8; ++x) {
                cd t(1.0);
                for (int h = 0; h < op.pad; ++h) {
                    const int p = __builtin_ctzll(op.fan_mask[h]);
                    if (p >= win[j] && p < win[j] + 3 && ((x >> (p - win[j])) & 1))
                        t *= cd(op.fan_ph[2 * h], op.fan_ph[2 * h + 1]);
                }
                put_c(r.ph, 8 + 8 * j + x, t);
            }
            r.hw[j] = uint64_t(win[j]);
        }
        out.push_back(r);
    }

    // a block of commuting diagonal rotations (backward pass): the element
    // factors of the register-slot entries and the common factor in u, the
    // thread-bit entries in lane / wave tables, the out-of-tile entries in
    // window tables (as for a fan); gradient entries in the slot order the
    // host assigned (in-tile by ascending compressed bit, then out-of-tile)
    void dgrad(const qcx::TileOp &op) {
        qcx::RtOp r{};
        r.kind = qcx::rt_code(qcx::RT_DGRAD, 0);
        const uint32_t in_mask = uint32_t(op.b1);
        for (int e = 0; e < E(); ++e) {
            cd g(op.u1[0], op.u1[1]);
            for (int c = 0; c < m; ++c)
                if (((in_mask >> c) & 1) && L.slot_of[c] < rb && ((e >> L.slot_of[c]) & 1))
                    g *= cd(op.u[2 * c], op.u[2 * c + 1]);
            put_c(r.u, e, g);
        }
        std::vector<cd> lane(64, cd(1.0)), wave(8, cd(1.0));
        int nt = 0;
        auto entry = [&](uint32_t loc) {
            r.w[1 + nt] = loc | (uint32_t(op.b0 + nt) << 8);
            ++nt;
        };
        for (int c = 0; c < m; ++c) {
            if (!((in_mask >> c) & 1)) continue;
            const int sl = L.slot_of[c];
            if (sl < rb) {
                entry(uint32_t(sl));
                continue;
            }
            const int tbit = sl - rb;
            entry(uint32_t(8 + tbit));
            const cd p(op.u[2 * c], op.u[2 * c + 1]);
            if (tbit < 6) {
                for (int l = 0; l < 64; ++l)
                    if ((l >> tbit) & 1) lane[l] *= p;
            } else {
                for (int w8 = 0; w8 < 8; ++w8)
                    if ((w8 >> (tbit - 6)) & 1) wave[w8] *= p;
            }
        }
        uint64_t hi_all = 0;
        for (int h = 0; h < op.pad; ++h) {
            hi_all |= op.fan_mask[h];
            entry(uint32_t(32 + __builtin_ctzll(op.fan_mask[h])));
        }
        r.nt = nt;
        const std::vector<int> win = windows_of(hi_all);
        if (win.size() > size_t(qcx::kRtWindows)) too_wide = true;
        r.w[0] = add_ctab(lblob, lane);
        for (int w8 = 0; w8 < 8; ++w8) put_c(r.ph, w8, wave[w8]);
        r.b = int(std::min(win.size(), size_t(qcx::kRtWindows)));
        for (int j = r.b; j < qcx::kRtWindows; ++j)   // unused windows: factor 1
            for (int x = 0; x < 8; ++x) put_c(r.ph, 8 + 8 * j + x, cd(1.0));
        for (int j = 0; j < r.b; ++j) {
            for (int x = 0; x < 8; ++x) {
                cd t(1.0);
                for (int h = 0; h < op.pad; ++h) {
                    const int p = __builtin_ctzll(op.fan_mask[h]);
                    if (p >= win[j] && p < win[j] + 3 && ((x >> (p - win[j])) & 1))
                        t *= cd(op.fan_ph[2 * h], op.fan_ph[2 * h + 1]);
                }
                put_c(r.ph, 8 + 8 * j + x, t);
            }
            r.hw[j] = uint64_t(win[j]);
        }
        out.push_back(r);
    }

    // a Hadamard followed by the fan on the same register slot: one op; two
    // such ops in a row on different slots: one RT_HFAN2 op and the second
    // one's data (the interpreter copies every element register once per
    // op, so fewer ops means fewer copies)
    // the element factors of a fan on slot S depend only on the register
    // bits above S: u at e equals u at e with the bits below S cleared
    bool upper_only(const qcx::RtOp &op, int S) const {
        for (int e = 0; e < E(); ++e) {
            if (!((e >> S) & 1)) continue;
            const int e0 = e & ~((1 << S) - 1);
            for (int c = 0; c < 2; ++c) {
                const bool same = is64() ? qcx::rt_vals<float>(op.u)[2 * e + c] == qcx::rt_vals<float>(op.u)[2 * e0 + c]
                                         : op.u[2 * e + c] == op.u[2 * e0 + c];
                if (!same) return false;
            }
        }
        return true;
    }

    // backward programs: real-rotation gradient steps on slots 0, 1, 2 (or
    // 0, 1, or 1, 0) in a row become one op, the later steps kept as its
    // data (with the exchange behind them, if any); so does a sign op with
    // the diagonal-rotation block behind it
    void fuse_grads() {
        std::vector<qcx::RtOp> f;
        f.swap(out);
        auto is_gr = [&](size_t i, int slot) {
            return i < f.size() && f[i].kind == qcx::rt_code(qcx::RT_GRADR, slot);
        };
        for (size_t i = 0; i < f.size(); ++i) {
            if (rb >= 3 && is_gr(i, 0) && is_gr(i + 1, 1) && is_gr(i + 2, 2)) {
                // an exchange right behind joins the op
                const bool x = i + 3 < f.size() && f[i + 3].kind == qcx::rt_code(qcx::RT_REMAP, 0);
                qcx::RtOp r = f[i];
                r.kind = qcx::rt_code(x ? qcx::RT_GRADR3X : qcx::RT_GRADR3, 0);
                out.push_back(r);
                out.push_back(f[i + 1]);
                out.push_back(f[i + 2]);
                if (x) out.push_back(f[i + 3]);
                i += x ? 3 : 2;
            } else if (rb >= 2 && is_gr(i, 0) && is_gr(i + 1, 1)) {
                const bool x = i + 2 < f.size() && f[i + 2].kind == qcx::rt_code(qcx::RT_REMAP, 0);
                qcx::RtOp r = f[i];
                r.kind = qcx::rt_code(x ? qcx::RT_GRADR2X : qcx::RT_GRADR2, 0);
                out.push_back(r);
                out.push_back(f[i + 1]);
                if (x) out.push_back(f[i + 2]);
                i += x ? 2 : 1;
            } else if (is_gr(i, 1) && is_gr(i + 1, 0)) {
                qcx::RtOp r = f[i];
                r.kind = qcx::rt_code(qcx::RT_GRADR2R, 0);
                out.push_back(r);
                out.push_back(f[i + 1]);
                i += 1;
            } else if (f[i].kind == qcx::rt_code(qcx::RT_SIGN, 0) && i + 1 < f.size() &&
                       f[i + 1].kind == qcx::rt_code(qcx::RT_DGRAD, 0)) {
                qcx::RtOp r = f[i];
                r.kind = qcx::rt_code(qcx::RT_SIGNDG, 0);
                out.push_back(r);
                out.push_back(f[i + 1]);
                i += 1;
            } else {
                out.push_back(f[i]);
            }
        }
    }

    // forward programs: unconditioned one-qubit steps on slots 0..3 (or
    // 0..2) in a row become one op, the later steps kept as its data
    void fuse_u1() {
        std::vector<qcx::RtOp> f;
        f.swap(out);
        auto is_u1 = [&](size_t i, int slot) {
            return i < f.size() && f[i].kind == qcx::rt_code(qcx::RT_U1, slot);
        };
        for (size_t i = 0; i < f.size(); ++i) {
            const int len = rb >= 4 && is_u1(i, 0) && is_u1(i + 1, 1) && is_u1(i + 2, 2) && is_u1(i + 3, 3) ? 4
                            : rb >= 3 && is_u1(i, 0) && is_u1(i + 1, 1) && is_u1(i + 2, 2)             ? 3
                                                                                                    : 1;
            // an exchange right behind the steps joins the op
            const bool x = (len == 4 || (len == 3 && rb == 3)) && i + len < f.size() &&
                           f[i + len].kind == qcx::rt_code(qcx::RT_REMAP, 0);
            qcx::RtOp r = f[i];
            if (len > 1)
                r.kind = qcx::rt_code(len == 4 ? (x ? qcx::RT_U1X4X : qcx::RT_U1X4)
                                               : (x ? qcx::RT_U1X3X : qcx::RT_U1X3), 0);
            out.push_back(r);
            for (int j = 1; j < len + (x ? 1 : 0); ++j) out.push_back(f[i + j]);
            i += len - 1 + (x ? 1 : 0);
        }
    }

    void fuse_h_fan() {
        std::vector<qcx::RtOp> f;
        f.reserve(out.size());
        for (size_t i = 0; i < out.size(); ++i) {
            const int k = out[i].kind;
            if (!adjoint && i + 1 < out.size() && k / 8 == qcx::RT_H &&
                out[i + 1].kind == qcx::rt_code(qcx::RT_FAN, k % 8)) {
                qcx::RtOp r = out[i + 1];
                r.kind = qcx::rt_code(qcx::RT_HFAN, k % 8);
                f.push_back(r);
                ++i;
            } else {
                f.push_back(out[i]);
            }
        }
        out.clear();
        for (size_t i = 0; i < f.size(); ++i) {
            const int k = f[i].kind;
            if (rb >= 4 && i + 3 < f.size() && k == qcx::rt_code(qcx::RT_HFAN, 0) &&
                f[i + 1].kind == qcx::rt_code(qcx::RT_HFAN, 1) &&
                f[i + 2].kind == qcx::rt_code(qcx::RT_HFAN, 2) &&
                f[i + 3].kind == qcx::rt_code(qcx::RT_HFAN, 3)) {
                qcx::RtOp r = f[i];
                bool upper = rb == 4;
                for (int k = 0; k < 4; ++k) upper = upper && upper_only(f[i + k], k);
                r.kind = qcx::rt_code(upper ? qcx::RT_HFAN4U : qcx::RT_HFAN4, 0);
                out.push_back(r);
                for (int j = 1; j < 4; ++j) out.push_back(f[i + j]);   // data of the later steps
                i += 3;
                continue;
            }
            if (i + 1 < f.size() && k / 8 == qcx::RT_HFAN && f[i + 1].kind / 8 == qcx::RT_HFAN &&
                f[i + 1].kind % 8 != k % 8 && k % 8 < rb && f[i + 1].kind % 8 < rb) {
                qcx::RtOp r = f[i];
                r.kind = qcx::rt_hfan2_code(k % 8, f[i + 1].kind % 8);
                out.push_back(r);
                out.push_back(f[i + 1]);   // data of the second step
                ++i;
            } else {
                out.push_back(f[i]);
            }
        }
    }

    void phases_of(const qcx::TileOp &op, int nt) {
        diag_terms(nt, op.pm_lo, op.pv_lo, op.pm_hi, op.pv_hi, op.u);
    }

    void lower(int i) {
        const qcx::TileOp &op = ops[i];
        ensure(need[i], i);
        switch (op.kind) {
        case qcx::TILE_DENSE1: u1(op.b0, op.u, op.cmask_lo, op.cval_lo, op.cmask_hi, op.cval_hi); break;
        case qcx::TILE_DIAG1: {
            qcx::RtOp r{};
            r.a = L.slot_of[op.b0];
            if (r.a < rb) {
                r.kind = qcx::rt_code(qcx::RT_DIAG1, r.a);
            } else {
                r.kind = qcx::rt_code(qcx::RT_DIAG1, qcx::kRtThreadSlot);
                r.a -= rb;
            }
            r.b = (op.u[0] == 1.0 && op.u[1] == 0.0) ? 1 : 0;
            for (int k = 0; k < 4; ++k) put(r.u, k, op.u[k]);
            out.push_back(r);
        } break;
        case qcx::TILE_DENSE2: {
            qcx::RtOp r{};
            r.a = L.slot_of[op.b0];
            r.b = L.slot_of[op.b1];
            r.hm = op.cmask_hi;
            r.hv = op.cval_hi;
            split(op.cmask_lo, op.cval_lo, r.tm, r.tv, r.rm, r.rv);
            r.kind = qcx::rt_code(qcx::RT_U2, (r.tm | r.rm) != 0 || r.hm != 0 ? 1 : 0);
            for (int k = 0; k < 32; ++k) put(r.u, k, op.u[k]);
            out.push_back(r);
        } break;
        case qcx::TILE_PHASE: {
            const uint32_t pm = op.cmask_lo, pv = op.cval_lo;
            const uint64_t hm = op.cmask_hi, hv = op.cval_hi;
            diag_terms(1, &pm, &pv, &hm, &hv, op.u);
        } break;
        case qcx::TILE_PHASES: phases_of(op, op.b0); break;
        case qcx::TILE_FAN: fan(op); break;
        case qcx::TILE_DGRAD: dgrad(op); break;
        case qcx::TILE_GRAD:
        case qcx::TILE_GRAD_APPLY:
        case qcx::TILE_GRAD_APPLY_REAL:
        case qcx::TILE_GRAD_APPLY_DIAG: {
            qcx::RtOp r{};
            const int sl = L.slot_of[op.b0];
            const int kind = op.kind == qcx::TILE_GRAD ? qcx::RT_GRAD0
                             : op.kind == qcx::TILE_GRAD_APPLY ? qcx::RT_GRAD
                             : op.kind == qcx::TILE_GRAD_APPLY_REAL ? qcx::RT_GRADR : qcx::RT_GRADD;
            r.kind = qcx::rt_code(kind, sl);
            r.b = op.b1;
            r.w[0] = uint32_t(op.pad);
            for (int k = 0; k < 8; ++k) put(r.u, k, op.u[k]);
            out.push_back(r);
        } break;
        case qcx::TILE_GRAD_APPLY2_DIAG_REAL: {
            qcx::RtOp r{};
            r.kind = qcx::rt_code(qcx::RT_GRAD2, L.slot_of[op.b0]);
            r.b = op.b1;
            r.w[0] = uint32_t(op.pad) & 0xffffu;
            r.w[1] = uint32_t(op.pad) >> 16;
            for (int k = 0; k < 8; ++k) {
                put(r.u, k, op.u[k]);
                put(r.ph, k, op.u1[k]);
            }
            out.push_back(r);
        } break;
        case qcx::TILE_XPERM:
            for (int k = 0; k < op.b0; ++k) {
                qcx::RtOp r{};
                r.a = L.slot_of[op.x_t[k]];
                r.kind = qcx::rt_code(qcx::RT_CX, r.a);
                r.hm = op.x_hm[k];
                r.hv = op.x_hv[k];
                split(op.x_cm[k], op.x_cv[k], r.tm, r.tv, r.rm, r.rv);
                out.push_back(r);
            }
            break;
        default: break;
        }
    }

    // global positions of the register and thread bits of layout l
    void positions(const RtLayout &l, uint32_t *thr, uint32_t *reg) const {
        uint32_t pos[32];
        for (int p = 0, j = 0; p < n; ++p)
            if ((P >> p) & 1) pos[j++] = uint32_t(p);
        for (int i = 0; i < rb; ++i) reg[i] = pos[l.bit_of[i]];
        for (int k = 0; k < m - rb; ++k) thr[k] = pos[l.bit_of[rb + k]];
    }

    void run(qcx::RtArgs &a) {
        need.resize(n_ops);
        for (int i = 0; i < n_ops; ++i) need[i] = need_of(ops[i]);
        initial_layout();
        const RtLayout first = L;
        for (int i = 0; i < n_ops; ++i) lower(i);
        fuse_h_fan();
        if (adjoint) fuse_grads();
        else fuse_u1();
        if (scale != 1.0 && !defer_scale) {
            qcx::RtOp r{};
            r.kind = qcx::rt_code(qcx::RT_SCALE, 0);
            put(r.u, 0, scale);
            out.push_back(r);
        }
        // the store wants most lanes on the lowest bits (runs of >= 16
        // contiguous amplitudes per wavefront store); otherwise one more
        // exchange puts the load's lanes back
        int low_lanes = 0;
        for (int k = 0; k < std::min(m - rb, 6); ++k)
            if (L.bit_of[rb + k] < 5) ++low_lanes;
        const bool lanes_ok = low_lanes >= std::min({m - rb, 6, 4});
        if (!lanes_ok) {
            RtLayout back = L;
            // lanes as at the load; the register bits stay where they are if
            // they are not lane bits there
            std::vector<int> lane_bits;
            for (int k = 0; k < std::min(m - rb, 6); ++k) lane_bits.push_back(first.bit_of[rb + k]);
            std::vector<bool> taken(m, false);
            for (int k = 0; k < (int)lane_bits.size(); ++k) {
                back.bit_of[rb + k] = lane_bits[k];
                taken[lane_bits[k]] = true;
            }
            int sl = 0;
            for (int i = 0; i < rb; ++i) {
                const int b = L.bit_of[i];
                if (!taken[b]) {
                    back.bit_of[sl++] = b;
                    taken[b] = true;
                }
            }
            for (int b = 0; b < m && sl < rb; ++b)
                if (!taken[b]) {
                    back.bit_of[sl++] = b;
                    taken[b] = true;
                }
            sl = rb + (int)lane_bits.size();
            for (int b = 0; b < m; ++b)
                if (!taken[b]) back.bit_of[sl++] = b;
            for (int s2 = 0; s2 < m; ++s2) back.slot_of[back.bit_of[s2]] = s2;
            emit_remap(back);
        }
        while (lblob.size() % 16) lblob.push_back(0);
        a = qcx::RtArgs{};
        a.st_scale = 1.0;
        a.lds_tab_bytes = uint32_t(lblob.size());
        a.m = m;
        a.tb = m - rb;
        a.n_tiles = uint64_t(1) << (n - m);
        a.n_ops = int(out.size());
        for (int p = 0, j = 0; p < n; ++p)
            if ((P >> p) & 1) a.pos[j++] = uint32_t(p);
        positions(first, a.ld_thr, a.ld_reg);
        positions(L, a.st_thr, a.st_reg);
    }
};

// Split the composite tile ops into ops that each need at most two register
// slots: a TILE_XPERM into one op per controlled-X gate (they commute), a
// TILE_KRON into one TILE_DENSE1 per bit, and the dense-then-diagonal pairs
// into their two halves.
void rt_expand(const std::vector<qcx::TileOp> &in, std::vector<qcx::TileOp> &out) {
    out.clear();
    for (const qcx::TileOp &op : in) {
        switch (op.kind) {
        case qcx::TILE_XPERM:
            for (int k = 0; k < op.b0; ++k) {
                qcx::TileOp x{};
                x.kind = qcx::TILE_XPERM;
                x.b0 = 1;
                x.x_cm[0] = op.x_cm[k];
                x.x_cv[0] = op.x_cv[k];
                x.x_t[0] = op.x_t[k];
                x.x_hm[0] = op.x_hm[k];
                x.x_hv[0] = op.x_hv[k];
                out.push_back(x);
            }
            break;
        case qcx::TILE_KRON:
            for (int j = 0; j < op.b0; ++j) {
                qcx::TileOp d{};
                d.kind = qcx::TILE_DENSE1;
                d.b0 = (op.b1 >> (5 * j)) & 31;
                for (int i = 0; i < 8; ++i) d.u[i] = op.u[8 * j + i];
                out.push_back(d);
            }
            break;
        case qcx::TILE_DENSE1_PHASES:
        case qcx::TILE_DENSE1_FAN: {
            qcx::TileOp d{};
            d.kind = qcx::TILE_DENSE1;
            d.b0 = op.b0;
            for (int i = 0; i < 8; ++i) d.u[i] = op.u1[i];
            out.push_back(d);
            qcx::TileOp p = op;
            if (op.kind == qcx::TILE_DENSE1_PHASES) {
                p.kind = qcx::TILE_PHASES;
                p.b0 = op.pad;
            } else {
                p.kind = qcx::TILE_FAN;
            }
            out.push_back(p);
        } break;
        default: out.push_back(op);
        }
    }
}

// RT program of one tile run (m tile bits P, TileOp list ops), as one
// host buffer: the RtOps, then the table blob (lane tables first).
// adjoint: a backward program for the two-vector kernel.
// scale_out: if given, the program leaves the product of its Hadamards'
// 1/sqrt2 factors out and returns it there (the caller applies it at a
// later store)
void rt_program(int n, int m, int dtype, uint64_t P, const std::vector<qcx::TileOp> &ops,
                qcx::RtArgs &a, std::vector<unsigned char> &buf, size_t &tab_off,
                bool adjoint = false, double *scale_out = nullptr) {
    std::vector<qcx::TileOp> flat;
    rt_expand(ops, flat);
    const int rb = adjoint ? qcx::rt_adj_reg_bits(dtype) : qcx::rt_reg_bits(dtype, m);
    RtLowering lw{n, m, rb, dtype, P, flat.data(), int(flat.size())};
    lw.adjoint = adjoint;
    lw.defer_scale = scale_out != nullptr && !adjoint;
    lw.run(a);
    if (scale_out) *scale_out = lw.defer_scale ? lw.scale : 1.0;
    if (lw.too_wide) a.lds_tab_bytes = ~0u;   // not expressible: the caller takes the LDS engine
    const size_t ob = lw.out.size() * sizeof(qcx::RtOp);
    tab_off = ob;
    buf.resize(ob + lw.lblob.size() + lw.gblob.size());
    std::memcpy(buf.data(), lw.out.data(), ob);
    if (!lw.lblob.empty()) std::memcpy(buf.data() + ob, lw.lblob.data(), lw.lblob.size());
    if (!lw.gblob.empty())
        std::memcpy(buf.data() + ob + lw.lblob.size(), lw.gblob.data(), lw.gblob.size());
}

// Plans of recently applied tiled circuits.  A circuit applied again with
// the same gates (matrices included), register size, precision and tile
// settings reuses its runs' programs; the device work is the same.
struct TiledPlanRun {
    uint64_t P = 0;
    int gate = -1;                      // the standalone gate (P == 0)
    bool rt = false;
    qcx::RtArgs ra{};
    size_t tab_off = 0;
    int n_ops = 0;                      // LDS-engine runs: TileOp count
    std::vector<unsigned char> bytes;   // register-tile program and tables, or the TileOps
};
struct TiledPlan {
    std::vector<unsigned char> key;
    std::vector<TiledPlanRun> runs;
    std::vector<unsigned char> blob;   // every run's bytes, 256-byte aligned
    std::vector<size_t> off;           // run i's bytes at blob + off[i]
};
constexpr size_t kPlanCacheEntries = 4;
constexpr size_t kPlanKeyMaxBytes = size_t(1) << 20;
std::mutex g_plan_mu;
std::vector<std::shared_ptr<const TiledPlan>> g_plans;   // most recent first

// the key of a tiled circuit; false if it is too large to keep
bool plan_key(const qc_state_t &s, int m, int ng, const qc_gate_t *gs, std::vector<unsigned char> &k) {
    size_t bytes = 5 * sizeof(int);
    for (int i = 0; i < ng; ++i)
        bytes += sizeof(int32_t) * (2 + gs[i].n_targets + 2 * gs[i].n_ctrls) +
                 sizeof(double) * 2 * (size_t(1) << (2 * gs[i].n_targets));
    if (bytes > kPlanKeyMaxBytes) return false;
    k.clear();
    k.reserve(bytes);
    auto put = [&](const void *p, size_t b) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        k.insert(k.end(), c, c + b);
    };
    const int hdr[5] = {s.n, s.dtype, m, g_knob_tile_engine.load(), ng};
    put(hdr, sizeof(hdr));
    for (int i = 0; i < ng; ++i) {
        const qc_gate_t &g = gs[i];
        put(&g.n_targets, sizeof(int32_t));
        put(&g.n_ctrls, sizeof(int32_t));
        put(g.targets, sizeof(int32_t) * g.n_targets);
        put(g.ctrls, sizeof(int32_t) * g.n_ctrls);
        put(g.ctrl_vals, sizeof(int32_t) * g.n_ctrls);
        put(g.matrix, sizeof(double) * 2 * (size_t(1) << (2 * g.n_targets)));
    }
    return true;
}

// one run: its bytes staged now, or already on the device at `dev`
int launch_plan_run(qc_state_t s, int m, const qc_gate_t *gs, const TiledPlanRun &pr, DevCtx *c,
                    qc_exec_stats_t &st, void *stream, void *dev = nullptr) {
    if (pr.P == 0) return apply_gate_unfused(s, gs[pr.gate], st, stream);
    const hipStream_t hs = (hipStream_t)stream;
    if (!dev) {
        const int rc = stage(c, pr.bytes.data(), pr.bytes.size(), hs, &dev);
        if (rc) return rc;
    }
    hipError_t e;
    if (pr.rt) {
        e = qcx::launch_rt_run(s.amp, s.dtype, pr.ra, static_cast<const qcx::RtOp *>(dev),
                               static_cast<const unsigned char *>(dev) + pr.tab_off, hs);
    } else {
        const qcx::TileArgs a = tile_args(s.n, m, pr.P, pr.n_ops);
        e = qcx::launch_tile_run(s.amp, s.dtype, s.n, a, static_cast<const qcx::TileOp *>(dev), hs);
    }
    if (e != hipSuccess) return hip_fail(e, "tile_run");
    st.launches += 1;
    st.sweeps += 1;
    st.state_bytes += sweep_bytes(s.n, s.dtype);
    return QC_OK;
}

int tiled_execute(qc_state_t s, int ng, const qc_gate_t *gs, qc_exec_stats_t &st,
                  void *stream) {
    DevCtx *c;
    int rc = get_ctx(&c);
    if (rc) return rc;
    const int n = s.n;
    const int m = tile_bits_for(s);
    auto plan = std::make_shared<TiledPlan>();
    const bool keep = plan_key(s, m, ng, gs, plan->key);
    if (keep) {
        std::shared_ptr<const TiledPlan> hit;
        {
            std::lock_guard<std::mutex> lk(g_plan_mu);
            for (size_t i = 0; i < g_plans.size(); ++i)
                if (g_plans[i]->key == plan->key) {
                    hit = g_plans[i];
                    g_plans.erase(g_plans.begin() + long(i));
                    g_plans.insert(g_plans.begin(), hit);
                    break;
                }
        }
        if (hit) {
            // the first program in a copy of its own and its launch, then
            // every later program in one copy (made while the first run is
            // on the GPU) and their launches back to back
            bool first = true;
            char *rest = nullptr;   // the later programs on the device, from blob offset rest_off
            size_t rest_off = 0;
            for (size_t i = 0; i < hit->runs.size(); ++i) {
                const TiledPlanRun &pr = hit->runs[i];
                void *dev = nullptr;
                if (pr.P != 0 && first) {
                    first = false;   // staged by launch_plan_run
                } else if (pr.P != 0) {
                    if (!rest) {
                        rest_off = hit->off[i];
                        void *d = nullptr;
                        if ((rc = stage(c, hit->blob.data() + rest_off, hit->blob.size() - rest_off,
                                        (hipStream_t)stream, &d)))
                            return rc;
                        rest = static_cast<char *>(d);
                    }
                    dev = rest + (hit->off[i] - rest_off);
                }
                if ((rc = launch_plan_run(s, m, gs, pr, c, st, stream, dev))) return rc;
            }
            return QC_OK;
        }
    }
    std::vector<TileRun> runs;
    form_runs(n, m, ng, gs, nullptr, runs);
    std::vector<qcx::TileOp> ops;
    // register tiles pay off when there are tiles enough for every CU;
    // a few tiles (small registers) are latency-bound per op, where the
    // LDS-resident engine's cheaper ops win
    const bool rt_ok = g_knob_tile_engine.load() == 1 && m >= qcx::rt_reg_bits(s.dtype, m) &&
                       n - m >= kRtMinTileBits;
    // Register-tile programs leave their Hadamards' 1/sqrt2 factors out; the
    // product is applied at the store of the last register-tile run before
    // a standalone gate or the end, or by a scaling op in front of an
    // LDS-engine run (each run is planned while the previous one runs)
    double pending = 1.0;
    plan->runs.resize(runs.size());
    for (size_t i = 0; i < runs.size(); ++i) {
        const TileRun &r = runs[i];
        TiledPlanRun &pr = plan->runs[i];
        pr.P = r.P;
        if (r.P == 0) {
            pr.gate = r.gates[0];
            if ((rc = launch_plan_run(s, m, gs, pr, c, st, stream))) return rc;
            continue;
        }
        ops.clear();
        tile_ops_for(n, gs, r.gates, r.P, ops);
        double scale = 1.0;
        if (rt_ok) rt_program(n, m, s.dtype, r.P, ops, pr.ra, pr.bytes, pr.tab_off, false, &scale);
        pr.rt = rt_ok && pr.ra.lds_tab_bytes <= kRtLdsTabMax;
        if (pr.rt) {
            pending *= scale;
            if (i + 1 == runs.size() || runs[i + 1].P == 0) {
                pr.ra.st_scale = pending;
                pending = 1.0;
            }
        } else {   // LDS-resident tiles (also for programs whose lane tables exceed the LDS budget)
            if (pending != 1.0) {
                qcx::TileOp sc{};
                sc.kind = qcx::TILE_DIAG1;
                sc.u[0] = sc.u[2] = pending;
                ops.insert(ops.begin(), sc);
                pending = 1.0;
            }
            pr.n_ops = int(ops.size());
            const unsigned char *b = reinterpret_cast<const unsigned char *>(ops.data());
            pr.bytes.assign(b, b + ops.size() * sizeof(qcx::TileOp));
        }
        if ((rc = launch_plan_run(s, m, gs, pr, c, st, stream))) return rc;
    }
    if (keep) {
        plan->off.resize(plan->runs.size(), 0);
        for (size_t i = 0; i < plan->runs.size(); ++i) {
            const std::vector<unsigned char> &b = plan->runs[i].bytes;
            if (b.empty()) continue;
            plan->blob.resize((plan->blob.size() + 255) & ~size_t(255));
            plan->off[i] = plan->blob.size();
            plan->blob.insert(plan->blob.end(), b.begin(), b.end());
        }
        if (plan->blob.size() > kRingBytes / 4) return QC_OK;   // too large to stage at once: not kept
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans.insert(g_plans.begin(), std::move(plan));
        if (g_plans.size() > kPlanCacheEntries) g_plans.pop_back();
    }
    return QC_OK;
}

}  // namespace

namespace {

// Block and selector qubits of a fused block.  Every qubit on which a
// member acts non-diagonally is a block qubit; qubits where all members act
// diagonally fill the block up to fuse_k qubits, lowest bit positions first,
// and the rest become selector qubits (high bit positions, so the low,
// contiguous address bits stay inside the tiles of the matrix-core kernel).
// With `widen`, blocks narrower than fuse_k are padded with untouched
// qubits.  Returns false when the members do not fit QC_MAX_FUSED block
// qubits and kMaxSel selector qubits.
bool assign_block(int n, const std::vector<const qc_gate_t *> &members, int fuse_k, bool widen,
                  int *bq, int &k, int *sq, int &ns) {
    uint64_t all = 0, nd = 0;
    for (auto *g : members) {
        all |= gate_mask(*g);
        nd |= gate_nd_mask(*g);
    }
    const int width = std::max(fuse_k, __builtin_popcountll(nd));
    if (width > QC_MAX_FUSED) return false;
    uint64_t q = nd;
    for (int lab = n - 1; lab >= 0 && __builtin_popcountll(q) < width; --lab)
        if (((all & ~q) >> lab) & 1) q |= uint64_t(1) << lab;
    const uint64_t sel = all & ~q;
    if (__builtin_popcountll(sel) > qcx::kMaxSel) return false;
    for (int lab = n - 1; widen && lab >= 0 && __builtin_popcountll(q) < fuse_k; --lab)
        if (!(((q | sel) >> lab) & 1)) q |= uint64_t(1) << lab;
    k = 0;
    ns = 0;
    for (int lab = 0; lab < n; ++lab) {
        if ((q >> lab) & 1) bq[k++] = lab;
        if ((sel >> lab) & 1) sq[ns++] = lab;
    }
    return true;
}

// QC_EXEC_FUSED: plan the blocks (one-step lookahead over `look`
// candidates) and launch each block as soon as the planner has chosen it,
// so the planning of the next block overlaps the device work.  complex64
// blocks are widened to 5 qubits so that every block runs on the
// matrix-core kernel (the extra qubits carry identity).
int fused_execute(qc_state_t s, int n_gates, const qc_gate_t *gates, int fuse_k, int look,
                  qc_exec_stats_t &st, void *stream) {
    const hipStream_t hs = (hipStream_t)stream;
    const double sweep = sweep_bytes(s.n, s.dtype);
    const bool widen = s.dtype == QC_C64 && fuse_k == 5;
    int rc = QC_OK;
    std::vector<const qc_gate_t *> members;
    fuse_plan_each(s.n, n_gates, gates, fuse_k, qcx::kMaxSel, look,
                   [&](const std::vector<int> &idx) {
        members.clear();
        for (int i : idx) members.push_back(&gates[i]);
        int bq[QC_MAX_FUSED], sq[qcx::kMaxSel], k = 0, ns = 0;
        if (!assign_block(s.n, members, fuse_k, widen, bq, k, sq, ns)) {
            // not expressible as one block (a gate with many controls)
            for (auto *g : members)
                if ((rc = apply_gate_unfused(s, *g, st, stream))) return false;
            return true;
        }
        rc = fused_apply(s, k, bq, ns, sq, block_matrices(k, bq, ns, sq, members), hs);
        if (rc) return false;
        st.launches += 1;
        st.sweeps += 1;
        st.fused_blocks += 1;
        st.state_bytes += sweep;
        return true;
    });
    return rc;
}

}  // namespace

extern "C" {

int qc_apply_fused_k(qc_state_t s, int k, const int *qubits, const double *u, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!u) return fail(QC_ERR_ARG, "matrix is NULL");
    if (k < 1 || k > QC_MAX_FUSED) return fail(QC_ERR_ARG, "k out of range");
    if (k > s.n) return fail(QC_ERR_QUBIT, "more gate qubits than register qubits");
    if ((rc = check_qubits(s.n, qubits, k, "target"))) return rc;
    return fused_apply(s, k, qubits, 0, nullptr, to_cd(u, 1 << k), (hipStream_t)stream);
}

int qc_apply_multiplexed(qc_state_t s, int k, const int *qubits, int n_sel, const int *sel_qubits,
                         const double *u, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!u) return fail(QC_ERR_ARG, "matrix is NULL");
    if (k < 1 || k > QC_MAX_FUSED) return fail(QC_ERR_ARG, "k out of range");
    if (n_sel < 0 || n_sel > QC_MAX_SEL) return fail(QC_ERR_ARG, "n_sel out of range");
    if (k + n_sel > s.n) return fail(QC_ERR_QUBIT, "more gate qubits than register qubits");
    if (n_sel > 0 && !sel_qubits) return fail(QC_ERR_ARG, "selector pointer is NULL");
    if (!qubits) return fail(QC_ERR_ARG, "target pointer is NULL");
    int all[QC_MAX_FUSED + QC_MAX_SEL];
    for (int j = 0; j < k; ++j) all[j] = qubits[j];
    for (int j = 0; j < n_sel; ++j) all[k + j] = sel_qubits[j];
    if ((rc = check_qubits(s.n, all, k + n_sel, "gate qubit"))) return rc;
    const int d = 1 << k;
    std::vector<cd> m(size_t(d) * d << n_sel);
    for (size_t i = 0; i < m.size(); ++i) m[i] = cd(u[2 * i], u[2 * i + 1]);
    return fused_apply(s, k, qubits, n_sel, sel_qubits, m, (hipStream_t)stream);
}

int qc_fuse_plan(int n, int n_gates, const qc_gate_t *gates, int fuse_k, int *block_of,
                 int *n_blocks) {
    if (n < 1 || n > QC_MAX_QUBITS) return fail(QC_ERR_ARG, "qubit count out of range");
    if (n_gates < 0 || (n_gates > 0 && (!gates || !block_of)) || !n_blocks)
        return fail(QC_ERR_ARG, "NULL argument");
    if (fuse_k < 1 || fuse_k > QC_MAX_FUSED) return fail(QC_ERR_ARG, "fuse_k out of range");
    for (int i = 0; i < n_gates; ++i) {
        int rc = check_gate(n, gates[i]);
        if (rc) return rc;
    }
    std::vector<int> bo;
    int nb = 0;
    fuse_plan(n, n_gates, gates, fuse_k, qcx::kMaxSel, g_knob_look.load(), bo, nb);
    std::copy(bo.begin(), bo.end(), block_of);
    *n_blocks = nb;
    return QC_OK;
}

int qc_block_matrices(int n_gates, const qc_gate_t *gates, int k, const int *qubits, int n_sel,
                      const int *sel_qubits, double *out) {
    if (k < 1 || k > QC_MAX_FUSED) return fail(QC_ERR_ARG, "k out of range");
    if (n_sel < 0 || n_sel > QC_MAX_SEL) return fail(QC_ERR_ARG, "selector count out of range");
    if (!qubits || (n_sel > 0 && !sel_qubits) || !out || (n_gates > 0 && !gates) || n_gates < 0)
        return fail(QC_ERR_ARG, "NULL argument");
    int all[QC_MAX_FUSED + QC_MAX_SEL];
    for (int j = 0; j < k; ++j) all[j] = qubits[j];
    for (int j = 0; j < n_sel; ++j) all[k + j] = sel_qubits[j];
    int rc = check_qubits(QC_MAX_QUBITS, all, k + n_sel, "block qubit");
    if (rc) return rc;
    std::vector<const qc_gate_t *> gs(static_cast<size_t>(n_gates));
    for (int i = 0; i < n_gates; ++i) {
        const qc_gate_t &g = gates[i];
        if ((rc = check_gate(QC_MAX_QUBITS, g))) return rc;
        auto in = [&](int q, int lo, int hi) {
            for (int j = lo; j < hi; ++j)
                if (all[j] == q) return true;
            return false;
        };
        const bool diag = matrix_is_diagonal(g.matrix, g.n_targets);
        for (int j = 0; j < g.n_targets; ++j)
            if (!in(g.targets[j], 0, k) && !(diag && in(g.targets[j], k, k + n_sel)))
                return fail(QC_ERR_QUBIT, "gate target outside the block (or non-diagonal on a selector)");
        for (int j = 0; j < g.n_ctrls; ++j)
            if (!in(g.ctrls[j], 0, k + n_sel)) return fail(QC_ERR_QUBIT, "gate control outside the block");
        gs[size_t(i)] = &g;
    }
    const std::vector<cd> m = block_matrices(k, qubits, n_sel, sel_qubits, gs);
    for (size_t i = 0; i < m.size(); ++i) {
        out[2 * i] = m[i].real();
        out[2 * i + 1] = m[i].imag();
    }
    return QC_OK;
}

namespace {

// Move the bit of label from[q] to label to[q] for every qubit q.
int relabel(qc_state_t s, const int *from, const int *to, qc_exec_stats_t &st, void *stream) {
    uint32_t sigma[QC_MAX_QUBITS];
    for (int q = 0; q < s.n; ++q) sigma[bitpos(s.n, from[q])] = uint32_t(bitpos(s.n, to[q]));
    int sweeps = 0;
    const hipError_t e = qcx::launch_permute_bits(s.amp, s.dtype, s.n, sigma, &sweeps,
                                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "permute");
    st.launches += sweeps;
    st.sweeps += sweeps;
    st.state_bytes += sweeps * sweep_bytes(s.n, s.dtype);
    return QC_OK;
}

bool is_swap_gate(const qc_gate_t &g) {
    if (g.n_targets != 2 || g.n_ctrls != 0) return false;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            const bool one = (r == c && (r == 0 || r == 3)) || (r == 1 && c == 2) || (r == 2 && c == 1);
            if (g.matrix[2 * (4 * r + c)] != (one ? 1.0 : 0.0) || g.matrix[2 * (4 * r + c) + 1] != 0.0)
                return false;
        }
    return true;
}

// SWAP gates leave the list: the gates after one are rewritten with its two
// qubits exchanged.  phys[q] receives the label that holds qubit q's bit
// once `out` has been applied.  Returns false (out untouched) if the list
// holds no SWAP.
bool defer_swaps(int n, int ng, const qc_gate_t *gs, std::vector<qc_gate_t> &out, int *phys) {
    int i0 = 0;
    while (i0 < ng && !is_swap_gate(gs[i0])) ++i0;
    if (i0 == ng) return false;
    for (int q = 0; q < n; ++q) phys[q] = q;
    out.assign(gs, gs + i0);
    for (int i = i0; i < ng; ++i) {
        const qc_gate_t &g = gs[i];
        if (is_swap_gate(g)) {
            std::swap(phys[g.targets[0]], phys[g.targets[1]]);
            continue;
        }
        qc_gate_t h = g;
        for (int j = 0; j < h.n_targets; ++j) h.targets[j] = phys[g.targets[j]];
        for (int j = 0; j < h.n_ctrls; ++j) h.ctrls[j] = phys[g.ctrls[j]];
        out.push_back(h);
    }
    return true;
}

}  // namespace

int qc_permute_qubits(qc_state_t s, const int *perm, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!perm) return fail(QC_ERR_ARG, "perm is NULL");
    if ((rc = check_qubits(s.n, perm, s.n, "perm entry"))) return rc;
    int id[QC_MAX_QUBITS];
    for (int q = 0; q < s.n; ++q) id[q] = q;
    qc_exec_stats_t st{};
    return relabel(s, id, perm, st, stream);
}

int qc_apply_circuit(qc_state_t s, int n_gates, const qc_gate_t *gates, int mode, int fuse_k,
                     qc_exec_stats_t *stats, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (n_gates < 0 || (n_gates > 0 && !gates)) return fail(QC_ERR_ARG, "gate list is NULL");
    if (mode != QC_EXEC_UNFUSED && mode != QC_EXEC_FUSED && mode != QC_EXEC_TILED)
        return fail(QC_ERR_ARG, "unknown mode");
    if (mode == QC_EXEC_FUSED && (fuse_k < 1 || fuse_k > QC_MAX_FUSED))
        return fail(QC_ERR_ARG, "fuse_k out of range");
    if (fuse_k > s.n) fuse_k = s.n;   // blocks cannot be wider than the register
    for (int i = 0; i < n_gates; ++i)
        if ((rc = check_gate(s.n, gates[i]))) return rc;
    qc_exec_stats_t st{};
    st.gates = n_gates;
    if (mode == QC_EXEC_UNFUSED) {
        for (int i = 0; i < n_gates; ++i)
            if ((rc = apply_gate_unfused(s, gates[i], st, stream))) return rc;
    } else {
        std::vector<qc_gate_t> rel;
        int phys[QC_MAX_QUBITS];
        const bool deferred = defer_swaps(s.n, n_gates, gates, rel, phys);
        const qc_gate_t *gl = deferred ? rel.data() : gates;
        const int ng = deferred ? int(rel.size()) : n_gates;
        if (ng > 0) {
            rc = mode == QC_EXEC_TILED
                     ? tiled_execute(s, ng, gl, st, stream)
                     : fused_execute(s, ng, gl, fuse_k, g_knob_look.load(), st, stream);
            if (rc) return rc;
        }
        if (deferred) {
            int id[QC_MAX_QUBITS];
            for (int q = 0; q < s.n; ++q) id[q] = q;
            if ((rc = relabel(s, phys, id, st, stream))) return rc;
        }
    }
    if (stats) *stats = st;
    return QC_OK;
}

int qc_probs(qc_state_t s, int m, const int *qubits, double *out_dev, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!out_dev) return fail(QC_ERR_ARG, "output pointer is NULL");
    if (m < 1 || m > s.n) return fail(QC_ERR_ARG, "m out of range");
    if (m != s.n && m > 24) return fail(QC_ERR_UNSUPPORTED, "marginal over more than 24 qubits");
    if ((rc = check_qubits(s.n, qubits, m, "qubit"))) return rc;
    int pos[QC_MAX_QUBITS];
    bool identity = (m == s.n);
    for (int j = 0; j < m; ++j) {
        pos[j] = bitpos(s.n, qubits[j]);
        if (qubits[j] != j) identity = false;
    }
    hipError_t e;
    if (m == s.n) {
        e = qcx::launch_probs_full(s.amp, s.dtype, s.n, pos, identity, out_dev, (hipStream_t)stream);
    } else {
        DevCtx *c;
        if ((rc = get_ctx(&c))) return rc;
        e = qcx::launch_probs_marginal(s.amp, s.dtype, s.n, m, pos, out_dev, c->work, kWorkElems,
                                       (hipStream_t)stream);
    }
    return e == hipSuccess ? QC_OK : hip_fail(e, "probs");
}

}  // extern "C"

// ---------------------------------------------------- allocation-free probs

// Partial sums of qc_probs_noalloc: a fixed device array instead of the
// allocated workspace.  Every GPU the library runs on holds its own copy
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it only names the symbol): the device address comes
// from hipGetSymbolAddress, once per device, kept in g_scratch_dev.
static __device__ __align__(256) double scratch[QC_PROBS_NOALLOC_SCRATCH];

namespace {

constexpr size_t kScratchElems = QC_PROBS_NOALLOC_SCRATCH;
double *g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

int scratch_address(double **out) {
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (d < 0 || d >= kMaxDevices) return fail(QC_ERR_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[d]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(QC_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[d] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[d];
    return QC_OK;
}

}  // namespace

extern "C" {

int qc_probs_noalloc(qc_state_t s, int m, const int *qubits, double *out_dev, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (!out_dev) return fail(QC_ERR_ARG, "output pointer is NULL");
    if (m < 1 || m > s.n) return fail(QC_ERR_ARG, "m out of range");
    if (m != s.n && m > 24) return fail(QC_ERR_UNSUPPORTED, "marginal over more than 24 qubits");
    if ((rc = check_qubits(s.n, qubits, m, "qubit"))) return rc;
    int pos[QC_MAX_QUBITS];
    bool identity = (m == s.n);
    for (int j = 0; j < m; ++j) {
        pos[j] = bitpos(s.n, qubits[j]);
        if (qubits[j] != j) identity = false;
    }
    const hipStream_t hs = (hipStream_t)stream;
    hipError_t e;
    if (m == s.n) {   // one output per amplitude: no partial sums at all
        e = qcx::launch_probs_full(s.amp, s.dtype, s.n, pos, identity, out_dev, hs);
    } else {
        const size_t need = qcx::probs_marginal_work(s.n, m);
        if (need > kScratchElems)
            return fail(QC_ERR_UNSUPPORTED, "marginal needs " + std::to_string(need) +
                                                " partial sums, more than the " +
                                                std::to_string(kScratchElems) +
                                                " of the static scratch array");
        double *work = nullptr;
        if ((rc = scratch_address(&work))) return rc;
        e = qcx::launch_probs_marginal(s.amp, s.dtype, s.n, m, pos, out_dev, work, kScratchElems,
                                       hs);
    }
    return e == hipSuccess ? QC_OK : hip_fail(e, "probs_noalloc");
}

}  // extern "C"

namespace {

// The terms no tile pass took (X bits spread wider than a tile) with the
// pair kernel, grouped by x mask; then out[0] = sum_t c_t v_t and
// out[1 + t] = v_t in the caller's order (where[t] = slot of term t).
int expect_finish(qc_state_t s, int n_terms, const std::vector<uint64_t> &xm,
                  const std::vector<uint64_t> &zm, const std::vector<int> &ph, const double *coeff,
                  int per_term, double *out_dev, DevCtx *c, hipStream_t hs, std::vector<int> &where,
                  int slot, std::vector<int> &order) {
    const int n = s.n;
    int rc;
    double *vals = c->work;
    double *part = c->work + ((n_terms + 255) & ~255);
    // pair kernel: group the remaining terms by x mask, preserving first-seen order
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return xm[a] < xm[b]; });
    for (size_t i = 0; i < order.size(); ++i) where[order[i]] = slot + int(i);
    vals += slot;
    size_t i0 = 0;
    while (i0 < order.size()) {
        size_t i1 = i0;
        while (i1 < order.size() && xm[order[i1]] == xm[order[i0]] &&
               i1 - i0 < size_t(qcx::kExpectMaxTerms))
            ++i1;
        const uint64_t x = xm[order[i0]];
        const int hpos = x ? 63 - __builtin_clzll(x) : -1;
        uint64_t zz[qcx::kExpectMaxTerms];
        int pp[qcx::kExpectMaxTerms];
        for (size_t i = i0; i < i1; ++i) {
            zz[i - i0] = zm[order[i]];
            pp[i - i0] = ph[order[i]];
        }
        hipError_t e = qcx::launch_expect_group(s.amp, s.dtype, n, x, hpos, int(i1 - i0), zz, pp,
                                                vals + i0, part, hs);
        if (e != hipSuccess) return hip_fail(e, "expect");
        i0 = i1;
    }
    vals = c->work;
    // combine in the caller's term order: out[0] = sum_t c_t v_t, out[1+t] = v_t
    std::vector<double> tab(size_t(2) * n_terms);
    for (int t = 0; t < n_terms; ++t) {
        tab[t] = coeff[t];
        tab[n_terms + t] = double(where[t]);
    }
    void *cdev = nullptr;
    if ((rc = stage(c, tab.data(), tab.size() * sizeof(double), hs, &cdev))) return rc;
    hipError_t e = qcx::launch_expect_combine(vals, static_cast<const double *>(cdev), n_terms,
                                              per_term, out_dev, hs);
    if (e != hipSuccess) return hip_fail(e, "expect_combine");
    return QC_OK;
}



// Register-tile passes (k_expect_reg, k_pauli_reg): a wavefront tile is 6
// lane bits and kExpRegB element bits.  The first pass has the six lowest
// bits on the lanes (512 contiguous bytes or more per load); later passes
// keep only the bits of one 128-byte run on the lanes (4 for complex64, 3
// for complex128) and put new bits on the other lanes and the elements, so a
// later pass covers up to 6 - LL + kExpRegB new bits.  A term is taken in
// the first pass whose tile holds its X bits all on the lanes or on one
// element bit; every diagonal term rides in the first pass.  Each launch
// lists its X terms, then its diagonal terms grouped by element mask (the
// ranges in hoff); ids gives the caller's term index of every entry.
// Terms that fit no pass are appended to `left`.
struct RegLaunch {
    qcx::ExpRegArgs a;
    std::vector<qcx::ExpRegTerm> terms;
    std::vector<int> ids;
};

// for_expect: the launches feed k_expect_reg, whose diagonal terms with Z
// bits outside the tile share at most kExpRegMaxC (zsign, zl) pairs per
// launch; diagonal terms that would need more than one launch beyond those
// the X terms of the first pass need go to `left` (one LDS tile pass takes
// any number of them)
void plan_register_passes(int n, int dtype, int n_terms, const std::vector<uint64_t> &xm,
                          const std::vector<uint64_t> &zm, const std::vector<int> &ph,
                          std::vector<RegLaunch> &launches, std::vector<int> &left,
                          bool for_expect) {
    constexpr int RB = qcx::kExpRegB;
    const int LL = dtype == QC_C64 ? 4 : 3;
    const uint64_t low6 = 63, lowL = (uint64_t(1) << LL) - 1;
    const int capL = 6 - LL + RB;
    std::vector<int> diag, rest;
    for (int t = 0; t < n_terms; ++t) {
        if (xm[t] == 0) diag.push_back(t);
        else if (__builtin_popcountll(xm[t] & ~low6) <= RB ||
                 __builtin_popcountll(xm[t] & ~lowL) <= capL)
            rest.push_back(t);
        else
            left.push_back(t);
    }
    // choose the new bits of a pass: the high X bits of the remaining terms
    // in order while they fit, then the bits most used by the rest, then the
    // lowest free ones
    auto choose = [&](uint64_t fixed, int cap) {
        uint64_t S = 0;
        for (int t : rest) {
            const uint64_t hb = xm[t] & ~fixed;
            if (__builtin_popcountll(S | hb) <= cap) S |= hb;
        }
        std::vector<int> cnt(n, 0);
        for (int t : rest)
            for (int p = 0; p < n; ++p)
                if (((xm[t] & ~fixed) >> p) & 1) ++cnt[p];
        while (__builtin_popcountll(S) < cap) {
            int best = -1;
            for (int p = 0; p < n; ++p)
                if (!((S | fixed) >> p & 1) && (best < 0 || cnt[p] > cnt[best])) best = p;
            if (best < 0) break;
            S |= uint64_t(1) << best;
        }
        return S;
    };
    bool first = true;
    while (first || !rest.empty()) {
        qcx::ExpRegArgs a{};
        uint64_t P;
        if (first) {
            const uint64_t S = choose(low6, RB);
            for (int k = 0; k < 6; ++k) a.lpos[k] = uint32_t(k);
            for (int i = 0, p = 0; p < n; ++p)
                if ((S >> p) & 1) a.rpos[i++] = uint32_t(p);
            P = low6 | S;
        } else {
            const uint64_t S = choose(lowL, capL);
            int k = 0, i = 0;
            for (; k < LL; ++k) a.lpos[k] = uint32_t(k);
            for (int p = 0; p < n; ++p) {
                if (!((S >> p) & 1)) continue;
                if (k < 6) a.lpos[k++] = uint32_t(p);   // the lowest new bits go to the lanes
                else a.rpos[i++] = uint32_t(p);
            }
            P = lowL | S;
        }
        // slot masks of a global bit mask
        auto on_lanes = [&](uint64_t m) {
            uint32_t r = 0;
            for (int k = 0; k < 6; ++k)
                if ((m >> a.lpos[k]) & 1) r |= 1u << k;
            return r;
        };
        auto on_elems = [&](uint64_t m) {
            uint32_t r = 0;
            for (int i = 0; i < RB; ++i)
                if ((m >> a.rpos[i]) & 1) r |= 1u << i;
            return r;
        };
        // a term whose X bits are all on the lanes, or one element bit
        std::vector<int> xs, stay;
        for (int t : rest) {
            const bool fits = (xm[t] & ~P) == 0 &&
                              (on_elems(xm[t]) == 0 ||
                               (on_lanes(xm[t]) == 0 && __builtin_popcount(on_elems(xm[t])) == 1));
            (fits ? xs : stay).push_back(t);
        }
        rest.swap(stay);
        std::vector<int> ds = first ? diag : std::vector<int>();
        const bool was_first = first;
        first = false;
        if (xs.empty() && ds.empty()) {
            if (was_first) continue;
            break;   // no progress: the caller's other paths take the rest
        }
        // diagonal terms grouped by their element mask
        std::stable_sort(ds.begin(), ds.end(),
                         [&](int p, int q) { return on_elems(zm[p]) < on_elems(zm[q]); });
        for (int j = 0, p = 0; p < n; ++p)
            if ((P >> p) & 1) a.pos[j++] = uint32_t(p);
        a.n_tiles = uint64_t(1) << (n - 6 - RB);
        // the transposed tile of complex64 expectation passes (loaded tile
        // bit j < 6 = lane bit j, 6 + i = element bit i).  First pass: the
        // element bits of the transposed tile are lane bits 0..3 and its
        // lane bits 0, 1 lane bits 4, 5 (DPP partners); later passes: its
        // element bits 2, 3 are lane bits 4, 5.  Padding of one amplitude
        // per 16 (first) or 64 (later) keeps both LDS access patterns free
        // of bank conflicts.
        const bool transpose = for_expect && dtype == QC_C64;
        static const uint32_t tl_first[6] = {4, 5, 6, 7, 8, 9}, te_first[4] = {0, 1, 2, 3};
        static const uint32_t tl_later[6] = {2, 3, 6, 7, 8, 9}, te_later[4] = {0, 1, 4, 5};
        const uint32_t *tl = was_first ? tl_first : tl_later, *te = was_first ? te_first : te_later;
        auto gpos = [&](uint32_t j) { return j < 6 ? a.lpos[j] : a.rpos[j - 6]; };
        auto on_tlanes = [&](uint64_t m) {
            uint32_t r = 0;
            for (int k = 0; k < 6; ++k)
                if ((m >> gpos(tl[k])) & 1) r |= 1u << k;
            return r;
        };
        auto on_telems = [&](uint64_t m) {
            uint32_t r = 0;
            for (int i = 0; i < RB; ++i)
                if ((m >> gpos(te[i])) & 1) r |= 1u << i;
            return r;
        };
        // an X term on one lane bit goes to the transposed tile where that
        // saves LDS permutes or DPP moves: lane bits 0..5 in the first pass,
        // 4 and 5 in the later ones
        auto to_transposed = [&](int t) {
            if (!transpose || on_elems(xm[t]) != 0 || __builtin_popcount(on_lanes(xm[t])) != 1) return false;
            return was_first || __builtin_ctz(on_lanes(xm[t])) >= 4;
        };
        auto term = [&](int t) {
            const bool tr = to_transposed(t);
            qcx::ExpRegTerm e{};
            e.z_hi = zm[t] & ~P;
            e.xl = tr ? on_tlanes(xm[t]) : on_lanes(xm[t]);
            e.xr = tr ? on_telems(xm[t]) : on_elems(xm[t]);
            e.zl = tr ? on_tlanes(zm[t]) : on_lanes(zm[t]);
            const uint32_t zr = tr ? on_telems(zm[t]) : on_elems(zm[t]);
            for (int el = 0; el < (1 << RB); ++el)
                if (__builtin_popcount(uint32_t(el) & zr) & 1) e.zsign |= 1u << el;
            e.ph = ph[t];
            e.hk = -1;
            e.ck = -1;
            // X terms: element bit i -> mode i; a lane bit below 4 -> DPP
            // partners, mode 4 + b; any other lane mask -> LDS permutes, mode 8
            int mode = 8;
            if (e.xr != 0) mode = __builtin_ctz(e.xr);
            else if (__builtin_popcount(e.xl) == 1 && e.xl < 16) mode = 4 + __builtin_ctz(e.xl);
            e.kind = 2 * mode + (ph[t] & 1);
            return e;
        };
        size_t xi = 0, di = 0;
        const size_t diag_launches =
            for_expect ? std::max<size_t>(1, (xs.size() + qcx::kExpRegMaxX - 1) / qcx::kExpRegMaxX) + 1
                       : ds.size();
        size_t n_launch = 0;
        while (xi < xs.size() || di < ds.size()) {
            if (di < ds.size() && n_launch == diag_launches) {
                left.insert(left.end(), ds.begin() + long(di), ds.end());
                di = ds.size();
                if (xi == xs.size()) break;
            }
            ++n_launch;
            const size_t x1 = std::min(xs.size(), xi + qcx::kExpRegMaxX);
            RegLaunch L;
            L.a = a;
            L.a.n_xb = 0;
            for (int k = 0; k < 6; ++k) L.a.tl[k] = tl[k];
            for (int i = 0; i < RB; ++i) L.a.te[i] = te[i];
            L.a.tsh = was_first ? 4 : 6;
            L.a.tpad = 1;
            for (int pass_b = 0; pass_b < 2; ++pass_b)   // untransposed terms first
                for (size_t k = xi; k < x1; ++k) {
                    if (to_transposed(xs[k]) != (pass_b == 1)) continue;
                    L.terms.push_back(term(xs[k]));
                    L.ids.push_back(xs[k]);
                    L.a.n_xb += pass_b;
                }
            L.a.n_x = int(x1 - xi);
            L.a.n_h = 0;
            L.a.n_c = 0;
            L.a.n_din = 0;
            // diagonal terms in order while the launch has room: at most
            // kExpRegMaxD, and at most kExpRegMaxC distinct (zsign, zl) pairs
            // among those with Z bits outside the tile
            size_t d1 = di;
            for (; d1 < ds.size() && d1 - di < size_t(qcx::kExpRegMaxD); ++d1) {
                const qcx::ExpRegTerm e = term(ds[d1]);
                if (!for_expect || e.z_hi == 0) continue;
                int c = 0;
                while (c < L.a.n_c && !(L.a.csign[c] == e.zsign && L.a.clane[c] == e.zl)) ++c;
                if (c == L.a.n_c) {
                    if (c == qcx::kExpRegMaxC) break;
                    L.a.csign[c] = e.zsign;
                    L.a.clane[c] = e.zl;
                    ++L.a.n_c;
                }
            }
            for (size_t k = di; k < d1; ++k) {
                qcx::ExpRegTerm e = term(ds[k]);
                if (!for_expect) {
                    // k_pauli_reg takes every diagonal term per lane
                } else if (e.z_hi == 0) {
                    ++L.a.n_din;
                } else {
                    int c = 0;
                    while (!(L.a.csign[c] == e.zsign && L.a.clane[c] == e.zl)) ++c;
                    e.ck = c;
                }
                const uint32_t zr = on_elems(zm[ds[k]]);
                int h = 0;
                while (h < L.a.n_h && L.a.hval[h] != zr) ++h;
                if (h == L.a.n_h) {
                    L.a.hoff[h] = uint32_t(k - di);
                    L.a.hval[L.a.n_h++] = zr;
                }
                e.hk = h;
                L.terms.push_back(e);
                L.ids.push_back(ds[k]);
            }
            L.a.n_d = int(d1 - di);
            L.a.hoff[L.a.n_h] = uint32_t(L.a.n_d);
            launches.push_back(std::move(L));
            xi = x1;
            di = d1;
        }
    }
    left.insert(left.end(), rest.begin(), rest.end());
}

// lam = H psi: register-tile passes (the first writes lam, the others add),
// then the gather kernel for the terms no pass takes; the gather kernel
// alone below 12 qubits.
int pauli_apply(qc_state_t psi, qc_state_t lam, const std::vector<qcx::PauliTermDev> &terms,
                DevCtx *c, hipStream_t hs) {
    const int nt = int(terms.size());
    std::vector<RegLaunch> launches;
    std::vector<int> left;
    if (psi.n >= 6 + qcx::kExpRegB + 2) {
        std::vector<uint64_t> xm(nt), zm(nt);
        std::vector<int> ph(nt);
        for (int t = 0; t < nt; ++t) {
            xm[t] = terms[t].x;
            zm[t] = terms[t].z;
            ph[t] = terms[t].ph;
        }
        plan_register_passes(psi.n, psi.dtype, nt, xm, zm, ph, launches, left, false);
    } else {
        for (int t = 0; t < nt; ++t) left.push_back(t);
    }
    bool written = false;
    // every pass's terms and coefficients in one copy
    std::vector<unsigned char> blob(16, 0);   // a valid device address for term-less passes
    std::vector<size_t> toff, coff;
    auto append = [&](const void *p, size_t bytes) {
        blob.resize((blob.size() + 255) & ~size_t(255));
        const size_t at = blob.size();
        const unsigned char *b = static_cast<const unsigned char *>(p);
        blob.insert(blob.end(), b, b + bytes);
        return at;
    };
    for (const RegLaunch &L : launches) {
        std::vector<double> coef(L.ids.size());
        for (size_t k = 0; k < L.ids.size(); ++k) coef[k] = terms[L.ids[k]].c;
        toff.push_back(append(L.terms.data(), L.terms.size() * sizeof(qcx::ExpRegTerm)));
        coff.push_back(append(coef.data(), coef.size() * sizeof(double)));
    }
    void *bdev = nullptr;
    if (!launches.empty()) {
        const int rc = stage(c, blob.data(), blob.size(), hs, &bdev);
        if (rc) return rc;
    }
    for (size_t i = 0; i < launches.size(); ++i) {
        const RegLaunch &L = launches[i];
        const unsigned char *base = static_cast<const unsigned char *>(bdev);
        hipError_t e = qcx::launch_pauli_reg(psi.amp, lam.amp, psi.dtype, L.a,
                                             reinterpret_cast<const qcx::ExpRegTerm *>(base + toff[i]),
                                             reinterpret_cast<const double *>(base + coff[i]), written, hs);
        if (e != hipSuccess) return hip_fail(e, "pauli_reg");
        written = true;
    }
    if (!left.empty()) {
        std::vector<qcx::PauliTermDev> rest;
        for (int t : left) rest.push_back(terms[t]);
        void *tdev = nullptr;
        int rc = stage(c, rest.data(), rest.size() * sizeof(qcx::PauliTermDev), hs, &tdev);
        if (rc) return rc;
        hipError_t e = qcx::launch_pauli_apply(psi.amp, lam.amp, psi.dtype, psi.n,
                                               static_cast<const qcx::PauliTermDev *>(tdev),
                                               int(rest.size()), written, hs);
        if (e != hipSuccess) return hip_fail(e, "pauli_apply");
    }
    return QC_OK;
}

int expect_register_passes(qc_state_t s, int n_terms, const std::vector<uint64_t> &xm,
                           const std::vector<uint64_t> &zm, const std::vector<int> &ph, DevCtx *c,
                           hipStream_t hs, double *vals, double *part, std::vector<int> &where,
                           int &slot, std::vector<int> &left) {
    std::vector<RegLaunch> launches;
    plan_register_passes(s.n, s.dtype, n_terms, xm, zm, ph, launches, left, true);
    // every pass's terms in one copy
    std::vector<unsigned char> blob;
    std::vector<size_t> off;
    for (const RegLaunch &L : launches) {
        blob.resize((blob.size() + 255) & ~size_t(255));
        off.push_back(blob.size());
        const unsigned char *b = reinterpret_cast<const unsigned char *>(L.terms.data());
        blob.insert(blob.end(), b, b + L.terms.size() * sizeof(qcx::ExpRegTerm));
    }
    void *bdev = nullptr;
    if (!launches.empty()) {
        if (blob.empty()) blob.resize(16, 0);   // a valid device address for term-less passes
        const int rc = stage(c, blob.data(), blob.size(), hs, &bdev);
        if (rc) return rc;
    }
    for (size_t i = 0; i < launches.size(); ++i) {
        const RegLaunch &L = launches[i];
        for (size_t k = 0; k < L.ids.size(); ++k) where[L.ids[k]] = slot + int(k);
        const void *tdev = static_cast<const unsigned char *>(bdev) + off[i];
        hipError_t e = qcx::launch_expect_reg(s.amp, s.dtype, L.a,
                                              static_cast<const qcx::ExpRegTerm *>(tdev),
                                              vals + slot, part, hs);
        if (e != hipSuccess) return hip_fail(e, "expect_reg");
        slot += L.a.n_x + L.a.n_d;
    }
    return QC_OK;
}

}  // namespace

extern "C" {
int qc_expect_pauli(qc_state_t s, int n_terms, const char *paulis, const double *coeff,
                    int per_term, double *out_dev, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (n_terms < 1 || n_terms > 65536) return fail(QC_ERR_ARG, "term count out of range");
    if (!paulis || !coeff || !out_dev) return fail(QC_ERR_ARG, "NULL argument");
    const int n = s.n;
    std::vector<uint64_t> xm(n_terms), zm(n_terms);
    std::vector<int> ph(n_terms);
    for (int t = 0; t < n_terms; ++t) {
        uint64_t x = 0, z = 0;
        int ny = 0;
        for (int q = 0; q < n; ++q) {
            const char ch = paulis[size_t(t) * n + q];
            const uint64_t b = uint64_t(1) << bitpos(n, q);
            switch (ch) {
            case 'I': break;
            case 'X': x |= b; break;
            case 'Y': x |= b; z |= b; ++ny; break;
            case 'Z': z |= b; break;
            default: return fail(QC_ERR_ARG, "Pauli character not in {I,X,Y,Z}");
            }
        }
        xm[t] = x;
        zm[t] = z;
        ph[t] = ny & 3;
    }
    DevCtx *c;
    if ((rc = get_ctx(&c))) return rc;
    const hipStream_t hs = (hipStream_t)stream;
    double *vals = c->work;                         // n_terms values
    double *part = c->work + ((n_terms + 255) & ~255);  // per-block partials
    std::vector<int> where(n_terms);
    int slot = 0;
    std::vector<int> order;   // terms left to the pair kernel
    // registers tiles first (every diagonal term and every term whose X
    // bits fit one of their passes); the LDS tile passes take the rest
    std::vector<int> left;
    if (n >= 6 + qcx::kExpRegB + 2) {
        if ((rc = expect_register_passes(s, n_terms, xm, zm, ph, c, hs, vals, part, where, slot,
                                         left)))
            return rc;
    } else {
        for (int t = 0; t < n_terms; ++t) left.push_back(t);
    }
    // Tile passes: the tile is the kExpectLowBits lowest bits plus up to
    // m - kExpectLowBits more; a term whose X bits all lie in a pass's tile
    // bits is evaluated in that pass (the pair j, j ^ x is in one tile), and
    // every diagonal term rides in the first pass.  Terms that fit no tile
    // (more X bits above the low ones than a tile has room for) are
    // evaluated one X mask at a time with the pair kernel.
    const int m = std::min(n, s.dtype == QC_C64 ? 12 : 11);
    const int L = std::min(qcx::kExpectLowBits, m);
    const uint64_t low = (uint64_t(1) << L) - 1;
    std::vector<int> rest, diag;
    for (int t : left) {
        if (xm[t] == 0) diag.push_back(t);
        else if (__builtin_popcountll(xm[t] & ~low) <= m - L) rest.push_back(t);
        else order.push_back(t);   // pair kernel
    }
    struct ExpPass {
        uint64_t P;
        std::vector<int> terms;
    };
    std::vector<ExpPass> passes;
    while (!rest.empty()) {
        uint64_t S = 0;
        for (int t : rest) {
            const uint64_t hb = xm[t] & ~low;
            if (__builtin_popcountll(S | hb) <= m - L) S |= hb;
        }
        for (int p = L; __builtin_popcountll(S) < m - L && p < n; ++p) S |= uint64_t(1) << p;
        ExpPass ps{low | S, {}};
        std::vector<int> left;
        for (int t : rest) ((xm[t] & ~ps.P) == 0 ? ps.terms : left).push_back(t);
        passes.push_back(std::move(ps));
        rest.swap(left);
    }
    if (!diag.empty()) {
        if (passes.empty()) {
            uint64_t P = 0;
            for (int p = 0; p < m; ++p) P |= uint64_t(1) << p;
            passes.push_back({P, {}});
        }
        passes[0].terms.insert(passes[0].terms.begin(), diag.begin(), diag.end());
    }
    // term values: tile-pass terms first (pass order), then the pair
    // kernel's terms grouped by x mask; combine permutes them back
    for (const ExpPass &ps : passes) {
        for (size_t k0 = 0; k0 < ps.terms.size(); k0 += qcx::kExpectTileMaxTerms) {
            const size_t k1 = std::min(ps.terms.size(), k0 + qcx::kExpectTileMaxTerms);
            std::vector<qcx::ExpectTerm> et(k1 - k0);
            for (size_t k = k0; k < k1; ++k) {
                const int t = ps.terms[k];
                uint32_t xc = 0, zc = 0;
                for (int p = 0, j = 0; p < n; ++p) {
                    if (!((ps.P >> p) & 1)) continue;
                    if ((xm[t] >> p) & 1) xc |= 1u << j;
                    if ((zm[t] >> p) & 1) zc |= 1u << j;
                    ++j;
                }
                qcx::ExpectTerm &e = et[k - k0];
                e.z_hi = zm[t] & ~ps.P;
                e.xc = xc;
                e.zc = zc;
                e.ph = ph[t];
                e.xtop = xc ? 31 - __builtin_clz(xc) : -1;
                where[t] = slot + int(k - k0);
            }
            void *tdev = nullptr;
            if ((rc = stage(c, et.data(), et.size() * sizeof(qcx::ExpectTerm), hs, &tdev))) return rc;
            const qcx::TileArgs a = tile_args(n, m, ps.P, 0);
            hipError_t e = qcx::launch_expect_tiles(s.amp, s.dtype, a,
                                                    static_cast<const qcx::ExpectTerm *>(tdev),
                                                    int(k1 - k0), vals + slot, part, hs);
            if (e != hipSuccess) return hip_fail(e, "expect_tiles");
            slot += int(k1 - k0);
        }
    }
    return expect_finish(s, n_terms, xm, zm, ph, coeff, per_term, out_dev, c, hs, where, slot,
                         order);
}
int qc_collapse(qc_state_t s, int q, int outcome, double *prob_dev, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (outcome != 0 && outcome != 1) return fail(QC_ERR_ARG, "outcome must be 0 or 1");
    if ((rc = check_qubits(s.n, &q, 1, "qubit"))) return rc;
    DevCtx *c;
    if ((rc = get_ctx(&c))) return rc;
    const hipStream_t hs = (hipStream_t)stream;
    const int p = bitpos(s.n, q);
    // P(0), P(1) into the workspace tail, then the rescale reads them there
    double *pr = c->work + kWorkElems - 2;
    hipError_t e = qcx::launch_probs_marginal(s.amp, s.dtype, s.n, 1, &p, pr, c->work,
                                              kWorkElems - 2, hs);
    if (e == hipSuccess) e = qcx::launch_collapse(s.amp, s.dtype, s.n, p, outcome, pr, prob_dev, hs);
    return e == hipSuccess ? QC_OK : hip_fail(e, "collapse");
}

int qc_reset(qc_state_t s, int q, int outcome, double *prob_dev, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (outcome != 0 && outcome != 1) return fail(QC_ERR_ARG, "outcome must be 0 or 1");
    if ((rc = check_qubits(s.n, &q, 1, "qubit"))) return rc;
    DevCtx *c;
    if ((rc = get_ctx(&c))) return rc;
    const hipStream_t hs = (hipStream_t)stream;
    const int p = bitpos(s.n, q);
    double *pr = c->work + kWorkElems - 2;
    hipError_t e = qcx::launch_probs_marginal(s.amp, s.dtype, s.n, 1, &p, pr, c->work,
                                              kWorkElems - 2, hs);
    if (e == hipSuccess) e = qcx::launch_reset(s.amp, s.dtype, s.n, p, outcome, pr, prob_dev, hs);
    return e == hipSuccess ? QC_OK : hip_fail(e, "reset");
}

int qc_reduced_state(qc_state_t src, int m, const int *qubits, const int *values, qc_state_t dst,
                     void *stream) {
    int rc = check_state(src);
    if (rc) return rc;
    if ((rc = check_state(dst))) return rc;
    if (m < 1 || m >= src.n) return fail(QC_ERR_ARG, "m out of range");
    if (!values) return fail(QC_ERR_ARG, "values pointer is NULL");
    if ((rc = check_qubits(src.n, qubits, m, "qubit"))) return rc;
    if (dst.n != src.n - m || dst.dtype != src.dtype)
        return fail(QC_ERR_ARG, "destination must have n - m qubits and the same dtype");
    int pos[QC_MAX_QUBITS], val[QC_MAX_QUBITS];
    for (int j = 0; j < m; ++j) {
        if (values[j] != 0 && values[j] != 1) return fail(QC_ERR_ARG, "values must be 0 or 1");
        pos[j] = bitpos(src.n, qubits[j]);
        val[j] = values[j];
    }
    hipError_t e = qcx::launch_reduced(src.amp, dst.amp, src.dtype, src.n, m, pos, val,
                                       (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "reduced_state");
}

int qc_sample(qc_state_t s, int shots, const double *u_dev, int64_t *out_dev, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (shots < 0 || (shots > 0 && (!u_dev || !out_dev))) return fail(QC_ERR_ARG, "NULL argument");
    DevCtx *c;
    if ((rc = get_ctx(&c))) return rc;
    hipError_t e = qcx::launch_sample(s.amp, s.dtype, s.n, u_dev, shots, out_dev, c->work,
                                      kWorkElems, (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "sample");
}

int qc_counts(qc_state_t s, int m, const int *qubits, int shots, const double *u_dev,
              int64_t *counts_dev, void *stream) {
    int rc = check_state(s);
    if (rc) return rc;
    if (m < 1 || m > s.n || m > QC_MAX_COUNT_QUBITS)
        return fail(QC_ERR_ARG, "m must be in [1, min(n, QC_MAX_COUNT_QUBITS)]");
    if (shots < 0 || shots > QC_MAX_COUNT_SHOTS)
        return fail(QC_ERR_ARG, "shots must be in [0, QC_MAX_COUNT_SHOTS]");
    if (!counts_dev || (shots > 0 && !u_dev)) return fail(QC_ERR_ARG, "NULL argument");
    if ((rc = check_qubits(s.n, qubits, m, "qubit"))) return rc;
    DevCtx *c;
    if ((rc = get_ctx(&c))) return rc;
    int pos[QC_MAX_QUBITS];
    for (int j = 0; j < m; ++j) pos[j] = bitpos(s.n, qubits[j]);
    // the sampled indices sit at the top of the workspace; the sampler's
    // chunk sums use at most 2^22 + 1 entries below them
    constexpr size_t kIdx = size_t(QC_MAX_COUNT_SHOTS);
    static_assert(kWorkElems - kIdx >= (size_t(2) << 21) + 1, "chunk-sum area");
    int64_t *idx = reinterpret_cast<int64_t *>(c->work + (kWorkElems - kIdx));
    const hipStream_t hs = (hipStream_t)stream;
    hipError_t e = qcx::launch_sample(s.amp, s.dtype, s.n, u_dev, shots, idx, c->work,
                                      kWorkElems - kIdx, hs);
    if (e == hipSuccess) e = qcx::launch_count(idx, shots, m, pos, counts_dev, hs);
    return e == hipSuccess ? QC_OK : hip_fail(e, "counts");
}

}  // extern "C"

namespace {

// Operand layout for the FP32 matrix-core kernel: see qc_fused_mfma.hip for
// the register mapping.  Three real 32x32 matrices in the order Ur, Ui,
// Ur + Ui (the three products of the 3M complex multiplication).
void mfma_operand_c64(const std::vector<cd> &u, std::vector<float> &out) {
    out.assign(3 * 32 * 32, 0.f);
    for (int r = 0; r < 32; ++r)
        for (int c = 0; c < 32; ++c) {
            const cd v = u[size_t(r) * 32 + c];
            out[0 * 1024 + r * 32 + c] = float(v.real());
            out[1 * 1024 + r * 32 + c] = float(v.imag());
            out[2 * 1024 + r * 32 + c] = float(v.real() + v.imag());
        }
}

// FP64 matrix of a one-qubit program op (rotations take theta[param]).
void op_matrix(const qc_op_t &op, const double *theta, qcx::Mat2d &m) {
    const double r2 = std::sqrt(0.5);
    double t = 0.0;
    if (op.kind == QC_OP_RX || op.kind == QC_OP_RY || op.kind == QC_OP_RZ) t = theta[op.param];
    const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
    for (int i = 0; i < 4; ++i) m.re[i] = m.im[i] = 0.0;
    switch (op.kind) {
    case QC_OP_RX: m.re[0] = c; m.im[1] = -s; m.im[2] = -s; m.re[3] = c; break;
    case QC_OP_RY: m.re[0] = c; m.re[1] = -s; m.re[2] = s; m.re[3] = c; break;
    case QC_OP_RZ: m.re[0] = c; m.im[0] = -s; m.re[3] = c; m.im[3] = s; break;
    case QC_OP_H: m.re[0] = r2; m.re[1] = r2; m.re[2] = r2; m.re[3] = -r2; break;
    case QC_OP_X: m.re[1] = 1; m.re[2] = 1; break;
    case QC_OP_Y: m.im[1] = -1; m.im[2] = 1; break;
    default: m.re[0] = 1; m.re[3] = -1; break;   // Z
    }
}

void mat_dagger(const qcx::Mat2d &a, qcx::Mat2d &d) {
    const int tr[4] = {0, 2, 1, 3};
    for (int i = 0; i < 4; ++i) {
        d.re[i] = a.re[tr[i]];
        d.im[i] = -a.im[tr[i]];
    }
}

bool is_rotation(int kind) { return kind == QC_OP_RX || kind == QC_OP_RY || kind == QC_OP_RZ; }

}  // namespace

extern "C" namespace {

// A diagonal gradient-and-apply op followed by a real one on the same bit
// (an inverse RZ and an inverse RY on one qubit in the backward pass)
// becomes one TILE_GRAD_APPLY2_DIAG_REAL op: one pass over both tiles'
// pairs instead of two.
void merge_grad_pairs(std::vector<qcx::TileOp> &ops) {
    auto plain = [](const qcx::TileOp &o) { return o.cmask_lo == 0 && o.cmask_hi == 0; };
    std::vector<qcx::TileOp> out;
    out.reserve(ops.size());
    for (size_t k = 0; k < ops.size(); ++k) {
        const qcx::TileOp &a = ops[k];
        if (k + 1 < ops.size() && a.kind == qcx::TILE_GRAD_APPLY_DIAG &&
            ops[k + 1].kind == qcx::TILE_GRAD_APPLY_REAL && ops[k + 1].b0 == a.b0 && plain(a) &&
            plain(ops[k + 1])) {
            const qcx::TileOp &b = ops[k + 1];
            qcx::TileOp mo{};
            mo.kind = qcx::TILE_GRAD_APPLY2_DIAG_REAL;
            mo.b0 = a.b0;
            mo.b1 = a.b1 | (b.b1 << 4);
            mo.pad = a.pad | (b.pad << 16);
            for (int i = 0; i < 8; ++i) {
                mo.u[i] = a.u[i];
                mo.u1[i] = b.u[i];
            }
            out.push_back(mo);
            ++k;
            continue;
        }
        out.push_back(a);
    }
    ops.swap(out);
}

// A pending block of diagonal rotations exp(-i t Z_q / 2) (or their
// inverses): the global bit of each, its gradient row (backward pass), the
// phase of the bit's set value relative to its clear value; the product of
// the clear values apart.  One entry per bit, at most 8 bits outside the
// tile (one window each), 48 entries.
struct DiagBlock {
    struct Ent {
        int pos, row;
        cd ph;
    };
    std::vector<Ent> ents;
    cd common = cd(1.0);
    bool empty() const { return ents.empty(); }
    size_t size() const { return ents.size(); }
    bool fits(int pos, uint64_t P) const {
        int n_out = 0;
        for (const Ent &d : ents) {
            if (d.pos == pos) return false;
            n_out += !((P >> d.pos) & 1);
        }
        return ents.size() < 48 && (((P >> pos) & 1) || n_out < 8);
    }
    void add(int pos, int row, const double *mu) {
        const cd d0(mu[0], mu[1]), d1(mu[6], mu[7]);
        common *= d0;
        ents.push_back({pos, row, d1 / d0});
    }
    // the TILE_DGRAD op: in-tile entries by ascending compressed bit, then
    // the out-of-tile ones; their gradient rows appended to `rows` in that
    // order when given (first slot b0 = rows->size())
    qcx::TileOp op(uint64_t P, std::vector<int32_t> *rows) const {
        qcx::TileOp o{};
        o.kind = qcx::TILE_DGRAD;
        o.b0 = rows ? int32_t(rows->size()) : 0;
        auto cidx = [&](int p) { return __builtin_popcountll(P & ((uint64_t(1) << p) - 1)); };
        std::vector<std::pair<int, int>> in;   // (compressed bit, entry)
        for (int i = 0; i < int(ents.size()); ++i)
            if ((P >> ents[i].pos) & 1) in.push_back({cidx(ents[i].pos), i});
        std::sort(in.begin(), in.end());
        for (const auto &ci : in) {
            o.b1 |= 1 << ci.first;
            o.u[2 * ci.first] = ents[ci.second].ph.real();
            o.u[2 * ci.first + 1] = ents[ci.second].ph.imag();
            if (rows) rows->push_back(ents[ci.second].row);
        }
        for (const Ent &d : ents) {
            if ((P >> d.pos) & 1) continue;
            o.fan_mask[o.pad] = uint64_t(1) << d.pos;
            o.fan_ph[2 * o.pad] = d.ph.real();
            o.fan_ph[2 * o.pad + 1] = d.ph.imag();
            ++o.pad;
            if (rows) rows->push_back(d.row);
        }
        o.u1[0] = common.real();
        o.u1[1] = common.imag();
        return o;
    }
    void clear() {
        ents.clear();
        common = cd(1.0);
    }
};

bool diag_gate(const qc_gate_t &g) {
    const double *mu = g.matrix;
    return g.n_targets == 1 && mu[2] == 0 && mu[3] == 0 && mu[4] == 0 && mu[5] == 0;
}

bool gate_touches(const qc_gate_t &g, int q) {
    for (int i = 0; i < g.n_targets; ++i)
        if (g.targets[i] == q) return true;
    for (int i = 0; i < g.n_ctrls; ++i)
        if (g.ctrls[i] == q) return true;
    return false;
}

}  // namespace

int qc_adjoint_grad(qc_state_t psi, qc_state_t lam, const qc_op_t *ops, int n_ops,
                               const double *theta, int n_params, int n_terms,
                               const char *paulis, const double *coeff, double *energy_dev,
                               double *grad_dev, void *stream) {
    int rc = check_state(psi);
    if (rc) return rc;
    if ((rc = check_state(lam))) return rc;
    if (psi.n != lam.n || psi.dtype != lam.dtype)
        return fail(QC_ERR_ARG, "psi and lam must have the same size and dtype");
    {
        const size_t bytes = (size_t(1) << psi.n) * (psi.dtype == QC_C64 ? 8 : 16);
        const char *a = (const char *)psi.amp, *b = (const char *)lam.amp;
        if (a < b + bytes && b < a + bytes) return fail(QC_ERR_ARG, "psi and lam overlap");
    }
    if (n_ops < 0 || (n_ops > 0 && !ops)) return fail(QC_ERR_ARG, "op list is NULL");
    if (n_params < 0 || (n_params > 0 && (!theta || !grad_dev)))
        return fail(QC_ERR_ARG, "theta or grad pointer is NULL");
    if (!energy_dev) return fail(QC_ERR_ARG, "energy pointer is NULL");
    if (n_terms < 1 || !paulis || !coeff) return fail(QC_ERR_ARG, "Hamiltonian is empty");
    const int n = psi.n;
    int n_rot = 0;
    for (int k = 0; k < n_ops; ++k) {
        const qc_op_t &o = ops[k];
        if (o.kind < QC_OP_RX || o.kind > QC_OP_CNOT) return fail(QC_ERR_ARG, "unknown op kind");
        const bool two = o.kind == QC_OP_CZ || o.kind == QC_OP_CNOT;
        const int q[2] = {o.q0, o.q1};
        if ((rc = check_qubits(n, q, two ? 2 : 1, "op qubit"))) return rc;
        if (is_rotation(o.kind)) {
            if (o.param < 0 || o.param >= n_params)
                return fail(QC_ERR_ARG, "rotation parameter index out of range");
            ++n_rot;
        }
    }
    std::vector<qcx::PauliTermDev> terms(n_terms);
    for (int t = 0; t < n_terms; ++t) {
        qcx::PauliTermDev T{};
        int ny = 0;
        for (int q = 0; q < n; ++q) {
            const uint64_t b = uint64_t(1) << bitpos(n, q);
            switch (paulis[size_t(t) * n + q]) {
            case 'I': break;
            case 'X': T.x |= b; break;
            case 'Y': T.x |= b; T.z |= b; ++ny; break;
            case 'Z': T.z |= b; break;
            default: return fail(QC_ERR_ARG, "Pauli character not in {I,X,Y,Z}");
            }
        }
        T.ph = ny & 3;
        T.c = coeff[t];
        terms[t] = T;
    }
    DevCtx *c;
    if ((rc = get_ctx(&c))) return rc;
    // two vectors share one 64 KiB LDS tile budget in the backward pass
    const int mb = std::min(n, psi.dtype == QC_C64 ? 12 : 11);
    const unsigned cols = qcx::adjoint_tile_grid(uint64_t(1) << (n - mb));
    const size_t need = size_t(n_rot) * cols + size_t(n_rot) + 1024;
    if (need > kWorkElems) return fail(QC_ERR_UNSUPPORTED, "too many rotations for the workspace");
    const hipStream_t hs = (hipStream_t)stream;
    hipError_t e;
    // gate lists: forward U_1..U_L and backward U_L^+..U_1^+ (one or two
    // qubits, at most one control), with FP64 matrices kept alive here
    std::vector<qc_gate_t> fwd(n_ops), bwd(n_ops);
    std::vector<double> mats(size_t(n_ops) * 16);
    std::vector<uint64_t> extra(n_ops, 0);
    std::vector<int> rot_row(n_ops, -1), gen_of(n_ops, 0);
    for (int k = 0, r = 0; k < n_ops; ++k) {
        const qc_op_t &o = ops[k];
        qc_gate_t g{};
        g.n_targets = 1;
        double *uf = &mats[size_t(k) * 16], *ub = uf + 8;
        if (o.kind == QC_OP_CZ || o.kind == QC_OP_CNOT) {
            g.targets[0] = o.q1;
            g.n_ctrls = 1;
            g.ctrls[0] = o.q0;
            g.ctrl_vals[0] = 1;
            const double z[8] = {1, 0, 0, 0, 0, 0, -1, 0}, x[8] = {0, 0, 1, 0, 1, 0, 0, 0};
            std::copy(o.kind == QC_OP_CZ ? z : x, (o.kind == QC_OP_CZ ? z : x) + 8, uf);
            std::copy(uf, uf + 8, ub);      // self-inverse
        } else {
            g.targets[0] = o.q0;
            qcx::Mat2d m, d;
            op_matrix(o, theta, m);
            mat_dagger(m, d);
            for (int i = 0; i < 4; ++i) {
                uf[2 * i] = m.re[i];
                uf[2 * i + 1] = m.im[i];
                ub[2 * i] = d.re[i];
                ub[2 * i + 1] = d.im[i];
            }
        }
        g.matrix = uf;
        fwd[k] = g;
        g.matrix = ub;
        bwd[n_ops - 1 - k] = g;
        if (is_rotation(o.kind)) {
            rot_row[n_ops - 1 - k] = r++;
            gen_of[n_ops - 1 - k] = o.kind == QC_OP_RX ? 1 : (o.kind == QC_OP_RY ? 2 : 3);
            extra[n_ops - 1 - k] = uint64_t(1) << bitpos(n, o.q0);   // reduction needs the bit
        }
    }
    // register-tile backward runs take the diagonal rotations of a layer as
    // one block (RT_DGRAD): every rotation with a non-diagonal matrix moves
    // later in the backward list past the gates that do not act on its
    // qubit (they commute with it and with its generator, so the gradients
    // are unchanged), which leaves a layer's diagonal rotations next to each
    // other; their bits then need not be tile bits
    const bool rt_bwd = g_knob_tile_engine.load() == 1 && mb == qcx::rt_adj_reg_bits(psi.dtype) + 9 &&
                        n - mb >= kRtMinTileBits;
    auto dblock_rot = [&](int k) { return rt_bwd && rot_row[k] >= 0 && gen_of[k] == 3 && diag_gate(bwd[k]); };
    if (rt_bwd) {
        for (int i = n_ops - 2; i >= 0; --i) {
            if (rot_row[i] < 0 || diag_gate(bwd[i])) continue;
            const int q = bwd[i].targets[0];
            for (int j = i; j + 1 < n_ops && !gate_touches(bwd[j + 1], q); ++j) {
                std::swap(bwd[j], bwd[j + 1]);
                std::swap(rot_row[j], rot_row[j + 1]);
                std::swap(gen_of[j], gen_of[j + 1]);
                std::swap(extra[j], extra[j + 1]);
            }
        }
        for (int k = 0; k < n_ops; ++k)
            if (dblock_rot(k)) extra[k] = 0;
    }
    // forward: phi = U_L .. U_1 psi in tile runs (at these sizes a fused
    // sweep is shorter than building its block matrices on the host)
    qc_exec_stats_t st{};
    if ((rc = tiled_execute(psi, n_ops, fwd.data(), st, stream))) return rc;
    // energy, then lam = H phi
    if ((rc = qc_expect_pauli(psi, n_terms, paulis, coeff, 0, energy_dev, stream))) return rc;
    if ((rc = pauli_apply(psi, lam, terms, c, hs))) return rc;
    // backward: tile runs over (phi, lam); each rotation's Im <lam|G|phi> is
    // taken in LDS right before its inverse is applied
    double *partial = c->work;
    double *g_op = c->work + size_t(n_rot) * cols;
    std::vector<TileRun> runs;
    form_runs(n, mb, n_ops, bwd.data(), extra.data(), runs);
    std::vector<qcx::TileOp> tops;
    std::vector<int32_t> slot_row;
    const bool rt = rt_bwd;
    const int max_slots = rt ? qcx::kRtAdjSlots : qcx::kAdjointMaxSlots;
    std::vector<unsigned char> rbuf;
    // the backward launches are planned first and their programs staged in
    // one copy (the forward runs, the energy and lambda are on the GPU
    // meanwhile), then launched back to back
    struct BwdLaunch {
        bool rt;
        qcx::RtArgs ra;
        qcx::TileArgs ta;
        size_t prog, tab_off, slots;
        int n_slots;
    };
    std::vector<BwdLaunch> launches;
    std::vector<unsigned char> blob;
    auto append = [&](const void *p, size_t bytes) {
        blob.resize((blob.size() + 255) & ~size_t(255));
        const size_t off = blob.size();
        const unsigned char *b = static_cast<const unsigned char *>(p);
        blob.insert(blob.end(), b, b + bytes);
        return off;
    };
    auto flush = [&](uint64_t P) -> int {
        if (tops.empty()) return QC_OK;
        merge_grad_pairs(tops);
        BwdLaunch L{};
        L.n_slots = int(slot_row.size());
        if (rt) {   // register tiles: both vectors in registers
            rt_program(n, mb, psi.dtype, P, tops, L.ra, rbuf, L.tab_off, true);
            bool has_dblock = false;
            for (const qcx::TileOp &o : tops) has_dblock = has_dblock || o.kind == qcx::TILE_DGRAD;
            if (L.ra.lds_tab_bytes > kRtLdsTabMax && has_dblock)   // the LDS engine has no such op
                return fail(QC_ERR_UNSUPPORTED, "backward program exceeds the register-tile table budget");
            L.rt = L.ra.lds_tab_bytes <= kRtLdsTabMax;
        }
        if (L.rt) {
            L.prog = append(rbuf.data(), rbuf.size());
        } else {
            L.ta = tile_args(n, mb, P, int(tops.size()));
            L.prog = append(tops.data(), tops.size() * sizeof(qcx::TileOp));
        }
        L.slots = slot_row.empty() ? 0 : append(slot_row.data(), slot_row.size() * sizeof(int32_t));
        launches.push_back(L);
        tops.clear();
        slot_row.clear();
        return QC_OK;
    };
    // the pending block of diagonal rotations and the blocks in the current
    // launch (16 lane tables at most)
    DiagBlock dblk;
    int dblocks = 0;
    auto emit_dblk = [&](TileOpBuilder &B, uint64_t P) {
        if (dblk.empty()) return;
        const qcx::TileOp op = dblk.op(P, &slot_row);
        // one-qubit gates the builder still holds on the block's tile bits
        // go out first
        B.add_op(op, uint32_t(op.b1));
        dblk.clear();
        ++dblocks;
    };
    for (const TileRun &r : runs) {
        if (r.P == 0) return fail(QC_ERR_UNSUPPORTED, "adjoint op cannot be tiled");
        TileOpBuilder B(n, r.P, tops);
        B.kron_max = 1;   // k_adjoint_tiles is compiled without TILE_KRON
        B.fans = false;   // nor with the fan ops
        B.xperms = false;   // nor with the X permutations
        dblocks = 0;
        for (int j : r.gates) {
            if (dblock_rot(j)) {
                const int pos = bitpos(n, bwd[j].targets[0]);
                if (!dblk.fits(pos, r.P)) emit_dblk(B, r.P);
                if (int(slot_row.size() + dblk.size()) + 1 > max_slots || (dblk.empty() && dblocks == 16)) {
                    emit_dblk(B, r.P);
                    B.finish();
                    if ((rc = flush(r.P))) return rc;
                    dblocks = 0;
                }
                dblk.add(pos, rot_row[j], bwd[j].matrix);
                continue;
            }
            // any other op after the block (diagonal gates without a
            // parameter commute with it and may stay behind)
            if (rot_row[j] >= 0 || !diag_gate(bwd[j])) emit_dblk(B, r.P);
            if (rot_row[j] >= 0) {
                if (int(slot_row.size()) == max_slots) {
                    B.finish();
                    if ((rc = flush(r.P))) return rc;
                }
                // the reduction and the inverse rotation share one pass
                qcx::TileOp gop{};
                const double *mu = bwd[j].matrix;
                const bool real = mu[1] == 0 && mu[3] == 0 && mu[5] == 0 && mu[7] == 0;
                const bool diag = mu[2] == 0 && mu[3] == 0 && mu[4] == 0 && mu[5] == 0;
                gop.kind = real ? qcx::TILE_GRAD_APPLY_REAL
                                : diag ? qcx::TILE_GRAD_APPLY_DIAG : qcx::TILE_GRAD_APPLY;
                gop.b0 = B.cidx(bitpos(n, bwd[j].targets[0]));
                gop.b1 = gen_of[j];
                gop.pad = int32_t(slot_row.size());
                for (int i = 0; i < 8; ++i) gop.u[i] = mu[i];
                slot_row.push_back(rot_row[j]);
                B.add_op(gop, 1u << gop.b0);
                continue;
            }
            B.add_gate(bwd[j]);
        }
        emit_dblk(B, r.P);
        B.finish();
        if ((rc = flush(r.P))) return rc;
    }
    if (!launches.empty()) {
        void *bdev = nullptr;
        if ((rc = stage(c, blob.data(), blob.size(), hs, &bdev))) return rc;
        const unsigned char *base = static_cast<const unsigned char *>(bdev);
        for (const BwdLaunch &L : launches) {
            const int32_t *sl = L.n_slots ? reinterpret_cast<const int32_t *>(base + L.slots) : nullptr;
            hipError_t e2;
            if (L.rt)
                e2 = qcx::launch_rt_adjoint(psi.amp, lam.amp, psi.dtype, L.ra,
                                            reinterpret_cast<const qcx::RtOp *>(base + L.prog),
                                            base + L.prog + L.tab_off, sl, L.n_slots, partial, cols, hs);
            else
                e2 = qcx::launch_adjoint_tiles(psi.amp, lam.amp, psi.dtype, L.ta,
                                               reinterpret_cast<const qcx::TileOp *>(base + L.prog), sl,
                                               L.n_slots, partial, cols, hs);
            if (e2 != hipSuccess) return hip_fail(e2, L.rt ? "rt_adjoint" : "adjoint_tiles");
        }
    }
    // grad[p] = sum of the rotation rows that use parameter p
    std::vector<int> csr(size_t(n_params) + 1 + size_t(n_rot), 0);
    {
        std::vector<std::vector<int>> users(n_params);
        int r = 0;
        for (int k = 0; k < n_ops; ++k)
            if (is_rotation(ops[k].kind)) users[ops[k].param].push_back(r++);
        int at = 0;
        for (int p = 0; p < n_params; ++p) {
            csr[p] = at;
            for (int u : users[p]) csr[size_t(n_params) + 1 + at++] = u;
        }
        csr[n_params] = at;
    }
    void *cdev = nullptr;
    if ((rc = stage(c, csr.data(), csr.size() * sizeof(int), hs, &cdev))) return rc;
    const int *ptr = static_cast<const int *>(cdev);
    e = qcx::launch_grad_finalize(partial, n_rot, int(cols), g_op, ptr, ptr + n_params + 1,
                                  n_params, grad_dev, hs);
    return e == hipSuccess ? QC_OK : hip_fail(e, "grad_finalize");
}

// ======================================================================
// batched persistent launch: host planner
// ======================================================================

struct qc_batch {
    int dtype = 0, keep = 0, n_circ = 0, grid = 0, n_groups = 0, G = 0, mmax = 0, n_phases = 0;
    size_t lds_bytes = 0;
    uint64_t arena_elems = 0;
    std::vector<qcx::BatchCircuit> circ_h;
    qcx::BatchCircuit *circ = nullptr;
    qcx::BatchPhase *phases = nullptr;
    qcx::TileOp *ops = nullptr;
    qcx::BatchTerm *terms = nullptr;
    qcx::BatchJob *jobs = nullptr;
    int32_t *group_jobs = nullptr;
    double *partial = nullptr;
    unsigned *barrier = nullptr;
};

namespace {

struct HostTerm {
    uint64_t x, z;
    int ph;
    double c;
};

uint32_t compress_mask(uint64_t mask, uint64_t P) {
    uint32_t out = 0;
    int j = 0;
    for (int p = 0; p < 64; ++p)
        if ((P >> p) & 1) {
            if ((mask >> p) & 1) out |= 1u << j;
            ++j;
        }
    return out;
}

qcx::BatchTerm make_term(const HostTerm &t, uint64_t P) {
    qcx::BatchTerm b{};
    b.xc = compress_mask(t.x, P);
    b.zc = compress_mask(t.z & P, P);
    b.z_hi = t.z & ~P;
    b.c = t.c;
    b.ph = t.ph;
    b.xtop = b.xc ? 31 - __builtin_clz(b.xc) : -1;
    return b;
}

qcx::BatchPhase make_phase(int n, int m, uint64_t P, int op_begin, int op_count, int flags) {
    qcx::BatchPhase ph{};
    ph.n_tiles = uint64_t(1) << (n - m);
    ph.m = m;
    ph.op_begin = op_begin;
    ph.op_count = op_count;
    ph.flags = flags;
    for (int p = 0, j = 0; p < n; ++p)
        if ((P >> p) & 1) ph.pos[j++] = uint32_t(p);
    return ph;
}

// Phases of one circuit: gate runs (as in the tiled executor), then the
// energy terms on the tile bits that hold their X/Y factors.
int plan_circuit(const qc_circuit_t &c, int mmax, bool keep, std::vector<qcx::BatchPhase> &phases,
                 std::vector<qcx::TileOp> &ops, std::vector<qcx::BatchTerm> &terms, double &cost) {
    const int n = c.n;
    const int m = std::min(n, mmax);
    const int low = std::min(m, 5);
    const uint64_t low_mask = (uint64_t(1) << low) - 1;
    const bool large = n > m;
    const int store = (large || keep) ? qcx::BATCH_STORE : 0;
    for (int i = 0; i < c.n_gates; ++i) {
        int rc = check_gate(n, c.gates[i]);
        if (rc) return rc;
        if (c.gates[i].n_targets > 2)
            return fail(QC_ERR_UNSUPPORTED, "batched circuits take gates with at most 2 targets");
    }
    std::vector<HostTerm> ht(c.n_terms);
    for (int t = 0; t < c.n_terms; ++t) {
        HostTerm h{};
        int ny = 0;
        for (int q = 0; q < n; ++q) {
            const uint64_t b = uint64_t(1) << bitpos(n, q);
            switch (c.paulis[size_t(t) * n + q]) {
            case 'I': break;
            case 'X': h.x |= b; break;
            case 'Y': h.x |= b; h.z |= b; ++ny; break;
            case 'Z': h.z |= b; break;
            default: return fail(QC_ERR_ARG, "Pauli character not in {I,X,Y,Z}");
            }
        }
        h.ph = ny & 3;
        h.c = c.coeff[t];
        ht[t] = h;
    }
    cost = 0.0;
    std::vector<int> pending(c.n_gates);
    for (int i = 0; i < c.n_gates; ++i) pending[i] = i;
    uint64_t last_P = 0;
    bool first = true;
    do {
        uint64_t P = low_mask, blocked = 0;
        std::vector<int> run, rest;
        for (int idx : pending) {
            const TileClass tc = tile_class(n, c.gates[idx]);
            if (!(tc.touch & blocked) && __builtin_popcountll(P | tc.tbits) <= m) {
                P |= tc.tbits;
                run.push_back(idx);
            } else {
                blocked |= tc.touch;
                rest.push_back(idx);
            }
        }
        for (int p = 0; __builtin_popcountll(P) < m && p < n; ++p) P |= uint64_t(1) << p;
        const int op_begin = int(ops.size());
        tile_ops_for(n, c.gates, run, P, ops);
        const int nops = int(ops.size()) - op_begin;
        phases.push_back(make_phase(n, m, P, op_begin, nops, (first ? qcx::BATCH_INIT : 0) | store));
        cost += double(uint64_t(1) << n) * (nops + 2);
        first = false;
        last_P = P;
        pending.swap(rest);
    } while (!pending.empty());
    // energy terms: on the last gate phase when their X/Y bits are tile bits,
    // else on read-only phases whose tile bits cover them
    std::vector<int> left;
    {
        qcx::BatchPhase &ph = phases.back();
        ph.term_begin = int(terms.size());
        for (int t = 0; t < c.n_terms; ++t) {
            if ((ht[t].x & ~last_P) == 0) terms.push_back(make_term(ht[t], last_P));
            else left.push_back(t);
        }
        ph.term_count = int(terms.size()) - ph.term_begin;
        cost += double(uint64_t(1) << n) * ph.term_count;
    }
    while (!left.empty()) {
        uint64_t P = low_mask;
        std::vector<int> take, rest;
        for (int t : left) {
            if (__builtin_popcountll(P | ht[t].x) <= m) {
                P |= ht[t].x;
                take.push_back(t);
            } else {
                rest.push_back(t);
            }
        }
        if (take.empty()) return fail(QC_ERR_UNSUPPORTED, "Pauli term wider than one tile");
        for (int p = 0; __builtin_popcountll(P) < m && p < n; ++p) P |= uint64_t(1) << p;
        qcx::BatchPhase ph = make_phase(n, m, P, int(ops.size()), 0, 0);
        ph.term_begin = int(terms.size());
        for (int t : take) terms.push_back(make_term(ht[t], P));
        ph.term_count = int(take.size());
        phases.push_back(ph);
        cost += double(uint64_t(1) << n) * (ph.term_count + 1);
        left.swap(rest);
    }
    return QC_OK;
}

template <typename T>
int upload(const std::vector<T> &v, T **dev) {
    const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (hipMalloc(dev, bytes) != hipSuccess) return fail(QC_ERR_NOMEM, "batch program allocation");
    if (!v.empty()) {
        hipError_t e = hipMemcpy(*dev, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    return QC_OK;
}

}  // namespace

extern "C" {

int qc_batch_destroy(qc_batch_t *b) {
    if (!b) return QC_OK;
    (void)hipFree(b->circ);
    (void)hipFree(b->phases);
    (void)hipFree(b->ops);
    (void)hipFree(b->terms);
    (void)hipFree(b->jobs);
    (void)hipFree(b->group_jobs);
    (void)hipFree(b->partial);
    (void)hipFree(b->barrier);
    delete b;
    return QC_OK;
}

int qc_batch_create(int n_circuits, const qc_circuit_t *circuits, int dtype, int keep_states,
                    qc_batch_t **out) {
    if (!out) return fail(QC_ERR_ARG, "output handle pointer is NULL");
    *out = nullptr;
    if (n_circuits < 1 || !circuits) return fail(QC_ERR_ARG, "empty batch");
    if (dtype != QC_C64 && dtype != QC_C128) return fail(QC_ERR_DTYPE, "unknown dtype");
    const int mmax = dtype == QC_C64 ? 13 : 12;
    const int G = qcx::kBatchGroup;
    std::vector<qcx::BatchCircuit> circ(n_circuits);
    std::vector<qcx::BatchPhase> phases;
    std::vector<qcx::TileOp> ops;
    std::vector<qcx::BatchTerm> terms;
    std::vector<double> cost(n_circuits);
    uint64_t arena = 0;
    for (int i = 0; i < n_circuits; ++i) {
        const qc_circuit_t &c = circuits[i];
        if (c.n < 1 || c.n > 30) return fail(QC_ERR_ARG, "batched circuit size out of range");
        if (c.n_gates < 0 || (c.n_gates > 0 && !c.gates)) return fail(QC_ERR_ARG, "gate list is NULL");
        if (c.n_terms < 1 || !c.paulis || !c.coeff) return fail(QC_ERR_ARG, "Hamiltonian is empty");
        const int begin = int(phases.size());
        int rc = plan_circuit(c, mmax, keep_states != 0, phases, ops, terms, cost[i]);
        if (rc) return rc;
        circ[i].n = c.n;
        circ[i].phase_begin = begin;
        circ[i].phase_count = int(phases.size()) - begin;
        circ[i].large = c.n > mmax;
        circ[i].arena_off = arena;
        if (circ[i].large || keep_states) arena += uint64_t(1) << c.n;
    }
    // persistent grid: resident workgroups only, in whole groups on 8 XCDs
    const size_t elem = dtype == QC_C64 ? 8 : 16;
    const size_t lds = (size_t(1) << mmax) * elem;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return fail(QC_ERR_HIP, "cannot query the compute-unit count");
    const int per_cu = std::min(qcx::batch_resident_blocks(dtype, lds), 2);
    if (per_cu < 1) return fail(QC_ERR_UNSUPPORTED, "batch kernel cannot be resident");
    const int grid = (per_cu * cus) / (8 * G) * (8 * G);
    if (grid < 8 * G) return fail(QC_ERR_UNSUPPORTED, "device too small for the batch grid");
    const int n_groups = grid / G;
    // jobs: bundles of G small circuits, one job per large circuit
    struct Job { qcx::BatchJob j; double cost; };
    std::vector<Job> jobs;
    std::vector<int> small, large;
    for (int i = 0; i < n_circuits; ++i) (circ[i].large ? large : small).push_back(i);
    std::stable_sort(small.begin(), small.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (size_t s0 = 0; s0 < small.size(); s0 += G) {
        Job J{};
        J.j.kind = 0;
        for (int r = 0; r < G; ++r) J.j.circ[r] = -1;
        for (int r = 0; r < G && s0 + r < small.size(); ++r) {
            J.j.circ[r] = small[s0 + r];
            J.cost = std::max(J.cost, cost[small[s0 + r]]);
        }
        jobs.push_back(J);
    }
    for (int i : large) {
        Job J{};
        J.j.kind = 1;
        for (int r = 0; r < G; ++r) J.j.circ[r] = -1;
        J.j.circ[0] = i;
        J.cost = cost[i] / G;
        jobs.push_back(J);
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job &a, const Job &b) { return a.cost > b.cost; });
    std::vector<double> load(n_groups, 0.0);
    std::vector<std::vector<qcx::BatchJob>> per_group(n_groups);
    for (const Job &J : jobs) {
        const int g = int(std::min_element(load.begin(), load.end()) - load.begin());
        load[g] += J.cost;
        per_group[g].push_back(J.j);
    }
    std::vector<qcx::BatchJob> job_list;
    std::vector<int32_t> group_jobs(n_groups + 1, 0);
    for (int g = 0; g < n_groups; ++g) {
        group_jobs[g] = int32_t(job_list.size());
        for (auto &j : per_group[g]) job_list.push_back(j);
    }
    group_jobs[n_groups] = int32_t(job_list.size());

    qc_batch_t *b = new qc_batch_t();
    b->dtype = dtype;
    b->keep = keep_states != 0;
    b->n_circ = n_circuits;
    b->grid = grid;
    b->n_groups = n_groups;
    b->G = G;
    b->mmax = mmax;
    b->lds_bytes = lds;
    b->arena_elems = arena;
    b->n_phases = int(phases.size());
    b->circ_h = circ;
    int rc;
    std::vector<double> zeros(size_t(n_circuits) * G, 0.0);
    std::vector<unsigned> zbar(n_groups + 1, 0u);
    if ((rc = upload(circ, &b->circ)) || (rc = upload(phases, &b->phases)) ||
        (rc = upload(ops, &b->ops)) || (rc = upload(terms, &b->terms)) ||
        (rc = upload(job_list, &b->jobs)) || (rc = upload(group_jobs, &b->group_jobs)) ||
        (rc = upload(zeros, &b->partial)) || (rc = upload(zbar, &b->barrier))) {
        qc_batch_destroy(b);
        return rc;
    }
    *out = b;
    return QC_OK;
}

int qc_batch_info(const qc_batch_t *b, uint64_t *arena_bytes, int *grid, int *phases) {
    if (!b) return fail(QC_ERR_ARG, "batch handle is NULL");
    if (arena_bytes) *arena_bytes = b->arena_elems * (b->dtype == QC_C64 ? 8 : 16);
    if (grid) *grid = b->grid;
    if (phases) *phases = b->n_phases;
    return QC_OK;
}

int qc_run_batch(qc_batch_t *b, void *arena_dev, double *energy_dev, void *stream) {
    if (!b) return fail(QC_ERR_ARG, "batch handle is NULL");
    if (!energy_dev) return fail(QC_ERR_ARG, "energy pointer is NULL");
    if (b->arena_elems && !arena_dev) return fail(QC_ERR_ARG, "batch needs an arena");
    qcx::BatchArgs a{};
    a.circ = b->circ;
    a.phases = b->phases;
    a.ops = b->ops;
    a.terms = b->terms;
    a.jobs = b->jobs;
    a.group_jobs = b->group_jobs;
    a.arena = arena_dev;
    a.energy = energy_dev;
    a.partial = b->partial;
    a.barrier = b->barrier;
    a.error = b->barrier + b->n_groups;
    a.n_groups = b->n_groups;
    a.G = b->G;
    hipError_t e = qcx::launch_batch(a, b->dtype, unsigned(b->grid), b->lds_bytes, (hipStream_t)stream);
    return e == hipSuccess ? QC_OK : hip_fail(e, "run_batch");
}

int qc_batch_state(const qc_batch_t *b, void *arena_dev, int i, qc_state_t *view) {
    if (!b || !view || !arena_dev) return fail(QC_ERR_ARG, "NULL argument");
    if (i < 0 || i >= b->n_circ) return fail(QC_ERR_ARG, "circuit index out of range");
    const qcx::BatchCircuit &c = b->circ_h[i];
    if (!c.large && !b->keep) return fail(QC_ERR_ARG, "this circuit's state is not kept");
    view->amp = static_cast<char *>(arena_dev) + c.arena_off * (b->dtype == QC_C64 ? 8 : 16);
    view->n = c.n;
    view->dtype = b->dtype;
    return QC_OK;
}

int qc_batch_status(qc_batch_t *b, int *flags) {
    if (!b || !flags) return fail(QC_ERR_ARG, "NULL argument");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    unsigned v = 0;
    e = hipMemcpy(&v, b->barrier + b->n_groups, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    *flags = int(v);
    return QC_OK;
}

int qc_autotune(qc_state_t scratch, int n_gates, const qc_gate_t *gates, int reps,
                qc_tune_entry_t *entries, int max_entries, int *n_entries, void *stream) {
    int rc = check_state(scratch);
    if (rc) return rc;
    if (!n_entries || (max_entries > 0 && !entries)) return fail(QC_ERR_ARG, "NULL argument");
    if (reps < 1 || reps > 100) return fail(QC_ERR_ARG, "reps must be 1..100");
    if (n_gates < 1 || !gates) return fail(QC_ERR_ARG, "empty gate list");
    for (int i = 0; i < n_gates; ++i)
        if ((rc = check_gate(scratch.n, gates[i]))) return rc;
    struct Cand { int mode, k, wg, tbits, tile_bits; };
    std::vector<Cand> cands{{QC_EXEC_UNFUSED, 0, 0, 0, 0}};
    {
        const int top = scratch.dtype == QC_C64 ? 13 : 12;
        for (int m = top; m >= top - 2; --m)
            if (m <= scratch.n || m == top) cands.push_back({QC_EXEC_TILED, 0, 0, 0, m});
    }
    for (int k = 2; k <= std::min(QC_MAX_FUSED, scratch.n); ++k) {
        if (scratch.dtype == QC_C64 && k == 5 && scratch.n >= 12) {
            for (int wg = 2; wg <= 5; ++wg) cands.push_back({QC_EXEC_FUSED, 5, wg, 12, 0});
            // 64 KiB workgroups: the knob's tile slots give 1 or 2 per CU
            if (scratch.n >= 13)
                for (int wg = 2; wg <= 4; wg += 2) cands.push_back({QC_EXEC_FUSED, 5, wg, 13, 0});
        } else {
            cands.push_back({QC_EXEC_FUSED, k, 0, 0, 0});
        }
    }
    const int saved_wg = g_knob_mfma.load();
    const int saved_tbits = g_knob_tbits.load();
    const int saved_tile_bits = g_knob_tile_bits.load();
    const hipStream_t hs = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(QC_ERR_HIP, "hipEventCreate");
    std::vector<qc_tune_entry_t> out;
    for (const Cand &c : cands) {
        if (c.wg) g_knob_mfma.store(c.wg);
        if (c.tbits) g_knob_tbits.store(c.tbits);
        g_knob_tile_bits.store(c.tile_bits ? c.tile_bits : saved_tile_bits);
        qc_exec_stats_t st{};
        std::vector<float> t;
        for (int r = 0; r <= reps && rc == QC_OK; ++r) {
            if ((rc = qc_state_init(scratch, 0, stream))) break;
            (void)hipEventRecord(e0, hs);
            rc = qc_apply_circuit(scratch, n_gates, gates, c.mode, c.k ? c.k : 5, &st, stream);
            (void)hipEventRecord(e1, hs);
            if (rc) break;
            if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(QC_ERR_HIP, "hipEventSynchronize"); break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t.push_back(ms);   // the first run is the warm-up
        }
        if (rc) break;
        std::sort(t.begin(), t.end());
        qc_tune_entry_t e{};
        e.mode = c.mode;
        e.fuse_k = c.k;
        e.mfma_wg_per_cu = c.wg ? c.wg : saved_wg;
        e.mfma_tile_bits = c.tbits ? c.tbits : saved_tbits;
        e.tile_bits = c.tile_bits ? c.tile_bits : saved_tile_bits;
        e.sweeps = int32_t(st.sweeps);
        e.ms = t[t.size() / 2];
        out.push_back(e);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_knob_mfma.store(saved_wg);
    g_knob_tbits.store(saved_tbits);
    g_knob_tile_bits.store(saved_tile_bits);
    if (rc) return rc;
    std::stable_sort(out.begin(), out.end(),
                     [](const qc_tune_entry_t &a, const qc_tune_entry_t &b) { return a.ms < b.ms; });
    if (!out.empty()) {
        g_knob_mfma.store(out[0].mfma_wg_per_cu);
        g_knob_tbits.store(out[0].mfma_tile_bits);
        g_knob_tile_bits.store(out[0].tile_bits);
    }
    const int n = std::min<int>(int(out.size()), max_entries);
    for (int i = 0; i < n; ++i) entries[i] = out[i];
    *n_entries = n;
    return QC_OK;
}

}  // extern "C"
