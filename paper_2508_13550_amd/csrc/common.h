// Internal declarations of the CSFMM library for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/csfmm.h"

namespace csfmm {

// Deepest quadtree level; a level-l cell is a square of side (pi/2)/2^l in
// the local angles of its face.  Morton keys hold 3 face bits and 2 bits per
// level.
constexpr int kMaxLevel = 20;
constexpr int kMaxDegree = 16;
constexpr int kAncStride = kMaxLevel + 2;

constexpr double kPi = 3.14159265358979323846;
constexpr double kPi4 = 0.78539816339744830962;  // pi/4
constexpr double kPi2 = 1.57079632679489661923;  // pi/2

// Error reporting (thread-local message behind csfmm_last_error).
void set_error(const char* fmt, ...);
void clear_error();

#define CSFMM_HIP_TRY(call)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            ::csfmm::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),       \
                               __FILE__, __LINE__);                                          \
            return (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)             \
                       ? CSFMM_E_OOM                                                         \
                       : CSFMM_E_HIP;                                                        \
        }                                                                                    \
    } while (0)

#define CSFMM_LAUNCH_CHECK()                                                                  \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess) {                                                               \
            ::csfmm::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_),    \
                               __FILE__, __LINE__);                                           \
            return CSFMM_E_HIP;                                                               \
        }                                                                                     \
    } while (0)

// Device allocation owned by a plan; freed in the plan's destructor.
struct DevArena {
    std::vector<void*> ptrs;
    int64_t bytes = 0;
    template <class T>
    int alloc(T** p, int64_t n) {
        *p = nullptr;
        if (n <= 0) n = 1;
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(T) * size_t(n));
        if (e != hipSuccess) {
            set_error("hipMalloc of %lld bytes failed: %s", (long long)(sizeof(T) * n),
                      hipGetErrorString(e));
            (void)hipGetLastError();
            return CSFMM_E_OOM;
        }
        ptrs.push_back(q);
        bytes += int64_t(sizeof(T)) * n;
        *p = static_cast<T*>(q);
        return CSFMM_OK;
    }
    void release() {
        for (void* q : ptrs) (void)hipFree(q);
        ptrs.clear();
        bytes = 0;
    }
};

// Several arena arrays in one hipMalloc: add() records where each array's
// pointer goes and its size, commit() allocates the sum (each array starting
// on a 256-byte boundary) and hands out the pointers.  `bytes` grows by what
// is allocated, padding included.
struct ArenaGroup {
    struct Item {
        void** p;
        size_t b;
    };
    std::vector<Item> items;
    template <class T>
    void add(T** p, int64_t n) {
        *p = nullptr;
        items.push_back(Item{(void**)p, sizeof(T) * size_t(n > 0 ? n : 1)});
    }
    int commit(DevArena& A) {
        size_t total = 0;
        for (const Item& it : items) total += (it.b + 255) / 256 * 256;
        char* base = nullptr;
        int rc = A.alloc(&base, int64_t(total));
        if (rc != CSFMM_OK) return rc;
        size_t o = 0;
        for (const Item& it : items) {
            *it.p = base + o;
            o += (it.b + 255) / 256 * 256;
        }
        items.clear();
        return CSFMM_OK;
    }
};

// Stream-ordered scratch for one build step: requests are carved (256-byte
// aligned) from chunks taken with hipMallocAsync on the stream, and every
// chunk goes back to the stream's pool when the object dies, after the work
// queued before that point.  A request larger than half a chunk gets a chunk
// of its own, so the open chunk keeps serving small requests.
struct Scratch {
    struct Chunk {
        char* base;
        size_t cap, used;
    };
    static constexpr size_t kChunk = size_t(8) << 20;
    hipStream_t s;
    std::vector<Chunk> chunks;  // the open chunk is the last one
    explicit Scratch(hipStream_t st) : s(st) {}
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
    int take(size_t cap, char** q) {
        void* v = nullptr;
        hipError_t e = hipMallocAsync(&v, cap, s);
        if (e != hipSuccess) {
            set_error("hipMallocAsync of %lld bytes failed: %s", (long long)cap,
                      hipGetErrorString(e));
            (void)hipGetLastError();
            return CSFMM_E_OOM;
        }
        *q = static_cast<char*>(v);
        return CSFMM_OK;
    }
    template <class T>
    int get(T** p, int64_t n) {
        *p = nullptr;
        const size_t b = (sizeof(T) * size_t(n > 0 ? n : 1) + 255) / 256 * 256;
        char* q = nullptr;
        if (b > kChunk / 2) {  // a full chunk of its own, placed before the open one
            int rc = take(b, &q);
            if (rc != CSFMM_OK) return rc;
            chunks.insert(chunks.empty() ? chunks.end() : chunks.end() - 1, Chunk{q, b, b});
            *p = reinterpret_cast<T*>(q);
            return CSFMM_OK;
        }
        if (chunks.empty() || chunks.back().cap - chunks.back().used < b) {
            int rc = take(kChunk, &q);
            if (rc != CSFMM_OK) return rc;
            chunks.push_back(Chunk{q, kChunk, 0});
        }
        Chunk& c = chunks.back();
        *p = reinterpret_cast<T*>(c.base + c.used);
        c.used += b;
        return CSFMM_OK;
    }
    ~Scratch() {
        for (const Chunk& c : chunks) (void)hipFreeAsync(c.base, s);
    }
};

// One quadtree forest over a point set, cells in breadth-first order.
struct Tree {
    int64_t n = 0;
    int32_t ncells = 0, nleaves = 0, depth = 0;
    int32_t max_leaf = 0;  // largest number of points in a leaf
    std::vector<int32_t> level_begin;   // host: first cell of each level, + end
    std::vector<int32_t> parents_begin; // host: first entry of each level in `parents`
    // sorted points (SoA) and their caller indices
    double *x = nullptr, *y = nullptr, *z = nullptr;
    double *u = nullptr, *v = nullptr;  // local coordinates in their leaf, [-1,1]
    int32_t* perm = nullptr;            // sorted position -> caller index
    // cells
    int32_t *level = nullptr, *face = nullptr, *ci = nullptr, *cj = nullptr;
    int32_t *begin = nullptr, *count = nullptr, *child0 = nullptr;
    int32_t* parent = nullptr;  // -1 for the six roots
    // per leaf (in `leaves` order): [0] = number of cells on the path from the
    // root to the leaf, then those cells, root first; stride kAncStride
    int32_t* leaf_anc = nullptr;
    // [ncells][4] box of each cell: xi_mid, eta_mid, half_xi, half_eta (the
    // cell itself, or its points' bounding rectangle with shrinking)
    double* box = nullptr;
    // shrinking: [ncells][2][p+1][p+1] 1-D factors of the parent-to-child
    // operator (xi, eta): the parent's polynomial k at the child's node m
    double* ops = nullptr;
    double* center = nullptr;  // [ncells][3]
    double* radius = nullptr;  // [ncells]
    // [ncells] leaves: a lower bound on the geodesic distance of the leaf's
    // points to its edges; 0 for the other cells
    double* gap = nullptr;
    double* prox = nullptr;    // [ncells][3][KS] proxy coordinates (SoA per cell)
    int32_t* leaves = nullptr;  // [nleaves] leaf cell ids (Morton order)
    int32_t* parents = nullptr; // non-leaf cells grouped by level (host offsets above)
};

// Interaction lists in CSR form by target cell.
enum ListKind { kPP = 0, kPC = 1, kCP = 2, kCC = 3 };

// Same-set plans: the PP entries of distinct leaves split by kernel symmetry.
// A pair of leaves {T, S} whose PP entry holds both ways ((T, S) and (S, T))
// is evaluated once, by its owner (pair_owner), for both directions: the
// owner's own targets take the row sums, the partner's targets the column
// sums, which go to a slot of the workspace and are added afterwards in list
// order.  Entries that hold one way only stay one-directional.
struct SymPP {
    bool on = false;
    int64_t n_own = 0, n_one = 0;  // owned pairs (as many are received), one-way entries
    int32_t *own_off = nullptr, *own_src = nullptr;    // [ncells+1], [n_own]; slot = index
    int32_t *recv_off = nullptr, *recv_slot = nullptr; // [ncells+1], [n_own]
    int32_t *one_off = nullptr, *one_src = nullptr;    // [ncells+1], [n_one]
};

struct Lists {
    int64_t cnt[4] = {0, 0, 0, 0};
    int32_t* off[4] = {nullptr, nullptr, nullptr, nullptr};  // [ncells_t + 1]
    int32_t* src[4] = {nullptr, nullptr, nullptr, nullptr};  // [cnt]
    int32_t* novl = nullptr;  // [ncells_t] leading PP entries whose cells overlap the target
    int32_t* ncl = nullptr;   // [ncells_t] FP32 form: the close PP entries that follow them
    int64_t n_close = 0;      // sum of ncl
    int32_t* far_targets = nullptr;  // target cells with CP or CC entries
    int32_t n_far_targets = 0;
    int64_t evals[4] = {0, 0, 0, 0};
    SymPP sym;
};

// Device-resident description of one (plan, workspace) pair: every pointer and
// size an eval kernel needs about one request.
struct ReqView {
    // target tree
    const int32_t *t_begin, *t_count, *t_child0, *t_leaf_anc, *t_leaves, *t_parents, *t_perm;
    const double *t_x, *t_y, *t_z, *t_u, *t_v, *t_center, *t_prox;
    // source tree
    const int32_t *s_begin, *s_count, *s_child0, *s_leaves, *s_parents, *s_perm;
    const double *s_x, *s_y, *s_z, *s_u, *s_v, *s_prox;
    // interaction lists
    const int32_t* off[4];
    const int32_t* src[4];
    const int32_t *novl, *ncl, *far_targets;
    // fixed operators, and the per-cell factors of shrunk trees (else NULL)
    const double *bm2m, *lag1d;
    const double *t_ops, *s_ops;
    // workspace
    double *ws, *wbar, *psi, *phinear, *phipc;
    int64_t nt, ns, psi_stride;
    int32_t p, K, KS, nb1;
    int32_t nleaves_t, nleaves_s;
    // symmetric PP split (SymPP) and its column-sum slots [n_own][kWaveLeaf]
    // (float in the FP32 form, double in FP64)
    const int32_t *own_off, *own_src, *recv_off, *recv_slot, *one_off, *one_src;
    void* sym_col;
};

// Target leaves of at most this many points take the one-wave-per-leaf path of
// the near-field tile kernel.
constexpr int kWaveLeaf = 64;

// Kernel argument of every eval launch: up to kMaxBatch requests; block b of
// the grid belongs to request r with prefix[r] <= b < prefix[r+1].
constexpr int kMaxBatch = 32;
struct Batch {
    int32_t n;
    const ReqView* v[kMaxBatch];
    const double* w[kMaxBatch];     // caller weights (caller order)
    double* out[kMaxBatch];         // caller outputs (caller order)
    int32_t vd[kMaxBatch];          // output components: 3 for Biot-Savart, else 1
    int32_t a0[kMaxBatch];          // M2M / L2L: first parent of the level in `parents`
    int32_t a1[kMaxBatch];          // M2M / L2L: number of parents at the level
    int32_t prefix[kMaxBatch + 1];
    int32_t prefix2[kMaxBatch + 1];  // tile launches: far-field blocks (prefix: near-field)
    int32_t mode;                    // tile launches: kTileNearPP or kTilePCFar
    int32_t leaf_wave[kMaxBatch];    // tile launches: request r's near field takes one wave per leaf
    int32_t wave_kernel;  // tile launches: near field only, all one wave per leaf: k_tile_wave
    int32_t sym[kMaxBatch];  // PP launches: request r takes the symmetric PP path (sym_path)
};

// Tile launch modes.  The PP near field needs no proxy weights, so it runs on
// a side stream while the upward pass runs; the PC near field (into its own
// buffer) and the CP + CC far field follow the upward pass.
enum TileMode { kTileNearPP = 1, kTilePCFar = 2 };

__device__ __forceinline__ void prefix_locate(const int32_t* prefix, int n, int blk, int& r,
                                              int& local) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= blk)
            lo = mid;
        else
            hi = mid - 1;
    }
    r = lo;
    local = blk - prefix[lo];
}

__device__ __forceinline__ void batch_locate(const Batch& b, int blk, int& r, int& local) {
    prefix_locate(b.prefix, b.n, blk, r, local);
}

__device__ __forceinline__ void batch_locate2(const Batch& b, int blk, int& r, int& local) {
    prefix_locate(b.prefix2, b.n, blk, r, local);
}

}  // namespace csfmm

struct csfmm_workspace_s;

struct csfmm_plan_s {
    int64_t nt = 0, ns = 0;
    bool same = false;
    int kernel = 1, p = 8, leaf = 64;
    double theta = 0.7;
    unsigned flags = 0;
    int K = 81, KS = 84;  // (p+1)^2 and its stride rounded up to 4
    csfmm::DevArena arena;
    csfmm::Tree tt, st_own;
    csfmm::Tree* st = nullptr;  // source tree (== &tt for a same-set plan)
    csfmm::Lists lists;
    // fixed interpolation operators (MFMA B operands)
    double* bm2m = nullptr;  // [4*KS][NB1], NB1 = roundup(KS,16)
    double* lag1d = nullptr; // [2][p+1][p+1] 1-D parent-at-child-node values (L2L factors)
    int nb1 = 0;
    // the plan's own workspace, used by csfmm_eval
    csfmm_workspace_s* ws0 = nullptr;
    int32_t* tc_status = nullptr;  // treecode stack-overflow flag (device)
    // optional per-stage timing with HIP events (ring of event sets)
    struct Timing {
        // P2M, M2M, PP (side stream), PC + CP + CC, L2L + L2P, and the span of
        // the two interaction launches (PP start to the eval stream's join)
        static constexpr int kStages = 6;
        static constexpr int kMain = 5;   // events on the eval stream per slot
        // + PP start/end on the side stream, + the join on the eval stream
        static constexpr int kEvents = kMain + 3;
        static constexpr int kSlots = 32;
        int on = 0;  // 0 off, 1 every stage, 2 the PP and the PC + far-field launches only
        std::vector<hipEvent_t> ev;  // [kSlots][kEvents]
        std::vector<int> pending;    // slot recorded and not yet read
        double sum_ms[kStages] = {0, 0, 0, 0, 0, 0};
        int64_t n = 0;
        int next = 0;
    } timing;
    ~csfmm_plan_s();
};

// Eval workspace bound to one plan: sorted weights, proxy weights, proxy
// potentials and near field, plus the device copy of the request view.
struct csfmm_workspace_s {
    csfmm_plan_s* plan = nullptr;
    csfmm::DevArena arena;
    double* ws = nullptr;       // [ns]
    double* wbar = nullptr;     // [ncells_s][KS]
    double* psi = nullptr;      // [3][ncells_t][KS]
    double* phinear = nullptr;  // [3][nt] PP near field
    double* phipc = nullptr;    // [3][nt] PC near field
    void* sym_col = nullptr;    // [n_own][kWaveLeaf] column sums of symmetric PP pairs
                                // (float in the FP32 form, double in FP64)
    csfmm::ReqView* dview = nullptr;  // device copy of dview_host
    csfmm::ReqView dview_host{};
    // side stream of the PP near field, with its fork and join events
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    ~csfmm_workspace_s();
};

namespace csfmm {
// Side streams are kept for reuse (creating one takes longer than building a
// small plan); a released stream has no work pending (destroying a workspace
// waits for the device first).
hipError_t acquire_side_stream(hipStream_t* s);
void release_side_stream(hipStream_t s);
}  // namespace csfmm

inline csfmm_workspace_s::~csfmm_workspace_s() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) csfmm::release_side_stream(side);
    arena.release();
}

inline csfmm_plan_s::~csfmm_plan_s() {
    for (hipEvent_t e : timing.ev) (void)hipEventDestroy(e);
    delete ws0;
    arena.release();
}

namespace csfmm {
int device_cus();  // compute units of the current device

// The near field of a target tree takes one wave per leaf when its leaves hold
// at most kWaveLeaf points and there are enough of them to give every SIMD a
// couple of waves; fewer leaves keep the block path, whose four waves share a
// leaf (measured on N = 6,144 in FP64: 0.48 ms per eval on the wave path,
// 0.20 on the block path).
inline bool leaf_wave_path(const csfmm::Tree& tt) {
    return tt.max_leaf <= kWaveLeaf && int64_t(tt.nleaves) >= 8 * int64_t(device_cus());
}

// The symmetric PP path: same-set plan (either form) whose target leaves take
// the one-wave-per-leaf path; an eval uses it for the scalar kernels
// (K(x, y) = K(y, x)), not for Biot-Savart.
inline bool sym_path_possible(const csfmm_plan_s* P) {
    return P->lists.sym.on && leaf_wave_path(P->tt) && P->lists.sym.n_own > 0;
}
// bytes of one column-sum value of the symmetric PP path
inline int64_t sym_value_bytes(const csfmm_plan_s* P) {
    return (P->flags & CSFMM_FP32_FORM) ? 4 : 8;
}
inline bool sym_path(const csfmm_plan_s* P, int kernel) {
    return sym_path_possible(P) && kernel != CSFMM_K_BIOT_SAVART;
}
}  // namespace csfmm

namespace csfmm {

// ---- building blocks (sort_scan.hip)
// exclusive scan of n int32 values; writes the total to *d_total (device)
// unless it is null; in == out is allowed
int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* d_total,
                       Scratch& S, hipStream_t s);
// exclusive scans of m arrays of n int32 values each (m <= 8), totals to
// d_totals[0..m) (device); one launch when n is small
int scan_exclusive_multi(const int32_t* const* in, int32_t* const* out, int m, int64_t n,
                         int32_t* d_totals, Scratch& S, hipStream_t s);
// stable LSD radix sort of (key, value) pairs on the low `bits` bits of the keys
int radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n, int bits, Scratch& S,
                   hipStream_t s);

// ---- plan (plan.hip)
int build_plan(csfmm_plan_s* P, const double* targets, const double* sources, hipStream_t s);

// ---- stage timing (eval.hip)
int timing_enable(csfmm_plan_s* P, int level);
int timing_collect(csfmm_plan_s* P);

// ---- eval (eval.hip)
int workspace_create(csfmm_plan_s* P, hipStream_t stream, csfmm_workspace_s** out);
struct EvalReq {
    csfmm_plan_s* plan;
    csfmm_workspace_s* ws;
    int kernel;
    const double* w;
    double* out;
};
// one packed eval of up to kMaxBatch requests (timing marks when n == 1)
int run_eval_batch(const EvalReq* reqs, int n, hipStream_t s);
int run_eval(csfmm_plan_s* P, int kernel, const double* weights, double* out, double* wbar_out,
             double* psi_out, double* near_out, hipStream_t s);
// upward pass on the plan's source tree, then the treecode (Algorithm 1)
int run_treecode(csfmm_plan_s* P, int kernel, const double* weights, double* out, hipStream_t s);

// ---- tile engine (tile.hip): b holds requests of one kernel and form
int launch_tile_batch(const Batch& b, int kernel, bool fp32, hipStream_t s);
int launch_sym_merge(const Batch& b, int kernel, bool fp32, hipStream_t s);

// Cubed sphere treecode (paper §7, Algorithm 1): one traversal of the source
// tree per target particle, FP64.
struct TcArgs {
    const double *tx, *ty, *tz;  // targets (sorted order of the target tree)
    const int32_t* tperm;        // sorted position -> caller index
    int64_t nt;
    const int32_t *sbegin, *scount, *schild0;  // source tree cells
    const double *scenter, *sradius;
    const double *sx, *sy, *sz, *sw;  // sorted source points and weights
    const double *sprox, *swbar;      // proxies [cell][3][KS], proxy weights [cell][KS]
    int K, KS, N0, nroots;            // roots are cells 0 .. nroots-1
    double theta2;                    // MAC^2
    double* out;                      // [nt] or [nt][3], caller order
    int32_t* status;                  // set to 1 by a wave whose stack overflows
};
int launch_treecode(const TcArgs& a, int kernel, hipStream_t s);
// Partial sums of the direct sum without allocation: 4 Mi doubles (32 MiB)
// of static device memory per device.
constexpr int64_t kDirectScratchDoubles = int64_t(1) << 22;
int launch_direct(const double* tgt, int64_t nt, const double* src, int64_t ns, const double* w,
                  int kernel, bool fp32, double* out, hipStream_t s, bool no_alloc = false);

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

}  // namespace csfmm
