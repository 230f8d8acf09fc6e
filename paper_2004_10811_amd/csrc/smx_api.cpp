// Host side of libsmx: the C ABI declared in include/smx.h.
//
// Responsibilities: argument and layout validation, the per-pattern plan
// (row sets R(g), gather/scatter tables, product tiles), device memory, and
// the stream-ordered driver of one evaluation:
//   gather + shift + Gershgorin bound -> Newton-Schulz steps (two batched
//   matrix-core products per step, converged groups skip on the device) ->
//   scatter of the own columns of D with energy/trace partials -> fixed-order
//   reduction.
#include "smx.h"
#include "smx_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace smx;

// Work memory of smx_evaluate_static: a fixed array in device memory, one
// copy per device, held until the process ends.  Host code never uses the
// array's name as an address (on the host it is only a stand-in for the
// symbol); each device's address is resolved once, at smx_create, and kept
// in g_scratch_ptr.  External linkage on purpose: the HIP runtime resolves a
// device variable by name among the code object's exported symbols, and an
// internal-linkage array would be a local symbol it cannot find.
__device__ __align__(256) unsigned char smx_static_scratch[SMX_STATIC_SCRATCH_BYTES];

namespace {

// Marker ranges (roctx) around the entry points and the phases they enqueue,
// for rocprofv3 --marker-trace; host-side spans (with host polling the
// iteration range lasts until the last step is launched).  Ranges still open
// when the scope ends (an early error return) are closed then.
struct TraceScope {
    int depth = 0;
    TraceScope() = default;
    explicit TraceScope(const char *name) { push(name); }
    void push(const char *name)
    {
        roctxRangePushA(name);
        depth++;
    }
    void pop()
    {
        if (depth > 0) {
            roctxRangePop();
            depth--;
        }
    }
    void next(const char *name)
    {
        pop();
        push(name);
    }
    ~TraceScope()
    {
        while (depth > 0) pop();
    }
    TraceScope(const TraceScope &) = delete;
    TraceScope &operator=(const TraceScope &) = delete;
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), bytes);
        if (e == hipSuccess) cap = std::max<size_t>(n, 1);
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    size_t bytes() const { return cap * sizeof(T); }
};

struct Plan {
    int32_t ngroups = 0;
    std::vector<GroupDesc> gd;
    std::vector<TileDesc> tiles;
    std::vector<int2> chunks;
    std::vector<RowInfo> rinfo;
    std::vector<int32_t> bmap;
    std::vector<int32_t> boffs;
    std::vector<ScatterDesc> scat;
    std::vector<int32_t> own_list;    // own columns of every group (submatrix column indices)
    std::vector<double> wtiles;       // live 64 x 64 wave tiles of one product, per group
    std::vector<TileDesc> tiles_full; // every tile (general products of the adjoint), XCD-ordered
    std::vector<int64_t> cptr;        // per stored block: its contributions from the groups (adjoint)
    std::vector<int4> contrib;        // (group, row offset, column offset, 0), ascending group per block
    // waves: consecutive group ranges [wave_g[w], wave_g[w+1]) whose slabs share one arena;
    // slab and own-column offsets (GroupDesc::off, thin_off) are relative to the wave
    std::vector<int32_t> wave_g;
    std::vector<int32_t> wave_of;      // wave of every group
    std::vector<int64_t> tile_beg;     // wave w's lower tiles: tiles[tile_beg[w] .. tile_beg[w+1])
    // size buckets of the one- and two-word products: groups with n_pad >= the
    // context's big_min_npad take 256 x 256 tiles (tiles_b), the others 128 x 128
    // tiles (tiles_s); per wave like tile_beg
    std::vector<char> big;
    std::vector<TileDesc> tiles_s, tiles_b;
    std::vector<int64_t> tiles_s_beg, tiles_b_beg;
    std::vector<double> wtiles2;       // live 16 x 16 blocks of one product on 256 x 256 tiles, per group
    // per-XCD work lists of the 128 x 128 bucket for the persistent word products:
    // wave w's lists start at tiles_sx[sx_wbeg[w]], list x at + xbeg[9 w + x]
    std::vector<TileDesc> tiles_sx;
    std::vector<int64_t> sx_wbeg;
    std::vector<int32_t> xbeg;
    std::vector<int64_t> chunk_beg;    // wave w's gather chunks (chunks are in group order)
    std::vector<int64_t> plist;        // stored blocks of the own columns of each wave (more than one wave)
    std::vector<int64_t> plist_beg;
    int64_t work_elems = 0;            // slab elements of the largest wave
    int64_t thin_elems = 0;            // own-column elements of the largest wave
    int64_t total_elems = 0;           // slab elements of all groups
    int32_t max_npad = 0, max_own = 0;
    int32_t nwaves() const { return (int32_t)wave_g.size() - 1; }
};

// Device addresses of a plan's tables and of the per-evaluation state: the
// context's own buffers, or places in the static scratch array.
struct DevView {
    const GroupDesc *gd = nullptr;
    const TileDesc *tiles = nullptr, *tiles_s = nullptr, *tiles_b = nullptr;
    const TileDesc *tiles_sx = nullptr;     // per-XCD lists of the persistent word products (context buffers only)
    const int32_t *xbeg = nullptr;
    const int2 *chunks = nullptr;
    const RowInfo *rinfo = nullptr;
    const int32_t *bmap = nullptr, *boffs = nullptr, *own = nullptr;
    const ScatterDesc *scat = nullptr;
    const int64_t *plist = nullptr;
    unsigned long long *scale = nullptr, *resid = nullptr;
    int32_t *done = nullptr, *kfinal = nullptr, *flags = nullptr, *ndone = nullptr;
    double *tdiag = nullptr, *tau_hist = nullptr, *pe = nullptr, *pn = nullptr, *ne = nullptr;
};

// Arena of one wave: three FP64 slabs X_a | X_b | W (24 bytes per element);
// in the reduced-precision modes the words of X_a, X_b and W (nw E 16-bit
// words each) start at byte 8E (over X_b and W, dead during the bulk) and reach 8E + 6 nw E bytes,
// i.e. 26 bytes per element with three BF16 words.
constexpr int64_t kArenaBytesPerElem = 26;

// Largest n_polish of the reduced-precision modes (the own-column polish
// evaluates a degree-3^n_polish polynomial by 3^n_polish - 1 thin products).
constexpr int32_t kMaxPolishMixed = 4;

// Default size bucket boundary of the one- and two-word products: groups whose
// padded dimension reaches it take 256 x 256 tiles (0: 128 x 128 tiles only).
constexpr int32_t kDefaultBigMinNpad = 0;

}  // namespace

struct smx_context {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // problem
    bool loaded = false;
    int32_t nblk = 0;
    int64_t nnzb = 0, nvals = 0;
    std::vector<int32_t> blk_size;
    std::vector<int64_t> col_ptr;
    std::vector<int32_t> row_idx;
    std::vector<int64_t> val_off;
    std::vector<int32_t> grp_ptr, grp_blocks;
    bool plan_dirty = true;
    Plan plan;
    // plan of the static-scratch evaluation (smx_evaluate_static): same groups
    // and tiles, waves sized to the fixed scratch array, tables kept in it
    bool splan_dirty = true;
    Plan splan;
    uint64_t splan_gen = 0;
    uint64_t uid = 0;                    // unique per context (owner tag of the scratch tables)
    int32_t splan_stride = -1;           // history stride the static layout was sized for

    // options
    double mu = 0.0, kT = 0.0;
    int32_t precision = SMX_FP64;
    int32_t iteration = SMX_ITER_NS2;         // sign iteration of the FP64 path and the bulk (smx_set_iteration)
    int32_t solver = SMX_SOLVER_ITERATIVE;    // smx_set_solver; kT > 0 always diagonalises
    double tol = 1e-12, switch_tol = 1e-3;
    int32_t max_iter = 100, n_polish = 2;

    // device: problem
    DevBuf<double> d_k, d_d;
    DevBuf<int64_t> d_valoff, d_mirror;
    DevBuf<int32_t> d_brow, d_bcol;
    // device: plan
    DevBuf<GroupDesc> d_gd;
    DevBuf<TileDesc> d_tiles, d_tiles_s, d_tiles_b, d_tiles_sx;
    DevBuf<int32_t> d_xbeg, d_tq;           // per-XCD list offsets, counters of the persistent word products
    DevBuf<int2> d_chunks;
    DevBuf<RowInfo> d_rinfo;
    DevBuf<int32_t> d_bmap, d_boffs;
    DevBuf<ScatterDesc> d_scat;
    // device: work
    DevBuf<double> d_arena;                 // one wave's slabs (see kArenaBytesPerElem), when no
                                            // caller work space is set
    int64_t ws_limit = 0;                   // arena byte limit (0: from free device memory)
    void *ws_ptr = nullptr;                 // caller work space (smx_set_workspace): arena, then polish pool
    size_t ws_bytes = 0;
    int32_t host_poll = 1;                  // 1: stop launching once every group is done (host polls);
                                            // 0: enqueue all max_iter steps, no host synchronisation
    int32_t tile_order = 0;                 // 0: XCD-aware launch order, 1: group by group
    int32_t kernel_variant = 0;             // operand stream of the word products (smx_set_kernel_variant)
    int32_t pers_nwg = 0;                   // workgroups of a persistent word-product launch (0: not yet known)
    int32_t big_min_npad = kDefaultBigMinNpad;   // 256 x 256 tiles from this n_pad on (smx_set_tile_shape)
    DevBuf<unsigned long long> d_scale, d_resid;
    DevBuf<int32_t> d_done, d_kfinal, d_flags, d_ndone;
    DevBuf<double> d_pe, d_pn, d_ne, d_check;
    DevBuf<int32_t> d_fsum;                 // flag counts of a static-scratch evaluation
    DevBuf<int32_t> d_own;
    DevBuf<double> d_tdiag, d_tau_hist;
    // frozen iteration (derivatives, mu search): step counts and scales of a previous evaluation
    DevBuf<int32_t> d_kfix;
    DevBuf<unsigned long long> d_sfix, d_scale_scratch;
    DevBuf<double> d_tx0, d_tx1, d_dnp, d_dn;    // mu tangent of the iterates, its reduction
    // eigensolver (finite temperature, Algorithm 1): per-row arrays indexed like the row tables
    DevBuf<double> d_ed, d_ee, d_etau, d_elam, d_elabs, d_ew, d_mus, d_npart, d_nval;
    DevBuf<int32_t> d_ebs, d_ebe;
    // adjoint
    DevBuf<TileDesc> d_tiles_full;
    DevBuf<int64_t> d_cptr;
    DevBuf<int4> d_contrib;
    DevBuf<double> d_adj, d_dk, d_dmu;
    bool contrib_ready = false;
    // D in another layout (smx_get_d_expanded)
    DevBuf<int64_t> d_xidx;
    DevBuf<double> d_xout;
    DevBuf<double> d_tpool;                      // own-column blocks of the FP64 polish (2 n_polish + 1)
    DevBuf<int64_t> d_plist;

    // host polling / timing
    int32_t *h_ndone = nullptr;
    int32_t h_ndone_cap = 0;
    std::vector<hipEvent_t> ev_poll;
    std::vector<hipEvent_t> ev_launch;   // two per product launch (before, after)
    std::vector<int32_t> launch_step;    // step k of each product launch
    std::vector<int32_t> launch_kind;    // 0/1 FP64 square/update, 2/3 word square/update (128 x 128
                                         // tiles), 4/5 polish, 6 tangent, 7/8 word square/update (256 x 256)
    std::vector<int32_t> launch_wave;    // wave of each product launch
    std::vector<int32_t> launch_subset;  // groups of the launch: 0 all, 1 the 128-tile bucket, 2 the 256-tile bucket
    std::vector<hipEvent_t> ev_wave;     // four per wave: start, iterate, scatter, end
    hipEvent_t ev_t0 = nullptr, ev_t3 = nullptr;

    // results of the last evaluation
    bool evaluated = false;
    int32_t steps_launched = 0;
    int32_t last_precision = SMX_FP64;
    int32_t last_iteration = SMX_ITER_NS2;
    bool last_eig = false;                     // last evaluation diagonalised the submatrices
    double last_kT = 0.0;
    int32_t last_stride = 0;
    int32_t last_polish = 0;             // FP64 polish steps after the bulk (0 in FP64 mode)
    int32_t last_max_iter = 0;
    int32_t last_fmt = -1, last_nw = 0;        // storage of the reduced-precision bulk
    bool use_kfix = false, use_sfix = false;  // frozen step counts / scales
    bool have_tangent = false;                 // last evaluation computed dN/dmu
    bool last_sfix = false;                    // last evaluation ran on the frozen scales
    bool eval_static = false;                  // last evaluation ran in the static scratch array
    int32_t debug_checks = 0;                  // smx_set_debug_checks
    bool guards_armed = false;                 // guard regions written before the last evaluation
    double last_mu = 0.0;                      // mu of the last evaluation (the adjoint's A_g)

    // step graphs (smx_set_graph)
    int32_t graph_steps = 0;                   // steps per graph; 0: direct launches
    uint64_t plan_gen = 0;                     // bumped whenever the plan is rebuilt
    hipStream_t cap_stream = nullptr;          // private stream for graph capture
    std::vector<hipGraphExec_t> graphs;        // [wave][chunk], captured on first use
    std::vector<uint64_t> graph_sig;
};

namespace {

int32_t fail(smx_ctx c, int32_t code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

std::string g_create_err;

// Per-device address of the static scratch array, resolved once per device
// (with that device current) by the first smx_create on it; and which
// context's plan tables the array holds (uid, plan generation).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_tried[kMaxDevices] = {};
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
uint64_t g_scratch_owner[kMaxDevices][2] = {};
std::atomic<uint64_t> g_ctx_uid{0};

void drop_graphs(smx_ctx c)
{
    for (hipGraphExec_t &g : c->graphs)
        if (g) (void)hipGraphExecDestroy(g);
    c->graphs.clear();
    c->graph_sig.clear();
}

#define HIP_TRY(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return fail((ctx), _e == hipErrorOutOfMemory ? SMX_E_NOMEM : SMX_E_HIP,          \
                        std::string(#expr) + ": " + hipGetErrorString(_e));                  \
    } while (0)

template <typename T>
hipError_t upload(DevBuf<T> &b, const std::vector<T> &v, hipStream_t st)
{
    hipError_t e = b.ensure(v.size());
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// Bytes of one wave's arena (three FP64 slabs, or the words of three
// iterates laid from byte 8E), rounded up to 256, and of its polish pool.
int64_t arena_bytes(const Plan &P) { return (kArenaBytesPerElem * P.work_elems + 255) / 256 * 256; }
int64_t pool_bytes(const Plan &P) { return (2 * kMaxPolishMixed + 1) * 8 * P.thin_elems; }

double *arena_base(smx_ctx c) { return c->ws_ptr ? static_cast<double *>(c->ws_ptr) : c->d_arena.p; }
double *pool_base(smx_ctx c)
{
    return c->ws_ptr ? reinterpret_cast<double *>(static_cast<char *>(c->ws_ptr) + arena_bytes(c->plan))
                     : c->d_tpool.p;
}
double *slab(smx_ctx c, int i) { return arena_base(c) + (size_t)i * (size_t)c->plan.work_elems; }

// XCD-aware launch order.  Workgroup b of a launch runs on XCD b % 8 (the
// dispatcher deals workgroups round-robin over the 8 XCDs), and every XCD has
// its own L2.  All tiles of one group go to one XCD, so the group's panels are
// fetched into one L2 and shared by its tiles; groups are dealt to XCDs
// greedily by work (n_pad x tiles), largest first.  Slot s of XCD x becomes
// workgroup 8 s + x; short lists are padded with idle tiles (group -1).
// The tiles of groups g0 .. g1 - 1 dealt to the 8 XCDs: all tiles of a group
// to one XCD, groups largest first to the XCD with the least work so far.
std::vector<std::vector<TileDesc>> xcd_deal(const Plan &P, int32_t g0, int32_t g1, const std::vector<TileDesc> &tiles)
{
    constexpr int kXcd = 8;
    const int32_t ng = g1 - g0;
    std::vector<int32_t> order(ng);
    for (int32_t g = 0; g < ng; g++) order[g] = g0 + g;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return P.gd[a].npad > P.gd[b].npad; });
    std::vector<std::vector<TileDesc>> per_group(ng), lists(kXcd);
    for (const TileDesc &t : tiles) per_group[t.x - g0].push_back(t);
    std::vector<double> load(kXcd, 0.0);
    for (int32_t g : order) {
        int best = 0;
        for (int x = 1; x < kXcd; x++)
            if (load[x] < load[best]) best = x;
        load[best] += (double)P.gd[g].npad * per_group[g - g0].size();
        for (const TileDesc &t : per_group[g - g0]) lists[best].push_back(t);
    }
    return lists;
}

void xcd_order(const Plan &P, int32_t g0, int32_t g1, std::vector<TileDesc> &tiles)
{
    constexpr int kXcd = 8;
    const auto lists = xcd_deal(P, g0, g1, tiles);
    size_t len = 0;
    for (const auto &l : lists) len = std::max(len, l.size());
    tiles.assign(len * kXcd, TileDesc{-1, 0});
    for (int x = 0; x < kXcd; x++)
        for (size_t q = 0; q < lists[x].size(); q++) tiles[q * kXcd + x] = lists[x][q];
}

int32_t build_plan(smx_ctx c, Plan &P)
{
    P = Plan();
    const int32_t nblk = c->nblk;
    const int32_t ng = (int32_t)c->grp_ptr.size() - 1;
    P.ngroups = ng;
    std::vector<int32_t> pos(nblk, -1);
    std::vector<char> mark(nblk, 0);
    P.scat.assign((size_t)c->nnzb, ScatterDesc{-1, 0, 0, 0});
    std::vector<int32_t> rows;
    rows.reserve(1024);
    for (int32_t g = 0; g < ng; g++) {
        rows.clear();
        for (int32_t q = c->grp_ptr[g]; q < c->grp_ptr[g + 1]; q++) {
            const int32_t j = c->grp_blocks[q];
            for (int64_t p = c->col_ptr[j]; p < c->col_ptr[j + 1]; p++) {
                const int32_t i = c->row_idx[p];
                if (!mark[i]) {
                    mark[i] = 1;
                    rows.push_back(i);
                }
            }
        }
        std::sort(rows.begin(), rows.end());
        const int32_t m = (int32_t)rows.size();
        GroupDesc d{};
        d.m = m;
        d.boff_off = (int32_t)P.boffs.size();
        int64_t n = 0;
        for (int32_t t = 0; t < m; t++) {
            mark[rows[t]] = 0;
            pos[rows[t]] = t;
            P.boffs.push_back((int32_t)n);
            n += c->blk_size[rows[t]];
        }
        P.boffs.push_back((int32_t)n);
        if (n > 60000) return fail(c, SMX_E_INVALID, "submatrix dimension above 60000 in group " + std::to_string(g));
        d.n = (int32_t)n;
        d.npad = (int32_t)(((std::max<int64_t>(n, 1) + kPad - 1) / kPad) * kPad);
        P.total_elems += (int64_t)d.npad * d.npad;
        d.rinfo_off = (int64_t)P.rinfo.size();
        for (int32_t t = 0; t < m; t++) {
            const int32_t b = c->blk_size[rows[t]];
            for (int32_t rr = 0; rr < b; rr++) P.rinfo.push_back(RowInfo{t, rr | (b << 16)});
        }
        for (int32_t r = d.n; r < d.npad; r++) P.rinfo.push_back(RowInfo{0, 0});
        d.map_off = (int64_t)P.bmap.size();
        P.bmap.resize(P.bmap.size() + (size_t)m * m, -1);
        for (int32_t tb = 0; tb < m; tb++) {
            const int32_t j = rows[tb];
            for (int64_t p = c->col_ptr[j]; p < c->col_ptr[j + 1]; p++) {
                const int32_t a = pos[c->row_idx[p]];
                if (a >= 0) P.bmap[(size_t)d.map_off + a + (size_t)m * tb] = (int32_t)p;
            }
        }
        d.own_off = (int32_t)P.own_list.size();
        int32_t ocol = 0;
        for (int32_t q = c->grp_ptr[g]; q < c->grp_ptr[g + 1]; q++) {
            const int32_t j = c->grp_blocks[q];
            const int32_t oj = P.boffs[d.boff_off + pos[j]];
            for (int64_t p = c->col_ptr[j]; p < c->col_ptr[j + 1]; p++) {
                const int32_t i = c->row_idx[p];
                const int32_t oi = P.boffs[d.boff_off + pos[i]];
                P.scat[p] = ScatterDesc{g, oi, oj, c->blk_size[i] | (c->blk_size[j] << 16), ocol, 0};
            }
            for (int32_t cc = 0; cc < c->blk_size[j]; cc++) P.own_list.push_back(oj + cc);
            ocol += c->blk_size[j];
        }
        d.m_own = ocol;
        P.max_npad = std::max(P.max_npad, d.npad);
        P.max_own = std::max(P.max_own, d.m_own);
        for (int32_t t = 0; t < m; t++) pos[rows[t]] = -1;
        const int32_t nt = (d.npad + kTile - 1) / kTile;
        for (int32_t r0 = 0; r0 < d.npad; r0 += 256) P.chunks.push_back(int2{g, r0});
        // issued flops of one product: live 64 x 64 wave tiles x K
        double wt = 0;
        for (int32_t ti = 0; ti < nt; ti++)
            for (int32_t tj = 0; tj <= ti; tj++)
                for (int wr = 0; wr < 2; wr++)
                    for (int wc = 0; wc < 2; wc++) {
                        if (ti * kTile + wr * 64 >= d.npad || tj * kTile + wc * 64 >= d.npad) continue;
                        if (ti == tj && wr < wc) continue;
                        wt += 1;
                    }
        P.wtiles.push_back(wt);
        // the same on 256 x 256 tiles: live 16 x 16 blocks (inside the matrix,
        // not entirely above the diagonal of a diagonal tile)
        const int32_t nt2 = (d.npad + kTile2 - 1) / kTile2;
        double wt2 = 0;
        for (int32_t ti = 0; ti < nt2; ti++)
            for (int32_t tj = 0; tj <= ti; tj++)
                for (int32_t r0 = 0; r0 < kTile2; r0 += 16)
                    for (int32_t c0 = 0; c0 < kTile2; c0 += 16) {
                        if (ti * kTile2 + r0 >= d.npad || tj * kTile2 + c0 >= d.npad) continue;
                        if (ti == tj && r0 + 15 < c0) continue;
                        wt2 += 1;
                    }
        P.wtiles2.push_back(wt2);
        P.gd.push_back(d);
    }
    for (int64_t p = 0; p < c->nnzb; p++)
        if (P.scat[p].g < 0) return fail(c, SMX_E_INVALID, "internal: stored block without a group");
    return SMX_OK;
}

// Device bytes one group adds to a wave: its share of the arena and of the
// own-column blocks of the FP64 polish (2 n_polish + 1 <= 9 of them).
int64_t group_bytes(const GroupDesc &d)
{
    return kArenaBytesPerElem * (int64_t)d.npad * d.npad + (2 * kMaxPolishMixed + 1) * 8 * (int64_t)d.npad * d.m_own;
}

// Split the groups into consecutive waves of at most `budget` bytes each
// (balanced: about total / ceil(total / budget) per wave), assign the
// wave-relative slab offsets, and build each wave's launch lists.
int32_t partition_waves(smx_ctx c, Plan &P, int64_t budget)
{
    const int32_t ng = P.ngroups;
    int64_t total = 0;
    for (int32_t g = 0; g < ng; g++) {
        const int64_t b = group_bytes(P.gd[g]);
        if (b > budget)
            return fail(c, SMX_E_NOMEM, "group " + std::to_string(g) + " needs " + std::to_string(b >> 20) +
                                            " MiB of work space, more than the " + std::to_string(budget >> 20) +
                                            " MiB available");
        total += b;
    }
    const int64_t nw0 = std::max<int64_t>(1, (total + budget - 1) / budget);
    const int64_t target = std::min<int64_t>(budget, (total + nw0 - 1) / nw0);
    P.wave_g.assign(1, 0);
    P.wave_of.assign((size_t)ng, 0);
    int64_t cur = 0;
    for (int32_t g = 0; g < ng; g++) {
        const int64_t b = group_bytes(P.gd[g]);
        if (cur > 0 && cur + b > target) {
            P.wave_g.push_back(g);
            cur = 0;
        }
        cur += b;
        P.wave_of[g] = (int32_t)P.wave_g.size() - 1;
    }
    P.wave_g.push_back(ng);
    const int32_t nw = P.nwaves();
    P.work_elems = P.thin_elems = 0;
    P.tiles.clear();
    P.tiles_full.clear();
    P.tile_beg.assign(1, 0);
    P.tiles_s.clear();
    P.tiles_b.clear();
    P.tiles_s_beg.assign(1, 0);
    P.tiles_b_beg.assign(1, 0);
    P.tiles_sx.clear();
    P.sx_wbeg.assign(1, 0);
    P.xbeg.clear();
    P.big.assign((size_t)ng, 0);
    for (int32_t g = 0; g < ng; g++) P.big[g] = c->big_min_npad > 0 && P.gd[g].npad >= c->big_min_npad;
    P.chunk_beg.assign(1, 0);
    P.plist.clear();
    P.plist_beg.assign(1, 0);
    size_t ch = 0;
    for (int32_t w = 0; w < nw; w++) {
        int64_t e = 0, t = 0;
        std::vector<TileDesc> tl, ts, tb;
        for (int32_t g = P.wave_g[w]; g < P.wave_g[w + 1]; g++) {
            GroupDesc &d = P.gd[g];
            d.off = e;
            e += (int64_t)d.npad * d.npad;
            d.thin_off = t;
            t += (int64_t)d.npad * d.m_own;
            const int32_t nt = (d.npad + kTile - 1) / kTile;
            for (int32_t ti = 0; ti < nt; ti++)
                for (int32_t tj = 0; tj <= ti; tj++) tl.push_back(TileDesc{g, (ti << 16) | tj});
            if (P.big[g]) {
                const int32_t nt2 = (d.npad + kTile2 - 1) / kTile2;
                for (int32_t ti = 0; ti < nt2; ti++)
                    for (int32_t tj = 0; tj <= ti; tj++) tb.push_back(TileDesc{g, (ti << 16) | tj});
            } else {
                for (int32_t ti = 0; ti < nt; ti++)
                    for (int32_t tj = 0; tj <= ti; tj++) ts.push_back(TileDesc{g, (ti << 16) | tj});
            }
        }
        P.work_elems = std::max(P.work_elems, e);
        P.thin_elems = std::max(P.thin_elems, t);
        {
            const auto lists = xcd_deal(P, P.wave_g[w], P.wave_g[w + 1], ts);
            int32_t off = 0;
            for (const auto &l : lists) {
                P.xbeg.push_back(off);
                P.tiles_sx.insert(P.tiles_sx.end(), l.begin(), l.end());
                off += (int32_t)l.size();
            }
            P.xbeg.push_back(off);
            P.sx_wbeg.push_back((int64_t)P.tiles_sx.size());
        }
        if (c->tile_order == 0) {
            xcd_order(P, P.wave_g[w], P.wave_g[w + 1], tl);
            if (!ts.empty()) xcd_order(P, P.wave_g[w], P.wave_g[w + 1], ts);
            if (!tb.empty()) xcd_order(P, P.wave_g[w], P.wave_g[w + 1], tb);
        }
        P.tiles.insert(P.tiles.end(), tl.begin(), tl.end());
        P.tile_beg.push_back((int64_t)P.tiles.size());
        P.tiles_s.insert(P.tiles_s.end(), ts.begin(), ts.end());
        P.tiles_s_beg.push_back((int64_t)P.tiles_s.size());
        P.tiles_b.insert(P.tiles_b.end(), tb.begin(), tb.end());
        P.tiles_b_beg.push_back((int64_t)P.tiles_b.size());
        while (ch < P.chunks.size() && P.chunks[ch].x < P.wave_g[w + 1]) ch++;
        P.chunk_beg.push_back((int64_t)ch);
    }
    if (nw == 1) {
        // every tile (general products of the adjoint), XCD-ordered
        for (int32_t g = 0; g < ng; g++) {
            const int32_t nt = (P.gd[g].npad + kTile - 1) / kTile;
            for (int32_t ti = 0; ti < nt; ti++)
                for (int32_t tj = 0; tj < nt; tj++) P.tiles_full.push_back(TileDesc{g, (ti << 16) | tj});
        }
        xcd_order(P, 0, ng, P.tiles_full);
    } else {
        std::vector<int64_t> cnt((size_t)nw + 1, 0);
        for (int64_t p = 0; p < c->nnzb; p++) cnt[(size_t)P.wave_of[P.scat[p].g] + 1]++;
        for (int32_t w = 0; w < nw; w++) cnt[w + 1] += cnt[w];
        P.plist_beg = cnt;
        P.plist.assign((size_t)c->nnzb, 0);
        for (int64_t p = 0; p < c->nnzb; p++) P.plist[(size_t)cnt[(size_t)P.wave_of[P.scat[p].g]]++] = p;
    }
    return SMX_OK;
}

// Host-side consistency check of everything the kernels will index with.
int32_t check_plan(smx_ctx c, const Plan &P)
{
    const int32_t nw = P.nwaves();
    if (nw < 1 || P.wave_g[0] != 0 || P.wave_g[nw] != P.ngroups || (int32_t)P.tile_beg.size() != nw + 1 ||
        (int32_t)P.chunk_beg.size() != nw + 1 || P.tile_beg[nw] != (int64_t)P.tiles.size() ||
        P.chunk_beg[nw] != (int64_t)P.chunks.size())
        return fail(c, SMX_E_INVALID, "internal: wave tables");
    for (int32_t w = 0; w < nw; w++) {
        if (P.wave_g[w + 1] <= P.wave_g[w]) return fail(c, SMX_E_INVALID, "internal: empty wave");
        for (int64_t q = P.tile_beg[w]; q < P.tile_beg[w + 1]; q++) {
            const TileDesc &t = P.tiles[(size_t)q];
            if (t.x == -1) continue;    // idle slot of the XCD-aware launch order
            if (t.x < P.wave_g[w] || t.x >= P.wave_g[w + 1]) return fail(c, SMX_E_INVALID, "internal: tile group");
            const GroupDesc &d = P.gd[t.x];
            const int ti = t.y >> 16, tj = t.y & 0xffff;
            if (tj > ti || ti * kTile >= d.npad) return fail(c, SMX_E_INVALID, "internal: tile index");
        }
        // size-bucket lists: every group of the wave in exactly one of them,
        // with its full set of lower tiles of that shape
        if ((int32_t)P.tiles_s_beg.size() != nw + 1 || (int32_t)P.tiles_b_beg.size() != nw + 1 ||
            P.tiles_s_beg[nw] != (int64_t)P.tiles_s.size() || P.tiles_b_beg[nw] != (int64_t)P.tiles_b.size() ||
            (int32_t)P.big.size() != P.ngroups)
            return fail(c, SMX_E_INVALID, "internal: size-bucket tables");
        std::vector<int64_t> seen((size_t)(P.wave_g[w + 1] - P.wave_g[w]), 0);
        for (int pass = 0; pass < 2; pass++) {
            const std::vector<TileDesc> &L = pass ? P.tiles_b : P.tiles_s;
            const std::vector<int64_t> &B = pass ? P.tiles_b_beg : P.tiles_s_beg;
            const int edge = pass ? kTile2 : kTile;
            for (int64_t q = B[w]; q < B[w + 1]; q++) {
                const TileDesc &t = L[(size_t)q];
                if (t.x == -1) continue;
                if (t.x < P.wave_g[w] || t.x >= P.wave_g[w + 1] || (P.big[t.x] != 0) != (pass == 1))
                    return fail(c, SMX_E_INVALID, "internal: size-bucket tile group");
                const int ti = t.y >> 16, tj = t.y & 0xffff;
                if (tj > ti || ti * edge >= P.gd[t.x].npad) return fail(c, SMX_E_INVALID, "internal: size-bucket tile");
                seen[(size_t)(t.x - P.wave_g[w])]++;
            }
        }
        for (int32_t g = P.wave_g[w]; g < P.wave_g[w + 1]; g++) {
            const int64_t nt = (P.gd[g].npad + (P.big[g] ? kTile2 : kTile) - 1) / (P.big[g] ? kTile2 : kTile);
            if (seen[(size_t)(g - P.wave_g[w])] != nt * (nt + 1) / 2)
                return fail(c, SMX_E_INVALID, "internal: size-bucket tile count");
        }
        for (int64_t q = P.chunk_beg[w]; q < P.chunk_beg[w + 1]; q++) {
            const int2 &ch = P.chunks[(size_t)q];
            if (ch.x < P.wave_g[w] || ch.x >= P.wave_g[w + 1] || ch.y < 0 || ch.y >= P.gd[ch.x].npad)
                return fail(c, SMX_E_INVALID, "internal: gather chunk");
        }
        if (nw > 1)
            for (int64_t q = P.plist_beg[w]; q < P.plist_beg[w + 1]; q++) {
                const int64_t p = P.plist[(size_t)q];
                if (p < 0 || p >= c->nnzb || P.wave_of[P.scat[p].g] != w)
                    return fail(c, SMX_E_INVALID, "internal: scatter list");
            }
    }
    if (nw > 1 && (P.plist_beg[nw] != c->nnzb || !P.tiles_full.empty()))
        return fail(c, SMX_E_INVALID, "internal: scatter list");
    for (const TileDesc &t : P.tiles_full) {
        if (t.x == -1) continue;
        if (t.x < 0 || t.x >= P.ngroups) return fail(c, SMX_E_INVALID, "internal: tile group");
        const GroupDesc &d = P.gd[t.x];
        const int ti = t.y >> 16, tj = t.y & 0xffff;
        if (ti * kTile >= d.npad || tj * kTile >= d.npad) return fail(c, SMX_E_INVALID, "internal: tile index");
    }
    for (const GroupDesc &d : P.gd) {
        if (d.npad % 16 || d.npad < d.n || d.off < 0 || d.off + (int64_t)d.npad * d.npad > P.work_elems)
            return fail(c, SMX_E_INVALID, "internal: group extent");
        if (d.rinfo_off + d.npad > (int64_t)P.rinfo.size() ||
            d.map_off + (int64_t)d.m * d.m > (int64_t)P.bmap.size() ||
            d.boff_off + d.m + 1 > (int64_t)P.boffs.size() || P.boffs[d.boff_off + d.m] != d.n)
            return fail(c, SMX_E_INVALID, "internal: group tables");
    }
    for (size_t q = 0; q < P.bmap.size(); q++)
        if (P.bmap[q] < -1 || P.bmap[q] >= c->nnzb) return fail(c, SMX_E_INVALID, "internal: block map");
    for (const RowInfo &r : P.rinfo)
        if (r.x < 0 || (r.y & 0xffff) >= (r.y >> 16 ? (r.y >> 16) : 1)) return fail(c, SMX_E_INVALID, "internal: row table");
    for (int64_t p = 0; p < c->nnzb; p++) {
        const ScatterDesc &s = P.scat[p];
        const GroupDesc &d = P.gd[s.g];
        if (s.oi + (s.bij & 0xffff) > d.n || s.oj + (s.bij >> 16) > d.n || s.ocol + (s.bij >> 16) > d.m_own)
            return fail(c, SMX_E_INVALID, "internal: scatter extent");
    }
    for (const GroupDesc &d : P.gd) {
        if (d.own_off + d.m_own > (int64_t)P.own_list.size() || d.thin_off < 0 ||
            d.thin_off + (int64_t)d.npad * d.m_own > P.thin_elems)
            return fail(c, SMX_E_INVALID, "internal: own-column tables");
        for (int32_t q = 0; q < d.m_own; q++)
            if (P.own_list[d.own_off + q] < 0 || P.own_list[d.own_off + q] >= d.n)
                return fail(c, SMX_E_INVALID, "internal: own-column index");
    }
    return SMX_OK;
}

template <typename T>
size_t vbytes(const std::vector<T> &v) { return v.size() * sizeof(T); }

int32_t ensure_plan(smx_ctx c)
{
    if (!c->plan_dirty) return SMX_OK;
    Plan &P = c->plan;
    int32_t st = build_plan(c, P);
    if (st) return st;
    // work space: release what depends on the plan, then size the waves to
    // the limit set by smx_set_workspace_limit or to the free device memory
    // left after the plan's tables (with 1 GiB held back, and no more than
    // 3/4 of the device)
    c->d_arena.release();
    c->d_tpool.release();
    c->d_tx0.release();
    c->d_tx1.release();
    c->d_adj.release();
    int64_t budget = c->ws_ptr ? (int64_t)c->ws_bytes - 512 : c->ws_limit;
    if (budget <= 0 && c->ws_ptr) return fail(c, SMX_E_NOMEM, "the work space is too small");
    if (budget <= 0) {
        size_t fr = 0, tot = 0;
        HIP_TRY(c, hipMemGetInfo(&fr, &tot));
        int64_t tiles_est = 0;
        for (const GroupDesc &d : P.gd) {
            const int64_t nt = (d.npad + kTile - 1) / kTile;
            tiles_est += nt * nt;
        }
        const int64_t tables = (int64_t)(vbytes(P.gd) + vbytes(P.chunks) + vbytes(P.rinfo) + vbytes(P.bmap) +
                                         vbytes(P.boffs) + vbytes(P.scat) + vbytes(P.own_list)) +
                               (int64_t)sizeof(TileDesc) * 2 * tiles_est + 8 * c->nnzb + 64 * (int64_t)P.ngroups;
        // at most 3/4 of the device in one allocation
        budget = std::min<int64_t>((int64_t)fr - tables - (int64_t)(1ll << 30), (int64_t)(tot / 4 * 3));
        if (budget <= 0) return fail(c, SMX_E_NOMEM, "no device memory left for the submatrix work space");
    }
    st = partition_waves(c, P, budget);
    if (st) return st;
    // a caller work space holds the largest wave's arena and pool side by side;
    // the largest arena and the largest pool may come from different waves, so
    // shrink the wave budget until both fit
    while (c->ws_ptr && arena_bytes(P) + pool_bytes(P) > (int64_t)c->ws_bytes) {
        budget = budget * 15 / 16;
        st = partition_waves(c, P, budget);
        if (st) return st;
    }
    st = check_plan(c, P);
    if (st) return st;
    HIP_TRY(c, upload(c->d_gd, P.gd, c->stream));
    HIP_TRY(c, upload(c->d_tiles, P.tiles, c->stream));
    HIP_TRY(c, upload(c->d_tiles_s, P.tiles_s, c->stream));
    HIP_TRY(c, upload(c->d_tiles_b, P.tiles_b, c->stream));
    HIP_TRY(c, upload(c->d_tiles_sx, P.tiles_sx, c->stream));
    HIP_TRY(c, upload(c->d_xbeg, P.xbeg, c->stream));
    HIP_TRY(c, upload(c->d_tiles_full, P.tiles_full, c->stream));
    HIP_TRY(c, upload(c->d_plist, P.plist, c->stream));
    c->contrib_ready = false;
    HIP_TRY(c, upload(c->d_chunks, P.chunks, c->stream));
    HIP_TRY(c, upload(c->d_rinfo, P.rinfo, c->stream));
    HIP_TRY(c, upload(c->d_bmap, P.bmap, c->stream));
    HIP_TRY(c, upload(c->d_boffs, P.boffs, c->stream));
    HIP_TRY(c, upload(c->d_scat, P.scat, c->stream));
    HIP_TRY(c, upload(c->d_own, P.own_list, c->stream));
    const size_t ng = (size_t)std::max(P.ngroups, 1);
    HIP_TRY(c, c->d_scale.ensure(ng));
    HIP_TRY(c, c->d_done.ensure(ng));
    HIP_TRY(c, c->d_kfinal.ensure(ng));
    HIP_TRY(c, c->d_flags.ensure(ng));
    HIP_TRY(c, c->d_ndone.ensure(1));
    HIP_TRY(c, c->d_pe.ensure((size_t)std::max<int64_t>(c->nnzb, 1)));
    HIP_TRY(c, c->d_pn.ensure((size_t)std::max<int64_t>(c->nnzb, 1)));
    HIP_TRY(c, c->d_ne.ensure(2));
    HIP_TRY(c, hipStreamSynchronize(c->stream));   // host vectors may change after return
    c->plan_dirty = false;
    c->plan_gen++;
    return SMX_OK;
}

int32_t validate_values(smx_ctx c)
{
    HIP_TRY(c, c->d_check.ensure(2));
    HIP_TRY(c, hipMemsetAsync(c->d_check.p, 0, 2 * sizeof(double), c->stream));
    HIP_TRY(c, launch_check_values(c->stream, c->nnzb, c->d_valoff.p, c->d_brow.p, c->d_bcol.p,
                                   c->d_mirror.p, c->d_k.p, c->d_check.p));
    double h[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(h, c->d_check.p, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!std::isfinite(h[1])) return fail(c, SMX_E_NONFINITE, "K holds NaN or Inf values");
    if (h[0] > 1e-12 * h[1]) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "K is not symmetric: max|K_IJ - K_JI^T| = %.3e > 1e-12 * max|K| = %.3e",
                      h[0], 1e-12 * h[1]);
        return fail(c, SMX_E_NOT_SYMMETRIC, buf);
    }
    return SMX_OK;
}

int32_t copy_values_in(smx_ctx c, const double *values, int32_t on_device)
{
    HIP_TRY(c, c->d_k.ensure((size_t)std::max<int64_t>(c->nvals, 1)));
    HIP_TRY(c, c->d_d.ensure((size_t)std::max<int64_t>(c->nvals, 1)));
    if (c->nvals > 0)
        HIP_TRY(c, hipMemcpyAsync(c->d_k.p, values, (size_t)c->nvals * sizeof(double),
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    return SMX_OK;
}

int32_t set_device(smx_ctx c)
{
    HIP_TRY(c, hipSetDevice(c->device));
    return SMX_OK;
}

int32_t need_sync_results(smx_ctx c)
{
    if (!c->evaluated) return fail(c, SMX_E_STATE, "no evaluation has been run");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SMX_OK;
}

// Per-group state of a static-scratch evaluation stays in the shared scratch
// array, which any later static evaluation on the device overwrites.
int32_t need_group_state(smx_ctx c)
{
    if (c->evaluated && c->eval_static)
        return fail(c, SMX_E_STATE, "per-group results of smx_evaluate_static are not kept (D, N, E and the "
                                    "convergence status are)");
    return need_sync_results(c);
}

// FP64 polish of the reduced-precision modes on the own columns.  With
// A_0(Z) = X Z (X the bulk result, FP64) and A_j(Z) = X_{k+j} Z =
// 1.5 A_{j-1}(Z) - 0.5 A_{j-1}(A_{j-1}(A_{j-1}(Z))), the own columns of the
// p-times polished sign are A_p(E), E the own-column selector (A_0(E) is a
// gather).  Thin blocks come from a pool of 2p + 1; the residual
// max|X_{k+p-1}^2 E - E| is taken on the innermost square of the last step.
int32_t own_polish(smx_ctx c, const Plan &P, const DevView &V, double *pool, int32_t g0, int32_t wng,
                   const XSource &x, const IterState &it, int32_t *result)
{
    hipStream_t st = c->stream;
    const int32_t nbuf = 2 * c->n_polish + 1;
    char used[2 * kMaxPolishMixed + 1] = {0};
    const int slot = c->max_iter + c->n_polish;
    hipError_t herr = hipSuccess;
    struct Poly {
        // own columns of A_j(Z) for Z in buffer zi (zi < 0: the selector E);
        // returns the result's buffer, or -1
        const Plan &P;
        const DevView &V;
        hipStream_t st;
        int32_t g0, wng, slot;
        const XSource &x;
        const IterState &it;
        char *used;
        int nbuf;
        double *pool;
        hipError_t &herr;
        double *buf(int i) const { return pool + (size_t)i * (size_t)P.thin_elems; }
        int take()
        {
            for (int i = 0; i < nbuf; i++)
                if (!used[i]) {
                    used[i] = 1;
                    return i;
                }
            return -1;
        }
        int apply(int j, int zi, bool top)
        {
            if (herr != hipSuccess) return -1;
            if (j == 1) {
                const int a = take();
                if (a < 0) return -1;
                herr = zi < 0 ? launch_own_gather(st, g0, wng, P.max_npad, V.gd, V.own, x, buf(a))
                              : launch_thin_mul(st, 0, g0, wng, P.max_npad, P.max_own, V.gd, x, buf(zi), nullptr,
                                                buf(a));
                const int b = take();
                if (b < 0) return -1;
                if (herr == hipSuccess)
                    herr = launch_thin_mul(st, 0, g0, wng, P.max_npad, P.max_own, V.gd, x, buf(a), nullptr, buf(b));
                if (top && herr == hipSuccess)
                    herr = launch_thin_resid(st, g0, wng, P.max_npad, P.max_own, V.gd, V.own, buf(b), it, slot);
                const int out = take();
                if (out < 0) return -1;
                if (herr == hipSuccess)
                    herr = launch_thin_mul(st, 1, g0, wng, P.max_npad, P.max_own, V.gd, x, buf(b), buf(a), buf(out));
                used[a] = used[b] = 0;
                return out;
            }
            const int aa = apply(j - 1, zi, false);
            if (aa < 0) return -1;
            const int bb = apply(j - 1, aa, false);
            if (bb < 0) return -1;
            if (top && herr == hipSuccess)
                herr = launch_thin_resid(st, g0, wng, P.max_npad, P.max_own, V.gd, V.own, buf(bb), it, slot);
            const int cc = apply(j - 1, bb, false);
            if (cc < 0) return -1;
            used[bb] = 0;
            if (herr == hipSuccess)
                herr = launch_thin_combine(st, g0, wng, P.max_npad, P.max_own, V.gd, buf(aa), buf(cc));
            used[aa] = 0;
            return cc;
        }
    } poly{P, V, st, g0, wng, slot, x, it, used, nbuf, pool, herr};
    const int r = poly.apply(c->n_polish, -1, true);
    if (herr != hipSuccess)
        return fail(c, herr == hipErrorOutOfMemory ? SMX_E_NOMEM : SMX_E_HIP,
                    std::string("own-column polish: ") + hipGetErrorString(herr));
    if (r < 0) return fail(c, SMX_E_INVALID, "internal: own-column polish ran out of buffers");
    *result = r;
    return SMX_OK;
}

}  // namespace

extern "C" {

int32_t smx_create(int32_t device, smx_ctx *out)
{
    if (!out) {
        g_create_err = "out is NULL";
        return SMX_E_INVALID;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n) {
        g_create_err = "no HIP device " + std::to_string(device) + " (" + hipGetErrorString(e) + ")";
        return SMX_E_HIP;
    }
    smx_ctx c = new (std::nothrow) smx_context();
    if (!c) {
        g_create_err = "host allocation failed";
        return SMX_E_NOMEM;
    }
    c->device = device;
    c->uid = ++g_ctx_uid;
    e = hipSetDevice(device);
    if (e == hipSuccess) e = hipEventCreate(&c->ev_t0);
    if (e == hipSuccess) e = hipEventCreate(&c->ev_t3);
    if (e == hipSuccess) e = c->d_ne.ensure(2);
    if (e == hipSuccess) e = c->d_fsum.ensure(2);
    if (e == hipSuccess && device < kMaxDevices) {
        // the static scratch array's address on this device (once per device)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_tried[device]) {
            void *ptr = nullptr;
            const hipError_t se = hipGetSymbolAddress(&ptr, HIP_SYMBOL(smx_static_scratch));
            g_scratch_tried[device] = true;
            g_scratch_err[device] = se;
            g_scratch_ptr[device] = se == hipSuccess ? ptr : nullptr;
            if (se != hipSuccess) (void)hipGetLastError();
        }
    }
    if (e != hipSuccess) {
        g_create_err = std::string("HIP initialisation failed: ") + hipGetErrorString(e);
        delete c;
        return SMX_E_HIP;
    }
    *out = c;
    return SMX_OK;
}

int32_t smx_destroy(smx_ctx c)
{
    if (!c) return SMX_E_INVALID;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto *b : {&c->d_k, &c->d_d, &c->d_arena, &c->d_pe, &c->d_pn, &c->d_ne, &c->d_check})
        b->release();
    c->d_fsum.release();
    c->d_xidx.release();
    c->d_xout.release();
    c->d_plist.release();
    c->d_valoff.release();
    c->d_mirror.release();
    c->d_brow.release();
    c->d_bcol.release();
    c->d_gd.release();
    c->d_tiles.release();
    c->d_tiles_s.release();
    c->d_tiles_sx.release();
    c->d_xbeg.release();
    c->d_tq.release();
    c->d_tiles_b.release();
    c->d_chunks.release();
    c->d_rinfo.release();
    c->d_bmap.release();
    c->d_boffs.release();
    c->d_scat.release();
    c->d_scale.release();
    c->d_resid.release();
    c->d_done.release();
    c->d_kfinal.release();
    c->d_flags.release();
    c->d_ndone.release();
    c->d_own.release();
    c->d_tdiag.release();
    c->d_tau_hist.release();
    c->d_kfix.release();
    c->d_sfix.release();
    c->d_scale_scratch.release();
    c->d_tx0.release();
    c->d_tx1.release();
    c->d_dnp.release();
    c->d_dn.release();
    c->d_tiles_full.release();
    c->d_cptr.release();
    c->d_contrib.release();
    c->d_adj.release();
    c->d_dk.release();
    c->d_dmu.release();
    c->d_tpool.release();
    for (auto *b : {&c->d_ed, &c->d_ee, &c->d_etau, &c->d_elam, &c->d_elabs, &c->d_ew, &c->d_mus, &c->d_npart,
                    &c->d_nval})
        b->release();
    c->d_ebs.release();
    c->d_ebe.release();
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_ndone) (void)hipHostFree(c->h_ndone);
    for (hipEvent_t ev : c->ev_poll) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : c->ev_launch) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : c->ev_wave) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : {c->ev_t0, c->ev_t3})
        if (ev) (void)hipEventDestroy(ev);
    delete c;
    return SMX_OK;
}

const char *smx_last_error(smx_ctx c)
{
    if (!c) return g_create_err.c_str();
    return c->err.c_str();
}

int32_t smx_set_stream(smx_ctx c, void *hip_stream)
{
    if (!c) return SMX_E_INVALID;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return SMX_OK;
}

int32_t smx_load_k(smx_ctx c, int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr,
                   const int32_t *row_idx, const double *values, int32_t values_on_device)
{
    if (!c) return SMX_E_INVALID;
    c->loaded = false;
    c->evaluated = false;
    c->plan_dirty = true;
    c->splan_dirty = true;
    c->use_kfix = c->use_sfix = false;
    if (nblk <= 0 || !blk_size || !col_ptr || !row_idx || !values)
        return fail(c, SMX_E_INVALID, "nblk must be positive and all arrays non-NULL");
    if (int32_t st = set_device(c)) return st;
    for (int32_t j = 0; j < nblk; j++)
        if (blk_size[j] < 1 || blk_size[j] > 1024)
            return fail(c, SMX_E_INVALID, "block size out of range 1..1024 at block " + std::to_string(j));
    if (col_ptr[0] != 0) return fail(c, SMX_E_INVALID, "col_ptr[0] must be 0");
    for (int32_t j = 0; j < nblk; j++)
        if (col_ptr[j + 1] < col_ptr[j]) return fail(c, SMX_E_INVALID, "col_ptr must be non-decreasing");
    const int64_t nnzb = col_ptr[nblk];
    if (nnzb > (int64_t)INT32_MAX) return fail(c, SMX_E_INVALID, "more than 2^31-1 stored blocks");
    c->nblk = nblk;
    c->nnzb = nnzb;
    c->blk_size.assign(blk_size, blk_size + nblk);
    c->col_ptr.assign(col_ptr, col_ptr + nblk + 1);
    c->row_idx.assign(row_idx, row_idx + nnzb);
    c->val_off.assign((size_t)nnzb + 1, 0);
    std::vector<int32_t> brow((size_t)nnzb), bcol((size_t)nnzb);
    std::vector<int64_t> mirror((size_t)nnzb);
    for (int32_t j = 0; j < nblk; j++) {
        bool has_diag = false;
        for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++) {
            const int32_t i = row_idx[p];
            if (i < 0 || i >= nblk) return fail(c, SMX_E_INVALID, "row index out of range in column " + std::to_string(j));
            if (p > col_ptr[j] && row_idx[p - 1] >= i)
                return fail(c, SMX_E_INVALID, "row indices must ascend strictly in column " + std::to_string(j));
            if (i == j) has_diag = true;
            c->val_off[p + 1] = c->val_off[p] + (int64_t)blk_size[i] * blk_size[j];
            brow[p] = blk_size[i];
            bcol[p] = blk_size[j];
        }
        if (!has_diag) return fail(c, SMX_E_INVALID, "diagonal block missing in column " + std::to_string(j));
    }
    // mirror positions: block (J, I) for every stored (I, J); the pattern must be symmetric
    for (int32_t j = 0; j < nblk; j++)
        for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; p++) {
            const int32_t i = row_idx[p];
            const int32_t *lo = row_idx + col_ptr[i], *hi = row_idx + col_ptr[i + 1];
            const int32_t *f = std::lower_bound(lo, hi, j);
            if (f == hi || *f != j)
                return fail(c, SMX_E_NOT_SYMMETRIC, "pattern is not symmetric: block (" + std::to_string(i) + "," +
                                                        std::to_string(j) + ") stored without its mirror");
            mirror[p] = col_ptr[i] + (f - lo);
        }
    c->nvals = c->val_off[nnzb];
    HIP_TRY(c, upload(c->d_valoff, c->val_off, c->stream));
    HIP_TRY(c, upload(c->d_mirror, mirror, c->stream));
    HIP_TRY(c, upload(c->d_brow, brow, c->stream));
    HIP_TRY(c, upload(c->d_bcol, bcol, c->stream));
    if (int32_t st = copy_values_in(c, values, values_on_device)) return st;
    if (int32_t st = validate_values(c)) return st;
    // default grouping: one group per block column
    c->grp_ptr.resize((size_t)nblk + 1);
    c->grp_blocks.resize((size_t)nblk);
    for (int32_t j = 0; j <= nblk; j++) c->grp_ptr[j] = j;
    for (int32_t j = 0; j < nblk; j++) c->grp_blocks[j] = j;
    c->loaded = true;
    return SMX_OK;
}

int32_t smx_update_values(smx_ctx c, const double *values, int32_t values_on_device)
{
    if (!c) return SMX_E_INVALID;
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (!values) return fail(c, SMX_E_INVALID, "values is NULL");
    if (int32_t st = set_device(c)) return st;
    c->evaluated = false;
    if (int32_t st = copy_values_in(c, values, values_on_device)) return st;
    if (int32_t st = validate_values(c)) {
        c->loaded = false;
        return st;
    }
    return SMX_OK;
}

int32_t smx_set_groups(smx_ctx c, int32_t ngroups, const int32_t *grp_ptr, const int32_t *grp_blocks)
{
    if (!c) return SMX_E_INVALID;
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (ngroups <= 0 || !grp_ptr || !grp_blocks) return fail(c, SMX_E_INVALID, "need ngroups > 0 and arrays");
    if (grp_ptr[0] != 0 || grp_ptr[ngroups] != c->nblk)
        return fail(c, SMX_E_INVALID, "groups must cover every block column exactly once");
    std::vector<char> seen((size_t)c->nblk, 0);
    for (int32_t g = 0; g < ngroups; g++) {
        if (grp_ptr[g + 1] <= grp_ptr[g]) return fail(c, SMX_E_INVALID, "empty group " + std::to_string(g));
        for (int32_t q = grp_ptr[g]; q < grp_ptr[g + 1]; q++) {
            const int32_t j = grp_blocks[q];
            if (j < 0 || j >= c->nblk || seen[j])
                return fail(c, SMX_E_INVALID, "block column listed twice or out of range in group " + std::to_string(g));
            seen[j] = 1;
        }
    }
    c->grp_ptr.assign(grp_ptr, grp_ptr + ngroups + 1);
    c->grp_blocks.assign(grp_blocks, grp_blocks + c->nblk);
    c->plan_dirty = true;
    c->splan_dirty = true;
    c->evaluated = false;
    c->use_kfix = c->use_sfix = false;
    return SMX_OK;
}

int32_t smx_set_mu(smx_ctx c, double mu)
{
    if (!c) return SMX_E_INVALID;
    if (!std::isfinite(mu)) return fail(c, SMX_E_INVALID, "mu must be finite");
    c->mu = mu;
    return SMX_OK;
}

int32_t smx_set_temperature(smx_ctx c, double kT)
{
    if (!c) return SMX_E_INVALID;
    if (!(kT >= 0.0) || !std::isfinite(kT)) return fail(c, SMX_E_INVALID, "kT must be finite and >= 0");
    c->kT = kT;
    return SMX_OK;
}

int32_t smx_set_precision(smx_ctx c, int32_t mode)
{
    if (!c) return SMX_E_INVALID;
    if (mode < SMX_FP64 || mode > SMX_FP16_2W) return fail(c, SMX_E_INVALID, "unknown precision mode");
    c->precision = mode;
    return SMX_OK;
}

int32_t smx_set_convergence(smx_ctx c, double tol, int32_t max_iter, int32_t n_polish, double switch_tol)
{
    if (!c) return SMX_E_INVALID;
    if (!(tol > 0.0) || max_iter < 1 || max_iter > 1000 || n_polish < 1 || n_polish > 10 || !(switch_tol > 0.0))
        return fail(c, SMX_E_INVALID, "need tol > 0, 1 <= max_iter <= 1000, 1 <= n_polish <= 10, switch_tol > 0");
    c->tol = tol;
    c->max_iter = max_iter;
    c->n_polish = n_polish;
    c->switch_tol = switch_tol;
    return SMX_OK;
}

int32_t smx_set_graph(smx_ctx c, int32_t steps_per_graph)
{
    if (!c) return SMX_E_INVALID;
    if (steps_per_graph < 0 || steps_per_graph > 64) return fail(c, SMX_E_INVALID, "steps_per_graph must be 0..64");
    if (int32_t st = set_device(c)) return st;
    if (steps_per_graph != c->graph_steps) drop_graphs(c);
    c->graph_steps = steps_per_graph;
    return SMX_OK;
}

int32_t smx_set_tile_order(smx_ctx c, int32_t order)
{
    if (!c) return SMX_E_INVALID;
    if (order != 0 && order != 1) return fail(c, SMX_E_INVALID, "order must be 0 (XCD-aware) or 1 (group by group)");
    if (order != c->tile_order) {
        c->tile_order = order;
        c->plan_dirty = true;
        c->splan_dirty = true;
        c->evaluated = false;
        c->contrib_ready = false;
    }
    return SMX_OK;
}

int32_t smx_set_debug_checks(smx_ctx c, int32_t on)
{
    if (!c) return SMX_E_INVALID;
    if (on != 0 && on != 1) return fail(c, SMX_E_INVALID, "on must be 0 or 1");
    c->debug_checks = on;
    c->guards_armed = false;
    return SMX_OK;
}

int32_t smx_set_kernel_variant(smx_ctx c, int32_t variant)
{
    if (!c) return SMX_E_INVALID;
    if (variant < 0 || variant > 2) return fail(c, SMX_E_INVALID, "variant must be 0, 1 or 2");
    if (variant != c->kernel_variant) drop_graphs(c);
    c->kernel_variant = variant;
    return SMX_OK;
}

int32_t smx_set_solver(smx_ctx c, int32_t solver)
{
    if (!c) return SMX_E_INVALID;
    if (solver != SMX_SOLVER_ITERATIVE && solver != SMX_SOLVER_EIG) return fail(c, SMX_E_INVALID, "unknown solver");
    c->solver = solver;
    return SMX_OK;
}

int32_t smx_set_iteration(smx_ctx c, int32_t kind)
{
    if (!c) return SMX_E_INVALID;
    if (kind != SMX_ITER_NS2 && kind != SMX_ITER_PADE3) return fail(c, SMX_E_INVALID, "unknown sign iteration");
    if (kind != c->iteration) drop_graphs(c);
    c->iteration = kind;
    return SMX_OK;
}

int32_t smx_set_tile_shape(smx_ctx c, int32_t big_min_npad)
{
    if (!c) return SMX_E_INVALID;
    if (big_min_npad < 0) return fail(c, SMX_E_INVALID, "big_min_npad must be >= 0");
    if (big_min_npad != c->big_min_npad) {
        c->big_min_npad = big_min_npad;
        c->plan_dirty = true;
        c->splan_dirty = true;
        c->evaluated = false;
        c->contrib_ready = false;
    }
    return SMX_OK;
}

int32_t smx_get_launch_config(smx_ctx c, int32_t *graph_steps, int32_t *tile_order, int32_t *big_min_npad,
                              int32_t *kernel_variant)
{
    if (!c) return SMX_E_INVALID;
    if (graph_steps) *graph_steps = c->graph_steps;
    if (tile_order) *tile_order = c->tile_order;
    if (big_min_npad) *big_min_npad = c->big_min_npad;
    if (kernel_variant) *kernel_variant = c->kernel_variant;
    return SMX_OK;
}

int32_t smx_set_workspace_limit(smx_ctx c, int64_t bytes)
{
    if (!c) return SMX_E_INVALID;
    if (bytes < 0) return fail(c, SMX_E_INVALID, "bytes must be >= 0");
    c->ws_limit = bytes;
    c->plan_dirty = true;
    c->evaluated = false;
    c->use_kfix = c->use_sfix = false;
    c->contrib_ready = false;
    return SMX_OK;
}

}  // extern "C"

namespace {

// Settings of one evaluation, derived from the context.
struct EvalMode {
    int fmt = -1, nw = 0;          // storage of the reduced-precision bulk (fmt < 0: FP64)
    bool mixed = false;
    bool pade = false;             // third-order Pade steps (three products) instead of Newton-Schulz
    bool eig = false;              // diagonalisation path (kT > 0, or SMX_SOLVER_EIG)
    bool tangent = false;          // the mu tangent rides along (frozen step counts)
    int32_t stride = 0;            // residual / tau history slots per group
    int32_t kmax = 0;              // last bulk step
};

int32_t eval_mode(smx_ctx c, EvalMode &m)
{
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    m.eig = c->kT > 0.0 || c->solver == SMX_SOLVER_EIG;
    if (m.eig) {
        if (c->precision != SMX_FP64)
            return fail(c, SMX_E_UNSUPPORTED, "the diagonalisation path (kT > 0 or SMX_SOLVER_EIG) runs in SMX_FP64");
        if (c->use_kfix || c->use_sfix)
            return fail(c, SMX_E_UNSUPPORTED, "frozen iteration (derivatives, mu search) follows the Newton-Schulz map");
        m.stride = c->max_iter + 2 + c->n_polish;
        return SMX_OK;
    }
    switch (c->precision) {
    case SMX_FP64: break;
    case SMX_FP16_2W: m.fmt = 0; m.nw = 2; break;
    case SMX_BF16_3W: m.fmt = 1; m.nw = 3; break;
    case SMX_BF16_1W: m.fmt = 1; m.nw = 1; break;
    case SMX_FP32: m.fmt = 2; m.nw = 2; break;       // one FP32 value = two 16-bit storage units
    default: return fail(c, SMX_E_UNSUPPORTED, "precision mode not implemented on the GPU path");
    }
    m.mixed = m.fmt >= 0;
    m.pade = c->iteration == SMX_ITER_PADE3;
    const bool frozen = c->use_kfix || c->use_sfix;
    if (frozen && m.pade)
        return fail(c, SMX_E_UNSUPPORTED, "frozen iteration (derivatives, mu search) follows the Newton-Schulz map only");
    if (frozen && m.mixed)
        return fail(c, SMX_E_UNSUPPORTED, "frozen iteration (derivatives, mu search) runs in SMX_FP64 only");
    if (m.mixed && c->max_iter <= c->n_polish)
        return fail(c, SMX_E_INVALID, "max_iter must exceed n_polish in reduced-precision modes");
    if (m.mixed && c->n_polish > kMaxPolishMixed)
        return fail(c, SMX_E_INVALID, "n_polish above " + std::to_string(kMaxPolishMixed) +
                                          " in a reduced-precision mode (the own-column polish costs 3^n_polish - 1 "
                                          "passes over each submatrix)");
    m.tangent = c->use_kfix;
    m.stride = c->max_iter + 2 + c->n_polish;
    m.kmax = m.mixed ? c->max_iter - c->n_polish : c->max_iter;
    return SMX_OK;
}

// Every allocation an evaluation needs except the arena and the polish pool:
// the plan, per-group state and histories, the pinned polling buffer, events,
// and the tangent buffers of frozen evaluations.
int32_t eval_prepare(smx_ctx c, const EvalMode &m)
{
    if (int32_t st = ensure_plan(c)) return st;
    const Plan &P = c->plan;
    const int32_t ng = P.ngroups;
    HIP_TRY(c, c->d_resid.ensure((size_t)ng * m.stride));
    HIP_TRY(c, c->d_tdiag.ensure(std::max<size_t>(P.rinfo.size(), 1)));
    HIP_TRY(c, c->d_tau_hist.ensure((size_t)ng * m.stride));
    if (c->h_ndone_cap < m.stride) {
        if (c->h_ndone) (void)hipHostFree(c->h_ndone);
        c->h_ndone = nullptr;
        c->h_ndone_cap = 0;
        HIP_TRY(c, hipHostMalloc(reinterpret_cast<void **>(&c->h_ndone), sizeof(int32_t) * m.stride));
        c->h_ndone_cap = m.stride;
    }
    while ((int32_t)c->ev_poll.size() < m.stride) {
        hipEvent_t ev;
        HIP_TRY(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        c->ev_poll.push_back(ev);
    }
    while ((int32_t)c->ev_wave.size() < 4 * P.nwaves()) {
        hipEvent_t ev;
        HIP_TRY(c, hipEventCreate(&ev));
        c->ev_wave.push_back(ev);
    }
    if (c->use_sfix) HIP_TRY(c, c->d_scale_scratch.ensure((size_t)std::max(ng, 1)));
    if (m.eig) {
        if (P.max_npad > kEigMaxN)
            return fail(c, SMX_E_UNSUPPORTED, "the diagonalisation path takes submatrices up to n = " +
                                                  std::to_string(kEigMaxN));
        const size_t nr = std::max<size_t>(P.rinfo.size(), 1);
        for (auto *b : {&c->d_ed, &c->d_ee, &c->d_etau, &c->d_elam, &c->d_elabs, &c->d_ew}) HIP_TRY(c, b->ensure(nr));
        HIP_TRY(c, c->d_ebs.ensure(nr));
        HIP_TRY(c, c->d_ebe.ensure(nr));
    }
    if (m.tangent) {
        HIP_TRY(c, c->d_tx0.ensure((size_t)P.work_elems));
        HIP_TRY(c, c->d_tx1.ensure((size_t)P.work_elems));
        HIP_TRY(c, c->d_dnp.ensure((size_t)std::max(ng, 1)));
        HIP_TRY(c, c->d_dn.ensure(2));
    }
    return SMX_OK;
}

// The library's own arena (and polish pool) when the caller set no work space.
int32_t ensure_arena(smx_ctx c, bool pool)
{
    if (c->ws_ptr) return SMX_OK;
    const Plan &P = c->plan;
    const size_t guard = c->debug_checks ? kGuardElems : 0;
    HIP_TRY(c, c->d_arena.ensure((size_t)(arena_bytes(P) / 8) + guard));
    if (pool)
        HIP_TRY(c, c->d_tpool.ensure((size_t)(2 * c->n_polish + 1) * (size_t)std::max<int64_t>(P.thin_elems, 1) +
                                     guard));
    return SMX_OK;
}

// ---- debug checks (smx_set_debug_checks) -------------------------------------
// Host validation of every plan table against the sizes it indexes, and guard
// regions of kGuardElems doubles, filled with a byte pattern, right after the
// extent an evaluation may write in the arena, the polish pool and D; smx_wait
// reads them back and reports any changed byte.

bool plan_tables_valid(const Plan &P, int64_t nnzb, int32_t big_tile, std::string &why)
{
    auto bad = [&](const std::string &s) {
        why = s;
        return false;
    };
    const int32_t ng = P.ngroups;
    for (int32_t g = 0; g < ng; g++) {
        const GroupDesc &d = P.gd[g];
        const std::string tag = "group " + std::to_string(g) + ": ";
        if (d.npad % 32 || d.n < 1 || d.n > d.npad || d.npad > P.max_npad) return bad(tag + "dimensions");
        if (d.off < 0 || d.off + (int64_t)d.npad * d.npad > P.work_elems) return bad(tag + "slab beyond the arena");
        if (d.thin_off < 0 || d.thin_off + (int64_t)d.npad * d.m_own > std::max<int64_t>(P.thin_elems, 1))
            return bad(tag + "own-column block beyond the pool");
        if (d.rinfo_off < 0 || d.rinfo_off + d.npad > (int64_t)P.rinfo.size()) return bad(tag + "row table");
        if (d.own_off < 0 || d.own_off + d.m_own > (int64_t)P.own_list.size() || d.m_own > P.max_own)
            return bad(tag + "own-column list");
        for (int32_t c = 0; c < d.m_own; c++)
            if (P.own_list[d.own_off + c] < 0 || P.own_list[d.own_off + c] >= d.n) return bad(tag + "own column");
        if (d.map_off < 0 || d.map_off + (int64_t)d.m * d.m > (int64_t)P.bmap.size()) return bad(tag + "block map");
        for (int64_t q = 0; q < (int64_t)d.m * d.m; q++) {
            const int32_t v = P.bmap[d.map_off + q];
            if (v < -1 || v >= nnzb) return bad(tag + "block map entry");
        }
        if (d.boff_off < 0 || d.boff_off + d.m + 1 > (int64_t)P.boffs.size()) return bad(tag + "block offsets");
        if (P.boffs[d.boff_off] != 0 || P.boffs[d.boff_off + d.m] != d.n) return bad(tag + "block offsets");
        for (int32_t b = 0; b < d.m; b++)
            if (P.boffs[d.boff_off + b + 1] <= P.boffs[d.boff_off + b]) return bad(tag + "block offsets");
        for (int32_t r = 0; r < d.n; r++) {
            const RowInfo ri = P.rinfo[d.rinfo_off + r];
            if (ri.x < 0 || ri.x >= d.m || (ri.y & 0xffff) >= (ri.y >> 16)) return bad(tag + "row table entry");
        }
    }
    auto tiles_ok = [&](const std::vector<TileDesc> &tl, int tile, const char *name) {
        for (const TileDesc &td : tl) {
            if (td.x < 0) continue;                              // idle slot
            if (td.x >= ng) return bad(std::string(name) + ": group out of range");
            const int32_t ti = td.y >> 16, tj = td.y & 0xffff, nt = (P.gd[td.x].npad + tile - 1) / tile;
            if (ti >= nt || tj > ti) return bad(std::string(name) + ": tile outside the lower triangle");
        }
        return true;
    };
    if (!tiles_ok(P.tiles, kTile, "tiles") || !tiles_ok(P.tiles_s, kTile, "128-tiles") ||
        !tiles_ok(P.tiles_b, big_tile, "256-tiles"))
        return false;
    for (const int2 &ch : P.chunks)
        if (ch.x < 0 || ch.x >= ng || ch.y < 0 || ch.y >= P.gd[ch.x].npad) return bad("gather chunk out of range");
    for (size_t q = 0; q < P.scat.size(); q++) {
        const ScatterDesc &s = P.scat[q];
        if (s.g < 0 || s.g >= ng) return bad("scatter descriptor " + std::to_string(q) + ": group");
        const GroupDesc &d = P.gd[s.g];
        const int32_t bi = s.bij & 0xffff, bj = s.bij >> 16;
        if (s.oi < 0 || s.oi + bi > d.n || s.oj < 0 || s.oj + bj > d.n || s.ocol < 0 || s.ocol + bj > d.m_own)
            return bad("scatter descriptor " + std::to_string(q) + ": block outside its submatrix");
    }
    return true;
}

constexpr unsigned char kGuardByte = 0xA5;

int32_t arm_guards(smx_ctx c, bool pool)
{
    c->guards_armed = false;
    if (!c->debug_checks) return SMX_OK;
    std::string why;
    if (!plan_tables_valid(c->plan, c->nnzb, kTile2, why)) return fail(c, SMX_E_INVALID, "debug check: plan table: " + why);
    HIP_TRY(c, c->d_d.ensure((size_t)std::max<int64_t>(c->nvals, 1) + kGuardElems));
    HIP_TRY(c, hipMemsetAsync(c->d_d.p + c->nvals, kGuardByte, kGuardElems * 8, c->stream));
    if (!c->ws_ptr) {
        HIP_TRY(c, hipMemsetAsync(c->d_arena.p + arena_bytes(c->plan) / 8, kGuardByte, kGuardElems * 8, c->stream));
        if (pool) {
            const size_t used = (size_t)(2 * c->n_polish + 1) * (size_t)std::max<int64_t>(c->plan.thin_elems, 1);
            HIP_TRY(c, hipMemsetAsync(c->d_tpool.p + used, kGuardByte, kGuardElems * 8, c->stream));
        }
    }
    c->guards_armed = true;
    return SMX_OK;
}

int32_t check_guards(smx_ctx c)
{
    if (!c->guards_armed) return SMX_OK;
    c->guards_armed = false;
    std::vector<unsigned char> h(kGuardElems * 8);
    struct G {
        const double *p;
        const char *name;
    };
    std::vector<G> gs = {{c->d_d.p + c->nvals, "D"}};
    if (!c->ws_ptr) {
        gs.push_back({c->d_arena.p + arena_bytes(c->plan) / 8, "arena"});
        if (c->d_tpool.p && c->d_tpool.cap >= (size_t)(2 * c->n_polish + 1) *
                                                   (size_t)std::max<int64_t>(c->plan.thin_elems, 1) + kGuardElems)
            gs.push_back({c->d_tpool.p + (size_t)(2 * c->n_polish + 1) * (size_t)std::max<int64_t>(c->plan.thin_elems, 1),
                          "polish pool"});
    }
    for (const G &g : gs) {
        HIP_TRY(c, hipMemcpy(h.data(), g.p, h.size(), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < h.size(); i++)
            if (h[i] != kGuardByte)
                return fail(c, SMX_E_HIP, std::string("debug check: the guard after the ") + g.name +
                                              " was overwritten at byte " + std::to_string(i));
    }
    return SMX_OK;
}

DevView ctx_view(smx_ctx c)
{
    DevView v;
    v.gd = c->d_gd.p;
    v.tiles = c->d_tiles.p;
    v.tiles_s = c->d_tiles_s.p;
    v.tiles_b = c->d_tiles_b.p;
    v.tiles_sx = c->d_tiles_sx.p;
    v.xbeg = c->d_xbeg.p;
    v.chunks = c->d_chunks.p;
    v.rinfo = c->d_rinfo.p;
    v.bmap = c->d_bmap.p;
    v.boffs = c->d_boffs.p;
    v.own = c->d_own.p;
    v.scat = c->d_scat.p;
    v.plist = c->d_plist.p;
    v.scale = c->d_scale.p;
    v.resid = c->d_resid.p;
    v.done = c->d_done.p;
    v.kfinal = c->d_kfinal.p;
    v.flags = c->d_flags.p;
    v.ndone = c->d_ndone.p;
    v.tdiag = c->d_tdiag.p;
    v.tau_hist = c->d_tau_hist.p;
    v.pe = c->d_pe.p;
    v.pn = c->d_pn.p;
    v.ne = c->d_ne.p;
    return v;
}

// Enqueue one evaluation on the context's stream.  `arena` holds the largest
// wave's three slabs (or the words of three iterates from byte 8E), `pool`
// the own-column blocks of the polish (2 n_polish + 1 of them).  With
// `timing`, HIP events bracket every product launch (smx_get_launch_profile);
// `graphs` allows the step graphs of smx_set_graph.  Nothing is allocated
// here unless `timing` or `graphs` ask for events or graph captures.
int32_t eval_enqueue(smx_ctx c, const EvalMode &m, const Plan &P, const DevView &V, double *arena, double *pool,
                     bool timing, bool graphs, bool events, bool poll)
{
    const int32_t ng = P.ngroups;
    const int32_t fmt = m.fmt, nw = m.nw;
    const bool mixed = m.mixed, tangent = m.tangent, pade = m.pade;
    const int32_t stride = m.stride, kmax = m.kmax;
    const int32_t nwave = P.nwaves();
    hipStream_t st = c->stream;
    IterState it;
    it.scale_bits = V.scale;
    it.resid_bits = V.resid;
    it.done = V.done;
    it.kfinal = V.kfinal;
    it.flags = V.flags;
    it.ndone = V.ndone;
    it.kfix = c->use_kfix ? c->d_kfix.p : nullptr;
    it.kact = -1;
    it.tdiag = V.tdiag;
    it.tau_hist = V.tau_hist;
    it.resid_stride = stride;
    if (c->use_sfix) it.scale_bits = c->d_sfix.p;           // the kernels read the frozen scales
    unsigned long long *gather_scale = c->use_sfix ? c->d_scale_scratch.p : it.scale_bits;
    TraceScope tr;
    if (events) HIP_TRY(c, hipEventRecord(c->ev_t0, st));
    HIP_TRY(c, hipMemsetAsync(gather_scale, 0, sizeof(unsigned long long) * ng, st));
    HIP_TRY(c, hipMemsetAsync(it.resid_bits, 0, sizeof(unsigned long long) * (size_t)ng * stride, st));
    HIP_TRY(c, hipMemsetAsync(it.done, 0, sizeof(int32_t) * ng, st));
    HIP_TRY(c, hipMemsetAsync(it.kfinal, 0, sizeof(int32_t) * ng, st));
    HIP_TRY(c, hipMemsetAsync(it.flags, 0, sizeof(int32_t) * ng, st));

    c->launch_step.clear();
    c->launch_kind.clear();
    c->launch_wave.clear();
    c->launch_subset.clear();
    int32_t wave = 0;
    int32_t subset = 0;
    auto timed = [&](int kind, int k, auto &&launch) -> hipError_t {
        const size_t idx = c->launch_step.size();
        while (c->ev_launch.size() < 2 * (idx + 1)) {
            hipEvent_t ev;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return e;
            c->ev_launch.push_back(ev);
        }
        hipError_t e = hipEventRecord(c->ev_launch[2 * idx], st);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(c->ev_launch[2 * idx + 1], st);
        c->launch_step.push_back(k);
        c->launch_kind.push_back(kind);
        c->launch_wave.push_back(wave);
        c->launch_subset.push_back(subset);
        return e;
    };
    const int64_t welems = P.work_elems;        // an operand's words take nw * welems 16-bit units
    double *xb[2] = {arena, arena + welems};
    double *wslab = arena + 2 * welems;
    unsigned short *wbase = reinterpret_cast<unsigned short *>(arena + welems);
    unsigned short *wb[2] = {wbase, wbase + (size_t)nw * welems};
    unsigned short *wwp = wbase + (size_t)2 * nw * welems;
    double *tb[2] = {c->d_tx0.p, c->d_tx1.p};
    double *thin_result = nullptr;
    int32_t launched = 0;
    const bool use_graphs = graphs && c->graph_steps > 0;
    // the register-prefetch stream indexes a group's words with 32-bit offsets
    const int32_t variant =
        (c->kernel_variant == 1 && (int64_t)std::max(nw, 1) * P.max_npad * P.max_npad < (int64_t)INT32_MAX) ? 1 : 0;
    // persistent word products (variant 2): Newton-Schulz, 2-word FP16 or
    // 1-word BF16, the 128 x 128 bucket, context buffers (not the static array)
    const bool persistent = c->kernel_variant == 2 && mixed && !pade && !tangent && V.tiles_sx &&
                            ((fmt == 0 && nw == 2) || (fmt == 1 && nw == 1));
    int32_t pers_nwg = 0;
    if (persistent) {
        if (c->pers_nwg <= 0) {
            hipDeviceProp_t prop;
            HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
            c->pers_nwg = prop.multiProcessorCount * words_persistent_blocks_per_cu(fmt, nw);
        }
        pers_nwg = c->pers_nwg;
        HIP_TRY(c, c->d_tq.ensure((size_t)(kmax + 1) * 16));
    }
    if (use_graphs) {
        // replayable step graphs: valid while everything baked into their
        // launches (plan, buffers, mode and convergence settings) is unchanged
        if (!c->cap_stream) HIP_TRY(c, hipStreamCreate(&c->cap_stream));
        const std::vector<uint64_t> sig = {
            c->plan_gen, (uint64_t)c->precision, (uint64_t)c->max_iter, (uint64_t)c->n_polish,
            (uint64_t)c->graph_steps, (uint64_t)tangent, (uint64_t)c->use_sfix, (uint64_t)c->use_kfix,
            (uint64_t)c->kernel_variant, (uint64_t)pade, (uint64_t)(uintptr_t)arena, (uint64_t)(uintptr_t)c->d_tx0.p, (uint64_t)(uintptr_t)c->d_tx1.p,
            (uint64_t)(uintptr_t)c->d_resid.p, (uint64_t)(uintptr_t)c->d_tdiag.p, (uint64_t)(uintptr_t)c->d_tau_hist.p,
            (uint64_t)(uintptr_t)c->d_sfix.p, (uint64_t)(uintptr_t)c->d_kfix.p,
            __builtin_bit_cast(uint64_t, c->tol), __builtin_bit_cast(uint64_t, c->switch_tol)};
        const size_t ngraph = (size_t)nwave * (size_t)(kmax / c->graph_steps + 1);
        if (sig != c->graph_sig || c->graphs.size() != ngraph) {
            drop_graphs(c);
            c->graph_sig = sig;
            c->graphs.assign(ngraph, nullptr);
        }
    }
    // waves run one after the other through the same arena; every group's
    // arithmetic is independent of the wave it falls in
    for (wave = 0; wave < nwave; wave++) {
        const int32_t g0 = P.wave_g[wave], wng = P.wave_g[wave + 1] - g0;
        const int ntiles = (int)(P.tile_beg[wave + 1] - P.tile_beg[wave]);
        const TileDesc *tl = V.tiles + P.tile_beg[wave];
        // one- and two-word products: the size buckets (128 x 128 and 256 x 256 tiles)
        const bool buckets = mixed && fmt != 2 && nw <= 2;
        const int nts = (int)(P.tiles_s_beg[wave + 1] - P.tiles_s_beg[wave]);
        const int ntb = (int)(P.tiles_b_beg[wave + 1] - P.tiles_b_beg[wave]);
        const TileDesc *tls = V.tiles_s + P.tiles_s_beg[wave], *tlb = V.tiles_b + P.tiles_b_beg[wave];
        tr.push("smx gather");
        if (events) HIP_TRY(c, hipEventRecord(c->ev_wave[4 * wave], st));
        HIP_TRY(c, hipMemsetAsync(it.ndone, 0, sizeof(int32_t), st));
        if (persistent)                         // the step launches (or their graphs) take fresh counters
            HIP_TRY(c, hipMemsetAsync(c->d_tq.p, 0, sizeof(int32_t) * (size_t)(kmax + 1) * 16, st));
        const int nch = (int)(P.chunk_beg[wave + 1] - P.chunk_beg[wave]);
        const int2 *chs = V.chunks + P.chunk_beg[wave];
        if (!mixed) {
            HIP_TRY(c, launch_gather(st, nch, chs, V.gd, V.rinfo, V.bmap, V.boffs, c->d_valoff.p,
                                     c->d_k.p, c->mu, xb[0], gather_scale));
        } else {
            // bounds first, then X_0 straight into the words (no FP64 copy of A_g)
            HIP_TRY(c, launch_gather_bound(st, nch, chs, V.gd, V.rinfo, V.bmap, V.boffs,
                                           c->d_valoff.p, c->d_k.p, c->mu, gather_scale));
            HIP_TRY(c, launch_gather_words(st, fmt, nw, nch, chs, V.gd, V.rinfo, V.bmap, V.boffs,
                                           c->d_valoff.p, c->d_k.p, c->mu, it.scale_bits, wb[0]));
        }
        if (tangent) HIP_TRY(c, launch_tangent_init(st, g0, wng, P.max_npad, V.gd, it.scale_bits, tb[0]));
        if (events) HIP_TRY(c, hipEventRecord(c->ev_wave[4 * wave + 1], st));
        tr.next("smx iterate");
        // one Newton-Schulz step of the wave on stream s (timed: HIP events around
        // each product launch; not inside a graph capture)
        auto step = [&](hipStream_t s, int32_t k, bool time_it) -> hipError_t {
            auto run = [&](int kind, auto &&launch) -> hipError_t { return time_it ? timed(kind, k, launch) : launch(); };
            hipError_t e = hipSuccess;
            // Newton-Schulz: square (W = 1.5 I - 0.5 X^2), update X W.  Pade:
            // square (T = X^2, into the buffer X_{k+1} will take), combine
            // (W = (15 I - 10 T + 3 T^2) / 8), update X W.
            if (!mixed) {
                if (!pade) {
                    e = run(0, [&] { return launch_ns_f64(s, 0, ntiles, tl, V.gd, xb[k & 1], xb[k & 1], wslab, it, k,
                                                          c->tol, c->max_iter, 0); });
                } else {
                    double *tt = xb[(k + 1) & 1];
                    e = run(0, [&] { return launch_ns_f64(s, 5, ntiles, tl, V.gd, xb[k & 1], xb[k & 1], tt, it, k,
                                                          c->tol, c->max_iter, 0); });
                    if (e == hipSuccess)
                        e = run(11, [&] { return launch_ns_f64(s, 6, ntiles, tl, V.gd, tt, tt, wslab, it, k, c->tol,
                                                               c->max_iter, 0); });
                }
                if (e == hipSuccess)
                    e = run(1, [&] { return launch_ns_f64(s, 1, ntiles, tl, V.gd, xb[k & 1], wslab, xb[(k + 1) & 1],
                                                          it, k, c->tol, c->max_iter, 0); });
                if (e == hipSuccess && tangent)
                    e = run(6, [&] { return launch_ns_f64(s, 2, ntiles, tl, V.gd, tb[k & 1], wslab, tb[(k + 1) & 1],
                                                          it, k, c->tol, c->max_iter, 0); });
            } else {
                // one launch per size bucket and product (one bucket of all
                // groups on 128 x 128 tiles when the mode has no 256 x 256 kernel)
                struct Bucket {
                    int n;
                    const TileDesc *tl;
                    bool big;
                    int sub;
                };
                const Bucket bk[2] = {buckets ? Bucket{nts, tls, false, 1} : Bucket{ntiles, tl, false, 0},
                                      Bucket{buckets ? ntb : 0, tlb, true, 2}};
                unsigned short *tw = wb[(k + 1) & 1];
                auto prod = [&](const Bucket &b, int mode, int kind128, int kind256, const unsigned short *x,
                                const unsigned short *y, unsigned short *o) -> hipError_t {
                    if (b.n <= 0) return hipSuccess;
                    subset = b.sub;
                    hipError_t r;
                    if (b.big)
                        r = run(kind256, [&] { return launch_ns_words256(s, fmt, nw, mode, b.n, b.tl, V.gd, x, y, o, it,
                                                                         k, c->switch_tol, kmax); });
                    else if (persistent && mode <= 1)
                        r = run(kind128, [&] {
                            return launch_ns_words_persistent(s, fmt, nw, mode, pers_nwg, V.tiles_sx + P.sx_wbeg[wave],
                                                              V.xbeg + 9 * wave, c->d_tq.p + ((size_t)k * 2 + mode) * 8,
                                                              V.gd, x, y, o, it, k, c->switch_tol, kmax);
                        });
                    else
                        r = run(kind128, [&] { return launch_ns_words(s, fmt, nw, mode, mode <= 1 ? variant : 0, b.n,
                                                                      b.tl, V.gd, x, y, o, it, k, c->switch_tol, kmax); });
                    subset = 0;
                    return r;
                };
                // squares of both buckets, then (Pade) their combines, then their
                // updates: a group's products keep their order, and the groups
                // are independent
                for (const Bucket &b : bk)
                    if (e == hipSuccess) e = pade ? prod(b, 2, 2, 7, wb[k & 1], wb[k & 1], tw)
                                                  : prod(b, 0, 2, 7, wb[k & 1], wb[k & 1], wwp);
                if (pade)
                    for (const Bucket &b : bk)
                        if (e == hipSuccess) e = prod(b, 3, 9, 10, tw, tw, wwp);
                for (const Bucket &b : bk)
                    if (e == hipSuccess) e = prod(b, 1, 3, 8, wb[k & 1], wwp, wb[(k + 1) & 1]);
            }
            return e;
        };
        // bulk steps: every group iterates until its own stopping rule.  With
        // host polling, the host reads the wave's finished-group counter one
        // step (or one graph of graph_steps steps) behind the device and stops
        // launching once all are done; without, every step up to the cap is
        // enqueued and finished groups skip on the device
        const int32_t S = use_graphs ? c->graph_steps : 1;
        const int32_t nchunk = kmax / S + 1;
        for (int32_t ch = 0; ch < nchunk; ch++) {
            const int32_t k0 = ch * S, k1 = std::min(k0 + S - 1, kmax);
            if (use_graphs) {
                hipGraphExec_t &ex = c->graphs[(size_t)wave * nchunk + ch];
                if (!ex) {
                    // capture on the private stream (capture does not run anything)
                    hipGraph_t gr = nullptr;
                    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                    hipError_t e = hipSuccess;
                    for (int32_t k = k0; k <= k1 && e == hipSuccess; k++) e = step(c->cap_stream, k, false);
                    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &gr);
                    HIP_TRY(c, e);
                    HIP_TRY(c, e2);
                    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(gr);
                    HIP_TRY(c, e);
                }
                HIP_TRY(c, hipGraphLaunch(ex, st));
            } else {
                HIP_TRY(c, step(st, k0, timing));
            }
            launched = std::max(launched, k1 + 1);
            if (poll) {
                HIP_TRY(c, hipMemcpyAsync(c->h_ndone + ch, it.ndone, sizeof(int32_t), hipMemcpyDeviceToHost, st));
                HIP_TRY(c, hipEventRecord(c->ev_poll[ch], st));
                if (ch >= 1) {
                    HIP_TRY(c, hipEventSynchronize(c->ev_poll[ch - 1]));
                    if (c->h_ndone[ch - 1] >= wng) break;
                }
            }
        }
        if (mixed) {
            // FP64 polish on the own columns: X_{k+p} E from the bulk result X,
            // read from its words (converted exactly on the fly)
            const XSource xs{nullptr, wb[0], wb[1], it.kfinal, fmt, nw};
            int32_t res = -1;
            tr.next("smx polish");
            if (int32_t e = own_polish(c, P, V, pool, g0, wng, xs, it, &res)) return e;
            thin_result = pool + (size_t)res * (size_t)P.thin_elems;
            HIP_TRY(c, launch_polish_flags(st, g0, wng, it, c->max_iter + c->n_polish, c->tol));
        }
        if (events) HIP_TRY(c, hipEventRecord(c->ev_wave[4 * wave + 2], st));
        tr.next("smx scatter");
        const int64_t nsc = nwave > 1 ? P.plist_beg[wave + 1] - P.plist_beg[wave] : c->nnzb;
        const int64_t *pl = nwave > 1 ? V.plist + P.plist_beg[wave] : nullptr;
        if (mixed)
            HIP_TRY(c, launch_scatter(st, nsc, pl, V.scat, c->d_valoff.p, V.gd, thin_result, nullptr, it,
                                      c->d_k.p, c->d_d.p, V.pe, V.pn, 1));
        else
            HIP_TRY(c, launch_scatter(st, nsc, pl, V.scat, c->d_valoff.p, V.gd, xb[0], xb[1], it, c->d_k.p,
                                      c->d_d.p, V.pe, V.pn, 0));
        if (tangent)
            HIP_TRY(c, launch_own_trace(st, g0, wng, V.gd, V.own, tb[0], tb[1], it.kfinal, c->d_dnp.p));
        if (events) HIP_TRY(c, hipEventRecord(c->ev_wave[4 * wave + 3], st));
        tr.pop();
    }
    HIP_TRY(c, launch_reduce(st, c->nnzb, V.pe, V.pn, V.ne));
    if (tangent) HIP_TRY(c, launch_reduce(st, ng, c->d_dnp.p, c->d_dnp.p, c->d_dn.p));
    c->have_tangent = tangent;
    c->last_sfix = c->use_sfix;
    if (events) HIP_TRY(c, hipEventRecord(c->ev_t3, st));
    c->steps_launched = launched;
    c->last_precision = c->precision;
    c->last_iteration = c->iteration;
    c->last_stride = stride;
    c->last_polish = mixed ? c->n_polish : 0;
    c->last_fmt = fmt;
    c->last_nw = nw;
    c->last_max_iter = c->max_iter;
    c->last_mu = c->mu;
    c->last_eig = false;
    c->last_kT = 0.0;
    c->evaluated = true;
    return SMX_OK;
}

// ---- diagonalisation path (finite temperature, Algorithm 1) -----------------
EigVecs eig_vecs(smx_ctx c)
{
    return EigVecs{c->d_ed.p, c->d_ee.p, c->d_etau.p, c->d_elam.p, c->d_elabs.p, c->d_ew.p, c->d_ebs.p, c->d_ebe.p};
}

// Decompose the groups of one wave at the context's mu: gather A_g - mu I
// into slab 0 (and its Gershgorin norm), tridiagonalise (reflectors stay in
// slab 0), eigenvalues and eigenvectors of T (slab 1, slab 2 as scratch),
// Y = Q^T E (thin block 0), C = S^T Y (thin block 1) with the weights and the
// unshifted eigenvalues.
int32_t eig_decompose_wave(smx_ctx c, const Plan &P, const DevView &V, double *arena, double *pool, int32_t wave,
                           hipEvent_t after_gather = nullptr)
{
    hipStream_t st = c->stream;
    const int32_t g0 = P.wave_g[wave], wng = P.wave_g[wave + 1] - g0;
    const int64_t E = P.work_elems;
    double *a = arena, *s = arena + E, *scr = arena + 2 * E;
    double *y = pool, *cb = pool + P.thin_elems;
    const EigVecs ev = eig_vecs(c);
    const int nch = (int)(P.chunk_beg[wave + 1] - P.chunk_beg[wave]);
    HIP_TRY(c, launch_gather(st, nch, V.chunks + P.chunk_beg[wave], V.gd, V.rinfo, V.bmap, V.boffs, c->d_valoff.p,
                             c->d_k.p, c->mu, a, V.scale));
    if (after_gather) HIP_TRY(c, hipEventRecord(after_gather, st));
    {
        // the Householder reduction dominates the path: timed like the product launches
        const size_t idx = c->launch_step.size();
        while (c->ev_launch.size() < 2 * (idx + 1)) {
            hipEvent_t evt;
            HIP_TRY(c, hipEventCreate(&evt));
            c->ev_launch.push_back(evt);
        }
        HIP_TRY(c, hipEventRecord(c->ev_launch[2 * idx], st));
        HIP_TRY(c, launch_eig_tridiag(st, g0, wng, V.gd, a, s, ev));     // s is free until the eigenvectors
        HIP_TRY(c, hipEventRecord(c->ev_launch[2 * idx + 1], st));
        c->launch_step.push_back(0);
        c->launch_kind.push_back(12);
        c->launch_wave.push_back(wave);
        c->launch_subset.push_back(0);
    }
    HIP_TRY(c, launch_eig_values_vectors(st, g0, wng, P.max_npad, V.gd, ev, s, scr));
    HIP_TRY(c, launch_eig_own_select(st, g0, wng, P.max_npad, P.max_own, V.gd, V.own, y));
    HIP_TRY(c, launch_eig_reflect(st, 1, g0, wng, P.max_own, V.gd, a, ev, y));
    HIP_TRY(c, launch_eig_thin(st, 0, g0, wng, P.max_npad, P.max_own, V.gd, ev, s, y, cb, c->mu, 0.0, c->kT, V.scale));
    return SMX_OK;
}

// D's own columns of the decomposed wave at mu0 + dmu: Z = S diag(g) C
// (thin block 2), G = Q Z, scatter of (E - G) / 2 with the energy and trace
// partials of the wave's stored blocks.
int32_t eig_apply_wave(smx_ctx c, const Plan &P, const DevView &V, double *arena, double *pool, int32_t wave,
                       double dmu)
{
    hipStream_t st = c->stream;
    const int32_t g0 = P.wave_g[wave], wng = P.wave_g[wave + 1] - g0;
    const int64_t E = P.work_elems;
    double *a = arena, *s = arena + E;
    double *cb = pool + P.thin_elems, *z = pool + 2 * P.thin_elems;
    const EigVecs ev = eig_vecs(c);
    HIP_TRY(c, launch_eig_thin(st, 1, g0, wng, P.max_npad, P.max_own, V.gd, ev, s, cb, z, c->mu, dmu, c->kT, V.scale));
    HIP_TRY(c, launch_eig_reflect(st, 0, g0, wng, P.max_own, V.gd, a, ev, z));
    IterState it{};
    it.scale_bits = V.scale;
    it.kfinal = V.kfinal;
    const int nwave = P.nwaves();
    const int64_t nsc = nwave > 1 ? P.plist_beg[wave + 1] - P.plist_beg[wave] : c->nnzb;
    const int64_t *pl = nwave > 1 ? V.plist + P.plist_beg[wave] : nullptr;
    HIP_TRY(c, launch_scatter(st, nsc, pl, V.scat, c->d_valoff.p, V.gd, z, nullptr, it, c->d_k.p, c->d_d.p, V.pe,
                              V.pn, 1));
    return SMX_OK;
}

// One evaluation on the diagonalisation path (all waves), then N and E.
int32_t eig_enqueue(smx_ctx c, const EvalMode &m, const Plan &P, const DevView &V, double *arena, double *pool)
{
    hipStream_t st = c->stream;
    const int32_t ng = P.ngroups;
    HIP_TRY(c, hipEventRecord(c->ev_t0, st));
    HIP_TRY(c, hipMemsetAsync(V.scale, 0, sizeof(unsigned long long) * ng, st));
    HIP_TRY(c, hipMemsetAsync(V.resid, 0, sizeof(unsigned long long) * (size_t)ng * m.stride, st));
    HIP_TRY(c, hipMemsetAsync(V.done, 0, sizeof(int32_t) * ng, st));
    HIP_TRY(c, hipMemsetAsync(V.kfinal, 0, sizeof(int32_t) * ng, st));
    HIP_TRY(c, hipMemsetAsync(V.flags, 0, sizeof(int32_t) * ng, st));
    c->launch_step.clear();
    c->launch_kind.clear();
    c->launch_wave.clear();
    c->launch_subset.clear();
    for (int32_t wave = 0; wave < P.nwaves(); wave++) {
        TraceScope tr("smx diagonalise");
        HIP_TRY(c, hipEventRecord(c->ev_wave[4 * wave], st));
        if (int32_t e = eig_decompose_wave(c, P, V, arena, pool, wave, c->ev_wave[4 * wave + 1])) return e;
        HIP_TRY(c, hipEventRecord(c->ev_wave[4 * wave + 2], st));
        tr.next("smx own columns of D");
        if (int32_t e = eig_apply_wave(c, P, V, arena, pool, wave, 0.0)) return e;
        HIP_TRY(c, hipEventRecord(c->ev_wave[4 * wave + 3], st));
    }
    HIP_TRY(c, launch_reduce(st, c->nnzb, V.pe, V.pn, V.ne));
    HIP_TRY(c, hipEventRecord(c->ev_t3, st));
    c->have_tangent = false;
    c->last_sfix = false;
    c->steps_launched = 0;
    c->last_precision = SMX_FP64;
    c->last_iteration = c->iteration;
    c->last_stride = m.stride;
    c->last_polish = 0;
    c->last_fmt = -1;
    c->last_nw = 0;
    c->last_max_iter = c->max_iter;
    c->last_mu = c->mu;
    c->last_eig = true;
    c->last_kT = c->kT;
    c->evaluated = true;
    return SMX_OK;
}

// ---- static scratch layout (smx_evaluate_static) ---------------------------
// The whole work memory of a static evaluation lies in the fixed scratch
// array, in this order: the plan's tables (group descriptors, tiles, gather
// chunks, row tables, block maps, block offsets, scatter descriptors, own-column
// lists, per-wave scatter lists), the per-evaluation state (scales, residual
// and trace histories, flags, counters, energy/trace partials), then one
// wave's arena and polish pool.  Only K, D and the two result scalars live in
// context memory allocated by earlier calls.
struct StaticLayout {
    int64_t gd = 0, tiles = 0, chunks = 0, rinfo = 0, bmap = 0, boffs = 0, scat = 0, own = 0, plist = 0;
    int64_t tiles_s = 0, tiles_b = 0;
    int64_t scale = 0, resid = 0, done = 0, kfinal = 0, flags = 0, ndone = 0, tdiag = 0, tau_hist = 0;
    int64_t pe = 0, pn = 0, arena = 0, pool = 0, end = 0;
};

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

StaticLayout static_layout(smx_ctx c, const Plan &P, int32_t stride)
{
    StaticLayout L;
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o += align256(std::max<int64_t>(bytes, 1));
        return at;
    };
    const int64_t ng = std::max(P.ngroups, 1);
    const int64_t nb = std::max<int64_t>(c->nnzb, 1);
    L.gd = take(vbytes(P.gd));
    L.tiles = take(vbytes(P.tiles));
    L.tiles_s = take(vbytes(P.tiles_s));
    L.tiles_b = take(vbytes(P.tiles_b));
    L.chunks = take(vbytes(P.chunks));
    L.rinfo = take(vbytes(P.rinfo));
    L.bmap = take(vbytes(P.bmap));
    L.boffs = take(vbytes(P.boffs));
    L.scat = take(vbytes(P.scat));
    L.own = take(vbytes(P.own_list));
    L.plist = take(vbytes(P.plist));
    L.scale = take(8 * ng);
    L.resid = take(8 * ng * stride);
    L.done = take(4 * ng);
    L.kfinal = take(4 * ng);
    L.flags = take(4 * ng);
    L.ndone = take(4);
    L.tdiag = take(8 * (int64_t)P.rinfo.size());
    L.tau_hist = take(8 * ng * stride);
    L.pe = take(8 * nb);
    L.pn = take(8 * nb);
    L.arena = take(arena_bytes(P));
    L.pool = take(pool_bytes(P));
    L.end = o;
    return L;
}

// Host-side plan of the static evaluation: waves sized so that tables, state,
// arena and pool fit the scratch array together.  Allocates host memory only.
int32_t static_plan(smx_ctx c, int32_t stride)
{
    if (!c->splan_dirty && c->splan_stride == stride) return SMX_OK;
    // earlier static evaluations may still be copying the old tables from the host
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    Plan &P = c->splan;
    c->splan_dirty = true;
    if (int32_t st = build_plan(c, P)) return st;
    const int64_t cap = (int64_t)SMX_STATIC_SCRATCH_BYTES;
    // first guess: everything but the arena and pool, with the tiles and
    // scatter lists at their one-wave sizes
    int64_t budget = cap - static_layout(c, P, stride).end - 8 * c->nnzb - 64 * 1024;
    for (;;) {
        if (budget <= 0)
            return fail(c, SMX_E_NOMEM, "the plan tables and iteration state need more than the " +
                                            std::to_string(cap >> 20) + " MiB static scratch array");
        if (int32_t st = partition_waves(c, P, budget)) {
            c->err = "static scratch array (" + std::to_string(cap >> 20) + " MiB): " + c->err;
            return st;
        }
        if (static_layout(c, P, stride).end <= cap) break;
        budget = budget * 15 / 16;
    }
    if (int32_t st = check_plan(c, P)) return st;
    c->splan_gen++;
    c->splan_stride = stride;
    c->splan_dirty = false;
    return SMX_OK;
}

template <typename T>
hipError_t upload_to(char *base, int64_t off, const std::vector<T> &v, hipStream_t st)
{
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(base + off, v.data(), vbytes(v), hipMemcpyHostToDevice, st);
}

}  // namespace

extern "C" {

int32_t smx_evaluate(smx_ctx c)
{
    if (!c) return SMX_E_INVALID;
    TraceScope tr("smx_evaluate");
    EvalMode m;
    if (int32_t st = eval_mode(c, m)) return st;
    if (int32_t st = set_device(c)) return st;
    c->evaluated = false;
    c->eval_static = false;
    if (int32_t st = eval_prepare(c, m)) return st;
    if (int32_t st = ensure_arena(c, m.mixed || m.eig)) return st;
    if (int32_t st = arm_guards(c, m.mixed || m.eig)) return st;
    if (m.eig) return eig_enqueue(c, m, c->plan, ctx_view(c), arena_base(c), pool_base(c));
    c->last_eig = false;
    return eval_enqueue(c, m, c->plan, ctx_view(c), arena_base(c), pool_base(c), true, true, true, c->host_poll != 0);
}


int32_t smx_evaluate_static(smx_ctx c)
{
    if (!c) return SMX_E_INVALID;
    TraceScope tr("smx_evaluate_static");
    EvalMode m;
    if (int32_t st = eval_mode(c, m)) return st;
    if (c->use_kfix || c->use_sfix)
        return fail(c, SMX_E_UNSUPPORTED, "frozen evaluations (derivatives, mu search) do not run in the static scratch");
    if (m.eig)
        return fail(c, SMX_E_UNSUPPORTED, "the diagonalisation path (kT > 0) does not run in the static scratch");
    if (int32_t st = set_device(c)) return st;
    void *sp = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (c->device < kMaxDevices && g_scratch_tried[c->device]) sp = g_scratch_ptr[c->device];
        if (!sp)
            return fail(c, SMX_E_HIP, std::string("the static scratch array has no address on this device: ") +
                                          hipGetErrorString(c->device < kMaxDevices ? g_scratch_err[c->device]
                                                                                    : hipErrorInvalidDevice));
    }
    c->evaluated = false;
    c->eval_static = false;
    if (int32_t st = static_plan(c, m.stride)) return st;
    const Plan &P = c->splan;
    const StaticLayout L = static_layout(c, P, m.stride);
    char *base = static_cast<char *>(sp);
    hipStream_t st = c->stream;
    {
        // the plan's tables, unless this context's current tables are already there
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        uint64_t *own = g_scratch_owner[c->device];
        if (own[0] != c->uid || own[1] != c->splan_gen) {
            HIP_TRY(c, upload_to(base, L.gd, P.gd, st));
            HIP_TRY(c, upload_to(base, L.tiles, P.tiles, st));
            HIP_TRY(c, upload_to(base, L.tiles_s, P.tiles_s, st));
            HIP_TRY(c, upload_to(base, L.tiles_b, P.tiles_b, st));
            HIP_TRY(c, upload_to(base, L.chunks, P.chunks, st));
            HIP_TRY(c, upload_to(base, L.rinfo, P.rinfo, st));
            HIP_TRY(c, upload_to(base, L.bmap, P.bmap, st));
            HIP_TRY(c, upload_to(base, L.boffs, P.boffs, st));
            HIP_TRY(c, upload_to(base, L.scat, P.scat, st));
            HIP_TRY(c, upload_to(base, L.own, P.own_list, st));
            HIP_TRY(c, upload_to(base, L.plist, P.plist, st));
            own[0] = c->uid;
            own[1] = c->splan_gen;
        }
    }
    DevView V;
    V.gd = reinterpret_cast<const GroupDesc *>(base + L.gd);
    V.tiles = reinterpret_cast<const TileDesc *>(base + L.tiles);
    V.tiles_s = reinterpret_cast<const TileDesc *>(base + L.tiles_s);
    V.tiles_b = reinterpret_cast<const TileDesc *>(base + L.tiles_b);
    V.chunks = reinterpret_cast<const int2 *>(base + L.chunks);
    V.rinfo = reinterpret_cast<const RowInfo *>(base + L.rinfo);
    V.bmap = reinterpret_cast<const int32_t *>(base + L.bmap);
    V.boffs = reinterpret_cast<const int32_t *>(base + L.boffs);
    V.scat = reinterpret_cast<const ScatterDesc *>(base + L.scat);
    V.own = reinterpret_cast<const int32_t *>(base + L.own);
    V.plist = reinterpret_cast<const int64_t *>(base + L.plist);
    V.scale = reinterpret_cast<unsigned long long *>(base + L.scale);
    V.resid = reinterpret_cast<unsigned long long *>(base + L.resid);
    V.done = reinterpret_cast<int32_t *>(base + L.done);
    V.kfinal = reinterpret_cast<int32_t *>(base + L.kfinal);
    V.flags = reinterpret_cast<int32_t *>(base + L.flags);
    V.ndone = reinterpret_cast<int32_t *>(base + L.ndone);
    V.tdiag = reinterpret_cast<double *>(base + L.tdiag);
    V.tau_hist = reinterpret_cast<double *>(base + L.tau_hist);
    V.pe = reinterpret_cast<double *>(base + L.pe);
    V.pn = reinterpret_cast<double *>(base + L.pn);
    V.ne = c->d_ne.p;
    // state that must start at zero is cleared inside (scales, histories,
    // flags, step counts, the finished-group counter); every other state
    // array and the arena are written before they are read
    if (int32_t e = eval_enqueue(c, m, P, V, reinterpret_cast<double *>(base + L.arena),
                                 reinterpret_cast<double *>(base + L.pool), false, false, false, false))
        return e;
    HIP_TRY(c, launch_count_flags(st, P.ngroups, V.flags, c->d_fsum.p));
    c->eval_static = true;
    return SMX_OK;
}

int32_t smx_wait(smx_ctx c)
{
    if (!c) return SMX_E_INVALID;
    if (int32_t st = need_sync_results(c)) return st;
    if (int32_t st = check_guards(c)) return st;
    int nc = 0, nf = 0;
    if (c->eval_static) {
        int32_t cnt[2] = {0, 0};
        HIP_TRY(c, hipMemcpy(cnt, c->d_fsum.p, sizeof cnt, hipMemcpyDeviceToHost));
        nc = cnt[0];
        nf = cnt[1];
    } else {
        std::vector<int32_t> fl((size_t)c->plan.ngroups);
        HIP_TRY(c, hipMemcpy(fl.data(), c->d_flags.p, fl.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int32_t f : fl) {
            nc += (f & 1) != 0;
            nf += (f & 2) != 0;
        }
    }
    if (nf) return fail(c, SMX_E_NONFINITE, std::to_string(nf) + " group(s) produced non-finite iterates");
    if (nc)
        return fail(c, SMX_E_NOT_CONVERGED,
                    std::to_string(nc) + " group(s) did not converge (FP64: max_iter reached; reduced precision: "
                                         "bulk left above switch_tol, or polished residual above tol)");
    return SMX_OK;
}

int32_t smx_get_d(smx_ctx c, double *out, int32_t out_on_device)
{
    if (!c) return SMX_E_INVALID;
    if (!out) return fail(c, SMX_E_INVALID, "out is NULL");
    if (int32_t st = need_sync_results(c)) return st;
    if (c->nvals > 0)
        HIP_TRY(c, hipMemcpyAsync(out, c->d_d.p, (size_t)c->nvals * sizeof(double),
                                  out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SMX_OK;
}

int32_t smx_get_d_expanded(smx_ctx c, const int64_t *index, int64_t n_out, double *out, int32_t out_on_device)
{
    if (!c) return SMX_E_INVALID;
    if (!out || (!index && c->nvals > 0)) return fail(c, SMX_E_INVALID, "index and out must not be NULL");
    if (n_out < 0) return fail(c, SMX_E_INVALID, "n_out < 0");
    if (int32_t st = need_sync_results(c)) return st;
    {
        std::vector<char> seen((size_t)n_out, 0);
        for (int64_t q = 0; q < c->nvals; q++) {
            const int64_t d = index[q];
            if (d < 0 || d >= n_out) return fail(c, SMX_E_INVALID, "index out of range at " + std::to_string(q));
            if (seen[(size_t)d]) return fail(c, SMX_E_INVALID, "index repeats position " + std::to_string(d));
            seen[(size_t)d] = 1;
        }
    }
    HIP_TRY(c, c->d_xidx.ensure((size_t)c->nvals));
    if (c->nvals > 0)
        HIP_TRY(c, hipMemcpyAsync(c->d_xidx.p, index, (size_t)c->nvals * sizeof(int64_t), hipMemcpyHostToDevice,
                                  c->stream));
    double *dst = out;
    if (!out_on_device) {
        HIP_TRY(c, c->d_xout.ensure((size_t)n_out));
        dst = c->d_xout.p;
    }
    HIP_TRY(c, launch_expand_values(c->stream, c->nvals, c->d_xidx.p, c->d_d.p, n_out, dst));
    if (!out_on_device && n_out > 0)
        HIP_TRY(c, hipMemcpyAsync(out, dst, (size_t)n_out * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SMX_OK;
}

static int32_t read_ne(smx_ctx c, double *ne)
{
    if (int32_t st = need_sync_results(c)) return st;
    HIP_TRY(c, hipMemcpy(ne, c->d_ne.p, 2 * sizeof(double), hipMemcpyDeviceToHost));
    return SMX_OK;
}

int32_t smx_trace(smx_ctx c, double *n_out)
{
    if (!c) return SMX_E_INVALID;
    if (!n_out) return fail(c, SMX_E_INVALID, "n_out is NULL");
    double ne[2];
    if (int32_t st = read_ne(c, ne)) return st;
    *n_out = ne[0];
    return SMX_OK;
}

int32_t smx_energy(smx_ctx c, double *e_out)
{
    if (!c) return SMX_E_INVALID;
    if (!e_out) return fail(c, SMX_E_INVALID, "e_out is NULL");
    double ne[2];
    if (int32_t st = read_ne(c, ne)) return st;
    *e_out = ne[1];
    return SMX_OK;
}

int32_t smx_get_group_info(smx_ctx c, int32_t *n_g, int32_t *iters, double *scale, double *resid)
{
    if (!c) return SMX_E_INVALID;
    if (int32_t st = need_group_state(c)) return st;
    const int32_t ng = c->plan.ngroups;
    std::vector<int32_t> kf((size_t)ng);
    std::vector<unsigned long long> sb((size_t)ng), rb((size_t)ng * c->last_stride);
    HIP_TRY(c, hipMemcpy(kf.data(), c->d_kfinal.p, kf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(sb.data(), c->last_sfix ? c->d_sfix.p : c->d_scale.p, sb.size() * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(rb.data(), c->d_resid.p, rb.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (int32_t g = 0; g < ng; g++) {
        if (n_g) n_g[g] = c->plan.gd[g].n;
        if (iters) iters[g] = kf[g] + c->last_polish;
        // FP64 mode: residual of the returned X_k; reduced-precision modes:
        // max|X_{k+p-1}^2 E - E| on the own columns, one step before the result
        const size_t slot = c->last_polish ? (size_t)(c->last_max_iter + c->last_polish) : (size_t)kf[g];
        double s, r;
        std::memcpy(&s, &sb[g], sizeof s);
        std::memcpy(&r, &rb[(size_t)g * c->last_stride + slot], sizeof r);
        if (scale) scale[g] = s;
        if (resid) resid[g] = r;
    }
    return SMX_OK;
}

int32_t smx_get_stats(smx_ctx c, smx_stats *out)
{
    if (!c) return SMX_E_INVALID;
    if (!out) return fail(c, SMX_E_INVALID, "out is NULL");
    if (int32_t st = need_group_state(c)) return st;
    const int32_t ng = c->plan.ngroups;
    std::vector<int32_t> n((size_t)ng), it((size_t)ng), fl((size_t)ng);
    std::vector<double> sc((size_t)ng), rs((size_t)ng);
    if (int32_t st = smx_get_group_info(c, n.data(), it.data(), sc.data(), rs.data())) return st;
    HIP_TRY(c, hipMemcpy(fl.data(), c->d_flags.p, fl.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    smx_stats s;
    std::memset(&s, 0, sizeof s);
    s.ngroups = ng;
    s.precision = c->last_precision;
    s.n_min = INT32_MAX;
    s.iters_min = INT32_MAX;
    double nsum = 0, isum = 0;
    for (int32_t g = 0; g < ng; g++) {
        s.n_min = std::min(s.n_min, n[g]);
        s.n_max = std::max(s.n_max, n[g]);
        s.iters_min = std::min(s.iters_min, it[g]);
        s.iters_max = std::max(s.iters_max, it[g]);
        s.n_not_converged += (fl[g] & 1) != 0;
        nsum += n[g];
        isum += it[g];
        s.resid_max = std::max(s.resid_max, rs[g]);
        // dense products: two per Newton-Schulz step, three per Pade step (the
        // polish of the reduced-precision modes is Newton-Schulz)
        const double nd = n[g];
        const double ppb = c->last_iteration == SMX_ITER_PADE3 ? 3.0 : 2.0;
        s.algo_flops += 2.0 * nd * nd * nd * (ppb * (it[g] - c->last_polish) + 2.0 * c->last_polish);
    }
    if (c->last_eig) {
        // Householder reduction (4/3 n^3) and the four thin passes over n x n
        // matrices with the m_own own columns (2 n^2 m_own each)
        s.algo_flops = 0;
        for (int32_t g = 0; g < ng; g++) {
            const double nd = n[g];
            s.algo_flops += 4.0 / 3.0 * nd * nd * nd + 8.0 * nd * nd * c->plan.gd[g].m_own;
        }
    }
    s.n_mean = ng ? nsum / ng : 0;
    s.iters_mean = ng ? isum / ng : 0;
    // issued matrix-core flops of the product kernels (live wave tiles, padding included)
    double exec = 0;
    {
        const Plan &P = c->plan;
        int npairs = 1;
        if (c->last_precision == SMX_FP16_2W) npairs = 3;
        if (c->last_precision == SMX_BF16_3W) npairs = 6;
        const bool buckets = c->last_precision == SMX_FP16_2W || c->last_precision == SMX_BF16_1W;
        const double ppb = c->last_iteration == SMX_ITER_PADE3 ? 3.0 : 2.0;
        for (int32_t g = 0; g < ng; g++) {
            const GroupDesc &d = P.gd[g];
            const double per = (buckets && P.big[g]) ? P.wtiles2[g] * 2.0 * 16 * 16 * d.npad
                                                     : P.wtiles[g] * 2.0 * 64 * 64 * d.npad;
            const double kb = it[g] - c->last_polish;     // bulk steps taken
            // the last step's square (and Pade combine) precede the stopping decision
            if (c->last_polish == 0) {
                exec += per * (ppb * kb + ppb - 1.0);
            } else {
                // bulk word products, then 3^p - 1 thin FP64 products of the own-column polish
                exec += per * npairs * (ppb * kb + ppb - 1.0);
                exec += (std::pow(3.0, c->last_polish) - 1.0) * 2.0 * (double)d.n * d.n * d.m_own;
            }
        }
    }
    s.exec_flops = c->last_eig ? s.algo_flops : exec;
    // phase times summed over the waves (the first wave's start includes the
    // state clears, the final reductions count as scatter)
    const int32_t nwave = c->plan.nwaves();
    s.nwaves = nwave;
    float ms = 0;
    for (int32_t w = 0; w < nwave; w++) {
        HIP_TRY(c, hipEventElapsedTime(&ms, w ? c->ev_wave[4 * w] : c->ev_t0, c->ev_wave[4 * w + 1]));
        s.time_gather_ms += ms;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_wave[4 * w + 1], c->ev_wave[4 * w + 2]));
        s.time_iterate_ms += ms;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_wave[4 * w + 2], c->ev_wave[4 * w + 3]));
        s.time_scatter_ms += ms;
    }
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_wave[4 * (nwave - 1) + 3], c->ev_t3));
    s.time_scatter_ms += ms;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_t0, c->ev_t3));
    s.time_total_ms = ms;
    double ws = 0;
    for (size_t b : {c->d_k.bytes(), c->d_d.bytes(), c->d_arena.bytes(), c->d_tpool.bytes(), c->d_tx0.bytes(), c->d_tx1.bytes(), c->d_adj.bytes(), c->d_bmap.bytes(),
                     c->d_rinfo.bytes(), c->d_scat.bytes(), c->d_resid.bytes(), c->d_tiles.bytes(),
                     c->d_tiles_full.bytes(), c->d_plist.bytes(), c->ws_ptr ? c->ws_bytes : (size_t)0})
        ws += (double)b;
    s.workspace_bytes = ws;
    *out = s;
    return SMX_OK;
}

int32_t smx_get_launch_profile(smx_ctx c, int32_t cap, float *ms, double *algo_flops, int32_t *kind,
                               int32_t *count)
{
    if (!c) return SMX_E_INVALID;
    if (int32_t st = need_group_state(c)) return st;
    const int32_t nl = (int32_t)c->launch_step.size();
    if (count) *count = nl;
    std::vector<int32_t> kf((size_t)c->plan.ngroups);
    HIP_TRY(c, hipMemcpy(kf.data(), c->d_kfinal.p, kf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int32_t l = 0; l < nl && l < cap; l++) {
        const int32_t kd = c->launch_kind[l];
        if (kind) kind[l] = kd;
        if (ms) {
            float t = 0;
            HIP_TRY(c, hipEventElapsedTime(&t, c->ev_launch[2 * l], c->ev_launch[2 * l + 1]));
            ms[l] = t;
        }
        if (algo_flops) {
            const int32_t k = c->launch_step[l], w = c->launch_wave[l], sub = c->launch_subset[l];
            double f = 0;
            for (int32_t g = c->plan.wave_g[w]; g < c->plan.wave_g[w + 1]; g++) {
                if (sub == 1 && c->plan.big[g]) continue;     // the launch covers one size bucket
                if (sub == 2 && !c->plan.big[g]) continue;
                bool active = true;                           // polish launches work on every group
                if (kd == 0 || kd == 2 || kd == 7 || kd >= 9) active = k <= kf[g];   // squares (and Pade combines)
                                                                                      // run up to the last step
                if (kd == 1 || kd == 3 || kd == 6 || kd == 8) active = k < kf[g];   // updates (and tangents) stop one earlier
                const double n = c->plan.gd[g].n;
                if (kd == 12) f += 4.0 / 3.0 * n * n * n;     // Householder reduction to tridiagonal form
                else if (active) f += 2.0 * n * n * n;
            }
            algo_flops[l] = f;
        }
    }
    return SMX_OK;
}

int32_t smx_get_launch_issued(smx_ctx c, int32_t cap, double *issued_flops, int32_t *count)
{
    if (!c) return SMX_E_INVALID;
    if (int32_t st = need_group_state(c)) return st;
    const int32_t nl = (int32_t)c->launch_step.size();
    if (count) *count = nl;
    if (!issued_flops) return SMX_OK;
    std::vector<int32_t> kf((size_t)c->plan.ngroups);
    HIP_TRY(c, hipMemcpy(kf.data(), c->d_kfinal.p, kf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    const Plan &P = c->plan;
    int npairs = 1;
    if (c->last_precision == SMX_FP16_2W) npairs = 3;
    if (c->last_precision == SMX_BF16_3W) npairs = 6;
    for (int32_t l = 0; l < nl && l < cap; l++) {
        const int32_t kd = c->launch_kind[l], k = c->launch_step[l], w = c->launch_wave[l];
        const int32_t sub = c->launch_subset[l];
        double f = 0;
        for (int32_t g = P.wave_g[w]; g < P.wave_g[w + 1]; g++) {
            if (sub == 1 && P.big[g]) continue;
            if (sub == 2 && !P.big[g]) continue;
            bool active = true;
            if (kd == 0 || kd == 2 || kd == 7 || kd >= 9) active = k <= kf[g];
            if (kd == 1 || kd == 3 || kd == 6 || kd == 8) active = k < kf[g];
            const GroupDesc &d = P.gd[g];
            if (kd == 12) {
                const double n = d.n;
                f += 4.0 / 3.0 * n * n * n;              // vector-unit work, no matrix cores
            } else if (active) {
                const bool word = kd == 2 || kd == 3 || kd == 7 || kd == 8 || kd == 9 || kd == 10;
                const double per = (kd == 7 || kd == 8 || kd == 10) ? P.wtiles2[g] * 2.0 * 16 * 16 * d.npad
                                                                     : P.wtiles[g] * 2.0 * 64 * 64 * d.npad;
                f += per * (word ? npairs : 1);
            }
        }
        issued_flops[l] = f;
    }
    return SMX_OK;
}

int32_t smx_get_submatrix(smx_ctx c, int32_t g, int32_t what, double *out, int32_t ld, int32_t *n_out)
{
    if (!c) return SMX_E_INVALID;
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (what != 0 && what != 1) return fail(c, SMX_E_INVALID, "what must be 0 or 1");
    if (int32_t st = set_device(c)) return st;
    if (what == 1 && !c->evaluated) return fail(c, SMX_E_STATE, "no evaluation has been run");
    if (what == 1 && c->eval_static)
        return fail(c, SMX_E_STATE, "the iterates of a static-scratch evaluation are not kept");
    if (int32_t st = ensure_plan(c)) return st;
    if (int32_t st = ensure_arena(c, false)) return st;
    const Plan &P = c->plan;
    if (g < 0 || g >= P.ngroups) return fail(c, SMX_E_INVALID, "group index out of range");
    const GroupDesc d = P.gd[g];
    if (n_out) *n_out = d.n;
    if (!out) return SMX_OK;
    if (ld < d.n) return fail(c, SMX_E_INVALID, "ld < n_g");
    if (what == 1 && P.wave_of[g] != P.nwaves() - 1)
        return fail(c, SMX_E_UNSUPPORTED, "the iterates of group " + std::to_string(g) +
                                              " were overwritten by a later wave (only the last wave's are kept)");
    const double *src = nullptr;
    double a = 1.0;
    if (what == 0) {
        // re-gather this group's chunks into a slab that what = 1 does not read:
        // the W slab in FP64 mode; after a reduced-precision evaluation the first
        // slab (the words of the iterates lie over the second and third)
        double *dst = (c->evaluated && c->last_polish) ? slab(c, 0) : slab(c, 2);
        std::vector<int2> ch;
        for (const int2 &x : P.chunks)
            if (x.x == g) ch.push_back(x);
        DevBuf<int2> dch;
        HIP_TRY(c, upload(dch, ch, c->stream));
        HIP_TRY(c, c->d_check.ensure((size_t)std::max(P.ngroups, 2)));
        HIP_TRY(c, hipMemsetAsync(c->d_check.p, 0, sizeof(double) * std::max(P.ngroups, 2), c->stream));
        HIP_TRY(c, launch_gather(c->stream, (int)ch.size(), dch.p, c->d_gd.p, c->d_rinfo.p, c->d_bmap.p,
                                 c->d_boffs.p, c->d_valoff.p, c->d_k.p, c->mu, dst,
                                 reinterpret_cast<unsigned long long *>(c->d_check.p)));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dch.release();
        src = dst + d.off;
    } else if (c->last_polish) {
        // reduced-precision modes: the bulk's last iterate, converted to FP64
        // from its words (the polish steps are computed on the own columns only)
        const unsigned short *w0 = reinterpret_cast<const unsigned short *>(slab(c, 1));
        const unsigned short *w1 = w0 + (size_t)c->last_nw * P.work_elems;
        HIP_TRY(c, launch_from_words(c->stream, c->last_fmt, c->last_nw, g, 1, d.npad, c->d_gd.p, w0, w1,
                                     c->d_kfinal.p, slab(c, 0)));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        src = slab(c, 0) + d.off;
    } else {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        int32_t kf = 0;
        unsigned long long sb = 0;
        HIP_TRY(c, hipMemcpy(&kf, c->d_kfinal.p + g, sizeof kf, hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(&sb, (c->last_sfix ? c->d_sfix.p : c->d_scale.p) + g, sizeof sb, hipMemcpyDeviceToHost));
        if (kf == 0) {
            double s;
            std::memcpy(&s, &sb, sizeof s);
            a = s > 0 ? 1.0 / s : 0.0;
        }
        src = slab(c, kf & 1) + d.off;
    }
    std::vector<double> tmp((size_t)d.npad * d.npad);
    HIP_TRY(c, hipMemcpy(tmp.data(), src, tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int32_t j = 0; j < d.n; j++)
        for (int32_t i = 0; i < d.n; i++) out[i + (size_t)j * ld] = a * tmp[i + (size_t)j * d.npad];
    return SMX_OK;
}

int32_t smx_set_frozen(smx_ctx c, int32_t on)
{
    if (!c) return SMX_E_INVALID;
    if (!on) {
        c->use_kfix = c->use_sfix = false;
        return SMX_OK;
    }
    if (int32_t st = need_group_state(c)) return st;
    if (c->last_iteration != SMX_ITER_NS2 || c->last_eig)
        return fail(c, SMX_E_UNSUPPORTED, "the frozen map (derivatives, mu search) is the Newton-Schulz one");
    const int32_t ng = c->plan.ngroups;
    std::vector<int32_t> kf((size_t)ng);
    HIP_TRY(c, hipMemcpy(kf.data(), c->d_kfinal.p, kf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int32_t &k : kf) k += c->last_polish;          // total steps, polish included
    HIP_TRY(c, upload(c->d_kfix, kf, c->stream));
    if (!c->last_sfix) {
        HIP_TRY(c, c->d_sfix.ensure((size_t)std::max(ng, 1)));
        HIP_TRY(c, hipMemcpyAsync(c->d_sfix.p, c->d_scale.p, sizeof(unsigned long long) * ng,
                                  hipMemcpyDeviceToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->use_kfix = c->use_sfix = true;
    return SMX_OK;
}

int32_t smx_dn_dmu(smx_ctx c, double *out)
{
    if (!c) return SMX_E_INVALID;
    if (!out) return fail(c, SMX_E_INVALID, "out is NULL");
    if (int32_t st = need_sync_results(c)) return st;
    if (!c->have_tangent) return fail(c, SMX_E_STATE, "the last evaluation was not frozen (smx_set_frozen)");
    double v[2];
    HIP_TRY(c, hipMemcpy(v, c->d_dn.p, sizeof v, hipMemcpyDeviceToHost));
    *out = -0.5 * v[0];
    return SMX_OK;
}

// Key of a tuning record: device, precision and the shape of the batch
// (groups, waves, sum and maximum of n_pad, work sum n_pad^3).
static std::string tune_key(smx_ctx c)
{
    hipDeviceProp_t prop;
    std::string dev = "gpu";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev = prop.gcnArchName;
    for (char &ch : dev)
        if (ch == ' ' || ch == ':') ch = '_';
    const Plan &P = c->plan;
    double s1 = 0, s3 = 0;
    for (const GroupDesc &d : P.gd) {
        s1 += d.npad;
        s3 += (double)d.npad * d.npad * d.npad;
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "v2|%s|p%d|g%d|w%d|n%.0f|m%d|c%.4e", dev.c_str(), c->precision, P.ngroups, P.nwaves(),
                  s1, P.max_npad, s3);
    return buf;
}

int32_t smx_autotune(smx_ctx c, int32_t reps, int32_t use_cache, int32_t *graph_steps_out, int32_t *tile_order_out,
                     double *best_ms_out)
{
    if (!c) return SMX_E_INVALID;
    TraceScope tr("smx_autotune");
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (reps < 1 || reps > 100) return fail(c, SMX_E_INVALID, "reps must be 1..100");
    if (int32_t st = set_device(c)) return st;
    if (int32_t st = ensure_plan(c)) return st;
    const char *path = std::getenv("SMX_TUNE_CACHE");
    std::string key = tune_key(c);
    int32_t best_g = -1, best_o = -1, best_b = -1;
    double best = INFINITY;
    if (use_cache && path) {
        if (FILE *f = std::fopen(path, "r")) {
            char line[512];
            while (std::fgets(line, sizeof line, f)) {
                char k[320];
                int g, o, b;
                double ms;
                if (std::sscanf(line, "%319s %d %d %d %lf", k, &g, &o, &b, &ms) == 5 && key == k && g >= 0 && g <= 64 &&
                    (o == 0 || o == 1) && b >= 0) {
                    best_g = g;
                    best_o = o;
                    best_b = b;
                    best = ms;
                }
            }
            std::fclose(f);
        }
    }
    const bool from_cache = best_g >= 0;
    if (!from_cache) {
        // candidates: launch order x step graphs x (one- and two-word products)
        // the size bucket boundary of the 256 x 256 tiles; each timed by device
        // time of whole evaluations
        const int32_t keep_g = c->graph_steps, keep_o = c->tile_order, keep_b = c->big_min_npad;
        std::vector<int32_t> shapes = {c->big_min_npad};
        if (c->precision == SMX_FP16_2W || c->precision == SMX_BF16_1W) shapes = {0, 384, 640, 896};
        for (int32_t b : shapes)
            for (int32_t o : {0, 1})
                for (int32_t g : {0, 2, 8}) {
                    if (int32_t st = smx_set_tile_shape(c, b)) return st;
                    if (int32_t st = smx_set_tile_order(c, o)) return st;
                    if (int32_t st = smx_set_graph(c, g)) return st;
                    double tmin = INFINITY;
                    for (int32_t r = 0; r <= reps; r++) {      // the first run captures graphs / warms up
                        int32_t st = smx_evaluate(c);
                        if (st == SMX_OK) st = smx_wait(c);
                        if (st != SMX_OK && st != SMX_E_NOT_CONVERGED) {
                            (void)smx_set_tile_shape(c, keep_b);
                            (void)smx_set_tile_order(c, keep_o);
                            (void)smx_set_graph(c, keep_g);
                            return st;
                        }
                        smx_stats sst;
                        if (int32_t e = smx_get_stats(c, &sst)) return e;
                        if (r > 0) tmin = std::min(tmin, sst.time_total_ms);
                    }
                    if (tmin < best) {
                        best = tmin;
                        best_g = g;
                        best_o = o;
                        best_b = b;
                    }
                }
        if (path)
            if (FILE *f = std::fopen(path, "a")) {
                std::fprintf(f, "%s %d %d %d %.6f\n", key.c_str(), best_g, best_o, best_b, best);
                std::fclose(f);
            }
    }
    if (int32_t st = smx_set_tile_shape(c, best_b)) return st;
    if (int32_t st = smx_set_tile_order(c, best_o)) return st;
    if (int32_t st = smx_set_graph(c, best_g)) return st;
    c->evaluated = false;
    if (graph_steps_out) *graph_steps_out = best_g;
    if (tile_order_out) *tile_order_out = best_o;
    if (best_ms_out) *best_ms_out = best;
    return SMX_OK;
}

// Gershgorin interval of the whole K (host copy of the values): every
// principal submatrix has its spectrum inside it (Cauchy interlacing).
static int32_t gershgorin_interval(smx_ctx c, double *lo, double *hi)
{
    std::vector<double> v((size_t)c->nvals);
    HIP_TRY(c, hipMemcpy(v.data(), c->d_k.p, v.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<int64_t> boff((size_t)c->nblk + 1, 0);
    for (int32_t j = 0; j < c->nblk; j++) boff[j + 1] = boff[j] + c->blk_size[j];
    const int64_t n = boff[c->nblk];
    std::vector<double> diag((size_t)n, 0.0), rad((size_t)n, 0.0);
    for (int32_t j = 0; j < c->nblk; j++) {
        const int32_t bj = c->blk_size[j];
        for (int64_t p = c->col_ptr[j]; p < c->col_ptr[j + 1]; p++) {
            const int32_t i = c->row_idx[p], bi = c->blk_size[i];
            const double *b = v.data() + c->val_off[p];
            for (int32_t cc = 0; cc < bj; cc++)
                for (int32_t rr = 0; rr < bi; rr++) {
                    const int64_t gi = boff[i] + rr, gj = boff[j] + cc;
                    if (gi == gj) diag[gi] = b[rr + (int64_t)cc * bi];
                    else rad[gi] += std::fabs(b[rr + (int64_t)cc * bi]);
                }
        }
    }
    double l = INFINITY, h = -INFINITY;
    for (int64_t i = 0; i < n; i++) {
        l = std::min(l, diag[i] - rad[i]);
        h = std::max(h, diag[i] + rad[i]);
    }
    *lo = l;
    *hi = h;
    return SMX_OK;
}

// Gershgorin scales s_g = ||K_sub - mu I||_inf of every group at mu (device gather into scratch).
static int32_t scales_at(smx_ctx c, double mu, std::vector<double> &out)
{
    const Plan &P = c->plan;
    const int32_t ng = P.ngroups;
    if (int32_t st = ensure_arena(c, false)) return st;
    HIP_TRY(c, c->d_scale_scratch.ensure((size_t)std::max(ng, 1)));
    HIP_TRY(c, hipMemsetAsync(c->d_scale_scratch.p, 0, sizeof(unsigned long long) * ng, c->stream));
    for (int32_t w = 0; w < P.nwaves(); w++)
        HIP_TRY(c, launch_gather(c->stream, (int)(P.chunk_beg[w + 1] - P.chunk_beg[w]), c->d_chunks.p + P.chunk_beg[w],
                                 c->d_gd.p, c->d_rinfo.p, c->d_bmap.p, c->d_boffs.p, c->d_valoff.p, c->d_k.p, mu,
                                 slab(c, 2), c->d_scale_scratch.p));
    std::vector<unsigned long long> b((size_t)ng);
    HIP_TRY(c, hipMemcpyAsync(b.data(), c->d_scale_scratch.p, b.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out.resize((size_t)ng);
    for (int32_t g = 0; g < ng; g++) std::memcpy(&out[g], &b[g], sizeof(double));
    return SMX_OK;
}

int32_t smx_find_mu(smx_ctx c, double n_target, double tol, int32_t max_steps, double *mu_out, int32_t *steps_out)
{
    if (!c) return SMX_E_INVALID;
    TraceScope tr("smx_find_mu");
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (!mu_out || !(tol > 0.0) || max_steps < 1) return fail(c, SMX_E_INVALID, "need mu_out, tol > 0, max_steps >= 1");
    if (c->precision != SMX_FP64) return fail(c, SMX_E_UNSUPPORTED, "the mu search runs in SMX_FP64");
    if (c->iteration != SMX_ITER_NS2)
        return fail(c, SMX_E_UNSUPPORTED, "the mu search follows the frozen Newton-Schulz map");
    if (int32_t st = set_device(c)) return st;
    if (int32_t st = ensure_plan(c)) return st;
    const int32_t ng = c->plan.ngroups;
    double lo, hi;
    if (int32_t st = gershgorin_interval(c, &lo, &hi)) return st;
    // scales valid over the whole bracket (the norm is convex in mu)
    std::vector<double> s_lo, s_hi;
    if (int32_t st = scales_at(c, lo, s_lo)) return st;
    if (int32_t st = scales_at(c, hi, s_hi)) return st;
    std::vector<unsigned long long> sb((size_t)ng);
    for (int32_t g = 0; g < ng; g++) {
        const double sv = std::max(s_lo[g], s_hi[g]);
        std::memcpy(&sb[g], &sv, sizeof sv);
    }
    HIP_TRY(c, upload(c->d_sfix, sb, c->stream));
    // step counts: a converged evaluation at the starting mu with those scales
    double mu = std::min(std::max(c->mu, lo), hi);
    c->mu = mu;
    c->use_sfix = true;
    c->use_kfix = false;
    int32_t st = smx_evaluate(c);
    if (st == SMX_OK) st = smx_wait(c);
    if (st != SMX_OK) {
        c->use_sfix = false;
        return st;
    }
    {
        std::vector<int32_t> kf((size_t)ng);
        HIP_TRY(c, hipMemcpy(kf.data(), c->d_kfinal.p, kf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_TRY(c, upload(c->d_kfix, kf, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    c->use_kfix = true;
    // safeguarded Newton on the frozen approximant N_k(mu) (increasing in mu)
    int32_t steps = 0;
    int32_t result = SMX_E_NOT_CONVERGED;
    double blo = lo, bhi = hi;
    for (steps = 1; steps <= max_steps; steps++) {
        c->mu = mu;
        st = smx_evaluate(c);
        if (st == SMX_OK) st = smx_wait(c);
        double nval = 0, dn = 0;
        if (st == SMX_OK) st = smx_trace(c, &nval);
        if (st == SMX_OK) st = smx_dn_dmu(c, &dn);
        if (st != SMX_OK) {
            result = st;
            break;
        }
        const double f = nval - n_target;
        if (std::fabs(f) <= tol) {
            result = SMX_OK;
            break;
        }
        if (f > 0) bhi = mu;
        else blo = mu;
        double next = (dn > 0) ? mu - f / dn : NAN;
        if (!(next > blo && next < bhi)) next = 0.5 * (blo + bhi);
        mu = next;
    }
    c->use_kfix = c->use_sfix = false;
    *mu_out = c->mu;
    if (steps_out) *steps_out = std::min(steps, max_steps);
    if (result == SMX_E_NOT_CONVERGED) return fail(c, SMX_E_NOT_CONVERGED, "mu search did not reach the tolerance");
    return result;
}

// Per stored block of K, the groups whose submatrix contains it, with the
// block's offsets there (the transpose of the gather), ascending in group.
int32_t smx_find_mu_eig(smx_ctx c, double n_target, double tol, int32_t max_steps, double *mu_out,
                        int32_t *steps_out)
{
    if (!c) return SMX_E_INVALID;
    TraceScope tr("smx_find_mu_eig");
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (!mu_out || !(tol > 0.0) || max_steps < 1) return fail(c, SMX_E_INVALID, "need mu_out, tol > 0, max_steps >= 1");
    if (c->precision != SMX_FP64) return fail(c, SMX_E_UNSUPPORTED, "the diagonalisation path runs in SMX_FP64");
    if (c->use_kfix || c->use_sfix) return fail(c, SMX_E_UNSUPPORTED, "unfreeze first (smx_set_frozen(ctx, 0))");
    if (int32_t st = set_device(c)) return st;
    EvalMode m;
    m.eig = true;
    m.stride = c->max_iter + 2 + c->n_polish;
    c->evaluated = false;
    c->eval_static = false;
    if (int32_t st = eval_prepare(c, m)) return st;
    if (int32_t st = ensure_arena(c, true)) return st;
    const Plan &P = c->plan;
    const DevView V = ctx_view(c);
    const int32_t ng = P.ngroups;
    hipStream_t st = c->stream;
    double *arena = arena_base(c), *pool = pool_base(c);
    // 1. every group's eigenvalues and Algorithm 1's weights, at mu0
    const double mu0 = c->mu;
    HIP_TRY(c, hipMemsetAsync(V.scale, 0, sizeof(unsigned long long) * ng, st));
    for (int32_t wave = 0; wave < P.nwaves(); wave++)
        if (int32_t e = eig_decompose_wave(c, P, V, arena, pool, wave)) return e;
    // 2. multisection on N(mu) = sum_g sum_l w_gl f(lambda_gl - mu), monotone in
    // mu: kM trial points per round inside the bracket, which every eigenvalue
    // (of every principal submatrix of K, by interlacing) lies in
    constexpr int kM = 128;
    double lo, hi;
    if (int32_t e = gershgorin_interval(c, &lo, &hi)) return e;
    lo -= 40.0 * c->kT + 1e-12 * std::max(1.0, std::fabs(lo));
    hi += 40.0 * c->kT + 1e-12 * std::max(1.0, std::fabs(hi));
    HIP_TRY(c, c->d_mus.ensure(kM));
    HIP_TRY(c, c->d_nval.ensure(kM));
    HIP_TRY(c, c->d_npart.ensure((size_t)std::max(ng, 1) * kM));
    std::vector<double> mus(kM), nv(kM);
    double best_mu = 0.5 * (lo + hi), best_n = NAN;
    int32_t steps = 0;
    bool found = false;
    while (steps < max_steps && !found) {
        for (int q = 0; q < kM; q++) mus[q] = lo + (hi - lo) * (q + 1) / (kM + 1);
        HIP_TRY(c, hipMemcpyAsync(c->d_mus.p, mus.data(), sizeof(double) * kM, hipMemcpyHostToDevice, st));
        HIP_TRY(c, launch_n_of_mu(st, ng, V.gd, eig_vecs(c), c->d_mus.p, kM, c->kT, V.scale, c->d_npart.p,
                                  c->d_nval.p));
        HIP_TRY(c, hipMemcpyAsync(nv.data(), c->d_nval.p, sizeof(double) * kM, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        steps++;
        int first = kM;                               // first trial point with N >= target
        for (int q = 0; q < kM; q++) {
            if (!std::isfinite(nv[q])) return fail(c, SMX_E_NONFINITE, "N(mu) is not finite");
            if (std::fabs(nv[q] - n_target) < (std::isnan(best_n) ? INFINITY : std::fabs(best_n - n_target))) {
                best_n = nv[q];
                best_mu = mus[q];
            }
            if (std::fabs(nv[q] - n_target) <= tol) found = true;
            if (first == kM && nv[q] >= n_target) first = q;
        }
        if (found) break;
        const double nlo = first > 0 ? mus[first - 1] : lo, nhi = first < kM ? mus[first] : hi;
        if (!(nhi - nlo > 2.220446049250313e-16 * std::max(std::fabs(nlo), std::fabs(nhi)))) break;
        lo = nlo;
        hi = nhi;
    }
    // 3. D at mu* from the stored decompositions (one wave), or a new
    // evaluation at mu* (the decompositions of earlier waves are gone)
    c->mu = best_mu;
    *mu_out = best_mu;
    if (steps_out) *steps_out = steps;
    if (P.nwaves() == 1) {
        const double mu_dec = c->mu;
        c->mu = mu0;                                  // the decomposition's shift
        HIP_TRY(c, hipEventRecord(c->ev_t0, st));
        HIP_TRY(c, hipMemsetAsync(V.kfinal, 0, sizeof(int32_t) * ng, st));
        HIP_TRY(c, hipMemsetAsync(V.flags, 0, sizeof(int32_t) * ng, st));
        HIP_TRY(c, hipMemsetAsync(V.resid, 0, sizeof(unsigned long long) * (size_t)ng * m.stride, st));
        HIP_TRY(c, hipEventRecord(c->ev_wave[0], st));
        HIP_TRY(c, hipEventRecord(c->ev_wave[1], st));
        HIP_TRY(c, hipEventRecord(c->ev_wave[2], st));
        int32_t e = eig_apply_wave(c, P, V, arena, pool, 0, mu_dec - mu0);
        c->mu = mu_dec;
        if (e) return e;
        HIP_TRY(c, hipEventRecord(c->ev_wave[3], st));
        HIP_TRY(c, launch_reduce(st, c->nnzb, V.pe, V.pn, V.ne));
        HIP_TRY(c, hipEventRecord(c->ev_t3, st));
        c->launch_step.clear();
        c->launch_kind.clear();
        c->launch_wave.clear();
        c->launch_subset.clear();
        c->have_tangent = false;
        c->last_sfix = false;
        c->last_precision = SMX_FP64;
        c->last_iteration = c->iteration;
        c->last_stride = m.stride;
        c->last_polish = 0;
        c->last_fmt = -1;
        c->last_nw = 0;
        c->last_max_iter = c->max_iter;
        c->last_mu = c->mu;
        c->last_eig = true;
        c->last_kT = c->kT;
        c->evaluated = true;
    } else {
        if (int32_t e = eig_enqueue(c, m, P, V, arena, pool)) return e;
    }
    if (!found)
        return fail(c, SMX_E_NOT_CONVERGED, "N(mu) = " + std::to_string(best_n) + " does not reach the target " +
                                                std::to_string(n_target) + " within tol (a step of N at T = 0?)");
    return SMX_OK;
}

int32_t smx_get_spectrum(smx_ctx c, double *lam, double *w)
{
    if (!c) return SMX_E_INVALID;
    if (int32_t st = need_group_state(c)) return st;
    if (!c->last_eig) return fail(c, SMX_E_STATE, "the last evaluation did not diagonalise the submatrices");
    const Plan &P = c->plan;
    const size_t nr = P.rinfo.size();
    std::vector<double> hl(nr), hw(nr);
    HIP_TRY(c, hipMemcpy(hl.data(), c->d_elabs.p, nr * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(hw.data(), c->d_ew.p, nr * sizeof(double), hipMemcpyDeviceToHost));
    size_t o = 0;
    for (const GroupDesc &d : P.gd)
        for (int32_t i = 0; i < d.n; i++, o++) {
            if (lam) lam[o] = hl[(size_t)d.rinfo_off + i];
            if (w) w[o] = hw[(size_t)d.rinfo_off + i];
        }
    return SMX_OK;
}

static int32_t ensure_contrib(smx_ctx c)
{
    if (c->contrib_ready) return SMX_OK;
    Plan &P = c->plan;
    std::vector<int64_t> cnt((size_t)c->nnzb + 1, 0);
    for (int32_t g = 0; g < P.ngroups; g++) {
        const GroupDesc &d = P.gd[g];
        for (int64_t q = 0; q < (int64_t)d.m * d.m; q++) {
            const int32_t p = P.bmap[(size_t)(d.map_off + q)];
            if (p >= 0) cnt[(size_t)p + 1]++;
        }
    }
    for (int64_t p = 0; p < c->nnzb; p++) cnt[(size_t)p + 1] += cnt[(size_t)p];
    P.cptr = cnt;
    P.contrib.assign((size_t)cnt[(size_t)c->nnzb], int4{0, 0, 0, 0});
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t g = 0; g < P.ngroups; g++) {
        const GroupDesc &d = P.gd[g];
        for (int32_t b = 0; b < d.m; b++)
            for (int32_t a = 0; a < d.m; a++) {
                const int32_t p = P.bmap[(size_t)(d.map_off + a + (int64_t)d.m * b)];
                if (p < 0) continue;
                P.contrib[(size_t)fill[(size_t)p]++] =
                    int4{g, P.boffs[d.boff_off + a], P.boffs[d.boff_off + b], 0};
            }
    }
    HIP_TRY(c, upload(c->d_cptr, P.cptr, c->stream));
    HIP_TRY(c, upload(c->d_contrib, P.contrib, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->contrib_ready = true;
    return SMX_OK;
}

int32_t smx_backward(smx_ctx c, double gE, double gN, const double *gD, int32_t gD_on_device, double *dK_out,
                     int32_t dK_on_device, double *dmu_out)
{
    if (!c) return SMX_E_INVALID;
    TraceScope tr("smx_backward");
    if (!dK_out && !dmu_out) return fail(c, SMX_E_INVALID, "nothing to compute (dK_out and dmu_out are NULL)");
    if (!std::isfinite(gE) || !std::isfinite(gN)) return fail(c, SMX_E_INVALID, "seeds must be finite");
    if (int32_t st = need_group_state(c)) return st;
    if (c->last_iteration != SMX_ITER_NS2 || c->last_eig)
        return fail(c, SMX_E_UNSUPPORTED, "the adjoint differentiates the Newton-Schulz map");
    if (int32_t st = set_device(c)) return st;
    if (c->plan.nwaves() != 1)
        return fail(c, SMX_E_UNSUPPORTED, "the adjoint needs every submatrix resident at once (one wave); "
                                          "raise the work-space limit");
    if (int32_t st = ensure_contrib(c)) return st;
    const Plan &P = c->plan;
    const int32_t ng = P.ngroups;
    hipStream_t st = c->stream;
    // the frozen map of the last evaluation: its step counts and scales
    std::vector<int32_t> kf((size_t)ng);
    HIP_TRY(c, hipMemcpy(kf.data(), c->d_kfinal.p, kf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t kmax = 0;
    for (int32_t &k : kf) {
        k += c->last_polish;
        kmax = std::max(kmax, k);
    }
    HIP_TRY(c, upload(c->d_kfix, kf, st));
    const unsigned long long *sptr = c->last_sfix ? c->d_sfix.p : c->d_scale.p;
    // slabs: Xbar, W, Z, Y, 8 segment iterates, checkpoints X_{8m}
    constexpr int kSeg = 8;
    const int32_t ncp = kmax / kSeg + 1;
    const int64_t E = P.work_elems;
    const size_t nslab = (size_t)(4 + kSeg + ncp);
    {
        size_t fr = 0, tot = 0;
        HIP_TRY(c, hipMemGetInfo(&fr, &tot));
        const size_t need = nslab * (size_t)E * sizeof(double);
        if (need > fr + c->d_adj.bytes())
            return fail(c, SMX_E_NOMEM, "adjoint needs " + std::to_string(need >> 20) + " MiB of device memory");
    }
    HIP_TRY(c, c->d_adj.ensure(nslab * (size_t)E));
    HIP_TRY(c, c->d_dk.ensure((size_t)std::max<int64_t>(c->nvals, 1)));
    HIP_TRY(c, c->d_dmu.ensure(2));
    HIP_TRY(c, c->d_dnp.ensure((size_t)std::max(ng, 1)));
    double *xb = c->d_adj.p, *wb = xb + E, *zb = wb + E, *yb = zb + E;
    double *seg[kSeg];
    for (int q = 0; q < kSeg; q++) seg[q] = yb + E * (q + 1);
    double *cp0 = yb + E * (kSeg + 1);
    auto cp = [&](int m) { return cp0 + E * m; };

    IterState it;
    it.scale_bits = const_cast<unsigned long long *>(sptr);
    it.resid_bits = c->d_resid.p;
    it.done = c->d_done.p;
    it.kfinal = c->d_kfinal.p;
    it.flags = c->d_flags.p;
    it.ndone = c->d_ndone.p;
    it.kfix = c->d_kfix.p;
    it.kact = -1;
    it.tdiag = c->d_tdiag.p;
    it.tau_hist = c->d_tau_hist.p;
    it.resid_stride = c->last_stride;
    const int scratch_slot = c->last_max_iter + 1;    // residual slot the adjoint squares may use
    const int nt = (int)P.tiles.size(), ntf = (int)P.tiles_full.size();
    const TileDesc *tl = c->d_tiles.p, *tf = c->d_tiles_full.p;

    // seed: Xbar_K = sym(-1/2 dL/dD at the own-column stored positions)
    HIP_TRY(c, hipMemsetAsync(xb, 0, sizeof(double) * (size_t)E, st));
    const double *gdp = nullptr;
    DevBuf<double> gdd;
    if (gD) {
        if (gD_on_device) {
            gdp = gD;
        } else {
            HIP_TRY(c, gdd.ensure((size_t)c->nvals));
            HIP_TRY(c, hipMemcpyAsync(gdd.p, gD, sizeof(double) * (size_t)c->nvals, hipMemcpyHostToDevice, st));
            gdp = gdd.p;
        }
    }
    HIP_TRY(c, launch_adj_seed(st, c->nnzb, c->d_scat.p, c->d_valoff.p, c->d_gd.p, c->d_k.p, gdp, gE, gN, xb));
    HIP_TRY(c, launch_symmetrize(st, ng, P.max_npad, c->d_gd.p, xb));

    // forward with checkpoints: X_0 = A / s_g, X_{k+1} = X_k W_k
    HIP_TRY(c, hipMemsetAsync(c->d_check.p, 0, 2 * sizeof(double), st));
    HIP_TRY(c, c->d_scale_scratch.ensure((size_t)std::max(ng, 1)));
    HIP_TRY(c, launch_gather(st, (int)P.chunks.size(), c->d_chunks.p, c->d_gd.p, c->d_rinfo.p, c->d_bmap.p,
                             c->d_boffs.p, c->d_valoff.p, c->d_k.p, c->last_mu, seg[0], c->d_scale_scratch.p));
    HIP_TRY(c, launch_scale_slab(st, ng, P.max_npad, c->d_gd.p, sptr, seg[0]));
    HIP_TRY(c, hipMemcpyAsync(cp(0), seg[0], sizeof(double) * (size_t)E, hipMemcpyDeviceToDevice, st));
    auto fwd_step = [&](int k, const double *x, double *xnext) -> int32_t {
        it.kact = k;
        HIP_TRY(c, launch_ns_f64(st, 0, nt, tl, c->d_gd.p, x, x, wb, it, scratch_slot, 0.0, c->last_max_iter, 1));
        HIP_TRY(c, launch_ns_f64(st, 1, nt, tl, c->d_gd.p, x, wb, xnext, it, scratch_slot, 0.0, c->last_max_iter, 1));
        return SMX_OK;
    };
    const int32_t mlast = (kmax > 0) ? (kmax - 1) / kSeg : 0;
    for (int32_t m = 0; m <= mlast; m++) {
        if (m > 0) HIP_TRY(c, hipMemcpyAsync(seg[0], cp(m), sizeof(double) * (size_t)E, hipMemcpyDeviceToDevice, st));
        for (int j = 0; j + 1 < kSeg && m * kSeg + j + 1 <= kmax - 1; j++)
            if (int32_t e = fwd_step(m * kSeg + j, seg[j], seg[j + 1])) return e;
        if (m < mlast)
            if (int32_t e = fwd_step(m * kSeg + kSeg - 1, seg[kSeg - 1], cp(m + 1))) return e;
    }
    // backward over the segments, the last one still in place
    for (int32_t m = mlast; m >= 0 && kmax > 0; m--) {
        if (m < mlast) {
            HIP_TRY(c, hipMemcpyAsync(seg[0], cp(m), sizeof(double) * (size_t)E, hipMemcpyDeviceToDevice, st));
            for (int j = 0; j + 1 < kSeg; j++)
                if (int32_t e = fwd_step(m * kSeg + j, seg[j], seg[j + 1])) return e;
        }
        const int32_t khi = std::min(m * kSeg + kSeg - 1, kmax - 1);
        for (int32_t k = khi; k >= m * kSeg; k--) {
            const double *x = seg[k - m * kSeg];
            it.kact = k;
            HIP_TRY(c, launch_ns_f64(st, 0, nt, tl, c->d_gd.p, x, x, wb, it, scratch_slot, 0.0, c->last_max_iter, 1));
            HIP_TRY(c, launch_ns_f64(st, 4, ntf, tf, c->d_gd.p, xb, wb, zb, it, scratch_slot, 0.0, c->last_max_iter, 1));
            HIP_TRY(c, launch_ns_f64(st, 4, ntf, tf, c->d_gd.p, xb, x, yb, it, scratch_slot, 0.0, c->last_max_iter, 1));
            HIP_TRY(c, launch_ns_f64(st, 3, nt, tl, c->d_gd.p, x, yb, xb, it, scratch_slot, 0.0, c->last_max_iter, 1,
                                     zb));
        }
    }
    // dK: transposed gather of Abar = Xbar_0 / s_g plus gE D; dL/dmu = -sum_g tr(Abar_g)
    HIP_TRY(c, launch_gather_t(st, c->nnzb, c->d_cptr.p, c->d_contrib.p, c->d_valoff.p, c->d_brow.p, c->d_bcol.p,
                               c->d_gd.p, sptr, xb, c->d_d.p, gE, c->d_dk.p));
    HIP_TRY(c, launch_diag_part(st, ng, c->d_gd.p, sptr, xb, c->d_dnp.p));
    HIP_TRY(c, launch_reduce(st, ng, c->d_dnp.p, c->d_dnp.p, c->d_dmu.p));
    if (dK_out && c->nvals > 0)
        HIP_TRY(c, hipMemcpyAsync(dK_out, c->d_dk.p, sizeof(double) * (size_t)c->nvals,
                                  dK_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    double dm[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(dm, c->d_dmu.p, sizeof dm, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    gdd.release();
    if (dmu_out) *dmu_out = dm[0];
    return SMX_OK;
}

int32_t smx_workspace_size(smx_ctx c, size_t *bytes)
{
    if (!c) return SMX_E_INVALID;
    if (!bytes) return fail(c, SMX_E_INVALID, "bytes is NULL");
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (int32_t st = set_device(c)) return st;
    if (int32_t st = ensure_plan(c)) return st;
    // every group resident at once: one wave's arena, then its polish pool
    int64_t e = 0, t = 0;
    for (const GroupDesc &d : c->plan.gd) {
        e += (int64_t)d.npad * d.npad;
        t += (int64_t)d.npad * d.m_own;
    }
    *bytes = (size_t)((kArenaBytesPerElem * e + 255) / 256 * 256 + (2 * kMaxPolishMixed + 1) * 8 * t + 512);
    return SMX_OK;
}

int32_t smx_set_workspace(smx_ctx c, void *dptr, size_t bytes)
{
    if (!c) return SMX_E_INVALID;
    if (int32_t st = set_device(c)) return st;
    if ((dptr == nullptr) != (bytes == 0)) return fail(c, SMX_E_INVALID, "dptr and bytes must both be set or both be 0");
    if (dptr) {
        if (reinterpret_cast<uintptr_t>(dptr) % 256) return fail(c, SMX_E_INVALID, "the work space must be 256-byte aligned");
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, dptr) != hipSuccess || attr.type != hipMemoryTypeDevice ||
            attr.device != c->device) {
            (void)hipGetLastError();
            return fail(c, SMX_E_INVALID, "the work space is not device memory of this context's device");
        }
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));      // no enqueued work may still use the old arena
    c->ws_ptr = dptr;
    c->ws_bytes = bytes;
    c->d_arena.release();
    c->d_tpool.release();
    drop_graphs(c);
    c->plan_dirty = true;
    c->evaluated = false;
    c->use_kfix = c->use_sfix = false;
    c->contrib_ready = false;
    return SMX_OK;
}

int32_t smx_set_host_poll(smx_ctx c, int32_t on)
{
    if (!c) return SMX_E_INVALID;
    if (on != 0 && on != 1) return fail(c, SMX_E_INVALID, "on must be 0 or 1");
    c->host_poll = on;
    return SMX_OK;
}

int32_t smx_get_history(smx_ctx c, int32_t cap, double *resid, double *tau, int32_t *nsteps)
{
    if (!c) return SMX_E_INVALID;
    if (cap < 0) return fail(c, SMX_E_INVALID, "cap must be >= 0");
    if (int32_t st = need_group_state(c)) return st;
    if (c->last_eig) return fail(c, SMX_E_STATE, "the diagonalisation path has no iteration history");
    const int32_t ng = c->plan.ngroups;
    const int32_t stride = c->last_stride;
    std::vector<int32_t> kf((size_t)ng);
    std::vector<unsigned long long> rb((size_t)ng * stride);
    std::vector<double> tb((size_t)ng * stride);
    HIP_TRY(c, hipMemcpy(kf.data(), c->d_kfinal.p, kf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(rb.data(), c->d_resid.p, rb.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(tb.data(), c->d_tau_hist.p, tb.size() * sizeof(double), hipMemcpyDeviceToHost));
    const bool has_tau = c->last_polish > 0;      // tau_k is computed by the reduced-precision bulk only
    for (int32_t g = 0; g < ng; g++) {
        const int32_t n = kf[g] + 1;
        if (nsteps) nsteps[g] = n;
        for (int32_t k = 0; k < cap; k++) {
            double r = NAN, t = NAN;
            if (k < n) {
                std::memcpy(&r, &rb[(size_t)g * stride + k], sizeof r);
                if (has_tau) t = tb[(size_t)g * stride + k];
            }
            if (resid) resid[(size_t)g * cap + k] = r;
            if (tau) tau[(size_t)g * cap + k] = t;
        }
    }
    return SMX_OK;
}

int32_t smx_get_sizes(smx_ctx c, int32_t *ngroups, int64_t *nvalues)
{
    if (!c) return SMX_E_INVALID;
    if (!c->loaded) return fail(c, SMX_E_STATE, "smx_load_k must come first");
    if (ngroups) *ngroups = (int32_t)c->grp_ptr.size() - 1;
    if (nvalues) *nvalues = c->nvals;
    return SMX_OK;
}

}  // extern "C"
