// Batched render plans: heterogeneous work items (volume, detector, pose,
// outputs) rendered in one execute, either by persistent kernels that pull
// ray tiles from device queues or by one workgroup per tile (chosen per
// output group, or fixed), optionally replayed from captured HIP graphs,
// with the launch shape chosen by timing candidates (autotuner).
//
// Groups.  Each execute call groups its items by output mode (image /
// image + counts / image + Jacobian / fused -ZNCC objective) and lays the
// tiles of each group out item after item.  Items of the objective group
// write per-tile moment sums to their own scratch; a finalize kernel, one
// workgroup per item, then reduces them in a fixed order into the item's
// loss and pose gradient.
//
// Queues.  The tile range of a group is split into 8 contiguous shares, one
// per XCD; a persistent workgroup first drains the share of the XCD it runs
// on (hardware dispatch is round-robin over the XCDs), so concurrently
// running workgroups of one XCD render neighbouring tiles of one pose and
// share that XCD's L2, and then helps the other shares.  The counters are
// reset by a small kernel at the start of every execute (no memset nodes in
// the graph).  Which workgroup renders a tile never changes a result: tiles
// are independent and each writes only its own pixels.
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "reduce_common.hpp"

namespace drr {

constexpr int kPlanModes = 4;   // groups: kImage, kCount, kJac, kNcc (see group_mode)
constexpr int kXcds = 8;
constexpr int kRing = 4;        // item tables in flight
constexpr size_t kMaxGraphsPerSlot = 16;   // captured launches kept per item table
constexpr int kMaxPlanItems = 8192;

struct PlanItem {
    VolArgs vol;
    DetArgs det;
    const float* pose;
    float* image;
    float* jac;
    int32_t* counts;
    const float* target;  // objective items
    float* loss;
    float* grad;
    double* partials;     // [tiles][kNccSums]
    int32_t tiles_x;
    int32_t tile_begin;   // first tile of this item within its group
    int32_t tiles;        // tiles of this item
    int32_t pad;
};

// Render mode of group g (groups are indexed 0..kPlanModes-1).
__host__ __device__ constexpr int group_mode(int g)
{
    return g == 0 ? kImage : (g == 1 ? kCount : (g == 2 ? kJac : kNcc));
}

struct PlanHeader {
    int32_t first[kPlanModes];     // first item of each group
    int32_t count[kPlanModes];     // items per group
    int32_t tiles[kPlanModes];     // tiles per group
    int32_t uniform[kPlanModes];   // tiles per item when all items of the group
                                   // have the same count, else 0
};
// the item table follows the header: keep its doubles aligned
static_assert(sizeof(PlanHeader) % 16 == 0, "PlanHeader size must keep items aligned");

struct Slot {
    PlanHeader* h_header = nullptr;   // pinned: header followed by items
    PlanItem* h_items = nullptr;
    char* d_block = nullptr;          // device copy of header + items
    int32_t* d_counters = nullptr;    // [kPlanModes][kXcds]
    hipEvent_t done = nullptr;
    bool used = false;
    std::map<std::vector<int>, hipGraphExec_t> graphs;   // by mode mask (+ flat grids)
};

// ------------------------------------------------------------------ kernels

__global__ void k_reset_counters(int32_t* c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// Item of tile t within group g: a division when all items of the group have
// the same tile count, else a binary search for the last item whose first
// tile is <= t.  Every operand is wave-uniform.
__device__ inline int item_of_tile(const PlanHeader* hdr, const PlanItem* items, int g, int t)
{
    const int u = hdr->uniform[g];
    if (u > 0) return t / u;
    const int first = hdr->first[g];
    int lo = 0, hi = hdr->count[g] - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[first + mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Next tile of group `g` for a workgroup on XCD `xcd`, or -1 when drained.
__device__ inline int next_tile(int32_t* counters, int total, int xcd, int* scan)
{
    while (*scan < kXcds) {
        const int q = (xcd + *scan) % kXcds;
        const int lo = (int)(((int64_t)total * q) / kXcds);
        const int hi = (int)(((int64_t)total * (q + 1)) / kXcds);
        const int t = atomicAdd(&counters[q], 1);
        if (lo + t < hi) return lo + t;
        ++*scan;
    }
    return -1;
}

template <int TW, int WX, int WY, int MODE>
__global__ __launch_bounds__(64 * WX * WY) void render_persistent(const char* __restrict__ block,
                                                                  int32_t* counters, int group)
{
    using S = TileShape<TW, WX, WY>;
    __shared__ int s_tile;
    __shared__ double lds[MODE == kNcc ? kNccSums * WX * WY : 1];
    static_assert(sizeof(lds) + sizeof(s_tile) <=
                      16 + tile_sum_lds_bytes(MODE == kNcc ? kNccSums : 0, WX * WY),
                  "static LDS budget");
    const PlanHeader* hdr = (const PlanHeader*)block;
    const PlanItem* items = (const PlanItem*)(block + sizeof(PlanHeader));
    const int first = hdr->first[group], total = hdr->tiles[group];
    int32_t* ctr = counters + group * kXcds;
    const int xcd = (int)(blockIdx.x % kXcds);
    int scan = 0;
    for (;;) {
        if (threadIdx.x == 0) s_tile = next_tile(ctr, total, xcd, &scan);
        __syncthreads();
        // uniform across the workgroup: keep the item lookup and the item's
        // fields in scalar registers
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t < 0) break;
        const PlanItem& it = items[first + item_of_tile(hdr, items, group, t)];
        const int local = t - it.tile_begin;
        const int ty = local / it.tiles_x, tx = local % it.tiles_x;
        TileOut o;
        o.image = it.image;
        o.jac = it.jac;
        o.counts = it.counts;
        o.aux = MODE == kNcc ? it.target : nullptr;
        o.partial = MODE == kNcc ? it.partials + (int64_t)local * kNccSums : nullptr;
        // (lean in the Jacobian modes: the loop over tiles and the item
        // fields would otherwise push them past 128 VGPRs, below four waves
        // per SIMD)
        render_tile<TW, WX, WY, MODE, full_depth<MODE>(), ModeTraits<MODE>::jac>(
            it.vol, it.det, it.pose, tx, ty, o, lds);
    }
    (void)sizeof(S);
}

// Flat strategy: one workgroup per tile (grid = the group's tile count), the
// hardware dispatcher as the queue, with the XCD-aware ordering of the
// direct launches.  No atomics; the grid size is fixed per execute.
template <int TW, int WX, int WY, int MODE>
__global__ __launch_bounds__(64 * WX * WY) void render_plan_flat(const char* __restrict__ block,
                                                                 int group)
{
    __shared__ double lds[MODE == kNcc ? kNccSums * WX * WY : 1];
    static_assert(sizeof(lds) <= 16 + tile_sum_lds_bytes(MODE == kNcc ? kNccSums : 0, WX * WY),
                  "static LDS budget");
    const PlanHeader* hdr = (const PlanHeader*)block;
    const PlanItem* items = (const PlanItem*)(block + sizeof(PlanHeader));
    const int t = (int)xcd_logical(blockIdx.x, gridDim.x);
    const PlanItem& it = items[hdr->first[group] + item_of_tile(hdr, items, group, t)];
    const int local = t - it.tile_begin;
    const int ty = local / it.tiles_x, tx = local % it.tiles_x;
    TileOut o;
    o.image = it.image;
    o.jac = it.jac;
    o.counts = it.counts;
    o.aux = MODE == kNcc ? it.target : nullptr;
    o.partial = MODE == kNcc ? it.partials + (int64_t)local * kNccSums : nullptr;
    // the flat grid serves small groups under the default strategy: the deep
    // pipeline keeps a lone wave's gathers in flight
    render_tile<TW, WX, WY, MODE, kDeepDepth>(it.vol, it.det, it.pose, tx, ty, o, lds);
}

// Loss and pose gradient of every objective item: workgroup i reduces the
// tile sums of item first + i in a fixed order.
__global__ __launch_bounds__(kReduceThreads) void k_plan_ncc_finalize(
    const char* __restrict__ block, int group)
{
    __shared__ double lds[kReduceThreads * kNccSums];
    const PlanHeader* hdr = (const PlanHeader*)block;
    const PlanItem* items = (const PlanItem*)(block + sizeof(PlanHeader));
    const PlanItem& it = items[hdr->first[group] + (int)blockIdx.x];
    sum_tile_partials<kNccSums>(it.partials, it.tiles, lds);
    ncc_from_sums(lds, (double)it.det.H * (double)it.det.W, it.loss, it.grad);
}

// ------------------------------------------------------------------ shapes

typedef void (*PersistentFn)(const char*, int32_t*, int);

template <int MODE>
static PersistentFn persistent_fn(int code)
{
    switch (code) {
    case 0: return render_persistent<8, 2, 2, MODE>;
    case 1: return render_persistent<8, 1, 1, MODE>;
    case 2: return render_persistent<8, 1, 4, MODE>;
    case 3: return render_persistent<16, 1, 4, MODE>;
    case 4: return render_persistent<4, 4, 1, MODE>;
    case 5: return render_persistent<8, 4, 1, MODE>;
    case 6: return render_persistent<4, 1, 4, MODE>;
    case 7: return render_persistent<2, 2, 2, MODE>;
    default: return render_persistent<1, 4, 1, MODE>;
    }
}

static PersistentFn kernel_for(int group, int code)
{
    switch (group_mode(group)) {
    case kImage: return persistent_fn<kImage>(code);
    case kCount: return persistent_fn<kCount>(code);
    case kJac: return persistent_fn<kJac>(code);
    default: return persistent_fn<kNcc>(code);
    }
}

typedef void (*FlatFn)(const char*, int);

template <int MODE>
static FlatFn flat_fn(int code)
{
    switch (code) {
    case 0: return render_plan_flat<8, 2, 2, MODE>;
    case 1: return render_plan_flat<8, 1, 1, MODE>;
    case 2: return render_plan_flat<8, 1, 4, MODE>;
    case 3: return render_plan_flat<16, 1, 4, MODE>;
    case 4: return render_plan_flat<4, 4, 1, MODE>;
    case 5: return render_plan_flat<8, 4, 1, MODE>;
    case 6: return render_plan_flat<4, 1, 4, MODE>;
    case 7: return render_plan_flat<2, 2, 2, MODE>;
    default: return render_plan_flat<1, 4, 1, MODE>;
    }
}

static FlatFn flat_kernel_for(int group, int code)
{
    switch (group_mode(group)) {
    case kImage: return flat_fn<kImage>(code);
    case kCount: return flat_fn<kCount>(code);
    case kJac: return flat_fn<kJac>(code);
    default: return flat_fn<kNcc>(code);
    }
}

enum Strategy { kPersistent = 0, kFlat = 1, kAuto = 2 };

// Group of an item: 0 image, 1 image + counts, 2 image + Jacobian,
// 3 objective.
static int group_of_flags(int32_t flags)
{
    if (flags & DRR_ITEM_NCC) return 3;
    if (flags & DRR_ITEM_JAC) return 2;
    if (flags & DRR_ITEM_COUNT) return 1;
    return 0;
}

// Upper bound of the static LDS of group g's plan kernels: the tile index
// and the block-sum buffer of the objective group.
static size_t plan_static_lds(int g, const ShapeInfo& sh)
{
    return 16 + tile_sum_lds_bytes(group_mode(g) == kNcc ? kNccSums : 0, sh.wx * sh.wy);
}

// Tiles of a detector for launch shape `code`.
static int64_t tiles_for(const drr_detector_desc& d, int code, int* tiles_x)
{
    const ShapeInfo& sh = kShapes[code];
    const int pxw = sh.tw * sh.wx, pxh = (64 / sh.tw) * sh.wy;
    const int tx = (d.width + pxw - 1) / pxw, ty = (d.height + pxh - 1) / pxh;
    if (tiles_x) *tiles_x = tx;
    return (int64_t)tx * ty;
}

}  // namespace drr

using namespace drr;

struct drr_plan {
    int max_items = 0;
    std::vector<drr_volume_desc> vols;
    std::vector<const void*> packed;
    int strategy = 0;          // kPersistent, kFlat or kAuto
    int tile_code = 0;
    int wg_per_cu = 0;         // requested workgroups per CU (0 = occupancy limit)
    int grid[kPlanModes] = {0, 0, 0, 0};   // persistent grid per group
    int num_cus = 0;
    bool use_graph = false;
    Slot slots[kRing];
    int next = 0;
    std::mutex mu;
};

namespace drr {

static size_t table_bytes(int max_items)
{
    return sizeof(PlanHeader) + (size_t)max_items * sizeof(PlanItem);
}

static int32_t compute_grids(drr_plan* p)
{
    const ShapeInfo& sh = kShapes[p->tile_code];
    const int threads = 64 * sh.wx * sh.wy;
    for (int m = 0; m < kPlanModes; ++m) {
        int occ = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, (const void*)kernel_for(m, p->tile_code), threads, 0);
        if (e != hipSuccess || occ < 1)
            return fail(DRR_EHIP, "occupancy query failed: %s", hipGetErrorString(e));
        int per = p->wg_per_cu > 0 && p->wg_per_cu < occ ? p->wg_per_cu : occ;
        p->grid[m] = per * p->num_cus;
        // whole multiples of the XCD count keep the XCD shares balanced
        p->grid[m] = ((p->grid[m] + kXcds - 1) / kXcds) * kXcds;
    }
    return DRR_OK;
}

// Fills slot `s` for the given items; returns the mode mask via *mask.
static int32_t stage_items(drr_plan* p, Slot& s, const drr_work_item* items, int n, int* mask)
{
    PlanHeader* h = s.h_header;
    int pos = 0;
    *mask = 0;
    for (int m = 0; m < kPlanModes; ++m) {
        h->first[m] = pos;
        h->count[m] = 0;
        h->uniform[m] = 0;
        int64_t tiles = 0, per = -1;
        for (int i = 0; i < n; ++i) {
            const drr_work_item& w = items[i];
            if (group_of_flags(w.flags) != m) continue;
            PlanItem& it = s.h_items[pos++];
            it.vol = vol_args(p->packed[w.volume], p->vols[w.volume]);
            it.det = det_args(w.det);
            it.pose = w.pose;
            it.image = w.image;
            it.jac = w.jac;
            it.counts = w.counts;
            it.target = w.target;
            it.loss = w.loss;
            it.grad = w.grad;
            it.partials = w.partials;
            const int64_t t = tiles_for(w.det, p->tile_code, &it.tiles_x);
            it.tiles = (int32_t)t;
            it.tile_begin = (int32_t)tiles;
            tiles += t;
            per = per == -1 || per == t ? t : 0;
            h->count[m]++;
        }
        if (per > 0 && per <= 0x7FFFFFFF) h->uniform[m] = (int32_t)per;
        if (tiles > 0x7FFFFFFF) return fail(DRR_ENOTSUP, "too many tiles in one execute");
        h->tiles[m] = (int32_t)tiles;
        if (tiles > 0) *mask |= 1 << m;
    }
    return DRR_OK;
}

// The objective group's losses and gradients, after its tiles are rendered.
static int32_t enqueue_finalize(Slot& s, int mask, hipStream_t st)
{
    constexpr int g = 3;
    if (!(mask & (1 << g))) return DRR_OK;
    hipLaunchKernelGGL(k_plan_ncc_finalize, dim3(s.h_header->count[g]), dim3(kReduceThreads), 0,
                       st, (const char*)s.d_block, g);
    return check_launch("plan objective finalize");
}

// Strategy of group m in the staged execute.
static int group_strategy(const drr_plan* p, const Slot& s, int m)
{
    if (p->strategy != kAuto) return p->strategy;
    return s.h_header->tiles[m] <= p->grid[m] ? kFlat : kPersistent;
}

static int32_t enqueue_kernels(drr_plan* p, Slot& s, int mask, hipStream_t st)
{
    const ShapeInfo& sh = kShapes[p->tile_code];
    const int threads = 64 * sh.wx * sh.wy;
    int32_t rc;
    bool counters_reset = false;
    for (int m = 0; m < kPlanModes; ++m) {
        if (!(mask & (1 << m))) continue;
        if (group_strategy(p, s, m) == kFlat) {
            const size_t lds = occupancy_lds(p->wg_per_cu, plan_static_lds(m, sh));
            hipLaunchKernelGGL(flat_kernel_for(m, p->tile_code), dim3(s.h_header->tiles[m]),
                               dim3(threads), lds, st, (const char*)s.d_block, m);
            if ((rc = check_launch("plan flat kernel"))) return rc;
            continue;
        }
        if (!counters_reset) {
            hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, st, s.d_counters,
                               kPlanModes * kXcds);
            if ((rc = check_launch("plan counter reset"))) return rc;
            counters_reset = true;
        }
        hipLaunchKernelGGL(kernel_for(m, p->tile_code), dim3(p->grid[m]), dim3(threads), 0, st,
                           (const char*)s.d_block, s.d_counters, m);
        if ((rc = check_launch("plan persistent kernel"))) return rc;
    }
    return enqueue_finalize(s, mask, st);
}

static void drop_graphs(Slot& s)
{
    for (auto& kv : s.graphs) (void)hipGraphExecDestroy(kv.second);
    s.graphs.clear();
}

static int32_t execute_locked(drr_plan* p, const drr_work_item* items, int n, hipStream_t st)
{
    Slot& s = p->slots[p->next];
    p->next = (p->next + 1) % kRing;
    if (s.used) {
        hipError_t e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return fail(DRR_EHIP, "plan slot wait: %s", hipGetErrorString(e));
    }
    int mask = 0;
    int32_t rc = stage_items(p, s, items, n, &mask);
    if (rc) return rc;
    const size_t bytes = sizeof(PlanHeader) + (size_t)n * sizeof(PlanItem);
    hipError_t e = hipMemcpyAsync(s.d_block, s.h_header, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(DRR_EHIP, "plan table copy: %s", hipGetErrorString(e));
    if (p->use_graph && st != nullptr) {
        // what the captured launches depend on: groups present, the
        // finalize grid, and each group's strategy with its flat grid size
        std::vector<int> key = {mask, s.h_header->count[3]};
        for (int m = 0; m < kPlanModes; ++m) {
            const int g = group_strategy(p, s, m);
            key.push_back(g);
            key.push_back(g == kFlat ? s.h_header->tiles[m] : 0);
        }
        auto found = s.graphs.find(key);
        if (found == s.graphs.end()) {
            // bound the cache: batches of ever new shapes would otherwise
            // keep one executable graph each (this slot's last launch has
            // completed, so its graphs are idle)
            if (s.graphs.size() >= kMaxGraphsPerSlot) drop_graphs(s);
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return fail(DRR_EHIP, "begin capture: %s", hipGetErrorString(e));
            rc = enqueue_kernels(p, s, mask, st);
            hipError_t e2 = hipStreamEndCapture(st, &g);
            if (rc) return rc;
            if (e2 != hipSuccess) return fail(DRR_EHIP, "end capture: %s", hipGetErrorString(e2));
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(DRR_EHIP, "graph instantiate: %s", hipGetErrorString(e));
            found = s.graphs.emplace(key, ge).first;
        }
        e = hipGraphLaunch(found->second, st);
        if (e != hipSuccess) return fail(DRR_EHIP, "graph launch: %s", hipGetErrorString(e));
    } else {
        rc = enqueue_kernels(p, s, mask, st);
        if (rc) return rc;
    }
    e = hipEventRecord(s.done, st);
    if (e != hipSuccess) return fail(DRR_EHIP, "plan event: %s", hipGetErrorString(e));
    s.used = true;
    return DRR_OK;
}

static int32_t validate_items(const drr_plan* p, const drr_work_item* items, int n)
{
    if (n < 0 || n > p->max_items)
        return fail(DRR_EINVAL, "plan execute: %d items (capacity %d)", n, p->max_items);
    if (n > 0 && !items) return fail(DRR_EINVAL, "plan execute: items is NULL");
    for (int i = 0; i < n; ++i) {
        const drr_work_item& w = items[i];
        if (w.volume < 0 || w.volume >= (int)p->vols.size())
            return fail(DRR_EINVAL, "item %d: volume index %d out of range", i, w.volume);
        int32_t rc = validate_detector(&w.det);
        if (rc) return rc;
        if (!w.pose) return fail(DRR_EINVAL, "item %d: NULL pose", i);
        if (!w.image && !(w.flags & DRR_ITEM_NCC))
            return fail(DRR_EINVAL, "item %d: NULL image", i);
        if ((w.flags & DRR_ITEM_JAC) && !w.jac) return fail(DRR_EINVAL, "item %d: NULL jac", i);
        if ((w.flags & DRR_ITEM_COUNT) && !w.counts)
            return fail(DRR_EINVAL, "item %d: NULL counts", i);
        const int kinds = ((w.flags & DRR_ITEM_JAC) ? 1 : 0) + ((w.flags & DRR_ITEM_COUNT) ? 1 : 0) +
                          ((w.flags & DRR_ITEM_NCC) ? 1 : 0);
        if (kinds > 1) return fail(DRR_EINVAL, "item %d: JAC, COUNT and NCC are exclusive", i);
        if (w.flags & ~(DRR_ITEM_JAC | DRR_ITEM_COUNT | DRR_ITEM_NCC))
            return fail(DRR_EINVAL, "item %d: unknown flags 0x%x", i, (unsigned)w.flags);
        if (w.flags & DRR_ITEM_NCC) {
            if (!w.target || !w.loss || !w.grad || !w.partials)
                return fail(DRR_EINVAL, "item %d: NULL target, loss, grad or partials", i);
            if ((int64_t)w.det.height * w.det.width < 2)
                return fail(DRR_EINVAL, "item %d: the objective needs at least 2 pixels", i);
        }
    }
    return DRR_OK;
}

// ------------------------------------------------------------------ autotune

static std::string tune_key(const drr_plan* p, const drr_work_item* items, int n)
{
    std::string k = "v2";
    for (const auto& v : p->vols) {
        char b[96];
        snprintf(b, sizeof b, "|%dx%dx%d@%.3g,%.3g,%.3g", v.nx, v.ny, v.nz, v.spacing[0],
                 v.spacing[1], v.spacing[2]);
        k += b;
    }
    int64_t px[kPlanModes] = {0, 0, 0, 0};
    for (int i = 0; i < n; ++i)
        px[group_of_flags(items[i].flags)] += (int64_t)items[i].det.height * items[i].det.width;
    char b[128];
    snprintf(b, sizeof b, "|n%d|px%lld,%lld,%lld", n, (long long)px[0], (long long)px[1],
             (long long)px[2]);
    k += b;
    if (px[3] > 0) {   // older cache lines (no objective items) keep their keys
        snprintf(b, sizeof b, ",%lld", (long long)px[3]);
        k += b;
    }
    return k;
}

static bool cache_lookup(const char* path, const std::string& key, int* strategy, int* code,
                         int* wpc)
{
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool hit = false;
    while (fgets(line, sizeof line, f)) {
        char k[900];
        int g, c, w;
        if (sscanf(line, "%899s %d %d %d", k, &g, &c, &w) == 4 && key == k &&
            (g == kPersistent || g == kFlat) && c >= 0 && c < kNumShapes && w >= 0) {
            *strategy = g;
            *code = c;
            *wpc = w;
            hit = true;
        }
    }
    fclose(f);
    return hit;
}

static void cache_store(const char* path, const std::string& key, int strategy, int code,
                        int wpc)
{
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d\n", key.c_str(), strategy, code, wpc);
    fclose(f);
}

static int32_t time_config(drr_plan* p, const drr_work_item* items, int n, hipStream_t st,
                           float* ms)
{
    int32_t rc = compute_grids(p);
    if (rc) return rc;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(DRR_EHIP, "autotune: event creation failed");
    rc = execute_locked(p, items, n, st);   // warm-up (also captures the graph)
    const int reps = 3;
    (void)hipEventRecord(a, st);
    for (int r = 0; r < reps && rc == DRR_OK; ++r) rc = execute_locked(p, items, n, st);
    (void)hipEventRecord(b, st);
    hipError_t e = hipEventSynchronize(b);
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    if (e != hipSuccess) return fail(DRR_EHIP, "autotune sync: %s", hipGetErrorString(e));
    *ms = t / reps;
    return DRR_OK;
}

static int32_t autotune(drr_plan* p, const drr_work_item* items, int n, hipStream_t st,
                        const char* cache)
{
    const std::string key = tune_key(p, items, n);
    int strategy = 0, code = 0, wpc = 0;
    if (cache_lookup(cache, key, &strategy, &code, &wpc)) {
        p->strategy = strategy;
        p->tile_code = code;
        p->wg_per_cu = wpc;
        return compute_grids(p);
    }
    float best = 1e30f;
    int best_code = 0, best_wpc = 0, best_strategy = kPersistent;
    // resident workgroups per CU: the register limit, or fewer (less cache
    // pressure from concurrent rays)
    const int wpcs[] = {0, 3, 4, 5, 6};
    for (int strat = kPersistent; strat <= kFlat; ++strat) {
        for (int c = 0; c < kNumShapes; ++c) {
            for (int w : wpcs) {
                p->strategy = strat;
                p->tile_code = c;
                p->wg_per_cu = w;
                for (Slot& s : p->slots) drop_graphs(s);
                float ms = 0.0f;
                int32_t rc = time_config(p, items, n, st, &ms);
                if (rc) return rc;
                if (ms < best) {
                    best = ms;
                    best_code = c;
                    best_wpc = w;
                    best_strategy = strat;
                }
            }
        }
    }
    for (Slot& s : p->slots) drop_graphs(s);
    p->strategy = best_strategy;
    p->tile_code = best_code;
    p->wg_per_cu = best_wpc;
    cache_store(cache, key, best_strategy, best_code, best_wpc);
    return compute_grids(p);
}

static void free_plan(drr_plan* p)
{
    for (Slot& s : p->slots) {
        if (s.used && s.done) (void)hipEventSynchronize(s.done);
        drop_graphs(s);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.h_header) (void)hipHostFree(s.h_header);
        if (s.d_block) (void)hipFree(s.d_block);
        if (s.d_counters) (void)hipFree(s.d_counters);
    }
    delete p;
}

}  // namespace drr

extern "C" {

int32_t drr_plan_create(const drr_plan_desc* desc, const drr_work_item* tune_items,
                        int32_t n_tune_items, void* stream, drr_plan** out)
{
    if (!desc || !out) return fail(DRR_EINVAL, "plan_create: NULL argument");
    *out = nullptr;
    if (desc->max_items < 1 || desc->max_items > kMaxPlanItems)
        return fail(DRR_EINVAL, "plan_create: max_items must be in [1, %d]", kMaxPlanItems);
    if (desc->n_volumes < 1 || !desc->volumes || !desc->packed)
        return fail(DRR_EINVAL, "plan_create: need at least one volume");
    drr_plan* p = new drr_plan();
    p->max_items = desc->max_items;
    p->use_graph = desc->use_graph != 0;
    for (int v = 0; v < desc->n_volumes; ++v) {
        int32_t rc = validate_volume(&desc->volumes[v]);
        if (rc || !desc->packed[v]) {
            delete p;
            return rc ? rc : fail(DRR_EINVAL, "plan_create: packed[%d] is NULL", v);
        }
        p->vols.push_back(desc->volumes[v]);
        p->packed.push_back(desc->packed[v]);
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        p->num_cus = 0;
    if (p->num_cus < 1) p->num_cus = 1;
    const size_t tb = table_bytes(p->max_items);
    for (Slot& s : p->slots) {
        if (hipHostMalloc((void**)&s.h_header, tb, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void**)&s.d_block, tb) != hipSuccess ||
            hipMalloc((void**)&s.d_counters, kPlanModes * kXcds * sizeof(int32_t)) !=
                hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
            free_plan(p);
            return fail(DRR_ENOMEM, "plan_create: allocation failed");
        }
        s.h_items = (PlanItem*)((char*)s.h_header + sizeof(PlanHeader));
    }
    if (!desc->autotune) {
        if (desc->tile_code >= kNumShapes) {
            free_plan(p);
            return fail(DRR_EINVAL, "plan_create: tile_code must be < %d", kNumShapes);
        }
        if (desc->strategy > kAuto) {
            free_plan(p);
            return fail(DRR_EINVAL, "plan_create: unknown strategy %d", desc->strategy);
        }
        // defaults: the launch shape the autotuner picks for the 512 x 512 x
        // 133 CT with 256 x 256 detectors (4 workgroups per CU keep the
        // gather working set in cache), and the strategy chosen per execute
        p->strategy = desc->strategy >= 0 ? desc->strategy : kAuto;
        p->tile_code = desc->tile_code >= 0 ? desc->tile_code : 4;
        p->wg_per_cu = desc->wg_per_cu >= 0 ? desc->wg_per_cu : 4;
    }
    int32_t rc = compute_grids(p);
    if (rc == DRR_OK && desc->autotune) {
        if (n_tune_items < 1 || !tune_items) {
            rc = fail(DRR_EINVAL, "plan_create: autotune needs sample items");
        } else if ((rc = validate_items(p, tune_items, n_tune_items)) == DRR_OK) {
            rc = autotune(p, tune_items, n_tune_items, as_stream(stream), desc->tune_cache_path);
        }
    }
    if (rc) {
        free_plan(p);
        return rc;
    }
    *out = p;
    return DRR_OK;
}

int32_t drr_plan_execute(drr_plan* plan, const drr_work_item* items, int32_t n_items,
                         void* stream)
{
    if (!plan) return fail(DRR_EINVAL, "plan_execute: NULL plan");
    std::lock_guard<std::mutex> lock(plan->mu);
    int32_t rc = validate_items(plan, items, n_items);
    if (rc) return rc;
    if (n_items == 0) return DRR_OK;
    return execute_locked(plan, items, n_items, as_stream(stream));
}

int32_t drr_plan_config(const drr_plan* plan, int32_t* strategy, int32_t* tile_code,
                        int32_t* wg_per_cu, int32_t* use_graph)
{
    if (!plan) return fail(DRR_EINVAL, "plan_config: NULL plan");
    if (strategy) *strategy = plan->strategy;
    if (tile_code) *tile_code = plan->tile_code;
    if (wg_per_cu) *wg_per_cu = plan->wg_per_cu;
    if (use_graph) *use_graph = plan->use_graph ? 1 : 0;
    return DRR_OK;
}

void drr_plan_destroy(drr_plan* plan)
{
    if (plan) free_plan(plan);
}

size_t drr_plan_item_workspace_bytes(const drr_detector_desc* det)
{
    if (!det || validate_detector(det) != DRR_OK) return 0;
    int64_t most = 0;
    for (int c = 0; c < kNumShapes; ++c) {
        const int64_t t = tiles_for(*det, c, nullptr);
        most = t > most ? t : most;
    }
    return (size_t)most * kNccSums * sizeof(double);
}

}  // extern "C"
