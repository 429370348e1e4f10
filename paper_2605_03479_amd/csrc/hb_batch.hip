// Batched form of the HB-UGKS pseudo step (see the batched section of hb_ugks.h).
//
// A batch holds many cases (each a full hb_ugks handle whose device memory is
// carved from the batch's pool).  One batch step advances every active case
// by one pseudo step with one launch per kernel phase over all of them (the
// update phase: one launch per (precision, N_T) group, since the level count
// is a template parameter), recorded once into a HIP graph and replayed.  The
// launch shape of each phase (threads per block for the update, blocks per
// CU of the persistent grid) is chosen by a tuner that times the candidates
// on the batch itself and remembers the winner per (precision, N_T, N_v).
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "hb_batch_kernels.h"
#include "hb_handle.h"

namespace {

using hb::CaseCtl;
using hb::CaseDev;
using hb::WorkItem;

// A work list on the device with the block ranges of its persistent launch.
struct DevList {
    std::vector<WorkItem> items;
    std::vector<double> cost;
    WorkItem *d_items = nullptr;
    int *d_bstart = nullptr;
    int grid = 0;
    int tpb = 0;

    void free_dev()
    {
        if (d_items) (void)hipFree(d_items);
        if (d_bstart) (void)hipFree(d_bstart);
        d_items = nullptr;
        d_bstart = nullptr;
        grid = 0;
    }
    // cut the list into `g` contiguous ranges of about equal cost and upload
    int upload(int g, int threads)
    {
        free_dev();
        tpb = threads;
        const int n = (int)items.size();
        if (n == 0) return HB_OK;
        g = std::max(1, std::min(g, n));
        std::vector<int> bs(g + 1, n);
        if (g == n) {  // one item per block
            for (int q = 0; q <= n; q++) bs[q] = q;
        }
        double tot = 0.0;
        for (double c : cost) tot += c;
        bs[0] = 0;
        double acc = 0.0;
        int k = g == n ? g : 1;
        for (int i = 0; i < n && k < g; i++) {
            acc += cost[i];
            while (k < g && acc >= tot * k / g) bs[k++] = i + 1;
        }
        for (; k < g; k++) bs[k] = n;
        for (int q = 1; q <= g; q++) bs[q] = std::max(bs[q], bs[q - 1]);
        if (hipMalloc((void **)&d_items, sizeof(WorkItem) * n) != hipSuccess ||
            hipMalloc((void **)&d_bstart, sizeof(int) * (g + 1)) != hipSuccess) {
            (void)hipGetLastError();
            free_dev();
            return HB_ENOMEM;
        }
        HIPOK(hipMemcpy(d_items, items.data(), sizeof(WorkItem) * n, hipMemcpyHostToDevice));
        HIPOK(hipMemcpy(d_bstart, bs.data(), sizeof(int) * (g + 1), hipMemcpyHostToDevice));
        grid = g;
        return HB_OK;
    }
};

// Launch shape of one phase: threads per block and persistent blocks per CU
// (0 = one item per block).
struct Shape {
    int tpb, per_cu;
};

struct UpdGroup {
    int prec = HB_FP64, NT = 1, Mt = 0;  // Mt: table stride, max(M, M_v)
    bool so = false;                     // non-temporal stores of the update (the cases' Params::stream_out)
    int max_nvp = 0;
    size_t lds = 0;
    DevList in, bn;
    Shape shape{256, 0};
};

// tuner memory: (precision, NT, nvp) -> shape of the update phase; (precision, 0, nvp) -> moments
std::map<std::tuple<int, int, int>, Shape> g_tuned;

template <int NT, typename TS, bool SO>
int set_batch_lds_so(size_t bytes)
{
    if (hipFuncSetAttribute((const void *)hb::kb_update_int<NT, TS, SO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes) != hipSuccess ||
        hipFuncSetAttribute((const void *)hb::kb_update_bnd<NT, TS, SO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes) != hipSuccess)
        return HB_EDEVICE;
    return HB_OK;
}
template <int NT, typename TS>
int set_batch_lds_t(size_t bytes)
{
    if (bytes <= 64 * 1024) return HB_OK;
    const int rc = set_batch_lds_so<NT, TS, false>(bytes);
    if constexpr (sizeof(TS) == 4) {
        if (rc == HB_OK) return set_batch_lds_so<NT, TS, true>(bytes);
    }
    return rc;
}

template <typename TS>
int set_batch_lds_p(int NT, size_t bytes)
{
    switch (NT) {
    case 1: return set_batch_lds_t<1, TS>(bytes);
    case 3: return set_batch_lds_t<3, TS>(bytes);
    case 5: return set_batch_lds_t<5, TS>(bytes);
    case 7: return set_batch_lds_t<7, TS>(bytes);
    case 9: return set_batch_lds_t<9, TS>(bytes);
    default: return set_batch_lds_t<11, TS>(bytes);
    }
}

template <int NT, typename TS, bool SO>
void launch_group_so(const UpdGroup &g, const CaseDev *cs, const CaseCtl *ctl, hipStream_t st, bool interior,
                     bool ring)
{
    if (interior && g.in.grid)
        hipLaunchKernelGGL((hb::kb_update_int<NT, TS, SO>), dim3(g.in.grid), dim3(g.in.tpb), g.lds, st, cs, ctl,
                           g.in.d_items, g.in.d_bstart);
    if (ring && g.bn.grid)
        hipLaunchKernelGGL((hb::kb_update_bnd<NT, TS, SO>), dim3(g.bn.grid), dim3(g.bn.tpb), g.lds, st, cs, ctl,
                           g.bn.d_items, g.bn.d_bstart);
}
template <int NT, typename TS>
void launch_group_t(const UpdGroup &g, const CaseDev *cs, const CaseCtl *ctl, hipStream_t st, bool interior,
                    bool ring)
{
    if constexpr (sizeof(TS) == 4) {
        if (g.so) {
            launch_group_so<NT, TS, true>(g, cs, ctl, st, interior, ring);
            return;
        }
    }
    launch_group_so<NT, TS, false>(g, cs, ctl, st, interior, ring);
}

template <typename TS>
void launch_group_p(const UpdGroup &g, const CaseDev *cs, const CaseCtl *ctl, hipStream_t st, bool in, bool rg)
{
    switch (g.NT) {
    case 1: launch_group_t<1, TS>(g, cs, ctl, st, in, rg); break;
    case 3: launch_group_t<3, TS>(g, cs, ctl, st, in, rg); break;
    case 5: launch_group_t<5, TS>(g, cs, ctl, st, in, rg); break;
    case 7: launch_group_t<7, TS>(g, cs, ctl, st, in, rg); break;
    case 9: launch_group_t<9, TS>(g, cs, ctl, st, in, rg); break;
    default: launch_group_t<11, TS>(g, cs, ctl, st, in, rg); break;
    }
}

void launch_group(const UpdGroup &g, const CaseDev *cs, const CaseCtl *ctl, hipStream_t st, bool in = true,
                  bool rg = true)
{
    if (g.prec == HB_MIXED) launch_group_p<float>(g, cs, ctl, st, in, rg);
    else launch_group_p<double>(g, cs, ctl, st, in, rg);
}

// Cases run phase by phase together.  Groups are sized so that the device
// footprint of their cases fits the Infinity Cache, and one group's whole step
// runs before the next group's: the stencil re-reads of the cell-per-block
// kernels then hit the cache instead of HBM, while small cases still share
// launches and fill the GPU.
struct CacheGroup {
    DevList mom[2], faces, cells, dts, resid;
    std::vector<UpdGroup> groups;
    Shape mom_shape[2]{{256, 0}, {256, 0}};
    int mom_nvp[2]{0, 0};
    size_t bytes = 0;

    void free_dev()
    {
        for (auto &m : mom) m.free_dev();
        faces.free_dev();
        cells.free_dev();
        dts.free_dev();
        resid.free_dev();
        for (auto &g : groups) {
            g.in.free_dev();
            g.bn.free_dev();
        }
    }
};

}  // namespace

// streams a batch step spreads its cache groups over
#define HB_BATCH_LANES 4

struct hb_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // the further streams of a batch step (default priority): cache group k
    // runs on lane k % HB_BATCH_LANES (lane 0 is `stream`), the lanes forked
    // from and joined to `stream` once per step
    hipStream_t side[HB_BATCH_LANES - 1]{};
    hipEvent_t fork = nullptr, join = nullptr;
    int num_cu = 256;
    HbPool pool;
    int max_cases = 0;
    std::vector<hb_ugks *> cases;  // slot -> handle (null: free)
    std::vector<char> active;
    CaseDev *d_cs = nullptr;
    CaseCtl *d_ctl = nullptr;
    // work lists of the current active set, per cache group
    std::vector<CacheGroup> cgs;
    size_t cache_bytes = 224u << 20;  // device footprint per cache group
    std::vector<int> ids;              // active slots
    int *d_ids = nullptr;
    double *d_res = nullptr;
    long *d_steps = nullptr;
    int *d_flags = nullptr;
    bool lists_valid = false;
    // captured step
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = true;
    long steps = 0;
};

static void drop_graph(hb_batch *B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

static void drop_lists(hb_batch *B)
{
    (void)hipStreamSynchronize(B->stream);  // nothing in flight reads the lists below
    drop_graph(B);
    for (auto &cg : B->cgs) cg.free_dev();
    B->cgs.clear();
    if (B->d_ids) (void)hipFree(B->d_ids);
    if (B->d_res) (void)hipFree(B->d_res);
    if (B->d_steps) (void)hipFree(B->d_steps);
    if (B->d_flags) (void)hipFree(B->d_flags);
    B->d_ids = nullptr;
    B->d_res = nullptr;
    B->d_steps = nullptr;
    B->d_flags = nullptr;
    B->lists_valid = false;
}

static int grid_of(const hb_batch *B, const DevList &L, int per_cu)
{
    return per_cu <= 0 ? (int)L.items.size() : per_cu * B->num_cu;
}

// Work lists of the active cases: cases sorted by (precision, N_T, max(M, M_v)) and
// packed into cache groups; within a group, in case order then the case's own.
static int build_lists(hb_batch *B)
{
    drop_lists(B);
    B->ids.clear();
    for (int s = 0; s < B->max_cases; s++)
        if (B->cases[s] && B->active[s]) B->ids.push_back(s);
    std::vector<int> order = B->ids;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const hb_ugks *x = B->cases[a], *y = B->cases[b];
        return std::make_tuple(x->precision, x->P.NT, x->P.Mt, x->P.stream_out) <
               std::make_tuple(y->precision, y->P.NT, y->P.Mt, y->P.stream_out);
    });
    for (int s : order) {
        const hb_ugks *H = B->cases[s];
        if (B->cgs.empty() ||
            (B->cache_bytes && B->cgs.back().bytes > 0 && B->cgs.back().bytes + H->bytes > B->cache_bytes))
            B->cgs.emplace_back();
        CacheGroup &cg = B->cgs.back();
        cg.bytes += H->bytes;
        const hb::Params &P = H->P;
        const int pm = H->precision == HB_MIXED ? 1 : 0;
        const double cc = (double)P.nvp * P.NT;
        cg.mom_nvp[pm] = std::max(cg.mom_nvp[pm], P.nvp);
        for (int c = 0; c < P.nc; c++) {
            cg.mom[pm].items.push_back({s, hb::strip_cell(c, P.nx, P.ny)});
            cg.mom[pm].cost.push_back(cc);
        }
        const int nf = ((P.nx + 1) * P.ny + P.nx * (P.ny + 1)) * P.NT;
        for (int k = 0; k < (nf + 127) / 128; k++) {
            cg.faces.items.push_back({s, k});
            cg.faces.cost.push_back(1.0);
        }
        for (int k = 0; k < H->cells_blocks; k++) {
            cg.cells.items.push_back({s, k});
            cg.cells.cost.push_back(1.0);
        }
        for (int k = 0; k < (P.nc + 127) / 128; k++) {
            cg.dts.items.push_back({s, k});
            cg.dts.cost.push_back(1.0);
        }
        cg.resid.items.push_back({s, 0});
        cg.resid.cost.push_back((double)H->cells_blocks);
        if (cg.groups.empty() || cg.groups.back().prec != H->precision || cg.groups.back().NT != P.NT ||
            cg.groups.back().Mt != P.Mt || cg.groups.back().so != (P.stream_out != 0)) {
            cg.groups.emplace_back();
            cg.groups.back().prec = H->precision;
            cg.groups.back().NT = P.NT;
            cg.groups.back().Mt = P.Mt;
            cg.groups.back().so = P.stream_out != 0;
        }
        UpdGroup &g = cg.groups.back();
        g.max_nvp = std::max(g.max_nvp, P.nvp);
        g.lds = std::max(g.lds, H->upd_lds);
        for (int ci = 0; ci < H->n_int; ci++) {
            g.in.items.push_back({s, hb::strip_cell(ci, P.nx - 4, P.ny - 4)});
            g.in.cost.push_back(cc);
        }
        for (int c : H->bnd_host) {
            g.bn.items.push_back({s, c});
            g.bn.cost.push_back(cc * 1.35);
        }
    }
    int rc = HB_OK;
    for (auto &cg : B->cgs) {
        for (int pm = 0; pm < 2; pm++) {
            auto t = g_tuned.find(std::make_tuple(pm ? HB_MIXED : HB_FP64, 0, cg.mom_nvp[pm]));
            if (t != g_tuned.end()) cg.mom_shape[pm] = t->second;
            if ((rc = cg.mom[pm].upload(grid_of(B, cg.mom[pm], cg.mom_shape[pm].per_cu), 256)) != HB_OK) return rc;
        }
        if ((rc = cg.faces.upload(grid_of(B, cg.faces, 0), 128)) != HB_OK) return rc;
        if ((rc = cg.cells.upload(grid_of(B, cg.cells, 0), 128)) != HB_OK) return rc;
        if ((rc = cg.dts.upload(grid_of(B, cg.dts, 0), 128)) != HB_OK) return rc;
        if ((rc = cg.resid.upload(grid_of(B, cg.resid, 0), 256)) != HB_OK) return rc;
        for (auto &g : cg.groups) {
            auto t = g_tuned.find(std::make_tuple(g.prec, g.NT, g.max_nvp));
            if (t != g_tuned.end()) g.shape = t->second;
            if (g.prec == HB_MIXED) rc = set_batch_lds_p<float>(g.NT, g.lds);
            else rc = set_batch_lds_p<double>(g.NT, g.lds);
            if (rc != HB_OK) return rc;
            if ((rc = g.in.upload(grid_of(B, g.in, g.shape.per_cu), g.shape.tpb)) != HB_OK) return rc;
            if ((rc = g.bn.upload(grid_of(B, g.bn, g.shape.per_cu), g.shape.tpb)) != HB_OK) return rc;
        }
    }
    const int n = (int)B->ids.size();
    if (n > 0) {
        if (hipMalloc((void **)&B->d_ids, sizeof(int) * n) != hipSuccess ||
            hipMalloc((void **)&B->d_res, sizeof(double) * 4 * n) != hipSuccess ||
            hipMalloc((void **)&B->d_steps, sizeof(long) * n) != hipSuccess ||
            hipMalloc((void **)&B->d_flags, sizeof(int) * n) != hipSuccess) {
            (void)hipGetLastError();
            return HB_ENOMEM;
        }
        HIPOK(hipMemcpy(B->d_ids, B->ids.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    }
    B->lists_valid = true;
    return HB_OK;
}

static void launch_moments(const CacheGroup &cg, int pm, const CaseDev *cs, const CaseCtl *ctl, hipStream_t st)
{
    const DevList &L = cg.mom[pm];
    if (!L.grid) return;
    if (pm == 0)
        hipLaunchKernelGGL(hb::kb_moments<double>, dim3(L.grid), dim3(256), 0, st, cs, ctl, L.d_items, L.d_bstart);
    else
        hipLaunchKernelGGL(hb::kb_moments<float>, dim3(L.grid), dim3(256), 0, st, cs, ctl, L.d_items, L.d_bstart);
}

// One cache group's phases of a step, on one stream.
static void enqueue_group(const CacheGroup &cg, const CaseDev *cs, const CaseCtl *ctl, hipStream_t st)
{
    launch_moments(cg, 0, cs, ctl, st);
    launch_moments(cg, 1, cs, ctl, st);
    if (cg.faces.grid)
        hipLaunchKernelGGL(hb::kb_faces, dim3(cg.faces.grid), dim3(128), 0, st, cs, ctl, cg.faces.d_items,
                           cg.faces.d_bstart);
    if (cg.cells.grid)
        hipLaunchKernelGGL(hb::kb_cells, dim3(cg.cells.grid), dim3(128), 0, st, cs, ctl, cg.cells.d_items,
                           cg.cells.d_bstart);
    if (cg.dts.grid)
        hipLaunchKernelGGL(hb::kb_dt, dim3(cg.dts.grid), dim3(128), 0, st, cs, ctl, cg.dts.d_items,
                           cg.dts.d_bstart);
    if (cg.resid.grid)
        hipLaunchKernelGGL(hb::kb_resid, dim3(cg.resid.grid), dim3(256), 0, st, cs, ctl, cg.resid.d_items,
                           cg.resid.d_bstart);
    for (auto &g : cg.groups) launch_group(g, cs, ctl, st);
}

// The launches of one batch step: per cache group, the phases in the order
// of the single-case step; then the buffer swap of every stepped case.  The
// cache groups hold disjoint cases, so they run on HB_BATCH_LANES streams in
// turn: one group's latency-bound phases (faces, cells, local steps,
// residual) and ring update then overlap another's moments and interior
// update.
static void enqueue_step(hb_batch *B)
{
    hipStream_t st = B->stream;
    const CaseDev *cs = B->d_cs;
    const CaseCtl *ctl = B->d_ctl;
    const int lanes = (int)std::min<size_t>(HB_BATCH_LANES, B->cgs.size());
    if (lanes > 1) {
        (void)hipEventRecord(B->fork, st);
        for (int l = 1; l < lanes; l++) (void)hipStreamWaitEvent(B->side[l - 1], B->fork, 0);
    }
    for (size_t k = 0; k < B->cgs.size(); k++) {
        const int l = (int)(k % HB_BATCH_LANES);
        enqueue_group(B->cgs[k], cs, ctl, l == 0 ? st : B->side[l - 1]);
    }
    for (int l = 1; l < lanes; l++) {
        (void)hipEventRecord(B->join, B->side[l - 1]);
        (void)hipStreamWaitEvent(st, B->join, 0);
    }
    const int n = (int)B->ids.size();
    if (n) hipLaunchKernelGGL(hb::kb_step_end, dim3((n + 127) / 128), dim3(128), 0, st, B->d_ctl, B->d_ids, n);
}

static int capture(hb_batch *B)
{
    drop_graph(B);
    if (!B->use_graph || B->ids.empty()) return HB_OK;
    if (hipStreamBeginCapture(B->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        B->use_graph = false;
        return HB_OK;
    }
    enqueue_step(B);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(B->stream, &g) != hipSuccess || !g) {
        (void)hipGetLastError();
        B->use_graph = false;
        return HB_OK;
    }
    if (hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        B->exec = nullptr;
        B->use_graph = false;
        return HB_OK;
    }
    B->graph = g;
    return HB_OK;
}

static int ensure_lists(hb_batch *B)
{
    if (B->lists_valid) return HB_OK;
    int rc = build_lists(B);
    if (rc != HB_OK) return rc;
    return capture(B);
}

static int check_slot(const hb_batch *B, int id)
{
    if (!B || id < 0 || id >= B->max_cases || !B->cases[id]) return HB_EINVAL;
    return HB_OK;
}

extern "C" {

int hb_batch_create(const hb_create_opts *opts, size_t pool_bytes, int max_cases, hb_batch_handle *out)
{
    if (!out || max_cases <= 0) return HB_EINVAL;
    *out = nullptr;
    const int dev = opts ? opts->device : 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev < 0 || dev >= ndev) return HB_EDEVICE;
    if (hipSetDevice(dev) != hipSuccess) return HB_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return HB_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HB_EDEVICE;
    hb_batch *B = new (std::nothrow) hb_batch();
    if (!B) return HB_ENOMEM;
    B->device = dev;
    B->stream = opts ? (hipStream_t)opts->stream : nullptr;
    if (!B->stream) {  // graph capture needs a stream of our own (default priority)
        if (hipStreamCreate(&B->stream) != hipSuccess) {
            delete B;
            return HB_EDEVICE;
        }
        B->own_stream = true;
    }
    bool ok = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&B->join, hipEventDisableTiming) == hipSuccess;
    for (int l = 0; ok && l < HB_BATCH_LANES - 1; l++)
        ok = hipStreamCreateWithFlags(&B->side[l], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        if (B->fork) (void)hipEventDestroy(B->fork);
        if (B->join) (void)hipEventDestroy(B->join);
        for (auto &sd : B->side)
            if (sd) (void)hipStreamDestroy(sd);
        if (B->own_stream) (void)hipStreamDestroy(B->stream);
        delete B;
        return HB_EDEVICE;
    }
    B->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    B->max_cases = max_cases;
    B->cases.assign(max_cases, nullptr);
    B->active.assign(max_cases, 0);
    if (pool_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete B;
            return HB_EDEVICE;
        }
        pool_bytes = opts && opts->hbm_budget_bytes ? opts->hbm_budget_bytes : fr / 10 * 9;
    }
    int rc = B->pool.init(pool_bytes);
    if (rc == HB_OK && (hipMalloc((void **)&B->d_cs, sizeof(CaseDev) * max_cases) != hipSuccess ||
                        hipMalloc((void **)&B->d_ctl, sizeof(CaseCtl) * max_cases) != hipSuccess)) {
        (void)hipGetLastError();
        rc = HB_ENOMEM;
    }
    if (rc != HB_OK) {
        if (B->d_cs) (void)hipFree(B->d_cs);
        B->pool.destroy();
        (void)hipEventDestroy(B->fork);
        (void)hipEventDestroy(B->join);
        for (auto &sd : B->side) (void)hipStreamDestroy(sd);
        if (B->own_stream) (void)hipStreamDestroy(B->stream);
        delete B;
        return rc;
    }
    *out = B;
    return HB_OK;
}

void hb_batch_destroy(hb_batch_handle B)
{
    if (!B) return;
    (void)hipSetDevice(B->device);
    (void)hipStreamSynchronize(B->stream);
    drop_lists(B);
    for (auto *H : B->cases)
        if (H) hb_ugks_destroy(H);
    if (B->d_cs) (void)hipFree(B->d_cs);
    if (B->d_ctl) (void)hipFree(B->d_ctl);
    B->pool.destroy();
    for (auto &sd : B->side) {
        (void)hipStreamSynchronize(sd);
        (void)hipStreamDestroy(sd);
    }
    (void)hipEventDestroy(B->fork);
    (void)hipEventDestroy(B->join);
    if (B->own_stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

int hb_batch_case_bytes(hb_batch_handle B, int precision, const hb_geometry *geo, int n_harmonics,
                        const hb_vgrid *vg, size_t *bytes)
{
    if (!B || !geo || !vg || !bytes) return HB_EINVAL;
    hb_create_opts o{B->device, B->stream, precision, 0};
    hb_handle H = nullptr;
    int rc = hb_ugks_create(&o, &H);
    if (rc != HB_OK) return rc;
    H->count_only = true;
    hb_wall w[4];
    for (auto &x : w) x = hb_wall{0, 0, 0, 1, 0, 0};
    rc = hb_ugks_set_case(H, geo, 1.0, 1.0, n_harmonics, w, vg, nullptr);
    *bytes = H->bytes;
    hb_ugks_destroy(H);
    return rc;
}

int hb_batch_add(hb_batch_handle B, int precision, const hb_geometry *geo, double Kn, double St, int n_harmonics,
                 const hb_wall walls[4], const hb_vgrid *vg, const hb_numerics *num, int *case_id)
{
    if (!B || !case_id) return HB_EINVAL;
    int slot = -1;
    for (int s = 0; s < B->max_cases && slot < 0; s++)
        if (!B->cases[s]) slot = s;
    if (slot < 0) return HB_ECAPACITY;
    hb_create_opts o{B->device, B->stream, precision, 0};
    hb_handle H = nullptr;
    int rc = hb_ugks_create(&o, &H);
    if (rc != HB_OK) return rc;
    H->pool = &B->pool;
    rc = hb_ugks_set_case(H, geo, Kn, St, n_harmonics, walls, vg, num);
    if (rc != HB_OK) {
        hb_ugks_destroy(H);
        return rc;
    }
    H->batch_owned = true;
    CaseDev cd{};
    cd.P = H->P;
    for (int k = 0; k < 2; k++) {
        cd.h[k] = H->h[k];
        cd.b[k] = H->b[k];
        cd.W[k] = H->W[k];
        cd.dt[k] = H->dt[k];
    }
    cd.feed = H->feed;
    cd.recx = H->recx;
    cd.recy = H->recy;
    cd.crec = H->crec;
    cd.rpart = H->rpart;
    cd.ring = H->ring;
    cd.flag = H->flag;
    cd.cells_blocks = H->cells_blocks;
    cd.ring_len = HB_RING;
    CaseCtl cc{H->cur, 0, H->step};
    (void)hipSetDevice(B->device);
    if (hipMemcpy(B->d_cs + slot, &cd, sizeof(cd), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->d_ctl + slot, &cc, sizeof(cc), hipMemcpyHostToDevice) != hipSuccess) {
        hb_ugks_destroy(H);
        return HB_EDEVICE;
    }
    B->cases[slot] = H;
    B->active[slot] = 1;
    B->lists_valid = false;
    *case_id = slot;
    return HB_OK;
}

int hb_batch_remove(hb_batch_handle B, int case_id)
{
    int rc = check_slot(B, case_id);
    if (rc != HB_OK) return rc;
    (void)hipSetDevice(B->device);
    HIPOK(hipStreamSynchronize(B->stream));
    drop_lists(B);  // the graph refers to the case
    hb_ugks_destroy(B->cases[case_id]);
    B->cases[case_id] = nullptr;
    B->active[case_id] = 0;
    return HB_OK;
}

int hb_batch_set_active(hb_batch_handle B, int case_id, int on)
{
    int rc = check_slot(B, case_id);
    if (rc != HB_OK) return rc;
    if ((B->active[case_id] != 0) != (on != 0)) {
        B->active[case_id] = on ? 1 : 0;
        B->lists_valid = false;
    }
    return HB_OK;
}

int hb_batch_step(hb_batch_handle B, int nsteps)
{
    if (!B || nsteps < 0) return HB_EINVAL;
    if (hipSetDevice(B->device) != hipSuccess) return HB_EDEVICE;
    int rc = ensure_lists(B);
    if (rc != HB_OK) return rc;
    if (B->ids.empty()) return HB_OK;
    for (int s = 0; s < nsteps; s++) {
        if (B->exec) HIPOK(hipGraphLaunch(B->exec, B->stream));
        else enqueue_step(B);
    }
    HIPOK(hipGetLastError());
    B->steps += nsteps;
    return HB_OK;
}

int hb_batch_residuals(hb_batch_handle B, double *res, long *steps, int *diverged, int *ids, int capacity)
{
    if (!B) return HB_EINVAL;
    if (hipSetDevice(B->device) != hipSuccess) return HB_EDEVICE;
    int rc = ensure_lists(B);
    if (rc != HB_OK) return rc;
    const int n = (int)B->ids.size();
    if (capacity < n) return HB_ECAPACITY;
    if (n == 0) return 0;
    hipLaunchKernelGGL(hb::kb_gather, dim3((n + 127) / 128), dim3(128), 0, B->stream, B->d_cs, B->d_ctl, B->d_ids, n,
                       B->d_res, B->d_steps, B->d_flags);
    HIPOK(hipGetLastError());
    HIPOK(hipStreamSynchronize(B->stream));
    if (res) HIPOK(hipMemcpy(res, B->d_res, sizeof(double) * 4 * n, hipMemcpyDeviceToHost));
    if (steps) HIPOK(hipMemcpy(steps, B->d_steps, sizeof(long) * n, hipMemcpyDeviceToHost));
    if (diverged) HIPOK(hipMemcpy(diverged, B->d_flags, sizeof(int) * n, hipMemcpyDeviceToHost));
    if (ids) std::memcpy(ids, B->ids.data(), sizeof(int) * n);
    return n;
}

int hb_batch_case(hb_batch_handle B, int case_id, hb_handle *out)
{
    int rc = check_slot(B, case_id);
    if (rc != HB_OK || !out) return HB_EINVAL;
    if (hipSetDevice(B->device) != hipSuccess) return HB_EDEVICE;
    HIPOK(hipStreamSynchronize(B->stream));
    CaseCtl cc{};
    HIPOK(hipMemcpy(&cc, B->d_ctl + case_id, sizeof(cc), hipMemcpyDeviceToHost));
    hb_ugks *H = B->cases[case_id];
    H->cur = cc.cur;
    H->step = cc.kstep;
    *out = H;
    return HB_OK;
}

int hb_batch_pool_info(hb_batch_handle B, size_t *capacity, size_t *in_use, size_t *largest_free)
{
    if (!B) return HB_EINVAL;
    if (capacity) *capacity = B->pool.size;
    if (in_use) *in_use = B->pool.in_use;
    if (largest_free) *largest_free = B->pool.largest_free();
    return HB_OK;
}

// Time each candidate launch shape of the update phase of every (precision,
// N_T) group and of the moments phase on the batch's own data, keep the
// fastest.  The timed kernels only read the current state and rewrite the
// next buffers (or the feeds), so repeating them changes nothing; one batch
// step is taken first so that every record they read is set.
int hb_batch_tune(hb_batch_handle B, int reps)
{
    if (!B || reps <= 0) return HB_EINVAL;
    if (hipSetDevice(B->device) != hipSuccess) return HB_EDEVICE;
    int rc = ensure_lists(B);
    if (rc != HB_OK) return rc;
    if (B->ids.empty()) return HB_OK;
    if ((rc = hb_batch_step(B, 1)) != HB_OK) return rc;
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    HIPOK(hipEventCreate(&e1));
    auto timeit = [&](auto &&launch) -> double {
        launch();  // warm-up
        (void)hipEventRecord(e0, B->stream);
        for (int r = 0; r < reps; r++) launch();
        (void)hipEventRecord(e1, B->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    const Shape upd_cands[] = {{256, 0}, {128, 0}, {64, 0}, {256, 2}, {256, 4}, {128, 4}, {128, 8}};
    std::map<std::tuple<int, int, int>, Shape> done;
    for (auto &cg : B->cgs)
        for (auto &g : cg.groups) {
            const auto key = std::make_tuple(g.prec, g.NT, g.max_nvp);
            if (done.count(key)) continue;
            double best = 1e300;
            Shape bs = g.shape;
            for (const Shape &c : upd_cands) {
                if ((rc = g.in.upload(grid_of(B, g.in, c.per_cu), c.tpb)) != HB_OK) break;
                if ((rc = g.bn.upload(grid_of(B, g.bn, c.per_cu), c.tpb)) != HB_OK) break;
                const double t = timeit([&] { launch_group(g, B->d_cs, B->d_ctl, B->stream); });
                if (t < best) {
                    best = t;
                    bs = c;
                }
            }
            if (rc != HB_OK) break;
            done[key] = bs;
            g_tuned[key] = bs;
        }
    const Shape mom_cands[] = {{256, 0}, {256, 2}, {256, 4}, {256, 8}};
    for (auto &cg : B->cgs)
        for (int pm = 0; pm < 2 && rc == HB_OK; pm++) {
            DevList &L = cg.mom[pm];
            const auto key = std::make_tuple(pm ? HB_MIXED : HB_FP64, 0, cg.mom_nvp[pm]);
            if (L.items.empty() || done.count(key)) continue;
            double best = 1e300;
            Shape bs = cg.mom_shape[pm];
            for (const Shape &c : mom_cands) {
                if ((rc = L.upload(grid_of(B, L, c.per_cu), 256)) != HB_OK) break;
                const double t = timeit([&] { launch_moments(cg, pm, B->d_cs, B->d_ctl, B->stream); });
                if (t < best) {
                    best = t;
                    bs = c;
                }
            }
            done[key] = bs;
            g_tuned[key] = bs;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != HB_OK) return rc;
    HIPOK(hipGetLastError());
    B->lists_valid = false;  // rebuild with the tuned shapes and capture again
    return ensure_lists(B);
}

int hb_batch_shapes(hb_batch_handle B, int *out, int capacity)
{
    // per distinct update group: precision, NT, padded velocities, threads per block, blocks per CU
    if (!B || !out) return HB_EINVAL;
    int rc = ensure_lists(B);
    if (rc != HB_OK) return rc;
    std::map<std::tuple<int, int, int>, Shape> seen;
    for (auto &cg : B->cgs)
        for (auto &g : cg.groups) seen[std::make_tuple(g.prec, g.NT, g.max_nvp)] = g.shape;
    const int n = (int)seen.size();
    if (capacity < 5 * n) return HB_ECAPACITY;
    int k = 0;
    for (auto &kv : seen) {
        out[5 * k + 0] = std::get<0>(kv.first);
        out[5 * k + 1] = std::get<1>(kv.first);
        out[5 * k + 2] = std::get<2>(kv.first);
        out[5 * k + 3] = kv.second.tpb;
        out[5 * k + 4] = kv.second.per_cu;
        k++;
    }
    return n;
}

int hb_batch_set_cache_bytes(hb_batch_handle B, size_t bytes)
{
    if (!B) return HB_EINVAL;
    B->cache_bytes = bytes;
    B->lists_valid = false;
    return HB_OK;
}

int hb_batch_use_graph(hb_batch_handle B, int on)
{
    if (!B) return HB_EINVAL;
    B->use_graph = on != 0;
    B->lists_valid = false;
    return HB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ serving
// Requests arrive at given times (seconds from the start of the run).  The
// loop admits every arrived request whose device footprint fits the pool now
// (FIFO, later requests may pass one that does not fit yet), advances the
// batch check_every steps at a time, and retires each case whose density
// residual (Eq. 43) is at or below tol: its harmonics go to the request's
// buffers and its memory returns to the pool at once.  Admission and checks
// happen only between chunks of check_every steps, so a request's step count
// and result do not depend on what else is in the mix.
namespace {
double wall_now()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

extern "C" int hb_serve_run(hb_batch_handle B, const hb_request *req, int n, double tol, int check_every,
                            long max_steps, double max_wall_s, hb_result *out, double *wall_s)
{
    if (!B || (n > 0 && (!req || !out)) || n < 0 || check_every <= 0 || max_steps <= 0 || !(tol > 0.0))
        return HB_EINVAL;
    for (int k = 0; k < B->max_cases; k++)
        if (B->cases[k]) return HB_ESTATE;  // the run owns the batch
    for (int k = 0; k < n; k++) {
        out[k] = hb_result{};
        out[k].status = HB_ESTATE;
        out[k].t_admit = out[k].t_done = -1.0;
    }
    std::vector<int> slot_req(B->max_cases, -1);
    std::vector<size_t> need(n, 0);
    for (int k = 0; k < n; k++) {
        int rc = hb_batch_case_bytes(B, req[k].precision, &req[k].geo, req[k].n_harmonics, &req[k].vg, &need[k]);
        if (rc != HB_OK) return rc;
    }
    const char *pv = std::getenv("HB_SERVE_PROGRESS");
    const bool progress = pv && *pv && std::strcmp(pv, "0") != 0;
    const double t0 = wall_now();
    int done = 0, next = 0, active = 0;
    std::vector<char> pending(n, 0);
    std::vector<double> res(4 * (size_t)B->max_cases);
    std::vector<long> steps(B->max_cases);
    std::vector<int> div(B->max_cases), ids(B->max_cases);
    while (done < n) {
        const double now = wall_now() - t0;
        while (next < n && req[next].arrival_s <= now) pending[next++] = 1;
        // admission in arrival order; a request that can never fit is refused
        for (int k = 0; k < next; k++) {
            if (!pending[k]) continue;
            if (need[k] > B->pool.size) {
                pending[k] = 0;
                out[k].status = HB_ENOMEM;
                out[k].t_done = now;
                done++;
                continue;
            }
            if (need[k] > B->pool.largest_free()) continue;
            int cid = -1;
            const hb_request &r = req[k];
            int rc = hb_batch_add(B, r.precision, &r.geo, r.Kn, r.St, r.n_harmonics, r.walls, &r.vg,
                                  r.has_numerics ? &r.num : nullptr, &cid);
            if (rc == HB_ENOMEM || rc == HB_ECAPACITY) continue;  // not now
            if (rc != HB_OK) return rc;
            pending[k] = 0;
            slot_req[cid] = k;
            out[k].t_admit = wall_now() - t0;
            out[k].bytes = need[k];
            active++;
        }
        if (active == 0) {
            if (next < n) {  // idle until the next arrival
                const double wait = req[next].arrival_s - (wall_now() - t0);
                if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            }
            continue;
        }
        int rc = hb_batch_step(B, check_every);
        if (rc != HB_OK) return rc;
        const int na = hb_batch_residuals(B, res.data(), steps.data(), div.data(), ids.data(), B->max_cases);
        if (na < 0) return na;
        // past the wall-clock cap every resident case retires as it stands and
        // the requests not yet admitted are left unserved (HB_ESTATE, t_admit -1)
        const bool capped = max_wall_s > 0.0 && wall_now() - t0 >= max_wall_s;
        for (int a = 0; a < na; a++) {
            const int cid = ids[a], k = slot_req[cid];
            if (k < 0) continue;
            const bool conv = res[4 * a] <= tol, bad = div[a] != 0, late = steps[a] >= max_steps || capped;
            if (!conv && !bad && !late) continue;
            hb_result &o = out[k];
            o.steps = steps[a];
            for (int q = 0; q < 4; q++) o.residual[q] = res[4 * a + q];
            o.status = bad ? HB_EDIVERGED : (conv ? HB_OK : HB_ESTATE);
            if (conv && !bad && req[k].re && req[k].im) {
                hb_handle H = nullptr;
                if ((rc = hb_batch_case(B, cid, &H)) != HB_OK) return rc;
                rc = hb_ugks_harmonics_out(H, req[k].var_mask, req[k].re, req[k].im, req[k].capacity);
                if (rc != HB_OK) o.status = rc;
            }
            if ((rc = hb_batch_remove(B, cid)) != HB_OK) return rc;
            slot_req[cid] = -1;
            o.t_done = wall_now() - t0;
            active--;
            done++;
        }
        if (progress) {
            std::fprintf(stderr, "serve: %.1f s, %d resident, %d of %d requests finished\n", wall_now() - t0, active,
                         done, n);
            std::fflush(stderr);
        }
        if (capped) {
            for (int k = 0; k < n; k++)
                if (out[k].t_admit < 0.0 && out[k].t_done < 0.0) done++;  // never admitted
            break;
        }
    }
    if (wall_s) *wall_s = wall_now() - t0;
    return HB_OK;
}
