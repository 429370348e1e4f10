// Batched form of the pseudo step: the same per-cell / per-face bodies as the
// single-case kernels, driven by work lists that span many cases.
//
// Every phase is one persistent launch: block k (in the XCD-contiguous order
// of xcd_cell) owns the contiguous item range [bstart[k], bstart[k+1]) of its
// work list, so the cells one XCD works on are neighbours and share its L2.
// Item ranges are cut on the host so that every block gets about the same
// cost.  A work item names a case and a unit of that case (a cell, or a block
// of threads for the per-thread phases); every case keeps exactly the
// single-case decomposition, so its arithmetic, and its residual summation
// order, are those of the single-case path: a case gives the same bits alone
// and in a batch.
#pragma once
#include "hb_kernels.h"

namespace hb {

// Static per-case data (set when the case joins the batch).
struct CaseDev {
    Params P;
    void *h[2], *b[2];
    double *W[2], *dt[2];
    double *feed, *recx, *recy, *crec, *rpart, *ring;
    int *flag;
    int cells_blocks, ring_len;
};

// Per-case step state, advanced on the device at the end of every batch step.
struct CaseCtl {
    int cur, pad;
    long kstep;
};

struct WorkItem {
    int cs, unit;
};

__device__ inline void item_range(const int *__restrict__ bstart, int &a, int &e)
{
    const int k = xcd_cell(blockIdx.x, gridDim.x);
    a = bstart[k];
    e = bstart[k + 1];
}

template <typename TS>
__global__ __launch_bounds__(256, sizeof(TS) == 4 ? HB_MOM_WAVES_MIXED : HB_MOM_WAVES) void kb_moments(const CaseDev *__restrict__ cs, const CaseCtl *__restrict__ ctl,
                                                  const WorkItem *__restrict__ items, const int *__restrict__ bstart)
{
    int a, e;
    item_range(bstart, a, e);
    for (int it = a; it < e; it++) {
        const WorkItem w = items[it];
        const CaseDev &C = cs[w.cs];
        const int cur = ctl[w.cs].cur;
        moments_cell<TS>(C.P, (const TS *)C.h[cur], (const TS *)C.b[cur], C.feed, w.unit);
        __syncthreads();
    }
}

__global__ __launch_bounds__(128) void kb_faces(const CaseDev *__restrict__ cs, const CaseCtl *__restrict__ ctl,
                                                const WorkItem *__restrict__ items, const int *__restrict__ bstart)
{
    int a, e;
    item_range(bstart, a, e);
    for (int it = a; it < e; it++) {
        const WorkItem w = items[it];
        const CaseDev &C = cs[w.cs];
        const int cur = ctl[w.cs].cur;
        faces_thread(C.P, C.feed, C.W[cur], C.dt[cur], C.recx, C.recy, w.unit * 128 + threadIdx.x);
    }
}

__global__ __launch_bounds__(128) void kb_cells(const CaseDev *__restrict__ cs, const CaseCtl *__restrict__ ctl,
                                                const WorkItem *__restrict__ items, const int *__restrict__ bstart)
{
    int a, e;
    item_range(bstart, a, e);
    for (int it = a; it < e; it++) {
        const WorkItem w = items[it];
        const CaseDev &C = cs[w.cs];
        const int cur = ctl[w.cs].cur;
        cells_block(C.P, C.feed, C.recx, C.recy, C.W[cur], C.dt[cur], C.W[1 - cur], C.crec, C.rpart, w.unit);
        __syncthreads();
    }
}

__global__ __launch_bounds__(128) void kb_dt(const CaseDev *__restrict__ cs, const CaseCtl *__restrict__ ctl,
                                             const WorkItem *__restrict__ items, const int *__restrict__ bstart)
{
    int a, e;
    item_range(bstart, a, e);
    for (int it = a; it < e; it++) {
        const WorkItem w = items[it];
        const CaseDev &C = cs[w.cs];
        const int nxt = 1 - ctl[w.cs].cur;
        dt_thread(C.P, C.W[nxt], C.dt[nxt], w.unit * 128 + threadIdx.x);
    }
}

__global__ __launch_bounds__(256) void kb_resid(const CaseDev *__restrict__ cs, const CaseCtl *__restrict__ ctl,
                                                const WorkItem *__restrict__ items, const int *__restrict__ bstart)
{
    int a, e;
    item_range(bstart, a, e);
    for (int it = a; it < e; it++) {
        const WorkItem w = items[it];
        const CaseDev &C = cs[w.cs];
        const int slot = (int)(ctl[w.cs].kstep % C.ring_len);
        resid_block(C.P, C.rpart, C.cells_blocks, C.ring, slot, C.flag);
        __syncthreads();
    }
}

// SO: every case of the work list stores its update non-temporally (the group
// is formed per store policy)
template <int NT, typename TS, bool SO = false>
__global__ __launch_bounds__(256, sizeof(TS) == 4 ? HB_UPD_WAVES_MIXED : HB_UPD_WAVES) void kb_update_int(const CaseDev *__restrict__ cs,
                                                                    const CaseCtl *__restrict__ ctl,
                                                                    const WorkItem *__restrict__ items,
                                                                    const int *__restrict__ bstart)
{
    int a, e;
    item_range(bstart, a, e);
    for (int it = a; it < e; it++) {
        const WorkItem w = items[it];
        const CaseDev &C = cs[w.cs];
        const int cur = ctl[w.cs].cur;
        update_int_cell<NT, TS, SO ? OUT_NT : 0>(C.P, (const TS *)C.h[cur], (const TS *)C.b[cur], C.recx, C.recy, C.crec, C.dt[cur],
                                (TS *)C.h[1 - cur], (TS *)C.b[1 - cur], C.W[1 - cur], w.unit);
        __syncthreads();
    }
}

template <int NT, typename TS, bool SO = false>
__global__ __launch_bounds__(256, 2) void kb_update_bnd(const CaseDev *__restrict__ cs, const CaseCtl *__restrict__ ctl,
                                                        const WorkItem *__restrict__ items,
                                                        const int *__restrict__ bstart)
{
    int a, e;
    item_range(bstart, a, e);
    for (int it = a; it < e; it++) {
        const WorkItem w = items[it];
        const CaseDev &C = cs[w.cs];
        const int cur = ctl[w.cs].cur;
        update_bnd_cell<NT, TS, SO ? OUT_NT : 0>(C.P, (const TS *)C.h[cur], (const TS *)C.b[cur], C.recx, C.recy, C.crec, C.dt[cur],
                                (TS *)C.h[1 - cur], (TS *)C.b[1 - cur], C.W[1 - cur], w.unit);
        __syncthreads();
    }
}

// end of a batch step: swap the buffers and count the step of every stepped case
__global__ void kb_step_end(CaseCtl *__restrict__ ctl, const int *__restrict__ ids, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        CaseCtl &c = ctl[ids[t]];
        c.cur = 1 - c.cur;
        c.kstep = c.kstep + 1;
    }
}

// latest residual (Eq. 43), step count and divergence flag of the listed cases
__global__ void kb_gather(const CaseDev *__restrict__ cs, const CaseCtl *__restrict__ ctl,
                          const int *__restrict__ ids, int n, double *__restrict__ res, long *__restrict__ steps,
                          int *__restrict__ flags)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int c = ids[t];
        const long ks = ctl[c].kstep;
        const int slot = ks > 0 ? (int)((ks - 1) % cs[c].ring_len) : 0;
        for (int k = 0; k < 4; k++) res[t * 4 + k] = ks > 0 ? cs[c].ring[slot * 4 + k] : 0.0;
        steps[t] = ks;
        flags[t] = *cs[c].flag;
    }
}

}  // namespace hb
