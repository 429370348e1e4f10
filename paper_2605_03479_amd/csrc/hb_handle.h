// Private host-side definitions shared by the single-case runtime
// (hb_runtime.hip) and the batched form (hb_batch.hip): the case handle and
// the device memory pool the batched form carves cases from.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

#include "hb_kernels.h"
#include "hb_ugks.h"

constexpr int HB_RING = 1024;  // residual ring entries per case
constexpr int HB_NKERN = 6;    // kernels of one pseudo step, in launch order
constexpr size_t HB_NOALLOC_DOUBLES = (size_t)4 << 20;  // scratch of hb_ugks_harmonics_out_noalloc (32 MiB)
constexpr int HB_MAX_DEVICES = 64;

struct HbBuf {
    void *p = nullptr;
    size_t n = 0;
};

// One device arena with first-fit allocation and coalescing frees.  Blocks
// are 256-byte aligned.  Not thread-safe (a batch is not).
struct HbPool {
    static constexpr size_t ALIGN = 256;
    char *base = nullptr;
    size_t size = 0, in_use = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> used_;  // offset -> length

    static size_t round(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

    int init(size_t bytes)
    {
        bytes = round(bytes);
        if (hipMalloc((void **)&base, bytes) != hipSuccess) {
            (void)hipGetLastError();
            base = nullptr;
            return HB_ENOMEM;
        }
        size = bytes;
        free_.clear();
        used_.clear();
        free_[0] = bytes;
        in_use = 0;
        return HB_OK;
    }
    void destroy()
    {
        if (base) (void)hipFree(base);
        base = nullptr;
        size = in_use = 0;
        free_.clear();
        used_.clear();
    }
    void *take(size_t n)
    {
        n = round(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used_[off] = n;
            in_use += n;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p)
    {
        if (!p) return;
        const size_t off = (size_t)((char *)p - base);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        in_use -= len;
        used_.erase(u);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {  // merge with the following free block
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {  // merge with the preceding free block
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    size_t largest_free() const
    {
        size_t m = 0;
        for (auto &f : free_) m = f.second > m ? f.second : m;
        return m;
    }
};

struct hb_ugks {
    int device = 0;
    hipStream_t stream = nullptr;
    // the boundary-ring update runs beside the interior update on this stream
    // (created on first use, default priority), forked from and joined to
    // `stream` by the two events
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    int precision = HB_FP64;
    size_t budget = 0;
    size_t bytes = 0;
    bool has_case = false;
    HbPool *pool = nullptr;    // device memory comes from here when set (batched form)
    bool count_only = false;   // set_case only sums the device bytes it would allocate
    bool batch_owned = false;  // stepped by a batch: hb_ugks_pseudo_step refuses it
    hb::Params P{};
    // device buffers
    std::vector<HbBuf> bufs;
    double *geo = nullptr;  // xf, yf, xc, yc, rdx, rdy, rcx, rcy, u1, w1
    double *vel = nullptr;  // vu, vv, vw
    int *veli = nullptr;    // viu, viv
    void *h[2]{}, *b[2]{};  // double (FP64) or float deviations from the rest Maxwellian (mixed)
    double *W[2]{}, *dt[2]{};
    double *vref = nullptr;
    std::vector<double> vref_host;
    double *feed = nullptr, *recx = nullptr, *recy = nullptr, *crec = nullptr, *rpart = nullptr, *ring = nullptr;
    int *flag = nullptr;
    double *lscale = nullptr;  // level-mass projection factors of the last step
    // mixed form: FP32 face and collision records, E(u_k) = exp(-u_k^2) in FP64 and FP32
    float *rx32 = nullptr, *ry32 = nullptr, *cr32 = nullptr, *er32 = nullptr, *vel32 = nullptr;
    double *ex64 = nullptr;
    // harmonics scratch: per-(var, level, cell) values, then [var][k][cell] re and im
    double *hvars = nullptr, *hre = nullptr, *him = nullptr;
    // time-domain form (one level, global step): wall inputs, physical time,
    // W at the start of the current period and the period residual
    hb_wall walls[4]{};
    double t_phys = 0.0;
    double *Wp = nullptr, *tdres = nullptr;
    int cur = 0;
    long step = 0;
    int cells_blocks = 0;
    size_t upd_lds = 0;
    int n_int = 0, n_bnd = 0;  // interior cells (>= 2 from every wall) and the boundary ring
    int *bnd_cells = nullptr;
    std::vector<int> bnd_host;  // the boundary-ring cells (host copy, for batched work lists)
    std::vector<int> perm;      // natural alpha -> internal alpha'
    std::vector<double> xf_host, yf_host;  // face coordinates (wall averages)
    // timing: one set of HB_NKERN + 1 events per timed step, read back lazily
    bool timing = false;
    std::vector<hipEvent_t> tev;
    size_t tused = 0;
    double kms[HB_NKERN]{};
    long klaunch[HB_NKERN]{};
};

#define HIPOK(x)                                  \
    do {                                          \
        if ((x) != hipSuccess) return HB_EDEVICE; \
    } while (0)
