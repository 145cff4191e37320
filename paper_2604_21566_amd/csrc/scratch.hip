// scratch.hip -- the fixed per-GPU device array behind bn_addsub_n_batch_noalloc.
//
// A chained add/sub scan (Sec. 3.1: the carry out of one chunk is the carry into the
// next, here resolved by decoupled look-back between workgroup tiles) keeps one status
// word per tile plus a small control block.  The context's workspace holds them for the
// ordinary entry points; for callers that cannot allocate at all, this file holds them
// in one file-scope device array instead.  Every GPU the library runs on gets its own
// copy of the array at its own address, taken once per device by scratch_setup() (from
// bn_create, with that device current) and kept until the process ends.  Host code uses
// only that address, never the array's name (which on the host is a stand-in, not a
// device address).
//
// Layout (bytes): [0, 512) the look-back control block (ScanCtl; epoch starts at 1),
// [512, 512 + 8 * BN_SCRATCH_MAX_TILES) the status words, then BN_SCRATCH_MAX_TILES
// bytes of fill codes (launches that defer their all-propagate tiles).  Every call on a device shares
// them: each chained launch tags its status words with an epoch of its own (a per-device
// host counter counting up from 2^61 for eager launches, the control block's counter
// for launches recorded into a graph), so nothing has to be cleared between calls; two
// calls that overlap in time on one GPU race on the array.
#include <atomic>
#include <mutex>

#include "bn_internal.h"

namespace {

constexpr size_t SCRATCH_CTL_BYTES = 512;
static_assert(sizeof(ScanCtl) <= SCRATCH_CTL_BYTES, "control block must fit its slot");
constexpr size_t SCRATCH_WORDS = (SCRATCH_CTL_BYTES + 9 * (size_t)BN_SCRATCH_MAX_TILES) / 8;

static __device__ __align__(256) u64 scratch[SCRATCH_WORDS];

// Host view of one device's copy of the array.
struct DevScratch {
    u64 *ptr = nullptr;                  // device address from hipGetSymbolAddress
    std::atomic<u64> host_epoch{1ull << 61};
    std::atomic<bool> ready{false};
};
constexpr int MAX_DEVICES = 64;
DevScratch g_dev[MAX_DEVICES];
std::mutex g_mu;

// Clear the array and start the control block's epoch at 1 (status words of 0 then
// match no epoch in use).
__global__ void k_scratch_init(u64 *p, u64 words) {
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < words; i += (u64)gridDim.x * blockDim.x)
        p[i] = (i == 0) ? 1ull : 0ull;  // word 0 is ScanCtl::epoch
}

}  // namespace

bn_status scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return BN_OK;  // the no-allocation entry point reports it
    std::lock_guard<std::mutex> lk(g_mu);
    DevScratch &d = g_dev[device];
    if (d.ready.load(std::memory_order_acquire)) return BN_OK;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return BN_EHIP;  // caller makes it current
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BN_EHIP;
    u64 *ptr = static_cast<u64 *>(p);
    hipLaunchKernelGGL(k_scratch_init, dim3(64), dim3(256), 0, nullptr, ptr, (u64)SCRATCH_WORDS);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return BN_EHIP;
    d.ptr = ptr;
    d.ready.store(true, std::memory_order_release);
    return BN_OK;
}

bool scratch_mem(int device, ScanMem *m) {
    if (device < 0 || device >= MAX_DEVICES) return false;
    DevScratch &d = g_dev[device];
    if (!d.ready.load(std::memory_order_acquire)) return false;
    m->ctl = reinterpret_cast<ScanCtl *>(d.ptr);
    m->status = d.ptr + SCRATCH_CTL_BYTES / 8;
    m->max_tiles = BN_SCRATCH_MAX_TILES;
    m->host_epoch = &d.host_epoch;
    m->dbg_mask = 1u;  // the self-help test hook applies; distances are not recorded here
    return true;
}
