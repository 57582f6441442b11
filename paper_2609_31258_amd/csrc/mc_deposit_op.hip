// mc_deposit_op.hip -- the cloud-in-cell charge deposit as a stand-alone
// operation on caller-owned device arrays ("Axisymmetric PIC space charge
// update": bilinear split of each pack's int64 charge onto the four nodes of
// its (r, z) cell, exact per pack).  Two entry points share the deposit
// kernels of the simulation context (k_deposit, k_deposit_sum):
//
//   mc_deposit_cic          scratch (copies of the grid for the blocks'
//                           flushes, two node-range slots) allocated per
//                           call with hipMalloc; synchronous.
//   mc_deposit_cic_noalloc  the same scratch in a file-scope device array,
//                           so the call allocates nothing; asynchronous.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>
#include <vector>

#include "mc_kernels.hpp"

using namespace mc;

namespace {

// Scratch of the allocation-free variant: the grid copies, then four int32
// range slots (lowest and highest node written; a dummy pair for the sum
// kernel's reset).  8 MiB of copies: 16 copies up to 65 536 nodes, fewer on
// larger grids, one copy at the largest grid the variant takes (1 048 576
// nodes, e.g. 256 x 4096).
constexpr int64_t kNoAllocCopyWords = (8ll << 20) / 8;
constexpr int64_t kNoAllocRangeWords = 2;  // four int32 slots
constexpr int64_t kNoAllocMaxNodes = kNoAllocCopyWords;

}  // namespace

// Every GPU that runs the variant holds its own copy of this array until the
// process ends.  Host code never uses the name as an address: it takes the
// device address from hipGetSymbolAddress (per device, below).
static __device__ __align__(256) unsigned long long scratch[kNoAllocCopyWords + kNoAllocRangeWords];

namespace {

// Range slots reset for one deposit: (INT32_MAX, -1) twice.
__global__ __launch_bounds__(64) void k_range_reset(int32_t *r) {
    if (threadIdx.x < 4) r[threadIdx.x] = (threadIdx.x & 1) ? -1 : INT32_MAX;
}

// The scratch copies start at zero: filled once per device by a kernel (the
// call may be recorded into a graph, where memset nodes are avoided).
__global__ __launch_bounds__(256) void k_fill_zero(unsigned long long *p, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0ull;
}

struct DeviceScratch {
    unsigned long long *ptr = nullptr;  // device address of `scratch` on this device
    bool cleared = false;               // the copies have been zeroed on this device
};

std::mutex g_scratch_mu;
std::vector<DeviceScratch> g_scratch;  // indexed by device ordinal

// The per-device address of `scratch`, looked up once with the device
// current; nullptr on failure.
unsigned long long *scratch_address(int dev, bool *first) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize((size_t)dev + 1);
    DeviceScratch &s = g_scratch[(size_t)dev];
    if (!s.ptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        s.ptr = static_cast<unsigned long long *>(p);
    }
    *first = !s.cleared;
    s.cleared = true;
    return s.ptr;
}

int32_t check_args(const mc_cic_packs *packs, const mc_grid *grid, const int64_t *q_out) {
    if (!packs || !grid || !q_out) return MC_EINVAL;
    if (grid->nr < 3 || grid->nz < 3 || !(grid->dr > 0.0) || !(grid->dz > 0.0)) return MC_EINVAL;
    if (packs->n < 0) return MC_EINVAL;
    if (packs->n > 0 && (!packs->x || !packs->y || !packs->z || !packs->q || !packs->status)) return MC_EINVAL;
    return MC_OK;
}

// The deposit kernels on caller arrays: copies and range slots given.
int32_t launch_deposit(const mc_cic_packs *packs, const mc_grid *grid, int64_t *q_out, unsigned long long *copies,
                       int32_t ncopies, int32_t *range, hipStream_t stream) {
    const int64_t nn = (int64_t)grid->nr * grid->nz;
    k_range_reset<<<1, 64, 0, stream>>>(range);
    if (packs->n > 0) {
        DepositArgs<double> a{};
        a.p.x = const_cast<double *>(packs->x);
        a.p.y = const_cast<double *>(packs->y);
        a.p.z = const_cast<double *>(packs->z);
        a.p.q = const_cast<int64_t *>(packs->q);
        a.p.status = const_cast<int32_t *>(packs->status);
        a.q = reinterpret_cast<unsigned long long *>(q_out);
        a.qrep = copies;
        a.range = range;
        a.n_slots = packs->n;
        a.nn = nn;
        a.inv_dr = 1.0 / grid->dr;
        a.inv_dz = 1.0 / grid->dz;
        a.nr = grid->nr;
        a.nz = grid->nz;
        a.nrep = ncopies;
        unsigned nb;
        deposit_shape(packs->n, &nb, &a.chunk);
        k_deposit<P64><<<nb, kDepositThreads, 0, stream>>>(a);
    }
    // every node of the output written: the sums over the range, zero elsewhere
    k_deposit_sum<<<(unsigned)std::min<int64_t>((nn + 255) / 256, kDepositSumBlocks), 256, 0, stream>>>(
        reinterpret_cast<unsigned long long *>(q_out), copies, ncopies, nn, range, nullptr, range + 2);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_EDEVICE;
}

}  // namespace

extern "C" {

int32_t mc_deposit_cic(const mc_cic_packs *packs, const mc_grid *grid, int64_t *q_out, void *stream) {
    int32_t rc = check_args(packs, grid, q_out);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nn = (int64_t)grid->nr * grid->nz;
    const int32_t ncopies = deposit_copies(nn);
    const size_t copy_bytes = (size_t)ncopies * (size_t)nn * 8;
    void *buf = nullptr;
    if (hipMalloc(&buf, copy_bytes + 256) != hipSuccess) return MC_ENOMEM;
    unsigned long long *copies = static_cast<unsigned long long *>(buf);
    int32_t *range = reinterpret_cast<int32_t *>(static_cast<char *>(buf) + copy_bytes);
    rc = hipMemsetAsync(copies, 0, copy_bytes, s) == hipSuccess ? MC_OK : MC_EDEVICE;
    if (!rc) rc = launch_deposit(packs, grid, q_out, copies, ncopies, range, s);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = MC_EDEVICE;
    (void)hipFree(buf);
    return rc;
}

int32_t mc_deposit_cic_noalloc(const mc_cic_packs *packs, const mc_grid *grid, int64_t *q_out, void *stream) {
    int32_t rc = check_args(packs, grid, q_out);
    if (rc) return rc;
    const int64_t nn = (int64_t)grid->nr * grid->nz;
    if (nn > kNoAllocMaxNodes) return MC_EINVAL;  // beyond the scratch array
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MC_EDEVICE;
    bool first = false;
    unsigned long long *base = scratch_address(dev, &first);
    if (!base) return MC_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (first) {
        k_fill_zero<<<256, 256, 0, s>>>(base, kNoAllocCopyWords);
        if (hipGetLastError() != hipSuccess) return MC_EDEVICE;
    }
    const int32_t ncopies = (int32_t)std::min<int64_t>(kDepositMaxCopies, kNoAllocCopyWords / nn);
    int32_t *range = reinterpret_cast<int32_t *>(base + kNoAllocCopyWords);
    return launch_deposit(packs, grid, q_out, base, ncopies, range, s);
}

}  // extern "C"
