// Batched 2D step of many domains (continuous batching): launchers of the
// persistent batch kernels.
#include "step_kernels.hpp"

#include <mutex>

// Batch table of fw2_batch_create_noalloc: file-scope device memory, one copy
// per GPU, held until the process ends.  In host code its name is only a
// stand-in: the device address of each GPU's copy comes from
// hipGetSymbolAddress with that GPU current (static_batch_table below).
static __device__ __align__(256) unsigned char scratch[sizeof(fw2::BatchTable)];

namespace fw2 {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];       // device address of `scratch`, per device
bool g_static_busy[kMaxDevices];       // a no-allocation batch holds the table

}  // namespace

hipError_t claim_static_batch_table(int device, BatchTable **table, bool *busy)
{
    std::lock_guard<std::mutex> lock(g_static_mu);
    *table = nullptr;
    *busy = false;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_static_ptr[device]) {                  // once per device, with it current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_static_ptr[device] = p;
    }
    if (g_static_busy[device]) {
        *busy = true;
        return hipSuccess;
    }
    g_static_busy[device] = true;
    *table = (BatchTable *)g_static_ptr[device];
    return hipSuccess;
}

void release_static_batch_table(int device)
{
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (device >= 0 && device < kMaxDevices) g_static_busy[device] = false;
}

namespace {

// One block per entry: its sources of the current step, then (after the
// block barrier, so the receivers see them) its receivers, then its step
// counter advanced.
__global__ void __launch_bounds__(256) batch_sparse(const BatchTable *__restrict__ T)
{
    const int d = blockIdx.x;
    if (d >= T->n) return;
    const BatchEntry &e = T->e[d];
    const long long step = *e.rcv.step;             // the entry's one counter (sources share it)
    if (step < e.n_steps && step < e.src.n_t)
        for (int q = threadIdx.x; q < e.src.n; q += blockDim.x) {
            const int64_t pi = padded_index(e.src.geo, e.src.idx[q]);
            e.src.p[pi] = e.src.p[pi] + e.src.w[q] * e.src.signals[(int64_t)e.src.sig[q] * e.src.n_t + step];
        }
    __syncthreads();
    if (step < e.n_steps && step < e.rcv.cap)
        for (int r = threadIdx.x; r < e.rcv.n; r += blockDim.x)
            e.rcv.trace[step * e.rcv.n + r] = e.rcv.p[padded_index(e.rcv.geo, e.rcv.idx[r])];
    __syncthreads();
    if (threadIdx.x == 0) e.rcv.step[0] = step + 1;
}

}  // namespace

// Persistent grid of a batch kernel: as many blocks as fit on the device at
// once (occupancy query), rounded down to a multiple of 8 XCDs, so that no
// block waits for a free slot while others hold tiles.
template <bool PRESSURE, int BX, int CLASS>
int batch_grid()
{
    static const int grid = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_phase<PRESSURE, BX, CLASS>, BX, 0) !=
                hipSuccess ||
            cus <= 0 || per_cu <= 0)
            return 2048;
        const int g = cus * per_cu;
        return g >= 8 ? g - g % 8 : g;
    }();
    return grid;
}

template <bool PRESSURE, int BX, int CLASS>
void launch_batch_class(const BatchTable *T, hipStream_t st)
{
    hipLaunchKernelGGL((batch_phase<PRESSURE, BX, CLASS>), dim3(batch_grid<PRESSURE, BX, CLASS>()), dim3(BX), 0, st, T);
}

template <bool PRESSURE>
void launch_batch_phase(const BatchTable *T, int bx, unsigned classes, hipStream_t st)
{
    if (bx == 64) {                                 // classes 0 and 2 (at most 4 mechanisms)
        if (classes & 1u) launch_batch_class<PRESSURE, 64, 0>(T, st);
        if (classes & 4u) launch_batch_class<PRESSURE, 64, 2>(T, st);
        return;
    }
    if (classes & 1u) launch_batch_class<PRESSURE, 256, 0>(T, st);
    if (classes & 2u) launch_batch_class<PRESSURE, 256, 1>(T, st);
    if (classes & 4u) launch_batch_class<PRESSURE, 256, 2>(T, st);
    if (classes & 8u) launch_batch_class<PRESSURE, 256, 3>(T, st);
}

hipError_t launch_batch_step(const BatchTable *T, int n_entries_max, int bx, unsigned classes, hipStream_t st)
{
    launch_batch_phase<true>(T, bx, classes, st);
    hipLaunchKernelGGL(batch_sparse, dim3(n_entries_max), dim3(256), 0, st, T);
    launch_batch_phase<false>(T, bx, classes, st);
    return hipGetLastError();
}

void prepare_batch_launches()
{
    (void)batch_grid<true, 64, 0>();
    (void)batch_grid<true, 64, 2>();
    (void)batch_grid<false, 64, 0>();
    (void)batch_grid<false, 64, 2>();
    (void)batch_grid<true, 256, 0>();
    (void)batch_grid<true, 256, 1>();
    (void)batch_grid<true, 256, 2>();
    (void)batch_grid<true, 256, 3>();
    (void)batch_grid<false, 256, 0>();
    (void)batch_grid<false, 256, 1>();
    (void)batch_grid<false, 256, 2>();
    (void)batch_grid<false, 256, 3>();
}

}  // namespace fw2
