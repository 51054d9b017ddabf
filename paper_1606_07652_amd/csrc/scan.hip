// Device-wide exclusive prefix sum (reduce-then-scan) used by the tree build.
#include "internal.h"

namespace rbf {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// Inclusive scan of one value per thread across a 256-thread block (4 waves of 64).
__device__ int block_inclusive_scan(int v, int *lds_waves) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    if (lane == kWave - 1) lds_waves[wave] = v;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < wave; ++w) add += lds_waves[w];
    __syncthreads();
    return v + add;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int *in, int *out, int *sums, int n) {
    __shared__ int lds[kScanThreads / kWave];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int local = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        local += v[k];
    }
    int incl = block_inclusive_scan(local, lds);
    int run = incl - local;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = incl;
}

__global__ void k_scan_add(int *out, const int *offs, int n) {
    int i = blockIdx.x * kScanTile + threadIdx.x;
    int add = offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k, i += kScanThreads)
        if (i < n) out[i] += add;
}

__global__ void k_total(const int *in, const int *ex, int n, int *tot) {
    *tot = (n > 0) ? ex[n - 1] + in[n - 1] : 0;
}

int scan_rec(const int *in, int *out, int n, hipStream_t s) {
    if (n <= 0) return RBF_OK;
    int nb = (n + kScanTile - 1) / kScanTile;
    int *sums = nullptr;
    RBF_HIP(hipMalloc(&sums, sizeof(int) * (size_t)nb * 2 + 64));
    int *soffs = sums + nb;
    k_scan_tiles<<<nb, kScanThreads, 0, s>>>(in, out, sums, n);
    RBF_HIP(hipGetLastError());
    if (nb > 1) {
        int rc = scan_rec(sums, soffs, nb, s);
        if (rc != RBF_OK) { (void)hipFree(sums); return rc; }
        k_scan_add<<<nb, kScanThreads, 0, s>>>(out, soffs, n);
        RBF_HIP(hipGetLastError());
    }
    RBF_HIP(hipStreamSynchronize(s));
    RBF_HIP(hipFree(sums));
    return RBF_OK;
}

}  // namespace

int exclusive_scan_i32(const int *in, int *out, int n, int *total, hipStream_t s) {
    // in and out may alias: keep the last input element for the total.
    int *tmp = nullptr;
    if (total) {
        RBF_HIP(hipMalloc(&tmp, sizeof(int) * 2));
        if (n > 0) RBF_HIP(hipMemcpyAsync(tmp, in + n - 1, sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    int rc = scan_rec(in, out, n, s);
    if (rc != RBF_OK) { if (tmp) (void)hipFree(tmp); return rc; }
    if (total) {
        int h[2] = {0, 0};
        if (n > 0) {
            RBF_HIP(hipMemcpyAsync(tmp + 1, out + n - 1, sizeof(int), hipMemcpyDeviceToDevice, s));
            RBF_HIP(hipMemcpyAsync(h, tmp, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
            RBF_HIP(hipStreamSynchronize(s));
        }
        *total = h[0] + h[1];
        RBF_HIP(hipFree(tmp));
    }
    return RBF_OK;
}

}  // namespace rbf
