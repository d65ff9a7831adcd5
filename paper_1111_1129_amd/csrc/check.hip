// check.hip -- lbm_check_adjacency: the checked mode of an adjacency list.
//
// The pull sweep reads, for list cell m and direction i = k + 1, the slot
// adj[k][base + m]: i * stride + base + m' for a fluid upstream cell m', or
// opp(i) * stride + base + m for a bounce-back (Sec. 2: the adjacency list;
// Sec. 7: the pull scheme).  Two properties make every sweep form safe and
// exact: each entry lies in rows 1..18 of the geometry's own columns
// [base, base + n) (so below 19 * stride, the bound every kernel relies on),
// and the 18 n entries of the geometry are a permutation of those 18 n slots
// (each referenced exactly once: the pull reads every population once, the
// adjoint and the in-place gather-scatter write every slot once).
//
// The check counts, per slot, how many entries reference it (one atomic add
// per entry, out-of-range entries counted apart and never used as an
// address), then counts the slots whose count is not exactly one.  It is a
// debugging and validation aid for adjacencies built or loaded outside the
// library; the library's own assembly is bit-exact with the oracle.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kChkBlock = 256;

__global__ void k_check_clear(uint32_t* p, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// counts[(row - 1) * n + (col - base)] += 1 for every entry (row, col) in
// range; out_of_range[0] += 1 otherwise
__global__ __launch_bounds__(kChkBlock) void k_check_refs(const uint32_t* __restrict__ adj,
                                                          int64_t base, int64_t n, int64_t stride,
                                                          uint32_t* __restrict__ counts,
                                                          unsigned long long* out_of_range) {
    const int64_t m = int64_t(blockIdx.x) * kChkBlock + threadIdx.x;
    if (m >= n) return;
    unsigned int bad = 0;
    for (int k = 0; k < Q - 1; ++k) {
        const uint64_t slot = adj[k * stride + base + m];
        const uint64_t row = slot / uint64_t(stride);
        const uint64_t col = slot % uint64_t(stride);
        if (row < 1 || row > uint64_t(Q - 1) || col < uint64_t(base) ||
            col >= uint64_t(base + n)) {
            ++bad;
            continue;
        }
        atomicAdd(&counts[int64_t(row - 1) * n + int64_t(col) - base], 1u);
    }
    if (bad) atomicAdd(out_of_range, static_cast<unsigned long long>(bad));
}

// not_once[0] += number of slots whose count is not 1
__global__ __launch_bounds__(kChkBlock) void k_check_once(const uint32_t* __restrict__ counts,
                                                          int64_t total,
                                                          unsigned long long* not_once) {
    unsigned int local = 0;
    for (int64_t i = int64_t(blockIdx.x) * kChkBlock + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * kChkBlock)
        local += counts[i] != 1u ? 1u : 0u;
    // wave sum, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off, 64);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(not_once, static_cast<unsigned long long>(local));
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_check_adjacency(int64_t base, int64_t n, int64_t stride,
                                          const uint32_t* adj, int64_t* result,
                                          void* workspace, size_t* ws_bytes, void* stream) {
    if (!ws_bytes || base < 0 || n < 0) return LBM_EINVAL;
    if (base > INT64_MAX - n) return LBM_EOVERFLOW;
    if (lbm_status st = check_layout(base + n, stride); st != LBM_OK) return st;
    const size_t off_counts = 256;  // the two 64-bit counters, then the slot counts
    const size_t need = off_counts + align_up(size_t(Q - 1) * size_t(n) * sizeof(uint32_t), 256);
    if (!workspace) {
        *ws_bytes = need;
        return LBM_OK;
    }
    if (*ws_bytes < need) return LBM_EWORKSPACE;
    if (!adj || !result) return LBM_EINVAL;
    result[0] = result[1] = 0;
    if (n == 0) return LBM_OK;
    hipStream_t s = as_stream(stream);
    char* ws = static_cast<char*>(workspace);
    auto* counters = reinterpret_cast<unsigned long long*>(ws);
    auto* counts = reinterpret_cast<uint32_t*>(ws + off_counts);
    const int64_t words = int64_t(need / sizeof(uint32_t));
    k_check_clear<<<dim3(unsigned((words + 255) / 256)), 256, 0, s>>>(reinterpret_cast<uint32_t*>(ws),
                                                                      words);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    k_check_refs<<<dim3(unsigned((n + kChkBlock - 1) / kChkBlock)), kChkBlock, 0, s>>>(
        adj, base, n, stride, counts, counters);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    const int64_t total = (Q - 1) * n;
    const int64_t blocks = std::min<int64_t>(4096, (total + kChkBlock - 1) / kChkBlock);
    k_check_once<<<dim3(unsigned(blocks)), kChkBlock, 0, s>>>(counts, total, counters + 1);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    unsigned long long host[2] = {0, 0};
    LBM_TRY_HIP(hipMemcpyAsync(host, counters, sizeof(host), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    result[0] = int64_t(host[0]);
    result[1] = int64_t(host[1]);
    return LBM_OK;
}
