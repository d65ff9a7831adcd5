// partition.hip -- communication analysis of the list cut into chunks
// (lbm_partition_stats).
//
// A solver on G devices would cut the 1-D list into G near-equal chunks
// (paper Sec. 2: chunk k = [floor(k n / G), floor((k+1) n / G)), sizes differ
// by at most one cell).  Sec. 7 / Fig. 7 characterise a cut by, per chunk,
// the number of neighbour chunks and the number of remote links (PDFs a
// chunk pulls from cells of other chunks).  One thread per cell walks its 18
// adjacency entries: a streaming entry (direction of the slot = direction of
// the entry) whose source cell lies in another chunk is a remote link; the
// pair (own chunk, source chunk) is recorded in a G x G bitmap.  Bounce-back
// entries never leave the cell.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kPartBlock = 256;
constexpr int64_t kMaxChunks = 16384;

// chunk of list cell m: the largest k with floor(k n / G) <= m
__device__ __forceinline__ int64_t chunk_of(int64_t m, int64_t n, int64_t G) {
    return ((m + 1) * G - 1) / n;
}

__global__ void k_zero_u32(uint32_t* p, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

__global__ __launch_bounds__(kPartBlock) void k_partition_links(
    const uint32_t* __restrict__ adj, int64_t n, int64_t stride, int64_t G, int64_t words,
    unsigned long long* __restrict__ remote, uint32_t* __restrict__ interface_cells,
    uint32_t* __restrict__ bitmap) {
    const int64_t m = int64_t(blockIdx.x) * kPartBlock + threadIdx.x;
    if (m >= n) return;
    const int64_t a = chunk_of(m, n, G);
    unsigned int links = 0;
    uint32_t slots[Q - 1];  // all 18 loads in flight before the first atomic
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) slots[k] = adj[k * stride + m];
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) {
        const int64_t slot = slots[k];
        const int64_t src = slot - (k + 1) * stride;
        if (src < 0 || src >= stride) continue;  // bounce-back (another row): own population
        if (src >= n) continue;  // not a listed cell of [0, n)
        const int64_t b = chunk_of(src, n, G);
        if (b == a) continue;
        ++links;
        atomicOr(&bitmap[a * words + (b >> 5)], 1u << (b & 31));
    }
    if (links) {
        atomicAdd(&remote[a], (unsigned long long)links);
        atomicAdd(&interface_cells[a], 1u);
    }
}

__global__ void k_partition_count(const uint32_t* __restrict__ bitmap, int64_t G, int64_t words,
                                  const unsigned long long* __restrict__ remote_tmp,
                                  const uint32_t* __restrict__ iface_tmp, int64_t* remote_links,
                                  int32_t* neighbours, int32_t* interface_cells) {
    const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= G) return;
    int32_t c = 0;
    for (int64_t w = 0; w < words; ++w) c += __popc(bitmap[a * words + w]);
    neighbours[a] = c;
    remote_links[a] = int64_t(remote_tmp[a]);
    interface_cells[a] = int32_t(iface_tmp[a]);
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_partition_stats(int64_t n, int64_t stride, const uint32_t* adj,
                                          int64_t n_chunks, int64_t* remote_links,
                                          int32_t* neighbours, int32_t* interface_cells,
                                          void* workspace, size_t* ws_bytes, void* stream) {
    if (!ws_bytes || n_chunks <= 0 || n_chunks > kMaxChunks) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    const int64_t G = n_chunks;
    const int64_t words = (G + 31) / 32;
    const size_t off_iface = align_up(size_t(G) * sizeof(unsigned long long), 256);
    const size_t off_bits = off_iface + align_up(size_t(G) * sizeof(uint32_t), 256);
    const size_t need = off_bits + align_up(size_t(G * words) * sizeof(uint32_t), 256);
    if (!workspace) {
        *ws_bytes = need;
        return LBM_OK;
    }
    if (*ws_bytes < need) return LBM_EWORKSPACE;
    if (!adj || !remote_links || !neighbours || !interface_cells || n <= 0) return LBM_EINVAL;
    hipStream_t s = as_stream(stream);
    char* ws = static_cast<char*>(workspace);
    auto* remote = reinterpret_cast<unsigned long long*>(ws);
    auto* iface = reinterpret_cast<uint32_t*>(ws + off_iface);
    auto* bits = reinterpret_cast<uint32_t*>(ws + off_bits);
    const int64_t zero_words = int64_t(need / sizeof(uint32_t));
    k_zero_u32<<<dim3(unsigned((zero_words + 255) / 256)), 256, 0, s>>>(reinterpret_cast<uint32_t*>(ws),
                                                                          zero_words);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    k_partition_links<<<dim3(unsigned((n + kPartBlock - 1) / kPartBlock)), kPartBlock, 0, s>>>(
        adj, n, stride, G, words, remote, iface, bits);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    k_partition_count<<<dim3(unsigned((G + 255) / 256)), 256, 0, s>>>(bits, G, words, remote, iface,
                                                                      remote_links, neighbours,
                                                                      interface_cells);
    return after_launch();
}
