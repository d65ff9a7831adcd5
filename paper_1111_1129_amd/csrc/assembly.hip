// assembly.hip -- assembly of the sparse representation on the GPU
// (lbm_build_adjacency).
//
// The paper's preprocessor (Sec. 3) numbers every box cell with an injective
// key, removes the gaps left by solid cells to get the contiguous index I_c,
// then finds each fluid cell's neighbours in the full representation.  Its
// distributed octree merge of incell runs computes, for every fluid cell, the
// number of fluid cells with a smaller key.  On one GPU that is an exclusive
// prefix count of fluid flags taken in key order, done here as a three-pass
// stream compaction:
//   1. count:  walk key positions in order, decode each to a box cell, test
//              its flag; per-wave ballot + popcount, per-tile total;
//   2. scan:   exclusive scan of the tile totals (one workgroup);
//   3. emit:   walk again; a lane's rank = tile offset + running total +
//              fluid lanes before it (mbcnt over the ballot mask); write
//              cell_of[rank] and index_of[cell];
//   4. adjacency: one thread per fluid cell, 18 neighbour lookups in index_of.
// All counts are exact integers, so the result does not depend on tile size
// or workgroup count (Sec. 8: the same sparse representation always).
//
// Key positions: lexicographic and blocked orders are walked through a
// gap-free "compact" position that decodes directly to the cell holding that
// rank among box cells; the Z curves, the Hilbert curve and the random order
// walk their own key space (a power of two, at most 8x the box) and skip
// positions that decode outside the box.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kScanBlock = 256;
constexpr int kItems = 16;
constexpr int64_t kTile = int64_t(kScanBlock) * kItems;
constexpr int kScanThreads = 1024;
constexpr uint64_t kMaxPositions = uint64_t(1) << 34;

struct KeySpace {
    int order;
    int h;             // random order: half width
    int64_t nx, ny, nz;
    int64_t b;         // blocked: block edge (clamped to the largest dim)
    uint64_t seed;     // random order
    int groups;        // Z curves: number of 1-bit (MORTON1) or 2-bit (MORTON2) groups
    uint64_t positions;
};

__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Inverse of the 4-round Feistel bijection used as the random ordering's key
// (forward round r: (L, R) -> (R, L ^ F_r(R))).
__device__ inline uint64_t feistel_inverse(uint64_t seed, int h, uint64_t v) {
    const uint64_t mask = (uint64_t(1) << h) - 1;
    uint64_t L = (v >> h) & mask, R = v & mask;
    for (int r = 3; r >= 0; --r) {
        const uint64_t prevR = L;
        const uint64_t prevL = R ^ (splitmix64(seed ^ (uint64_t(r) << 32) ^ prevR) & mask);
        L = prevL;
        R = prevR;
    }
    return (L << h) | R;
}

// Cell of the Hilbert key p on the 2^B cube: split p into the three
// transposed words (x's bit the most significant of each 3-bit digit), undo
// the Gray code, then undo the per-level reflections and exchanges from the
// lowest level up (the inverse of Skilling's coordinates-to-index transform).
__device__ inline void hilbert_decode(uint64_t p, int B, int64_t& x, int64_t& y, int64_t& z) {
    uint32_t X[3] = {0u, 0u, 0u};
    for (int j = 0; j < B; ++j) {
        X[0] |= uint32_t((p >> (3 * j + 2)) & 1) << j;
        X[1] |= uint32_t((p >> (3 * j + 1)) & 1) << j;
        X[2] |= uint32_t((p >> (3 * j)) & 1) << j;
    }
    if (B > 0) {
        const uint32_t end = 2u << (B - 1);
        uint32_t t = X[2] >> 1;
        X[2] ^= X[1];
        X[1] ^= X[0];
        X[0] ^= t;
        for (uint32_t q = 2; q != end; q <<= 1) {
            const uint32_t low = q - 1;
            for (int i = 2; i >= 0; --i) {
                if (X[i] & q) {
                    X[0] ^= low;
                } else {
                    const uint32_t swap = (X[0] ^ X[i]) & low;
                    X[0] ^= swap;
                    X[i] ^= swap;
                }
            }
        }
    }
    x = X[0];
    y = X[1];
    z = X[2];
}

// Box cell (linear index) at key position p, or -1 if p is a gap.
__device__ inline int64_t decode(const KeySpace& ks, uint64_t p) {
    const int64_t nx = ks.nx, ny = ks.ny, nz = ks.nz;
    switch (ks.order) {
    case LBM_ORDER_LEX:
        return int64_t(p);
    case LBM_ORDER_BLOCKED: {
        const int64_t b = ks.b;
        int64_t r = int64_t(p);
        const int64_t slab = b * nx * ny;  // every z-slab of blocks but the last is full
        const int64_t Z = r / slab;
        r -= Z * slab;
        const int64_t z0 = Z * b, bz = min(b, nz - z0);
        const int64_t row = b * nx * bz;
        const int64_t Y = r / row;
        r -= Y * row;
        const int64_t y0 = Y * b, by = min(b, ny - y0);
        const int64_t blk = b * by * bz;
        const int64_t X = r / blk;
        r -= X * blk;
        const int64_t x0 = X * b, bx = min(b, nx - x0);
        const int64_t xi = r % bx, t = r / bx;
        const int64_t yi = t % by, zi = t / by;
        return (x0 + xi) + nx * ((y0 + yi) + ny * (z0 + zi));
    }
    case LBM_ORDER_MORTON1: {
        int64_t x = 0, y = 0, z = 0;
        for (int k = 0; k < ks.groups; ++k) {
            x |= int64_t((p >> (3 * k)) & 1) << k;
            y |= int64_t((p >> (3 * k + 1)) & 1) << k;
            z |= int64_t((p >> (3 * k + 2)) & 1) << k;
        }
        if (x >= nx || y >= ny || z >= nz) return -1;
        return x + nx * (y + ny * z);
    }
    case LBM_ORDER_MORTON2: {
        int64_t x = 0, y = 0, z = 0;
        for (int k = 0; k < ks.groups; ++k) {
            x |= int64_t((p >> (6 * k)) & 3) << (2 * k);
            y |= int64_t((p >> (6 * k + 2)) & 3) << (2 * k);
            z |= int64_t((p >> (6 * k + 4)) & 3) << (2 * k);
        }
        if (x >= nx || y >= ny || z >= nz) return -1;
        return x + nx * (y + ny * z);
    }
    case LBM_ORDER_HILBERT: {
        int64_t x, y, z;
        hilbert_decode(p, ks.groups, x, y, z);
        if (x >= nx || y >= ny || z >= nz) return -1;
        return x + nx * (y + ny * z);
    }
    default: {  // random
        const uint64_t lin = feistel_inverse(ks.seed, ks.h, p);
        return lin < uint64_t(nx * ny * nz) ? int64_t(lin) : -1;
    }
    }
}

__device__ __forceinline__ bool fluid_at(const KeySpace& ks, const uint8_t* __restrict__ flag,
                                         uint64_t p, int64_t& lin) {
    lin = p < ks.positions ? decode(ks, p) : -1;
    return lin >= 0 && flag[lin] != 0;
}

__global__ __launch_bounds__(kScanBlock) void k_count(KeySpace ks, const uint8_t* __restrict__ flag,
                                                      uint32_t* __restrict__ tile_count) {
    __shared__ uint32_t wave_sum[kScanBlock / 64];
    const uint64_t t0 = uint64_t(blockIdx.x) * kTile;
    uint32_t mine = 0;
#pragma unroll 4
    for (int j = 0; j < kItems; ++j) {
        int64_t lin;
        const bool fl = fluid_at(ks, flag, t0 + uint64_t(j) * kScanBlock + threadIdx.x, lin);
        mine += __popcll(__ballot(fl));  // same value in every lane of the wave
    }
    if ((threadIdx.x & 63) == 0) wave_sum[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) s += wave_sum[w];
        tile_count[blockIdx.x] = s;
    }
}

// Exclusive scan of n tile counts in place, total written to *total.
__global__ __launch_bounds__(kScanThreads) void k_scan(uint32_t* __restrict__ v, int64_t n,
                                                       int64_t* __restrict__ total) {
    __shared__ uint64_t wave_tot[kScanThreads / 64];
    const int tid = threadIdx.x;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t lo = min(n, tid * per), hi = min(n, lo + per);
    uint64_t local = 0;
    for (int64_t i = lo; i < hi; ++i) local += v[i];
    // inclusive scan of `local` across the workgroup
    const int lane = tid & 63, wave = tid >> 6;
    uint64_t x = local;
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wave_tot[wave] = x;
    __syncthreads();
    uint64_t before = 0;
    for (int w = 0; w < wave; ++w) before += wave_tot[w];
    uint64_t run = before + x - local;  // exclusive prefix of this thread's chunk
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t c = v[i];
        v[i] = uint32_t(run);
        run += c;
    }
    if (tid == kScanThreads - 1) *total = int64_t(before + x);
}

__global__ __launch_bounds__(kScanBlock) void k_emit(KeySpace ks, const uint8_t* __restrict__ flag,
                                                     const uint32_t* __restrict__ tile_offset,
                                                     int32_t* __restrict__ index_of,
                                                     int32_t* __restrict__ cell_of) {
    __shared__ uint32_t wave_cnt[kScanBlock / 64];
    const uint64_t t0 = uint64_t(blockIdx.x) * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t running = tile_offset[blockIdx.x];
    for (int j = 0; j < kItems; ++j) {
        int64_t lin;
        const bool fl = fluid_at(ks, flag, t0 + uint64_t(j) * kScanBlock + threadIdx.x, lin);
        const uint64_t mask = __ballot(fl);
        // fluid lanes below this one in the wave
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                                         __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
        if (lane == 0) wave_cnt[wave] = uint32_t(__popcll(mask));
        __syncthreads();
        uint32_t woff = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kScanBlock / 64; ++w) {
            woff += (w < wave) ? wave_cnt[w] : 0u;
            tot += wave_cnt[w];
        }
        if (fl) {
            const uint32_t r = running + woff + below;
            cell_of[r] = int32_t(lin);
            index_of[lin] = int32_t(r);
        } else if (lin >= 0) {
            index_of[lin] = -1;
        }
        running += tot;
        __syncthreads();
    }
}

struct AdjGeom {
    int32_t nx, ny, nz;
    uint32_t periodic;
    int64_t base, stride;
};

// One thread per fluid cell.  The 18 upstream box indices are computed
// first without branches (a neighbour outside a non-periodic face reads the
// cell's own entry and is then discarded), so the 18 index_of gathers are all
// in flight at once instead of one round trip each.
__global__ __launch_bounds__(256) void k_adjacency(const int32_t* __restrict__ cell_of,
                                                   const int32_t* __restrict__ index_of, int64_t nf,
                                                   AdjGeom g, uint32_t* __restrict__ adj) {
    const int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (m >= nf) return;
    const uint32_t lin = uint32_t(cell_of[m]);
    const uint32_t nx = uint32_t(g.nx), ny = uint32_t(g.ny);
    const int32_t x = int32_t(lin % nx);
    const uint32_t yz = lin / nx;
    const int32_t y = int32_t(yz % ny);
    const int32_t z = int32_t(yz / ny);
    const int64_t self = g.base + m;
    const int32_t dims[3] = {g.nx, g.ny, g.nz};
    uint32_t at[Q - 1];
    uint32_t outside = 0;  // bit k: the upstream cell of direction k + 1 is outside the box
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) {
        const int i = k + 1;
        int32_t q[3] = {x - vel_x(i), y - vel_y(i), z - vel_z(i)};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool lo = q[d] < 0, hi = q[d] >= dims[d];
            const bool wrap = (g.periodic >> d) & 1u;
            if ((lo || hi) && !wrap) outside |= 1u << k;
            q[d] = lo ? q[d] + dims[d] : (hi ? q[d] - dims[d] : q[d]);
        }
        const uint32_t ql = uint32_t(q[0]) + nx * (uint32_t(q[1]) + ny * uint32_t(q[2]));
        at[k] = ((outside >> k) & 1u) ? lin : ql;
    }
    int32_t up[Q - 1];
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) up[k] = index_of[at[k]];
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) {
        const int i = k + 1;
        const bool stream = !((outside >> k) & 1u) && up[k] >= 0;
        const uint64_t slot = stream ? uint64_t(i) * uint64_t(g.stride) + uint64_t(g.base) + uint64_t(up[k])
                                     : uint64_t(opp(i)) * uint64_t(g.stride) + uint64_t(self);
        adj[int64_t(k) * g.stride + self] = uint32_t(slot);
    }
}

static int bits_for(int64_t n) {
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

static int feistel_half_bits(uint64_t n_box) {
    int h = 1;
    while (h < 31 && (uint64_t(1) << (2 * h)) < n_box) ++h;
    return h;
}

// Fills ks; returns LBM_OK or an error for unusable geometry/order.
static lbm_status make_keyspace(const lbm_geom& g, KeySpace& ks) {
    ks = KeySpace{};
    ks.order = g.order;
    ks.nx = g.nx;
    ks.ny = g.ny;
    ks.nz = g.nz;
    const int64_t n_box = int64_t(g.nx) * g.ny * g.nz;
    const int64_t dmax = std::max<int64_t>({g.nx, g.ny, g.nz});
    switch (g.order) {
    case LBM_ORDER_LEX:
        ks.positions = uint64_t(n_box);
        break;
    case LBM_ORDER_BLOCKED:
        if (g.order_param == 0) return LBM_EINVAL;
        // blocks wider than the box order cells exactly like blocks as wide as it
        ks.b = std::min<int64_t>(int64_t(g.order_param), dmax);
        ks.positions = uint64_t(n_box);
        break;
    case LBM_ORDER_MORTON1:
    case LBM_ORDER_HILBERT: {
        ks.groups = bits_for(dmax);
        if (3 * ks.groups > 62) return LBM_EOVERFLOW;
        ks.positions = uint64_t(1) << (3 * ks.groups);
        break;
    }
    case LBM_ORDER_MORTON2: {
        ks.groups = (bits_for(dmax) + 1) / 2;
        if (6 * ks.groups > 62) return LBM_EOVERFLOW;
        ks.positions = uint64_t(1) << (6 * ks.groups);
        break;
    }
    case LBM_ORDER_RANDOM:
        ks.h = feistel_half_bits(uint64_t(n_box));
        ks.seed = g.order_param;
        ks.positions = uint64_t(1) << (2 * ks.h);
        break;
    default:
        return LBM_EINVAL;
    }
    if (ks.positions > kMaxPositions) return LBM_EOVERFLOW;
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_build_adjacency(const lbm_geom* g, const uint8_t* flag, int64_t base,
                                          int64_t stride, int32_t* index_of, int32_t* cell_of,
                                          uint32_t* adj, int64_t cap, int64_t* n_fluid,
                                          void* workspace, size_t* ws_bytes, void* stream) {
    if (!g || !ws_bytes) return LBM_EINVAL;
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return LBM_EINVAL;
    const int64_t n_box = int64_t(g->nx) * g->ny * g->nz;
    if (n_box >= kBoxLimit) return LBM_EOVERFLOW;
    KeySpace ks;
    if (lbm_status st = make_keyspace(*g, ks); st != LBM_OK) return st;
    const int64_t tiles = int64_t((ks.positions + kTile - 1) / kTile);

    // workspace: tile counts | total | index_of scratch (only if index_of is NULL)
    const size_t off_total = align_up(size_t(tiles) * sizeof(uint32_t), 256);
    const size_t off_index = off_total + 256;
    const size_t need = off_index + (index_of ? 0 : align_up(size_t(n_box) * sizeof(int32_t), 256));
    if (!workspace) {
        *ws_bytes = need;
        return LBM_OK;
    }
    if (*ws_bytes < need) return LBM_EWORKSPACE;
    if (!flag || !n_fluid) return LBM_EINVAL;
    if (base < 0 || cap < 0) return LBM_EINVAL;
    if (adj && !stride_fits(stride)) return LBM_EOVERFLOW;

    char* ws = static_cast<char*>(workspace);
    uint32_t* tile_count = reinterpret_cast<uint32_t*>(ws);
    int64_t* total = reinterpret_cast<int64_t*>(ws + off_total);
    int32_t* idx = index_of ? index_of : reinterpret_cast<int32_t*>(ws + off_index);
    hipStream_t s = as_stream(stream);

    k_count<<<dim3(unsigned(tiles)), dim3(kScanBlock), 0, s>>>(ks, flag, tile_count);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    k_scan<<<1, kScanThreads, 0, s>>>(tile_count, tiles, total);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    int64_t nf = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&nf, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    *n_fluid = nf;
    if (!cell_of) return LBM_OK;  // count-only pass
    if (nf > cap) return LBM_ECAPACITY;
    if (adj && stride < base + nf) return LBM_EINVAL;

    k_emit<<<dim3(unsigned(tiles)), dim3(kScanBlock), 0, s>>>(ks, flag, tile_count, idx, cell_of);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    if (adj && nf > 0) {
        AdjGeom ag{g->nx, g->ny, g->nz, g->periodic, base, stride};
        k_adjacency<<<dim3(unsigned((nf + 255) / 256)), dim3(256), 0, s>>>(cell_of, idx, nf, ag, adj);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    }
    return LBM_OK;
}
