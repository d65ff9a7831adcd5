// batch.hip -- sweeps of many geometries that each keep their own TRT
// parameters, one launch per step or all steps in one persistent launch
// (lbm_step with per-segment parameters or persistent = 1, lbm_step_batch).
//
// Several geometries share one set of [19][stride] PDF arrays and one
// adjacency list, each in its own column range (a segment); their adjacency
// entries already carry the segment's base, so one sweep over [0, n)
// advances all of them.  Here the TRT constants (s+, s-, the force terms) are
// read per tile from a small table in the caller's workspace instead of being
// kernel arguments: entry k holds parameter set k, and a per-tile index says
// which set a tile uses.  When any segment selects a set other than 0, every
// segment starts on a tile boundary (256 cells), so a tile never holds cells
// of two segments and the choice stays uniform over the workgroup (scalar
// loads, no per-lane branch).  A tile no segment touches uses set 0; the
// cells of a segment's last tile past its end (which no other segment may
// claim) run with the segment's set.
//
// The adjacency is read as the full uint32 list, as 16-bit codes, or as 8-bit
// codes in the tiles that have them (the choice the code-reading sweeps
// make), and the arithmetic per cell is that of every other sweep, so a
// member's state is bitwise what a solo run of that member gives.
//
// Persistent launch: a cooperative grid of one 1024-thread workgroup per CU
// walks the tiles in groups of 4 (XCD-chunked like the per-step sweep's
// tiles), each wave its own quarter-tiles, with a grid-wide barrier between
// steps (two levels, every wait bounded):
//  * census at kernel start: each workgroup reads its XCD from the XCC_ID
//    hardware register and counts itself into xcd_size[xcd];
//  * per step, every thread waits for its own stores to be acknowledged by
//    the XCD's L2 (s_waitcnt 0), the workgroup arrives on xcd_count[xcd];
//    the last arrival of an XCD writes that L2 back (one agent-scope release
//    per XCD instead of one per workgroup) and increments the global count;
//    every workgroup polls the global count with relaxed loads and takes one
//    acquire fence (L1/L2 invalidate) when all XCDs have arrived.
// Past the spin limit a workgroup raises the error flag and every workgroup
// leaves the kernel, so the launch always drains; the host then reports
// LBM_EBARRIER.  The grid never exceeds one workgroup per CU: for the FP32
// sweep both the occupancy query and the compiler's resource report give 7
// co-resident workgroups per CU (70 VGPRs), yet a grid of 7 per CU once
// stalled in the census with 6 per CU arrived -- slots that neither model
// counts were unavailable -- so only one slot per CU is relied on.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kBBlock = kCodeTile;            // one workgroup = one tile of 256 cells
constexpr long kSpinLimit = 1L << 27;         // polls of ~256 clocks: ~14 s, far above any step
constexpr size_t kBarrierBytes = 256;         // workspace: barrier block
constexpr int kParamsPerFill = 32;            // parameter sets per table-writing launch
constexpr int kSegsPerFill = 256;             // segments per tile-index-writing launch

// One parameter set as the sweep reads it (FP64, host-computed).
struct ParamEntry {
    double sp, sm;       // s+ = 1/tau+, s- = 1/tau-
    double F[NPAIR];     // 3 w c.G of the odd member of each pair
    double pad;
};
static_assert(sizeof(ParamEntry) == 96, "ParamEntry layout");

struct ParamChunk {
    int count;
    ParamEntry e[kParamsPerFill];
};

struct SegTiles {
    int32_t first, last, param;  // tiles [first, last) use parameter set `param`
};

struct SegChunk {
    int count;
    SegTiles s[kSegsPerFill];
};

// Table and per-tile index in the workspace.
struct ParamTable {
    const ParamEntry* entries;  // n_params entries
    const int32_t* tile_param;  // per tile, or nullptr: every tile uses entry 0
};

__global__ void k_write_params(ParamEntry* dst, ParamChunk chunk) {
    const int i = threadIdx.x;
    if (i < chunk.count) dst[i] = chunk.e[i];
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// One workgroup per segment of the chunk: mark its tiles.
__global__ void k_mark_tiles(int32_t* tile_param, SegChunk chunk) {
    const SegTiles st = chunk.s[blockIdx.x];
    for (int32_t t = st.first + int32_t(threadIdx.x); t < st.last; t += blockDim.x) tile_param[t] = st.param;
}

// The TRT constants of a tile (uniform over the wave: scalar loads; the
// table is read-only for the launch, which the __restrict__ kernel
// arguments tell the compiler, so the loads stay scalar after the sweep's
// first stores).
__device__ __forceinline__ TrtConst tile_const(const ParamEntry* __restrict__ entries,
                                               const int32_t* __restrict__ tile_param, int64_t tile) {
    const int32_t k = tile_param ? tile_param[tile] : 0;
    const ParamEntry& e = entries[k];
    TrtConst c;
    c.sp = e.sp;
    c.sm = e.sm;
    c.G[0] = c.G[1] = c.G[2] = 0.0;  // the sweep uses the force through F only
#pragma unroll
    for (int q = 0; q < NPAIR; ++q) c.F[q] = e.F[q];
    return c;
}

// Where a tile's slots come from: SRC is the narrowest form the launch may
// use, each tile takes what its record allows (8-bit codes in a narrow tile,
// the full list in a tile with escapes, else 16-bit codes).
enum BatchSrc { kAdj = 0, kC16 = 1, kC8 = 2 };

template <int ST, bool PBB, bool NT, int SRC>
__device__ __forceinline__ void sweep_tile(const typename Storage<ST>::T* __restrict__ src,
                                           typename Storage<ST>::T* __restrict__ dst,
                                           const int8_t* __restrict__ codes8,
                                           const int16_t* __restrict__ codes,
                                           const int32_t* __restrict__ tile_rec,
                                           const uint32_t* __restrict__ adj,
                                           const double* __restrict__ ns, int64_t tile, int64_t m,
                                           int64_t stride, const TrtConst& c) {
    if constexpr (SRC == kAdj) {
        update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
    } else {
        const int32_t* rec = tile_rec + tile * kCodeRec;  // uniform over the workgroup
        if (SRC == kC8 && rec[Q] != 0)
            update_cell_coded<ST, PBB, NT, int8_t>(src, dst, codes8, rec, ns, m, stride, c);
        else if (rec[Q - 1] != 0)
            update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
        else
            update_cell_coded<ST, PBB, NT, int16_t>(src, dst, codes, rec, ns, m, stride, c);
    }
}

// One launch per step, constants from the table.
template <int ST, bool PBB, bool NT, int SRC>
__global__ __launch_bounds__(kBBlock) void k_trt_table(const typename Storage<ST>::T* __restrict__ src,
                                                       typename Storage<ST>::T* __restrict__ dst,
                                                       const int8_t* __restrict__ codes8,
                                                       const int16_t* __restrict__ codes,
                                                       const int32_t* __restrict__ tile_rec,
                                                       const uint32_t* __restrict__ adj,
                                                       const double* __restrict__ ns, int64_t n,
                                                       int64_t stride,
                                                       const ParamEntry* __restrict__ entries,
                                                       const int32_t* __restrict__ tile_param,
                                                       int chunk_shift) {
    const int64_t tile = logical_block(chunk_shift);
    const int64_t m = tile * kBBlock + threadIdx.x;
    if (m >= n) return;
    const TrtConst c = tile_const(entries, tile_param, tile);
    sweep_tile<ST, PBB, NT, SRC>(src, dst, codes8, codes, tile_rec, adj, ns, tile, m, stride, c);
}

// ---------------------------------------------------------------------------
// persistent launch
// ---------------------------------------------------------------------------
// barrier block layout (uint32 words): [0] global count, [1] error flag,
// [8..16) per-XCD arrivals, [16..24) per-XCD workgroup counts
struct Barrier {
    unsigned int* count;
    int* error;
    unsigned int* xcd_count;
    unsigned int* xcd_size;
};

__device__ __forceinline__ int xcc_id() {
    // hardware register XCC_ID, bits [3:0]: the XCD this wave runs on
    return int(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (NXCD - 1));
}

__device__ bool wait_at_least(unsigned int* cnt, unsigned int target, int* err) {
    long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(4);  // 4 x 64 clocks between polls
        if (++spins > kSpinLimit ||
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Persistent workgroups are 1024 threads (16 waves, one workgroup per CU):
// a pass of the walk covers a group of 4 consecutive tiles, one tile per
// quarter of the waves, and every wave walks its own quarter-tiles without
// waiting for the others; the waves of a workgroup meet only at the grid
// barrier between steps.  16 independent waves per CU (4 per SIMD, the
// occupancy of the FP64 one-launch-per-step sweep; the narrower storages
// allow more, which measured no faster at 6 per SIMD) keep many loads in
// flight; a 256-thread workgroup per CU (one wave per SIMD) left each tile's
// dependent loads exposed and ran at about 60 % of the per-step rate.
constexpr int kPThreads = 1024;
constexpr int kPWaves = kPThreads / 64;
constexpr int kGroupTiles = kPWaves / (kBBlock / 64);  // 4 tiles per pass

template <int ST, bool PBB, bool NT, int SRC>
__global__ __launch_bounds__(kPThreads) void k_trt_persistent(typename Storage<ST>::T* fa,
                                                              typename Storage<ST>::T* fb,
                                                              const int8_t* __restrict__ codes8,
                                                              const int16_t* __restrict__ codes,
                                                              const int32_t* __restrict__ tile_rec,
                                                              const uint32_t* __restrict__ adj,
                                                              const double* __restrict__ ns,
                                                              int64_t n, int64_t stride,
                                                              const ParamEntry* __restrict__ entries,
                                                              const int32_t* __restrict__ tile_param,
                                                              int n_steps, int chunk_shift,
                                                              Barrier bar) {
    __shared__ int ok;
    __shared__ unsigned int populated;
    const int xcc = xcc_id();
    // census
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&bar.xcd_size[xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(bar.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        ok = wait_at_least(bar.count, gridDim.x, bar.error);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unsigned int p = 0;
        for (int x = 0; x < NXCD; ++x)
            p += __hip_atomic_load(&bar.xcd_size[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        populated = p;
    }
    __syncthreads();
    if (!ok) return;
    const unsigned int mine =
        __hip_atomic_load(&bar.xcd_size[xcc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    // the wave index is uniform over the wave; readfirstlane lets the compiler
    // see it, so the tile index, its record and its parameter set stay scalar
    // (scalar loads); derived from threadIdx they were per-lane vector loads
    // that each iteration waited for, and the walk ran ~36 % slower
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    const int lane = int(threadIdx.x) & 63;
    const int64_t tiles = (n + kBBlock - 1) / kBBlock;
    const int64_t groups = (tiles + kGroupTiles - 1) / kGroupTiles;
    const int64_t q = int64_t(NXCD) << chunk_shift;
    const int64_t vgroups = (groups + q - 1) / q * q;  // virtual groups, relabelled like workgroups
    const int64_t my_tile_in_group = wave / (kBBlock / 64);
    const int64_t my_quarter = (wave % (kBBlock / 64)) * 64 + lane;
    unsigned int gen = 0;
    for (int step = 0; step < n_steps; ++step) {
        const auto* src = (step & 1) ? fb : fa;
        auto* dst = (step & 1) ? fa : fb;
        for (int64_t v = blockIdx.x; v < vgroups; v += gridDim.x) {
            const int64_t grp = ((v >> (3 + chunk_shift)) << (3 + chunk_shift)) +
                                ((v & (NXCD - 1)) << chunk_shift) +
                                ((v >> 3) & ((int64_t(1) << chunk_shift) - 1));
            const int64_t tile = grp * kGroupTiles + my_tile_in_group;
            const int64_t m = tile * kBBlock + my_quarter;
            if (grp < groups && m < n) {
                const TrtConst c = tile_const(entries, tile_param, tile);
                sweep_tile<ST, PBB, NT, SRC>(src, dst, codes8, codes, tile_rec, adj, ns, tile, m,
                                             stride, c);
            }
        }
        if (step + 1 == n_steps) break;
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores acknowledged by the L2
        __syncthreads();
        ++gen;
        if (threadIdx.x == 0) {
            const unsigned int prev =
                __hip_atomic_fetch_add(&bar.xcd_count[xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (prev + 1 == gen * mine) {
                // last workgroup of this XCD: write the XCD's L2 back, then arrive
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(bar.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            ok = wait_at_least(bar.count, gridDim.x + gen * populated, bar.error);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (!ok) return;
    }
}

__global__ void k_fill_u32(unsigned int* p, int count, unsigned int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchLaunch {
    int64_t n, stride;
    const int8_t* codes8;
    const int16_t* codes;
    const int32_t* rec;
    const uint32_t* adj;
    const double* ns;
    void* fa;
    void* fb;
    int n_steps;
    int chunk_shift;             // per-step launch: runs of tiles per XCD
    int chunk_shift_persistent;  // persistent launch: runs of 4-tile groups per XCD
    ParamTable tab;
    void* barrier;  // persistent only
};

template <int ST, bool PBB, bool NT, int SRC>
lbm_status launch_table_steps(const BatchLaunch& L, hipStream_t s) {
    using T = typename Storage<ST>::T;
    T* a = static_cast<T*>(L.fa);
    T* b = static_cast<T*>(L.fb);
    const dim3 g{unsigned(grid_blocks(L.n, kBBlock, L.chunk_shift))}, blk{unsigned(kBBlock)};
    for (int k = 0; k < L.n_steps; ++k) {
        const T* src = (k & 1) ? b : a;
        T* dst = (k & 1) ? a : b;
        k_trt_table<ST, PBB, NT, SRC><<<g, blk, 0, s>>>(src, dst, L.codes8, L.codes, L.rec, L.adj,
                                                        L.ns, L.n, L.stride, L.tab.entries,
                                                        L.tab.tile_param, L.chunk_shift);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    }
    return LBM_OK;
}

template <int ST, bool PBB, bool NT, int SRC>
lbm_status launch_persistent_t(const BatchLaunch& L, hipStream_t s) {
    using T = typename Storage<ST>::T;
    auto kern = k_trt_persistent<ST, PBB, NT, SRC>;
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    LBM_TRY_HIP(hipGetDevice(&dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return LBM_EHIP;
    LBM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                             kPThreads, 0));
    if (per_cu < 1) return LBM_EHIP;
    // one workgroup per CU at most (see the file header), a multiple of the XCD count
    const int64_t tiles = (L.n + kBBlock - 1) / kBBlock;
    const int64_t groups = (tiles + kGroupTiles - 1) / kGroupTiles;
    int64_t grid = std::min<int64_t>(cus, (groups + NXCD - 1) / NXCD * NXCD);
    grid = grid / NXCD * NXCD;
    if (grid < NXCD || grid > cus) return LBM_EHIP;

    unsigned int* w = static_cast<unsigned int*>(L.barrier);
    Barrier bar{w, reinterpret_cast<int*>(w + 1), w + 8, w + 16};
    // clear with a kernel (no memset node if the caller captures the stream)
    k_fill_u32<<<1, 64, 0, s>>>(w, 24, 0u);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;

    T* a = static_cast<T*>(L.fa);
    T* b = static_cast<T*>(L.fb);
    const int8_t* c8 = L.codes8;
    const int16_t* c16 = L.codes;
    const int32_t* rec = L.rec;
    const uint32_t* adj = L.adj;
    const double* ns = L.ns;
    int64_t n = L.n, stride = L.stride;
    const ParamEntry* entries = L.tab.entries;
    const int32_t* tile_param = L.tab.tile_param;
    int steps = L.n_steps, cs = L.chunk_shift_persistent;
    void* args[] = {&a, &b, &c8, &c16, &rec, &adj, &ns, &n, &stride, &entries, &tile_param, &steps,
                    &cs, &bar};
    LBM_TRY_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(unsigned(grid)),
                                           dim3(kPThreads), args, 0, s));
    int err = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&err, bar.error, sizeof(int), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return err ? LBM_EBARRIER : LBM_OK;
}

template <int ST, bool PBB, bool NT>
lbm_status launch_batch_src(const BatchLaunch& L, bool persistent, hipStream_t s) {
    if (persistent) {
        if (L.codes8) return launch_persistent_t<ST, PBB, NT, kC8>(L, s);
        if (L.codes) return launch_persistent_t<ST, PBB, NT, kC16>(L, s);
        return launch_persistent_t<ST, PBB, NT, kAdj>(L, s);
    }
    if (L.codes8) return launch_table_steps<ST, PBB, NT, kC8>(L, s);
    if (L.codes) return launch_table_steps<ST, PBB, NT, kC16>(L, s);
    return launch_table_steps<ST, PBB, NT, kAdj>(L, s);
}

template <int ST>
lbm_status launch_batch_st(const BatchLaunch& L, bool nt, bool persistent, hipStream_t s) {
    if (L.ns) return nt ? launch_batch_src<ST, true, true>(L, persistent, s)
                        : launch_batch_src<ST, true, false>(L, persistent, s);
    return nt ? launch_batch_src<ST, false, true>(L, persistent, s)
              : launch_batch_src<ST, false, false>(L, persistent, s);
}

// Workspace of a table launch: barrier block | parameter table | tile index.
struct BatchWs {
    size_t table_off, tiles_off, total;
};

inline BatchWs batch_ws(int32_t n_params, bool per_tile, int64_t n) {
    BatchWs w;
    w.table_off = kBarrierBytes;
    w.tiles_off = w.table_off + align_up(size_t(n_params) * sizeof(ParamEntry), 256);
    const int64_t tiles = (n + kBBlock - 1) / kBBlock;
    w.total = w.tiles_off + (per_tile ? align_up(size_t(std::max<int64_t>(tiles, 1)) * sizeof(int32_t), 256) : 0);
    return w;
}

static_assert(kSegmentAlign == kBBlock, "segments start on sweep tiles");

size_t step_batch_workspace(int32_t n_params, const lbm_segment* seg, int32_t n_seg, int64_t n) {
    return batch_ws(n_params, uses_param_sets(seg, n_seg), n).total;
}

// Every argument has been validated by the entry point; the workspace holds
// at least step_batch_workspace() bytes.
lbm_status step_batch(const lbm_params* p, int32_t n_params, const lbm_segment* seg,
                      int32_t n_seg, int64_t n, int64_t stride, const int8_t* codes8,
                      const int16_t* codes, const int32_t* tile_records, const uint32_t* adj,
                      const double* ns, void* f_a, void* f_b, int32_t n_steps, bool persistent,
                      void* workspace, hipStream_t s) {
    const bool per_tile = uses_param_sets(seg, n_seg);
    const BatchWs w = batch_ws(n_params, per_tile, n);
    char* ws = static_cast<char*>(workspace);
    auto* entries = reinterpret_cast<ParamEntry*>(ws + w.table_off);
    auto* tile_param = per_tile ? reinterpret_cast<int32_t*>(ws + w.tiles_off) : nullptr;
    // parameter table, written from kernel arguments (nothing host-resident
    // has to outlive the call)
    for (int32_t k0 = 0; k0 < n_params; k0 += kParamsPerFill) {
        ParamChunk ch;
        ch.count = std::min<int32_t>(kParamsPerFill, n_params - k0);
        for (int i = 0; i < ch.count; ++i) {
            const TrtConst c = make_trt_const(p[k0 + i]);
            ParamEntry& e = ch.e[i];
            e.sp = c.sp;
            e.sm = c.sm;
            for (int q = 0; q < NPAIR; ++q) e.F[q] = c.F[q];
            e.pad = 0.0;
        }
        k_write_params<<<1, 64, 0, s>>>(entries + k0, ch);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    }
    if (per_tile) {
        const int64_t tiles = (n + kBBlock - 1) / kBBlock;
        k_fill_i32<<<dim3(unsigned((tiles + 255) / 256)), 256, 0, s>>>(tile_param, tiles, 0);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
        for (int32_t k0 = 0; k0 < n_seg; k0 += kSegsPerFill) {
            SegChunk ch;
            ch.count = 0;
            for (int32_t k = k0; k < std::min<int32_t>(n_seg, k0 + kSegsPerFill); ++k) {
                if (seg[k].n == 0) continue;
                SegTiles& t = ch.s[ch.count++];
                t.first = int32_t(seg[k].base / kBBlock);
                t.last = int32_t((seg[k].base + seg[k].n + kBBlock - 1) / kBBlock);
                t.param = seg[k].param_index;
            }
            if (ch.count == 0) continue;
            k_mark_tiles<<<ch.count, 256, 0, s>>>(tile_param, ch);
            if (hipGetLastError() != hipSuccess) return LBM_EHIP;
        }
    }
    BatchLaunch L{n, stride, codes8, codes, tile_records, adj, ns, f_a, f_b, n_steps,
                  chunk_shift_for(p[0].flags, n, kBBlock), chunk_shift_for(p[0].flags, n, kPThreads),
                  ParamTable{entries, tile_param}, ws};
    const bool nt = (p[0].flags & LBM_FLAG_NONTEMPORAL) != 0;
    switch (p[0].storage) {
    case LBM_F64: return launch_batch_st<LBM_F64>(L, nt, persistent, s);
    case LBM_F64_SHIFTED: return launch_batch_st<LBM_F64_SHIFTED>(L, nt, persistent, s);
    case LBM_F32: return launch_batch_st<LBM_F32>(L, nt, persistent, s);
    case LBM_F32_SHIFTED: return launch_batch_st<LBM_F32_SHIFTED>(L, nt, persistent, s);
    case LBM_F16_SHIFTED: return launch_batch_st<LBM_F16_SHIFTED>(L, nt, persistent, s);
    case LBM_F16_SHIFTED_SCALED: return launch_batch_st<LBM_F16_SHIFTED_SCALED>(L, nt, persistent, s);
    default: return LBM_EINVAL;
    }
}

}  // namespace lbm
