// Rows kept in leaf order during a tree (for deep trees and many classes).
//
// A level's histograms need, per slot tile, only the rows of the tile's
// leaves. With rows in their original order, a tile of leaf slots that does
// not fit in LDS beside the others makes every block of every tile scan all
// rows (the histograms of all leaves of a deep level of a many-class problem
// are far larger than the LDS of the whole chip). So here,
// after the split of level l is chosen, the rows are moved by a stable
// partition on the new leaf bit: rows whose bit is 0 first, then rows whose
// bit is 1, each group in its previous order. Since the rows were already
// sorted by their leaf index below bit l, they end up sorted by the full
// leaf index (a least-significant-digit radix step), so the rows of any run
// of consecutive leaves are one contiguous range.
//
// Moved per row: the bins of every feature (16-row tiled layout, staged in
// LDS so that whole 16-byte segments are written), the gradient statistics
// the histogram reads, the original row id and the leaf index. Level 0 reads
// the problem's own arrays; level l writes buffer l % 2 and level l + 1
// reads it. After the last level's split the leaf index of every row is
// written back to the problem's leaf array (original order) for the leaf
// solve and the approx update.
//
// The histogram of a partitioned level runs the lanes-over-features tile
// over the row range of each slot tile only (chunks of the range, one block
// per chunk x feature group x class), and a merge that sums each slot tile's
// chunks.
#include <algorithm>
#include <vector>

#include "common.h"
#include "kernels_dev.h"

namespace cbh {

constexpr int kPartThreads = 256;
constexpr int64_t kPartRows = 1024;                // positions per partition block
constexpr int kPartSegs = 64;                      // 16-row segments per partition block
constexpr int kPartFeat = 16;                      // features staged per LDS round
constexpr int kPartLdsLeaves = 4096;               // leaf counters kept in LDS up to this L

}  // namespace cbh

struct cbh_part {
    cbh_ctx* ctx = nullptr;
    int64_t n = 0, n_pad = 0, n_pb = 0;
    int32_t F = 0, K = 0, depth = 0, loss = 0;
    uint8_t* bins[2] = {nullptr, nullptr};      // tiled [n_pad / 16][F][16]
    const uint8_t** cols[2] = {nullptr, nullptr};   // device: column f -> bins + 16 f
    int64_t* seg = nullptr;                     // device [F]: 16 F
    float* g[2] = {nullptr, nullptr};           // [K][n_pad]
    float* h[2] = {nullptr, nullptr};           // [K][n_pad] (not for RMSE)
    uint32_t* gq[2] = {nullptr, nullptr};       // [K][n_pad] int16 code pairs
    int32_t* order[2] = {nullptr, nullptr};     // original row of each position
    uint16_t* code[2] = {nullptr, nullptr};     // leaf of each position (0xffff: padding)
    int64_t* off[2] = {nullptr, nullptr};       // [2^(depth-1) + 1] first position of each leaf
    uint32_t* zl = nullptr;                     // [2^(depth-2)] rows of each leaf with bit 0
    int64_t* blk = nullptr;                     // [n_pb + 1] zeros per block, then their prefix
    int64_t* cp = nullptr;                      // [2^(depth-1) + 1] chunk prefix of slot tiles, in
                                                // the tiles' processing order
    int32_t* tord = nullptr;                    // [2 * 2^(depth-1)]: tile at each place of that
                                                // order, then the place of each tile
    int32_t* tleaf = nullptr;                   // [2^(depth-1)] child a subtraction build accumulates
};

namespace cbh {

// Exclusive prefix over 256 threads of one value each; `total` gets the sum.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* sh,
                                                       uint32_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    uint32_t wb = 0;
    for (int i = 0; i < w; ++i) wb += sh[i];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return wb + x - v;
}

// Exclusive prefix over `count` items by one block of 1024 threads, each
// taking a contiguous run; get(i) gives item i, put(i, prefix) receives it.
// Returns the total (in every thread).
template <class Get, class Put>
__device__ int64_t block_scan_1024(int64_t count, Get get, Put put, int64_t* sh) {
    const int64_t per = (count + 1023) / 1024;
    const int64_t i0 = min(count, int64_t(threadIdx.x) * per), i1 = min(count, i0 + per);
    int64_t s = 0;
    for (int64_t i = i0; i < i1; ++i) s += get(i);
    sh[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 run sums
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t y = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    const int64_t total = sh[1023];
    int64_t run = sh[threadIdx.x] - s;
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t v = get(i);
        put(i, run);
        run += v;
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ bool split_bit(const uint8_t* col, int64_t st, int64_t pos, int k) {
    return col != nullptr && (int)*seg_ptr(col, st, pos) > k;
}

// Rows with bit 0 per block (blk) and per current leaf (zl, added).
__global__ __launch_bounds__(kPartThreads) void part_count_kernel(
    const uint8_t* const* __restrict__ cols, const int64_t* __restrict__ seg, int32_t F,
    const cbh_split* __restrict__ split, int64_t n, const uint16_t* __restrict__ code, int32_t L,
    uint32_t* __restrict__ zl, int64_t* __restrict__ blk) {
    extern __shared__ uint32_t zc[];
    __shared__ uint32_t sh[8];
    const bool lds_cnt = L <= kPartLdsLeaves;
    if (lds_cnt)
        for (int i = threadIdx.x; i < L; i += kPartThreads) zc[i] = 0u;
    __syncthreads();
    const cbh_split sp = *split;
    const bool none = sp.feature < 0 || sp.feature >= F;
    const uint8_t* col = none ? nullptr : cols[sp.feature];
    const int64_t st = none ? 16 : seg_stride_of(seg, sp.feature);
    const int64_t p0 = int64_t(blockIdx.x) * kPartRows + int64_t(threadIdx.x) * 4;
    // this thread's 4 rows (one half of a 16-row segment's quarter): bins
    // and leaf codes in one load each where aligned
    uint32_t zbits = 0u, lf[4] = {0u, 0u, 0u, 0u};
    const uint8_t* pb = col ? seg_ptr(col, st, p0) : nullptr;
    if (p0 + 4 <= n && (!pb || (reinterpret_cast<uintptr_t>(pb) & 3) == 0) &&
        (!code || (reinterpret_cast<uintptr_t>(code + p0) & 7) == 0)) {
        const uint32_t bw = pb ? *reinterpret_cast<const uint32_t*>(pb) : 0u;
        const uint2 cw = code ? *reinterpret_cast<const uint2*>(code + p0) : make_uint2(0u, 0u);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!(pb && (int)((bw >> (8 * j)) & 255u) > sp.border)) zbits |= 1u << j;
            lf[j] = ((j < 2 ? cw.x : cw.y) >> (16 * (j & 1))) & 0xffffu;
        }
    } else {
        for (int j = 0; j < 4; ++j) {
            const int64_t pos = p0 + j;
            if (pos >= n) break;
            if (!split_bit(col, st, pos, sp.border)) zbits |= 1u << j;
            lf[j] = code ? (uint32_t)code[pos] : 0u;
        }
    }
    const uint32_t zeros = (uint32_t)__popc(zbits);
    // per-leaf zero counts: the rows are in leaf order, so the lanes of a
    // wave mostly share one leaf; each distinct leaf of a row slot gets one
    // atomic add of its lanes' sum instead of one add per row
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        bool pending = (zbits >> j) & 1u;
        while (__any(pending)) {
            const uint64_t act = __ballot(pending);
            const int leader = __ffsll((unsigned long long)act) - 1;
            const uint32_t l0 = __shfl(lf[j], leader, 64);
            const bool mine = pending && lf[j] == l0;
            const uint32_t cnt = (uint32_t)__popcll(__ballot(mine));
            if (lane == leader) {
                if (lds_cnt) atomicAdd(&zc[l0], cnt);
                else atomicAdd(&zl[l0], cnt);
            }
            pending = pending && !mine;
        }
    }
    uint32_t tot;
    (void)block_excl_scan256(zeros, sh, tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
    if (lds_cnt)
        for (int i = threadIdx.x; i < L; i += kPartThreads)
            if (zc[i]) atomicAdd(&zl[i], zc[i]);
}

// One block: block zero counts -> exclusive prefix (blk[n_pb] = all zeros);
// leaf offsets of the 2L new leaves (leaf v < L: the zeros of old leaf v;
// v >= L: the ones of old leaf v - L); zl cleared for the next level.
__global__ __launch_bounds__(1024) void part_scan_kernel(int64_t* __restrict__ blk, int64_t n_pb,
                                                         uint32_t* __restrict__ zl, int32_t L,
                                                         const int64_t* __restrict__ off_old,
                                                         int64_t n, int64_t* __restrict__ off_new) {
    __shared__ int64_t sh[1024];
    const int64_t nz = block_scan_1024(
        n_pb, [&](int64_t i) { return blk[i]; }, [&](int64_t i, int64_t e) { blk[i] = e; }, sh);
    if (threadIdx.x == 0) blk[n_pb] = nz;
    auto count = [&](int64_t v) -> int64_t {
        if (v < L) return (int64_t)zl[v];
        const int64_t u = v - L;
        const int64_t old = off_old ? off_old[u + 1] - off_old[u] : n;
        return old - (int64_t)zl[u];
    };
    (void)block_scan_1024(2 * int64_t(L), count, [&](int64_t v, int64_t e) { off_new[v] = e; },
                          sh);
    if (threadIdx.x == 0) off_new[2 * L] = n;
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += 1024) zl[i] = 0u;
}

struct PartMove {
    const uint8_t* const* src_cols;
    const int64_t* src_seg;
    uint8_t* dst_bins;             // tiled, segment stride 16 F
    int32_t F, K, level;
    const cbh_split* split;
    int64_t n, n_pad, n_pb;
    const int64_t* blk;            // exclusive zero prefix per block, total at [n_pb]
    const int32_t* src_order;      // NULL: identity
    int32_t* dst_order;
    const uint16_t* src_code;      // NULL: leaf 0
    uint16_t* dst_code;
    const float* src_g;            // each NULL when not moved
    const float* src_h;
    const uint32_t* src_gq;
    int64_t src_stride;            // elements between classes in the source
    float* dst_g;
    float* dst_h;
    uint32_t* dst_gq;
};

// The stable partition itself, one block per kPartRows positions:
//   1. wave 0 (lane = 16-row segment) finds the rows' bits and destinations,
//      and for each destination run the source row of every destination
//      (inv);
//   2. all threads move row ids, leaf indices and statistics (4 rows each);
//   3. the bins, kPartFeat features per round: consecutive threads read
//      consecutive 16-byte (segment, feature) pieces (each segment's features
//      contiguously) and store them unchanged in LDS, one row of bytes per
//      feature (rows padded so that different features fall on different
//      banks; the next round's pieces are loaded while this one is written).
//      Then every destination segment of the block's two runs (its zero rows
//      go to [Zb, Zb + nzb), its one rows to [O0, O0 + nob)) is gathered
//      byte by byte through inv and written, features fastest: whole
//      segments as one 16-byte store, the partial ones at the run ends byte
//      by byte (the neighbouring block owns their other bytes).
constexpr int kPartSrcRow = kPartRows + 16;   // bytes per staged feature (65 x 16)
constexpr int kPartRun = kPartRows + 32;      // destination slots per run

__global__ __launch_bounds__(kPartThreads) void part_scatter_kernel(PartMove m) {
    __shared__ __align__(16) uint8_t stage[kPartFeat * kPartSrcRow];
    __shared__ uint16_t inv[2][kPartRun];      // source row of destination base + i
    __shared__ int32_t rel[kPartRows];        // destination - base of its run
    __shared__ uint32_t segbits[kPartSegs], segvalid[kPartSegs];
    __shared__ uint32_t nzb_sh;
    const cbh_split sp = *m.split;
    const bool none = sp.feature < 0 || sp.feature >= m.F;
    const int64_t P0 = int64_t(blockIdx.x) * kPartRows;
    const int64_t Zb = m.blk[blockIdx.x], NZ = m.blk[m.n_pb];
    const int64_t O0 = NZ + (P0 - Zb);
    const int64_t base[2] = {Zb & ~int64_t(15), O0 & ~int64_t(15)};
    if (threadIdx.x < 64) {
        const int sg = threadIdx.x;
        const uint8_t* scol = none ? nullptr : m.src_cols[sp.feature];
        const int64_t sst = none ? 16 : seg_stride_of(m.src_seg, sp.feature);
        const int64_t p0 = P0 + 16 * sg;
        uint32_t bits = 0u, valid = 0u;
        const uint8_t* sb = scol ? scol + (p0 >> 4) * sst : nullptr;
        if (sb && p0 + 16 <= m.n && ((reinterpret_cast<uintptr_t>(sb) & 15) == 0)) {
            // the segment's 16 bins of the split feature in one load
            const uint4 w = gld_u4(sb);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
            valid = 0xffffu;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if ((int)((ws[j >> 2] >> (8 * (j & 3))) & 255u) > sp.border) bits |= 1u << j;
        } else {
            for (int j = 0; j < 16; ++j) {
                const int64_t pos = p0 + j;
                if (pos >= m.n) break;
                valid |= 1u << j;
                if (split_bit(scol, sst, pos, sp.border)) bits |= 1u << j;
            }
        }
        const uint32_t zmask = valid & ~bits;
        const uint32_t nz = (uint32_t)__popc(zmask);
        uint32_t x = nz;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (sg >= d) x += y;
        }
        const uint32_t zt = x - nz;
        if (sg == 63) nzb_sh = x;
        segbits[sg] = bits;
        segvalid[sg] = valid;
        for (int j = 0; j < 16; ++j) {
            if (!((valid >> j) & 1u)) break;
            const int64_t zb = Zb + zt + __popc(zmask & ((1u << j) - 1u));
            const int r = (bits >> j) & 1u;
            const int64_t d = r ? NZ + (p0 + j - zb) : zb;
            const int32_t rl = (int32_t)(d - base[r]);
            rel[16 * sg + j] = rl;
            inv[r][rl] = (uint16_t)(16 * sg + j);
        }
    }
    __syncthreads();
    const int64_t nzb = nzb_sh;
    const int64_t nvb = min(kPartRows, m.n - P0);
    const int64_t nob = nvb - nzb;
    // row ids, leaf indices and statistics: the thread's rows i = t + 256 q,
    // each class's loads of all of them issued before their stores (source
    // and destination are different copies)
    {
        constexpr int kQ = kPartRows / kPartThreads;
        int64_t pos[kQ], dst[kQ];
        bool ok[kQ];
        uint32_t bitv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int i = threadIdx.x + kPartThreads * q;
            ok[q] = i < nvb;
            pos[q] = P0 + i;
            bitv[q] = ok[q] ? (segbits[i >> 4] >> (i & 15)) & 1u : 0u;
            dst[q] = ok[q] ? base[bitv[q]] + rel[i] : 0;
        }
        const int32_t* __restrict__ so = m.src_order;
        const uint16_t* __restrict__ sc = m.src_code;
        int32_t ov[kQ];
        uint32_t cv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            ov[q] = ok[q] ? (so ? so[pos[q]] : (int32_t)pos[q]) : 0;
            cv[q] = ok[q] && sc ? (uint32_t)sc[pos[q]] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            if (!ok[q]) continue;
            m.dst_order[dst[q]] = ov[q];
            m.dst_code[dst[q]] = (uint16_t)(cv[q] | (bitv[q] << m.level));
        }
        const float* __restrict__ sg = m.src_g;
        const float* __restrict__ sh = m.src_h;
        const uint32_t* __restrict__ sq = m.src_gq;
        for (int c = 0; c < m.K; ++c) {
            const int64_t so_c = int64_t(c) * m.src_stride, do_c = int64_t(c) * m.n_pad;
            float gv[kQ], hv[kQ];
            uint32_t qv[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                gv[q] = ok[q] && m.dst_g ? sg[so_c + pos[q]] : 0.f;
                hv[q] = ok[q] && m.dst_h ? sh[so_c + pos[q]] : 0.f;
                qv[q] = ok[q] && m.dst_gq ? sq[so_c + pos[q]] : 0u;
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                if (!ok[q]) continue;
                if (m.dst_g) m.dst_g[do_c + dst[q]] = gv[q];
                if (m.dst_h) m.dst_h[do_c + dst[q]] = hv[q];
                if (m.dst_gq) m.dst_gq[do_c + dst[q]] = qv[q];
            }
        }
    }
    const int64_t run0[2] = {Zb, O0}, run1[2] = {Zb + nzb, O0 + nob};
    const int64_t s0[2] = {run0[0] >> 4, run0[1] >> 4};
    const int64_t ns[2] = {nzb ? ((run1[0] + 15) >> 4) - s0[0] : 0,
                           nob ? ((run1[1] + 15) >> 4) - s0[1] : 0};
    const int64_t dstride = 16 * int64_t(m.F);
    const int64_t seg0 = P0 >> 4;
    // thread t owns pieces c = t + 256 q (q < 4) of a round: segment c / 16,
    // feature f0 + c % 16
    constexpr int kPieces = kPartSegs * kPartFeat / kPartThreads;
    uint4 w[kPieces];
    auto load_round = [&](int f0) {
        const int nfe = min(kPartFeat, m.F - f0);
#pragma unroll
        for (int q = 0; q < kPieces; ++q) {
            const int c = threadIdx.x + kPartThreads * q;
            const int sg = c / kPartFeat, fi = c % kPartFeat;
            const uint32_t valid = segvalid[sg];
            w[q] = make_uint4(0u, 0u, 0u, 0u);
            if (fi >= nfe || !valid) continue;
            const int f = f0 + fi;
            const uint8_t* src = m.src_cols[f] + (seg0 + sg) * seg_stride_of(m.src_seg, f);
            if (valid == 0xffffu && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
                w[q] = gld_u4(src);
            } else {
                uint32_t t[4] = {0u, 0u, 0u, 0u};
                for (int j = 0; j < 16; ++j)
                    if ((valid >> j) & 1u) t[j >> 2] |= gld_u8(src + j) << (8 * (j & 3));
                w[q] = make_uint4(t[0], t[1], t[2], t[3]);
            }
        }
    };
    load_round(0);
    for (int f0 = 0; f0 < m.F; f0 += kPartFeat) {
        const int nfe = min(kPartFeat, m.F - f0);
#pragma unroll
        for (int q = 0; q < kPieces; ++q) {
            const int c = threadIdx.x + kPartThreads * q;
            const int sg = c / kPartFeat, fi = c % kPartFeat;
            if (fi >= nfe || !segvalid[sg]) continue;
            *reinterpret_cast<uint4*>(stage + fi * kPartSrcRow + 16 * sg) = w[q];
        }
        __syncthreads();
        if (f0 + kPartFeat < m.F) load_round(f0 + kPartFeat);
        const int64_t nseg = ns[0] + ns[1];
        for (int64_t it = threadIdx.x; it < nseg * nfe; it += kPartThreads) {
            const int fi = (int)(it % nfe);
            const int64_t q = it / nfe;
            const int r = q < ns[0] ? 0 : 1;
            const int64_t s = s0[r] + (r ? q - ns[0] : q);
            const int64_t lo = max(run0[r], 16 * s), hi = min(run1[r], 16 * s + 16);
            if (lo >= hi) continue;
            const uint8_t* srow = stage + fi * kPartSrcRow;
            const uint16_t* iv = inv[r] + (16 * s - base[r]);
            uint8_t* to = m.dst_bins + s * dstride + 16 * int64_t(f0 + fi);
            if (lo == 16 * s && hi == 16 * s + 16) {
                uint32_t t[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int p = 0; p < 16; ++p)
                    t[p >> 2] |= (uint32_t)srow[iv[p]] << (8 * (p & 3));
                *reinterpret_cast<uint4*>(to) = make_uint4(t[0], t[1], t[2], t[3]);
            } else {
                for (int64_t p = lo; p < hi; ++p) to[p - 16 * s] = srow[iv[p - 16 * s]];
            }
        }
        __syncthreads();
    }
}

// After the last level's split: leaf index of every row, in original order.
__global__ __launch_bounds__(256) void part_leaf_kernel(const uint8_t* const* __restrict__ cols,
                                                        const int64_t* __restrict__ seg, int32_t F,
                                                        const cbh_split* __restrict__ split,
                                                        int64_t n, int32_t level,
                                                        const int32_t* __restrict__ order,
                                                        const uint16_t* __restrict__ code,
                                                        uint16_t* __restrict__ leaf) {
    const cbh_split sp = *split;
    const bool none = sp.feature < 0 || sp.feature >= F;
    const uint8_t* col = none ? nullptr : cols[sp.feature];
    const int64_t st = none ? 16 : seg_stride_of(seg, sp.feature);
    for (int64_t pos = int64_t(blockIdx.x) * 256 + threadIdx.x; pos < n;
         pos += int64_t(gridDim.x) * 256) {
        const uint32_t bit = split_bit(col, st, pos, sp.border) ? 1u : 0u;
        const int64_t row = order ? order[pos] : pos;
        leaf[row] = (uint16_t)((code ? (uint32_t)code[pos] : 0u) | (bit << level));
    }
}

// Chunks of every slot tile: tile t holds leaves [t lt, min((t+1) lt, L)),
// i.e. positions [off[t lt], off[...]) and the 16-row segments over them.
// With tleaf (a build by subtraction: lt = 1, n_tiles = L / 2 parents), tile
// t is parent t and holds only its child with fewer rows, leaf t or t + L / 2
// (the lower one on a tie), whose leaf index goes to tleaf[t].
// The tiles are processed largest first (their rows, descending; ties by
// index): blocks start in index order, and leaves differ in size by orders
// of magnitude, so the chunks of a large leaf started last would leave most
// CUs idle while they finish. tord[q] is the tile at place q, tord[n_tiles +
// t] the place of tile t, and cp the exclusive prefix of chunks by place
// (total at [n_tiles]). Beyond kTileSort tiles the order is the index order.
constexpr int kTileSort = 2048;

__global__ __launch_bounds__(1024) void part_tiles_kernel(const int64_t* __restrict__ off,
                                                          int32_t L, int32_t lt, int32_t n_tiles,
                                                          int64_t segs_per_chunk,
                                                          int64_t* __restrict__ cp,
                                                          int32_t* __restrict__ tord,
                                                          int32_t* __restrict__ tleaf) {
    __shared__ int64_t sh[1024];
    __shared__ int64_t rows_sh[kTileSort];
    __shared__ int32_t ord_sh[kTileSort];
    auto first_leaf = [&](int64_t t) -> int64_t {
        if (!tleaf) return t * lt;
        const int64_t hi = t + n_tiles;
        return off[hi + 1] - off[hi] < off[t + 1] - off[t] ? hi : t;
    };
    auto range = [&](int64_t t, int64_t& a, int64_t& b) {
        const int64_t v = first_leaf(t);
        a = off[v];
        b = tleaf ? off[v + 1] : off[min((t + 1) * int64_t(lt), int64_t(L))];
    };
    auto chunks = [&](int64_t t) -> int64_t {
        int64_t a, b;
        range(t, a, b);
        if (a >= b) return 0;
        return (((b + 15) >> 4) - (a >> 4) + segs_per_chunk - 1) / segs_per_chunk;
    };
    const bool sorted = n_tiles <= kTileSort;
    if (sorted) {
        for (int t = threadIdx.x; t < n_tiles; t += 1024) {
            int64_t a, b;
            range(t, a, b);
            rows_sh[t] = b - a;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < n_tiles; t += 1024) {
            const int64_t rt = rows_sh[t];
            int q = 0;
            for (int u = 0; u < n_tiles; ++u) {
                const int64_t ru = rows_sh[u];
                q += (ru > rt || (ru == rt && u < t)) ? 1 : 0;
            }
            ord_sh[q] = t;
            tord[n_tiles + t] = q;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n_tiles; q += 1024) tord[q] = ord_sh[q];
    } else {
        for (int t = threadIdx.x; t < n_tiles; t += 1024) {
            tord[t] = t;
            tord[n_tiles + t] = t;
        }
    }
    const int64_t tot = block_scan_1024(
        n_tiles, [&](int64_t q) { return chunks(sorted ? ord_sh[q] : q); },
        [&](int64_t q, int64_t e) { cp[q] = e; }, sh);
    if (tleaf)
        for (int t = threadIdx.x; t < n_tiles; t += 1024) tleaf[t] = (int32_t)first_leaf(t);
    if (threadIdx.x == 0) cp[n_tiles] = tot;
}

struct PartHist {
    const uint8_t* const* cols;
    const int64_t* seg;
    const float* g;
    const float* h;
    const uint32_t* gq;
    const uint16_t* code;
    const int64_t* off;
    const int64_t* cp;             // chunk prefix by place in the processing order
    const int32_t* tord;           // tile at each place
    const int32_t* tleaf;          // subtraction: the leaf tile t (a parent) accumulates, or NULL
    uint32_t* partials;            // [chunk][lt][F][B][wpc]
    int64_t n_pad, n_items, segs_per_chunk;
    int32_t F, B, K, L, lt, n_tiles, n_fgroups, wpc;
};

// Block -> (class, feature group, chunk). Chunks go to the XCDs in turn
// (chunk gc to XCD gc mod 8; block b runs on XCD b mod 8), and each chunk's
// group and class blocks are neighbours on its XCD, the classes of one group
// adjacent (they read the same bins). Leaves, and so chunks, differ in size,
// and neighbouring leaves tend to be alike (they share their high split
// bits): a contiguous range of chunks per XCD would leave some XCDs with far
// more rows than others. The chunk's slot tile is found by binary search
// over cp.
template <int PREC, int RM, int W>
__global__ __launch_bounds__(kHistThreads) void hist_part_kernel(PartHist a) {
    extern __shared__ __align__(16) uint32_t lds[];
    const int64_t per_gc = int64_t(a.n_fgroups) * a.K;
    const int64_t bx = blockIdx.x >> 3;
    const int64_t gc = (bx / per_gc) * 8 + (blockIdx.x & 7);
    if (gc * per_gc >= a.n_items) return;
    const int64_t r = bx % per_gc;
    const int c = (int)(r % a.K);
    const int fg = (int)(r / a.K);
    if (gc >= a.cp[a.n_tiles]) return;
    int lo = 0, hi = a.n_tiles - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.cp[mid] <= gc) lo = mid; else hi = mid - 1;
    }
    const int t = a.tord[lo];
    const int64_t j = gc - a.cp[lo];
    const uint32_t s0 = a.tleaf ? (uint32_t)a.tleaf[t] : (uint32_t)t * (uint32_t)a.lt;
    const uint32_t ns = a.tleaf ? 1u : min((uint32_t)a.lt, (uint32_t)a.L - s0);
    const int64_t pa = a.off[s0], pb = a.off[s0 + ns];
    const int64_t sa = (pa >> 4) + j * a.segs_per_chunk;
    const int64_t sb = min((pb + 15) >> 4, sa + a.segs_per_chunk);
    LpfBlock b;
    b.bins = a.cols;
    b.seg = a.seg;
    b.g = a.g + int64_t(c) * a.n_pad;
    b.h = a.h ? a.h + int64_t(c) * a.n_pad : nullptr;
    b.gq = a.gq ? a.gq + int64_t(c) * a.n_pad : nullptr;
    b.rowcode = a.code;
    b.F = a.F;
    b.B = a.B;
    b.wpc = a.wpc;
    b.coff = c * (a.wpc / a.K);
    lpf_zero<PREC, W>(a.B, ns, lds);
    __syncthreads();
    // With one slot per tile, every row of a segment inside the tile's range
    // is in the slot: no per-row code is needed there (mode 0). Only the
    // tile's first and last segments can hold rows of neighbouring leaves (or
    // padding rows): mode 2 checks their codes.
    const bool head = ns == 1 && j == 0 && (pa & 15) != 0;
    const bool tail = ns == 1 && sb == ((pb + 15) >> 4) && (pb & 15) != 0;
    const int64_t ia = sa + (head ? 1 : 0), ib = sb - (tail ? 1 : 0);
    if (ns == 1 && ia < ib) {
        if (head) lpf_accumulate<PREC, RM, W, 2>(b, sa * 16, ia * 16, fg, s0, ns, lds);
        lpf_accumulate<PREC, RM, W, 0>(b, ia * 16, ib * 16, fg, s0, ns, lds);
        if (tail) lpf_accumulate<PREC, RM, W, 2>(b, ib * 16, sb * 16, fg, s0, ns, lds);
    } else {
        lpf_accumulate<PREC, RM, W, 2>(b, sa * 16, sb * 16, fg, s0, ns, lds);
    }
    __syncthreads();
    lpf_flush<PREC, RM, W>(b, fg, s0, ns, a.partials + gc * (int64_t(a.lt) * a.F * a.B * a.wpc),
                           s0, lds);
}

// Output (cell, class) units (cell = leaf, feature, bin): the sum of the
// unit's slot tile's chunks, in chunk order, with the arithmetic of the other
// merges (two-float: TwoSum of the (hi, lo) parts). One thread per unit, so
// consecutive threads read the consecutive classes' words of a cell.
// Subtraction (tleaf != NULL; lt = 1, L = the number of parents): unit cell
// (p, f, b) sums parent p's tile, which is leaf tleaf[p]; the sibling leaf
// gets parent - sum (a two-float difference, exact for int16 sums and counts,
// a float difference for FP32).
__device__ __forceinline__ float2 f2_sub_pair(float2 P, float2 r) {
    const float t = P.x - r.x;
    const float bp = t - P.x;
    const float e = ((P.x - (t - bp)) + (-r.x - bp)) + (P.y - r.y);
    const float dh = t + e;
    return make_float2(dh, e - (dh - t));
}

template <int PREC>
__global__ __launch_bounds__(256) void part_merge_kernel(const uint32_t* __restrict__ part,
                                                         const int64_t* __restrict__ cp,
                                                         const int32_t* __restrict__ tplace,
                                                         int32_t L, int32_t lt, int32_t F,
                                                         int32_t B, int32_t K, int32_t wpc,
                                                         int32_t rmse, void* __restrict__ out,
                                                         const int32_t* __restrict__ tleaf,
                                                         const void* __restrict__ parent) {
    const int64_t fb = int64_t(F) * B, cells_lt = int64_t(lt) * fb;
    const int64_t units = int64_t(L) * fb * K;
    const int64_t cw = cells_lt * wpc;                  // words per chunk partial
    for (int64_t u = int64_t(blockIdx.x) * 256 + threadIdx.x; u < units;
         u += int64_t(gridDim.x) * 256) {
        const int64_t cell = u / K;
        const int c = (int)(u % K);
        const int64_t v = cell / fb, rest = cell % fb;
        const int64_t t = v / lt;
        const int64_t q = tplace[t];
        const int64_t g0 = cp[q];
        const int nch = (int)(cp[q + 1] - g0);
        const uint32_t* p = part + g0 * cw + ((v - t * lt) * fb + rest) * wpc;
        // where the sum goes, and (subtraction) the sibling's cell
        int64_t dst = cell, sib = -1;
        if (tleaf) {
            const int64_t leaf = tleaf[v];
            dst = leaf * fb + rest;
            sib = (leaf == v ? v + L : v) * fb + rest;
        }
        if constexpr (PREC == CBH_PREC_FP32) {
            float g = 0.f, hh = 0.f;
            uint32_t cnt = 0;
            for (int ch = 0; ch < nch; ++ch) {
                const uint2 w = *reinterpret_cast<const uint2*>(p + ch * cw + 2 * c);
                g += __uint_as_float(w.x);
                if (rmse) cnt += w.y; else hh += __uint_as_float(w.y);
            }
            float* of = reinterpret_cast<float*>(out);
            uint32_t* ou = reinterpret_cast<uint32_t*>(out);
            of[dst * 2 * K + 2 * c] = g;
            if (rmse) ou[dst * 2 * K + 2 * c + 1] = cnt;
            else of[dst * 2 * K + 2 * c + 1] = hh;
            if (sib >= 0) {
                const float* pf = reinterpret_cast<const float*>(parent);
                const uint32_t* pu = reinterpret_cast<const uint32_t*>(parent);
                const int64_t e = cell * 2 * K + 2 * c;
                of[sib * 2 * K + 2 * c] = pf[e] - g;
                if (rmse) ou[sib * 2 * K + 2 * c + 1] = pu[e + 1] - cnt;
                else of[sib * 2 * K + 2 * c + 1] = pf[e + 1] - hh;
            }
        } else if constexpr (PREC == CBH_PREC_TWOFLOAT) {
            float S[2] = {0.f, 0.f}, E[2] = {0.f, 0.f};
            uint32_t cnt = 0;
            for (int ch = 0; ch < nch; ++ch) {
                const uint4 w = *reinterpret_cast<const uint4*>(p + ch * cw + 4 * c);
                const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int st = 0; st < 2; ++st) {
                    if (st == 1 && rmse) {
                        cnt += ww[2];
                        continue;
                    }
                    const float hi = __uint_as_float(ww[2 * st]);
                    const float lo = __uint_as_float(ww[2 * st + 1]);
                    const float tt = S[st] + hi;
                    const float bp = tt - S[st];
                    const float e = (S[st] - (tt - bp)) + (hi - bp);
                    S[st] = tt;
                    E[st] += e + lo;
                }
            }
            float2 r[2];
#pragma unroll
            for (int st = 0; st < 2; ++st) {
                const float hs = S[st] + E[st];
                r[st] = make_float2(hs, E[st] - (hs - S[st]));
            }
            if (rmse) r[1] = make_float2(__uint_as_float(cnt), 0.f);
            float2* o = reinterpret_cast<float2*>(out) + dst * 2 * K + 2 * c;
            o[0] = r[0];
            o[1] = r[1];
            if (sib >= 0) {
                const float2* P = reinterpret_cast<const float2*>(parent) + cell * 2 * K + 2 * c;
                float2* os = reinterpret_cast<float2*>(out) + sib * 2 * K + 2 * c;
                os[0] = f2_sub_pair(P[0], r[0]);
                os[1] = rmse ? make_float2(__uint_as_float(__float_as_uint(P[1].x) - cnt), 0.f)
                             : f2_sub_pair(P[1], r[1]);
            }
        } else {
            int64_t gs = 0, hs = 0;
            for (int ch = 0; ch < nch; ++ch) {
                const uint64_t w = *reinterpret_cast<const uint64_t*>(p + ch * cw + 2 * c);
                hs += (int64_t)(uint32_t)(w & 0xffffffffull);
                gs += (int64_t)(int32_t)(uint32_t)(w >> 32);
            }
            int64_t* o = reinterpret_cast<int64_t*>(out) + 2 * (dst * K + c);
            o[0] = gs;
            o[1] = hs;
            if (sib >= 0) {
                const int64_t* P = reinterpret_cast<const int64_t*>(parent) + 2 * (cell * K + c);
                int64_t* os = reinterpret_cast<int64_t*>(out) + 2 * (sib * K + c);
                os[0] = P[0] - gs;
                os[1] = P[1] - hs;
            }
        }
    }
}

void part_init_attrs(int max_lds) {
    const void* fns[] = {
        (const void*)hist_part_kernel<CBH_PREC_FP32, 0, 32>,
        (const void*)hist_part_kernel<CBH_PREC_FP32, 0, 16>,
        (const void*)hist_part_kernel<CBH_PREC_FP32, 0, 8>,
        (const void*)hist_part_kernel<CBH_PREC_FP32, 0, 4>,
        (const void*)hist_part_kernel<CBH_PREC_FP32, 1, 32>,
        (const void*)hist_part_kernel<CBH_PREC_FP32, 1, 16>,
        (const void*)hist_part_kernel<CBH_PREC_FP32, 1, 8>,
        (const void*)hist_part_kernel<CBH_PREC_FP32, 1, 4>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 0, 32>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 0, 16>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 0, 8>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 0, 4>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 1, 32>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 1, 16>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 1, 8>,
        (const void*)hist_part_kernel<CBH_PREC_TWOFLOAT, 1, 4>,
        (const void*)hist_part_kernel<CBH_PREC_INT16, 0, 32>,
        (const void*)hist_part_kernel<CBH_PREC_INT16, 0, 16>,
        (const void*)hist_part_kernel<CBH_PREC_INT16, 0, 8>,
        (const void*)hist_part_kernel<CBH_PREC_INT16, 0, 4>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 0, 32>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 0, 16>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 0, 8>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 0, 4>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 1, 32>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 1, 16>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 1, 8>,
        (const void*)hist_part_kernel<CBH_PREC_F64, 1, 4>};
    for (const void* f : fns)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
}

template <int PREC, int RM>
static void launch_part_hist(const PartHist& a, int W, unsigned grid, size_t lds, hipStream_t s) {
    switch (W) {
        case 32: hist_part_kernel<PREC, RM, 32><<<grid, kHistThreads, lds, s>>>(a); break;
        case 16: hist_part_kernel<PREC, RM, 16><<<grid, kHistThreads, lds, s>>>(a); break;
        case 8: hist_part_kernel<PREC, RM, 8><<<grid, kHistThreads, lds, s>>>(a); break;
        default: hist_part_kernel<PREC, RM, 4><<<grid, kHistThreads, lds, s>>>(a); break;
    }
}

// Plan of a build over rows in leaf order: a slot tile reads only its own
// rows, so more tiles cost no re-reads; the widest lane group whose tile of
// one slot fits the LDS (fewest feature groups, so the statistics are read
// fewest times), as many slots per tile as the LDS budget holds (at least
// one, at most 64; one slot lets the block skip the row codes inside its
// range), and chunks of at least min_rows rows sized so that the blocks of
// the whole level reach target_blocks (8 times that with several classes).
// A build by subtraction (sub) takes one parent per tile and reads about half
// the rows, which the chunk sizing assumes.
static HistPlan plan_part(const HistKnobs& kn, int64_t n, int32_t F, int32_t B, int32_t K,
                          int32_t L, int32_t precision, int max_lds, bool sub = false) {
    HistPlan p;
    p.kind = 1;
    p.words_per_cell = words_per_cell(precision, K);
    const uint32_t cs = precision == CBH_PREC_INT16 ? 8 : 16;
    int32_t W = kn.lpf_w > 0 ? std::min(kn.lpf_w, 32) : 32;
    while (W > 4 && int64_t(B) * lpf_record_bytes(W, cs) > max_lds) W /= 2;
    p.fb = W;
    const int64_t slot_bytes = int64_t(B) * lpf_record_bytes(W, cs);
    const int64_t budget = std::min<int64_t>(kn.lds_budget, max_lds);
    p.lt = sub ? 1
               : (int32_t)std::max<int64_t>(
                     1, std::min<int64_t>({int64_t(L), 64, budget / slot_bytes}));
    p.n_ltiles = sub ? L / 2 : (L + p.lt - 1) / p.lt;
    if (sub) n = std::max<int64_t>(1, n / 2);
    p.n_fgroups = (F + W - 1) / W;
    const int64_t per_chunk = int64_t(p.n_fgroups) * K;     // blocks per chunk of rows
    // the K class blocks of one (chunk, feature group) read the same bins,
    // which stay in L2 only if their row range is short; and leaves differ in
    // size by orders of magnitude, so short chunks also even out the blocks'
    // work (measured on 5*10^7 rows, 10 classes, depth 10: 32 times the
    // block target took the builds of a tree from 257 to 241 ms, at the cost
    // of more partial tiles to merge)
    const int64_t target = int64_t(std::max<int32_t>(1, kn.target_blocks)) * (K > 1 ? 32 : 1);
    int64_t rows = std::max<int64_t>(kn.min_rows, n * per_chunk / target);
    rows = align_up(std::min<int64_t>(rows, align_up(n, 16)), 16);
    if (precision == CBH_PREC_INT16) rows = std::min<int64_t>(rows, 65536);
    p.rows_per_chunk = rows;
    p.n_chunks = (int32_t)((n + rows - 1) / rows);
    p.rep = 1;
    p.lds_bytes = int64_t(p.lt) * slot_bytes;
    p.n_blocks = (int64_t(p.n_chunks) + p.n_ltiles) * per_chunk;
    return p;
}

static void free_part(cbh_part* p) {
    void* bufs[] = {p->bins[0], p->bins[1], p->cols[0], p->cols[1], p->seg,   p->g[0],
                    p->g[1],    p->h[0],    p->h[1],    p->gq[0],   p->gq[1], p->order[0],
                    p->order[1], p->code[0], p->code[1], p->off[0], p->off[1], p->zl,
                    p->blk,     p->cp,      p->tord,    p->tleaf};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

static int check_part(const cbh_part* part, const cbh_problem* prob) {
    CBH_ARG(part != nullptr, "partition is NULL");
    CBH_ARG(prob->n == part->n && prob->n_features == part->F && prob->K == part->K &&
                prob->depth == part->depth && prob->loss == part->loss,
            "problem does not match the partition (n, features, K, depth, loss)");
    CBH_ARG(count_stat(prob) || part->h[0] != nullptr,
            "the partition holds no h (made for RMSE without row weights), the problem needs it");
    CBH_REQUIRE(!packed_bins(prob), CBH_EUNSUPPORTED,
                "leaf-ordered rows take byte bins (the problem has packed bins)");
    return CBH_OK;
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int cbh_part_create(cbh_ctx* ctx, const cbh_problem* prob, cbh_part** out) {
    clear_error();
    CBH_ARG(ctx && out, "NULL argument");
    *out = nullptr;
    int rc = validate_problem(prob);
    if (rc) return rc;
    CBH_REQUIRE(!packed_bins(prob), CBH_EUNSUPPORTED,
                "leaf-ordered rows take byte bins (the problem has packed bins)");
    if (rc) return rc;
    CBH_REQUIRE(prob->depth <= 16, CBH_EUNSUPPORTED, "depth must be <= 16");
    cbh_part* p = new cbh_part();
    p->ctx = ctx;
    p->n = prob->n;
    p->n_pad = align_up(prob->n, 16);
    p->n_pb = (p->n + kPartRows - 1) / kPartRows;
    p->F = prob->n_features;
    p->K = prob->K;
    p->depth = prob->depth;
    p->loss = prob->loss;
    const int64_t np = p->n_pad, F = p->F, K = p->K;
    const int64_t half = int64_t(1) << std::max(0, p->depth - 1);
    auto alloc = [&](void** ptr, int64_t bytes) -> bool {
        if (hipMalloc(ptr, (size_t)std::max<int64_t>(bytes, 256)) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            return false;
        }
        return true;
    };
    bool ok = true;
    for (int b = 0; b < 2 && ok; ++b) {
        ok = alloc((void**)&p->bins[b], np * F) && alloc((void**)&p->cols[b], F * 8) &&
             alloc((void**)&p->g[b], K * np * 4) && alloc((void**)&p->gq[b], K * np * 4) &&
             alloc((void**)&p->order[b], np * 4) && alloc((void**)&p->code[b], np * 2) &&
             alloc((void**)&p->off[b], (2 * half + 1) * 8);
        if (ok && !count_stat(prob)) ok = alloc((void**)&p->h[b], K * np * 4);
    }
    ok = ok && alloc((void**)&p->seg, F * 8) && alloc((void**)&p->zl, half * 4) &&
         alloc((void**)&p->blk, (p->n_pb + 1) * 8) && alloc((void**)&p->cp, (half + 1) * 8) &&
         alloc((void**)&p->tord, 2 * half * 4) && alloc((void**)&p->tleaf, half * 4);
    if (!ok) {
        free_part(p);
        delete p;
        set_error("partition buffers (%lld rows x %lld features) do not fit in device memory",
                  (long long)prob->n, (long long)F);
        return CBH_ENOMEM;
    }
    // padding positions keep code 0xffff (never a slot), zero statistics
    std::vector<const uint8_t*> colv(F);
    std::vector<int64_t> segv(F, 16 * F);
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2; ++b) {
        for (int64_t f = 0; f < F; ++f) colv[f] = p->bins[b] + 16 * f;
        if (e == hipSuccess) e = hipMemcpy(p->cols[b], colv.data(), F * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(p->code[b], 0xff, np * 2);
        if (e == hipSuccess) e = hipMemset(p->g[b], 0, K * np * 4);
        if (e == hipSuccess) e = hipMemset(p->gq[b], 0, K * np * 4);
        if (e == hipSuccess && p->h[b]) e = hipMemset(p->h[b], 0, K * np * 4);
        if (e == hipSuccess) e = hipMemset(p->bins[b], 0, np * F);
    }
    if (e == hipSuccess) e = hipMemcpy(p->seg, segv.data(), F * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->zl, 0, half * 4);
    if (e != hipSuccess) {
        free_part(p);
        delete p;
        set_error("partition set-up failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    *out = p;
    return CBH_OK;
}

void cbh_part_destroy(cbh_part* part) {
    if (!part) return;
    (void)hipDeviceSynchronize();
    free_part(part);
    delete part;
}

int cbh_part_split(cbh_ctx* ctx, cbh_part* part, const cbh_problem* prob, int32_t level,
                   int32_t precision, const cbh_split* split, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr && split != nullptr, "NULL argument");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    rc = check_part(part, prob);
    if (rc) return rc;
    CBH_ARG(level >= 0 && level < prob->depth, "level %d outside [0, depth)", level);
    hipStream_t s = (hipStream_t)stream;
    const int src = (level + 1) & 1, dst = level & 1;   // level l reads (l-1) % 2, writes l % 2
    const bool first = level == 0;
    const uint8_t* const* scols = first ? prob->bins : part->cols[src];
    const int64_t* sseg = first ? prob->seg_stride : part->seg;
    const int32_t* sorder = first ? nullptr : part->order[src];
    const uint16_t* scode = first ? nullptr : part->code[src];
    const int F = part->F;
    if (level == prob->depth - 1) {
        const unsigned grid =
            (unsigned)std::min<int64_t>((part->n + 255) / 256, int64_t(ctx->num_cus) * 16);
        part_leaf_kernel<<<grid, 256, 0, s>>>(scols, sseg, F, split, part->n, level, sorder, scode,
                                              prob->leaf);
        CBH_LAUNCHED();
        return CBH_OK;
    }
    const int32_t L = 1 << level;
    const size_t cnt_lds = L <= kPartLdsLeaves ? size_t(L) * 4 : 0;
    part_count_kernel<<<(unsigned)part->n_pb, kPartThreads, cnt_lds, s>>>(
        scols, sseg, F, split, part->n, scode, L, part->zl, part->blk);
    CBH_LAUNCHED();
    part_scan_kernel<<<1, 1024, 0, s>>>(part->blk, part->n_pb, part->zl, L,
                                         first ? nullptr : part->off[src], part->n, part->off[dst]);
    CBH_LAUNCHED();
    PartMove m;
    m.src_cols = scols;
    m.src_seg = sseg;
    m.dst_bins = part->bins[dst];
    m.F = F;
    m.K = part->K;
    m.level = level;
    m.split = split;
    m.n = part->n;
    m.n_pad = part->n_pad;
    m.n_pb = part->n_pb;
    m.blk = part->blk;
    m.src_order = sorder;
    m.dst_order = part->order[dst];
    m.src_code = scode;
    m.dst_code = part->code[dst];
    const bool q = precision == CBH_PREC_INT16;
    const bool rm = count_stat(prob);
    m.src_g = q ? nullptr : (first ? prob->g : part->g[src]);
    m.src_h = (q || rm) ? nullptr : (first ? prob->h : part->h[src]);
    m.src_gq = q ? (first ? reinterpret_cast<const uint32_t*>(prob->gq) : part->gq[src]) : nullptr;
    m.src_stride = first ? prob->n : part->n_pad;
    m.dst_g = q ? nullptr : part->g[dst];
    m.dst_h = (q || rm) ? nullptr : part->h[dst];
    m.dst_gq = q ? part->gq[dst] : nullptr;
    part_scatter_kernel<<<(unsigned)part->n_pb, kPartThreads, 0, s>>>(m);
    CBH_LAUNCHED();
    return CBH_OK;
}

static int part_build(cbh_ctx* ctx, cbh_part* part, const cbh_problem* prob, int32_t level,
                      int32_t precision, const void* parent_hist, void* hist_out,
                      void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr && hist_out != nullptr, "NULL argument");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    rc = check_part(part, prob);
    if (rc) return rc;
    CBH_ARG(level >= 1 && level < prob->depth, "level %d outside [1, depth)", level);
    const bool sub = parent_hist != nullptr;
    CBH_ARG(parent_hist != hist_out, "parent_hist must not be hist_out");
    hipStream_t s = (hipStream_t)stream;
    const int src = (level + 1) & 1;   // written by the split of level - 1
    const int L = 1 << level;
    const int F = part->F, B = prob->max_bins, K = part->K;
    const int rmse = count_stat(prob);
    const HistKnobs kn = knobs_for(ctx, F, B, K, level, precision, prob->n, sub ? 3 : 2);
    const HistPlan plan = plan_part(kn, prob->n, F, B, K, L, precision, ctx->max_lds, sub);
    const int64_t spc = std::max<int64_t>(1, plan.rows_per_chunk / 16);
    const int64_t n_tiles = plan.n_ltiles;
    const int64_t max_chunks = (part->n_pad / 16 + n_tiles + spc - 1) / spc + n_tiles + 1;
    const int64_t cell_words = int64_t(plan.lt) * F * B * plan.words_per_cell;
    rc = ensure_ws(ctx, max_chunks * cell_words * 4, stream);
    if (rc) return rc;
    part_tiles_kernel<<<1, 1024, 0, s>>>(part->off[src], L, plan.lt, (int32_t)n_tiles, spc,
                                          part->cp, part->tord, sub ? part->tleaf : nullptr);
    CBH_LAUNCHED();
    PartHist a;
    const bool q = precision == CBH_PREC_INT16;
    a.cols = part->cols[src];
    a.seg = part->seg;
    a.g = part->g[src];
    a.h = part->h[src];
    a.gq = q ? part->gq[src] : nullptr;
    a.code = part->code[src];
    a.off = part->off[src];
    a.cp = part->cp;
    a.tord = part->tord;
    a.tleaf = sub ? part->tleaf : nullptr;
    a.partials = (uint32_t*)ctx->ws;
    a.n_pad = part->n_pad;
    a.n_items = max_chunks * plan.n_fgroups * K;
    a.segs_per_chunk = spc;
    a.F = F;
    a.B = B;
    a.K = K;
    a.L = L;
    a.lt = plan.lt;
    a.n_tiles = (int32_t)n_tiles;
    a.n_fgroups = plan.n_fgroups;
    a.wpc = plan.words_per_cell;
    const unsigned grid = (unsigned)(8 * ((max_chunks + 7) / 8) * plan.n_fgroups * K);
    const size_t lds = (size_t)plan.lds_bytes;
    switch (precision) {
        case CBH_PREC_FP32:
            if (rmse) launch_part_hist<CBH_PREC_FP32, 1>(a, plan.fb, grid, lds, s);
            else launch_part_hist<CBH_PREC_FP32, 0>(a, plan.fb, grid, lds, s);
            break;
        case CBH_PREC_TWOFLOAT:
            if (rmse) launch_part_hist<CBH_PREC_TWOFLOAT, 1>(a, plan.fb, grid, lds, s);
            else launch_part_hist<CBH_PREC_TWOFLOAT, 0>(a, plan.fb, grid, lds, s);
            break;
        case CBH_PREC_F64:
            if (rmse) launch_part_hist<CBH_PREC_F64, 1>(a, plan.fb, grid, lds, s);
            else launch_part_hist<CBH_PREC_F64, 0>(a, plan.fb, grid, lds, s);
            break;
        default:
            launch_part_hist<CBH_PREC_INT16, 0>(a, plan.fb, grid, lds, s);
            break;
    }
    CBH_LAUNCHED();
    // merge units: every leaf, or (subtraction) every parent, which writes both children
    const int Lm = sub ? L / 2 : L;
    const int64_t units = int64_t(Lm) * F * B * K;
    const unsigned mg =
        (unsigned)std::min<int64_t>((units + 255) / 256, int64_t(ctx->num_cus) * 16);
    const int32_t* tl = sub ? part->tleaf : nullptr;
    switch (out_prec(precision)) {
        case CBH_PREC_FP32:
            part_merge_kernel<CBH_PREC_FP32><<<mg, 256, 0, s>>>(
                (const uint32_t*)ctx->ws, part->cp, part->tord + n_tiles, Lm, plan.lt, F, B, K,
                plan.words_per_cell,
                rmse, hist_out, tl, parent_hist);
            break;
        case CBH_PREC_TWOFLOAT:
            part_merge_kernel<CBH_PREC_TWOFLOAT><<<mg, 256, 0, s>>>(
                (const uint32_t*)ctx->ws, part->cp, part->tord + n_tiles, Lm, plan.lt, F, B, K,
                plan.words_per_cell,
                rmse, hist_out, tl, parent_hist);
            break;
        default:
            part_merge_kernel<CBH_PREC_INT16><<<mg, 256, 0, s>>>(
                (const uint32_t*)ctx->ws, part->cp, part->tord + n_tiles, Lm, plan.lt, F, B, K,
                plan.words_per_cell,
                rmse, hist_out, tl, parent_hist);
            break;
    }
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_part_build_histograms(cbh_ctx* ctx, cbh_part* part, const cbh_problem* prob,
                              int32_t level, int32_t precision, void* hist_out, void* stream) {
    return part_build(ctx, part, prob, level, precision, nullptr, hist_out, stream);
}

int cbh_part_build_histograms_sub(cbh_ctx* ctx, cbh_part* part, const cbh_problem* prob,
                                  int32_t level, int32_t precision, const void* parent_hist,
                                  void* hist_out, void* stream) {
    if (!parent_hist) {
        clear_error();
        set_error("parent_hist is NULL");
        return CBH_EINVAL;
    }
    return part_build(ctx, part, prob, level, precision, parent_hist, hist_out, stream);
}

}  // extern "C"
