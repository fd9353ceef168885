// Output-key work items (SEG_BKT): the sparse product's merge-and-sort step
// as one scatter pass and one in-LDS sort per work item.  Included by
// pm_kernels.hip.
//
// The result of Section 2 (every term pair (i, j) of the pp-matrix of Fig. 1
// contributes a_i b_j to the monomial alpha_i + beta_j; equal monomials are
// summed, zero sums dropped, the result sorted ascending) is produced in four
// steps.  Like Algorithm 1, the output-key space is cut into intervals whose
// pair counts are balanced and each interval is merged by one worker
// independently; the intervals here come from an exact count instead of the
// grid sample of Section 5, and the merge is an LDS radix sort instead of a
// heap or tree.
//   k_bk_count    every pair of a generation tile (rows x columns of the
//                 pp-matrix) adds one to the fine bin of its compressed key;
//                 a tile's pairs fall into few bins (rows and columns are
//                 sorted), so bins are first aggregated in an LDS table
//   k_bk_cut      per super-bin of BK_SB fine bins: greedy cut of the bins
//                 into work items of at most BK_CAP pairs (pointer doubling
//                 over the greedy successor of every bin)
//   k_bk_scan     work-item (ticket) and staging offsets of every super-bin
//   k_bk_winfo    work-item descriptors
//   k_bk_scatter  every pair of a tile goes to its work item's staging range;
//                 a tile touches few work items, so its items are claimed per
//                 (tile, work item) and written as long contiguous runs
//   k_bk_reduce   per work item: like-term sums in a direct LDS accumulator
//                 (exact rings, narrow key ranges) or after an LDS radix sort
//                 by key (FP64: by key, then row, so equal monomials sum in
//                 row-major order), zero removal; result terms to staging
//   k_bk_oscan    result offsets (prefix of the work items' term counts)
//   k_bk_copy     result terms to h, keys decompressed
#pragma once

namespace pm {

constexpr int BK_T = 256;            // threads of the tile kernels
constexpr int BK_H1 = 2048;          // LDS table slots of the bin count
constexpr int BK_H3 = 1024;          // LDS table slots of the scatter
constexpr u32 BK_EMPTY = 0xFFFFFFFFu;
constexpr int BC_T = 1024;           // threads of the cut kernels (4 bins each)
constexpr int BC_LV = 6;             // greedy steps 1, 2, 4, ..., 2^BC_LV kept per bin
constexpr int BR_T = 1024;           // threads of the work-item kernel
constexpr int BR_IPT = BK_CAP / BR_T;
constexpr int BR_NW = BR_T / 64;
static_assert(BR_T * BR_IPT == BK_CAP, "work-item capacity");
static_assert(BC_T * 4 == BK_SB, "cut kernel covers one super-bin");

// Generation tile t of the launch: rows [i0, i0+rm) x columns [j0, j0+cn) of
// product q, laid out as rm rows of 2^tnl slots (slots past cn are empty).
struct BkTile {
    const u32 *kf, *kg;
    i64 bin_off, sb_first;
    u32 i0, j0, rm, cn, tnl, fs, nb;
    i32 q;
};

// The tile fields of one product, kept while a workgroup's consecutive tiles
// belong to it (the product search and descriptor loads then happen once per
// product instead of once per tile).
struct BkProd {
    i64 t_lo = 0, t_hi = 0;  // the product's tiles [t_lo, t_hi) of the launch
    BkTile base;             // every field but i0, j0, rm, cn
    u32 tiles_n = 1, na = 0;
};

__device__ inline BkTile bk_tile(const Ctx &C, i64 t, BkProd &P) {
    if (t < P.t_lo || t >= P.t_hi) {
        const int bq = seg_search(C.bk_tile_pre, C.nbk, t);
        const int q = C.bk_seg[bq];
        const DevSeg &s = C.segs[q];
        P.t_lo = C.bk_tile_pre[bq];
        P.t_hi = C.bk_tile_pre[bq + 1];
        const u32 *ck = (const u32 *)C.ck;
        BkTile &B = P.base;
        B.kf = ck + s.ck_f;
        B.kg = ck + s.ck_g;
        B.bin_off = s.bk_bin_off;
        B.sb_first = s.bk_sb_first;
        B.tnl = (u32)s.bk_tnl;
        B.fs = (u32)s.bk_fs;
        B.nb = (u32)s.nb;
        B.q = q;
        P.tiles_n = (u32)s.bk_tiles_n;
        P.na = (u32)s.na;
    }
    BkTile T = P.base;
    const u32 tm = (u32)BK_TILE >> T.tnl, tn = 1u << T.tnl;
    const u32 lt = (u32)(t - P.t_lo);  // tiles of one product: fewer than 2^32
    const u32 tr = lt / P.tiles_n, tc = lt - tr * P.tiles_n;
    T.i0 = tr * tm;
    T.j0 = tc * tn;
    T.rm = min(tm, P.na - T.i0);
    T.cn = min(tn, T.nb - T.j0);
    return T;
}

// Slot p of the tile: pair (i0 + p / 2^tnl, j0 + p mod 2^tnl).  With at least
// 64 columns a wave's lanes hold consecutive columns of one row, so their keys
// ascend along the lanes.
__device__ inline bool bk_slot(const BkTile &T, u32 p, u32 &r, u32 &c) {
    r = p >> T.tnl;
    c = p & ((1u << T.tnl) - 1);
    return r < T.rm && c < T.cn;
}

// Runs of equal values along the lanes: lanes whose value differs from the
// lane below, and invalid lanes, start a run.  Returns the mask of run starts.
__device__ inline u64 bk_run_starts(bool valid, u32 v) {
    // the lower neighbour's value through a DPP wave shift (lane 0 keeps ~v)
    const u32 prev = (u32)__builtin_amdgcn_update_dpp((int)~v, (int)v, 0x138, 0xF, 0xF, false);
    const bool head = valid && prev != v;
    return __ballot(head) | ~__ballot(valid);
}

// Length of the run starting at this lane (a run start) given the start mask.
__device__ inline u32 bk_run_len(u64 starts) {
    const u32 lane = lane_id();
    const u64 above = lane == 63 ? 0ull : (starts & (~0ull << (lane + 1)));
    const u32 end = above ? (u32)__ffsll((unsigned long long)above) - 1 : 64u;
    return end - lane;
}

__device__ inline u32 bk_hash(u32 key, int log2n) { return (key * 2654435761u) >> (32 - log2n); }

// Adds `add` to key's slot of an LDS open-addressing table (2^log2n slots).
// Returns the slot, or -1 when 64 probes found no room.  With occ, a newly
// claimed slot is also appended to occ (its first nocc_max entries; *nocc
// counts every claim).
__device__ inline int bk_table_add(u32 *keys, u32 *cnt, int log2n, u32 key, u32 add,
                                   unsigned short *occ = nullptr, u32 *nocc = nullptr, u32 nocc_max = 0) {
    u32 h = bk_hash(key, log2n);
    const u32 m = (1u << log2n) - 1;
#pragma unroll 1
    for (int probe = 0; probe < 64; probe++) {
        const u32 old = atomicCAS(&keys[h], BK_EMPTY, key);
        if (old == BK_EMPTY || old == key) {
            atomicAdd(&cnt[h], add);
            if (occ && old == BK_EMPTY) {
                const u32 at = atomicAdd(nocc, 1u);
                if (at < nocc_max) occ[at] = (unsigned short)h;
            }
            return (int)h;
        }
        h = (h + 1) & m;
    }
    return -1;
}

// Slot of key in the table, or -1 after max_probes probes.
__device__ inline int bk_table_find(const u32 *keys, int log2n, u32 key, int max_probes = 64) {
    u32 h = bk_hash(key, log2n);
    const u32 m = (1u << log2n) - 1;
#pragma unroll 1
    for (int probe = 0; probe < max_probes; probe++) {
        if (keys[h] == key) return (int)h;
        h = (h + 1) & m;
    }
    return -1;
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

// A load through a pointer known to address global memory (a generic pointer
// taken from a descriptor otherwise becomes a flat access).
template <typename T>
__device__ inline T gload(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

// Calls f(valid, key, r, c) for every slot of the tile, a wave's 64 lanes
// together (f may use wave-wide operations).  Tiles of at least 64 columns
// keep each lane's column keys in registers and take a row's key from a
// register of the lane that loaded it, so the loop does no memory access;
// narrower tiles walk the slots in order.
template <typename F>
__device__ inline void bk_tile_pairs(const BkTile &T, F &&f) {
    const u32 lane = lane_id();
    if (T.tnl >= 6) {
        const u32 w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const u32 nm = 1u << (T.tnl - 6);  // 64-column chunks, at most 4
        u32 b[BK_TN_MAX / 64];
#pragma unroll
        for (u32 m = 0; m < BK_TN_MAX / 64; m++) {
            const u32 c = 64 * m + lane;
            b[m] = m < nm && c < T.cn ? gload(T.kg + T.j0 + c) : 0;
        }
        for (u32 rb = 0; rb < T.rm; rb += 64) {
            const u32 areg = rb + lane < T.rm ? gload(T.kf + T.i0 + rb + lane) : 0;
            const u32 rend = min(T.rm - rb, 64u);
            for (u32 r = w; r < rend; r += BK_T / 64) {
                const u32 a = (u32)__builtin_amdgcn_readlane((int)areg, (int)r);
                // one copy of f: the chunk's column keys picked by selects
#pragma unroll 1
                for (u32 m = 0; m < nm; m++) {
                    static_assert(BK_TN_MAX / 64 == 4, "four column chunks");
                    const u32 bm = m == 0 ? b[0] : m == 1 ? b[1] : m == 2 ? b[2] : b[3];
                    const u32 c = 64 * m + lane;
                    f(c < T.cn, a + bm, rb + r, c);
                }
            }
        }
    } else {
        const u32 slots = T.rm << T.tnl;
        for (u32 p0 = 0; p0 < slots; p0 += BK_T) {
            u32 r, c;
            const bool valid = bk_slot(T, p0 + threadIdx.x, r, c);
            u32 key = 0;
            if (valid) key = gload(T.kf + T.i0 + r) + gload(T.kg + T.j0 + c);
            f(valid, key, r, c);
        }
    }
}

// ---------------------------------------------------------------------------
// k_bk_count: pair counts of the fine bins.  Work queue over generation
// tiles; a tile's bins are counted in an LDS table, added to the global
// counts, and listed for the scatter (up to BK_TL entries per tile).
// ---------------------------------------------------------------------------
constexpr int BK_TL = 512;            // bins listed per tile, at most
constexpr u32 BK_TL_NONE = 0xFFFFFFFFu;

__global__ __launch_bounds__(BK_T) void k_bk_count(Ctx C) {
    __shared__ u32 s_key[BK_H1], s_cnt[BK_H1];
    __shared__ unsigned short s_occ[BK_TL];  // slots claimed by the tile, in claim order
    __shared__ u32 s_nocc[2], s_ovf[2];      // by tile parity: reset one tile ahead
    for (int e = threadIdx.x; e < BK_H1; e += BK_T) {
        s_key[e] = BK_EMPTY;
        s_cnt[e] = 0;
    }
    if (threadIdx.x < 2) {
        s_nocc[threadIdx.x] = 0;
        s_ovf[threadIdx.x] = 0;
    }
    const u32 lane = lane_id();
    BkProd P;
    u32 par = 0;
    // tiles are equal work: a static round robin (no shared queue counter)
    for (i64 t = blockIdx.x; t < C.bk_ntiles; t += gridDim.x, par ^= 1u) {
        __syncthreads();
        const BkTile T = bk_tile(C, t, P);
        u32 *hist = C.bk_hist + T.bin_off;
        bk_tile_pairs(T, [&](bool valid, u32 key, u32, u32) {
            const u32 bin = valid ? key >> T.fs : BK_EMPTY;
            const u64 starts = bk_run_starts(valid, bin);
            if (valid && ((starts >> lane) & 1)) {
                const u32 len = bk_run_len(starts);
                if (bk_table_add(s_key, s_cnt, ilog2c(BK_H1), bin, len, s_occ, &s_nocc[par], BK_TL) < 0) {
                    atomicAdd(&hist[bin], len);
                    s_ovf[par] = 1;
                }
            }
        });
        __syncthreads();
        // global counts, and the tile's list of (bin, count) when its bins
        // fit the list (then only the claimed slots are visited)
        const u32 nocc = s_nocc[par];
        const bool listed = nocc <= (u32)BK_TL && !s_ovf[par];
        if (listed) {
            u64 *list = C.bk_tlist + t * BK_TL;
            for (u32 e = threadIdx.x; e < nocc; e += BK_T) {
                const u32 sl = s_occ[e];
                const u32 k = s_key[sl], c = s_cnt[sl];
                atomicAdd(&hist[k], c);
                list[e] = ((u64)k << 32) | c;
                s_key[sl] = BK_EMPTY;
                s_cnt[sl] = 0;
            }
        } else {
            for (int sl = threadIdx.x; sl < BK_H1; sl += BK_T) {
                const u32 k = s_key[sl];
                if (k != BK_EMPTY) {
                    atomicAdd(&hist[k], s_cnt[sl]);
                    s_key[sl] = BK_EMPTY;
                    s_cnt[sl] = 0;
                }
            }
        }
        if (threadIdx.x == 0) {
            C.bk_tcnt[t] = listed ? nocc : BK_TL_NONE;
            s_nocc[par ^ 1u] = 0;  // the next tile's counters (last read by the previous tile)
            s_ovf[par ^ 1u] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Greedy cut of one super-bin (BK_SB fine bins, four per thread) into work
// items: a work item starting at bin b takes the following bins while their
// pairs stay within BK_CAP (a bin over BK_CAP alone) and, for exact rings, at
// most bk_span_bins bins (a key span of BR_RANK_SPAN).  nxt(b) is where that
// work item ends; the work-item starts are the orbit of bin 0 under nxt.  The
// orbit is marked by pointer doubling: nxt^(2^l) for l <= BC_LV, then jumps of
// 2^(BC_LV-1), ..., 1 from every marked bin, repeated from nxt^(2^BC_LV) of the
// phase's start until the orbit leaves the super-bin.
// ---------------------------------------------------------------------------
struct BkCutLds {
    u32 pre[BK_SB + 1];
    unsigned short jmp[BC_LV + 1][BK_SB + 1];
    unsigned char on[BK_SB + 1];
    u32 scan[BC_T / 64];
    u32 start;
};

__device__ inline void bk_sb_locate(const Ctx &C, i64 gsb, int &q, i64 &lsb) {
    const int bq = seg_search(C.bk_sb_pre, C.nbk, gsb);
    q = C.bk_seg[bq];
    lsb = gsb - C.bk_sb_pre[bq];
}

__global__ __launch_bounds__(BC_T) void k_bk_cut(Ctx C) {
    __shared__ BkCutLds L;
    const i64 gsb = blockIdx.x;
    int q;
    i64 lsb;
    bk_sb_locate(C, gsb, q, lsb);
    const i64 b0 = C.segs[q].bk_bin_off + lsb * BK_SB;
    const int t = threadIdx.x;
    const uint4 hv = *(const uint4 *)(C.bk_hist + b0 + 4 * t);
    const u32 h[4] = {hv.x, hv.y, hv.z, hv.w};
    u32 tot;
    const u32 ex = block_excl_scan<u32, BC_T>(h[0] + h[1] + h[2] + h[3], L.scan, tot);
    if (tot == 0) {
        if (t == 0) {
            C.bk_sbtot[gsb] = 0;
            C.bk_sbwi[gsb] = 0;
        }
        return;
    }
    {
        u32 run = ex;
        for (int k = 0; k < 4; k++) {
            L.pre[4 * t + k] = run;
            run += h[k];
        }
        if (t == BC_T - 1) L.pre[BK_SB] = tot;
    }
    __syncthreads();
    const int span_bins = C.segs[q].bk_span_bins;
    for (int k = 0; k < 4; k++) {
        const int b = 4 * t + k;
        const u32 lim = L.pre[b] + (u32)BK_CAP;  // pairs < 2^32 per product
        int e = b + 1;
        if (L.pre[e] <= lim && lim >= L.pre[b]) {
            int lo = e, hi = BK_SB;  // largest e in [lo, hi] with pre[e] <= lim
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.pre[mid] <= lim) lo = mid;
                else hi = mid - 1;
            }
            e = lo;
        }
        if (span_bins > 0 && e > b + span_bins) e = b + span_bins;
        L.jmp[0][b] = (unsigned short)e;
        L.on[b] = 0;
    }
    if (t == 0) {
        L.jmp[0][BK_SB] = BK_SB;
        L.on[BK_SB] = 0;
    }
    __syncthreads();
    for (int l = 1; l <= BC_LV; l++) {
        for (int k = 0; k < 4; k++) {
            const int b = 4 * t + k;
            L.jmp[l][b] = L.jmp[l - 1][L.jmp[l - 1][b]];
        }
        if (t == 0) L.jmp[l][BK_SB] = BK_SB;
        __syncthreads();
    }
    if (t == 0) {
        L.on[0] = 1;
        L.start = 0;
    }
    __syncthreads();
    while (true) {
        for (int l = BC_LV - 1; l >= 0; l--) {
            for (int k = 0; k < 4; k++) {
                const int b = 4 * t + k;
                if (L.on[b]) L.on[L.jmp[l][b]] = 1;
            }
            __syncthreads();
        }
        const u32 s = L.start;
        const u32 nx = L.jmp[BC_LV][s];
        __syncthreads();
        if (nx >= (u32)BK_SB) break;
        if (t == 0) {
            L.on[nx] = 1;
            L.start = nx;
        }
        __syncthreads();
    }
    u32 f[4], nf = 0;
    for (int k = 0; k < 4; k++) {
        f[k] = L.on[4 * t + k];
        nf += f[k];
    }
    u32 nwi;
    u32 wi = block_excl_scan<u32, BC_T>(nf, L.scan, nwi);
    unsigned short wb[4];
    for (int k = 0; k < 4; k++) {
        wi += f[k];
        wb[k] = (unsigned short)(wi - 1);
    }
    uint2 o;
    o.x = (u32)wb[0] | ((u32)wb[1] << 16);
    o.y = (u32)wb[2] | ((u32)wb[3] << 16);
    *(uint2 *)(C.bk_wbin + b0 + 4 * t) = o;
    if (t == 0) {
        C.bk_sbtot[gsb] = tot;
        C.bk_sbwi[gsb] = nwi;
    }
}

// Ticket and staging offsets of every super-bin (one workgroup).
__global__ __launch_bounds__(BC_T) void k_bk_scan(Ctx C) {
    __shared__ u64 s_scan[BC_T / 64];
    u64 ct = 0, cp = 0;
    for (i64 b = 0; b < C.bk_nsb; b += BC_T) {
        const i64 i = b + threadIdx.x;
        const u64 w = i < C.bk_nsb ? C.bk_sbwi[i] : 0, p = i < C.bk_nsb ? C.bk_sbtot[i] : 0;
        u64 tw, tp;
        const u64 ew = block_excl_scan<u64, BC_T>(w, s_scan, tw);
        const u64 ep = block_excl_scan<u64, BC_T>(p, s_scan, tp);
        if (i < C.bk_nsb) {
            C.bk_sbtb[i] = (u32)(ct + ew);
            C.bk_sbpre[i] = cp + ep;
        }
        ct += tw;
        cp += tp;
    }
    if (threadIdx.x == 0) {
        if ((i64)ct > C.bk_wi_bound) {  // never planned: keep every ticket inside the work-item arrays
            atomicOr(&C.counters[CNT_ERR_SPIN], 8u);
            ct = (u64)C.bk_wi_bound;
        }
        C.bk_sbtb[C.bk_nsb] = (u32)ct;
    }
}

// Work-item descriptors: the first bin of a work item writes its start and
// staging offset, the last bin its end.
__global__ __launch_bounds__(BC_T) void k_bk_winfo(Ctx C) {
    __shared__ u32 s_scan[BC_T / 64];
    const i64 gsb = blockIdx.x;
    if (C.bk_sbwi[gsb] == 0) return;
    int q;
    i64 lsb;
    bk_sb_locate(C, gsb, q, lsb);
    const i64 b0 = C.segs[q].bk_bin_off + lsb * BK_SB;
    const int t = threadIdx.x;
    const uint4 hv = *(const uint4 *)(C.bk_hist + b0 + 4 * t);
    const u32 h[4] = {hv.x, hv.y, hv.z, hv.w};
    const uint2 wv = *(const uint2 *)(C.bk_wbin + b0 + 4 * t);
    const u32 wb[4] = {wv.x & 0xFFFF, wv.x >> 16, wv.y & 0xFFFF, wv.y >> 16};
    const u32 wprev = t > 0 ? (u32)C.bk_wbin[b0 + 4 * t - 1] : BK_EMPTY;
    const u32 wnext = t < BC_T - 1 ? (u32)C.bk_wbin[b0 + 4 * t + 4] : BK_EMPTY;
    u32 tot;
    u32 pre = block_excl_scan<u32, BC_T>(h[0] + h[1] + h[2] + h[3], s_scan, tot);
    const u32 tb = C.bk_sbtb[gsb];
    const u64 pb = C.bk_sbpre[gsb];
    for (int k = 0; k < 4; k++) {
        const u32 b = 4 * t + k;
        const u32 before = k ? wb[k - 1] : wprev;
        const u32 after = k < 3 ? wb[k + 1] : wnext;
        if ((i64)(tb + wb[k]) >= C.bk_wi_bound) break;
        BkWi &w = C.bk_wi[tb + wb[k]];
        const u32 tk = tb + wb[k];
        if (before != wb[k]) {
            w.bin_lo = (u32)(lsb * BK_SB + b);
            w.off = pb + pre;
            w.q = q;
            w.first = tk == C.bk_sbtb[C.segs[q].bk_sb_first];
        }
        pre += h[k];
        if (after != wb[k]) {
            w.bin_hi = (u32)(lsb * BK_SB + b + 1);
            w.end = pb + pre;
            w.last = tk + 1 == C.bk_sbtb[C.segs[q].bk_sb_first + C.segs[q].bk_nsb];
        }
    }
}

// ---------------------------------------------------------------------------
// k_bk_scatter: every pair to its work item.  A tile listed by the count
// knows its bins: each bin's work item is looked up once, the tile's pairs of
// one work item claim one contiguous range of the work item's staging, each
// bin gets its place inside that range, and one pass over the pairs writes
// each run of lanes to consecutive slots of its bin's place.  An unlisted
// tile (more bins than the list holds) counts its pairs per work item in an
// LDS table first, then claims per work item (or per run when the table
// overflows) and writes in a second pass.
// ---------------------------------------------------------------------------
__device__ inline u32 bk_ticket(const Ctx &C, const BkTile &T, u32 bin) {
    const i64 gsb = T.sb_first + (bin >> BK_SB_LOG);
    const u32 tk = C.bk_sbtb[gsb] + (u32)C.bk_wbin[T.bin_off + bin];
    return (i64)tk < C.bk_wi_bound ? tk : (u32)(C.bk_wi_bound - 1);  // only after a flagged error
}

// Writes item (key, pair index) of lane runs that share `cls`: a run start
// claims len slots from claim(cls, len) and every lane of the run writes to
// its slot.  Whole wave.
template <typename Claim>
__device__ inline void bk_write_runs(const Ctx &C, const BkTile &T, bool ok, u32 cls, u32 key, u32 r, u32 c,
                                     Claim &&claim) {
    const u32 lane = lane_id();
    const u64 starts = bk_run_starts(ok, cls);
    const bool head = ok && ((starts >> lane) & 1);
    u64 pos = 0;
    if (head) pos = claim(cls, bk_run_len(starts));
    const u64 below = starts & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    const u32 src = 63 - (u32)__clzll((long long)below);
    const u32 plo = __shfl((u32)pos, src, 64), phi = __shfl((u32)(pos >> 32), src, 64);
    if (ok) {
        const u64 at = (((u64)phi << 32) | plo) + (lane - src);
        const u32 x = (T.i0 + r) * T.nb + (T.j0 + c);
        if (at < (u64)C.bk_nstage) C.bk_stage[at] = ((u64)x << 32) | key;
        else atomicOr(&C.counters[CNT_ERR_SPIN], 8u);
    }
}

__global__ __launch_bounds__(BK_T) void k_bk_scatter(Ctx C) {
    constexpr int HB = 2 * BK_TL;   // bin table of a listed tile
    __shared__ u32 s_key[BK_H3], s_cnt[BK_H3];   // work-item table
    __shared__ u64 s_cur[BK_H3];
    __shared__ u32 s_bkey[HB];
    __shared__ u64 s_bcur[HB];
    __shared__ unsigned short s_wocc[BK_TL];  // work-item slots claimed by a listed tile
    __shared__ u32 s_nw;
    __shared__ u32 s_ovf;
    for (int e = threadIdx.x; e < BK_H3; e += BK_T) {
        s_key[e] = BK_EMPTY;
        s_cnt[e] = 0;
    }
    for (int e = threadIdx.x; e < HB; e += BK_T) s_bkey[e] = BK_EMPTY;
    if (threadIdx.x == 0) {
        s_ovf = 0;
        s_nw = 0;
    }
    const u32 lane = lane_id();
    BkProd P;
    for (i64 t = blockIdx.x; t < C.bk_ntiles; t += gridDim.x) {
        __syncthreads();
        const BkTile T = bk_tile(C, t, P);
        const u32 nl = C.bk_tcnt[t];
        if (nl != BK_TL_NONE) {
            // the tile's bins: work item, place inside the tile's piece of it
            const u64 *list = C.bk_tlist + t * BK_TL;
            u32 bslot = 0, tslot = 0, boff = 0;
            const bool mine = threadIdx.x < nl;  // nl <= BK_TL = 2 * BK_T: two bins per thread at most
            const bool mine2 = threadIdx.x + BK_T < nl;
            u32 bslot2 = 0, tslot2 = 0, boff2 = 0;
            if (mine) {
                const u64 ent = list[threadIdx.x];
                const u32 bin = (u32)(ent >> 32), cnt = (u32)ent;
                u32 h = bk_hash(bin, ilog2c(HB));
                while (atomicCAS(&s_bkey[h], BK_EMPTY, bin) != BK_EMPTY) h = (h + 1) & (HB - 1);
                bslot = h;
                const u32 tk = bk_ticket(C, T, bin);
                u32 g = bk_hash(tk, ilog2c(BK_H3));
                while (true) {
                    const u32 old = atomicCAS(&s_key[g], BK_EMPTY, tk);
                    if (old == BK_EMPTY) s_wocc[atomicAdd(&s_nw, 1u)] = (unsigned short)g;
                    if (old == BK_EMPTY || old == tk) break;
                    g = (g + 1) & (BK_H3 - 1);
                }
                tslot = g;
                boff = atomicAdd(&s_cnt[g], cnt);
            }
            if (mine2) {
                const u64 ent = list[threadIdx.x + BK_T];
                const u32 bin = (u32)(ent >> 32), cnt = (u32)ent;
                u32 h = bk_hash(bin, ilog2c(HB));
                while (atomicCAS(&s_bkey[h], BK_EMPTY, bin) != BK_EMPTY) h = (h + 1) & (HB - 1);
                bslot2 = h;
                const u32 tk = bk_ticket(C, T, bin);
                u32 g = bk_hash(tk, ilog2c(BK_H3));
                while (true) {
                    const u32 old = atomicCAS(&s_key[g], BK_EMPTY, tk);
                    if (old == BK_EMPTY) s_wocc[atomicAdd(&s_nw, 1u)] = (unsigned short)g;
                    if (old == BK_EMPTY || old == tk) break;
                    g = (g + 1) & (BK_H3 - 1);
                }
                tslot2 = g;
                boff2 = atomicAdd(&s_cnt[g], cnt);
            }
            __syncthreads();
            // one claim per work item of the tile (at most nl <= BK_TL of them)
            const u32 nw = s_nw;
            for (u32 e = threadIdx.x; e < nw; e += BK_T) {
                const u32 g = s_wocc[e];
                const u32 k = s_key[g];
                s_cur[g] = C.bk_wi[k].off + atomicAdd(&C.bk_fill[k], s_cnt[g]);
            }
            __syncthreads();
            if (mine) s_bcur[bslot] = s_cur[tslot] + boff;
            if (mine2) s_bcur[bslot2] = s_cur[tslot2] + boff2;
            __syncthreads();
            bk_tile_pairs(T, [&](bool valid, u32 key, u32 r, u32 c) {
                const u32 bin = valid ? key >> T.fs : BK_EMPTY;
                bk_write_runs(C, T, valid, bin, key, r, c, [&](u32 b, u32 len) -> u64 {
                    // every bin of the tile was inserted (inserts probe without
                    // limit, so a find may need up to HB probes)
                    const int e = bk_table_find(s_bkey, ilog2c(HB), b, HB);
                    if (e < 0) return (u64)C.bk_nstage;  // never planned: flagged, nothing written
                    return atomicAdd((unsigned long long *)&s_bcur[e], (unsigned long long)len);
                });
            });
            __syncthreads();
            // clear what the tile claimed
            if (mine) s_bkey[bslot] = BK_EMPTY;
            if (mine2) s_bkey[bslot2] = BK_EMPTY;
            for (u32 e = threadIdx.x; e < nw; e += BK_T) {
                const u32 g = s_wocc[e];
                s_key[g] = BK_EMPTY;
                s_cnt[g] = 0;
            }
            if (threadIdx.x == 0) s_nw = 0;  // read by every thread before the last barrier
        } else {
            // count per work item, claim, then write
            bk_tile_pairs(T, [&](bool valid, u32 key, u32, u32) {
                u32 tk = valid ? bk_ticket(C, T, key >> T.fs) : BK_EMPTY;
                if (valid && (i64)tk >= C.bk_wi_bound) tk = BK_EMPTY;
                const bool ok = valid && tk != BK_EMPTY;
                const u64 starts = bk_run_starts(ok, tk);
                if (ok && ((starts >> lane) & 1)) {
                    if (bk_table_add(s_key, s_cnt, ilog2c(BK_H3), tk, bk_run_len(starts)) < 0) s_ovf = 1;
                }
            });
            __syncthreads();
            const bool ovf = s_ovf != 0;
            if (!ovf) {
                for (int e = threadIdx.x; e < BK_H3; e += BK_T) {
                    const u32 k = s_key[e];
                    if (k != BK_EMPTY) s_cur[e] = C.bk_wi[k].off + atomicAdd(&C.bk_fill[k], s_cnt[e]);
                }
            }
            __syncthreads();
            bk_tile_pairs(T, [&](bool valid, u32 key, u32 r, u32 c) {
                u32 tk = valid ? bk_ticket(C, T, key >> T.fs) : BK_EMPTY;
                const bool ok = valid && (i64)tk < C.bk_wi_bound;
                bk_write_runs(C, T, ok, tk, key, r, c, [&](u32 k, u32 len) -> u64 {
                    const int e = ovf ? -1 : bk_table_find(s_key, ilog2c(BK_H3), k);
                    if (e >= 0) return atomicAdd((unsigned long long *)&s_cur[e], (unsigned long long)len);
                    return C.bk_wi[k].off + atomicAdd(&C.bk_fill[k], len);
                });
            });
            __syncthreads();
            for (int e = threadIdx.x; e < BK_H3; e += BK_T) {
                s_key[e] = BK_EMPTY;
                s_cnt[e] = 0;
            }
            if (threadIdx.x == 0) s_ovf = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// k_bk_reduce: one work item at a time (work queue in key order).
// ---------------------------------------------------------------------------
// Thread coordinates taken through an opaque copy of the thread index once per
// work item: index and shuffle-address arithmetic then stays inside the loop
// instead of being held in registers for the whole kernel.
struct Thr {
    u32 tid, lane, w;
};
__device__ inline Thr br_thr() {
    u32 t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return Thr{t, t & 63u, t >> 6};
}
__device__ inline u32 shfl_o(u32 v, u32 src) { return (u32)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v); }
__device__ inline u64 shfl_o64(u64 v, u32 src) {
    return ((u64)shfl_o((u32)(v >> 32), src) << 32) | shfl_o((u32)v, src);
}
__device__ inline u64 wave_sum_o(u64 v, u32 lane) {
#pragma unroll
    for (u32 d = 32; d >= 1; d >>= 1) v += shfl_o64(v, lane ^ d);
    return v;
}
// Exclusive scan over the BR_T threads; scratch holds BR_NW entries.  Two
// barriers; every thread calls it.
__device__ inline u32 br_excl_scan(u32 v, u32 *scratch, u32 &total, const Thr &h) {
    u32 x = v;
#pragma unroll
    for (u32 d = 1; d < 64; d <<= 1) {
        const u32 y = shfl_o(x, h.lane >= d ? h.lane - d : h.lane);
        if (h.lane >= d) x += y;
    }
    if (h.lane == 63) scratch[h.w] = x;
    __syncthreads();
    u32 pre = 0, tot = 0;
#pragma unroll
    for (u32 i = 0; i < (u32)BR_NW; i++) {
        const u32 sv = scratch[i];
        if (i < h.w) pre += sv;
        tot += sv;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// LDS of the work-item kernel (one 64 KB region M, reused by phase):
//   direct accumulation (exact rings, key span <= BK_DIRECT): acc[BK_DIRECT]
//     u64 cells indexed by local key; cell order is key order, so no sort
//   LSD sort: local keys (and, for FP64, rows) by load position, a 16-bit
//     permutation and per-wave digit counters; after the sort the products
//     a_i b_j (held in registers until then) overlay the keys (cval)
//   rounds of a work item over BK_CAP pairs: the round's items (key, pair
//     index) are staged through stk / stx
//   ranked accumulation (exact rings, key span <= BR_RANK_SPAN): a presence
//     bitmap over the span gives every present key its rank among the
//     present keys (prefix of per-word popcounts); acc[rank] accumulates and
//     rkey[rank] holds the key, so cell order is again key order
template <bool F64>
struct BrLds {
    static constexpr int LK = 0, IK = 32 << 10;
    static constexpr int PERM = F64 ? (64 << 10) : (32 << 10);
    static constexpr int CNT = PERM + (16 << 10);               // [BR_NW][256] u32
    static constexpr int LKS = CNT + BR_NW * 256 * 4;           // FP64: sorted keys
    static constexpr int RKEY = 64 << 10;                       // exact rings: u32[BK_CAP]
    static constexpr int BM = RKEY + (32 << 10);                // u64[BR_RANK_SPAN / 64]
    static constexpr int PRE = BM + (32 << 10);                 // u16[BR_RANK_SPAN / 64]
    static constexpr int BYTES = F64 ? LKS + (32 << 10) : PRE + (8 << 10);
    static_assert(F64 || CNT + BR_NW * 256 * 4 <= (64 << 10), "exact-ring sort arrays fit under the products");
};
constexpr int BK_DIRECT = 8192;  // cells of the direct accumulator (64 KB)
constexpr u32 BR_RANK_SPAN = 1u << BK_RANK_LOG;  // key span of the presence bitmap (32 KB)
static_assert(BK_DIRECT == BR_T * BR_IPT, "each thread owns BR_IPT accumulator cells");
static_assert(BR_RANK_SPAN / 64 == BR_T * 4, "each thread scans four bitmap words");

template <int RING>
struct BrCtx {
    static constexpr bool F64 = RING == RING_F64;
    unsigned char *mem;
    __device__ u32 *lk() { return (u32 *)(mem + BrLds<F64>::LK); }
    __device__ u32 *ik() { return (u32 *)(mem + BrLds<F64>::IK); }
    __device__ unsigned short *perm() { return (unsigned short *)(mem + BrLds<F64>::PERM); }
    __device__ u32 *cnt() { return (u32 *)(mem + BrLds<F64>::CNT); }
    __device__ u32 *lks() { return (u32 *)(mem + BrLds<F64>::LKS); }
    __device__ u64 *cval() { return (u64 *)mem; }
    __device__ u64 *acc() { return (u64 *)mem; }
    __device__ u32 *stk() { return (u32 *)mem; }
    __device__ u32 *stx() { return (u32 *)(mem + (32 << 10)); }
    __device__ u32 *rkey() { return (u32 *)(mem + BrLds<F64>::RKEY); }
    __device__ u64 *bm() { return (u64 *)(mem + BrLds<F64>::BM); }
    __device__ unsigned short *pre() { return (unsigned short *)(mem + BrLds<F64>::PRE); }
};

// Sequence position of register slot k in the striped layout.
__device__ inline u32 br_seq(u32 k, const Thr &h) { return h.w * (BR_IPT * 64) + k * 64 + h.lane; }

// Register slot k's load position, two 16-bit positions per register.
struct BrPerm {
    u32 w[BR_IPT / 2];
    __device__ u32 get(int k) const { return (w[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu; }
    __device__ void set(int k, u32 v) {
        const u32 sh = (k & 1) * 16;
        w[k >> 1] = (w[k >> 1] & ~(0xFFFFu << sh)) | (v << sh);
    }
};

// One stable LSD pass over digit [sh, sh+width) of src[] (indexed by load
// position).  pv.get(k): load position of the item at sequence position
// br_seq(k); items at sequence positions >= m are padding and take the
// largest digit, so they stay behind the m real items.  On return pv holds
// the new order, striped, or blocked (thread t: positions t*BR_IPT + k).
// Ranks among a wave's items of the same digit come from one ballot per digit
// bit: the lanes agreeing with this lane on every bit are its peers.
template <int RING>
__device__ inline void br_pass(BrCtx<RING> &B, BrPerm &pv, const u32 *src, u32 sh, u32 width, u32 m, bool blocked,
                               u32 *s_scan, const Thr &h) {
    const u32 lane = h.lane, w = h.w;
    const u32 mask = (1u << width) - 1, nd = 1u << width;
    u32 *cnt = B.cnt();
    for (u32 e = h.tid; e < BR_NW * 256; e += BR_T) cnt[e] = 0;
    __syncthreads();
    u32 rd[BR_IPT];  // rank among the wave's items of the same digit | digit << 16
    const u64 below = (1ull << lane) - 1;
#pragma unroll
    for (int k = 0; k < BR_IPT; k++) {
        const u32 seq = br_seq(k, h);
        const u32 d = seq < m ? (src[pv.get(k)] >> sh) & mask : mask;
        u64 peers = ~0ull;
        for (u32 b = 0; b < width; b++) {
            const u64 bal = __ballot((d >> b) & 1);
            const u32 mb = 0u - ((d >> b) & 1u);           // all ones where this lane's bit is set
            const u64 agree = ~(bal ^ (((u64)mb << 32) | mb));
            peers &= agree;
        }
        u32 *cell = cnt + w * 256 + d;
        const u32 c0 = *cell;
        const u32 r = (u32)__popcll(peers & below);
        if (r == 0) *cell = c0 + (u32)__popcll(peers);
        rd[k] = (c0 + r) | (d << 16);
    }
    __syncthreads();
    // digit-major, wave-minor offsets
    {
        const u32 d = h.tid;
        u32 col = 0;
        if (d < nd) {
            for (u32 ww = 0; ww < BR_NW; ww++) {
                const u32 v = cnt[ww * 256 + d];
                cnt[ww * 256 + d] = col;
                col += v;
            }
        }
        u32 tot;
        const u32 base = br_excl_scan(d < nd ? col : 0, s_scan, tot, h);
        if (d < nd)
            for (u32 ww = 0; ww < BR_NW; ww++) cnt[ww * 256 + d] += base;
    }
    __syncthreads();
    unsigned short *perm = B.perm();
#pragma unroll
    for (int k = 0; k < BR_IPT; k++) perm[cnt[w * 256 + (rd[k] >> 16)] + (rd[k] & 0xFFFFu)] = (unsigned short)pv.get(k);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BR_IPT; k++) pv.set(k, perm[blocked ? h.tid * BR_IPT + k : br_seq(k, h)]);
    __syncthreads();
}

__device__ inline u32 bitlen64(u64 x) { return x ? 64 - (u32)__clzll((long long)x) : 0; }

// Exact rings: segmented inclusive scan operator on (run started, sum).
template <int RING>
__device__ inline void seg_combine(u32 &f, u64 &v, u32 f2, u64 v2) {
    v = f2 ? v2 : ring_add<RING>(v, v2);
    f |= f2;
}

// Exclusive segmented scan over the workgroup: (flag, value) of the threads
// before this one, combined left to right.
template <int RING>
__device__ inline u64 br_seg_scan(u32 flag, u64 val, u32 *s_f, u64 *s_v, const Thr &h) {
    const u32 lane = h.lane, w = h.w;
    u32 f = flag;
    u64 v = val;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const u32 src = lane >= (u32)d ? lane - d : lane;
        const u32 fu = shfl_o(f, src);
        const u64 vu = shfl_o64(v, src);
        if (lane >= (u32)d) {
            u32 ff = fu;
            u64 vv = vu;
            seg_combine<RING>(ff, vv, f, v);
            f = ff;
            v = vv;
        }
    }
    if (lane == 63) {
        s_f[w] = f;
        s_v[w] = v;
    }
    u32 fe = shfl_o(f, lane ? lane - 1 : 0);
    u64 ve = shfl_o64(v, lane ? lane - 1 : 0);
    if (lane == 0) {
        fe = 0;
        ve = 0;
    }
    __syncthreads();
    u32 cf = 0;
    u64 cv = 0;
    for (u32 ww = 0; ww < w; ww++) seg_combine<RING>(cf, cv, s_f[ww], s_v[ww]);
    seg_combine<RING>(cf, cv, fe, ve);
    __syncthreads();
    return cv;
}

// k_bk_reduce: work items from a queue in key order.  A work item of at most
// BK_CAP pairs is loaded once: each pair's product a_i b_j is formed from its
// index (operand gathers in staging order, where neighbouring items share rows
// and nearby columns), then its like terms are summed either in a direct LDS
// accumulator (exact rings, key span <= BK_DIRECT) or after a stable LDS
// radix sort.  Its result terms (compressed key, coefficient) go to the
// work item's own staging range and its count to bk_u; k_bk_oscan and
// k_bk_copy place them.  A work item over BK_CAP pairs (one fine bin holding
// that many) is processed in rounds of key sub-ranges chosen from histograms;
// it takes its result offset from a look-back over the product's earlier work
// items, which publish their counts as soon as they are known, and writes its
// result terms directly.
// The fields of one product that the work-item kernel uses, in scalar
// registers (a descriptor read with vector loads would be re-read per item,
// since the kernel also writes global memory).
struct BrSeg {
    const u64 *fc, *gc;
    u64 *hk, *hc;
    i64 na, cap, var_off, sb_first;
    u64 lo_key;
    u32 nb, fs;
    Div32 nb_div;
};

__device__ inline BrSeg load_br_seg(const Ctx &C, int q) {
    const DevSeg &d = C.segs[q];
    BrSeg r;
    r.fc = (const u64 *)uniform64((i64)d.fc);
    r.gc = (const u64 *)uniform64((i64)d.gc);
    r.hk = (u64 *)uniform64((i64)d.hk);
    r.hc = (u64 *)uniform64((i64)d.hc);
    r.na = uniform64(d.na);
    r.cap = uniform64(d.cap);
    r.var_off = uniform64(d.var_off);
    r.sb_first = uniform64(d.bk_sb_first);
    r.lo_key = (u64)uniform64((i64)d.lo_key);
    r.nb = uniform32((u32)d.nb);
    r.fs = uniform32((u32)d.bk_fs);
    r.nb_div.m = uniform32(d.nb_div.m);
    r.nb_div.s1 = uniform32(d.nb_div.s1);
    r.nb_div.s2 = uniform32(d.nb_div.s2);
    r.nb_div.d = uniform32(d.nb_div.d);
    return r;
}

template <int RING>
__global__ __launch_bounds__(BR_T) __attribute__((amdgpu_waves_per_eu(4))) void k_bk_reduce(Ctx C) {
    constexpr bool F64 = RING == RING_F64;
    __shared__ __align__(16) unsigned char s_mem[BrLds<F64>::BYTES];
    __shared__ u32 s_scan[BR_NW];
    __shared__ u32 s_segf[BR_NW];
    __shared__ u64 s_segv[BR_NW];
    __shared__ u32 s_firstk[BR_T + 1], s_lastk[BR_T];
    __shared__ u32 s_hist[1024];
    __shared__ u64 s_pre;
    __shared__ u32 s_tn;
    __shared__ u32 s_m;
    BrCtx<RING> B{s_mem};
    const i64 ntk = (i64)C.bk_sbtb[C.bk_nsb];
    // work items from a queue; the next ticket is taken while the current
    // work item runs, and its descriptor loaded at the end of it
    if (threadIdx.x == 0) s_pre = atomicAdd(&C.counters[CNT_BK_REDUCE], 1u);
    __syncthreads();
    i64 t = (i64)uniform32((u32)s_pre);
    BkWi wn;
    if (t < ntk) wn = C.bk_wi[t];
    int qc = -1;  // product whose fields are held in s
    BrSeg s;
    while (t < ntk) {
        __syncthreads();  // every thread has read the ticket
        if (threadIdx.x == 0) s_tn = atomicAdd(&C.counters[CNT_BK_REDUCE], 1u);
        // the work item's and its product's fields, in scalar registers
        BkWi W;
        W.bin_lo = uniform32(wn.bin_lo);
        W.bin_hi = uniform32(wn.bin_hi);
        W.off = (u64)uniform64((i64)wn.off);
        W.end = (u64)uniform64((i64)wn.end);
        W.q = (i32)uniform32((u32)wn.q);
        if (W.q != qc) {
            s = load_br_seg(C, W.q);
            qc = W.q;
        }
        const u32 kbase = W.bin_lo << s.fs;
        const u64 span = (u64)(W.bin_hi - W.bin_lo) << s.fs;
        const u64 n = W.end - W.off;
        const bool fat = n > (u64)BK_CAP;
        const u32 nb = s.nb;
        const Div32 nbd = s.nb_div;
        const u32 ibits = bitlen64((u64)(s.na - 1));
        // a work item over BK_CAP pairs is a single fine bin: at most 2^fs
        // result terms, whose coefficients go to a range of bk_fatc (its
        // staging is read again by every round)
        u64 fbase = 0;
        if (fat) {
            if (threadIdx.x == 0) {
                const u64 want = min(n, (u64)1 << s.fs);
                u64 b = atomicAdd((unsigned long long *)C.bk_fatfill, (unsigned long long)want);
                if (b + want > (u64)C.bk_fat_cap) {  // never planned
                    atomicOr(&C.counters[CNT_ERR_SPIN], 16u);
                    b = ~0ull;
                }
                s_pre = b;
            }
            __syncthreads();
            fbase = (u64)uniform64((i64)s_pre);
        }
        u64 acc = 0;  // result terms of the earlier rounds
        u64 lo = 0;   // first key (relative to kbase) of the next round
        while (lo < span) {
            const Thr h = br_thr();  // opaque again for each round
            const u32 tid = h.tid;
            u64 hi = span;
            if (fat) {
                // the round's key range [lo, hi): at most BK_CAP items, from
                // 1024-bucket histograms of the remaining range, refined while
                // the first bucket alone holds more
                u64 a = lo, b = span;
                while (true) {
                    const u64 wdt = (b - a + 1023) / 1024;
                    for (u32 e = tid; e < 1024; e += BR_T) s_hist[e] = 0;
                    __syncthreads();
                    for (u64 e = tid; e < n; e += BR_T) {
                        const u64 lk = (u32)C.bk_stage[W.off + e] - kbase;
                        if (lk >= a && lk < b) atomicAdd(&s_hist[(lk - a) / wdt], 1u);
                    }
                    __syncthreads();
                    u32 run = 0, fit = 0;
                    for (u32 e = 0; e < 1024 / BR_T; e++) run += s_hist[tid * (1024 / BR_T) + e];
                    u32 tot;
                    u32 ex = br_excl_scan(run, s_scan, tot, h);
                    for (u32 e = 0; e < 1024 / BR_T; e++) {
                        ex += s_hist[tid * (1024 / BR_T) + e];
                        fit += ex <= (u32)BK_CAP ? 1u : 0u;
                    }
                    u32 nfit;
                    (void)br_excl_scan(fit, s_scan, nfit, h);
                    if (nfit == 0) {
                        if (wdt == 1) {  // one monomial with more than BK_CAP pairs: never planned
                            if (tid == 0) atomicOr(&C.counters[CNT_ERR_SPIN], 4u);
                            hi = a + 1;
                            break;
                        }
                        b = a + wdt;
                        continue;
                    }
                    hi = nfit == 1024 ? b : min(b, a + (u64)nfit * wdt);
                    break;
                }
                // stage the round's items in LDS
                u32 m0 = 0;
                for (u64 e0 = 0; e0 < n; e0 += BR_T) {
                    const u64 e = e0 + tid;
                    u64 it = 0;
                    bool in = false;
                    if (e < n) {
                        it = C.bk_stage[W.off + e];
                        const u64 lk = (u32)it - kbase;
                        in = lk >= lo && lk < hi;
                    }
                    u32 tot;
                    const u32 at = m0 + br_excl_scan(in ? 1u : 0u, s_scan, tot, h);
                    if (in && at < (u32)BK_CAP) {
                        B.stk()[at] = (u32)it;
                        B.stx()[at] = (u32)(it >> 32);
                    }
                    m0 += tot;
                }
                if (tid == 0) s_m = min(m0, (u32)BK_CAP);
                __syncthreads();
            }
            const u32 m = fat ? uniform32(s_m) : (u32)n;
            const u32 rbase = kbase + (u32)lo;  // smallest key of the round
            const u32 kbits = bitlen64(hi - lo - 1);
            const bool direct = !F64 && hi - lo <= (u64)BK_DIRECT;
            const bool ranked = !F64 && !direct && hi - lo <= (u64)BR_RANK_SPAN;
            // load: register slot k holds the item at load position br_seq(k)
            u32 ks[BR_IPT], xs[BR_IPT];
#pragma unroll
            for (int k = 0; k < BR_IPT; k++) {
                const u32 lp = br_seq(k, h);
                xs[k] = 0;
                ks[k] = rbase;
                if (lp < m) {
                    if (fat) {
                        ks[k] = B.stk()[lp];
                        xs[k] = B.stx()[lp];
                    } else {
                        const u64 it = C.bk_stage[W.off + lp];
                        ks[k] = (u32)it;
                        xs[k] = (u32)(it >> 32);
                    }
                }
            }
            if (fat) __syncthreads();  // the staging overlays the accumulator and the sort arrays
            // the product a_i b_j of slot k's pair (operand gathers in load
            // order, where neighbouring items share rows and nearby columns)
            auto product = [&](int k, u32 &row) -> u64 {
                u32 i = div32(xs[k], nbd), j = xs[k] - i * nb;
                if ((i64)i >= s.na) {  // a staging slot never written: internal error
                    atomicOr(&C.counters[CNT_ERR_SPIN], 8u);
                    i = 0;
                    j = 0;
                }
                row = i;
                return ring_mul<RING>(gload(s.fc + i), gload(s.gc + j));
            };
            // this thread's results: slots k with bit k of em set, key rbase +
            // kk[k], coefficient val[k], in key order across the workgroup
            u32 kk[BR_IPT];
            u64 val[BR_IPT];
            u32 em = 0;
            if (direct || ranked) {
                if constexpr (!F64) {
                    // cells in key order: the local key itself (direct) or its
                    // rank among the round's present keys (ranked)
                    u64 *cell = B.acc();
                    u32 *rkey = B.rkey();
                    u64 *bm = B.bm();
                    unsigned short *pre = B.pre();
                    const u32 nw = ranked ? (u32)((hi - lo + 63) >> 6) : 0;
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) cell[k * BR_T + tid] = 0;
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        if ((u32)e * BR_T + tid < nw) bm[e * BR_T + tid] = 0;
                    __syncthreads();
                    u32 ncell = BK_DIRECT;
                    if (ranked) {
#pragma unroll
                        for (int k = 0; k < BR_IPT; k++) {
                            if (br_seq(k, h) < m) {
                                const u32 kl = ks[k] - rbase;
                                atomicOr((unsigned long long *)&bm[kl >> 6], 1ull << (kl & 63));
                            }
                        }
                        __syncthreads();
                        // rank of a word's first key: prefix of the popcounts
                        // (thread t: words 4t .. 4t + 3)
                        u32 pc[4], sum = 0;
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const u32 wd = tid * 4 + e;
                            pc[e] = wd < nw ? (u32)__popcll(bm[wd]) : 0u;
                            sum += pc[e];
                        }
                        u32 ex = br_excl_scan(sum, s_scan, ncell, h);
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const u32 wd = tid * 4 + e;
                            if (wd < nw) pre[wd] = (unsigned short)ex;
                            ex += pc[e];
                        }
                        __syncthreads();
                    }
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) {
                        if (br_seq(k, h) < m) {
                            const u32 kl = ks[k] - rbase;
                            u32 c = kl;
                            if (ranked) {
                                const u32 wd = kl >> 6;
                                c = pre[wd] + (u32)__popcll(bm[wd] & ((1ull << (kl & 63)) - 1));
                                rkey[c] = kl;
                            }
                            u32 row;
                            ring_atomic_acc<RING>(cell + c, product(k, row));
                        }
                        if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                    }
                    __syncthreads();
                    // striped read-back: slot k of a wave's lanes is the run of
                    // cells br_seq(k, .), so a wave's cells are contiguous
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) {
                        const u32 c = br_seq(k, h);
                        kk[k] = c;
                        val[k] = 0;
                        if (c < ncell) {
                            if (ranked) kk[k] = rkey[c];
                            val[k] = ring_cell_final<RING>(cell[c]);
                            if (!ring_is_zero<RING>(val[k])) em |= 1u << k;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < BR_IPT; k++) {
                    const u32 lp = br_seq(k, h);
                    if (lp < m) {
                        B.lk()[lp] = ks[k] - rbase;
                        if constexpr (F64) B.ik()[lp] = div32(xs[k], nbd);
                    }
                }
                __syncthreads();
                // LSD passes: for FP64 the row first (least significant), then the key
                BrPerm pv;
#pragma unroll
                for (int k = 0; k < BR_IPT; k++) pv.set(k, br_seq(k, h));
                const u32 pk = (kbits + 7) / 8, pi = F64 ? (ibits + 7) / 8 : 0;
                const u32 np = pk + pi;
                if (np == 0) {
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) {
                        pv.set(k, tid * BR_IPT + k);
                        if (F64) B.perm()[tid * BR_IPT + k] = (unsigned short)(tid * BR_IPT + k);
                    }
                } else {
                    for (u32 ps = 0; ps < np; ps++) {
                        const bool onrow = ps < pi;
                        const u32 bits = onrow ? ibits : kbits, npass = onrow ? pi : pk, idx = onrow ? ps : ps - pi;
                        const u32 wd = (bits + npass - 1) / npass;
                        const u32 sh = idx * wd, width = min(wd, bits - sh);
                        br_pass<RING>(B, pv, onrow ? B.ik() : B.lk(), sh, width, m, ps == np - 1, s_scan, h);
                    }
                }
                // this thread's sorted items are positions p0 .. p0 + BR_IPT - 1
                const u32 p0 = tid * BR_IPT;
#pragma unroll
                for (int k = 0; k < BR_IPT; k++) kk[k] = B.lk()[pv.get(k)];
                s_firstk[tid] = kk[0];
                s_lastk[tid] = kk[BR_IPT - 1];
                if (tid == 0) s_firstk[BR_T] = 0;
                if (F64) {
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) B.lks()[p0 + k] = kk[k];
                }
                __syncthreads();
                // the products, by load position, over the keys
#pragma unroll
                for (int k = 0; k < BR_IPT; k++) {
                    const u32 lp = br_seq(k, h);
                    if (lp < m) {
                        u32 row;
                        B.cval()[lp] = product(k, row);
                    }
                    if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
                const bool hd0 = p0 < m && (tid == 0 || s_lastk[tid - 1] != kk[0]);
                if constexpr (!F64) {
                    // run sums by a segmented scan (exact rings: any order)
                    u32 fl = 0;
                    u64 run = 0;
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) {
                        if (p0 + k < m) {
                            const u64 c = B.cval()[pv.get(k)];
                            const bool hk = k ? kk[k] != kk[k - 1] : hd0;
                            if (hk) {
                                run = c;
                                fl = 1;
                            } else {
                                run = ring_add<RING>(run, c);
                            }
                        }
                        val[k] = run;
                    }
                    const u64 carry = br_seg_scan<RING>(fl, run, s_segf, s_segv, h);
                    bool seen = false;
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) {
                        const bool v = p0 + k < m;
                        seen = seen || (v && (k ? kk[k] != kk[k - 1] : hd0));
                        const bool endr = k < BR_IPT - 1 ? (p0 + k + 1 >= m || kk[k + 1] != kk[k])
                                                         : (p0 + BR_IPT >= m || s_firstk[tid + 1] != kk[k]);
                        if (!seen) val[k] = ring_add<RING>(carry, val[k]);
                        if (v && endr && !ring_is_zero<RING>(val[k])) em |= 1u << k;
                    }
                } else {
                    // FP64: the thread holding a run's first item adds the run
                    // left to right (rows ascending within a key: row-major order)
                    const unsigned short *perm = B.perm();
                    const u32 *lks = B.lks();
#pragma unroll
                    for (int k = 0; k < BR_IPT; k++) {
                        const u32 p = p0 + k;
                        val[k] = 0;
                        if (p < m && (k ? kk[k] != kk[k - 1] : hd0)) {
                            u64 sum = B.cval()[perm[p]];
                            for (u32 e = p + 1; e < m && lks[e] == kk[k]; e++)
                                sum = ring_add<RING>(sum, B.cval()[perm[e]]);
                            val[k] = sum;
                            if (!ring_is_zero<RING>(sum)) em |= 1u << k;
                        }
                    }
                }
            }
            // result terms: keys to bk_rkey, coefficients to the work item's
            // own staging range (its pairs are all loaded) or to bk_fatc
            u32 u;
            if (direct || ranked) {
                // striped: wave-local ranks by ballot, then the waves' prefix
                u32 rk[BR_IPT], before = 0;
#pragma unroll
                for (int k = 0; k < BR_IPT; k++) {
                    const u64 bal = __ballot((em >> k) & 1u);
                    rk[k] = before + mbcnt(bal);
                    before += (u32)__popcll(bal);
                }
                if (h.lane == 0) s_scan[h.w] = before;
                __syncthreads();
                u32 wpre = 0, tot = 0;
#pragma unroll
                for (u32 i = 0; i < (u32)BR_NW; i++) {
                    const u32 v = s_scan[i];
                    if (i < h.w) wpre += v;
                    tot += v;
                }
                u = tot;
#pragma unroll
                for (int k = 0; k < BR_IPT; k++) {
                    if ((em >> k) & 1) {
                        const u64 at = acc + wpre + rk[k];
                        C.bk_rkey[W.off + at] = rbase + kk[k];
                        if (!fat) C.bk_stage[W.off + at] = val[k];
                        else if (fbase != ~0ull) C.bk_fatc[fbase + at] = val[k];
                    }
                }
            } else {
                const u32 rb = br_excl_scan((u32)__popc(em), s_scan, u, h);
                u64 at = acc + rb;
#pragma unroll
                for (int k = 0; k < BR_IPT; k++) {
                    if ((em >> k) & 1) {
                        C.bk_rkey[W.off + at] = rbase + kk[k];
                        if (!fat) C.bk_stage[W.off + at] = val[k];
                        else if (fbase != ~0ull) C.bk_fatc[fbase + at] = val[k];
                        at++;
                    }
                }
            }
            acc += u;
            lo = hi;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            C.bk_u[t] = (u32)acc | (fat ? 0x80000000u : 0u);
            if (fat) C.bk_fbase[t] = fbase;
        }
        __syncthreads();
        t = (i64)uniform32(s_tn);
        if (t < ntk) wn = C.bk_wi[t];
    }
}

// Result offsets: per product, the exclusive prefix of the work items'
// result counts in ticket (key) order; the product's term count (one
// workgroup, BO_IPT work items per thread per chunk, every load of a chunk
// issued before the first use).
constexpr int BO_IPT = 8;
__global__ __launch_bounds__(BC_T) void k_bk_oscan(Ctx C) {
    __shared__ u64 s_v[BC_T / 64];
    __shared__ u32 s_f[BC_T / 64];
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    const i64 ntk = (i64)C.bk_sbtb[C.bk_nsb];
    u64 carry = 0;  // running sum of the product in progress at the chunk's start
    for (i64 b = 0; b < ntk; b += (i64)BC_T * BO_IPT) {
        const i64 t0 = b + (i64)threadIdx.x * BO_IPT;
        u32 v[BO_IPT];
        u32 fl = 0, la = 0;  // bit e: work item t0 + e is its product's first / last
#pragma unroll
        for (int e = 0; e < BO_IPT; e++) {
            const i64 t = t0 + e;
            v[e] = 0;
            if (t < ntk) {
                v[e] = C.bk_u[t] & 0x7FFFFFFFu;
                fl |= (C.bk_wi[t].first ? 1u : 0u) << e;
                la |= (C.bk_wi[t].last ? 1u : 0u) << e;
            }
        }
        // the thread's (restarted, sum since its last restart)
        u32 fi = fl ? 1u : 0u;
        u64 vi = 0;
#pragma unroll
        for (int e = 0; e < BO_IPT; e++) vi = ((fl >> e) & 1u) ? (u64)v[e] : vi + v[e];
        // inclusive segmented scan over the wave's threads
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const u32 fu = __shfl_up(fi, d, 64);
            const u64 vu = ((u64)__shfl_up((u32)(vi >> 32), d, 64) << 32) | __shfl_up((u32)vi, d, 64);
            if (lane >= (u32)d) {
                if (!fi) vi += vu;
                fi |= fu;
            }
        }
        if (lane == 63) {
            s_v[w] = vi;
            s_f[w] = fi;
        }
        // this thread's exclusive part within the wave
        u32 fe = __shfl_up(fi, 1, 64);
        u64 ve = ((u64)__shfl_up((u32)(vi >> 32), 1, 64) << 32) | __shfl_up((u32)vi, 1, 64);
        if (lane == 0) {
            fe = 0;
            ve = 0;
        }
        __syncthreads();
        u64 cin = carry;  // the chunk carry, then the earlier waves, then the earlier lanes
        for (u32 ww = 0; ww < w; ww++) cin = s_f[ww] ? s_v[ww] : cin + s_v[ww];
        cin = fe ? ve : cin + ve;
        u64 run = cin;
#pragma unroll
        for (int e = 0; e < BO_IPT; e++) {
            const i64 t = t0 + e;
            run = ((fl >> e) & 1u) ? (u64)v[e] : run + v[e];
            if (t < ntk) {
                C.bk_opre[t] = run - v[e];
                if ((la >> e) & 1u) *C.segs[C.bk_wi[t].q].n_out = (i64)run;
            }
        }
        u64 ctot = carry;
        for (u32 ww = 0; ww < BC_T / 64; ww++) ctot = s_f[ww] ? s_v[ww] : ctot + s_v[ww];
        __syncthreads();
        carry = ctot;
    }
}

// Compressed key to packed key with the product's variable fields held in
// LDS (vl[5 v .. 5 v + 4]: shift, then the division by the range).
__device__ inline u64 decompress_lds(u32 ck, const u32 *vl, int nvars, u64 lo_key) {
    u64 key = lo_key;
    for (int v = nvars - 1; v >= 0; v--) {
        const Div32 dv{vl[5 * v + 1], vl[5 * v + 2], vl[5 * v + 3], vl[5 * v + 4]};
        const u32 q = div32(ck, dv);
        key += (u64)(ck - q * dv.d) << vl[5 * v];
        ck = q;
    }
    return key;
}

// Result terms of every work item to its offset in h, keys decompressed
// (BK_CP terms per thread per batch, loads issued before the stores).
constexpr int BK_CP = 8;
__global__ __launch_bounds__(BK_T) void k_bk_copy(Ctx C) {
    __shared__ u32 s_vl[5 * MAX_VARS];
    const i64 ntk = (i64)C.bk_sbtb[C.bk_nsb];
    const int nvars = C.nvars;
    int qc = -1;
    u64 *hk = nullptr, *hc = nullptr;
    i64 cap = 0;
    u64 lo_key = 0;
    for (i64 t = blockIdx.x; t < ntk; t += gridDim.x) {
        const u32 uv = C.bk_u[t];
        const u32 uw = uv & 0x7FFFFFFFu;
        const bool fat = (uv >> 31) != 0;
        const u64 fb = fat ? C.bk_fbase[t] : 0;
        const u64 P = C.bk_opre[t];
        const i32 q = C.bk_wi[t].q;
        const u64 off = C.bk_wi[t].off;
        if (fat && fb == ~0ull) continue;  // its coefficients were not kept (flagged)
        if (q != qc) {
            const DevSeg &s = C.segs[q];
            __syncthreads();
            const VarParam *vp = C.vars + s.var_off;
            for (int v = threadIdx.x; v < nvars; v += BK_T) {
                s_vl[5 * v] = vp[v].shift;
                s_vl[5 * v + 1] = vp[v].rdiv.m;
                s_vl[5 * v + 2] = vp[v].rdiv.s1;
                s_vl[5 * v + 3] = vp[v].rdiv.s2;
                s_vl[5 * v + 4] = vp[v].rdiv.d;
            }
            hk = s.hk;
            hc = s.hc;
            cap = s.cap;
            lo_key = s.lo_key;
            __syncthreads();
            qc = q;
        }
        const u32 *rk = C.bk_rkey + off;
        const u64 *rc = fat ? C.bk_fatc + fb : C.bk_stage + off;
        for (u32 r0 = 0; r0 < uw; r0 += BK_T * BK_CP) {
            u32 ck[BK_CP];
            u64 cv[BK_CP];
#pragma unroll
            for (int e = 0; e < BK_CP; e++) {
                const u32 r = r0 + e * BK_T + threadIdx.x;
                ck[e] = 0;
                cv[e] = 0;
                if (r < uw) {
                    ck[e] = rk[r];
                    cv[e] = rc[r];
                }
            }
#pragma unroll
            for (int e = 0; e < BK_CP; e++) {
                const u32 r = r0 + e * BK_T + threadIdx.x;
                const u64 at = P + r;
                if (r < uw && (i64)at < cap) {
                    hk[at] = decompress_lds(ck[e], s_vl, nvars, lo_key);
                    hc[at] = cv[e];
                }
            }
        }
    }
}

}  // namespace pm
