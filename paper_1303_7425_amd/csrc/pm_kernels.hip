// gfx950 kernels of the sparse polynomial product h = f * g.
//
// Pipeline for one launch (a batch of one or more products, "segments"):
//   k_stats      validation + per-variable exponent ranges of every operand
//   k_compress   operand keys -> mixed-radix indices in the product's degree box
//   k_tile       f-block x g-block tile of term products expanded into LDS and
//                combined there with an LDS hash (exact rings); unique pairs go
//                to a staging buffer (sparse) or into the degree-box array (dense)
//   k_seg_prepare per-product sizes, sort partitions, sort blocks
//   k_count      digit counts per sort block before each radix pass
//   k_onesweep   one stable LSD radix pass (8-bit digit); a workgroup ranks one
//                sort block's partitions in order from precomputed positions;
//                SEG_RAW products sort pair indices alone and regenerate their
//                keys from the operands' compressed keys
//   k_head_count run heads per reduce partition, k_head_scan their prefix
//   k_reduce     segmented like-term reduction + key decompression
//   k_zero_compact removal of runs that cancelled to zero
//   k_compact    dense path: degree-box cells -> sorted non-zero terms
//
// The schoolbook product P = sum_{i,j} a_i b_j x^{alpha_i + beta_j} and the
// canonical (sorted, summed, zero-free) result are defined in Section 2 of the
// paper (problem statement, Fig. 1, Algorithm 1).  The paper's own GPU kernel
// builds a per-interval 16-ary tree with atomics (Section 6.3); here the merge
// and sort step is redesigned for CDNA4 as LDS combine + global radix sort.
#include <type_traits>

#include "pm_internal.hpp"

namespace pm {

// ---------------------------------------------------------------------------
// k_stats: one workgroup per (segment, operand side).  Per-variable min/max of
// the exponents, strict ascending order, key bits outside the fields, and
// coefficient range.  out[(q*2+side)*2*nvars + v] = min, [... + nvars + v] = max.
// One sweep over the terms per group of eight variables, four independent
// loads in flight per thread (1024 threads: an operand of a few thousand
// terms takes one or two steps); the checks ride along with the first group.
// ---------------------------------------------------------------------------
constexpr int ST_T = 1024;

// A 64-bit value from another lane through a DPP move of both halves (lanes
// without a source keep their own value: harmless for min and max).
template <int CTRL>
__device__ inline u64 dpp_u64(u64 v) {
    const u32 lo = (u32)__builtin_amdgcn_update_dpp((int)(u32)v, (int)(u32)v, CTRL, 0xF, 0xF, false);
    const u32 hi = (u32)__builtin_amdgcn_update_dpp((int)(u32)(v >> 32), (int)(u32)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((u64)hi << 32) | lo;
}

// Minimum (MAX: maximum) over the wave, valid in lane 63: shifts by 1, 2, 4
// and 8 within each row of 16 lanes, then row 15 and lane 31 broadcasts.
template <bool MAX>
__device__ inline u64 wave_minmax_u64(u64 v) {
    auto op = [](u64 a, u64 b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
    v = op(v, dpp_u64<0x111>(v));
    v = op(v, dpp_u64<0x112>(v));
    v = op(v, dpp_u64<0x114>(v));
    v = op(v, dpp_u64<0x118>(v));
    v = op(v, dpp_u64<0x142>(v));
    v = op(v, dpp_u64<0x143>(v));
    return v;
}

__global__ __launch_bounds__(ST_T) void k_stats(const DevSeg *segs, int nvars, int bits, int ring, u64 *out,
                                                     u32 *flags) {
    constexpr int G = 8, U = 4, NW = ST_T / 64;
    const int q = blockIdx.x >> 1, side = blockIdx.x & 1;
    const DevSeg &s = segs[q];
    const i64 n = side ? s.nb : s.na;
    const u64 *k = side ? s.gk : s.fk;
    const u64 *c = side ? s.gc : s.fc;
    const u64 mask = bits == 64 ? ~0ull : ((1ull << bits) - 1);
    const int used = nvars * bits;
    __shared__ u64 s_mn[G][NW], s_mx[G][NW];
    __shared__ u32 s_flag;
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    u32 fl = 0;
    u64 *o = out + (i64)(q * 2 + side) * 2 * nvars;
    for (int v0 = 0; v0 < nvars; v0 += G) {
        u64 mn[G], mx[G];
        u32 sh[G];
#pragma unroll
        for (int u = 0; u < G; u++) {
            mn[u] = ~0ull;
            mx[u] = 0;
            sh[u] = v0 + u < nvars ? (u32)((nvars - 1 - (v0 + u)) * bits) : 0u;
        }
        for (i64 i0 = threadIdx.x; i0 < n; i0 += U * ST_T) {
            u64 kk[U], kp[U], cc[U];
#pragma unroll
            for (int r = 0; r < U; r++) {
                const i64 i = i0 + (i64)r * ST_T;
                kk[r] = i < n ? k[i] : 0;
                kp[r] = (v0 == 0 && i > 0 && i < n) ? k[i - 1] : 0;
                cc[r] = (v0 == 0 && i < n) ? c[i] : 0;
            }
#pragma unroll
            for (int r = 0; r < U; r++) {
                const i64 i = i0 + (i64)r * ST_T;
                if (i >= n) continue;
                if (v0 == 0) {
                    if (used < 64 && (kk[r] >> used) != 0) fl |= ST_BADBITS;
                    if (i > 0 && !(kk[r] > kp[r])) fl |= ST_UNSORTED;
                    if (ring == RING_MODP && cc[r] >= P61) fl |= ST_RANGE;
                    if (ring == RING_MODQ && cc[r] >= Q64) fl |= ST_RANGE;
                    if (ring == RING_F64 && ((cc[r] >> 52) & 0x7ff) == 0x7ff) fl |= ST_RANGE;
                }
#pragma unroll
                for (int u = 0; u < G; u++) {
                    const u64 e = (kk[r] >> sh[u]) & mask;
                    mn[u] = e < mn[u] ? e : mn[u];
                    mx[u] = e > mx[u] ? e : mx[u];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < G; u++) {
            mn[u] = wave_minmax_u64<false>(mn[u]);
            mx[u] = wave_minmax_u64<true>(mx[u]);
            if (lane_id() == 63) {
                s_mn[u][threadIdx.x >> 6] = mn[u];
                s_mx[u][threadIdx.x >> 6] = mx[u];
            }
        }
        __syncthreads();
        if (threadIdx.x < G && v0 + (int)threadIdx.x < nvars) {
            const int u = threadIdx.x;
            u64 a = s_mn[u][0], b = s_mx[u][0];
            for (int w = 1; w < NW; w++) {
                a = s_mn[u][w] < a ? s_mn[u][w] : a;
                b = s_mx[u][w] > b ? s_mx[u][w] : b;
            }
            o[v0 + u] = a;
            o[nvars + v0 + u] = b;
        }
        __syncthreads();
    }
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (threadIdx.x == 0) flags[q * 2 + side] = s_flag;
}

// ---------------------------------------------------------------------------
// Fill a u64 region (the per-call zeroed state: counters, range counters of
// the radix passes, look-back words, dense box).  A kernel, so that graph
// replays stay valid.
// ---------------------------------------------------------------------------
__global__ void k_fill(u64 *p, i64 n, u64 v) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_set32(u32 *p, u32 v) { *p = v; }

// ---------------------------------------------------------------------------
// k_compress: operand keys -> mixed-radix index.  Term t of the flattened list
// [seg0.f, seg0.g, seg1.f, ...] located through cpre (exclusive prefix).
// ---------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(NTHREADS) void k_compress(Ctx C, const i64 *cpre, i64 total) {
    for (i64 t = (i64)blockIdx.x * NTHREADS + threadIdx.x; t < total; t += (i64)gridDim.x * NTHREADS) {
        i32 idx = seg_search(cpre, 2 * C.nseg, t);
        const int q = idx >> 1, side = idx & 1;
        const DevSeg &s = C.segs[q];
        const i64 i = t - cpre[idx];
        const u64 key = side ? s.gk[i] : s.fk[i];
        const VarParam *vp = C.vars + s.var_off;
        u64 ck = 0;
        for (int v = 0; v < C.nvars; v++) {
            u64 e = (key >> vp[v].shift) & vp[v].mask;
            ck += (e - (side ? vp[v].ming : vp[v].minf)) * vp[v].stride;
        }
        ((K *)C.ck)[(side ? s.ck_g : s.ck_f) + i] = (K)ck;
    }
}

constexpr int MAX_PROBE = 32;

template <typename K>
__device__ inline K lds_cas(K *p, K cmp, K val) {
    if constexpr (sizeof(K) == 4) {
        return (K)atomicCAS((unsigned int *)p, (unsigned int)cmp, (unsigned int)val);
    } else {
        return (K)atomicCAS((unsigned long long *)p, (unsigned long long)cmp, (unsigned long long)val);
    }
}

template <typename K>
__device__ inline u32 hash_slot(K ck, int hb) {
    if constexpr (sizeof(K) == 4) {
        return ((u32)ck * 2654435761u) >> (32 - hb);
    } else {
        return (u32)(((u64)ck * 0x9E3779B97F4A7C15ull) >> (64 - hb));
    }
}

// ---------------------------------------------------------------------------
// k_tile: persistent work queue over the tiles of all SEG_COMBINE / SEG_DENSE
// products.  A tile is rows [i0, i0+TM) of f times columns [j0, j0+TN) of g:
// a TM x TN block of the pp-matrix (Fig. 1).  Each term product is inserted
// into an LDS open-addressing table keyed by its mixed-radix monomial index
// and accumulated there exactly (mod p or modulo 2^64).  The table's non-zero
// entries then go either to the product's staging array (sparse; the offset
// comes from a look-back over the product's earlier tiles, so the staging is
// dense) or into the degree-box array (dense).  One launch takes the tiles
// [t_begin, t_end): a large product runs as several bounded launches, so work
// on other streams is not kept off the device for the whole product.
// ---------------------------------------------------------------------------
template <typename K, int RING, int TM, int TN, int HB>
__global__ __launch_bounds__(NTHREADS) void k_tile(Ctx C, i64 t_begin, i64 t_end) {
    constexpr int HS = 1 << HB;
    constexpr int SPT = HS / NTHREADS;
    const K EMPTY = (K)~(K)0;
    __shared__ K s_fk[TM], s_gk[TN];
    __shared__ u64 s_fc[TM], s_gc[TN];
    __shared__ K s_hk[HS + HS / 16];   // padded: slot h lives at h + h/16
    __shared__ u64 s_hv[HS + HS / 16];
    __shared__ u32 s_scan[NTHREADS / 64];
    __shared__ i64 s_tile;
    __shared__ u64 s_base;
    auto pad = [](int h) { return h + (h >> 4); };

    const i64 tb = C.tb_tile;
    while (true) {
        if (threadIdx.x == 0) s_tile = t_begin + (i64)atomicAdd(&C.counters[CNT_TILE], 1u) * tb;
        __syncthreads();
        const i64 t0 = s_tile;
        if (t0 >= t_end) break;
        __syncthreads();
        for (i64 t = t0; t < min(t0 + tb, t_end); t++) {
        const i32 ts = seg_search(C.tile_pre, C.ntseg, t);
        const int q = C.tile_seg[ts];
        const DevSeg &s = C.segs[q];
        const i64 local = t - C.tile_pre[ts];
        const i64 i0 = (local / s.tiles_n) * TM, j0 = (local % s.tiles_n) * TN;
        const int tm = (int)min((i64)TM, s.na - i0), tn = (int)min((i64)TN, s.nb - j0);
        const bool dense = s.mode == SEG_DENSE;
        const K *ck = (const K *)C.ck;
        for (int e = threadIdx.x; e < TM; e += NTHREADS)
            if (e < tm) {
                s_fk[e] = ck[s.ck_f + i0 + e];
                s_fc[e] = s.fc[i0 + e];
            }
        for (int e = threadIdx.x; e < TN; e += NTHREADS)
            if (e < tn) {
                s_gk[e] = ck[s.ck_g + j0 + e];
                s_gc[e] = s.gc[j0 + e];
            }
        for (int e = threadIdx.x; e < HS; e += NTHREADS) {
            s_hk[pad(e)] = EMPTY;
            s_hv[pad(e)] = 0;
        }
        __syncthreads();
        // expand + combine
        const int max_probe = dense ? MAX_PROBE : HS;
        for (int e = threadIdx.x; e < TM * TN; e += NTHREADS) {
            const int i = e / TN, j = e % TN;
            if (i >= tm || j >= tn) continue;
            const u64 c = ring_mul<RING>(s_fc[i], s_gc[j]);
            if (c == 0) continue;
            const K key = s_fk[i] + s_gk[j];
            u32 h = hash_slot<K>(key, HB);
            bool found = false;
            for (int probe = 0; probe < max_probe; probe++) {
                K old = lds_cas<K>(&s_hk[pad(h)], EMPTY, key);
                if (old == EMPTY || old == key) {
                    found = true;
                    break;
                }
                h = (h + 1) & (HS - 1);
            }
            if (found) {
                ring_atomic_acc<RING>(&s_hv[pad(h)], c);
            } else if (dense) {
                // table region saturated: accumulate this product in the box directly
                ring_atomic_acc<RING>(C.box + s.stage_base + (u64)key, c);
            } else {
                // cannot happen: combine tiles hold at most half as many products as slots
                atomicOr(&C.counters[CNT_ERR_SPIN], 4u);
            }
        }
        __syncthreads();
        // compaction of the table: thread owns slots [tid*SPT, tid*SPT+SPT)
        u32 cnt = 0;
        for (int r = 0; r < SPT; r++) {
            const int h = pad(threadIdx.x * SPT + r);
            if (s_hk[h] != EMPTY && !ring_is_zero<RING>(ring_cell_final<RING>(s_hv[h]))) cnt++;
        }
        u32 total;
        u32 off = block_excl_scan<u32>(cnt, s_scan, total);
        if (dense) {
            u64 *box = C.box + s.stage_base;
            for (int r = 0; r < SPT; r++) {
                const int h = pad(threadIdx.x * SPT + r);
                if (s_hk[h] == EMPTY) continue;
                u64 v = ring_cell_final<RING>(s_hv[h]);
                if (!ring_is_zero<RING>(v)) ring_atomic_acc<RING>(box + (u64)s_hk[h], v);
            }
        } else {
            // dense staging offset: look-back over this product's earlier tiles
            const i64 tfirst = C.tile_pre[ts];
            if (threadIdx.x < 64) {
                const u64 pre = lookback_wave(C.look_tile, tfirst, t, 202u, total, &C.counters[CNT_ERR_SPIN]);
                if (threadIdx.x == 0) {
                    s_base = pre;
                    if (t == C.tile_pre[ts + 1] - 1) C.dyn[q].fill = pre + total;
                }
            }
            __syncthreads();
            const i64 base = s.stage_base + (i64)s_base + off;
            K *sk = (K *)C.stA_k;
            u64 *sv = (u64 *)C.stA_v;
            u32 w = 0;
            for (int r = 0; r < SPT; r++) {
                const int h = pad(threadIdx.x * SPT + r);
                if (s_hk[h] == EMPTY) continue;
                u64 v = ring_cell_final<RING>(s_hv[h]);
                if (ring_is_zero<RING>(v)) continue;
                sk[base + w] = s_hk[h];
                sv[base + w] = v;
                w++;
            }
        }
        __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// SEG_RAW products: pair (i, j) of the pp-matrix has index x = i*nb + j; the
// sort carries (key, x) and the reduction regenerates a_i * b_j from x.
// ---------------------------------------------------------------------------
// Wave-uniform value held in scalar registers.
__device__ inline i64 uniform64(i64 v) {
    const u32 lo = __builtin_amdgcn_readfirstlane((u32)(u64)v);
    const u32 hi = __builtin_amdgcn_readfirstlane((u32)((u64)v >> 32));
    return (i64)(((u64)hi << 32) | lo);
}
__device__ inline u32 uniform32(u32 v) { return __builtin_amdgcn_readfirstlane(v); }

// The fields of one product that a sort pass uses, kept in registers while
// consecutive partitions belong to the same product.
struct OsSeg {
    i64 first, n_q, lo;
    i64 ck_f, ck_g;
    u32 nb;
    Div32 nb_div;
};

__device__ inline OsSeg load_os_seg(const Ctx &C, int q) {
    const DevSeg &s = C.segs[q];
    OsSeg r;
    r.first = uniform64(C.ppre[q]);
    r.n_q = uniform64(C.dyn[q].n);
    r.lo = uniform64(s.stage_base);
    r.ck_f = uniform64(s.ck_f);
    r.ck_g = uniform64(s.ck_g);
    r.nb = uniform32((u32)s.nb);
    r.nb_div.m = uniform32(s.nb_div.m);
    r.nb_div.s1 = uniform32(s.nb_div.s1);
    r.nb_div.s2 = uniform32(s.nb_div.s2);
    r.nb_div.d = uniform32(s.nb_div.d);
    return r;
}

template <typename K>
__device__ inline K raw_key_os(const OsSeg &s, const K *ck, u32 x) {
    const u32 i = div32(x, s.nb_div);
    const u32 j = x - i * s.nb;
    return ck[s.ck_f + i] + ck[s.ck_g + j];
}

// ---------------------------------------------------------------------------
// Per-product sizes and sort partitions (one workgroup).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTHREADS) void k_seg_prepare(Ctx C) {
    __shared__ i64 s_scan[NTHREADS / 64];
    __shared__ i64 s_carry, s_ccarry, s_rcarry;
    if (threadIdx.x == 0) s_carry = s_ccarry = s_rcarry = 0;
    __syncthreads();
    for (int b = 0; b < C.nseg; b += NTHREADS) {
        const int q = b + threadIdx.x;
        i64 np = 0;
        if (q < C.nseg) {
            const DevSeg &s = C.segs[q];
            i64 n = 0;
            if (s.mode == SEG_COMBINE) n = (i64)C.dyn[q].fill;
            else if (s.mode == SEG_RAW) n = s.na * s.nb;
            C.dyn[q].n = n;
            np = (n + PART - 1) / PART;
            C.dyn[q].nparts = np;
            if ((s.mode == SEG_COMBINE || s.mode == SEG_RAW || s.mode == SEG_EMPTY) && n == 0) *s.n_out = 0;
        }
        i64 tot;
        i64 off = block_excl_scan<i64>(np, s_scan, tot);
        i64 ctot;
        const i64 nbq = (np + C.pblk - 1) / C.pblk;
        const i64 coff = block_excl_scan<i64>(nbq, s_scan, ctot);
        i64 rtot;
        const i64 roff = block_excl_scan<i64>((nbq + RNG - 1) / RNG, s_scan, rtot);
        if (q < C.nseg) {
            C.dyn[q].part_first = s_carry + off;
            C.ppre[q] = s_carry + off;
            C.chpre[q] = s_ccarry + coff;
            C.rpre[q] = s_rcarry + roff;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_carry += tot;
            s_ccarry += ctot;
            s_rcarry += rtot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        C.ppre[C.nseg] = s_carry;
        C.chpre[C.nseg] = s_ccarry;
        C.rpre[C.nseg] = s_rcarry;
    }
}

// ---------------------------------------------------------------------------
// Sort blocks.  Each product's sort partitions are cut into blocks of pblk
// consecutive partitions (pblk chosen so that the blocks about fill the
// resident grid), and the blocks into ranges of RNG blocks (chpre / rpre:
// block and range prefixes over products).  Before every radix pass the
// counting kernel writes each block's digit histogram (ctot) and adds it into
// its range's counter (rtot, one set per pass parity).  A radix pass
// takes one block at a time: its first position per digit is the digit base
// (keys of the product with a smaller digit) plus the counts of the earlier
// ranges (k_range_scan) and of the range's earlier blocks; it then ranks the
// block's partitions in order and carries the positions itself.  No look-back
// between workgroups; a work queue over blocks balances uneven products.
// ---------------------------------------------------------------------------
// Where a radix pass takes its items from.  SM_STAGED: (key, payload) pairs
// in the staging buffers (LDS-combined products).  SEG_RAW products carry
// only the pair index x = i*nb + j, whose key ck(alpha_i) + ck(beta_j) is
// regenerated from the compressed operand keys (a few tens of KB, cache
// resident) whenever it is needed: SM_GEN (first pass) takes x from the
// position, SM_INDEX (later passes) reads x from the staging buffer.
enum { SM_STAGED = 0, SM_GEN = 1, SM_INDEX = 2 };

// Digit counts (digit `pass`) of one sort block by CNT_T threads: CNT_G
// groups of NTHREADS, each counting its own partitions of the block into its
// own LDS histogram, so that CNT_G partitions' loads are in flight together.
// Writes the block's histogram, adds it into its range's counter of this
// pass's parity, and clears the other parity's row of the range for the next
// pass (the first block of each range does).  Staged keys and pair indices:
// each thread takes IPT consecutive items (16-byte loads; products start on
// 64-item boundaries) and counts runs of equal digits in a register, so the
// LDS sees one add per run: after the low digits are sorted, neighbouring
// keys mostly share their high digits, and per-item adds would collide in
// LDS.  Regenerated keys read the product's compressed operand keys (f's
// then g's, contiguous) from a copy in dynamic LDS (KL: every product of the
// launch fits), else from global memory: LDS serves a 64-lane gather in a
// few cycles, the vector cache about one line per cycle.  Generated pair indices run along the
// lanes, so that the LDS reads of g's keys hit distinct banks.
constexpr int CNT_G = 3;
constexpr int CNT_T = CNT_G * NTHREADS;

template <typename K, int SM, bool KL>
__global__ __launch_bounds__(CNT_T) __attribute__((amdgpu_waves_per_eu(6))) void k_count(Ctx C, int pass, const K *__restrict__ kin,
                                                 const u32 *__restrict__ xin) {
    __shared__ u32 s_h[CNT_G][RADIX];
    __shared__ u32 s_hg[RADIX];  // SM_GEN: histogram of g's low digit, per product
    extern __shared__ __align__(16) unsigned char s_dyn[];
    K *s_ck = (K *)s_dyn;
    const int shift = C.dsh[pass];
    const u32 dmask = (1u << C.dbits[pass]) - 1u;
    u64 *rt = C.rtot + (i64)(pass & 1) * C.nrng * RADIX;
    u64 *rz = C.rtot + (i64)((pass + 1) & 1) * C.nrng * RADIX;
    const K *ck = (const K *)C.ck;
    const i64 nblk = C.chpre[C.nseg];
    const int grp = (int)threadIdx.x / NTHREADS;
    const int tid = (int)threadIdx.x % NTHREADS;
    int cur_q = -1;
    OsSeg sq{};
    for (i64 b = blockIdx.x; b < nblk; b += gridDim.x) {
        s_h[grp][tid] = 0;  // RADIX == NTHREADS
        const int q = seg_search(C.chpre, C.nseg, b);
        if (q != cur_q) {
            sq = load_os_seg(C, q);
            cur_q = q;
            if constexpr (KL) {
                const i64 m = sq.ck_g - sq.ck_f + sq.nb;  // f's and g's compressed keys
                __syncthreads();  // the previous product's copy is no longer read
                for (i64 t = threadIdx.x; t < m; t += CNT_T) s_ck[t] = ck[sq.ck_f + t];
            }
            if constexpr (SM == SM_GEN) {
                __syncthreads();
                if (grp == 0) s_hg[tid] = 0;
                __syncthreads();
                const K *g0 = KL ? s_ck + (sq.ck_g - sq.ck_f) : ck + sq.ck_g;
                for (i64 t = threadIdx.x; t < sq.nb; t += CNT_T) atomicAdd(&s_hg[(u32)g0[t] & dmask], 1u);
            }
        }
        const i64 bl = b - C.chpre[q];
        const i64 r = C.rpre[q] + bl / RNG;
        const i64 p0 = sq.first + bl * C.pblk;
        const i64 p1 = min(sq.first + (sq.n_q + PART - 1) / PART, p0 + C.pblk);
        const K *kf = KL ? s_ck : ck + sq.ck_f;
        const K *kg = kf + (sq.ck_g - sq.ck_f);
        if (grp == 0 && bl % RNG == 0) rz[r * RADIX + tid] = 0;
        __syncthreads();
        if constexpr (SM == SM_GEN) {
            // Pass 0 counts the block's pairs x in [x0, x1) in generation
            // order (shift 0).  The digit of a_i + b_j is that of (a_i mod
            // 2^w) + (b_j mod 2^w), so a full row i of g contributes g's
            // low-digit histogram rotated by a_i: count[t] += hg[(t - a_i) mod 2^w].
            // Partial rows at the block's ends (and products with short
            // rows) are counted item by item.
            const u32 nb = sq.nb;
            const u32 x0 = (u32)((p0 - sq.first) * PART);
            const u32 x1 = (u32)min(sq.n_q, (p1 - sq.first) * PART);
            const u32 i0 = div32(x0, sq.nb_div), i1 = div32(x1 - 1, sq.nb_div);
            const bool rows = nb >= 4 * RADIX && i1 >= i0 + 2;
            const u32 e0 = rows ? (i0 + 1) * nb : x1;  // end of the first directly counted range
            const u32 s1 = rows ? i1 * nb : x1;        // start of the second
            for (u32 x = x0 + threadIdx.x; x < e0; x += CNT_T) {
                const u32 i = div32(x, sq.nb_div);
                atomicAdd(&s_h[0][(u32)(kf[i] + kg[x - i * nb]) & dmask], 1u);
            }
            for (u32 x = s1 + threadIdx.x; x < x1; x += CNT_T) {
                const u32 i = div32(x, sq.nb_div);
                atomicAdd(&s_h[0][(u32)(kf[i] + kg[x - i * nb]) & dmask], 1u);
            }
            if (rows && grp == 0 && (u32)tid <= dmask) {
                u32 acc = 0;
                for (u32 i = i0 + 1; i < i1; i++) acc += s_hg[((u32)tid - (u32)kf[i]) & dmask];
                if (acc) atomicAdd(&s_h[0][tid], acc);
            }
        }
        for (i64 p = p0 + grp; SM != SM_GEN && p < p1; p += CNT_G) {
            const i64 c = p - sq.first;
            const int n = (int)min((i64)PART, sq.n_q - c * PART);
            if constexpr (SM == SM_GEN) {
                // items tid + k * NTHREADS below n, in two halves (registers)
                u32 prev = 0, cnt = 0;
#pragma unroll 1
                for (int h = 0; h < IPT; h += IPT / 2) {
                    K key[IPT / 2];
#pragma unroll
                    for (int k = 0; k < IPT / 2; k++) {
                        const int idx = tid + (h + k) * NTHREADS;
                        const u32 x = (u32)(c * PART + idx);
                        const u32 i = div32(x, sq.nb_div);
                        key[k] = idx < n ? kf[i] + kg[x - i * sq.nb] : (K)0;
                    }
#pragma unroll
                    for (int k = 0; k < IPT / 2; k++) {
                        const u32 dk = (u32)(key[k] >> shift) & dmask;
                        if (tid + (h + k) * NTHREADS < n) {
                            if (cnt && dk != prev) {
                                atomicAdd(&s_h[grp][prev], cnt);
                                cnt = 0;
                            }
                            prev = dk;
                            cnt++;
                        }
                    }
                }
                if (cnt) atomicAdd(&s_h[grp][prev], cnt);
                continue;
            }
            K key[IPT];
            int nv;
            {
                nv = min(max(n - tid * IPT, 0), IPT);
                const i64 at = sq.lo + c * PART + (i64)tid * IPT;
                if constexpr (SM == SM_INDEX) {
                    u32 x[IPT];
                    if (nv == IPT) {
#pragma unroll
                        for (int k = 0; k < IPT; k += 4) {
                            const uint4 w = *(const uint4 *)(xin + at + k);
                            __builtin_memcpy(&x[k], &w, 16);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < IPT; k++) x[k] = k < nv ? xin[at + k] : 0u;
                    }
#pragma unroll
                    for (int k = 0; k < IPT; k++) {
                        const u32 i = div32(x[k], sq.nb_div);
                        key[k] = k < nv ? kf[i] + kg[x[k] - i * sq.nb] : (K)0;
                    }
                } else {
                    constexpr int VW = 16 / (int)sizeof(K);
                    if (nv == IPT) {
#pragma unroll
                        for (int k = 0; k < IPT; k += VW) {
                            const uint4 w = *(const uint4 *)(kin + at + k);
                            __builtin_memcpy(&key[k], &w, 16);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < IPT; k++) key[k] = k < nv ? kin[at + k] : (K)0;
                    }
                }
            }
            u32 prev = (u32)(key[0] >> shift) & dmask, cnt = 0;
#pragma unroll
            for (int k = 0; k < IPT; k++) {
                const u32 dk = (u32)(key[k] >> shift) & dmask;
                if (k < nv) {
                    if (dk != prev) {
                        atomicAdd(&s_h[grp][prev], cnt);
                        prev = dk;
                        cnt = 0;
                    }
                    cnt++;
                }
            }
            if (cnt) atomicAdd(&s_h[grp][prev], cnt);
        }
        __syncthreads();
        if (grp == 0) {
            u32 v = 0;
#pragma unroll
            for (int g2 = 0; g2 < CNT_G; g2++) v += s_h[g2][tid];
            C.ctot[b * RADIX + tid] = v;
            if (v) atomicAdd((unsigned long long *)&rt[r * RADIX + tid], (unsigned long long)v);
        }
        __syncthreads();
    }
}

// Per product: the ranges' counters of this pass become each range's first
// position per digit inside the product (exclusive prefix over the product's
// ranges, in place), and the digit bases (stage_base + keys with a smaller
// digit) go to pbase.  Range loads in batches.
__global__ __launch_bounds__(NTHREADS) void k_range_scan(Ctx C, int pass) {
    constexpr int B = 16;
    __shared__ u64 s_scan[NTHREADS / 64];
    u64 *rt = C.rtot + (i64)(pass & 1) * C.nrng * RADIX;
    const int d = threadIdx.x;  // RADIX == NTHREADS
    for (int q = blockIdx.x; q < C.nseg; q += gridDim.x) {
        const i64 r0 = C.rpre[q], r1 = C.rpre[q + 1];
        u64 run = 0;
        for (i64 rr = r0; rr < r1; rr += B) {
            u64 v[B];
#pragma unroll
            for (int k = 0; k < B; k++) v[k] = rr + k < r1 ? rt[(rr + k) * RADIX + d] : 0;
#pragma unroll
            for (int k = 0; k < B; k++) {
                if (rr + k < r1) rt[(rr + k) * RADIX + d] = run;
                run += v[k];
            }
        }
        u64 all;
        C.pbase[(i64)q * RADIX + d] = (u64)C.segs[q].stage_base + block_excl_scan<u64>(run, s_scan, all);
    }
}

// First position per digit (thread d) of local block bl of product q: digit
// base + the range's first position + the counts of the range's earlier
// blocks (at most RNG - 1 loads, in batches).  Without the range scan (every
// product has at most RSUM_MAX ranges) the digit bases and the range's first
// position are summed here from the product's range counters.  Whole
// workgroup (a block scan).
template <int NT>
__device__ inline u64 block_start(const Ctx &C, int pass, int q, i64 bl, u64 stage_base, u64 *s_scan64) {
    constexpr int B = 8;
    const int d = threadIdx.x;
    const bool dig = d < RADIX;
    const u64 *rt = C.rtot + (i64)(pass & 1) * C.nrng * RADIX;
    const i64 b0 = C.chpre[q], r0 = C.rpre[q];
    const i64 r = bl / RNG;
    u64 pos;
    if (C.rscan) {
        pos = dig ? C.pbase[(i64)q * RADIX + d] + rt[(r0 + r) * RADIX + d] : 0;
    } else {
        const i64 nr = C.rpre[q + 1] - r0;  // at most RSUM_MAX
        u64 before = 0, total = 0;
        if (dig) {
            for (int k0 = 0; k0 < RSUM_MAX; k0 += B) {
                u64 v[B];
#pragma unroll
                for (int k = 0; k < B; k++) v[k] = k0 + k < nr ? rt[(r0 + k0 + k) * RADIX + d] : 0;
#pragma unroll
                for (int k = 0; k < B; k++) {
                    total += v[k];
                    if (k0 + k < r) before += v[k];
                }
            }
        }
        u64 all;
        pos = stage_base + block_excl_scan<u64, NT>(total, s_scan64, all) + before;
    }
    if (dig) {
        for (i64 bb = r * RNG; bb < bl; bb += B) {
            u64 v[B];
#pragma unroll
            for (int k = 0; k < B; k++) v[k] = bb + k < bl ? C.ctot[(b0 + bb + k) * RADIX + d] : 0;
#pragma unroll
            for (int k = 0; k < B; k++) pos += v[k];
        }
    }
    return pos;
}

// ---------------------------------------------------------------------------
// k_onesweep: one stable LSD radix pass over digit `pass` of every product's
// items: (key, coefficient) for SEG_COMBINE, the pair index alone for
// SEG_RAW (see SM_*).  A workgroup takes one sort block at a time and its
// partitions (PART consecutive items) in order.  Ranks come from per-wave
// ballot "match" masks (peers with the same digit) and per-wave digit
// counters in LDS; a digit's position is the block's running position for
// that digit, which starts from block_start's offsets and grows by each
// partition's digit count.  WK: the pass also writes the keys (always for
// staged items; for pair indices only in the last pass, for the reduction).
// ---------------------------------------------------------------------------
constexpr int OS_IPT = PART / OS_T;  // items per thread (OS_T = 512: 8 waves)

// DG: the pass keeps each item's digit rather than its key in LDS (passes of
// regenerated keys; one that writes keys regenerates them again), which
// leaves LDS room for a copy of the operands' compressed keys.

// The key ck(alpha_i) + ck(beta_j) of pair index x = i*nb + j.
template <typename K>
__device__ inline K regen_key(const OsSeg &s, const K *kf, const K *kg, u32 x) {
    const u32 i = div32(x, s.nb_div);
    return kf[i] + kg[x - i * s.nb];
}
template <typename K, typename V, bool DG = false>
struct OsSmem {
    static constexpr int NW = OS_T / 64;
    // waves per SIMD the registers are held to (with the LDS copy of the
    // operand keys, two workgroups per CU)
    static constexpr int OCC = (DG ? 2 : os_resident((int)sizeof(K), (int)sizeof(V))) * OS_T / 256;
    using KS = std::conditional_t<DG, unsigned char, K>;
    KS k[PART];
    V v[PART];
    u32 wh[NW][RADIX];
    u32 loff[RADIX];
    u32 goff[RADIX];  // digit's first position minus its local offset, from the product start, mod 2^32
    u32 scan[NW];
    u64 scan64[NW];
};

// Loads partition c (n items, warp-striped: item k of lane l in wave w is
// w*64*OS_IPT + k*64 + l) into registers.  Items past the end of a partial
// partition carry the all-ones key: they rank last in the last digit, i.e. at
// sorted positions [n, PART), so the valid items' positions are unaffected;
// only that digit's count and the global writes account for them.
template <typename K, typename V, int SM>
__device__ __forceinline__ void os_load(const Ctx &C, const OsSeg &s, i64 c, int n, const K *__restrict__ kin,
                                        const V *__restrict__ vin, const K *kf, const K *kg, K (&key)[OS_IPT],
                                        V (&val)[OS_IPT]) {
    // an opaque copy of the thread index: keeps the per-item index and
    // address arithmetic here instead of holding sixteen of each in
    // registers for the whole kernel
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int wbase = (tid >> 6) * 64 * OS_IPT + (tid & 63);
    const i64 start = s.lo + c * PART;
    // kf, kg: f's and g's compressed keys (an LDS copy or global memory)
    if constexpr (SM == SM_GEN) {
#pragma unroll
        for (int k = 0; k < OS_IPT; k++) {
            const int idx = wbase + k * 64;
            const u32 x = (u32)(c * PART + idx);
            const u32 i = div32(x, s.nb_div);
            key[k] = idx < n ? kf[i] + kg[x - i * s.nb] : ~(K)0;
            val[k] = (V)x;
        }
    } else if constexpr (SM == SM_INDEX) {
#pragma unroll
        for (int k = 0; k < OS_IPT; k++) {
            const int idx = wbase + k * 64;
            val[k] = idx < n ? vin[start + idx] : (V)0;
        }
#pragma unroll
        for (int k = 0; k < OS_IPT; k++) {
            const int idx = wbase + k * 64;
            const u32 i = div32((u32)val[k], s.nb_div);
            key[k] = idx < n ? kf[i] + kg[(u32)val[k] - i * s.nb] : ~(K)0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < OS_IPT; k++) {
            const int idx = wbase + k * 64;
            key[k] = idx < n ? kin[start + idx] : ~(K)0;
        }
        // payloads are only permuted: their loads overlap the ranking
#pragma unroll
        for (int k = 0; k < OS_IPT; k++) {
            const int idx = wbase + k * 64;
            val[k] = idx < n ? vin[start + idx] : (V)0;
        }
    }
}

// One partition (c, n items) whose items are in key/val.  Ranks them, places
// them in LDS in sorted order, then, while the sorted items are written out,
// loads the next partition (cn, nn items; nn = 0: none) into key/val.  `run`
// (thread d) is digit d's next position in the staging buffer.  Expects the
// wave digit counters S.wh zeroed and leaves them zeroed.
template <typename K, typename V, int SM, bool WK, bool DG>
__device__ __forceinline__ void os_partition(Ctx &C, OsSmem<K, V, DG> &S, const OsSeg &s, int pass, int n, i64 cn,
                                             int nn, const K *__restrict__ kin, const V *__restrict__ vin,
                                             K *__restrict__ kout, V *__restrict__ vout, K (&key)[OS_IPT],
                                             V (&val)[OS_IPT], u64 &run, const K *kf, const K *kg) {
    constexpr int NW = OsSmem<K, V, DG>::NW;
    using KS = typename OsSmem<K, V, DG>::KS;
    const int shift = C.dsh[pass];
    const u32 dmask = (1u << C.dbits[pass]) - 1u;
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const u32 w = (u32)tid >> 6;
    u32 rk[OS_IPT];
    // Per-wave stable ranking.  A lane's peers are the lanes whose digit
    // equals its own: per digit bit, the ballot of lanes with the bit set,
    // XNOR this lane's bit widened to all ones or zeros, keeps the lanes that
    // agree (every lane is active here: missing items carry a key).  Each
    // lane reads its digit's wave counter, and the first lane of each peer
    // group adds the group's size without waiting for the value (a wave's
    // LDS operations stay in order, so the next slot reads the sum).
#pragma unroll
    for (int k = 0; k < OS_IPT; k++) {
        const u32 d = (u32)((key[k] >> shift) & dmask);
        u32 t[RADIX_BITS];
        u64 m[RADIX_BITS];
#pragma unroll
        for (int b = 0; b < RADIX_BITS; b++) {
            t[b] = (u32)((i32)(d << (31 - b)) >> 31);
            asm volatile("" : "+v"(t[b]));  // the ballot tests t itself, which the masks reuse
        }
#pragma unroll
        for (int b = 0; b < RADIX_BITS; b++) m[b] = __ballot(t[b] != 0);
        // peers & ~(t ^ m): truth table 0x84 over (t, peers, m)
        u32 pl = ~0u, ph = ~0u;
#pragma unroll
        for (int b = 0; b < RADIX_BITS; b++) {
            pl = __builtin_amdgcn_bitop3_b32(t[b], pl, (u32)m[b], 0x84);
            ph = __builtin_amdgcn_bitop3_b32(t[b], ph, (u32)(m[b] >> 32), 0x84);
        }
        const u32 before = __builtin_amdgcn_mbcnt_hi(ph, __builtin_amdgcn_mbcnt_lo(pl, 0u));
        rk[k] = S.wh[w][d] + before;
        if (before == 0) atomicAdd(&S.wh[w][d], (u32)(__popc(pl) + __popc(ph)));
    }
    __syncthreads();
    // digit totals, wave prefixes, local digit offsets (thread d < RADIX
    // holds digit d); this partition's digit positions from the block's
    // running positions
    const int d = tid;
    const bool dig = d < RADIX;
    u32 tot = 0;
    if (dig) {
#pragma unroll
        for (int ww = 0; ww < NW; ww++) {
            const u32 x = S.wh[ww][d];
            S.wh[ww][d] = tot;
            tot += x;
        }
    }
    u32 all;
    const u32 loff = block_excl_scan<u32, OS_T>(tot, S.scan, all);
    if (dig) {
        if (d == dmask) tot -= (u32)(PART - n);  // the items past n rank last in the top digit
        S.loff[d] = loff;
        S.goff[d] = (u32)(run - (u64)s.lo) - loff;
        run += tot;
    }
    __syncthreads();
    // keys and payloads into LDS in sorted order
#pragma unroll
    for (int k = 0; k < OS_IPT; k++) {
        const u32 dk = (u32)((key[k] >> shift) & dmask);
        const u32 pos = S.loff[dk] + S.wh[w][dk] + rk[k];
        S.k[pos] = DG ? (KS)dk : (KS)key[k];
        S.v[pos] = val[k];
    }
    __syncthreads();
    if (nn > 0) os_load<K, V, SM>(C, s, cn, nn, kin, vin, kf, kg, key, val);
#pragma unroll
    for (int e = 0; e < NW * RADIX / OS_T; e++) (&S.wh[0][0])[tid + e * OS_T] = 0;
    // sorted item i of digit d goes to goff[d] + i; a position outside the
    // product (only possible with inconsistent counts) is flagged, and in a
    // full partition clamped so that the stores stay unconditional
    K *kq = kout + s.lo;
    V *vq = vout + s.lo;
    const u32 span32 = (u32)s.n_q;
    bool bad = false;
    if (n == PART) {
#pragma unroll
        for (int k = 0; k < OS_IPT; k++) {
            const u32 i = (u32)tid + (u32)(k * OS_T);
            const KS kv = S.k[i];
            const V vv = S.v[i];
            u32 rel = S.goff[DG ? (u32)kv : (u32)(kv >> shift) & dmask] + i;
            bad |= rel >= span32;
            rel = min(rel, span32 - 1u);
            if constexpr (WK) kq[rel] = DG ? regen_key(s, kf, kg, (u32)vv) : (K)kv;
            vq[rel] = vv;
        }
    } else {
#pragma unroll
        for (int k = 0; k < OS_IPT; k++) {
            const u32 i = (u32)tid + (u32)(k * OS_T);
            if (i < (u32)n) {
                const KS kv = S.k[i];
                const u32 rel = S.goff[DG ? (u32)kv : (u32)(kv >> shift) & dmask] + i;
                if (rel < span32) {
                    const V vv = S.v[i];
                    if constexpr (WK) kq[rel] = DG ? regen_key(s, kf, kg, (u32)vv) : (K)kv;
                    vq[rel] = vv;
                } else {
                    bad = true;
                }
            }
        }
    }
    if (bad) atomicOr(&C.counters[CNT_ERR_SPIN], 2u);
    __syncthreads();
}

// KL: regenerated keys read each product's compressed operand keys from a
// copy in dynamic LDS (every product of the launch fits), else from global
// memory.
template <typename K, typename V, int SM, bool WK, bool KL>
__global__ __launch_bounds__(OS_T) __attribute__((amdgpu_waves_per_eu(OsSmem<K, V, KL && SM != SM_STAGED>::OCC))) void k_onesweep(Ctx C, int pass, const K *__restrict__ kin,
                                                        const V *__restrict__ vin, K *__restrict__ kout,
                                                        V *__restrict__ vout) {
    constexpr bool DG = KL && SM != SM_STAGED;
    constexpr int NW = OsSmem<K, V, DG>::NW;
    __shared__ OsSmem<K, V, DG> S;
    __shared__ i64 s_b;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    K *s_ck = (K *)s_dyn;
    const K *ck = (const K *)C.ck;
    const i64 nblk = C.chpre[C.nseg];
    int cur_q = -1;
    OsSeg sq{};
    const K *kf = nullptr, *kg = nullptr;
    for (int e = threadIdx.x; e < NW * RADIX; e += OS_T) (&S.wh[0][0])[e] = 0;
    K key[OS_IPT];
    V val[OS_IPT];
    while (true) {
        // blocks are independent: the queue only balances uneven products
        if (threadIdx.x == 0) s_b = (i64)atomicAdd(&C.counters[CNT_SORT + pass], 1u);
        __syncthreads();
        const i64 b = s_b;
        __syncthreads();
        if (b >= nblk) break;
        const int q = seg_search(C.chpre, C.nseg, b);
        if (q != cur_q) {
            sq = load_os_seg(C, q);
            cur_q = q;
            kf = ck + sq.ck_f;
            if constexpr (KL) {  // the previous block ended with a barrier
                const i64 m = sq.ck_g - sq.ck_f + sq.nb;  // f's and g's compressed keys, contiguous
                for (i64 t = threadIdx.x; t < m; t += OS_T) s_ck[t] = kf[t];
                kf = s_ck;
                __syncthreads();
            }
            kg = kf + (sq.ck_g - sq.ck_f);
        }
        const i64 bl = b - C.chpre[q];
        const i64 c0 = bl * C.pblk;
        const i64 c1 = min((sq.n_q + PART - 1) / PART, c0 + C.pblk);
        os_load<K, V, SM>(C, sq, c0, (int)min((i64)PART, sq.n_q - c0 * PART), kin, vin, kf, kg, key, val);
        u64 run = block_start<OS_T>(C, pass, q, bl, (u64)sq.lo, S.scan64);
        for (i64 c = c0; c < c1; c++) {
            const int n = (int)min((i64)PART, sq.n_q - c * PART);
            const int nn = c + 1 < c1 ? (int)min((i64)PART, sq.n_q - (c + 1) * PART) : 0;
            os_partition<K, V, SM, WK, DG>(C, S, sq, pass, n, c + 1, nn, kin, vin, kout, vout, key, val, run, kf, kg);
        }
    }
}

// ---------------------------------------------------------------------------
// Result slots without look-back.  k_head_count: the number of runs (distinct
// keys) that start in each reduce partition of the sorted staging, into
// pcnt[p]; k_head_scan: per product, the exclusive prefix over its partitions,
// i.e. the slot of each partition's first run.
// ---------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(NTHREADS) void k_head_count(Ctx C, const K *__restrict__ kin) {
    __shared__ u32 s_scan[NTHREADS / 64];
    const i64 nparts = C.ppre[C.nseg];
    int cur_q = -1;
    OsSeg sq{};
    for (i64 p = blockIdx.x; p < nparts; p += gridDim.x) {
        const int q = (cur_q >= 0 && p < sq.first + (sq.n_q + PART - 1) / PART) ? cur_q : seg_search(C.ppre, C.nseg, p);
        if (q != cur_q) {
            sq = load_os_seg(C, q);
            cur_q = q;
        }
        const i64 c = p - sq.first;
        const i64 start = sq.lo + c * PART;
        const int n = (int)min((i64)PART, sq.n_q - c * PART);
        // loads at clamped positions (n >= 1; a product's first item reads
        // itself as its predecessor), every value taken after all are issued:
        // otherwise each load sits under its bounds branch and is waited for there
        K key[IPT], prev[IPT];
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const int i = (int)threadIdx.x + r * NTHREADS;
            const i64 at = start + (i < n ? i : n - 1);
            key[r] = kin[at];
            prev[r] = kin[(at > sq.lo) ? at - 1 : at];
        }
#pragma unroll
        for (int r = 0; r < IPT; r++) asm volatile("" : "+v"(key[r]), "+v"(prev[r]));
        u32 h = 0;
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const int i = (int)threadIdx.x + r * NTHREADS;
            if (i < n && ((i == 0 && c == 0) || key[r] != prev[r])) h++;
        }
        u32 tot;
        (void)block_excl_scan<u32>(h, s_scan, tot);
        if (threadIdx.x == 0) C.pcnt[p] = tot;
    }
}

constexpr int HS_T = 1024;  // k_head_scan threads (a product's partitions in few steps)

__global__ __launch_bounds__(HS_T) void k_head_scan(Ctx C) {
    __shared__ u64 s_scan[HS_T / 64];
    for (int q = blockIdx.x; q < C.nseg; q += gridDim.x) {
        const i64 p0 = C.ppre[q], np = C.ppre[q + 1] - p0;
        const i64 B = (np + HS_T - 1) / HS_T;  // partitions per thread, blocked
        const i64 b0 = p0 + (i64)threadIdx.x * B, b1 = min(p0 + np, b0 + B);
        u64 t = 0;
#pragma unroll 8
        for (i64 p = b0; p < b1; p++) t += C.pcnt[p];
        u64 all;
        u64 run = block_excl_scan<u64, HS_T>(t, s_scan, all);
#pragma unroll 8
        for (i64 p = b0; p < b1; p++) {
            const u64 v = C.pcnt[p];
            C.pcnt[p] = run;
            run += v;
        }
    }
}

// ---------------------------------------------------------------------------
// k_reduce: sorted staging -> result.  SEG_RAW items carry the pair index,
// from which each term product a_i * b_j is formed.  FP64: a run of equal
// keys is summed by the thread that owns its first element, left to right in
// staging order (the row-major (i, j) order of the pp-matrix, as the sort is
// stable and SEG_RAW items start in index order).  Exact rings: each thread
// sums the runs inside its items and a segmented scan over the workgroup
// completes the runs that cross threads.  The partition's last run is
// followed into the next partitions by one wave, 64 items at a time, adding
// in order.  Every run gets the result slot given by its rank among the
// product's runs, which is known from the keys alone: the partition's first
// slot comes from k_head_count and k_head_scan.  A run whose sum cancels to
// zero leaves a slot with a zero coefficient; k_zero_compact removes those
// slots afterwards (only products that have any).  Results are staged in LDS
// and written out contiguously with the key decompressed to the packed
// exponent layout.
// ---------------------------------------------------------------------------

// The fields of one product that the reduction uses, kept in scalar
// registers while consecutive partitions belong to the same product.
struct RdSeg {
    i64 first, n_q, lo, nparts, cap, var_off;
    const u64 *fc, *gc;
    u64 *hk, *hc;
    i64 *n_out;
    u64 lo_key;
    u32 nb;
    Div32 nb_div;
};

template <typename T>
__device__ inline T *uniform_ptr(T *p) {
    return (T *)(uintptr_t)uniform64((i64)(uintptr_t)p);
}

__device__ inline RdSeg load_rd_seg(const Ctx &C, int q) {
    const DevSeg &s = C.segs[q];
    RdSeg r;
    r.first = uniform64(C.ppre[q]);
    r.n_q = uniform64(C.dyn[q].n);
    r.nparts = uniform64(C.dyn[q].nparts);
    r.lo = uniform64(s.stage_base);
    r.cap = uniform64(s.cap);
    r.var_off = uniform64(s.var_off);
    r.fc = uniform_ptr(s.fc);
    r.gc = uniform_ptr(s.gc);
    r.hk = uniform_ptr(s.hk);
    r.hc = uniform_ptr(s.hc);
    r.n_out = uniform_ptr(s.n_out);
    r.lo_key = (u64)uniform64((i64)s.lo_key);
    r.nb = uniform32((u32)s.nb);
    r.nb_div.m = uniform32(s.nb_div.m);
    r.nb_div.s1 = uniform32(s.nb_div.s1);
    r.nb_div.s2 = uniform32(s.nb_div.s2);
    r.nb_div.d = uniform32(s.nb_div.d);
    return r;
}

template <typename K, typename V, int RING>
__device__ inline u64 item_value_rd(const RdSeg &s, V v) {
    if constexpr (sizeof(V) == 8) {
        return (u64)v;
    } else {
        const u32 i = div32((u32)v, s.nb_div);
        const u32 j = (u32)v - i * s.nb;
        return ring_mul<RING>(s.fc[i], s.gc[j]);
    }
}

constexpr u32 TAG_ZCOMPACT = 201u;
// The reduction runs 512-thread workgroups with 8 items per thread (one
// partition of PART items): the same LDS per workgroup as 256 x 16, twice the
// waves per CU to hide its load and gather latencies.
constexpr int RED_T = 512, RED_IPT = PART / RED_T;

template <typename K, typename V, int RING>
// three workgroups of 4-byte keys per CU (LDS), two of 8-byte keys
__global__ __launch_bounds__(RED_T) __attribute__((amdgpu_waves_per_eu(sizeof(K) == 4 ? 6 : 4))) void k_reduce(Ctx C, const K *__restrict__ kin, const V *__restrict__ vin) {
    constexpr int PADN = PART + PART / 16;
    __shared__ K s_k[PADN];
    __shared__ u64 s_v[PADN];
    __shared__ u32 s_scan[RED_T / 64];
    __shared__ int s_wp[RED_T / 64];
    __shared__ int s_cont;
    __shared__ u64 s_ws[RED_T / 64];
    __shared__ i64 s_p, s_pn;
    __shared__ u64 s_base;
    __shared__ u32 s_z;
    auto pad = [](int i) { return i + (i >> 4); };
    const i64 nparts = C.ppre[C.nseg];
    u32 *ticket = &C.counters[CNT_REDUCE];
    if (threadIdx.x == 0) s_p = (i64)atomicAdd(ticket, 1u);
    __syncthreads();
    i64 p = s_p;
    int q = -1;
    RdSeg s{};
    while (p < nparts) {
        if (q < 0 || p >= s.first + s.nparts) {
            q = seg_search(C.ppre, C.nseg, p);
            s = load_rd_seg(C, q);
        }
        const i64 first = s.first;
        const i64 c = p - first;
        const i64 n_q = s.n_q;
        const i64 start = s.lo + c * PART;
        const i64 send = s.lo + n_q;
        const int n = (int)min((i64)PART, n_q - c * PART);
        if (threadIdx.x == 0) {
            s_z = 0;
            s_cont = -1;
        }
        // opaque thread index: per-item index arithmetic stays in the loop
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        // keys and raw payloads, register-blocked and coalesced
        K kr[RED_IPT];
        V vr[RED_IPT];
#pragma unroll
        for (int r = 0; r < RED_IPT; r++) {
            const int i = tid + r * RED_T;
            kr[r] = i < n ? kin[start + i] : (K)0;
            vr[r] = i < n ? vin[start + i] : (V)0;
        }
#pragma unroll
        for (int r = 0; r < RED_IPT; r++) {
            const int i = tid + r * RED_T;
            if (i < n) s_k[pad(i)] = kr[r];
        }
        const K prevk = c > 0 ? kin[start - 1] : (K)0;
        __syncthreads();
        // run heads among this thread's items [b0, b0 + RED_IPT); publish the count
        const int b0 = tid * RED_IPT;
        u32 hm = 0;
        {
            K kp = b0 == 0 ? prevk : s_k[pad(b0 > 0 ? b0 - 1 : 0)];
            bool hp = !(b0 == 0 && c == 0);
#pragma unroll
            for (int r = 0; r < RED_IPT; r++) {
                if (b0 + r < n) {
                    const K key = s_k[pad(b0 + r)];
                    if (!hp || key != kp) hm |= 1u << r;
                    kp = key;
                    hp = true;
                }
            }
        }
        u32 total;
        const u32 off = block_excl_scan<u32, RED_T>((u32)__popc(hm), s_scan, total);
        if (threadIdx.x == 0) s_base = C.pcnt[p];
        // item values: the operand gathers of all of a thread's items in flight together
        {
            u64 xv[RED_IPT];
            if constexpr (sizeof(V) == 8) {
#pragma unroll
                for (int r = 0; r < RED_IPT; r++) xv[r] = (u64)vr[r];
            } else {
                u64 fa[RED_IPT], gb[RED_IPT];
#pragma unroll
                for (int r = 0; r < RED_IPT; r++) {
                    const int i = tid + r * RED_T;
                    const u32 a = i < n ? div32((u32)vr[r], s.nb_div) : 0u;
                    const u32 b = i < n ? (u32)vr[r] - a * (u32)s.nb : 0u;
                    fa[r] = s.fc[a];
                    gb[r] = s.gc[b];
                }
#pragma unroll
                for (int r = 0; r < RED_IPT; r++) xv[r] = ring_mul<RING>(fa[r], gb[r]);
            }
#pragma unroll
            for (int r = 0; r < RED_IPT; r++) {
                const int i = tid + r * RED_T;
                if (i < n) s_v[pad(i)] = xv[r];
            }
        }
        __syncthreads();
        // each head's run sum replaces the head's value in LDS
        if constexpr (RING == RING_F64) {
            // FP64: the head's thread adds its run left to right (the oracle's order)
            {
                int open = -1;
                u64 acc = 0;
#pragma unroll
                for (int r = 0; r < RED_IPT; r++) {
                    if (b0 + r < n) {
                        const u64 v = s_v[pad(b0 + r)];
                        if ((hm >> r) & 1) {
                            if (open >= 0) s_v[pad(b0 + open)] = acc;
                            open = r;
                            acc = v;
                        } else if (open >= 0) {
                            acc = ring_add<RING>(acc, v);
                        }
                    }
                }
                if (open >= 0) {
                    // the last run may continue into the next threads' items and partitions
                    const K key = s_k[pad(b0 + open)];
                    int j = b0 + RED_IPT;
                    while (j < n && s_k[pad(j)] == key) acc = ring_add<RING>(acc, s_v[pad(j++)]);
                    s_v[pad(b0 + open)] = acc;
                    if (j >= n && n > 0) s_cont = b0 + open;  // continues past the partition
                }
            }
        } else {
            // exact rings: a segmented scan over the threads.  Each thread
            // sums the runs that start and end inside its items, and offers
            // (position of its last head or -1, sum from there to its end; or
            // with no head, the sum of all its items); the scan hands each
            // thread the run still open on its left, which it completes when
            // it holds a head.  The thread holding the partition's last item
            // completes the last open run, following it into the next
            // partitions when it continues there.
            int lp = -1;
            u64 ls = 0, pre = 0;
#pragma unroll
            for (int r = 0; r < RED_IPT; r++) {
                if (b0 + r < n) {
                    const u64 v = s_v[pad(b0 + r)];
                    if ((hm >> r) & 1) {
                        if (lp >= 0) s_v[pad(lp)] = ls;
                        lp = b0 + r;
                        ls = v;
                    } else if (lp >= 0) {
                        ls = ring_add<RING>(ls, v);
                    } else {
                        pre = ring_add<RING>(pre, v);
                    }
                }
            }
            // inclusive scan of (p, s): (p1, s1) + (p2, s2) = p2 >= 0 ? (p2, s2) : (p1, s1 + s2)
            int ip = lp;
            u64 is = lp >= 0 ? ls : pre;
            const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int po = __shfl_up(ip, off, 64);
                const u64 so = __shfl_up(is, off, 64);
                if (lane >= off && ip < 0) {
                    ip = po;
                    is = ring_add<RING>(so, is);
                }
            }
            if (lane == 63) {
                s_wp[wv] = ip;
                s_ws[wv] = is;
            }
            int ep = __shfl_up(ip, 1, 64);
            u64 es = __shfl_up(is, 1, 64);
            if (lane == 0) {
                ep = -1;
                es = 0;
            }
            __syncthreads();
            // the carry from earlier waves, then this wave's earlier lanes
            int cp = -1;
            u64 cs = 0;
            for (int w2 = 0; w2 < wv; w2++) {
                if (s_wp[w2] >= 0) {
                    cp = s_wp[w2];
                    cs = s_ws[w2];
                } else {
                    cs = ring_add<RING>(cs, s_ws[w2]);
                }
            }
            if (ep >= 0) {
                cp = ep;
                cs = es;
            } else {
                cs = ring_add<RING>(cs, es);
            }
            if (lp >= 0 && cp >= 0) s_v[pad(cp)] = ring_add<RING>(cs, pre);  // the open run ends before my first head
            if (b0 < n && b0 + RED_IPT >= n) {
                // the partition's last open run: combine the carry with this thread's part
                int fp = lp >= 0 ? lp : cp;
                u64 fs = lp >= 0 ? ls : ring_add<RING>(cs, pre);
                if (fp >= 0) {
                    s_v[pad(fp)] = fs;
                    s_cont = fp;  // may continue past the partition
                }
            }
            // a run still open at this thread's end is completed by the thread
            // holding the next head or the partition's last item
            __syncthreads();
        }
        // the partition's last run may continue into the next partitions: wave 0
        // reads 64 items at a time and adds the matching prefix (left to right)
        if constexpr (RING == RING_F64) __syncthreads();
        if (tid < 64) {
            const int cp = s_cont;
            if (cp >= 0) {
                const K key = s_k[pad(cp)];
                u64 acc = s_v[pad(cp)];
                for (i64 g = start + n; g < send; g += 64) {
                    const i64 gi = g + tid;
                    const bool m = gi < send && kin[gi] == key;
                    const u64 mb = __ballot(m);
                    const int cnt = mb == ~0ull ? 64 : __builtin_ctzll(~mb);
                    const u64 v = tid < cnt ? item_value_rd<K, V, RING>(s, vin[gi]) : 0;
                    for (int t = 0; t < cnt; t++) acc = ring_add<RING>(acc, __shfl(v, t, 64));
                    if (cnt < 64) break;
                }
                if (tid == 0) s_v[pad(cp)] = acc;
            }
        }
        __syncthreads();
        u32 tk = 0;
        if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);  // next partition
        // gather this thread's runs, then stage them by slot in LDS
        K ok[RED_IPT];
        u64 ov[RED_IPT];
#pragma unroll
        for (int r = 0; r < RED_IPT; r++) {
            ok[r] = s_k[pad(b0 + r)];
            ov[r] = s_v[pad(b0 + r)];
        }
        __syncthreads();
        u32 o = off, zc = 0;
#pragma unroll
        for (int r = 0; r < RED_IPT; r++) {
            if ((hm >> r) & 1) {
                s_k[o] = ok[r];
                s_v[o] = ov[r];
                zc += ring_is_zero<RING>(ov[r]) ? 1u : 0u;
                o++;
            }
        }
        if (zc) atomicAdd(&s_z, zc);
        __syncthreads();
        const u64 base = s_base;
        const VarParam *vp = C.vars + s.var_off;
        for (int i = threadIdx.x; i < (int)total; i += RED_T) {
            const u64 pos = base + i;
            if ((i64)pos < s.cap) {
                s.hk[pos] = decompress<K>(s_k[i], vp, C.nvars, s.lo_key);
                s.hc[pos] = s_v[i];
            }
        }
        if (threadIdx.x == 0) {
            if (c == s.nparts - 1) {
                *s.n_out = (i64)(base + total);
                C.dyn[q].heads = (i64)(base + total);
            }
            if (s_z) {
                atomicAdd(&C.dyn[q].zeros, (unsigned long long)s_z);
                atomicOr(&C.counters[CNT_ZEROS], 1u);
            }
            s_pn = (i64)tk;
        }
        __syncthreads();
        p = s_pn;
    }
}

// ---------------------------------------------------------------------------
// k_zero_compact: removes the cancelled (zero-coefficient) slots that
// k_reduce left in the results of products that have any, in place and in
// order.  Partition c of product q covers result slots [c*PART, (c+1)*PART)
// up to min(heads, capacity).  A partition's writes land at or below its own
// slots, and only after every earlier partition has published, i.e. read its
// slots; so in-place compaction is safe.  When the slots exceed the capacity
// (truncation), *n_out reports the slot count, which is the capacity that
// avoids it, and the coefficients after the compacted prefix are zeroed.
// ---------------------------------------------------------------------------
template <int RING>
__global__ __launch_bounds__(NTHREADS) void k_zero_compact(Ctx C) {
    __shared__ u64 s_k[PART];
    __shared__ u64 s_v[PART];
    __shared__ u32 s_scan[NTHREADS / 64];
    __shared__ i64 s_p;
    __shared__ u64 s_base;
    if (__hip_atomic_load(&C.counters[CNT_ZEROS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
    const i64 nparts = C.ppre[C.nseg];
    while (true) {
        if (threadIdx.x == 0) s_p = (i64)atomicAdd(&C.counters[CNT_ZCOMPACT], 1u);
        __syncthreads();
        const i64 p = s_p;
        __syncthreads();
        if (p >= nparts) break;
        const int q = seg_search(C.ppre, C.nseg, p);
        const DevSeg &s = C.segs[q];
        if (C.dyn[q].zeros == 0) continue;
        const i64 heads = C.dyn[q].heads;
        const i64 lim = min(heads, s.cap);
        const i64 first = C.ppre[q];
        const i64 lo = (p - first) * PART;
        if (lo >= lim) continue;
        const int n = (int)min((i64)PART, lim - lo);
        for (int i = threadIdx.x; i < n; i += NTHREADS) {
            s_k[i] = s.hk[lo + i];
            s_v[i] = s.hc[lo + i];
        }
        __syncthreads();
        const int b0 = (int)threadIdx.x * IPT;
        u64 kk[IPT], vv[IPT];
        u32 m = 0;
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            kk[r] = s_k[b0 + r];
            vv[r] = s_v[b0 + r];
            if (b0 + r < n && !ring_is_zero<RING>(vv[r])) m |= 1u << r;
        }
        u32 total;
        const u32 off = block_excl_scan<u32>((u32)__popc(m), s_scan, total);
        if (threadIdx.x < 64) {
            if (threadIdx.x == 0) lb_publish(C.look_red + p, first, p, TAG_ZCOMPACT, total);
            const u64 pre = lookback_wave_resolve(C.look_red, first, p, TAG_ZCOMPACT, total, &C.counters[CNT_ERR_SPIN]);
            if (threadIdx.x == 0) s_base = pre;
        }
        __syncthreads();
        u32 o = off;
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            if ((m >> r) & 1) {
                s_k[o] = kk[r];
                s_v[o] = vv[r];
                o++;
            }
        }
        __syncthreads();
        const u64 base = s_base;
        for (int i = threadIdx.x; i < (int)total; i += NTHREADS) {
            s.hk[base + i] = s_k[i];
            s.hc[base + i] = s_v[i];
        }
        if (lo + n == lim) {
            // last partition: clear the coefficients behind the compacted result
            for (i64 i = (i64)(base + total) + threadIdx.x; i < lim; i += NTHREADS) s.hc[i] = 0;
            if (threadIdx.x == 0) *s.n_out = heads > s.cap ? heads : (i64)(base + total);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_compact: dense path.  Cells of each product's degree box, in mixed-radix
// (= lexicographic) order, become the sorted result; a cell is a term when its
// accumulated value is non-zero.
// ---------------------------------------------------------------------------
template <int RING>
__global__ __launch_bounds__(NTHREADS) void k_compact(Ctx C) {
    __shared__ u32 s_scan[NTHREADS / 64];
    __shared__ i64 s_p;
    __shared__ u64 s_base;
    const i64 tb = C.tb_cmp;
    while (true) {
        if (threadIdx.x == 0) s_p = (i64)atomicAdd(&C.counters[CNT_COMPACT], 1u) * tb;
        __syncthreads();
        const i64 p0 = s_p;
        if (p0 >= C.ndparts) break;
        __syncthreads();
        for (i64 p = p0; p < min(p0 + tb, C.ndparts); p++) {
        const i32 ds = seg_search(C.dpart_pre, C.ndseg, p);
        const int q = C.dseg[ds];
        const DevSeg &s = C.segs[q];
        const i64 first = C.dpart_pre[ds];
        const i64 c = p - first;
        const i64 nparts = C.dpart_pre[ds + 1] - first;
        const i64 c0 = c * PART;
        const i64 b0 = c0 + (i64)threadIdx.x * IPT;
        u64 val[IPT];
        u32 mask = 0;
        // the product's box in registers, and every load at a clamped cell
        // (the box has at least one), so that the IPT loads are in flight
        // together instead of one per branch
        const i64 sbound = uniform64(s.stage_bound);
        const u64 *boxq = C.box + uniform64(s.stage_base);
        const i64 last = sbound - 1;
        u64 raw[IPT];
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const i64 cell = b0 + r;
            raw[r] = boxq[cell < last ? cell : last];
        }
        // every value is taken here (the compiler would otherwise move each
        // load under its cell's bounds branch and wait for it there)
#pragma unroll
        for (int r = 0; r < IPT; r++) asm volatile("" : "+v"(raw[r]));
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            const bool in = b0 + r < sbound;
            val[r] = in ? ring_cell_final<RING>(raw[r]) : 0;
            if (in && !ring_is_zero<RING>(val[r])) mask |= 1u << r;
        }
        const u32 cnt = (u32)__popc(mask);
        u32 total;
        const u32 off = block_excl_scan<u32>(cnt, s_scan, total);
        if (threadIdx.x < 64) {
            const u64 pre = lookback_wave(C.look_cmp, first, p, 201u, total, &C.counters[CNT_ERR_SPIN]);
            if (threadIdx.x == 0) s_base = pre;
        }
        __syncthreads();
        const u64 base = s_base + off;
        const VarParam *vp = C.vars + s.var_off;
        u32 r2 = 0;
#pragma unroll
        for (int r = 0; r < IPT; r++) {
            if (!(mask & (1u << r))) continue;
            const u64 pos = base + r2++;
            if ((i64)pos < s.cap) {
                s.hk[pos] = decompress<u64>((u64)(b0 + r), vp, C.nvars, s.lo_key);
                s.hc[pos] = val[r];
            }
        }
        if (c == nparts - 1 && threadIdx.x == 0) *s.n_out = (i64)(s_base + total);
        __syncthreads();
        }
    }
}

}  // namespace pm

#include "pm_ival.hpp"
#include "pm_bkt.hpp"
static_assert(pm::BK_TL == 512, "workspace layout sizes the tile lists for 512 bins");

// ===========================================================================
// Host-side launch sequence
// ===========================================================================
#include <string.h>

#include "pm_launch.hpp"

#include <mutex>
#include <string>
#include <vector>

namespace pm {

// Event-pair recorder around kernel launches (see pm_profile_enable).
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<std::string> names;
    struct Rec {
        int name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    std::vector<double> ms;
    std::vector<int64_t> count;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    int begin(const char *name, hipStream_t st) {
        std::lock_guard<std::mutex> lk(mu);
        if (!on) return -1;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return -1;
        int id = -1;
        for (size_t i = 0; i < names.size(); i++)
            if (names[i] == name) id = (int)i;
        if (id < 0) {
            names.push_back(name);
            ms.push_back(0);
            count.push_back(0);
            id = (int)names.size() - 1;
        }
        Rec r{id, get(), get()};
        (void)hipEventRecord(r.a, st);
        recs.push_back(r);
        return (int)recs.size() - 1;
    }
    void end(int rec, hipStream_t st) {
        if (rec < 0) return;
        std::lock_guard<std::mutex> lk(mu);
        if (rec < (int)recs.size()) (void)hipEventRecord(recs[rec].b, st);
    }
    void collect() {
        for (auto &r : recs) {
            (void)hipEventSynchronize(r.b);
            float t = 0;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                ms[r.name] += t;
                count[r.name] += 1;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
};
static Profiler g_prof;

struct ProfScope {
    int rec;
    hipStream_t st;
    ProfScope(const char *name, hipStream_t s) : rec(g_prof.begin(name, s)), st(s) {}
    ~ProfScope() { g_prof.end(rec, st); }
};

int profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (on) {
        g_prof.collect();
        g_prof.names.clear();
        g_prof.ms.clear();
        g_prof.count.clear();
    }
    g_prof.on = on != 0;
    return 0;
}

int profile_read(int i, char *name, int cap, double *total_ms, int64_t *launches) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.collect();
    const int n = (int)g_prof.names.size();
    if (i >= 0 && i < n) {
        if (name && cap > 0) {
            strncpy(name, g_prof.names[i].c_str(), cap - 1);
            name[cap - 1] = 0;
        }
        if (total_ms) *total_ms = g_prof.ms[i];
        if (launches) *launches = g_prof.count[i];
    }
    return n;
}

static int device_cus_cached() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

static inline int grid_for(int64_t work, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>(work, cap)); }

// ---------------------------------------------------------------------------
// Ceiling of the degree-box path's inner loop (for roofline reporting): the
// same per-pair work as k_tile's expand-and-combine step on a 64 x 64 tile
// (operand keys and coefficients read from LDS, one ring product, the hash of
// the key, one LDS compare-and-swap that finds the key's slot and one LDS
// atomic accumulation), repeated over `tiles` tiles per workgroup, with no
// HBM traffic and no table flush.  Keys i*8 + j give 567 distinct slots per
// tile, about seven pairs per monomial.
// ---------------------------------------------------------------------------
__device__ u64 g_ceiling_sink[1 << 14];

template <int RING>
__global__ __launch_bounds__(NTHREADS) void k_dense_ceiling(int tiles) {
    constexpr int TM = 64, TN = 64, HB = 12, HS = 1 << HB;
    const u32 EMPTY = ~0u;
    __shared__ u32 s_fk[TM], s_gk[TN];
    __shared__ u64 s_fc[TM], s_gc[TN];
    __shared__ u32 s_hk[HS + HS / 16];
    __shared__ u64 s_hv[HS + HS / 16];
    auto pad = [](int h) { return h + (h >> 4); };
    for (int e = threadIdx.x; e < TM; e += NTHREADS) {
        s_fk[e] = (u32)e * 8u;
        s_fc[e] = ((u64)(e + 1) * 0x9E3779B97F4A7C15ull + blockIdx.x) >> 4;  // < 2^60 < p
    }
    for (int e = threadIdx.x; e < TN; e += NTHREADS) {
        s_gk[e] = (u32)e;
        s_gc[e] = ((u64)(e + 7) * 0xC2B2AE3D27D4EB4Full) >> 4;
    }
    for (int e = threadIdx.x; e < HS + HS / 16; e += NTHREADS) {
        s_hk[e] = EMPTY;
        s_hv[e] = 0;
    }
    __syncthreads();
    for (int t = 0; t < tiles; t++) {
        for (int e = threadIdx.x; e < TM * TN; e += NTHREADS) {
            const int i = e / TN, j = e % TN;
            const u64 c = ring_mul<RING>(s_fc[i], s_gc[j]);
            const u32 key = s_fk[i] + s_gk[j];
            u32 h = hash_slot<u32>(key, HB);
            for (int probe = 0; probe < HS; probe++) {
                const u32 old = lds_cas<u32>(&s_hk[pad(h)], EMPTY, key);
                if (old == EMPTY || old == key) break;
                h = (h + 1) & (HS - 1);
            }
            ring_atomic_acc<RING>(&s_hv[pad(h)], c);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) g_ceiling_sink[blockIdx.x & ((1 << 14) - 1)] = s_hv[pad(hash_slot<u32>(0, HB))];
}

hipError_t launch_dense_ceiling(int ring, int grid, int tiles, hipStream_t st) {
    if (ring == RING_MODP) hipLaunchKernelGGL(k_dense_ceiling<RING_MODP>, dim3(grid), dim3(NTHREADS), 0, st, tiles);
    else if (ring == RING_MODQ) hipLaunchKernelGGL(k_dense_ceiling<RING_MODQ>, dim3(grid), dim3(NTHREADS), 0, st, tiles);
    else hipLaunchKernelGGL(k_dense_ceiling<RING_I64>, dim3(grid), dim3(NTHREADS), 0, st, tiles);
    return hipGetLastError();
}

hipError_t launch_stats(const DevSeg *segs, int nseg, int nvars, int bits, int ring, u64 *out, u32 *flags,
                        hipStream_t st) {
    ProfScope ps("stats", st);
    hipLaunchKernelGGL(k_stats, dim3(2 * nseg), dim3(ST_T), 0, st, segs, nvars, bits, ring, out, flags);
    return hipGetLastError();
}

template <typename K, int RING>
static void launch_tile(const Plan &P, const Ctx &C, hipStream_t st, int grid, i64 only = -1) {
    ProfScope ps("tile_combine", st);
    // launches of about TILE_LAUNCH_PAIRS term pairs each (about a millisecond
    // on the dense path); the tile ticket restarts at each launch.  only >= 0:
    // that launch alone.
    const i64 tile_pairs = (i64)TILE_CFGS[P.tile_cfg].tm * TILE_CFGS[P.tile_cfg].tn;
    const i64 per = std::max<i64>(1, TILE_LAUNCH_PAIRS / tile_pairs);
    for (i64 b = only >= 0 ? only * per : 0; b < P.ntiles; b += per) {
        const i64 e = std::min<i64>(P.ntiles, b + per);
        if (b > 0) hipLaunchKernelGGL(k_set32, dim3(1), dim3(1), 0, st, C.counters + CNT_TILE, 0u);
        const int g = (int)std::min<i64>(grid, e - b);
        switch (P.tile_cfg) {
            case 0: hipLaunchKernelGGL((k_tile<K, RING, 32, 64, 12>), dim3(g), dim3(NTHREADS), 0, st, C, b, e); break;
            case 1: hipLaunchKernelGGL((k_tile<K, RING, 64, 64, 12>), dim3(g), dim3(NTHREADS), 0, st, C, b, e); break;
            default: hipLaunchKernelGGL((k_tile<K, RING, 128, 128, 12>), dim3(g), dim3(NTHREADS), 0, st, C, b, e); break;
        }
        if (only >= 0) break;
    }
}

int64_t tile_launches(const Plan &P) {
    if (P.ntiles <= 0) return 0;
    const i64 tile_pairs = (i64)TILE_CFGS[P.tile_cfg].tm * TILE_CFGS[P.tile_cfg].tn;
    const i64 per = std::max<i64>(1, TILE_LAUNCH_PAIRS / tile_pairs);
    return (P.ntiles + per - 1) / per;
}

template <typename K, typename V, int RING>
static void launch_sort_reduce(const Plan &P, const Ctx &C, hipStream_t st, int cus) {
    {
        ProfScope ps("seg_prepare", st);
        hipLaunchKernelGGL(k_seg_prepare, dim3(1), dim3(NTHREADS), 0, st, C);
    }
    const int nblk_bound = (int)std::min<int64_t>(P.nparts_bound / P.pblk + P.nseg + 1, (int64_t)cus * 16);
    const int g = std::max(1, std::min(nblk_bound, cus * (P.kl ? 2 : os_resident((int)sizeof(K), (int)sizeof(V)))));
    K *ka = (K *)C.stA_k, *kb = (K *)C.stB_k;
    V *va = (V *)C.stA_v, *vb = (V *)C.stB_v;
    for (int pass = 0; pass < P.passes; pass++) {
        const bool gen = P.raw && pass == 0;
        const bool last = pass == P.passes - 1;
        // pair-index sorts regenerate keys (P.ix) while the operands' compressed
        // keys stay cache resident; otherwise the generating pass writes the
        // keys and later passes move (key, index) pairs
        const bool ix = P.raw && P.ix;
        {
            ProfScope ps("count", st);
            if constexpr (sizeof(V) == 4) {  // SEG_RAW: pair indices
                // every product's operand keys fit the LDS copy (P.ck_fit)
                const size_t dyn = (size_t)P.ck_lds * sizeof(K);
                const u32 *xa = (const u32 *)va;
                if (gen && P.ck_fit) hipLaunchKernelGGL((k_count<K, SM_GEN, true>), dim3(nblk_bound), dim3(CNT_T), dyn, st, C, 0, ka, xa);
                else if (gen) hipLaunchKernelGGL((k_count<K, SM_GEN, false>), dim3(nblk_bound), dim3(CNT_T), 0, st, C, 0, ka, xa);
                else if (ix) hipLaunchKernelGGL((k_count<K, SM_INDEX, true>), dim3(nblk_bound), dim3(CNT_T), dyn, st, C, pass, ka, xa);
                else hipLaunchKernelGGL((k_count<K, SM_STAGED, false>), dim3(nblk_bound), dim3(CNT_T), 0, st, C, pass, ka, xa);
            } else {
                hipLaunchKernelGGL((k_count<K, SM_STAGED, false>), dim3(nblk_bound), dim3(CNT_T), 0, st, C, pass, ka, (const u32 *)nullptr);
            }
            if (P.rscan) hipLaunchKernelGGL(k_range_scan, dim3(grid_for(P.nseg, cus * 4)), dim3(NTHREADS), 0, st, C, pass);
        }
        // profile names: the generating pass, passes that move items only,
        // and the last pass of a pair-index sort (it also writes the keys)
        ProfScope ps(gen ? "onesweep_gen" : (ix && last) ? "onesweep_last" : "onesweep", st);
        if constexpr (sizeof(V) == 4) {
            // pair-index passes hold the operand keys in LDS (P.kl: two
            // workgroups per CU, every product fits); the grid g matches
            const size_t dyn = P.kl ? (size_t)P.ck_lds * sizeof(K) : 0;
            if (gen && !ix) hipLaunchKernelGGL((k_onesweep<K, V, SM_GEN, true, false>), dim3(g), dim3(OS_T), 0, st, C, 0, ka, va, kb, vb);
            else if (!ix) hipLaunchKernelGGL((k_onesweep<K, V, SM_STAGED, true, false>), dim3(g), dim3(OS_T), 0, st, C, pass, ka, va, kb, vb);
            else if (P.kl) {
                if (gen && last) hipLaunchKernelGGL((k_onesweep<K, V, SM_GEN, true, true>), dim3(g), dim3(OS_T), dyn, st, C, 0, ka, va, kb, vb);
                else if (gen) hipLaunchKernelGGL((k_onesweep<K, V, SM_GEN, false, true>), dim3(g), dim3(OS_T), dyn, st, C, 0, ka, va, kb, vb);
                else if (last) hipLaunchKernelGGL((k_onesweep<K, V, SM_INDEX, true, true>), dim3(g), dim3(OS_T), dyn, st, C, pass, ka, va, kb, vb);
                else hipLaunchKernelGGL((k_onesweep<K, V, SM_INDEX, false, true>), dim3(g), dim3(OS_T), dyn, st, C, pass, ka, va, kb, vb);
            } else {
                if (gen && last) hipLaunchKernelGGL((k_onesweep<K, V, SM_GEN, true, false>), dim3(g), dim3(OS_T), 0, st, C, 0, ka, va, kb, vb);
                else if (gen) hipLaunchKernelGGL((k_onesweep<K, V, SM_GEN, false, false>), dim3(g), dim3(OS_T), 0, st, C, 0, ka, va, kb, vb);
                else if (last) hipLaunchKernelGGL((k_onesweep<K, V, SM_INDEX, true, false>), dim3(g), dim3(OS_T), 0, st, C, pass, ka, va, kb, vb);
                else hipLaunchKernelGGL((k_onesweep<K, V, SM_INDEX, false, false>), dim3(g), dim3(OS_T), 0, st, C, pass, ka, va, kb, vb);
            }
        } else {
            hipLaunchKernelGGL((k_onesweep<K, V, SM_STAGED, true, false>), dim3(g), dim3(OS_T), 0, st, C, pass, ka, va, kb, vb);
        }
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    {
        ProfScope ps("head_count", st);
        hipLaunchKernelGGL((k_head_count<K>), dim3(grid_for(P.nparts_bound, cus * 8)), dim3(NTHREADS), 0, st, C, ka);
        hipLaunchKernelGGL(k_head_scan, dim3(grid_for(P.nseg, cus * 4)), dim3(HS_T), 0, st, C);
    }
    {
        ProfScope ps("reduce", st);
        hipLaunchKernelGGL((k_reduce<K, V, RING>), dim3(grid_for(P.nparts_bound, cus * 3)), dim3(RED_T), 0, st, C,
                           ka, va);
    }
    ProfScope ps("zero_compact", st);
    hipLaunchKernelGGL((k_zero_compact<RING>), dim3(grid_for(P.nparts_bound, cus * 2)), dim3(NTHREADS), 0, st, C);
}

template <int RING>
static void launch_bkt(const Plan &P, const Ctx &C, hipStream_t st, int cus) {
    {
        ProfScope ps("bk_count", st);
        hipLaunchKernelGGL(k_bk_count, dim3(grid_for(P.bk_ntiles, cus * 8)), dim3(BK_T), 0, st, C);
    }
    {
        ProfScope ps("bk_cut", st);
        hipLaunchKernelGGL(k_bk_cut, dim3(P.bk_nsb), dim3(BC_T), 0, st, C);
        hipLaunchKernelGGL(k_bk_scan, dim3(1), dim3(BC_T), 0, st, C);
        hipLaunchKernelGGL(k_bk_winfo, dim3(P.bk_nsb), dim3(BC_T), 0, st, C);
    }
    {
        ProfScope ps("bk_scatter", st);
        hipLaunchKernelGGL(k_bk_scatter, dim3(grid_for(P.bk_ntiles, cus * 8)), dim3(BK_T), 0, st, C);
    }
    {
        ProfScope ps("bk_reduce", st);
        // one resident workgroup per CU: 1024 threads and 140-150 KB of LDS
        const int per_cu = 1;
        hipLaunchKernelGGL((k_bk_reduce<RING>), dim3(grid_for(P.bk_wi_bound, cus * per_cu)), dim3(BR_T), 0, st, C);
    }
    ProfScope ps("bk_place", st);
    hipLaunchKernelGGL(k_bk_oscan, dim3(1), dim3(BC_T), 0, st, C);
    hipLaunchKernelGGL(k_bk_copy, dim3(grid_for(P.bk_wi_bound, cus * 8)), dim3(BK_T), 0, st, C);
}

template <typename K, int RING>
static void launch_typed(const Plan &P, const Ctx &C, hipStream_t st, int cus, int part, i64 chunk) {
    if (part == PART_CHUNK) {
        if constexpr (RING != RING_F64) launch_tile<K, RING>(P, C, st, grid_for(P.ntiles, cus * 8), chunk);
        return;
    }
    if (part != PART_TAIL && P.nck > 0) {
        ProfScope ps("compress", st);
        hipLaunchKernelGGL((k_compress<K>), dim3(grid_for((P.nck + NTHREADS - 1) / NTHREADS, cus * 16)), dim3(NTHREADS),
                           0, st, C, (const i64 *)((const char *)C.segs - P.o_segs + P.o_cpre), (i64)P.nck);
    }
    if (P.ntiles > 0 && part != PART_TAIL) {
        if constexpr (RING != RING_F64)
            launch_tile<K, RING>(P, C, st, grid_for(P.ntiles, cus * 8), part == PART_HEAD ? 0 : -1);
    }
    if (part == PART_HEAD) return;
    if (P.nival > 0) {
        if constexpr (sizeof(K) == 4) {
            {
                ProfScope ps("ival_split", st);
                hipLaunchKernelGGL((k_ival_sample<K>), dim3(16, P.nseg), dim3(NTHREADS), 0, st, C);
                hipLaunchKernelGGL((k_ival_split<K>), dim3(P.nseg), dim3(NTHREADS), 0, st, C);
            }
            {
                ProfScope ps("ival", st);
                hipLaunchKernelGGL((k_ival<K, RING>), dim3(P.iv_grid), dim3(NTHREADS), 0, st, C);
            }
            ProfScope ps("ival_concat", st);
            hipLaunchKernelGGL(k_ival_scan, dim3(P.nival), dim3(NTHREADS), 0, st, C);
            hipLaunchKernelGGL((k_ival_copy<K>), dim3(grid_for(P.iv_items, cus * 8)), dim3(NTHREADS), 0, st, C);
        }
    }
    if (P.nbk > 0) {
        if constexpr (sizeof(K) == 4) launch_bkt<RING>(P, C, st, cus);
    }
    if (P.nsparse > 0) {
        if (P.raw) {
            launch_sort_reduce<K, u32, RING>(P, C, st, cus);
        } else {
            if constexpr (RING != RING_F64) launch_sort_reduce<K, u64, RING>(P, C, st, cus);
        }
    } else if (P.nseg > 0) {
        // products without a sort still need n_out = 0 when an operand is empty
        hipLaunchKernelGGL(k_seg_prepare, dim3(1), dim3(NTHREADS), 0, st, C);
    }
    if (P.ndparts > 0) {
        ProfScope ps("compact", st);
        if constexpr (RING != RING_F64)
            hipLaunchKernelGGL((k_compact<RING>), dim3(grid_for(P.ndparts, cus * 8)), dim3(NTHREADS), 0, st, C);
    }
}

hipError_t launch_pipeline(const Plan &P, const Ctx &C, hipStream_t st, int cus, int part, int64_t chunk) {
    // per-call zeroed state
    const size_t zbytes = P.r_zero.bytes;
    u64 *zp = (u64 *)((char *)C.segs - P.o_segs + P.r_zero.off);
    if (part == PART_ALL || part == PART_HEAD) {
        ProfScope ps("fill", st);
        hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)(zbytes / 8 + 255) / 256, cus * 8)), dim3(256), 0, st, zp,
                           (i64)(zbytes / 8), 0ull);
    }
    if (P.ksize == 4) {
        if (P.ring == RING_MODP) launch_typed<u32, RING_MODP>(P, C, st, cus, part, chunk);
        else if (P.ring == RING_MODQ) launch_typed<u32, RING_MODQ>(P, C, st, cus, part, chunk);
        else if (P.ring == RING_I64) launch_typed<u32, RING_I64>(P, C, st, cus, part, chunk);
        else launch_typed<u32, RING_F64>(P, C, st, cus, part, chunk);
    } else {
        if (P.ring == RING_MODP) launch_typed<u64, RING_MODP>(P, C, st, cus, part, chunk);
        else if (P.ring == RING_MODQ) launch_typed<u64, RING_MODQ>(P, C, st, cus, part, chunk);
        else if (P.ring == RING_I64) launch_typed<u64, RING_I64>(P, C, st, cus, part, chunk);
        else launch_typed<u64, RING_F64>(P, C, st, cus, part, chunk);
    }
    return hipGetLastError();
}

static i32 ticket_batch(int64_t work, int grid) {
    int64_t b = work / (2 * (int64_t)std::max(grid, 1));
    return (i32)std::max<int64_t>(1, std::min<int64_t>(b, 16));
}

Ctx make_ctx(const Plan &P, void *ws) {
    char *b = (char *)ws;
    Ctx C;
    C.segs = (DevSeg *)(b + P.o_segs);
    C.dyn = (DevSegDyn *)(b + P.o_dyn);
    C.vars = (VarParam *)(b + P.o_vars);
    C.tile_pre = (const i64 *)(b + P.o_tile_pre);
    C.tile_seg = (const i32 *)(b + P.o_tile_seg);
    C.dpart_pre = (const i64 *)(b + P.o_dpart_pre);
    C.dseg = (const i32 *)(b + P.o_dseg);
    C.ppre = (i64 *)(b + P.o_ppre);
    C.ck = b + P.o_ck;
    C.stA_k = b + P.o_stAk;
    C.stA_v = b + P.o_stAv;
    C.stB_k = b + P.o_stBk;
    C.stB_v = b + P.o_stBv;
    C.box = (u64 *)(b + P.o_box);
    C.pcnt = (u64 *)(b + P.o_pcnt);
    C.ctot = (u64 *)(b + P.o_ctot);
    C.chpre = (i64 *)(b + P.o_chpre);
    C.rpre = (i64 *)(b + P.o_rpre);
    C.rtot = (u64 *)(b + P.o_rtot);
    C.nrng = P.nrng;
    C.pbase = (u64 *)(b + P.o_pbase);
    C.rscan = P.rscan;
    C.look_red = (u64 *)(b + P.o_look_red);
    C.look_cmp = (u64 *)(b + P.o_look_cmp);
    C.look_tile = (u64 *)(b + P.o_look_tile);
    C.counters = (u32 *)(b + P.o_counters);
    C.nseg = P.nseg;
    C.ntseg = (i32)P.tile_seg.size();
    C.ndseg = (i32)P.dseg.size();
    C.nvars = P.nvars;
    C.bits = P.bits;
    C.passes = P.passes;
    for (int i = 0; i < MAX_PASSES; i++) {
        C.dsh[i] = P.dsh[i];
        C.dbits[i] = P.dbits[i];
    }
    C.pblk = P.pblk;
    C.ring = P.ring;
    C.ntiles = P.ntiles;
    C.raw = P.raw;
    C.iv_samp = b + P.o_iv_samp;
    C.iv_spl = b + P.o_iv_spl;
    C.iv_cur = (u32 *)(b + P.o_iv_cur);
    C.iv_maxrows = P.iv_maxrows;
    C.iv_items_arr = (IvalItem *)(b + P.o_iv_items);
    C.iv_off = (u64 *)(b + P.o_iv_off);
    C.iv_pre = (const i64 *)(b + P.o_iv_pre);
    C.iv_seg = (const i32 *)(b + P.o_iv_seg);
    C.nivseg = (i32)P.iv_seg.size();
    C.iv_items = P.iv_items;
    const int cus = device_cus_cached();
    // A ticket may cover several consecutive work items only where no
    // look-back follows: a batch's first item would otherwise wait for the
    // previous batch's last one and serialise the queue.
    C.tb_tile = P.raw ? ticket_batch(P.ntiles, cus * 8) : 1;
    C.tb_sort = 1;
    C.tb_cmp = 1;
    C.ndparts = P.ndparts;
    C.bk_hist = (u32 *)(b + P.o_bk_hist);
    C.bk_wbin = (unsigned short *)(b + P.o_bk_wbin);
    C.bk_sbtot = (u32 *)(b + P.o_bk_sbtot);
    C.bk_sbwi = (u32 *)(b + P.o_bk_sbwi);
    C.bk_sbtb = (u32 *)(b + P.o_bk_sbtb);
    C.bk_sbpre = (u64 *)(b + P.o_bk_sbpre);
    C.bk_wi = (BkWi *)(b + P.o_bk_wi);
    C.bk_fill = (u32 *)(b + P.o_bk_fill);
    C.bk_fatc = (u64 *)(b + P.o_bk_fatc);
    C.bk_fbase = (u64 *)(b + P.o_bk_fbase);
    C.bk_fatfill = (u64 *)(b + P.o_bk_fatfill);
    C.bk_fat_cap = P.bk_fat_cap;
    C.bk_stage = (u64 *)(b + P.o_bk_stage);
    C.bk_rkey = (u32 *)(b + P.o_bk_rkey);
    C.bk_u = (u32 *)(b + P.o_bk_u);
    C.bk_opre = (u64 *)(b + P.o_bk_opre);
    C.bk_tlist = (u64 *)(b + P.o_bk_tlist);
    C.bk_tcnt = (u32 *)(b + P.o_bk_tcnt);
    C.bk_tile_pre = (const i64 *)(b + P.o_bk_tile_pre);
    C.bk_seg = (const i32 *)(b + P.o_bk_seg);
    C.bk_sb_pre = (const i64 *)(b + P.o_bk_sb_pre);
    C.nbk = P.nbk;
    C.bk_ntiles = P.bk_ntiles;
    C.bk_nsb = P.bk_nsb;
    C.bk_wi_bound = P.bk_wi_bound;
    C.bk_nstage = P.bk_nstage;
    return C;
}

}  // namespace pm
