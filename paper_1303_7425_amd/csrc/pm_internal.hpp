// Internal definitions shared by the host planner and the gfx950 kernels of
// the sparse polynomial product.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;
typedef int32_t i32;

constexpr u64 P61 = (1ull << 61) - 1;

enum Ring : int { RING_MODP = 0, RING_F64 = 1, RING_I64 = 2, RING_MODQ = 3 };

// How one product (a "segment" of a launch) is computed.
enum SegMode : int {
    SEG_EMPTY = 0,    // an operand is empty: n_out = 0
    SEG_COMBINE = 1,  // tiles combined in LDS, then global radix sort + segmented reduction
    SEG_RAW = 2,      // pair indices sorted by key (products regenerated), then reduction
    SEG_DENSE = 3,    // accumulated directly into the degree box, then compaction
    SEG_IVAL = 4,     // output-key intervals owned by workgroups, merged in LDS (no global sort)
    SEG_BKT = 5,      // pairs scattered once into output-key work items, each sorted and summed in LDS
};

// Output-key work items (SEG_BKT).  The compressed key range of a product is
// cut into fine bins of 2^fs keys; a counting pass over the term pairs gives
// each bin's pair count, consecutive bins are grouped greedily into work
// items of at most BK_CAP pairs (a single bin over BK_CAP forms its own), one
// pass scatters every pair into its work item, and one workgroup per work
// item sorts and sums it in LDS.
constexpr int BK_TILE = 8192;          // term pairs per generation tile (rows x power-of-two columns)
constexpr int BK_TN_MAX = 256;         // columns of a generation tile, at most
constexpr int BK_SB_LOG = 12;
constexpr int BK_SB = 1 << BK_SB_LOG;  // fine bins per super-bin (the unit of the greedy cut)
constexpr int BK_CAP = 8192;           // pairs of a work item sorted in one LDS pass
constexpr int BK_BIN_PAIRS = 8;        // about this many term pairs per fine bin
constexpr long long TILE_LAUNCH_PAIRS = 1ll << 27;  // term pairs per tile-kernel launch (about 1 ms dense)
constexpr int BK_RANK_LOG = 18;        // exact rings: key span (log2) a work item sums by rank in LDS

// One work item: fine bins [bin_lo, bin_hi) of product q (bins local to the
// product), its items at [off, end) of the staging array.
struct BkWi {
    u32 bin_lo, bin_hi;
    u64 off, end;
    i32 q;
    u32 first, last;  // the product's first / last work item
    u32 pad;
};

constexpr int IV_SAMPLES_MAX = 4096;   // grid samples per product ((l+1)^2, l <= 63)

constexpr int NTHREADS = 256;          // threads per workgroup (4 wave64s)
constexpr int IPT = 16;                // items per thread in sort / reduce partitions
constexpr int PART = NTHREADS * IPT;   // items per partition
constexpr int RNG = 64;                // sort blocks per range
constexpr int PBLK_MAX = 32;           // sort partitions per sort block, at most
constexpr int RSUM_MAX = 16;           // products with at most this many ranges need no range scan
// Radix-pass workgroups (512 threads) resident per CU: three when keys and
// payloads are 4 bytes each (LDS and registers allow it), else two.
constexpr int OS_T = 512;
constexpr int os_resident(int ksize, int vsize) { return ksize + vsize <= 8 ? 3 : 2; }
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;

// LDS bytes of a radix-pass workgroup that keeps each item's digit byte (dg)
// or its key, its payload, the per-wave digit counters and the digit offsets
// (an upper bound of the kernel's shared block).
constexpr size_t os_lds_bytes(int ksize, int vsize, bool dg) {
    return (size_t)PART * ((dg ? 1 : ksize) + vsize) + (size_t)(OS_T / 64) * RADIX * 4 + 2 * RADIX * 4 + 256;
}
// Pair-index radix passes hold a copy of the operands' compressed keys (ck
// entries) in LDS when two such workgroups still fit a CU's 160 KB.
constexpr bool os_keys_in_lds(int64_t ck, int ksize, int vsize) {
    return ck > 0 && 2 * (os_lds_bytes(ksize, vsize, true) + (size_t)ck * ksize) <= ((size_t)160 << 10);
}
constexpr int MAX_PASSES = 8;
constexpr int MAX_VARS = 64;

// Unsigned 32-bit division by an invariant divisor d >= 1 (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994):
// q = (t + ((n - t) >> s1)) >> s2 with t = mulhi(m, n).
struct Div32 {
    u32 m, s1, s2, d;
};

inline Div32 make_div32(u32 d) {
    int l = 0;
    while (l < 32 && (1ull << l) < d) l++;
    Div32 r;
    r.m = (u32)(((((unsigned __int128)1) << 32) * ((((unsigned __int128)1) << l) - d)) / d + 1);
    r.s1 = l < 1 ? l : 1;
    r.s2 = l > 1 ? l - 1 : 0;
    r.d = d;
    return r;
}

__host__ __device__ inline u32 div32(u32 n, const Div32 &dv) {
#ifdef __HIP_DEVICE_COMPILE__
    u32 t = __umulhi(dv.m, n);
#else
    u32 t = (u32)(((u64)dv.m * n) >> 32);
#endif
    return (t + ((n - t) >> dv.s1)) >> dv.s2;
}

// Per-product descriptor, uploaded once per call.
struct DevSeg {
    const u64 *fk, *fc, *gk, *gc;  // operand keys / coefficient bits
    i64 na, nb;
    i64 ck_f, ck_g;                // offsets of the compressed operand keys
    i64 stage_base;                // first staging slot (sparse) or first box cell (dense)
    i64 stage_bound;               // staging slots (sparse) or box cells (dense)
    i64 tile_first;                // first tile of this product in the tile queue
    i64 tiles_n;                   // tiles along g
    Div32 nb_div;                  // division by nb: pair index -> (row, column) (SEG_RAW)
    i64 dpart_first;               // first compaction partition (SEG_DENSE)
    i64 var_off;                   // offset of this product's VarParam entries
    i64 iv_l;                      // grid parameter l (SEG_IVAL): (l+1)^2 samples
    i64 iv_samp_off, iv_spl_off;   // offsets of its samples and splitters
    i64 bk_bin_off;                // SEG_BKT: first fine bin in the launch's bin arrays (multiple of BK_SB)
    i64 bk_sb_first, bk_nsb;       // first super-bin (launch-wide index) and super-bins
    i64 bk_tile_first;             // first generation tile
    i64 bk_tiles_n;                // generation tiles along g
    i32 bk_fs;                     // fine shift: bin = compressed key >> bk_fs
    i32 bk_tnl;                    // log2 of the generation tile's columns (rows: BK_TILE >> bk_tnl)
    u64 lo_key;                    // packed key of the smallest output exponent vector
    u64 *hk, *hc;                  // result arrays
    i64 *n_out;
    i64 cap;
    i32 mode;
    i32 bk_span_bins;              // SEG_BKT: most fine bins per work item (0: no limit)
};

// Values produced on the device during a call.
struct DevSegDyn {
    unsigned long long fill;       // staged pairs (SEG_COMBINE)
    i64 n;                         // pairs to sort
    i64 part_first;                // first sort / reduce partition
    i64 nparts;
    i64 heads;                     // distinct keys after the sort (result slots incl. cancelled ones)
    unsigned long long zeros;      // slots whose sum cancelled to zero
};

// Per product and variable: field position and the mixed-radix compression.
// compressed(alpha) = sum_v (alpha_v - min_v) * stride_v, strides taken over the
// output ranges range_v = max_f+max_g-min_f-min_g+1, so compressed(f_i) +
// compressed(g_j) is the mixed-radix index of alpha_i+beta_j in the degree box
// and preserves the lexicographic order.
struct VarParam {
    u32 shift;
    u32 pad;
    u64 mask;
    u64 minf, ming;
    u64 range;
    u64 stride;
    Div32 rdiv;  // division by range (when range < 2^32)
};

// Launch-wide context passed by value to every kernel.
struct Ctx {
    DevSeg *segs;
    DevSegDyn *dyn;
    VarParam *vars;
    const i64 *tile_pre;    // [ntseg+1] exclusive tile prefix over tiled segments
    const i32 *tile_seg;    // [ntseg] segment index of each tiled segment
    const i64 *dpart_pre;   // [ndseg+1] compaction partition prefix over SEG_DENSE segments
    const i32 *dseg;
    i64 *ppre;              // [nseg+1] sort partition prefix (device computed)
    void *ck;               // compressed operand keys
    void *stA_k, *stA_v;
    void *stB_k, *stB_v;
    u64 *box;
    u64 *pcnt;                  // per-partition run-head counts, then first result slots [nparts_bound]
    u64 *ctot;                  // digit counts of the current radix pass per sort block [nblocks][RADIX]
    u64 *rtot;                  // the same per range of RNG blocks [2][nrng][RADIX], by pass parity
    i64 nrng;                   // range rows per parity
    u64 *pbase;                 // [nseg][RADIX] digit bases of the current radix pass
    i32 rscan;                  // k_range_scan runs (some product may have more than RSUM_MAX ranges)
    i64 *chpre;                 // [nseg+1] sort-block prefix over products (device computed)
    i64 *rpre;                  // [nseg+1] range prefix over products (device computed)
    u64 *look_red;              // reduce lookback [nparts_bound]
    u64 *look_cmp;              // dense compaction lookback [ndparts]
    u64 *look_tile;             // staging offsets of combined tiles [ntiles]
    u32 *counters;              // work-queue tickets and error flags
    void *iv_samp, *iv_spl;     // grid samples / interval bounds (SEG_IVAL)
    u32 *iv_cur;                // per-workgroup row cursors
    i64 iv_maxrows;
    struct IvalItem *iv_items_arr;
    u64 *iv_off;                // result offset of every interval
    const i64 *iv_pre;          // [nivseg+1] interval-item prefix over SEG_IVAL products
    const i32 *iv_seg;
    i32 nivseg;
    i64 iv_items;
    i32 nseg, ntseg, ndseg;
    i32 nvars, bits, passes, ring;
    unsigned char dsh[MAX_PASSES], dbits[MAX_PASSES];  // digit shift and width of each radix pass
    i64 pblk;                   // sort partitions per sort block
    i64 ntiles, ndparts;
    i32 raw;                    // sparse products carry pair indices (SEG_RAW) instead of values
    // SEG_BKT (output-key work items)
    u32 *bk_hist;               // [bins] term pairs per fine bin (zeroed per call)
    unsigned short *bk_wbin;    // [bins] work item of each bin, numbered inside its super-bin
    u32 *bk_sbtot, *bk_sbwi;    // [nsb] pairs and work items of each super-bin
    u32 *bk_sbtb;               // [nsb+1] first work item (ticket) of each super-bin; [nsb]: all
    u64 *bk_sbpre;              // [nsb] first staging slot of each super-bin
    BkWi *bk_wi;                // [wi bound] work items by ticket
    u32 *bk_fill;               // [wi bound] staged items per work item so far (zeroed per call)
    u64 *bk_fatc;               // result coefficients of work items over BK_CAP pairs
    u64 *bk_fbase;              // [wi bound] their first slot in bk_fatc
    u64 *bk_fatfill;            // slots of bk_fatc taken (zeroed per call)
    i64 bk_fat_cap;             // slots of bk_fatc
    u64 *bk_stage;              // staged items: (pair index << 32) | compressed key; then result coefficients
    u32 *bk_rkey;               // [staging slots] compressed keys of the result terms
    u32 *bk_u;                  // [wi bound] result terms of each work item (bit 31: coefficients in bk_fatc)
    u64 *bk_opre;               // [wi bound] first result slot of each work item
    u64 *bk_tlist;              // [tiles][BK_TL] (bin << 32 | pairs) of each generation tile
    u32 *bk_tcnt;               // [tiles] entries of the tile's list (all ones: not listed)
    const i64 *bk_tile_pre;     // [nbk+1] generation-tile prefix over SEG_BKT products
    const i32 *bk_seg;          // [nbk] their segment indices
    const i64 *bk_sb_pre;       // [nbk+1] super-bin prefix over SEG_BKT products
    i32 nbk;
    i64 bk_ntiles, bk_nsb;
    i64 bk_wi_bound;            // work-item slots (tickets beyond are an internal error)
    i64 bk_nstage;              // staging slots
    i32 tb_tile, tb_sort, tb_cmp;  // consecutive work items handed out per work-queue ticket
};

// counters[] slots
enum Counter : int {
    CNT_TILE = 0,
    CNT_HIST = 1,
    CNT_SORT = 2,                   // + pass (MAX_PASSES slots)
    CNT_REDUCE = CNT_SORT + MAX_PASSES,
    CNT_COMPACT,
    CNT_IVAL,
    CNT_ERR_SPIN,                   // a lookback wait hit its iteration bound
    CNT_ZEROS,                      // some product of the launch has cancelled terms
    CNT_ZCOMPACT,
    CNT_BK_REDUCE,                  // work items of the in-LDS sort and sum
    CNT_COUNT
};

// Validation flags reported by the statistics kernel.
enum StatFlag : u32 { ST_UNSORTED = 1, ST_BADBITS = 2, ST_RANGE = 4 };

// ---------------------------------------------------------------------------
// Ring arithmetic on 64-bit coefficient words
// ---------------------------------------------------------------------------
__host__ __device__ inline u64 addmod61(u64 a, u64 b) {
    u64 s = a + b;  // < 2^62
    return s >= P61 ? s - P61 : s;
}

// a * b mod 2^61-1 for a, b < 2^61: the 122-bit product is split at bit 61 and
// folded twice (2^61 = 1 mod p).
__device__ inline u64 mulmod61(u64 a, u64 b) {
    u64 lo = a * b;
    u64 hi = __umul64hi(a, b);
    u64 r = (lo & P61) + ((lo >> 61) | (hi << 3));
    r = (r & P61) + (r >> 61);
    return r >= P61 ? r - P61 : r;
}

// Any u64 to its residue in [0, p).
__host__ __device__ inline u64 reduce61(u64 x) {
    u64 r = (x & P61) + (x >> 61);
    return r >= P61 ? r - P61 : r;
}

// Arithmetic mod the prime q = 2^64 - 59, using 2^64 = 59 (mod q).
constexpr u64 Q64 = 0xFFFFFFFFFFFFFFC5ull;
constexpr u64 Q64_C = 59;

__host__ __device__ inline u64 addmodq(u64 a, u64 b) {
    u64 s = a + b;
    if (s < a) s += Q64_C;  // wrapped past 2^64: s + 59 < q
    return s >= Q64 ? s - Q64 : s;
}

// x = hi * 2^64 + lo  ->  hi * 59 + lo, folded until it fits, then one
// conditional subtraction.
__device__ inline u64 foldq(u64 hi, u64 lo) {
    const u64 t_lo = hi * Q64_C, t_hi = __umul64hi(hi, Q64_C);  // t_hi < 59
    u64 s = lo + t_lo;
    const u64 k = t_hi + (s < lo ? 1u : 0u);                       // <= 59
    const u64 s2 = s + k * Q64_C;
    s = s2 < s ? s2 + Q64_C : s2;                                   // a second wrap leaves s2 < 59^2
    return s >= Q64 ? s - Q64 : s;
}

__device__ inline u64 mulmodq(u64 a, u64 b) { return foldq(__umul64hi(a, b), a * b); }

template <int RING>
__device__ inline u64 ring_mul(u64 a, u64 b) {
    if constexpr (RING == RING_MODP) {
        return mulmod61(a, b);
    } else if constexpr (RING == RING_MODQ) {
        return mulmodq(a, b);
    } else if constexpr (RING == RING_I64) {
        return a * b;  // two's-complement product modulo 2^64
    } else {
        return (u64)__double_as_longlong(__longlong_as_double((long long)a) * __longlong_as_double((long long)b));
    }
}

template <int RING>
__device__ inline u64 ring_add(u64 a, u64 b) {
    if constexpr (RING == RING_MODP) {
        return addmod61(a, b);
    } else if constexpr (RING == RING_MODQ) {
        return addmodq(a, b);
    } else if constexpr (RING == RING_I64) {
        return a + b;
    } else {
        return (u64)__double_as_longlong(__longlong_as_double((long long)a) + __longlong_as_double((long long)b));
    }
}

template <int RING>
__device__ inline bool ring_is_zero(u64 a) {
    if constexpr (RING == RING_F64) {
        return (a << 1) == 0;  // +0.0 or -0.0
    } else {
        return a == 0;
    }
}

// Order-free exact accumulation into a 64-bit cell (LDS or global).
//   mod p: the cell holds a value congruent to the sum; a wrap past 2^64 is
//          compensated by adding 8, since 2^64 = 8 (mod 2^61-1).
//   mod q: the same with 2^64 = 59 (mod 2^64-59).
//   int64: plain wrapping addition.
template <int RING>
__device__ inline void ring_atomic_acc(u64 *cell, u64 c) {
    if constexpr (RING == RING_MODP || RING == RING_MODQ) {
        constexpr u64 WRAP = RING == RING_MODP ? 8 : Q64_C;
        u64 add = c;
        while (true) {
            u64 old = atomicAdd((unsigned long long *)cell, (unsigned long long)add);
            if (old + add >= old) break;
            add = WRAP;
        }
    } else {
        atomicAdd((unsigned long long *)cell, (unsigned long long)c);
    }
}

template <int RING>
__device__ inline u64 ring_cell_final(u64 x) {
    if constexpr (RING == RING_MODP) {
        return reduce61(x);
    } else if constexpr (RING == RING_MODQ) {
        return x >= Q64 ? x - Q64 : x;
    } else {
        return x;
    }
}

// ---------------------------------------------------------------------------
// Wave64 / workgroup primitives
// ---------------------------------------------------------------------------
__device__ inline u32 lane_id() { return __lane_id(); }

// popcount(mask & lanes below this one)
__device__ inline u32 mbcnt(u64 mask) {
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

template <typename T>
__device__ inline T wave_incl_scan(T x) {
    const u32 lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= (u32)d) x += y;
    }
    return x;
}

// Exclusive scan over the 256 threads of a workgroup.  `scratch` holds 4 T.
// Contains two barriers; every thread must call it.
template <typename T, int NT = NTHREADS>
__device__ inline T block_excl_scan(T v, T *scratch, T &total) {
    const u32 lane = lane_id();
    const u32 w = threadIdx.x >> 6;
    T x = wave_incl_scan(v);
    if (lane == 63) scratch[w] = x;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) {
        T s = scratch[i];
        if ((u32)i < w) pre += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// Lookback words: [63:56] tag, [55:54] flag, [53:0] value.
constexpr u64 LB_AGG = 1, LB_INC = 2;
__device__ inline u64 lb_pack(u32 tag, u64 flag, u64 value) { return ((u64)tag << 56) | (flag << 54) | value; }
__device__ inline void lb_store(u64 *p, u64 v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline u64 lb_load(u64 *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

constexpr u32 LB_SPIN_LIMIT = 1u << 24;

__device__ inline u64 wave_sum_u64(u64 v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Decoupled look-back: partition p publishes its own aggregate, later its
// inclusive prefix; a successor sums the words of its predecessors back to the
// nearest inclusive prefix.  Partitions are taken from a work queue in order,
// so every earlier partition belongs to a running or finished workgroup and
// each wait ends (a bounded spin flags an error instead of hanging).
//
// Publishes partition p's own aggregate: its inclusive prefix when p is the
// product's first partition.  Publishing early, and resolving the prefix
// later, gives the predecessors time to publish theirs.
__device__ inline void lb_publish(u64 *slot, i64 first, i64 p, u32 tag, u64 value) {
    lb_store(slot, lb_pack(tag, p == first ? LB_INC : LB_AGG, value));
}

// Wave-cooperative decoupled look-back for one counter per partition.  All
// 64 lanes of one wave call it with the same (first, p); lane l inspects
// predecessor p-1-l, so one round trip covers 64 predecessors.  Returns the
// exclusive prefix of `value` over partitions [first, p) in every lane.  The
// partition has already published its aggregate with lb_publish.
__device__ inline u64 lookback_wave_resolve(u64 *look, i64 first, i64 p, u32 tag, u64 value, u32 *err) {
    const u32 lane = lane_id();
    if (p == first) return 0;
    u64 prefix = 0;
    i64 top = p - 1;
    while (true) {
        const i64 j = top - (i64)lane;
        u64 val = 0;
        bool inc = true;
        if (j >= first) {
            u64 v = lb_load(look + j);
            u32 spins = 0;
            while ((u32)(v >> 56) != tag && spins < LB_SPIN_LIMIT) {
                spins++;
                v = lb_load(look + j);
            }
            if ((u32)(v >> 56) != tag) {
                atomicOr(err, 1u);
            } else {
                inc = ((v >> 54) & 3) == LB_INC;
                val = v & ((1ull << 54) - 1);
            }
        }
        const u64 im = __ballot(inc);
        if (im) {
            const u32 k = (u32)__ffsll((unsigned long long)im) - 1;  // nearest predecessor with a prefix
            prefix += wave_sum_u64(lane <= k ? val : 0);
            break;
        }
        prefix += wave_sum_u64(val);
        top -= 64;
    }
    if (lane == 0) lb_store(look + p, lb_pack(tag, LB_INC, prefix + value));
    return prefix;
}

__device__ inline u64 lookback_wave(u64 *look, i64 first, i64 p, u32 tag, u64 value, u32 *err) {
    if (lane_id() == 0) lb_publish(look + p, first, p, tag, value);
    return lookback_wave_resolve(look, first, p, tag, value, err);
}

// Largest index s in [0, n) with pre[s] <= x (pre ascending, pre[0] = 0).
__device__ inline i32 seg_search(const i64 *pre, i32 n, i64 x) {
    i32 lo = 0, hi = n - 1;
    while (lo < hi) {
        i32 mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Mixed-radix index back to the packed key.
template <typename K>
__device__ inline u64 decompress(K ck, const VarParam *vp, int nvars, u64 lo_key) {
    u64 key = lo_key;
    if constexpr (sizeof(K) == 4) {
        for (int v = nvars - 1; v >= 0; v--) {
            const u32 q = div32((u32)ck, vp[v].rdiv);
            key += (u64)((u32)ck - q * vp[v].rdiv.d) << vp[v].shift;
            ck = q;
        }
    } else {
        for (int v = nvars - 1; v >= 0; v--) {
            K r = (K)vp[v].range;
            K e;
            if (r == 0) {  // range 2^64: a single full-width variable
                e = ck;
                ck = 0;
            } else {
                e = ck % r;
                ck /= r;
            }
            key += (u64)e << vp[v].shift;
        }
    }
    return key;
}

// Grid sample t of Section 5 over an na x nb pp-matrix with parameter l
// ((l + 1)^2 samples, Fig. 2 with l = 8 has 81): sample row r = t / (l + 1)
// lies at row r * floor(na / l); its column c = t % (l + 1) lies at
// c * floor(nb / l), shifted by floor(nb / (2 l)) on odd sample rows (the
// staggered grid); both clamped to the matrix.  l = 0 is the single sample
// (0, 0).  Shared by the sampling kernel and the host helper pm_ival_grid.
__host__ __device__ inline void ival_grid_point(i64 na, i64 nb, i64 l, i64 t, i64 &i, i64 &j) {
    const i64 r = t / (l + 1), c = t % (l + 1);
    const i64 di = l ? na / l : 0, dj = l ? nb / l : 0, st = l ? nb / (2 * l) : 0;
    const i64 ri = r * di, cj = (r & 1) * st + c * dj;
    i = ri < na - 1 ? ri : na - 1;
    j = cj < nb - 1 ? cj : nb - 1;
}

}  // namespace pm
