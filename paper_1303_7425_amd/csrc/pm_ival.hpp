// Output-key interval path (SEG_IVAL), included by pm_kernels.hip.
//
// This is the structure of Algorithm 1 mapped onto the GPU:
//   step 1   k_ival_sample / k_ival_split: exponents alpha_i + beta_j sampled on
//            the staggered grid of Section 5 over the pp-matrix (Fig. 1),
//            sorted, duplicates removed, bracketed by gamma_11 and
//            gamma_end = gamma_{na,nb} + 1: half-open intervals [S_k, S_{k+1})
//            that together hold every term product exactly once.
//   step 2   k_ival: one work item per interval.  FindEdge as a binary search
//            per row gives the first column of each row inside the interval
//            (rows are increasing, Section 2); the workgroup then walks the
//            interval in LDS-sized batches of key sub-ranges (chosen from a
//            1024-bucket histogram of the interval's keys), generates each
//            batch's term pairs in row-major order, sorts them by key in LDS
//            (stable radix passes) and sums equal keys left to right: the
//            MergeSort role of Algorithm 1, with no global sort and no
//            communication between intervals.
//   concat   k_ival_scan / k_ival_copy: interval results are concatenated in
//            ascending interval order (Algorithm 1's last line) and the keys
//            decompressed.
// Because every pair of one monomial lies in one interval and is visited in
// row-major order, FP64 sums are the plain row-major schoolbook sums.

namespace pm {

constexpr int IV_CAP = PART;      // term pairs per LDS batch
constexpr int IV_NB = 512;        // histogram buckets per key range (9 bits per level)
constexpr int IV_LEVELS = 4;      // nested refinements of an over-full bucket (32-bit keys)

// Work-item bookkeeping, one entry per (product, interval).
struct IvalItem {
    unsigned long long ostart;    // first staging slot of this interval's results
    unsigned long long ocount;    // result terms of this interval
};

template <typename K>
__device__ inline u32 lower_bound_dev(const K *a, u32 n, K x) {
    u32 lo = 0, hi = n;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Grid samples of Section 5 (ival_grid_point), one exponent sum each.
template <typename K>
__global__ __launch_bounds__(NTHREADS) void k_ival_sample(Ctx C) {
    const int q = blockIdx.y;
    const DevSeg &s = C.segs[q];
    if (s.mode != SEG_IVAL) return;
    const i64 l = s.iv_l;
    const i64 ns = (l + 1) * (l + 1);
    const K *ck = (const K *)C.ck;
    K *samp = (K *)C.iv_samp + s.iv_samp_off;
    for (i64 t = (i64)blockIdx.x * NTHREADS + threadIdx.x; t < ns; t += (i64)gridDim.x * NTHREADS) {
        i64 i, j;
        ival_grid_point(s.na, s.nb, l, t, i, j);
        samp[t] = ck[s.ck_f + i] + ck[s.ck_g + j];
    }
}

// Sort the samples of one product (bitonic in LDS), drop duplicates, bracket
// with gamma_11 and gamma_end.  One workgroup per product.
template <typename K>
__global__ __launch_bounds__(NTHREADS) void k_ival_split(Ctx C) {
    constexpr int SMAX = IV_SAMPLES_MAX;
    __shared__ K s_v[SMAX];
    __shared__ u32 s_scan[NTHREADS / 64];
    const int q = blockIdx.x;
    const DevSeg &s = C.segs[q];
    if (s.mode != SEG_IVAL) return;
    const K *ck = (const K *)C.ck;
    const K *samp = (const K *)C.iv_samp + s.iv_samp_off;
    const int ns = (int)((s.iv_l + 1) * (s.iv_l + 1));
    int n2 = 1;
    while (n2 < ns) n2 <<= 1;
    const K KMAX = (K)~(K)0;
    for (int t = threadIdx.x; t < n2; t += NTHREADS) s_v[t] = t < ns ? samp[t] : KMAX;
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < n2; t += NTHREADS) {
                const int p = t ^ j;
                if (p > t) {
                    const K a = s_v[t], b = s_v[p];
                    const bool up = (t & k) == 0;
                    if ((a > b) == up) {
                        s_v[t] = b;
                        s_v[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    const K kmin = ck[s.ck_f] + ck[s.ck_g];
    const K kend = ck[s.ck_f + s.na - 1] + ck[s.ck_g + s.nb - 1] + 1;
    // keep sample t when it is distinct from its predecessor and inside (kmin, kend)
    K *spl = (K *)C.iv_spl + s.iv_spl_off;
    u32 base = 1;
    for (int b = 0; b < n2; b += NTHREADS) {
        const int t = b + threadIdx.x;
        bool keep = false;
        K v = 0;
        if (t < ns) {
            v = s_v[t];
            keep = v > kmin && v < kend && (t == 0 || s_v[t - 1] != v);
        }
        u32 tot;
        const u32 off = block_excl_scan<u32>(keep ? 1u : 0u, s_scan, tot);
        if (keep) spl[base + off] = v;
        base += tot;
    }
    if (threadIdx.x == 0) {
        spl[0] = kmin;
        spl[base] = kend;
        C.dyn[q].n = base;  // number of intervals
    }
}

// LDS radix sort of m <= IV_CAP (key, payload) items by the low `bits` bits of
// the key, stable.  Items live in s_k / s_x; 8-bit digits, ranks from per-wave
// ballot match masks as in k_onesweep.
__device__ __noinline__ void lds_sort_pairs(u32 *s_k, u32 *s_x, int m, int bits, u32 (*s_wh)[RADIX], u32 *s_scan) {
    constexpr int NW = NTHREADS / 64;
    const u32 lane = lane_id(), w = threadIdx.x >> 6;
    for (int shift = 0; shift < bits; shift += RADIX_BITS) {
        for (int d = threadIdx.x; d < NW * RADIX; d += NTHREADS) (&s_wh[0][0])[d] = 0;
        u32 key[IPT], x[IPT], rd[IPT];  // rd: rank within the wave's digit (low 16 bits) | digit << 16
#pragma unroll
        for (int k = 0; k < IPT; k++) {
            const int idx = (int)w * 64 * IPT + k * 64 + (int)lane;
            key[k] = idx < m ? s_k[idx] : 0u;
            x[k] = idx < m ? s_x[idx] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IPT; k++) {
            const int idx = (int)w * 64 * IPT + k * 64 + (int)lane;
            const bool valid = idx < m;
            const u32 d = (key[k] >> shift) & (RADIX - 1);
            u64 peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < RADIX_BITS; b++) {
                const u64 mm = __ballot((d >> b) & 1);
                peers &= ((d >> b) & 1) ? mm : ~mm;
            }
            const u32 before = mbcnt(peers);
            const u32 cnt = (u32)__popcll(peers);
            u32 old = valid ? s_wh[w][d] : 0;
            if (valid && before == 0) s_wh[w][d] = old + cnt;
            rd[k] = (old + before) | (d << 16);
        }
        __syncthreads();
        {
            const int d = threadIdx.x;
            u32 tot = 0;
#pragma unroll
            for (int ww = 0; ww < NW; ww++) {
                const u32 v = s_wh[ww][d];
                s_wh[ww][d] = tot;
                tot += v;
            }
            u32 all;
            const u32 loff = block_excl_scan<u32>(tot, s_scan, all);
#pragma unroll
            for (int ww = 0; ww < NW; ww++) s_wh[ww][d] += loff;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IPT; k++) {
            const int idx = (int)w * 64 * IPT + k * 64 + (int)lane;
            if (idx < m) {
                const u32 pos = s_wh[w][rd[k] >> 16] + (rd[k] & 0xFFFFu);
                s_k[pos] = key[k];
                s_x[pos] = x[k];
            }
        }
        __syncthreads();
    }
}

// k_ival: persistent queue of (product, interval) items.
template <typename K, int RING>
__global__ __launch_bounds__(NTHREADS) void k_ival(Ctx C) {
    constexpr int NW = NTHREADS / 64;
    __shared__ u32 s_k[IV_CAP];          // batch keys relative to the batch start
    __shared__ u32 s_x[IV_CAP];          // batch pair indices
    __shared__ u32 s_wh[NW][RADIX];
    __shared__ u32 s_hist[IV_LEVELS][IV_NB + 1];
    __shared__ u32 s_scan[NTHREADS / 64];
    __shared__ i64 s_item;
    __shared__ unsigned long long s_ob;
    __shared__ u32 s_run;                // results written so far by this interval
    __shared__ u64 s_v[IV_CAP];          // run sums (one per head)
    __shared__ K rlo[IV_LEVELS], rhi[IV_LEVELS];   // key sub-range of each refinement level
    __shared__ int sh[IV_LEVELS], nxt[IV_LEVELS];  // bucket shift and next bucket per level

    const K *ck = (const K *)C.ck;
    u32 *cur = C.iv_cur + (i64)blockIdx.x * C.iv_maxrows;
    while (true) {
        if (threadIdx.x == 0) s_item = (i64)atomicAdd(&C.counters[CNT_IVAL], 1u);
        __syncthreads();
        const i64 it = s_item;
        if (it >= C.iv_items) break;
        const i32 qs = seg_search(C.iv_pre, C.nivseg, it);
        const int q = C.iv_seg[qs];
        const DevSeg &s = C.segs[q];
        const i64 k = it - C.iv_pre[qs];
        if (k >= C.dyn[q].n) {  // fewer distinct splitters than samples
            __syncthreads();
            continue;
        }
        const K *spl = (const K *)C.iv_spl + s.iv_spl_off;
        const K lo = spl[k], hi = spl[k + 1];
        const K *cf = ck + s.ck_f;
        const K *cg = ck + s.ck_g;
        const u32 na = (u32)s.na, nb = (u32)s.nb;
        const u32 R = (na + NTHREADS - 1) / NTHREADS;  // rows per thread, blocked
        const u32 r0 = threadIdx.x * R, r1 = min(na, r0 + R);
        // FindEdge: first column of each row with key >= lo
        for (u32 i = r0; i < r1; i++) {
            const K a = cf[i];
            cur[i] = a >= lo ? 0u : lower_bound_dev<K>(cg, nb, (K)(lo - a));
        }
        if (threadIdx.x == 0) s_run = 0;
        __syncthreads();

        // depth-first walk over key sub-ranges: level 0 is [lo, hi).  The level
        // state is uniform and lives in LDS; every update is made by thread 0
        // and published by the barrier that follows it.
        int lev = 0;
        if (threadIdx.x == 0) {
            rlo[0] = lo;
            rhi[0] = hi;
        }
        __syncthreads();
        bool need_hist = true;
        bool reserved = false;
        while (lev >= 0) {
            if (need_hist) {
                const K width = rhi[lev] - rlo[lev];
                int b = 0;
                while (b < (int)(8 * sizeof(K)) && ((K)1 << b) < width) b++;  // bits of width-1, rounded
                if (threadIdx.x == 0) {
                    sh[lev] = b > 9 ? b - 9 : 0;
                    nxt[lev] = 0;
                }
                for (int e = threadIdx.x; e <= IV_NB; e += NTHREADS) s_hist[lev][e] = 0;
                __syncthreads();
                for (u32 i = r0; i < r1; i++) {
                    const K a = cf[i];
                    for (u32 j = cur[i]; j < nb; j++) {
                        const K key = a + cg[j];
                        if (key >= rhi[lev]) break;
                        atomicAdd(&s_hist[lev][(u32)((key - rlo[lev]) >> sh[lev])], 1u);
                    }
                }
                __syncthreads();
                // exclusive prefix in place: s_hist[lev][b] = pairs in buckets < b
                {
                    constexpr int BPT = IV_NB / NTHREADS;
                    u32 v[BPT], t = 0;
#pragma unroll
                    for (int r = 0; r < BPT; r++) {
                        v[r] = s_hist[lev][threadIdx.x * BPT + r];
                        t += v[r];
                    }
                    u32 tot;
                    u32 off = block_excl_scan<u32>(t, s_scan, tot);
#pragma unroll
                    for (int r = 0; r < BPT; r++) {
                        s_hist[lev][threadIdx.x * BPT + r] = off;
                        off += v[r];
                    }
                    if (threadIdx.x == 0) s_hist[lev][IV_NB] = tot;
                    if (!reserved && threadIdx.x == 0) s_ob = tot ? atomicAdd(&C.dyn[q].fill, (unsigned long long)tot) : 0;
                }
                reserved = true;
                need_hist = false;
                __syncthreads();
            }
            const int b0 = nxt[lev];
            const K width = rhi[lev] - rlo[lev];
            const int nbk = (int)min((u64)IV_NB, ((u64)(width - 1) >> sh[lev]) + 1);
            if (b0 >= nbk) {
                lev--;
                continue;
            }
            // largest b1 > b0 with pairs(b0..b1) <= IV_CAP
            const u32 base = s_hist[lev][b0];
            int lo_b = b0 + 1, hi_b = nbk;
            while (lo_b < hi_b) {
                const int mid = (lo_b + hi_b + 1) >> 1;
                if (s_hist[lev][mid] - base <= (u32)IV_CAP) lo_b = mid;
                else hi_b = mid - 1;
            }
            int b1 = lo_b;
            const u32 m = s_hist[lev][b1] - base;
            const K klo = rlo[lev] + ((K)b0 << sh[lev]);
            K khi = (b1 >= nbk) ? rhi[lev] : rlo[lev] + ((K)b1 << sh[lev]);
            if (m > (u32)IV_CAP) {
                // one bucket holds too many pairs: refine it (its width is 2^sh;
                // four levels of 9 bits reach single monomials for 32-bit keys)
                if (sh[lev] > 0) {
                    if (lev + 1 >= IV_LEVELS) {  // cannot happen for 32-bit keys
                        __syncthreads();
                        if (threadIdx.x == 0) {
                            atomicOr(&C.counters[CNT_ERR_SPIN], 8u);
                            nxt[lev] = b1;
                        }
                        __syncthreads();
                        continue;
                    }
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        nxt[lev] = b1;
                        rlo[lev + 1] = klo;
                        rhi[lev + 1] = khi;
                    }
                    __syncthreads();
                    lev++;
                    need_hist = true;
                    continue;
                }
                // a single monomial with more than IV_CAP pairs: sum its pairs in
                // row-major order, IV_CAP at a time
                __syncthreads();
                if (threadIdx.x == 0) nxt[lev] = b1;
                u64 acc = 0;
                bool have = false;
                while (true) {
                    u32 c = 0;
                    for (u32 i = r0; i < r1; i++) {
                        const u32 j = cur[i];
                        if (j < nb && cf[i] + cg[j] == klo) c++;
                    }
                    u32 tot;
                    const u32 off = block_excl_scan<u32>(c, s_scan, tot);
                    if (tot == 0) break;
                    const u32 take = min(tot, (u32)IV_CAP);
                    u32 o = off;
                    for (u32 i = r0; i < r1; i++) {
                        const u32 j = cur[i];
                        if (j < nb && cf[i] + cg[j] == klo) {
                            if (o < take) {
                                s_x[o] = i * nb + j;
                                cur[i] = j + 1;
                            }
                            o++;
                        }
                    }
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        for (u32 e = 0; e < take; e++) {
                            const u32 x = s_x[e];
                            const u32 ii = div32(x, s.nb_div);
                            const u64 v = ring_mul<RING>(s.fc[ii], s.gc[x - ii * nb]);
                            acc = have ? ring_add<RING>(acc, v) : v;
                            have = true;
                        }
                        s_v[0] = acc;
                    }
                    __syncthreads();
                    acc = s_v[0];
                    have = true;
                    __syncthreads();
                }
                if (threadIdx.x == 0 && have && !ring_is_zero<RING>(acc)) {
                    const u64 rel = s_ob + s_run;
                    if ((i64)rel < s.stage_bound) {
                        ((K *)C.stB_k)[(u64)s.stage_base + rel] = klo;
                        ((u64 *)C.stB_v)[(u64)s.stage_base + rel] = acc;
                    } else {
                        atomicOr(&C.counters[CNT_ERR_SPIN], 16u);
                    }
                    s_run = s_run + 1;
                }
                __syncthreads();
                continue;
            }
            __syncthreads();
            if (threadIdx.x == 0) nxt[lev] = b1;
            __syncthreads();
            if (m == 0) continue;
            // generate the batch in row-major order
            u32 c = 0;
            for (u32 i = r0; i < r1; i++) {
                const K a = cf[i];
                for (u32 j = cur[i]; j < nb && a + cg[j] < khi; j++) c++;
            }
            u32 tot;
            u32 o = block_excl_scan<u32>(c, s_scan, tot);
            for (u32 i = r0; i < r1; i++) {
                const K a = cf[i];
                u32 j = cur[i];
                for (; j < nb; j++) {
                    const K key = a + cg[j];
                    if (key >= khi) break;
                    if (o < (u32)IV_CAP) {
                        s_k[o] = (u32)(key - klo);
                        s_x[o] = i * nb + j;
                    }
                    o++;
                }
                cur[i] = j;
            }
            if (tot > (u32)IV_CAP) {  // histogram and walk disagree: cannot happen
                if (threadIdx.x == 0) atomicOr(&C.counters[CNT_ERR_SPIN], 16u);
                tot = IV_CAP;
            }
            __syncthreads();
            int kb = 0;
            while (kb < 32 && ((u64)1 << kb) < (u64)(khi - klo)) kb++;
            lds_sort_pairs(s_k, s_x, (int)tot, kb, s_wh, s_scan);
            // run sums: thread t owns items [t*IPT, t*IPT+IPT)
            const int i0 = threadIdx.x * IPT;
            u32 mask = 0;
            int open = -1;
            u64 acc = 0;
            for (int r = 0; r < IPT; r++) {
                const int e = i0 + r;
                if (e >= (int)tot) break;
                const u32 kk = s_k[e];
                const bool head = e == 0 || kk != s_k[e - 1];
                const u32 x = s_x[e];
                const u32 ii = div32(x, s.nb_div);
                const u64 v = ring_mul<RING>(s.fc[ii], s.gc[x - ii * nb]);
                if (head) {
                    if (open >= 0) {
                        s_v[i0 + open] = acc;
                        if (!ring_is_zero<RING>(acc)) mask |= 1u << open;
                    }
                    open = r;
                    acc = v;
                } else if (open >= 0) {
                    acc = ring_add<RING>(acc, v);
                }
            }
            if (open >= 0) {
                const u32 kk = s_k[i0 + open];
                for (int e = i0 + IPT; e < (int)tot && s_k[e] == kk; e++) {
                    const u32 x = s_x[e];
                    const u32 ii = div32(x, s.nb_div);
                    acc = ring_add<RING>(acc, ring_mul<RING>(s.fc[ii], s.gc[x - ii * nb]));
                }
                s_v[i0 + open] = acc;
                if (!ring_is_zero<RING>(acc)) mask |= 1u << open;
            }
            u32 rt;
            const u32 ro = block_excl_scan<u32>((u32)__popc(mask), s_scan, rt);
            const u64 rel0 = s_ob + s_run + ro;
            u32 w = 0;
            bool over = false;
            for (int r = 0; r < IPT; r++) {
                if (mask & (1u << r)) {
                    if ((i64)(rel0 + w) < s.stage_bound) {
                        ((K *)C.stB_k)[(u64)s.stage_base + rel0 + w] = klo + (K)s_k[i0 + r];
                        ((u64 *)C.stB_v)[(u64)s.stage_base + rel0 + w] = s_v[i0 + r];
                    } else {
                        over = true;
                    }
                    w++;
                }
            }
            if (over) atomicOr(&C.counters[CNT_ERR_SPIN], 16u);
            __syncthreads();
            if (threadIdx.x == 0) s_run = s_run + rt;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            IvalItem &I = C.iv_items_arr[it];
            I.ostart = s.stage_base + s_ob;
            I.ocount = s_run;
        }
        __syncthreads();
    }
}

// Result offsets of every interval of every product (one workgroup per
// product), then n_out.
__global__ __launch_bounds__(NTHREADS) void k_ival_scan(Ctx C) {
    __shared__ unsigned long long s_scan[NTHREADS / 64];
    __shared__ unsigned long long s_carry;
    const int qs = blockIdx.x;
    const int q = C.iv_seg[qs];
    const DevSeg &s = C.segs[q];
    const i64 first = C.iv_pre[qs], nint = C.dyn[q].n;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (i64 b = 0; b < nint; b += NTHREADS) {
        const i64 k = b + threadIdx.x;
        const unsigned long long c = k < nint ? C.iv_items_arr[first + k].ocount : 0;
        unsigned long long tot;
        const unsigned long long off = block_excl_scan<unsigned long long>(c, s_scan, tot);
        if (k < nint) C.iv_off[first + k] = s_carry + off;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *s.n_out = (i64)s_carry;
}

// Concatenate: interval results to their place in h, keys decompressed.
template <typename K>
__global__ __launch_bounds__(NTHREADS) void k_ival_copy(Ctx C) {
    for (i64 it = blockIdx.x; it < C.iv_items; it += gridDim.x) {
        const i32 qs = seg_search(C.iv_pre, C.nivseg, it);
        const int q = C.iv_seg[qs];
        const DevSeg &s = C.segs[q];
        const i64 k = it - C.iv_pre[qs];
        if (k >= C.dyn[q].n) continue;
        const IvalItem I = C.iv_items_arr[it];
        const u64 dst = C.iv_off[it];
        const VarParam *vp = C.vars + s.var_off;
        const u64 send = (u64)s.stage_base + (u64)s.stage_bound;
        for (u64 e = threadIdx.x; e < I.ocount; e += NTHREADS) {
            const u64 pos = dst + e;
            if ((i64)pos < s.cap && I.ostart + e < send) {
                s.hk[pos] = decompress<K>(((const K *)C.stB_k)[I.ostart + e], vp, C.nvars, s.lo_key);
                s.hc[pos] = ((const u64 *)C.stB_v)[I.ostart + e];
            }
        }
    }
}

}  // namespace pm
