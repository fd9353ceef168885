// Exact integer coefficients beyond one machine word (ring PM_Z192).
//
// The paper's benchmark section sums integer coefficients exactly in a
// three-word accumulator.  Here the coefficients are 192-bit two's-complement
// integers and the product is formed from three modular products that the
// exact-ring kernels already compute, followed by the Chinese remainder
// theorem:
//   m1 = 2^64          (the int64 ring: wrapping arithmetic)
//   m2 = 2^61 - 1      (the mod-p ring)
//   m3 = 2^64 - 59     (the mod-q ring)
// M = m1 m2 m3 is about 2^189, so every integer in (-M/2, M/2) is recovered
// from its three residues.  An output coefficient is bounded by
// min(n_f, n_g) max|a_i| max|b_j|; the call is refused (PM_EOVERFLOW) unless
// that bound is below 2^187.
//
// Steps, all enqueued on the caller's stream:
//   k_z_residues   each operand coefficient -> its three residues, and the
//                  bit length of its magnitude (read back for the bound)
//   three products through the ordinary pipeline, one per modulus
//   k_z_place      the three sorted result lists are merged by key (a term's
//                  place is its index plus its rank in the other two lists);
//                  a monomial whose coefficient vanishes modulo one m_k is
//                  missing from that list only
//   k_z_heads / k_z_head_scan / k_z_union
//                  equal neighbours of the merged list collapse into one
//                  union entry holding the three residues (0 where missing)
//   k_z_crt        Garner's form of the Chinese remainder theorem, signed
//                  result as three words; zero never occurs (a key is in the
//                  union only if some residue is non-zero)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/polymul.h"
#include "pm_api_internal.hpp"

namespace pm {

namespace {

constexpr int ZT = 256;       // threads of the element-wise kernels
constexpr int ZCH = 4096;     // merged slots per head-count block (ZT x 16)
constexpr int ZS_T = 1024;    // threads of the block-sum scan

constexpr u64 powmod(u64 a, u64 e, u64 m) {
    unsigned __int128 r = 1, b = a % m;
    while (e) {
        if (e & 1) r = r * b % m;
        b = b * b % m;
        e >>= 1;
    }
    return (u64)r;
}
constexpr u64 P61C = (1ull << 61) - 1;
constexpr u64 INV_M1_P = powmod(8, P61C - 2, P61C);         // (2^64)^-1 mod p, 2^64 = 8
constexpr u64 INV_M1_Q = powmod(Q64_C, Q64 - 2, Q64);       // (2^64)^-1 mod q, 2^64 = 59
constexpr u64 INV_P_Q = powmod(P61C, Q64 - 2, Q64);         // p^-1 mod q
constexpr unsigned __int128 PQ = (unsigned __int128)P61C * Q64;
static_assert(INV_M1_P == (1ull << 58), "8 * 2^58 = 2^61 = 1 (mod p)");

// Workspace regions of one PM_Z192 product.
struct ZLayout {
    size_t ctr, fr, gr, subk, subc, mkey, mres, msrc, bsum, ukey, ures, sub, total;
    int64_t bound, nblk;
};

size_t zal(size_t x) { return (x + 255) & ~(size_t)255; }

ZLayout z_layout(int64_t na, int64_t nb, int64_t bound, int64_t sub_bytes) {
    ZLayout z{};
    const size_t B = (size_t)std::max<int64_t>(bound, 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = zal(o + bytes);
        return at;
    };
    z.bound = (int64_t)B;
    z.nblk = (int64_t)((3 * B + ZCH - 1) / ZCH);
    z.ctr = take(64);
    z.fr = take(3 * 8 * (size_t)std::max<int64_t>(na, 1));
    z.gr = take(3 * 8 * (size_t)std::max<int64_t>(nb, 1));
    z.subk = take(3 * 8 * B);
    z.subc = take(3 * 8 * B);
    z.mkey = take(3 * 8 * B);
    z.mres = take(3 * 8 * B);
    z.msrc = take(3 * B);
    z.bsum = take(8 * (size_t)z.nblk);
    z.ukey = take(8 * B);
    z.ures = take(3 * 8 * B);
    z.sub = take((size_t)sub_bytes);
    z.total = o;
    return z;
}

// Counters at z.ctr: [0] u32 magnitude bits of f, [1] of g; then i64 union
// size at +8 and the three sub-product term counts at +16.
struct ZCtr {
    u32 bits[2];
    i64 nu;
    i64 nsub[3];
};

__device__ inline u64 fold_p(u64 x) {  // any u64 -> [0, p)
    u64 r = (x & P61C) + (x >> 61);
    return r >= P61C ? r - P61C : r;
}
__device__ inline u64 mod_q(u64 x) { return x >= Q64 ? x - Q64 : x; }
__device__ inline u64 submod_p(u64 a, u64 b) { return a >= b ? a - b : a + P61C - b; }
__device__ inline u64 submod_q(u64 a, u64 b) { return a >= b ? a - b : a + (Q64 - b); }

// Residues of a 192-bit two's-complement value w (least significant word first):
// U = w0 + 2^64 w1 + 2^128 w2 and, when negative, v = U - 2^192.
//   mod p: 2^64 = 8, 2^128 = 64, 2^192 = 2^9;  mod q: 2^64 = 59, powers of 59.
__global__ __launch_bounds__(ZT) void k_z_residues(const u64 *w, i64 n, u64 *r1, u64 *r2, u64 *r3, u32 *bits) {
    __shared__ u32 s_b[ZT / 64];
    u32 mb = 0;
    for (i64 i = (i64)blockIdx.x * ZT + threadIdx.x; i < n; i += (i64)gridDim.x * ZT) {
        const u64 w0 = w[3 * i], w1 = w[3 * i + 1], w2 = w[3 * i + 2];
        const bool neg = (w2 >> 63) != 0;
        r1[i] = w0;
        u64 p = addmod61(addmod61(fold_p(w0), mulmod61(fold_p(w1), 8)), mulmod61(fold_p(w2), 64));
        if (neg) p = submod_p(p, 1ull << 9);
        r2[i] = p;
        u64 q = addmodq(addmodq(mod_q(w0), mulmodq(mod_q(w1), Q64_C)), mulmodq(mod_q(w2), Q64_C * Q64_C));
        if (neg) q = submod_q(q, Q64_C * Q64_C * Q64_C);
        r3[i] = q;
        // magnitude: two's-complement negation of a negative value
        u64 m0 = w0, m1 = w1, m2 = w2;
        if (neg) {
            m0 = ~w0 + 1;
            const u64 c0 = m0 == 0 ? 1 : 0;
            m1 = ~w1 + c0;
            const u64 c1 = (c0 && m1 == 0) ? 1 : 0;
            m2 = ~w2 + c1;
        }
        const u32 b = m2 ? 192 - (u32)__clzll((long long)m2)
                         : m1 ? 128 - (u32)__clzll((long long)m1) : m0 ? 64 - (u32)__clzll((long long)m0) : 0;
        mb = b > mb ? b : mb;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const u32 o = (u32)__shfl_xor((int)mb, d, 64);
        mb = o > mb ? o : mb;
    }
    if ((threadIdx.x & 63) == 0) s_b[threadIdx.x >> 6] = mb;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 m = 0;
        for (int k = 0; k < ZT / 64; k++) m = s_b[k] > m ? s_b[k] : m;
        atomicMax(bits, m);
    }
}

// Number of entries of the ascending list a[0..n) below x (or <= x).
__device__ inline i64 z_rank(const u64 *a, i64 n, u64 x, bool inclusive) {
    i64 lo = 0, hi = n;
    while (lo < hi) {
        const i64 mid = (lo + hi) >> 1;
        if (a[mid] < x || (inclusive && a[mid] == x)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merged order of the three lists, equal keys in list order: entry i of list
// X goes to i + (entries of earlier lists <= key) + (of later lists < key).
__global__ __launch_bounds__(ZT) void k_z_place(const u64 *subk, const u64 *subc, const ZCtr *ctr, i64 B, u64 *mkey,
                                                u64 *mres, unsigned char *msrc) {
    const int X = blockIdx.y;
    const i64 n = min(ctr->nsub[X], B);
    const u64 *k = subk + X * B;
    for (i64 i = (i64)blockIdx.x * ZT + threadIdx.x; i < n; i += (i64)gridDim.x * ZT) {
        const u64 key = k[i];
        i64 pos = i;
        for (int Y = 0; Y < 3; Y++)
            if (Y != X) pos += z_rank(subk + Y * B, min(ctr->nsub[Y], B), key, Y < X);
        mkey[pos] = key;
        mres[pos] = subc[X * B + i];
        msrc[pos] = (unsigned char)X;
    }
}

__device__ inline i64 z_len(const ZCtr *ctr, i64 B) {
    return min(ctr->nsub[0], B) + min(ctr->nsub[1], B) + min(ctr->nsub[2], B);
}

// Union heads (a slot whose key differs from its predecessor) per block of ZCH slots.
__global__ __launch_bounds__(ZT) void k_z_heads(const u64 *mkey, const ZCtr *ctr, i64 B, i64 *bsum) {
    __shared__ u32 s[ZT / 64];
    const i64 L = z_len(ctr, B);
    const i64 b0 = (i64)blockIdx.x * ZCH;
    u32 c = 0;
    for (int k = 0; k < ZCH / ZT; k++) {
        const i64 t = b0 + (i64)k * ZT + threadIdx.x;
        if (t < L && (t == 0 || mkey[t] != mkey[t - 1])) c++;
    }
    for (int d = 32; d >= 1; d >>= 1) c += (u32)__shfl_xor((int)c, d, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (int k = 0; k < ZT / 64; k++) t += s[k];
        bsum[blockIdx.x] = t;
    }
}

// Exclusive prefix of the block counts (one workgroup); the union size goes
// to the counters and to the caller's n_out.
__global__ __launch_bounds__(ZS_T) void k_z_head_scan(i64 *bsum, i64 nblk, ZCtr *ctr, i64 *n_out) {
    __shared__ i64 s[ZS_T / 64];
    i64 carry = 0;
    for (i64 b = 0; b < nblk; b += ZS_T) {
        const i64 i = b + threadIdx.x;
        const i64 v = i < nblk ? bsum[i] : 0;
        i64 x = v;
        const int lane = threadIdx.x & 63;
        for (int d = 1; d < 64; d <<= 1) {
            const i64 y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) s[threadIdx.x >> 6] = x;
        __syncthreads();
        i64 pre = 0, tot = 0;
        for (int w = 0; w < ZS_T / 64; w++) {
            if (w < (int)(threadIdx.x >> 6)) pre += s[w];
            tot += s[w];
        }
        if (i < nblk) bsum[i] = carry + pre + x - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctr->nu = carry;
        *n_out = carry;
    }
}

// Union entries: keys, and each slot's residue in its list's column.
__global__ __launch_bounds__(ZT) void k_z_union(const u64 *mkey, const u64 *mres, const unsigned char *msrc,
                                                const ZCtr *ctr, i64 B, const i64 *bpre, u64 *ukey, u64 *ures) {
    __shared__ u32 s[ZT / 64];
    const i64 L = z_len(ctr, B);
    const i64 b0 = (i64)blockIdx.x * ZCH;
    i64 base = bpre[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < ZCH / ZT; k++) {
        const i64 t = b0 + (i64)k * ZT + threadIdx.x;
        const bool in = t < L;
        const bool head = in && (t == 0 || mkey[t] != mkey[t - 1]);
        const u64 bal = __ballot(head);
        const u32 below = (u32)__popcll(bal & ((1ull << lane) - 1));
        if (lane == 0) s[w] = (u32)__popcll(bal);
        __syncthreads();
        u32 wpre = 0, tot = 0;
        for (int v = 0; v < ZT / 64; v++) {
            if (v < w) wpre += s[v];
            tot += s[v];
        }
        // union index of slot t: heads up to and including t, minus one
        const i64 u = base + wpre + below + (head ? 1 : 0) - 1;
        if (in) {
            if (head) ukey[u] = mkey[t];
            ures[3 * u + msrc[t]] = mres[t];
        }
        base += tot;
        __syncthreads();
    }
}

// Garner: x = r1 + 2^64 (v2 + p v3) with v2 = (r2 - r1) / 2^64 mod p and
// v3 = ((r3 - r1) / 2^64 - v2) / p mod q; x in [0, M) is taken as x - M when
// x >= M/2, which (writing x = r1 + 2^64 Y) is 2 Y + r1 / 2^63 >= p q.
__global__ __launch_bounds__(ZT) void k_z_crt(const u64 *ukey, const u64 *ures, const ZCtr *ctr, u64 *hk, u64 *hc,
                                              i64 cap) {
    const i64 n = min(ctr->nu, cap);
    for (i64 u = (i64)blockIdx.x * ZT + threadIdx.x; u < n; u += (i64)gridDim.x * ZT) {
        const u64 r1 = ures[3 * u], r2 = ures[3 * u + 1], r3 = ures[3 * u + 2];
        const u64 v2 = mulmod61(submod_p(r2, fold_p(r1)), INV_M1_P);
        const u64 t = mulmodq(submod_q(r3, mod_q(r1)), INV_M1_Q);
        const u64 v3 = mulmodq(submod_q(t, v2), INV_P_Q);  // v2 < p < q is already reduced mod q
        unsigned __int128 Y = (unsigned __int128)v3 * P61C + v2;  // < p q + p < 2^125
        if (2 * Y + (r1 >> 63) >= PQ) Y -= PQ;                   // negative: two's complement in 128 bits
        hk[u] = ukey[u];
        hc[3 * u] = r1;
        hc[3 * u + 1] = (u64)Y;
        hc[3 * u + 2] = (u64)(Y >> 64);
    }
}

__global__ void k_z_fill(u64 *p, i64 n) {
    for (i64 i = (i64)blockIdx.x * ZT + threadIdx.x; i < n; i += (i64)gridDim.x * ZT) p[i] = 0;
}

__global__ void k_z_zero_count(i64 *n_out) { *n_out = 0; }

int grid_of(i64 n, int cap) { return (int)std::max<i64>(1, std::min<i64>((n + ZT - 1) / ZT, cap)); }

}  // namespace

// Bound and workspace of a PM_Z192 product: the plan of the int64 product of
// the same operands (its keys decide the bound and the pipeline's workspace),
// plus the residue, merge and union regions.
int z192_bound(HostStage &hs, const pm_layout *L, const pm_cpoly *f, const pm_cpoly *g, int64_t *max_terms,
               int64_t *ws_bytes, hipStream_t st, const Tuning &tune) {
    pm_layout l64 = *L;
    l64.ring = PM_I64;
    int64_t b = 0, w = 0;
    int rc = bound_impl(hs, &l64, 1, f, g, &b, &w, st, tune);
    if (rc) return rc;
    if (max_terms) *max_terms = b;
    if (ws_bytes) *ws_bytes = (int64_t)z_layout(f->n, g->n, b, w).total;
    return PM_OK;
}

int z192_mul(HostStage &hs, const pm_layout *L, const pm_cpoly *f, const pm_cpoly *g, const pm_poly *h, void *ws,
             int64_t ws_bytes, hipStream_t st, const Tuning &tune) {
    if (!ws) return PM_ENOMEM;
    if ((uintptr_t)ws & 255) return PM_EINVAL;
    if (f->n == 0 || g->n == 0) {
        hipLaunchKernelGGL(k_z_zero_count, dim3(1), dim3(1), 0, st, (i64 *)h->n_out);
        return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
    }
    // the int64 plan sizes everything (validates keys; the coefficient words
    // themselves need no range check); its statistics use the workspace
    pm_layout l64 = *L;
    l64.ring = PM_I64;
    const size_t need0 = stats_region_bytes(1, (int)L->nvars) + sizeof(DevSeg);
    if (ws_bytes < (int64_t)need0) return PM_ENOMEM;
    Plan P0;
    int rc = stats_and_plan(hs, &l64, 1, f, g, ws, st, tune, P0);
    if (rc) return rc;
    const int64_t B = P0.bound[0], wsub = (int64_t)P0.total;
    const ZLayout z = z_layout(f->n, g->n, B, wsub);
    if ((int64_t)z.total > ws_bytes) return PM_ENOMEM;
    char *base = (char *)ws;
    ZCtr *ctr = (ZCtr *)(base + z.ctr);
    u64 *fr = (u64 *)(base + z.fr), *gr = (u64 *)(base + z.gr);
    const i64 na = f->n, nb = g->n;
    hipError_t e = hipMemsetAsync(ctr, 0, sizeof(ZCtr), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_z_residues, dim3(grid_of(na, 1024)), dim3(ZT), 0, st, (const u64 *)f->coefs, na, fr,
                           fr + na, fr + 2 * na, &ctr->bits[0]);
        hipLaunchKernelGGL(k_z_residues, dim3(grid_of(nb, 1024)), dim3(ZT), 0, st, (const u64 *)g->coefs, nb, gr,
                           gr + nb, gr + 2 * nb, &ctr->bits[1]);
        e = hipGetLastError();
    }
    u32 bits[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(bits, ctr->bits, sizeof(bits), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error("exact-integer residues", e);
        return PM_EDEVICE;
    }
    // |c| <= min(na, nb) (2^bf - 1)(2^bg - 1) < 2^(bf + bg + bitlen(min(na, nb)))
    const i64 mn = std::min(na, nb);
    int lm = 0;
    while ((i64(1) << lm) <= mn && lm < 63) lm++;
    if ((int)bits[0] + (int)bits[1] + lm > 187) return PM_EOVERFLOW;
    // one product per modulus, results side by side
    const int rings[3] = {PM_I64, PM_MODP61, PM_MODQ64};
    u64 *subk = (u64 *)(base + z.subk), *subc = (u64 *)(base + z.subc);
    for (int X = 0; X < 3; X++) {
        pm_layout lx = *L;
        lx.ring = rings[X];
        const pm_cpoly fx{f->n, f->keys, fr + X * na};
        const pm_cpoly gx{g->n, g->keys, gr + X * nb};
        const pm_poly hx{B, &ctr->nsub[X], subk + X * B, subc + X * B};
        rc = mul_impl(hs, &lx, 1, &fx, &gx, &hx, base + z.sub, (int64_t)(z.total - z.sub), st, tune, nullptr);
        if (rc) return rc;
    }
    u64 *mkey = (u64 *)(base + z.mkey), *mres = (u64 *)(base + z.mres);
    unsigned char *msrc = (unsigned char *)(base + z.msrc);
    i64 *bsum = (i64 *)(base + z.bsum);
    u64 *ukey = (u64 *)(base + z.ukey), *ures = (u64 *)(base + z.ures);
    hipLaunchKernelGGL(k_z_fill, dim3(grid_of(3 * B, 2048)), dim3(ZT), 0, st, ures, (i64)(3 * B));
    hipLaunchKernelGGL(k_z_place, dim3(grid_of(B, 2048), 3), dim3(ZT), 0, st, (const u64 *)subk, (const u64 *)subc,
                       (const ZCtr *)ctr, (i64)B, mkey, mres, msrc);
    hipLaunchKernelGGL(k_z_heads, dim3((unsigned)z.nblk), dim3(ZT), 0, st, (const u64 *)mkey, (const ZCtr *)ctr,
                       (i64)B, bsum);
    hipLaunchKernelGGL(k_z_head_scan, dim3(1), dim3(ZS_T), 0, st, bsum, (i64)z.nblk, ctr, (i64 *)h->n_out);
    hipLaunchKernelGGL(k_z_union, dim3((unsigned)z.nblk), dim3(ZT), 0, st, (const u64 *)mkey, (const u64 *)mres,
                       (const unsigned char *)msrc, (const ZCtr *)ctr, (i64)B, (const i64 *)bsum, ukey, ures);
    if (h->capacity > 0)
        hipLaunchKernelGGL(k_z_crt, dim3(grid_of(B, 2048)), dim3(ZT), 0, st, (const u64 *)ukey, (const u64 *)ures,
                           (const ZCtr *)ctr, (u64 *)h->keys, (u64 *)h->coefs, (i64)h->capacity);
    e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("exact-integer merge", e);
        return PM_EDEVICE;
    }
    return PM_OK;
}

}  // namespace pm
