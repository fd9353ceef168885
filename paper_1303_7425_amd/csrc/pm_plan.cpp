// Host planner: see pm_plan.hpp.
#include "pm_plan.hpp"

#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/polymul.h"

namespace pm {

static std::mutex g_tune_mu;
struct TuneChoice {
    int tile_cfg, combine, digits;
};
static std::map<TuneClass, TuneChoice> g_tune_cache;

bool tune_lookup(const TuneClass &c, int &tile_cfg, int &combine, int &digits) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(c);
    if (it == g_tune_cache.end()) return false;
    tile_cfg = it->second.tile_cfg;
    combine = it->second.combine;
    digits = it->second.digits;
    return true;
}

void tune_store(const TuneClass &c, int tile_cfg, int combine, int digits) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[c] = {tile_cfg, combine, digits};
}

void tune_reset() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
}

// Text file, one choice per line: ring dense log2pairs tile_cfg combine digits.
int tune_save(const char *path) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = fopen(path, "w");
    if (!f) return PM_EINVAL;
    fprintf(f, "# polymul tuning: ring dense log2pairs tile_cfg combine digits\n");
    for (auto &kv : g_tune_cache)
        fprintf(f, "%d %d %d %d %d %d\n", kv.first.ring, kv.first.dense, kv.first.log2pairs, kv.second.tile_cfg,
                kv.second.combine, kv.second.digits);
    return fclose(f) == 0 ? PM_OK : PM_EINVAL;
}

int tune_load(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return PM_EINVAL;
    std::vector<std::pair<TuneClass, TuneChoice>> got;
    char line[256];
    int rc = PM_OK;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        int r, d, l, t, c, g;
        if (sscanf(line, "%d %d %d %d %d %d", &r, &d, &l, &t, &c, &g) != 6 || r < 0 || r > 4 || d < 0 || d > 1 ||
            l < 0 || l > 127 || t < -1 || t >= N_TILE_CFGS || c < -1 || c > 3 || g < -1 || g > 1) {
            rc = PM_EINVAL;
            break;
        }
        got.push_back({TuneClass{r, d, l}, TuneChoice{t, c, g}});
    }
    fclose(f);
    if (rc != PM_OK) return rc;  // nothing is taken from a malformed file
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &e : got) g_tune_cache[e.first] = e.second;
    return PM_OK;
}

// Digit widths of the radix passes over the keys' significant bits: 8 bits
// per pass with the remainder in the last (RADIX_DIGITS_GREEDY), or the same
// number of passes with widths as equal as possible, wider ones first
// (RADIX_DIGITS_BALANCED): fewer digit values give longer runs per digit and
// fuller cache lines in the scatter.
void set_digits(Plan &P, int schedule) {
    int shift = 0;
    for (int p = 0; p < P.passes; p++) {
        int w;
        if (schedule == RADIX_DIGITS_GREEDY) {
            w = std::min(RADIX_BITS, std::max(1, P.max_bits - shift));
        } else {
            const int rest = std::max(P.passes, P.max_bits - shift), left = P.passes - p;
            w = std::min(RADIX_BITS, (rest + left - 1) / left);
        }
        P.dsh[p] = (unsigned char)shift;
        P.dbits[p] = (unsigned char)w;
        shift += w;
    }
}

int log2_floor(uint64_t x) {
    int b = -1;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t stats_region_bytes(int nseg, int nvars) {
    return align256(stats_bytes(nseg, nvars)) + align256((size_t)nseg * 2 * sizeof(uint32_t));
}

static int bitlen128(unsigned __int128 x) {
    int b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

int plan_build(int nvars, int bits, int ring, const std::vector<SegInput> &in, const uint64_t *stats,
               const uint32_t *flags, const Tuning &tune_in, Plan &P, int cus) {
    const int S = (int)in.size();
    P = Plan();
    P.nseg = S;
    P.nvars = nvars;
    P.bits = bits;
    P.ring = ring;
    const uint64_t fmask = bits == 64 ? ~0ull : ((1ull << bits) - 1);

    // validation verdicts, most fundamental first
    uint32_t all = 0;
    for (int q = 0; q < S; q++) all |= flags[2 * q] | flags[2 * q + 1];
    if (all & ST_BADBITS) return PM_EINVAL;
    if (all & ST_UNSORTED) return PM_EUNSORTED;
    if (all & ST_RANGE) return PM_ERANGE;

    P.segs.resize(S);
    P.vars.resize((size_t)S * nvars);
    P.bound.assign(S, 0);
    std::vector<unsigned __int128> box(S, 0);
    int max_bits = 0;
    bool need_u64 = false;
    for (int q = 0; q < S; q++) {
        DevSeg &d = P.segs[q];
        d = DevSeg();
        d.fk = in[q].fk;
        d.fc = in[q].fc;
        d.gk = in[q].gk;
        d.gc = in[q].gc;
        d.na = in[q].na;
        d.nb = in[q].nb;
        d.var_off = (int64_t)q * nvars;
        if (d.na == 0 || d.nb == 0) {
            d.mode = SEG_EMPTY;
            continue;
        }
        const uint64_t *st = stats + (size_t)q * 4 * nvars;  // f: min[nv] max[nv], g: min[nv] max[nv]
        const uint64_t *fmin = st, *fmax = st + nvars, *gmin = st + 2 * nvars, *gmax = st + 3 * nvars;
        unsigned __int128 b = 1;
        bool big = false;
        uint64_t lo_key = 0;
        for (int v = 0; v < nvars; v++) {
            if (fmax[v] > fmask - gmax[v]) return PM_EOVERFLOW;
            unsigned __int128 r = (unsigned __int128)(fmax[v] + gmax[v]) - (fmin[v] + gmin[v]) + 1;
            VarParam &vp = P.vars[(size_t)q * nvars + v];
            vp.shift = (uint32_t)((nvars - 1 - v) * bits);
            vp.mask = fmask;
            vp.minf = fmin[v];
            vp.ming = gmin[v];
            vp.range = (uint64_t)r;  // 0 encodes 2^64 (one full-width variable)
            if (r <= 0xFFFFFFFFull) vp.rdiv = make_div32((uint32_t)r);
            lo_key += (fmin[v] + gmin[v]) << vp.shift;
            if (!big) {
                b *= r;
                if (b >> 64) big = true;
            }
        }
        // strides: stride_v = prod_{w > v} range_w
        unsigned __int128 st_acc = 1;
        for (int v = nvars - 1; v >= 0; v--) {
            VarParam &vp = P.vars[(size_t)q * nvars + v];
            vp.stride = (uint64_t)st_acc;
            unsigned __int128 r = vp.range ? vp.range : ((unsigned __int128)1 << 64);
            st_acc *= r;
            if (st_acc >> 65) st_acc = (unsigned __int128)1 << 65;  // only reached when box > 2^64
        }
        d.lo_key = lo_key;
        box[q] = big ? ((unsigned __int128)1 << 64) : b;
        const unsigned __int128 prod = (unsigned __int128)d.na * (unsigned __int128)d.nb;
        const unsigned __int128 bnd = std::min(prod, box[q]);
        P.bound[q] = (int64_t)bnd;
        // path
        // the degree box when it is small against the pairs, and also for a
        // product that no sparse path can take (their staged items address
        // pairs with 32 bits)
        const bool sparse_too_big = prod > (unsigned __int128)0xFFFFFFFFull;
        const bool can_dense = tune_in.allow_dense && ring != RING_F64 && box[q] <= (unsigned __int128)tune_in.dense_max_cells &&
                               ((double)box[q] * tune_in.dense_ratio <= (double)prod || sparse_too_big);
        if (can_dense) {
            d.mode = SEG_DENSE;
        } else {
            d.mode = SEG_RAW;  // decided for the whole launch below
            int kb = bitlen128(box[q] - 1);
            max_bits = std::max(max_bits, kb);
        }
        if (box[q] > (unsigned __int128)0xFFFFFFFFull) need_u64 = true;
    }
    P.ksize = need_u64 ? 8 : 4;
    P.passes = (max_bits + RADIX_BITS - 1) / RADIX_BITS;
    P.max_bits = max_bits;

    // automatic settings: the autotuner's choice for the largest product's class
    Tuning tune = tune_in;
    {
        int big = -1;
        unsigned __int128 bigp = 0;
        for (int q = 0; q < S; q++) {
            const unsigned __int128 pr = (unsigned __int128)P.segs[q].na * P.segs[q].nb;
            if (P.segs[q].mode != SEG_EMPTY && pr > bigp) {
                bigp = pr;
                big = q;
            }
        }
        if (big >= 0) {
            TuneClass tc{ring, P.segs[big].mode == SEG_DENSE ? 1 : 0, log2_floor((uint64_t)bigp)};
            int tcfg, comb, dig;
            if (tune_lookup(tc, tcfg, comb, dig)) {
                if (tune.tile_cfg < 0) tune.tile_cfg = tcfg;
                if (tune.combine < 0) tune.combine = comb;
                if (tune.digits < 0) tune.digits = dig;
            }
        }
    }

    // one sort mode per launch: pair indices (products regenerated in the
    // reduction, FP64 summed in row-major order) or LDS-combined coefficients
    // (exact rings only; needs a free hash sentinel, i.e. box < 2^(8*ksize)).
    bool idx_fits = true, sentinel_ok = true;
    for (int q = 0; q < S; q++) {
        if (P.segs[q].mode != SEG_RAW) continue;
        if ((unsigned __int128)P.segs[q].na * P.segs[q].nb > 0xFFFFFFFFull) idx_fits = false;
        if (box[q] >= ((unsigned __int128)1 << 64)) sentinel_ok = false;
    }
    // output-key intervals: 32-bit compressed keys and 32-bit pair indices
    if (P.ksize == 4 && idx_fits && tune.combine == 2) {
        for (int q = 0; q < S; q++) {
            if (P.segs[q].mode != SEG_RAW) continue;
            DevSeg &d = P.segs[q];
            d.mode = SEG_IVAL;
            const double target = std::max(1.0, (double)d.na * (double)d.nb / 32768.0);
            int64_t l = (int64_t)std::ceil(std::sqrt(target)) - 1;
            l = std::max<int64_t>(0, std::min<int64_t>(l, 63));
            l = std::min<int64_t>(l, std::min(d.na, d.nb));
            d.iv_l = l;
        }
    }
    // output-key work items: products with 32-bit compressed keys and pair
    // indices whose single monomials can never hold more than BK_CAP pairs
    // (at most min(na, nb) pairs share a monomial)
    // (automatic for the exact rings; FP64 sorts each work item by row and key
    // in LDS, slower than the pair-index sort, so only on request)
    if (P.ksize == 4 && (tune.combine == 3 || (tune.combine == -1 && ring != RING_F64))) {
        for (int q = 0; q < S; q++) {
            DevSeg &d = P.segs[q];
            if (d.mode != SEG_RAW) continue;
            if ((unsigned __int128)d.na * d.nb > 0xFFFFFFFFull || std::min(d.na, d.nb) > BK_CAP) continue;
            d.mode = SEG_BKT;
        }
        idx_fits = true;
        sentinel_ok = true;
        for (int q = 0; q < S; q++) {
            if (P.segs[q].mode != SEG_RAW) continue;
            if ((unsigned __int128)P.segs[q].na * P.segs[q].nb > 0xFFFFFFFFull) idx_fits = false;
            if (box[q] >= ((unsigned __int128)1 << 64)) sentinel_ok = false;
        }
    }
    bool combine = ring != RING_F64 && sentinel_ok && (tune.combine == 1 || !idx_fits);
    if (!combine && !idx_fits) return PM_ENOMEM;  // FP64 product of more than 2^32 - 1 term pairs
    P.raw = combine ? 0 : 1;
    P.vsize = combine ? 8 : 4;
    for (int q = 0; q < S; q++)
        if (P.segs[q].mode == SEG_RAW && combine) P.segs[q].mode = SEG_COMBINE;
    // the combine path stages at most one item per term pair and addresses a
    // product's staging slots and sort partitions with 32-bit positions
    for (int q = 0; q < S; q++)
        if (P.segs[q].mode == SEG_COMBINE && (unsigned __int128)P.segs[q].na * P.segs[q].nb > 0xFFFFFFFFull)
            return PM_ENOMEM;
    bool any_sparse = false;
    for (int q = 0; q < S; q++) any_sparse |= P.segs[q].mode == SEG_RAW || P.segs[q].mode == SEG_COMBINE;
    if (!any_sparse) P.passes = 0;
    if (P.raw && any_sparse && P.passes == 0) P.passes = 1;  // pass 0 also generates the items
    set_digits(P, tune.digits == RADIX_DIGITS_GREEDY ? RADIX_DIGITS_GREEDY : RADIX_DIGITS_BALANCED);

    // tile shape: explicit, or the largest one that still gives >= 512 tiles
    // over the tiled products (at least two per compute unit); the sparse
    // combine path keeps the smallest table load (32 x 64 into 4096 slots).
    int64_t tiled_pairs = 0;
    bool any_combine = false;
    for (int q = 0; q < S; q++) {
        const DevSeg &d = P.segs[q];
        if (d.mode == SEG_COMBINE || d.mode == SEG_DENSE) tiled_pairs += d.na * d.nb;
        if (d.mode == SEG_COMBINE) any_combine = true;
    }
    if (tune.tile_cfg >= 0 && tune.tile_cfg < N_TILE_CFGS && (!any_combine || tile_cfg_combines(tune.tile_cfg))) {
        P.tile_cfg = tune.tile_cfg;
    } else if (any_combine) {
        P.tile_cfg = 0;
    } else {
        // a degree box with few pairs per cell (under 16) gives tiles with few
        // like terms: a tile of more pairs than table slots would overflow
        // its table into global atomics, so the shape stays at 64 x 64
        int top = N_TILE_CFGS - 1;
        for (int q = 0; q < S; q++) {
            const DevSeg &d = P.segs[q];
            if (d.mode == SEG_DENSE && (unsigned __int128)d.na * d.nb < 16 * box[q]) top = std::min(top, 1);
        }
        P.tile_cfg = 0;
        for (int c = top; c >= 0; c--) {
            if (tiled_pairs / ((int64_t)TILE_CFGS[c].tm * TILE_CFGS[c].tn) >= 512) {
                P.tile_cfg = c;
                break;
            }
        }
    }
    const TileCfg tc = TILE_CFGS[P.tile_cfg];

    // queues and offsets
    P.tile_pre.push_back(0);
    P.dpart_pre.push_back(0);
    P.cpre.push_back(0);
    int64_t nstage = 0, nbox = 0, nck = 0;
    for (int q = 0; q < S; q++) {
        DevSeg &d = P.segs[q];
        d.ck_f = nck;
        nck += d.na;
        d.ck_g = nck;
        nck += d.nb;
        P.cpre.push_back(P.cpre.back() + d.na);
        P.cpre.push_back(P.cpre.back() + d.nb);
        if (d.mode == SEG_COMBINE || d.mode == SEG_DENSE) {
            const int64_t tmn = (d.na + tc.tm - 1) / tc.tm, tnn = (d.nb + tc.tn - 1) / tc.tn;
            d.tile_first = P.tile_pre.back();
            d.tiles_n = tnn;
            P.tile_seg.push_back(q);
            P.tile_pre.push_back(P.tile_pre.back() + tmn * tnn);
        }
        if (d.mode == SEG_RAW) d.nb_div = make_div32((uint32_t)d.nb);
        if (d.mode == SEG_IVAL) {
            d.nb_div = make_div32((uint32_t)d.nb);
            d.stage_base = nstage;
            d.stage_bound = d.na * d.nb;
            nstage += (d.stage_bound + 63) & ~(int64_t)63;
            d.iv_samp_off = P.iv_nsamp;
            P.iv_nsamp += (d.iv_l + 1) * (d.iv_l + 1);
            d.iv_spl_off = P.iv_nspl;
            P.iv_nspl += (d.iv_l + 1) * (d.iv_l + 1) + 2;
            if (P.iv_pre.empty()) P.iv_pre.push_back(0);
            P.iv_seg.push_back(q);
            P.iv_pre.push_back(P.iv_pre.back() + (d.iv_l + 1) * (d.iv_l + 1) + 1);
            P.iv_maxrows = std::max<int64_t>(P.iv_maxrows, d.na);
            P.nival++;
        }
        if (d.mode == SEG_COMBINE || d.mode == SEG_RAW) {
            d.stage_base = nstage;
            d.stage_bound = d.na * d.nb;
            nstage += (d.stage_bound + 63) & ~(int64_t)63;  // products start on 64-item boundaries
            P.nparts_bound += (d.stage_bound + PART - 1) / PART;
            P.nsparse++;
        }
        if (d.mode == SEG_BKT) {
            // fine bins of about BK_BIN_PAIRS pairs each (at least one super-bin)
            const uint64_t pairs = (uint64_t)d.na * (uint64_t)d.nb;
            const uint64_t target = std::max<uint64_t>(BK_SB, pairs / BK_BIN_PAIRS);
            const uint64_t cells = (uint64_t)box[q];
            int fs = 0;
            while (((cells + (1ull << fs) - 1) >> fs) > target) fs++;
            const int64_t nbins = (int64_t)((cells + (1ull << fs) - 1) >> fs);
            const int64_t nsb = (nbins + BK_SB - 1) / BK_SB;
            d.bk_fs = fs;
            // exact rings: work items span at most 2^BK_RANK_LOG keys, so each
            // one is summed by rank in LDS without a sort
            d.bk_span_bins = (ring != RING_F64 && fs <= BK_RANK_LOG) ? (1 << (BK_RANK_LOG - fs)) : 0;
            d.bk_bin_off = P.bk_nbins;
            d.bk_sb_first = P.bk_nsb;
            d.bk_nsb = nsb;
            P.bk_nbins += nsb * BK_SB;
            P.bk_nsb += nsb;
            // generation tiles: up to BK_TN_MAX columns (a power of two), BK_TILE slots
            int tnl = 0;
            while ((1ll << tnl) < d.nb && (1 << tnl) < BK_TN_MAX) tnl++;
            d.bk_tnl = tnl;
            const int64_t tm = BK_TILE >> tnl, tn = 1ll << tnl;
            d.bk_tiles_n = (d.nb + tn - 1) / tn;
            d.bk_tile_first = P.bk_ntiles;
            if (P.bk_tile_pre.empty()) P.bk_tile_pre.push_back(0), P.bk_sb_pre.push_back(0);
            P.bk_ntiles += ((d.na + tm - 1) / tm) * d.bk_tiles_n;
            P.bk_tile_pre.push_back(P.bk_ntiles);
            P.bk_sb_pre.push_back(P.bk_nsb);
            P.bk_seg.push_back(q);
            // two consecutive work items of a super-bin hold more than BK_CAP
            // pairs, so a super-bin of p pairs has at most 2 ceil(p / BK_CAP) + 1
            // (or the first spans bk_span_bins bins)
            const int64_t span_items = d.bk_span_bins ? 2 * nsb * ((BK_SB + d.bk_span_bins - 1) / d.bk_span_bins) : 0;
            P.bk_wi_bound += 2 * (int64_t)((pairs + BK_CAP - 1) / BK_CAP) + 3 * nsb + 1 + span_items;
            P.bk_nstage += (int64_t)pairs;
            // a work item over BK_CAP pairs is one fine bin: at most 2^fs result terms
            const uint64_t fat_items = pairs / (BK_CAP + 1);
            P.bk_fat_cap += (int64_t)std::min<uint64_t>(pairs, fat_items << fs);
            d.nb_div = make_div32((uint32_t)d.nb);
            P.nbk++;
        }
        if (d.mode == SEG_DENSE) {
            d.stage_base = nbox;
            d.stage_bound = (int64_t)box[q];
            nbox += d.stage_bound;
            d.dpart_first = P.dpart_pre.back();
            P.dseg.push_back(q);
            P.dpart_pre.push_back(P.dpart_pre.back() + (d.stage_bound + PART - 1) / PART);
            P.ndense++;
        }
    }
    P.ntiles = P.tile_pre.back();
    P.ndparts = P.dpart_pre.back();
    P.nstage = nstage;
    if (P.iv_pre.empty()) P.iv_pre.push_back(0);
    P.iv_items = P.iv_pre.back();
    P.iv_grid = (int)std::max<int64_t>(1, std::min<int64_t>(P.iv_items, (int64_t)cus * 2));
    P.nbox = nbox;
    P.nck = nck;
    // digit counts of pair-index sorts regenerate keys from an LDS copy of
    // the product's compressed operand keys, up to 64 KB (two workgroups per
    // CU); larger products read them from global memory
    // Pair-index sorts regenerate each key from the operands' compressed keys
    // while those stay cache resident (gathers that hit in L2) and every
    // product's keys fit the digit count's LDS copy; otherwise (over 1 MB of
    // them in one launch, as in large batches, or a product with more than
    // 64 KB of them) the generating pass writes the keys and later passes
    // carry them.
    P.ck_fit = 1;
    P.ck_lds = 0;
    for (int q = 0; q < S; q++) {
        const int64_t m = P.segs[q].na + P.segs[q].nb;
        if (P.segs[q].mode != SEG_RAW) continue;
        if (m * P.ksize <= (64 << 10)) P.ck_lds = std::max<int64_t>(P.ck_lds, m);
        else P.ck_fit = 0;
    }
    if (!P.ck_fit) P.ck_lds = 0;
    P.ix = P.ck_fit && (int64_t)nck * P.ksize <= (int64_t)1 << 20;

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    P.r_stats.off = take(stats_bytes(S, nvars));
    P.r_stats.bytes = stats_bytes(S, nvars);
    P.r_flags.off = take((size_t)S * 2 * 4);
    P.r_flags.bytes = (size_t)S * 2 * 4;
    const size_t desc0 = off;
    P.o_segs = take(sizeof(DevSeg) * S);
    P.o_vars = take(sizeof(VarParam) * S * nvars);
    P.o_tile_pre = take(8 * P.tile_pre.size());
    P.o_tile_seg = take(4 * std::max<size_t>(1, P.tile_seg.size()));
    P.o_dpart_pre = take(8 * P.dpart_pre.size());
    P.o_dseg = take(4 * std::max<size_t>(1, P.dseg.size()));
    P.o_cpre = take(8 * P.cpre.size());
    P.o_iv_pre = take(8 * P.iv_pre.size());
    P.o_iv_seg = take(4 * std::max<size_t>(1, P.iv_seg.size()));
    P.o_bk_tile_pre = take(8 * std::max<size_t>(1, P.bk_tile_pre.size()));
    P.o_bk_seg = take(4 * std::max<size_t>(1, P.bk_seg.size()));
    P.o_bk_sb_pre = take(8 * std::max<size_t>(1, P.bk_sb_pre.size()));
    P.r_desc.off = desc0;
    P.r_desc.bytes = off - desc0;
    const size_t zero0 = off;
    P.o_dyn = take(sizeof(DevSegDyn) * S);
    P.o_counters = take(4 * CNT_COUNT);
    P.o_look_red = take((size_t)8 * std::max<int64_t>(1, P.nparts_bound));
    P.o_look_cmp = take((size_t)8 * std::max<int64_t>(1, P.ndparts));
    P.o_look_tile = take((size_t)8 * std::max<int64_t>(1, P.ntiles));
    P.o_box = take((size_t)8 * std::max<int64_t>(1, nbox));
    P.o_bk_hist = take((size_t)4 * std::max<int64_t>(1, P.bk_nbins));
    P.o_bk_fill = take((size_t)4 * std::max<int64_t>(1, P.bk_wi_bound));
    P.o_bk_fatfill = take(8);
    // sort blocks fill the radix passes' resident workgroups
    P.kl = P.raw && P.ix && os_keys_in_lds(P.ck_lds, P.ksize, P.vsize);
    const int64_t resident = (int64_t)cus * (P.kl ? 2 : os_resident(P.ksize, P.vsize));
    // A workgroup's pass time goes with the blocks it takes times pblk: when
    // some pblk up to PBLK_MAX makes one block per resident workgroup, take
    // the smallest; otherwise (many rounds, where the ticket queue balances
    // finer blocks better) blocks of at most 16 partitions.
    P.pblk = 0;
    for (int64_t pb = 1; pb <= PBLK_MAX && !P.pblk; pb++) {
        int64_t nb = 0;
        for (int q = 0; q < S; q++) {
            const DevSeg &d = P.segs[q];
            if (d.mode != SEG_RAW && d.mode != SEG_COMBINE) continue;
            nb += ((d.stage_bound + PART - 1) / PART + pb - 1) / pb;
        }
        if (nb <= resident) P.pblk = pb;
    }
    if (!P.pblk) P.pblk = std::max<int64_t>(1, std::min<int64_t>(16, (P.nparts_bound + resident - 1) / resident));
    // range counters of the radix passes, two sets by pass parity (zeroed here,
    // then each counting kernel clears the other set for the next pass)
    P.nrng = (P.nparts_bound / P.pblk + S + 1) / RNG + S + 1;
    P.rscan = 0;
    for (int q = 0; q < S; q++) {
        const DevSeg &d = P.segs[q];
        if (d.mode != SEG_RAW && d.mode != SEG_COMBINE) continue;
        const int64_t np = (d.stage_bound + PART - 1) / PART, nb = (np + P.pblk - 1) / P.pblk;
        if ((nb + RNG - 1) / RNG > RSUM_MAX) P.rscan = 1;
    }
    P.o_rtot = take((size_t)8 * RADIX * 2 * P.nrng);
    P.r_zero.off = zero0;
    P.r_zero.bytes = off - zero0;
    P.o_ppre = take((size_t)8 * (S + 1));
    P.o_chpre = take((size_t)8 * (S + 1));
    P.o_rpre = take((size_t)8 * (S + 1));
    P.o_pbase = take((size_t)8 * RADIX * S);
    P.o_pcnt = take((size_t)8 * std::max<int64_t>(1, P.nparts_bound));
    P.o_ctot = take((size_t)8 * RADIX * (P.nparts_bound / P.pblk + S + 1));
    P.o_iv_samp = take((size_t)P.ksize * std::max<int64_t>(1, P.iv_nsamp));
    P.o_iv_spl = take((size_t)P.ksize * std::max<int64_t>(1, P.iv_nspl));
    P.o_iv_cur = take((size_t)4 * std::max<int64_t>(1, (int64_t)P.iv_grid * P.iv_maxrows));
    P.o_iv_items = take((size_t)16 * std::max<int64_t>(1, P.iv_items));
    P.o_iv_off = take((size_t)8 * std::max<int64_t>(1, P.iv_items));
    P.o_ck = take((size_t)P.ksize * std::max<int64_t>(1, nck));
    P.o_bk_wbin = take((size_t)2 * std::max<int64_t>(1, P.bk_nbins));
    P.o_bk_sbtot = take((size_t)4 * std::max<int64_t>(1, P.bk_nsb));
    P.o_bk_sbwi = take((size_t)4 * std::max<int64_t>(1, P.bk_nsb));
    P.o_bk_sbtb = take((size_t)4 * (P.bk_nsb + 1));
    P.o_bk_sbpre = take((size_t)8 * std::max<int64_t>(1, P.bk_nsb));
    P.o_bk_wi = take(sizeof(BkWi) * std::max<int64_t>(1, P.bk_wi_bound));
    P.o_bk_stage = take((size_t)8 * std::max<int64_t>(1, P.bk_nstage));
    P.o_bk_rkey = take((size_t)4 * std::max<int64_t>(1, P.bk_nstage));
    P.o_bk_tlist = take((size_t)8 * 512 * std::max<int64_t>(1, P.bk_ntiles));  // BK_TL bins per tile
    P.o_bk_tcnt = take((size_t)4 * std::max<int64_t>(1, P.bk_ntiles));
    P.o_bk_u = take((size_t)4 * std::max<int64_t>(1, P.bk_wi_bound));
    P.o_bk_opre = take((size_t)8 * std::max<int64_t>(1, P.bk_wi_bound));
    P.o_bk_fbase = take((size_t)8 * std::max<int64_t>(1, P.bk_wi_bound));
    P.o_bk_fatc = take((size_t)8 * std::max<int64_t>(1, P.bk_fat_cap));
    const int64_t nstageA = P.nival ? 1 : nstage;
    P.o_stAk = take((size_t)P.ksize * std::max<int64_t>(1, nstageA));
    P.o_stAv = take((size_t)P.vsize * std::max<int64_t>(1, nstageA));
    P.o_stBk = take((size_t)P.ksize * std::max<int64_t>(1, nstage));
    P.o_stBv = take((size_t)(P.nival ? 8 : P.vsize) * std::max<int64_t>(1, nstage));
    P.total = off;
    return PM_OK;
}

}  // namespace pm
