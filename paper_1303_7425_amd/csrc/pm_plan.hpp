// Host-side planning of one launch (a batch of products): per-product
// compression of the exponent keys into the degree box, the choice between
// the dense and the sparse path, tile and radix parameters, and the layout of
// the caller's workspace.  Pure host code.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "pm_internal.hpp"

namespace pm {

struct TileCfg {
    int tm, tn, hb;
};

// Tile shapes the kernels are instantiated for.  The sparse combine needs a
// table of at least twice the tile's products (so a free slot always exists);
// dense tiles may saturate their table and fall back to the box.
constexpr TileCfg TILE_CFGS[] = {{32, 64, 12}, {64, 64, 12}, {128, 128, 12}};
inline bool tile_cfg_combines(int c) { return 2 * TILE_CFGS[c].tm * TILE_CFGS[c].tn <= (1 << TILE_CFGS[c].hb); }
constexpr int N_TILE_CFGS = 3;

struct Tuning {
    int tile_cfg = -1;       // -1: choose automatically
    int combine = -1;        // sparse path: -1 auto, 0 pair-index sort, 1 LDS tile combine + sort, 2 key intervals,
                             // 3 output-key work items (one scatter, in-LDS sort per work item)
    int allow_dense = 1;     // permit the degree-box path
    int digits = -1;         // radix digit schedule: -1 auto, RADIX_DIGITS_GREEDY, RADIX_DIGITS_BALANCED
    double dense_ratio = 2;  // dense when box * dense_ratio <= na * nb
    int64_t dense_max_cells = int64_t(1) << 35;  // 256 GiB of u64 cells
};

// Autotuner cache: size class -> (tile_cfg, combine, digits).  Thread-safe.
struct TuneClass {
    int ring, dense, log2pairs;
    bool operator<(const TuneClass &o) const {
        if (ring != o.ring) return ring < o.ring;
        if (dense != o.dense) return dense < o.dense;
        return log2pairs < o.log2pairs;
    }
};
bool tune_lookup(const TuneClass &c, int &tile_cfg, int &combine, int &digits);
void tune_store(const TuneClass &c, int tile_cfg, int combine, int digits);
void tune_reset();
int tune_save(const char *path);
int tune_load(const char *path);
int log2_floor(uint64_t x);
struct Plan;
void set_digits(Plan &P, int schedule);

enum { RADIX_DIGITS_GREEDY = 0, RADIX_DIGITS_BALANCED = 1 };

struct Region {
    size_t off = 0, bytes = 0;
};

struct Plan {
    int nseg = 0, nvars = 0, bits = 0, ring = 0;
    int ksize = 4;
    int passes = 0;
    int max_bits = 0;                       // significant bits of the compressed sort keys
    unsigned char dsh[MAX_PASSES] = {}, dbits[MAX_PASSES] = {};  // digit shift and width per radix pass
    int tile_cfg = 0;
    std::vector<DevSeg> segs;
    std::vector<VarParam> vars;
    std::vector<int64_t> bound;     // result-size bound per product
    std::vector<int64_t> tile_pre, dpart_pre, cpre;
    std::vector<int32_t> tile_seg, dseg;
    int64_t ntiles = 0, ndparts = 0, nparts_bound = 0;
    int64_t pblk = 1;   // sort partitions per sort block (blocks about fill the resident grid)
    int raw = 1;        // sparse products sort (key, pair index); else (key, coefficient)
    int nival = 0;      // products on the output-key interval path
    std::vector<int64_t> iv_pre;
    std::vector<int32_t> iv_seg;
    int64_t iv_items = 0, iv_maxrows = 0, iv_nsamp = 0, iv_nspl = 0;
    int iv_grid = 1;
    int vsize = 4;      // payload bytes of a sort item
    // output-key work items (SEG_BKT)
    int nbk = 0;
    std::vector<int64_t> bk_tile_pre, bk_sb_pre;
    std::vector<int32_t> bk_seg;
    int64_t bk_ntiles = 0, bk_nsb = 0, bk_nbins = 0, bk_wi_bound = 0, bk_nstage = 0, bk_fat_cap = 0;
    size_t o_bk_hist = 0, o_bk_wbin = 0, o_bk_sbtot = 0, o_bk_sbwi = 0, o_bk_sbtb = 0, o_bk_sbpre = 0;
    size_t o_bk_tlist = 0, o_bk_tcnt = 0, o_bk_rkey = 0, o_bk_u = 0, o_bk_opre = 0, o_bk_wi = 0, o_bk_fill = 0, o_bk_fatc = 0, o_bk_fbase = 0, o_bk_fatfill = 0, o_bk_stage = 0, o_bk_tile_pre = 0, o_bk_seg = 0, o_bk_sb_pre = 0;
    int64_t nstage = 0, nbox = 0, nck = 0;
    int nsparse = 0, ndense = 0;
    // workspace layout
    Region r_stats, r_flags, r_desc, r_zero;
    size_t o_segs = 0, o_vars = 0, o_tile_pre = 0, o_tile_seg = 0, o_dpart_pre = 0, o_dseg = 0, o_cpre = 0;
    size_t o_dyn = 0, o_counters = 0, o_look_red = 0, o_look_cmp = 0, o_look_tile = 0, o_box = 0;
    size_t o_iv_samp = 0, o_iv_spl = 0, o_iv_cur = 0, o_iv_items = 0, o_iv_off = 0, o_iv_pre = 0, o_iv_seg = 0;
    size_t o_ppre = 0, o_ck = 0, o_stAk = 0, o_stAv = 0, o_stBk = 0, o_stBv = 0;
    size_t o_pcnt = 0, o_ctot = 0, o_rtot = 0, o_chpre = 0, o_rpre = 0, o_pbase = 0;
    int64_t ck_lds = 0;       // compressed operand keys a digit-count workgroup copies to LDS (entries)
    int ix = 1;               // pair-index sorts regenerate keys in every pass (else carry them)
    int ck_fit = 0;           // every pair-index product's compressed operand keys fit ck_lds
    int kl = 0;               // pair-index radix passes copy the operand keys to LDS (two workgroups per CU)
    int64_t nrng = 1;         // range rows of the radix-pass counters
    int rscan = 0;            // some product may have more than RSUM_MAX ranges
    size_t total = 0;
};

// Byte size of the statistics block written by the validation kernel.
inline size_t stats_bytes(int nseg, int nvars) { return (size_t)nseg * 2 * 2 * nvars * 8; }

struct SegInput {
    const uint64_t *fk, *fc, *gk, *gc;
    int64_t na, nb;
};

// Returns PM_OK or an error code.  `stats` holds [nseg][2 sides][min|max][nvars]
// and `flags` [nseg][2].  Output pointers of the segments are filled later.
int plan_build(int nvars, int bits, int ring, const std::vector<SegInput> &in, const uint64_t *stats,
               const uint32_t *flags, const Tuning &tune, Plan &plan, int cus = 256);

// Byte size of the region holding the statistics, for a call with nseg products.
size_t stats_region_bytes(int nseg, int nvars);

}  // namespace pm
