// Planner for one Strassen multiply (see plan.hpp).
//
// Recursion depth k (Algorithm 2 recurses until the block size is reached; here
// the leaf size is n_pad / 2^k).  Workspace regions, in order:
//   div_a[l], div_b[l]  binary32 operand blocks written by the divide of
//                       level l: 5 per node (the other two operands are views
//                       of the parent's quadrants; 4 and three views for
//                       Winograd's variant), 7 at level 0 when the user
//                       matrix must be zero-padded on the fly and 7 at the
//                       last level of the binary32 path from depth 2 on,
//                       whose divide also forms level depth-2 (not stored);
//   leaf_a, leaf_b      16-bit paths: the split leaf operands (P planes each,
//                       B side transposed), written by the split, which forms
//                       the last divide level (the last two from depth 2 on);
//   leaf_m              the 7^k leaf products;
//   comb[l]             combine output of level 1 <= l <= depth-2 (level
//                       depth-1 is folded into the pass of level depth-2).
//                       These reuse the
//                       front of the workspace: the divide outputs are dead
//                       once the leaf products are formed, and comb[l] never
//                       overlaps comb[l+1] (read while comb[l] is written).
//   pad_a, pad_b        depth-0 binary32 only: zero-padded copies.
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>

#include "../../include/stark.h"

namespace stk {

int64_t pow7(int l) {
    int64_t p = 1;
    for (int i = 0; i < l; ++i) p *= 7;
    return p;
}

int64_t padded_size(int64_t n, int depth) {
    const int64_t q = kLeafGranule << depth;
    return (n + q - 1) / q * q;
}

int max_depth_for(int64_t n) {
    int k = 0;
    while (k < STARK_MAX_DEPTH && k < STK_MAXD - 1) {
        // depth k+1 is usable while padding adds at most a quarter to the
        // minimal padded edge and every leaf keeps at least one 64-wide tile
        const int64_t np = padded_size(n, k + 1);
        if ((np >> (k + 1)) < kLeafGranule || 4 * np > 5 * padded_size(n, 0)) break;
        ++k;
    }
    return k;
}

int tile_candidates(const Plan& p, int out[3]) {
    const int classes[3] = {64, 128, 256};
    int me = 0;
    while (classes[me] != p.tile) ++me;
    int k = 0;
    out[k++] = p.tile;
    for (int j : {me - 1, me + 1})
        if (j >= 0 && j < 3 && p.leaf % classes[j] == 0) out[k++] = classes[j];
    return k;
}

int planes_for(int precision) {
    if (precision & ~(STARK_PRECISION_MASK | STARK_WINOGRAD | STARK_FUSED | STARK_PEEL | STARK_PAD)) return -1;
    switch (precision & STARK_PRECISION_MASK) {
        case STARK_FP32: return 0;
        case STARK_BF16X3: return 2;
        case STARK_BF16X6: return 3;
        case STARK_FP16X3: return 2;
        default: return -1;
    }
}

static int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// One candidate plan: the residue `peel` peeled off (0: none), otherwise n
// zero-padded to a multiple of granule * 2^depth.  Arguments already checked.
static std::string build_plan(int64_t n, int depth, int precision, Plan& p, int tile, int peel, int64_t granule);

std::string make_plan(int64_t n, int depth, int precision, Plan& p, int tile) {
    p = Plan();
    if (n <= 0) return "n must be positive";
    if (n > (int64_t)1 << 20) return "n too large";
    if (depth < 0 || depth > max_depth_for(n)) return "depth out of range for n";
    if (planes_for(precision) < 0) return "unknown precision";
    if ((precision & STARK_PEEL) && (precision & STARK_PAD)) return "STARK_PEEL and STARK_PAD exclude each other";
    // Sizes off the grid of the leaf GEMM's tiles.  Candidates: peel the
    // residue r = n mod 64 * 2^depth (the recursion runs on the leading
    // (n - r)^2 core in place; border and fix-up are classical; r <= 64), or
    // zero-pad to a multiple of G * 2^depth for a tile edge G of 64, 128 or
    // 256 (a wider tile class needs a leaf it divides; at most a quarter more
    // edge than the 64-multiple).  Peeling reads A and B once more for the
    // border and multiplies 2 r n (2n - r) more on the vector units; padding
    // adds the padded edge's share of the recursion's work.  The candidate of
    // least modelled time is taken (STARK_PEEL: the peeled one when there is
    // one; STARK_PAD: only padded ones); a forced tile class must divide the
    // leaf of the candidate, and where none does, n is padded to a multiple
    // of the tile edge times 2^depth.
    const int64_t g = kLeafGranule << depth;
    const int64_t r = n % g;
    const bool can_peel = depth >= 1 && r >= 1 && r <= kPeelMaxResidue && n - r >= g;
    const int64_t pad_limit = (5 * padded_size(n, depth)) / 4;   // at most a quarter more edge
    std::string first_error;
    bool have = false;
    double best = 0.0;
    auto consider = [&](int peel, int64_t granule) {
        Plan c;
        const std::string e = build_plan(n, depth, precision, c, tile, peel, granule);
        if (!e.empty()) {
            if (first_error.empty()) first_error = e;
            return;
        }
        const double t = model_seconds(c);
        if (!have || t < best) {
            p = c;
            best = t;
            have = true;
        }
    };
    if (can_peel && !(precision & STARK_PAD)) consider((int)r, 0);
    if (!(can_peel && (precision & STARK_PEEL))) {
        int64_t last = -1;
        for (int64_t granule : {kLeafGranule, 2 * kLeafGranule, 4 * kLeafGranule}) {
            const int64_t q = granule << depth;
            const int64_t np = (n + q - 1) / q * q;
            if (np == last || (granule > kLeafGranule && np > pad_limit)) continue;
            last = np;
            consider(0, granule);
        }
        // a forced tile class no candidate allows: pad to its multiple even
        // beyond the quarter (batches put small problems on the class of the
        // rest)
        if (!have && tile > 0) consider(0, tile);
    }
    return have ? "" : first_error;
}

static std::string build_plan(int64_t n, int depth, int precision, Plan& p, int tile, int peel, int64_t granule) {
    p = Plan();
    const int planes = planes_for(precision);
    p.n = n;
    p.depth = depth;
    p.precision = precision;
    p.variant = (precision & STARK_WINOGRAD) ? 1 : 0;
    p.planes = planes;
    p.peel = peel;
    if (peel) {
        p.np = n - peel;
    } else {
        const int64_t q = granule << depth;
        p.np = (n + q - 1) / q * q;
    }
    p.leaf = p.np >> depth;
    // level 0 reads A, B (and writes C) element by element with bounds: the
    // user matrices of a padded size are smaller than np, and the rows of a
    // peeled one are not 16-byte aligned unless n is a multiple of 4 (then
    // the core is read and written like an unpadded matrix)
    p.padded = (p.np != n) && !(p.peel && n % 4 == 0);
    // Leaf GEMM tile class: the largest whose tiles still fill most of the
    // chip -- 256-wide tiles run one block per CU (256 CUs), 128-wide two;
    // measured, 256-wide tiles beat 128-wide ones down to about 3/4 of a
    // wave of tiles and 128-wide tiles beat 64-wide ones above about 3/4 of
    // their two waves.
    {
        const int64_t leaves = pow7(depth);
        const int64_t t256 = leaves * (p.leaf / 256) * (p.leaf / 256);
        const int64_t t128 = leaves * (p.leaf / 128) * (p.leaf / 128);
        if (p.leaf % 256 == 0 && t256 >= 192) p.tile = 256;
        else if (p.leaf % 128 == 0 && t128 >= 384) p.tile = 128;
        else p.tile = 64;
    }
    if (tile != 0) {
        if (tile != 64 && tile != 128 && tile != 256) return "tile must be 64, 128 or 256";
        if (p.leaf % tile != 0) return "tile does not divide the leaf";
        p.tile = tile;
    }
    for (int l = 0; l < STK_MAXD; ++l) {
        p.div_a[l] = p.div_b[l] = p.comb[l] = -1;
        p.div_slots[l] = 0;
    }
    const int64_t N = p.np * p.np;
    int64_t off = 0;
    if ((precision & STARK_PRECISION_MASK) == STARK_FP16X3) {
        // 2 x kScaleParts partial maxima, then e_A, e_B (kept apart from the
        // regions the combine outputs reuse)
        p.scale = off;
        off = align256(off + (2 * kScaleParts + 2) * 4);
    }
    if (depth == 0) {
        if (planes == 0) {
            if (p.padded) {
                p.pad_a = off; off = align256(off + N * 4);
                p.pad_b = off; off = align256(off + N * 4);
            }
        } else {
            p.leaf_a = off; off = align256(off + planes * N * 2);
            p.leaf_b = off; off = align256(off + planes * N * 2);
        }
        p.leaf_m = -1;   // the product goes straight to C
        p.fp32_levels = 0;
        p.bytes = (size_t)(off > 0 ? off : 256);
        return "";
    }
    // Binary32 leaves with Algorithm 1 on 256-wide tiles: the leaf GEMM forms
    // the last level's operands from the level above while it copies its
    // tiles (one add per element, as the divide would), so the divide stops
    // a level early -- unless the level above is the padded user matrix
    // (depth 1 with padding: its bounded reads cannot be direct copies).
    p.fuse = planes == 0 && p.variant == 0 && p.tile == 256 && (precision & STARK_FUSED) &&
             !(depth == 1 && p.padded);
    // binary32 levels whose operands the divide stores: every level, or all
    // but the last with fused leaves
    const int stored = p.fuse ? depth - 1 : depth;
    // 16-bit paths: the split forms the last level (from depth 2 on, the last
    // two) on the fly, so only the levels above are stored in binary32
    p.fp32_levels = planes == 0 ? stored : depth >= 2 ? depth - 2 : 0;
    for (int l = 0; l < p.fp32_levels; ++l) {
        // binary32 path from two stored levels on: level stored-2 is formed
        // on the fly by the divide of level stored-1, which then stores all
        // seven operands
        if (planes == 0 && stored >= 2 && l == stored - 2) continue;
        const bool all7 = (l == 0 && p.padded) || (planes == 0 && stored >= 2 && l == stored - 1);
        const int slots = all7 ? 7 : p.variant ? 4 : 5;
        const int64_t h = (p.np >> l) >> 1;
        const int64_t sz = (int64_t)slots * pow7(l) * h * h * 4;
        p.div_slots[l] = slots;
        p.div_a[l] = off; off = align256(off + sz);
        p.div_b[l] = off; off = align256(off + sz);
    }
    if (planes > 0) {
        const int64_t sz = pow7(depth) * planes * p.leaf * p.leaf * 2;
        p.leaf_a = off; off = align256(off + sz);
        p.leaf_b = off; off = align256(off + sz);
    }
    const int64_t dead_end = off;
    p.leaf_m = off;
    off = align256(off + pow7(depth) * p.leaf * p.leaf * 4);
    int64_t c = p.scale >= 0 ? align256(p.scale + (2 * kScaleParts + 2) * 4) : 0;
    // level depth-1 is combined together with depth-2 and never stored
    for (int l = depth - 2; l >= 1; --l) {
        const int64_t m = p.np >> l;
        p.comb[l] = c;
        c = align256(c + pow7(l) * m * m * 4);
    }
    if (c > dead_end) throw std::logic_error("combine outputs do not fit the divide region");
    p.bytes = (size_t)off;
    return "";
}

ProbDesc make_desc(const Plan& p, const float* A, const float* B, float* C, void* ws) {
    ProbDesc d{};
    d.A = A;
    d.B = B;
    d.C = C;
    d.ws = static_cast<char*>(ws);
    d.n = p.peel ? p.np : p.n;
    d.ldu = p.n;
    d.peel = p.peel;
    d.np = p.np;
    d.leaf = p.leaf;
    d.depth = p.depth;
    d.planes = p.planes;
    d.bounded0 = p.padded ? 1 : 0;
    d.gemm_tile = p.tile;
    for (int l = 0; l < STK_MAXD; ++l) {
        d.div_a[l] = p.div_a[l] >= 0 ? p.div_a[l] / 4 : -1;
        d.div_b[l] = p.div_b[l] >= 0 ? p.div_b[l] / 4 : -1;
        d.div_slots[l] = p.div_slots[l];
        d.comb[l] = p.comb[l] >= 0 ? p.comb[l] / 4 : -1;
    }
    d.leaf_a = p.leaf_a >= 0 ? p.leaf_a / 2 : -1;
    d.leaf_b = p.leaf_b >= 0 ? p.leaf_b / 2 : -1;
    d.leaf_m = p.leaf_m >= 0 ? p.leaf_m / 4 : -1;
    d.pad_a = p.pad_a >= 0 ? p.pad_a / 4 : -1;
    d.pad_b = p.pad_b >= 0 ? p.pad_b / 4 : -1;
    d.fp16 = (p.precision & STARK_PRECISION_MASK) == STARK_FP16X3 ? 1 : 0;
    d.variant = p.variant;
    d.scale = p.scale >= 0 ? p.scale / 4 : -1;
    return d;
}

Work plan_work(const Plan& p) {
    Work w{};
    const double L = (double)p.leaf, E = 4.0;
    const double leaves = (double)pow7(p.depth);
    w.leaf_flops = 2.0 * L * L * L * leaves;
    const int prods = p.planes == 0 ? 1 : p.planes == 2 ? 3 : 6;
    w.mfma_flops = w.leaf_flops * prods;
    for (int l = 0; l < p.fp32_levels; ++l) {
        if (p.div_slots[l] == 0) continue;
        const double h = (double)(p.np >> l) / 2.0;
        // per side: read the 4 quadrants of every node (a level formed from
        // the unstored level above reads each grandparent operand once
        // instead), write `slots` blocks per node
        const double reads = (l > 0 && p.div_slots[l - 1] == 0) ? (double)pow7(l - 1) * 16.0 * h * h
                                                                : (double)pow7(l) * 4.0 * h * h;
        w.divide_bytes += 2.0 * (reads + (double)pow7(l) * p.div_slots[l] * h * h) * E;
    }
    if (p.planes > 0) {
        // per side: read the source operand once (depth >= 2: the level-
        // (depth-2) operand of edge 4L; depth 1: the matrix, 4 L^2; depth 0:
        // L^2), write every leaf operand as P 16-bit planes
        const double src = p.depth >= 2 ? (double)pow7(p.depth - 2) * 16.0 : p.depth == 1 ? 4.0 : 1.0;
        w.split_bytes = 2.0 * (src * L * L * E + leaves * p.planes * L * L * 2.0);
    }
    // combine: the two deepest levels in one pass (read the 49 grandchildren,
    // write the level-(depth-2) output), the others one level at a time
    int l = p.depth - 1;
    if (p.depth >= 2) {
        w.combine_bytes += (double)pow7(p.depth - 2) * (49.0 + 16.0) * L * L * E;
        l = p.depth - 3;
    }
    for (; l >= 0; --l) {
        const double h = (double)(p.np >> l) / 2.0;
        w.combine_bytes += (double)pow7(l) * (7.0 + 4.0) * h * h * E;
    }
    if (p.pad_a >= 0) w.pad_bytes = 2.0 * ((double)p.n * p.n * E + (double)p.np * p.np * E);
    if (p.peel) {
        // border: rows np..n-1 (all n columns) and columns np..n-1 of rows
        // 0..np-1, each an inner product of length n; fix-up: r terms per
        // core output.  The border kernel reads A and B once.
        const double n = (double)p.n, nc = (double)p.np, r = (double)p.peel;
        w.peel_flops = 2.0 * n * r * (n + nc) + 2.0 * r * nc * nc;
        w.peel_bytes = 2.0 * n * n * E;
    }
    return w;
}

ModelParts model_parts(const Plan& p) {
    const Work w = plan_work(p);
    const bool split = p.planes > 0;
    // matrix-core rate of each tile class on full waves of tiles, fitted to a
    // sweep of sizes 700 .. 12288 at depths 0 .. 3 and n = 16384 at depths
    // 0 .. 4 (16-bit: 1.45 / 1.0 / 0.55 PFLOP/s, binary32: 125 / 110 / 95
    // TFLOP/s for 256 / 128 / 64-wide tiles)
    const double rate = split ? (p.tile == 256 ? 1.45e15 : p.tile == 128 ? 1.0e15 : 0.55e15)
                              : (p.tile == 256 ? 125e12 : p.tile == 128 ? 110e12 : 95e12);
    const double rows = (split && p.planes == 3 && p.tile == 256) ? 2.0 : 1.0;  // 256 x 128 tiles
    const double klen = (double)p.leaf / ((double)p.leaf + 128.0);   // per-tile start and store cost
    ModelParts m;
    m.tiles = (double)pow7(p.depth) * rows * (double)(p.leaf / p.tile) * (double)(p.leaf / p.tile);
    m.gemm_s = w.mfma_flops / (rate * klen);
    m.launches = 1 + (p.pad_a >= 0 ? 1 : 0) + (split ? 1 : 0) + (p.scale >= 0 ? 2 : 0);
    for (int l = 0; l < p.fp32_levels; ++l) m.launches += p.div_slots[l] > 0 ? 1 : 0;
    m.launches += p.depth >= 2 ? p.depth - 1 : p.depth;
    if (p.peel) m.launches += 1;
    const double bytes = w.divide_bytes + w.split_bytes + w.combine_bytes + w.pad_bytes + w.peel_bytes;
    // streaming rates of the same fit (the binary32 divide and combine run
    // near the 5 TB/s they reach alone; the split passes that write binary16
    // planes lower); peeled plans: border and fix-up products on the vector
    // units
    const double bw = split ? 3.5e12 : 5e12;
    m.stream_s = bytes / bw + w.peel_flops / kPeelRate;
    return m;
}

double wave_fill(double tiles) {
    // waves of 256 tiles: the last one partly empty (576 tiles take three)
    return tiles > 0.0 ? tiles / (256.0 * std::ceil(tiles / 256.0)) : 1.0;
}

double model_seconds(const Plan& p) {
    const ModelParts m = model_parts(p);
    return m.gemm_s / wave_fill(m.tiles) + m.stream_s + m.launches * 10e-6;
}

int model_max_depth(int64_t n, int precision) {
    // BF16X3 loses about a factor 2 of accuracy per level (16-bit split):
    // at most one level keeps it near 1e-5
    int dmax = std::min(max_depth_for(n), 3);
    if ((precision & STARK_PRECISION_MASK) == STARK_BF16X3) dmax = std::min(dmax, 1);
    return dmax;
}

int model_depth(int64_t n, int precision) {
    const int dmax = model_max_depth(n, precision);
    int best = 0;
    double best_s = 0.0;
    for (int d = 0; d <= dmax; ++d) {
        Plan p;
        if (!make_plan(n, d, precision, p).empty()) continue;
        const double s = model_seconds(p);
        if (d == 0 || s < best_s) { best = d; best_s = s; }
    }
    return best;
}

std::string plan_batch(int count, const int64_t* n, int precision, std::vector<Plan>& plans,
                       const std::vector<char>& fixed) {
    constexpr int kClasses[3] = {256, 128, 64};
    struct Cand {
        bool ok = false;
        Plan p;
        ModelParts m{};
    };
    // cand[i][c]: problem i's cheapest plan on tile class kClasses[c]
    std::vector<std::array<Cand, 3>> cand(count);
    for (int i = 0; i < count; ++i) {
        if (fixed[i]) continue;
        std::string first_error;
        bool any = false;
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d <= model_max_depth(n[i], precision); ++d) {
                Plan p;
                const std::string e = make_plan(n[i], d, precision, p, kClasses[c]);
                if (!e.empty()) {
                    if (first_error.empty()) first_error = e;
                    continue;
                }
                const ModelParts m = model_parts(p);
                Cand& k = cand[i][c];
                if (!k.ok || m.gemm_s + m.stream_s < k.m.gemm_s + k.m.stream_s) {
                    k.ok = true;
                    k.p = p;
                    k.m = m;
                }
                any = true;
            }
        if (!any) return "problem " + std::to_string(i) + ": " + first_error;
    }
    // choice[i]: class index of problem i; -1 for fixed problems
    auto cost = [&](const std::vector<int>& choice) {
        double gemm[3] = {0, 0, 0}, tiles[3] = {0, 0, 0}, stream = 0.0;
        for (int i = 0; i < count; ++i) {
            const Plan& p = choice[i] < 0 ? plans[i] : cand[i][choice[i]].p;
            const ModelParts m = choice[i] < 0 ? model_parts(p) : cand[i][choice[i]].m;
            const int c = p.tile == 256 ? 0 : p.tile == 128 ? 1 : 2;
            gemm[c] += m.gemm_s;
            tiles[c] += m.tiles;
            stream += m.stream_s;
        }
        double t = stream;
        for (int c = 0; c < 3; ++c)
            if (tiles[c] > 0.0) t += gemm[c] / wave_fill(tiles[c]) + 10e-6;
        return t;
    };
    std::vector<int> best, choice(count);
    double best_t = 0.0;
    auto consider = [&]() {
        const double t = cost(choice);
        if (best.empty() || t < best_t) {
            best = choice;
            best_t = t;
        }
    };
    for (int c = 0; c < 3; ++c) {   // one class for the whole batch
        bool ok = true;
        for (int i = 0; i < count && ok; ++i) {
            choice[i] = fixed[i] ? -1 : c;
            ok = fixed[i] || cand[i][c].ok;
        }
        if (ok) consider();
    }
    for (int i = 0; i < count; ++i) {   // every problem on its own best class
        choice[i] = -1;
        if (fixed[i]) continue;
        for (int c = 0; c < 3; ++c) {
            const Cand& k = cand[i][c];
            if (k.ok && (choice[i] < 0 || k.m.gemm_s + k.m.stream_s <
                                              cand[i][choice[i]].m.gemm_s + cand[i][choice[i]].m.stream_s))
                choice[i] = c;
        }
    }
    consider();
    for (int i = 0; i < count; ++i)
        if (best[i] >= 0) plans[i] = cand[i][best[i]].p;
    return "";
}

}  // namespace stk
