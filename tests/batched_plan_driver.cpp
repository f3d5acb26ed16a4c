// CPU check of the batched planner and workspace layouts of the host runtime.
//
// This driver includes csrc/api.cpp itself, so it exercises the very functions
// the batched entry points call (plan_for_launch, plan_batched, plan_fits,
// bat_layout, adjb_layout) without a GPU: no kernel is launched.  For every
// ensemble file given (raw int64 offsets, S + 1 values) and every combination
// of chip size, blocks per CU, block size, rows per lane and work units per
// wave, it plans as a
// launch would and then walks every unit the way the kernels address memory:
// system, row block and part in range, j range inside the system's padded
// records, part slot inside the partial region, tables inside their regions,
// and the reduction list (every row block of every split system once).
// It also checks that a plan larger than a workspace's regions is refused.
// Prints one line per ensemble and exits non-zero on the first violation.
#include "api.cpp"

#include <cstdio>
#include <fstream>

namespace {

int g_bad = 0;

#define EXPECT(cond, ...)                                                                          \
    do {                                                                                           \
        if (!(cond)) {                                                                             \
            std::fprintf(stderr, "violation: %s: ", #cond);                                       \
            std::fprintf(stderr, __VA_ARGS__);                                                     \
            std::fprintf(stderr, "\n");                                                            \
            if (++g_bad > 20) std::exit(1);                                                        \
        }                                                                                          \
    } while (0)

// Walk one plan against the regions of a layout (partial slot of `dbl` doubles per row).
void walk(const BatchPlan &p, const std::vector<int64_t> &off, int ipl, size_t rec_bytes_, size_t rec_off,
          size_t unit_off, size_t next_off, size_t red_off, size_t red_end, size_t part_off, size_t part_end,
          int64_t max_slots, int dbl, const char *what)
{
    const int64_t S = (int64_t)off.size() - 1;
    const int64_t rows = 64 * ipl;
    EXPECT(p.poff.size() == off.size() && p.systab.size() == 3 * (size_t)S, "%s: table sizes", what);
    EXPECT(rec_off + (size_t)p.npad_total * rec_bytes_ <= unit_off, "%s: records overrun", what);
    EXPECT(unit_off + p.units.size() * sizeof(int32_t) <= next_off, "%s: unit table overruns (%zu units)",
           what, p.units.size() / 4);
    EXPECT(p.n_slots * ipl <= 2 * max_slots, "%s: slots %lld x ipl %d > 2 x %lld", what,
           (long long)p.n_slots, ipl, (long long)max_slots);
    std::vector<int64_t> seen((size_t)std::max<int64_t>(p.n_slots, 1), 0);
    int64_t pairs = 0;
    for (size_t u = 0; u < p.units.size() / 4; ++u) {
        const int64_t s = p.units[4 * u], rb = p.units[4 * u + 1], part = p.units[4 * u + 2];
        EXPECT(s >= 0 && s < S, "%s: unit %zu system %lld", what, u, (long long)s);
        if (s < 0 || s >= S) continue;
        const int64_t ns = off[s + 1] - off[s], po = p.poff[s], pe = p.poff[s + 1];
        const int64_t nparts = p.systab[3 * s], plen = p.systab[3 * s + 1], slot0 = p.systab[3 * s + 2];
        EXPECT(pe - po == round_up(ns, 64), "%s: padded length of system %lld", what, (long long)s);
        EXPECT(rb >= 0 && rb * rows < ns, "%s: unit %zu row block %lld of %lld rows", what, u, (long long)rb,
               (long long)ns);
        EXPECT(part >= 0 && part < nparts, "%s: unit %zu part %lld of %lld", what, u, (long long)part,
               (long long)nparts);
        const int64_t jb = po + part * plen, je = std::min(jb + plen, pe);
        EXPECT(jb >= po && jb < je && je <= pe && pe <= p.npad_total, "%s: j range of unit %zu", what, u);
        EXPECT((jb - po) % 64 == 0 && (je - jb) % 64 == 0, "%s: j range of unit %zu not whole chunks", what, u);
        const int64_t last_row = po + std::min(ns, (rb + 1) * rows) - 1;
        EXPECT(last_row < pe, "%s: rows of unit %zu", what, u);
        pairs += (std::min(ns, (rb + 1) * rows) - rb * rows) * (je - jb);
        if (nparts > 1) {
            const int64_t slot = slot0 + rb * nparts + part;
            EXPECT(slot >= 0 && slot < p.n_slots, "%s: unit %zu slot %lld of %lld", what, u, (long long)slot,
                   (long long)p.n_slots);
            const size_t hi = part_off + ((size_t)slot * rows + rows) * dbl * sizeof(double);
            EXPECT(hi <= part_end, "%s: unit %zu slot %lld ends past the partial region", what, u,
                   (long long)slot);
            if (slot >= 0 && slot < p.n_slots) ++seen[(size_t)slot];
        }
    }
    for (int64_t k = 0; k < p.n_slots; ++k) EXPECT(seen[(size_t)k] == 1, "%s: slot %lld written %lld times",
                                                     what, (long long)k, (long long)seen[(size_t)k]);
    // the reduction list: every row block of every split system exactly once, inside its region,
    // and each row block's slots inside the slot range
    EXPECT(red_off + p.red.size() * sizeof(int32_t) <= red_end, "%s: reduction list overruns", what);
    std::vector<int64_t> want_red;
    for (int64_t s = 0; s < S; ++s)
        if (p.systab[3 * s] > 1)
            for (int64_t rb = 0; rb * rows < off[s + 1] - off[s]; ++rb) {
                want_red.push_back(s);
                want_red.push_back(rb);
            }
    EXPECT(want_red.size() == p.red.size(), "%s: reduction list has %zu entries, want %zu", what,
           p.red.size() / 2, want_red.size() / 2);
    for (size_t k = 0; k < std::min(want_red.size(), p.red.size()); ++k)
        EXPECT(want_red[k] == p.red[k], "%s: reduction list entry %zu", what, k / 2);
    for (size_t k = 0; k + 1 < p.red.size(); k += 2) {
        const int64_t s = p.red[k], rb = p.red[k + 1];
        const int64_t last = p.systab[3 * s + 2] + (rb + 1) * p.systab[3 * s] - 1;
        EXPECT(last < p.n_slots, "%s: row block (%lld, %lld) reads slot %lld of %lld", what, (long long)s,
               (long long)rb, (long long)last, (long long)p.n_slots);
    }
    int64_t want = 0;
    for (int64_t s = 0; s < S; ++s) want += (off[s + 1] - off[s]) * round_up(off[s + 1] - off[s], 64);
    EXPECT(pairs == want, "%s: units cover %lld row x record pairs, want %lld", what, (long long)pairs,
           (long long)want);
}

// The batched symmetric tiles' plan: every system's upper triangle of blocks exactly once, slot
// partials inside the system's slots and the workspace's bound, the reduction list over every
// row block of 256, records inside their region.
// a plan of the symmetric tiles against a workspace: its unit and record capacities and its
// partial region, which holds row_bytes per slot row (16 for the forward's four FP32 sums, 16 or
// 32 for the adjoint's three or six)
void walk_bsym(const BatchPlan &p, const std::vector<int64_t> &off, int64_t max_units, int64_t max_records,
               size_t part_bytes, size_t row_bytes)
{
    const int64_t S = (int64_t)off.size() - 1;
    EXPECT((int64_t)p.units.size() / 4 <= max_units, "bsym: %zu tiles > %lld", p.units.size() / 4,
           (long long)max_units);
    EXPECT(p.npad_total <= max_records, "bsym: %lld records > %lld", (long long)p.npad_total,
           (long long)max_records);
    EXPECT((size_t)p.n_slots * row_bytes <= part_bytes, "bsym: %lld slot rows exceed the partial region",
           (long long)p.n_slots);
    EXPECT((int64_t)p.red.size() / 2 <= red_capacity(off.back(), S), "bsym: reduction list overruns");
    std::vector<std::vector<char>> seen((size_t)S);
    int64_t slot_end = 0;
    for (int64_t s = 0; s < S; ++s) {
        const int64_t ns = off[s + 1] - off[s], pn = p.poff[s + 1] - p.poff[s], nb = p.systab[3 * s];
        EXPECT(pn == round_up(ns, 256) && nb * 256 == pn, "bsym: system %lld padding", (long long)s);
        EXPECT(p.systab[3 * s + 2] == slot_end, "bsym: system %lld slot base", (long long)s);
        slot_end += nb * pn;
        seen[(size_t)s].assign((size_t)(nb * nb), 0);
    }
    EXPECT(slot_end == p.n_slots, "bsym: slot count");
    bool diag_seen = false;
    for (size_t u = 0; u < p.units.size() / 4; ++u) {
        const int64_t s = p.units[4 * u], b1 = p.units[4 * u + 1], b2 = p.units[4 * u + 2];
        EXPECT(s >= 0 && s < S, "bsym: tile %zu system %lld", u, (long long)s);
        if (s < 0 || s >= S) continue;
        const int64_t nb = p.systab[3 * s], pn = p.poff[s + 1] - p.poff[s];
        EXPECT(b1 >= 0 && b1 <= b2 && b2 < nb, "bsym: tile %zu blocks (%lld, %lld) of %lld", u, (long long)b1,
               (long long)b2, (long long)nb);
        if (b1 < 0 || b1 > b2 || b2 >= nb) continue;
        EXPECT(!diag_seen || b1 == b2, "bsym: off-diagonal tile %zu after the diagonal ones", u);
        diag_seen = diag_seen || b1 == b2;
        char &c = seen[(size_t)s][(size_t)(b1 * nb + b2)];
        EXPECT(!c, "bsym: tile (%lld, %lld, %lld) twice", (long long)s, (long long)b1, (long long)b2);
        c = 1;
        // the slots this tile writes: (b2, rows of b1) and (b1, rows of b2)
        const int64_t hi = p.systab[3 * s + 2] + std::max(b1, b2) * pn + std::max(b1, b2) * 256 + 255;
        EXPECT(hi < p.n_slots, "bsym: tile %zu writes past the slot partials", u);
        EXPECT(p.poff[s] + b2 * 256 + 255 < p.npad_total, "bsym: tile %zu reads past the records", u);
    }
    for (int64_t s = 0; s < S; ++s) {
        const int64_t nb = p.systab[3 * s];
        for (int64_t b1 = 0; b1 < nb; ++b1)
            for (int64_t b2 = b1; b2 < nb; ++b2)
                EXPECT(seen[(size_t)s][(size_t)(b1 * nb + b2)], "bsym: tile (%lld, %lld, %lld) missing", (long long)s,
                       (long long)b1, (long long)b2);
    }
    size_t k = 0;
    for (int64_t s = 0; s < S; ++s)
        for (int64_t rb = 0; rb * 256 < off[s + 1] - off[s]; ++rb, k += 2)
            EXPECT(k + 1 < p.red.size() && p.red[k] == s && p.red[k + 1] == rb, "bsym: reduction list entry %zu",
                   k / 2);
    EXPECT(k == p.red.size(), "bsym: reduction list length");
}

}  // namespace

int main(int argc, char **argv)
{
    nbody_law law{};
    law.kind = NBODY_LAW_LJC_LINEAR;
    law.precision = NBODY_FP32_KAHAN;
    law.coulomb_k = 332.0637;
    law.dielectric = 4.0;
    for (int a = 1; a < argc; ++a) {
        std::ifstream f(argv[a], std::ios::binary);
        std::vector<int64_t> off;
        int64_t v;
        while (f.read(reinterpret_cast<char *>(&v), sizeof v)) off.push_back(v);
        if (off.empty() || off[0] != 0) {
            std::fprintf(stderr, "%s: bad offsets file\n", argv[a]);
            return 2;
        }
        const int64_t S = (int64_t)off.size() - 1, n = off.back();
        const BatWs lay = bat_layout(&law, n, S);
        const AdjBatWs alay = adjb_layout(&law, n, S);
        int plans = 0;
        int64_t max_units = 0, max_slots_used = 0;
        for (int cus : {80, 256, 304})
            for (int per_cu = 1; per_cu <= 16; ++per_cu)
                for (int block : {64, 128, 192, 256})
                    for (int ipl : {1, 2, 4})
                    for (int upw : {1, 8, 64}) {
                        const int64_t resident = (int64_t)cus * per_cu * (block / 64);
                        const int64_t max_red = red_capacity(n, S);
                        const PlanChoice pc = plan_for_launch(off.data(), S, ipl, resident, lay.max_slots, upw);
                        const BatchPlan &p = *pc.plan;
                        EXPECT(plan_fits(p, ipl, lay.max_units, lay.max_records, lay.max_slots, max_red),
                               "forward plan (cus %d, per_cu %d, block %d, ipl %d, upw %d)", cus, per_cu, block,
                               ipl, upw);
                        walk(p, off, ipl, rec_bytes(law.kind, law.precision), lay.rec_off, lay.unit_off,
                             lay.off_off, lay.red_off, lay.part_off, lay.part_off, lay.ticket_off, lay.max_slots, 4,
                             "forward");
                        max_units = std::max<int64_t>(max_units, (int64_t)p.units.size() / 4);
                        max_slots_used = std::max<int64_t>(max_slots_used, p.n_slots * ipl);
                        if (ipl <= 2) {       // the batched adjoint runs up to 2 rows per lane
                            const PlanChoice pa =
                                plan_for_launch(off.data(), S, ipl, resident, alay.max_slots, upw);
                            EXPECT(plan_fits(*pa.plan, ipl, alay.max_units, alay.max_records, alay.max_slots,
                                             max_red),
                                   "adjoint plan (cus %d, per_cu %d, block %d, ipl %d)", cus, per_cu, block, ipl);
                            walk(*pa.plan, off, ipl, adj_rec_bytes(law.kind, law.precision), alay.rec_off,
                                 alay.unit_off, alay.off_off, alay.red_off, alay.part_off, alay.part_off,
                                 alay.ticket_off, alay.max_slots, 8, "adjoint");
                        }
                        ++plans;
                        // a workspace whose regions are one unit / one slot too small refuses the plan
                        if (!p.units.empty())
                            EXPECT(!plan_fits(p, ipl, (int64_t)p.units.size() / 4 - 1, lay.max_records,
                                              lay.max_slots, max_red), "undersized unit table accepted");
                        if (p.n_slots > 0)
                            EXPECT(!plan_fits(p, ipl, lay.max_units, lay.max_records,
                                              (p.n_slots * ipl + 1) / 2 - 1, max_red),
                                   "undersized slot region accepted");
                        if (!p.red.empty())
                            EXPECT(!plan_fits(p, ipl, lay.max_units, lay.max_records, lay.max_slots,
                                              (int64_t)p.red.size() / 2 - 1), "undersized reduction list accepted");
                    }
        // the symmetric tiles, for the laws that have them, where every system fits
        {
            nbody_law grav{};
            grav.kind = NBODY_LAW_GRAVITY;
            grav.precision = NBODY_FP32_KAHAN;
            for (const nbody_law *lw : {(const nbody_law *)&law, (const nbody_law *)&grav}) {
                const BatWs blay = bat_layout(lw, n, S);
                const bool takes = bsym_takes(lw, off.data(), S, false);
                bool fits = true;
                for (int64_t s = 0; s < S; ++s) fits = fits && off[s + 1] - off[s] <= kBSymMaxSystem;
                EXPECT(takes == fits, "bsym_takes %d for an ensemble whose systems fit: %d", (int)takes, (int)fits);
                EXPECT(!bsym_takes(lw, off.data(), S, true), "bsym_takes with exclusion lists");
                if (takes) walk_bsym(plan_bsym(off.data(), S), off, blay.max_units, blay.max_records, blay.part_bytes, 16);
                // the batched adjoint's tiles, in the adjoint's workspace
                const AdjBatWs alay = adjb_layout(lw, n, S);
                const bool atakes = bsym_adj_takes(lw, off.data(), S, false);
                EXPECT(atakes == fits, "bsym_adj_takes %d for an ensemble whose systems fit: %d", (int)atakes, (int)fits);
                EXPECT(!bsym_adj_takes(lw, off.data(), S, true), "bsym_adj_takes with exclusion lists");
                if (atakes)
                    walk_bsym(plan_bsym(off.data(), S), off, alay.max_units, alay.max_records, alay.part_bytes,
                              (size_t)(bsym_adj_sums(lw->kind) + 3) / 4 * 16);
            }
        }
        std::printf("%s: S=%lld n=%lld plans=%d max_units=%lld/%lld max_slot_rows=%lld/%lld violations=%d\n",
                    argv[a], (long long)S, (long long)n, plans, (long long)max_units, (long long)lay.max_units,
                    (long long)max_slots_used * 64, (long long)lay.max_slots * 128, g_bad);
    }
    return g_bad ? 1 : 0;
}
