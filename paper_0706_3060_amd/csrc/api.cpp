// Host runtime behind the C ABI of include/nbody.h: argument validation,
// workspace carving, launch-configuration choice (heuristic, forced or
// measured), kernel sequencing on the caller's stream, error reporting and
// the measurement hooks.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <unistd.h>

#include "../../include/nbody.h"
#include "adjoint.h"
#include "jerk.h"
#include "kernels.h"
#include "noalloc.h"
#include "probe.h"

namespace {

using namespace nbk;

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(NBODY_EHIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr int64_t kMaxPartialRows = int64_t(1) << 25;   // split partial buffer budget (rows; 1 GiB at 4 columns)
constexpr int kMaxSplit = 64;
constexpr int kTargetWaves = 4096;                      // 4 resident waves per SIMD on 256 CUs
// A candidate replaces the best so far only when it is faster by more than
// this fraction: launch-to-launch noise is a few tenths of a percent, and the
// earlier candidates (the model's ranking within each staging/unroll group)
// should win a tie, so that the choice repeats from run to run.
constexpr double kTuneMargin = 0.005;

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool is_f32(int prec) { return prec != NBODY_FP64; }

size_t rec_bytes(int law, int prec)
{
    const size_t t = is_f32(prec) ? 4 : 8;
    return law == NBODY_LAW_GRAVITY ? 4 * t : 8 * t;
}

size_t adj_rec_bytes(int law, int prec)
{
    const size_t t = is_f32(prec) ? 4 : 8;
    return law == NBODY_LAW_GRAVITY ? 8 * t : 16 * t;
}

// Largest j split for `rows` output rows against `nj` j records: the split
// partials of every row must fit the partial buffer, and every split keeps at
// least one 64-record chunk.
int max_split_rows(int64_t rows, int64_t nj)
{
    const int64_t rpad = round_up(std::max<int64_t>(rows, 1), 64);
    const int64_t jpad = round_up(std::max<int64_t>(nj, 1), 64);
    const int64_t by_ws = std::max<int64_t>(1, kMaxPartialRows / rpad);
    const int64_t by_len = std::max<int64_t>(1, jpad / 64);
    return (int)std::min<int64_t>(kMaxSplit, std::min(by_ws, by_len));
}

int max_split(int64_t npad) { return npad <= 0 ? 1 : max_split_rows(npad, npad); }

// ------------------------------------------------------ symmetric tiles
// j_stage 2 selects the symmetric pair tiles (symmetric.hip): gravity (forces,
// leapfrog, the position adjoint) or the LJC laws (forces, leapfrog), FP32 pair
// arithmetic and Kahan or FP64 tile sums, whole systems.
// j_tile is the block edge in records, 1024 (16 chunks, for N up to
// kSymSmallMax) or 2048 (32 chunks); ipl picks the workgroup shape (2: 512
// threads of 2 i chunks per wave, 4: 256 threads of 4).  Each row gets one FP32
// partial per block, so the partial buffer is npad^2 / (64 blk) x 16 bytes
// (8 GiB at N = 2^20); above kSymMaxN (32 GiB of partials) the one-sided
// kernels, whose partials are O(N), take over.
constexpr int kBatchUnitsPerWave = 8;    // the rule's work units per resident wave (batched j_split)
constexpr int kBSymWaves = 4;            // waves (one tile each) per workgroup of the batched symmetric tiles
constexpr int kSymStage = 2;
constexpr int64_t kSymSmallMax = int64_t(1) << 18;
constexpr int64_t kSymMinN = int64_t(1) << 15;       // the rule's threshold for whole systems
constexpr int64_t kSymSplit4Below = int64_t(1) << 16; // four j parts below this size
constexpr int64_t kSymMaxN = int64_t(1) << 21;
// j parts per tile above 1 (j_split 2 or 4 with j_stage 2) for systems up to this size, where a
// whole-tile launch fills the chip only a few rounds deep
constexpr int64_t kSymSplitMaxN = int64_t(1) << 17;

// The acceleration-and-jerk tiles (symjerk.hip, j_stage 2 of the jerk entry point): gravity
// with FP32 pair arithmetic, whole systems of up to kSymJerkMaxN particles, one workgroup shape
// (8 waves of 2 i chunks, blocks of 1024 records) and 1 or 2 j parts; each row gets one FP32
// partial of 32 bytes per block and part (8 GiB at kSymJerkMaxN).
constexpr int64_t kSymJerkMaxN = int64_t(1) << 19;
bool symjerk_ok(int law, int prec)
{
    return law == NBODY_LAW_GRAVITY && (prec == NBODY_FP32_KAHAN || prec == NBODY_FP32_FP64ACC);
}
int64_t symjerk_npad(int64_t n) { return round_up(std::max<int64_t>(n, 1), (int64_t)kSymJerkBlk * 64); }
int symjerk_max_split(int64_t n) { return n <= kSymSplitMaxN ? 2 : 1; }
size_t symjerk_partial_bytes(int64_t n, int split)
{
    const int64_t np = symjerk_npad(n);
    return (size_t)split * (size_t)(np / ((int64_t)kSymJerkBlk * 64)) * (size_t)np * 8 * sizeof(float);
}

// LJC(linear)'s single-system adjoint over unordered pairs: the batched adjoint's tiles
// (bsym_adj.hip, one wave per tile of two 256-record blocks) over one whole system, FP32 pair
// arithmetic, up to kSymAdjLjcMaxN atoms (32 bytes of slot partials per atom and block: 8 GiB
// at 2^18).  The rule takes them from kSymAdjLjcMinN atoms: measured per call 1.03-1.08x the
// one-sided adjoint at 16,384 atoms, 1.3x at 24,576, and per kernel 1.37x at 32,768, 1.43x at
// 65,536 and 1.53x at 131,072 (at 8,192 the 528 tiles leave most of the chip idle and the
// one-sided kernel is faster).
constexpr int64_t kSymAdjLjcMinN = int64_t(1) << 14;
constexpr int64_t kSymAdjLjcMaxN = int64_t(1) << 18;
bool symadj_ljc_ok(int law, int prec)
{
    return law == NBODY_LAW_LJC_LINEAR && (prec == NBODY_FP32_KAHAN || prec == NBODY_FP32_FP64ACC);
}
size_t symadj_ljc_partial_bytes(int64_t n)
{
    const int64_t np = round_up(std::max<int64_t>(n, 1), kBSymRecords);
    return (size_t)(np / kBSymRecords) * (size_t)np * 8 * sizeof(float);
}

bool sym_eligible(int api, int law, int prec)
{
    if (prec != NBODY_FP32_KAHAN && prec != NBODY_FP32_FP64ACC) return false;
    const bool fwd = api == NBODY_API_FORCES || api == NBODY_API_LEAPFROG;
    if (law == NBODY_LAW_GRAVITY) return fwd || api == NBODY_API_BACKWARD;
    return fwd;                                         // the three LJC dielectrics
}

// the symmetric tiles' pair operator of a forward law
int sym_op_of(int law)
{
    switch (law) {
    case NBODY_LAW_GRAVITY: return SYM_FORCE;
    case NBODY_LAW_LJC_LINEAR: return SYM_LJC;
    case NBODY_LAW_LJC_CONSTANT: return SYM_LJC_CONST;
    default: return SYM_LJC_SIG;
    }
}

// block edge in chunks for a requested j_tile and system size
int sym_blk(int j_tile, int64_t n) { return (j_tile <= 1024 && n <= kSymSmallMax) ? 16 : 32; }
int64_t sym_npad(int64_t n, int blk) { return round_up(std::max<int64_t>(n, 1), (int64_t)blk * 64); }
size_t sym_partial_bytes(int64_t n, int blk, int split = 1)
{
    const int64_t np = sym_npad(n, blk);
    return (size_t)split * (size_t)(np / ((int64_t)blk * 64)) * (size_t)np * 4 * sizeof(float);
}
// the largest j-part count allowed for n rows, blocks of blk chunks and `waves` waves per
// workgroup (every part needs at least as many chunks as the workgroup has waves)
int sym_max_split(int64_t n, int blk, int waves)
{
    if (n > kSymSplitMaxN) return 1;
    int s = 4;
    while (s > 1 && blk / s < waves) s /= 2;
    return s;
}
// the largest partial buffer any allowed block edge and j-part count needs for n rows
size_t sym_max_partial_bytes(int64_t n)
{
    size_t b = sym_partial_bytes(n, 32, sym_max_split(n, 32, 4));
    if (n <= kSymSmallMax) b = std::max(b, sym_partial_bytes(n, 16, sym_max_split(n, 16, 4)));
    return b;
}

int validate_law(const nbody_law *law, bool backward)
{
    if (!law) return fail(NBODY_EINVAL, "law is NULL");
    if (law->kind < NBODY_LAW_GRAVITY || law->kind > NBODY_LAW_LJC_SIGMOIDAL)
        return fail(NBODY_EINVAL, "unknown law kind %d", law->kind);
    if (law->precision < NBODY_FP64 || law->precision > NBODY_FP32_PLAIN)
        return fail(NBODY_EINVAL, "unknown precision %d", law->precision);
    if (law->kind == NBODY_LAW_GRAVITY) {
        if (!(law->softening >= 0.0) || !std::isfinite(law->softening))
            return fail(NBODY_EINVAL, "softening must be finite and >= 0 (got %g)", law->softening);
        if (!std::isfinite(law->G)) return fail(NBODY_EINVAL, "G must be finite");
    } else {
        if (law->kind != NBODY_LAW_LJC_SIGMOIDAL &&
            (!(law->dielectric > 0.0) || !std::isfinite(law->dielectric)))
            return fail(NBODY_EINVAL, "dielectric D must be finite and > 0 (got %g)", law->dielectric);
        if (!std::isfinite(law->coulomb_k) || law->coulomb_k < 0.0)
            return fail(NBODY_EINVAL, "coulomb_k must be finite and >= 0");
        if (law->kind == NBODY_LAW_LJC_SIGMOIDAL)
            for (int c = 0; c < 4; ++c)
                if (!std::isfinite(law->zeta[c])) return fail(NBODY_EINVAL, "zeta coefficients must be finite");
        if (law->kind >= NBODY_LAW_LJC_CONSTANT && law->precision == NBODY_FP32_PLAIN)
            return fail(NBODY_ENOTSUP, "FP32_PLAIN is provided for gravity and LJC(linear) only");
    }
    if (backward && law->precision == NBODY_FP32_PLAIN)
        return fail(NBODY_ENOTSUP, "the adjoint is provided for FP64, FP32_FP64ACC and FP32_KAHAN");
    if (backward && law->kind > NBODY_LAW_LJC_LINEAR)
        return fail(NBODY_ENOTSUP, "the adjoint is provided for gravity and LJC(linear)");
    return NBODY_OK;
}

// ------------------------------------------------------------ configuration
struct Cfg {
    int block = 256, ipl = 1, j_tile = 256, j_split = 1, j_stage = 0;
};

std::mutex g_mu;
constexpr int kNumApi = 7;
bool g_override_set[kNumApi] = {false, false, false, false, false, false, false};
Cfg g_override[kNumApi];

using TuneKey = std::tuple<int, int, int, int, int, int>;   // api, law, prec, pot, nbucket, sbucket
std::map<TuneKey, std::pair<Cfg, double>> g_tuned;
uint64_t g_cfg_version = 0;   // bumped (under g_mu) whenever an override or a tuned entry changes

int size_bucket(int64_t n)
{
    int b = 0;
    while ((int64_t(1) << b) < n && b < 62) ++b;
    return b;
}

int max_ipl(int api, int prec)
{
    if (api == NBODY_API_BATCHED || api == NBODY_API_BACKWARD) return 4;
    return is_f32(prec) ? 8 : 4;
}

bool ipl_ok(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }

Cfg sanitize(Cfg c, int api, int law, int prec, int64_t npad)
{
    if (c.j_stage == kSymStage && ((api == NBODY_API_BATCHED && bsym_supported(law, prec)) ||
                                   (api == NBODY_API_BACKWARD_BATCHED && bsym_adj_supported(law, prec)))) {
        c.block = kBSymWaves * 64;                    // the batched symmetric tiles' fixed shape
        c.ipl = kBSymRecords / 64;
        c.j_tile = kBSymRecords;
        c.j_split = 1;
        return c;
    }
    if (c.j_stage == kSymStage) {
        if (api == NBODY_API_BACKWARD && symadj_ljc_ok(law, prec) && npad <= kSymAdjLjcMaxN) {
            c.block = kBSymWaves * 64;                  // the batched adjoint tiles' fixed shape
            c.ipl = kBSymRecords / 64;
            c.j_tile = kBSymRecords;
            c.j_split = 1;
            return c;
        }
        if (api == NBODY_API_JERK && symjerk_ok(law, prec) && npad <= kSymJerkMaxN) {
            c.block = kSymThreads;                      // the jerk tiles' one shape
            c.ipl = 2;
            c.j_tile = kSymJerkBlk * 64;
            c.j_split = c.j_split >= 2 ? symjerk_max_split(npad) : 1;
            return c;
        }
        if (sym_eligible(api, law, prec) && npad <= kSymMaxN) {
            // two workgroup shapes: 8 waves of 2 i chunks, or 4 waves of 4 i chunks
            const bool four = c.ipl >= 4 && c.block <= 256;
            c.block = four ? 256 : kSymThreads;
            c.ipl = four ? 4 : 2;
            c.j_tile = sym_blk(c.j_tile, npad) * 64;
            // j parts per tile: 1, 2 or 4, as many as requested and allowed
            const int smax = sym_max_split(npad, c.j_tile / 64, c.block / 64);
            int sp = 1;
            while (sp * 2 <= std::min(c.j_split, smax)) sp *= 2;
            c.j_split = sp;
            return c;
        }
        c.j_stage = 1;                                  // other laws, precisions, entry points, sizes
    }
    c.j_stage = std::max(0, std::min(c.j_stage, 1));
    // the one-sided, batched, adjoint and jerk kernels are built for up to 256 threads
    c.block = std::max(64, std::min(c.block, 256)) / 64 * 64;
    c.ipl = std::min(c.ipl, max_ipl(api, prec));
    if (law >= NBODY_LAW_LJC_CONSTANT) c.ipl = std::min(c.ipl, 2);
    if (api == NBODY_API_JERK || api == NBODY_API_HERMITE) c.ipl = std::min(c.ipl, 2);
    if (c.j_stage == 1) c.ipl = std::min(c.ipl, 4);    // LDS staging: up to 4 rows per lane
    if (api == NBODY_API_BATCHED || api == NBODY_API_BACKWARD_BATCHED)
        c.j_split = std::max(1, std::min(c.j_split, 64));      // work units per resident wave
    else
        c.j_split = std::max(1, std::min(c.j_split, max_split(npad)));
    if (api == NBODY_API_BACKWARD_BATCHED) c.ipl = std::min(c.ipl, 2);
    return c;
}

int device_cus();

// Resident waves of the all-pairs kernel for this configuration (whole chip).
// The occupancy query is a runtime call of a few microseconds; its answer
// depends only on the kernel and the block size, so it is asked once.
int64_t resident_waves(int law, int prec, int ipl, bool pot, int js, int block)
{
    using Key = std::tuple<int, int, int, int, int, int>;
    static std::map<Key, int64_t> cache;
    static std::mutex mu;
    const Key key(law, prec, ipl, pot ? 1 : 0, js, block);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int bpc = forces_blocks_per_cu(law, prec, ipl, pot ? 1 : 0, js, block);
    const int64_t r = bpc > 0 ? (int64_t)bpc * (block / 64) * device_cus() : 0;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = r;
    return r;
}

// Resident workgroups per CU of the batched forward and adjoint kernels (asked once per variant).
int batched_blocks_per_cu_cached(int law, int prec, int ipl, bool pot, int js, int block, bool excl)
{
    using Key = std::tuple<int, int, int, int, int, int, int>;
    static std::map<Key, int> cache;
    static std::mutex mu;
    const Key key(law, prec, ipl, pot ? 1 : 0, js, block, excl ? 1 : 0);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int r = batched_max_blocks_per_cu(law, prec, ipl, pot ? 1 : 0, js, block, excl ? 1 : 0);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = r;
    return r;
}

// Modelled time of one evaluation of `rows` rows against `nj` j records with
// a j split of s (seconds, up to a common scale): waves run in rounds of
// `resident` concurrent waves, each doing 1/s of the j range, plus the
// fixed-order reduction of the split partials.
double split_cost(int64_t rows, int64_t nj, int64_t waves, int64_t resident, int s,
                  double pairs_per_s)
{
    const double w = (double)waves * s;
    const double R = (double)std::max<int64_t>(resident, 1);
    const double fill = w >= R ? std::ceil(w / R) * R / w : R / w;
    const double t_compute = (double)rows * (double)nj / pairs_per_s * fill;
    const double t_reduce = s > 1 ? 5e-6 + (double)rows * s * 32.0 / 4e11 : 0.0;
    return t_compute + t_reduce;
}

// as resident_waves, for the acceleration-and-jerk kernel
int64_t resident_waves_jerk(int prec, int ipl, bool pot, int js, int block)
{
    using Key = std::tuple<int, int, int, int, int>;
    static std::map<Key, int64_t> cache;
    static std::mutex mu;
    const Key key(prec, ipl, pot ? 1 : 0, js, block);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int bpc = jerk_blocks_per_cu(prec, ipl, pot ? 1 : 0, js, block);
    const int64_t r = bpc > 0 ? (int64_t)bpc * (block / 64) * device_cus() : 0;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = r;
    return r;
}

double nominal_rate(int law, int prec)
{
    const bool f32 = is_f32(prec);
    if (law == NBODY_LAW_GRAVITY) return f32 ? 3.3e12 : 1.4e12;
    if (law == NBODY_LAW_LJC_SIGMOIDAL) return f32 ? 1.2e12 : 0.4e12;
    return f32 ? 1.8e12 : 0.6e12;
}

// splits 1..smax ordered by modelled cost for `rows` output rows against `nj`
// records (jerk: the acceleration-and-jerk kernel, about twice the flops)
std::vector<int> ranked_splits(int law, int prec, int64_t rows, int64_t nj, int ipl, bool pot, int js,
                               int block, int smax, bool jerk = false)
{
    const int64_t waves = (rows + 64 * ipl - 1) / (64 * ipl);
    const int64_t R = jerk ? resident_waves_jerk(prec, ipl, pot, js, block)
                           : resident_waves(law, prec, ipl, pot, js, block);
    std::vector<std::pair<double, int>> c;
    for (int sp = 1; sp <= smax; ++sp) {
        double cost;
        if (R > 0) {
            cost = split_cost(rows, nj, waves, R, sp, nominal_rate(law, prec) * (jerk ? 0.5 : 1.0));
        } else {   // occupancy unknown: aim at kTargetWaves waves
            cost = std::abs(std::log((double)(waves * sp) / kTargetWaves)) + 0.01 * sp;
        }
        c.push_back({cost, sp});
    }
    std::stable_sort(c.begin(), c.end());
    std::vector<int> out;
    for (auto &e : c) out.push_back(e.second);
    return out;
}

// n output rows against nj j records (nj = n for a whole system)
Cfg heuristic(int api, int law, int prec, int64_t n, int64_t nj, int64_t S, bool pot, bool allow_sym = true)
{
    Cfg c;
    if (allow_sym && sym_eligible(api, law, prec) && n == nj && n >= kSymMinN && n <= kSymMaxN) {
        c.j_stage = kSymStage;
        c.j_tile = n <= kSymSmallMax ? 1024 : 2048;
        // 4 waves of 4 i chunks (half the cross-lane moves per pair, 4 waves per SIMD) against
        // 8 waves of 2 (6 waves per SIMD): for gravity measured 5-7 % faster with the
        // potential, and from N = 2^17 without it.  For LJC(linear) and LJC(constant) the
        // 8-wave shape is as fast or up to 5 % faster with the energies, the 4-wave one 15-20 %
        // faster without them; the sigmoidal dielectric's longer sequence leaves the 4-wave
        // shape three waves per SIMD, and 8 waves of 2 are 10 % faster either way.
        // (the adjoint has no potential, whatever the caller's flag says)
        const bool with_pot = pot && api != NBODY_API_BACKWARD;
        const bool four = law == NBODY_LAW_GRAVITY ? (with_pot || n > (int64_t(1) << 17))
                                                   : (!with_pot && law != NBODY_LAW_LJC_SIGMOIDAL);
        c.ipl = four ? 4 : 2;
        c.block = four ? 256 : kSymThreads;
        // up to 2^17 the 2,080 to 8,256 tiles fill the chip only 2 to 8 rounds deep, and the
        // last round is partly empty: two j parts per tile (one workgroup each) halve the
        // rounds' length, measured 4-10 % faster per call (kernel and slot reduction) at
        // N = 65,536 to 131,072; four parts shorten the kernel further but double the
        // reduction's reads again.  Below 65,536 (from 32,768) the 528 to 2,080 tiles fill the
        // chip less than two rounds deep: four parts (the 8-wave shape takes two), measured at
        // 32,768 and 49,152 particles 1.24-1.34x the one-sided kernel per call for gravity's
        // forces, 1.32-1.40x for LJC(linear)'s with the energies and 1.37-1.45x for gravity's
        // adjoint (at 16,384 the one-sided kernels are as fast or faster)
        c.j_split = n < kSymSplit4Below ? 4 : (n <= kSymSplitMaxN ? 2 : 1);
        return sanitize(c, api, law, prec, round_up(n, 64));
    }
    const int64_t npad = round_up(std::max<int64_t>(std::max(n, nj), 1), 64);
    const int smax = max_split_rows(n, nj);
    if (api == NBODY_API_BATCHED || api == NBODY_API_BACKWARD_BATCHED) {
        c.ipl = 1;
        c.block = 256;
        c.j_tile = 256;
        c.j_split = kBatchUnitsPerWave;
        c.j_stage = is_f32(prec) ? 1 : 0;
        // the symmetric tiles for systems of 512 particles on average and more (smaller ones
        // lose too much to the padding of 256-record blocks and the diagonal tiles; a launch
        // with a system above 8192 particles runs one-sided all the same)
        // (the batched adjoint's tiles: 1.77 against 2.42-2.47 ms for the 256-system LJC ensemble)
        const bool tiles = api == NBODY_API_BATCHED ? bsym_supported(law, prec) : bsym_adj_supported(law, prec);
        if (allow_sym && tiles && n >= 512 * std::max<int64_t>(S, 1)) {
            c.j_stage = kSymStage;
            return sanitize(c, api, law, prec, 64);
        }
        return c;
    }
    if (is_f32(prec)) {
        c.ipl = 1;
        c.j_tile = 256;
        c.j_stage = 1;
    } else {
        c.ipl = n >= (1 << 18) ? 2 : 1;
        c.j_tile = 1024;
        c.j_stage = 0;
    }
    if (api == NBODY_API_HERMITE) {
        // the block steps' kernel shape: the precision's default staging (LDS for
        // FP32, which keeps the short j ranges of small due sets fast); the split
        // follows the due count (hermite_split_table)
        c.ipl = 1;
        c.j_split = ranked_splits(law, prec, n, nj, c.ipl, pot, c.j_stage, c.block, smax, true)[0];
        return sanitize(c, api, law, prec, npad);
    }
    if (api == NBODY_API_JERK && allow_sym && symjerk_ok(law, prec) && n == nj && n >= kSymMinN &&
        n <= kSymJerkMaxN) {
        // whole systems from 32,768 particles: the symmetric tiles, in two j parts up to 2^17
        // (the tiles fill the chip only a few rounds deep there); measured 1.19x the one-sided
        // kernel per call at 32,768, 1.27x at 49,152 (at 16,384 the one-sided kernel is faster)
        c.j_stage = kSymStage;
        c.j_split = 2;
        return sanitize(c, api, law, prec, npad);
    }
    if (api == NBODY_API_JERK) {
        // Measured on gfx950: the jerk kernel runs 6-9 % faster with scalar staging of
        // its 32-byte records than through LDS (N = 65,536), and best with 24 parts
        // or more (N = 65,536: 24 parts 2 % ahead of 32; N = 262,144: 24 and 32
        // within 0.4 %, 4 % ahead of 8), up to 32 where that keeps 24k waves.
        c.ipl = 1;
        c.j_stage = 0;
        c.j_tile = is_f32(prec) ? 256 : 1024;
        const int64_t waves = (n + 63) / 64;
        const int64_t want = std::min<int64_t>(32, std::max<int64_t>(24, (24576 + waves - 1) / waves));
        c.j_split = (int)std::max<int64_t>(1, std::min<int64_t>(want, smax));
        return sanitize(c, api, law, prec, npad);
    }
    if (api == NBODY_API_BACKWARD && allow_sym && symadj_ljc_ok(law, prec) && n == nj && n >= kSymAdjLjcMinN &&
        n <= kSymAdjLjcMaxN) {
        c.j_stage = kSymStage;
        return sanitize(c, api, law, prec, npad);
    }
    if (api == NBODY_API_BACKWARD) {
        c.ipl = std::min(c.ipl, 2);
        c.j_stage = is_f32(prec) ? 1 : 0;
        // at least kTargetWaves waves, and up to 8 j parts while that keeps the
        // waves under 32768: the adjoint kernels gain from several waves per
        // SIMD to switch between (measured at N = 262,144: split 1 41.5 ms,
        // 2 38.4, 4 36.8, 8 35.6)
        const int64_t waves = (n + 64 * c.ipl - 1) / (64 * c.ipl);
        const int64_t target = std::max<int64_t>(kTargetWaves, std::min<int64_t>(32768, waves * 8));
        int split = 1;
        while (split < kMaxSplit && waves * split < target) split *= 2;
        c.j_split = split;
        return sanitize(c, api, law, prec, npad);
    }
    if (is_f32(prec)) {
        // Measured on gfx950 (gravity, FP32 + Kahan, one row per lane, LDS staging): 32
        // parts is the best split from N = 16,384 to 2^20 (ahead of 8 parts by 6 % at
        // N = 131,072, 3 % at 262,144, 1.5 % at 524,288 and 0.7 % at 2^20; 24 to 64
        // within 1 % of each other at N = 65,536); the round-quantisation model alone
        // stops at 5 and loses up to a fifth at N = 65,536.
        c.j_split = (int)std::max<int64_t>(1, std::min<int64_t>(32, smax));
        return sanitize(c, api, law, prec, npad);
    }
    c.j_split = ranked_splits(law, prec, n, nj, c.ipl, pot, c.j_stage, c.block, smax)[0];
    return sanitize(c, api, law, prec, npad);
}

bool is_batched_api(int api) { return api == NBODY_API_BATCHED || api == NBODY_API_BACKWARD_BATCHED; }

// Second component of a tuning key: the system count for the batched entry
// points, the j-record count otherwise (so that a row subset of a large system
// is not served the configuration tuned for a whole system of that row count).
int tune_sbucket(int api, int64_t S, int64_t nj) { return size_bucket(is_batched_api(api) ? S : nj); }

// NBODY_TUNE_CACHE names a tuning file shared between processes: it is read at
// the first configuration lookup of the process (when it exists) and written
// again after every autotuning run.  A file tuned on another device is not
// used (one stderr line says why) and is replaced by the next run's results.
const char *tune_cache_path()
{
    const char *p = getenv("NBODY_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

void tune_cache_load_once()
{
    static std::once_flag once;
    std::call_once(once, [] {
        const char *p = tune_cache_path();
        if (!p) return;
        FILE *f = fopen(p, "r");
        if (!f) return;  // nothing tuned yet
        fclose(f);
        if (nbody_tune_load(p) != NBODY_OK)
            fprintf(stderr, "nbody: tuning cache %s not used: %s\n", p, nbody_last_error());
    });
}

void tune_cache_store()
{
    const char *p = tune_cache_path();
    if (p && nbody_tune_save(p) != NBODY_OK)
        fprintf(stderr, "nbody: tuning cache %s not written: %s\n", p, nbody_last_error());
}

// The configuration for n output rows in S systems; nj j records (0: nj = n).
Cfg choose(int api, const nbody_law *law, int64_t n, int64_t S, bool pot, int64_t nj = 0)
{
    tune_cache_load_once();
    if (nj <= 0) nj = n;
    const int64_t npad = round_up(std::max<int64_t>(std::max(n, nj), 1), 64);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_override_set[api]) return sanitize(g_override[api], api, law->kind, law->precision, npad);
    const int sb = tune_sbucket(api, S, nj);
    auto it = g_tuned.find(TuneKey(api, law->kind, law->precision, pot ? 1 : 0, size_bucket(n), sb));
    if (it == g_tuned.end() && (api == NBODY_API_LEAPFROG || api == NBODY_API_HERMITE))
        // a leapfrog step runs the forces kernel, a Hermite step the jerk kernel
        it = g_tuned.find(TuneKey(api == NBODY_API_LEAPFROG ? NBODY_API_FORCES : NBODY_API_JERK,
                                  law->kind, law->precision, pot ? 1 : 0, size_bucket(n), sb));
    // (the jerk's symmetric tiles evaluate whole systems: not a shape for the block steps, which
    // a shared Hermite step takes from the jerk's own configuration)
    if (it != g_tuned.end() && api == NBODY_API_HERMITE && it->second.first.j_stage == kSymStage)
        it = g_tuned.end();
    if (it != g_tuned.end()) return sanitize(it->second.first, api, law->kind, law->precision, npad);
    return heuristic(api, law->kind, law->precision, n, nj, S, pot);
}

// c, or the rule's one-sided configuration when c selects the symmetric tiles
// (which evaluate whole systems only: not row subsets or exclusion lists)
Cfg one_sided(const Cfg &c, int api, const nbody_law *law, int64_t n, int64_t nj, bool pot)
{
    if (c.j_stage != kSymStage) return c;
    return heuristic(api, law->kind, law->precision, n, nj, 1, pot, false);
}

// ------------------------------------------------------------ measurement
bool g_timing = false;
struct TimedLaunch {
    hipEvent_t a, b;
};
std::vector<TimedLaunch> g_timed;
double g_timed_ms = 0.0;
int64_t g_timed_count = 0;

struct Timer {
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    explicit Timer(hipStream_t st, bool allowed = true) : s(st)
    {
        {
            std::lock_guard<std::mutex> lk(g_mu);
            on = allowed && g_timing;
        }
        if (on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
        else
            on = false;
    }
    void stop()
    {
        if (!on) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_mu);
        g_timed.push_back({a, b});
        on = false;
    }
};

// ------------------------------------------------------------ workspace
struct FwdWs {
    size_t rec_off, part_off, scratch_off, total;
};

FwdWs fwd_layout(int api, const nbody_law *law, int64_t n)
{
    FwdWs w{};
    const int64_t npad = round_up(std::max<int64_t>(n, 1), 64);
    const bool sym = sym_eligible(api, law->kind, law->precision) && n <= kSymMaxN;
    // the symmetric tiles pad the records to whole blocks and keep one FP32 partial per
    // row and block; the one-sided split keeps [split][rows][4] FP64 partials
    const int64_t nrec = sym ? sym_npad(n, 32) : npad;
    size_t part = (size_t)max_split(npad) * (size_t)npad * 4 * sizeof(double);
    if (sym) part = std::max(part, sym_max_partial_bytes(n));
    size_t off = 0;
    w.rec_off = off;
    off = align256(off + (size_t)nrec * rec_bytes(law->kind, law->precision));
    w.part_off = off;
    off = align256(off + part);
    w.scratch_off = off;
    if (api == NBODY_API_LEAPFROG) off = align256(off + (size_t)npad * 3 * sizeof(double));
    w.total = off;
    return w;
}

struct AdjWs {
    size_t rec_off, part_off, type_off, total;
};

// Partials of the per-type gradient sums (blocks x types x 2 doubles).
constexpr int64_t kTypePartDoubles = 32768;

AdjWs adj_layout(const nbody_law *law, int64_t n)
{
    AdjWs w{};
    const int64_t npad = round_up(std::max<int64_t>(n, 1), 64);
    // the gravity position adjoint may run as symmetric pair tiles: records padded to whole
    // blocks and one FP32 partial per row and block, as the forward's
    const bool sym = sym_eligible(NBODY_API_BACKWARD, law->kind, law->precision) && n <= kSymMaxN;
    // LJC(linear)'s: records padded to whole 256-record blocks, 32 bytes per row and block
    const bool ljs = symadj_ljc_ok(law->kind, law->precision) && n <= kSymAdjLjcMaxN;
    int64_t nrec = sym ? sym_npad(n, 32) : npad;
    if (ljs) nrec = std::max(nrec, round_up(std::max<int64_t>(n, 1), kBSymRecords));
    size_t part = (size_t)max_split(npad) * (size_t)npad * 8 * sizeof(double);
    if (sym) part = std::max(part, sym_max_partial_bytes(n));
    if (ljs) part = std::max(part, symadj_ljc_partial_bytes(n));
    size_t off = 0;
    w.rec_off = off;
    off = align256(off + (size_t)nrec * adj_rec_bytes(law->kind, law->precision));
    w.part_off = off;
    off = align256(off + part);
    w.type_off = off;
    off = align256(off + (size_t)kTypePartDoubles * sizeof(double));
    w.total = off;
    return w;
}

// Acceleration + jerk (and the Hermite integrator): records, split partials
// and, for the integrator, the new acceleration / jerk of the evaluated rows,
// the due list and the scheduling scratch.
constexpr int kSchedBlocks = 1024;
constexpr int64_t kBlockLog = 1024;   // block steps enqueued between two host read-backs, at most

struct JerkWs {
    size_t rec_off, part_off, a1_off, j1_off, list_off, pmin_off, pcnt_off, out_off, log_off, table_off, total;
};

JerkWs jerk_layout(int api, const nbody_law *law, int64_t n)
{
    JerkWs w{};
    const int64_t npad = round_up(std::max<int64_t>(n, 1), 64);
    const size_t t = is_f32(law->precision) ? 4 : 8;
    // the symmetric tiles' records (padded to whole blocks) and slot partials, for the sizes
    // they take
    const bool sym = symjerk_ok(law->kind, law->precision) && n <= kSymJerkMaxN;
    const int64_t nrec = sym ? std::max(npad, symjerk_npad(n)) : npad;
    size_t part = (size_t)max_split(npad) * (size_t)npad * 8 * sizeof(double);
    if (sym) part = std::max(part, symjerk_partial_bytes(n, symjerk_max_split(n)));
    size_t off = 0;
    w.rec_off = off;
    off = align256(off + (size_t)nrec * 8 * t);
    w.part_off = off;
    off = align256(off + part);
    if (api == NBODY_API_HERMITE) {
        w.a1_off = off;
        off = align256(off + (size_t)npad * 3 * sizeof(double));
        w.j1_off = off;
        off = align256(off + (size_t)npad * 3 * sizeof(double));
        w.list_off = off;
        off = align256(off + (size_t)npad * sizeof(int64_t));
        w.pmin_off = off;
        off = align256(off + (size_t)kSchedBlocks * sizeof(double));
        w.pcnt_off = off;
        off = align256(off + (size_t)kSchedBlocks * sizeof(int64_t));
        w.out_off = off;
        off = align256(off + sizeof(BlockState));
        w.log_off = off;
        off = align256(off + (size_t)kBlockLog * (sizeof(int64_t) + sizeof(double)));
        w.table_off = off;
        off = align256(off + (size_t)(npad / 64) * sizeof(int));
    }
    w.total = off;
    return w;
}

// Partial slots of the batched forward's j parts: a slot holds the part sums
// of one row block (64 x ipl rows, 4 doubles each); the buffer is sized for
// kMaxBatchSlots slots of 128 rows.
constexpr int64_t kMaxBatchSlots = int64_t(1) << 15;
constexpr int64_t kMinJUnit = 256;

int64_t batch_slot_cap(int64_t n_total, int64_t S)
{
    // j parts are at least kMinJUnit records: at most (row blocks) x (pn / kMinJUnit + 1)
    const int64_t rb = n_total / 64 + std::max<int64_t>(S, 1) + 1;
    const int64_t parts = (n_total + 64 * std::max<int64_t>(S, 1)) / kMinJUnit + 1;
    const double bound = (double)rb * (double)parts;
    return bound < (double)kMaxBatchSlots ? (int64_t)bound : kMaxBatchSlots;
}

struct BatWs {
    size_t rec_off, unit_off, off_off, poff_off, systab_off, red_off, part_off, ticket_off, total;
    size_t part_bytes;       // the partial region
    int64_t max_slots;       // partial budget: max_slots slots of 128 rows
    int64_t max_units;       // capacity of the unit table
    int64_t max_records;     // capacity of the record buffer
};

// the batched symmetric tiles apply to this law and precision
bool law_has_bsym(const nbody_law *law) { return bsym_supported(law->kind, law->precision); }

// row blocks of an ensemble (any rows per lane): at most one per 64 rows plus one per system
int64_t red_capacity(int64_t n_total, int64_t S) { return n_total / 64 + std::max<int64_t>(S, 1) + 1; }

// The batched symmetric tiles (systems of at most kBSymMaxSystem particles, padded to blocks of
// kBSymRecords): their tiles, and their FP32 slot partials (one per row and block of its system),
// bounded over every ensemble of n_total particles in S systems.
int64_t bsym_blocks_bound(int64_t n_total, int64_t S) { return n_total / kBSymRecords + std::max<int64_t>(S, 1); }
int64_t bsym_units_bound(int64_t n_total, int64_t S)
{
    return bsym_blocks_bound(n_total, S) * (kBSymMaxSystem / kBSymRecords + 1) / 2 + 1;
}
size_t bsym_slot_bytes_bound(int64_t n_total, int64_t S)
{
    return (size_t)(n_total + (int64_t)(kBSymRecords - 1) * std::max<int64_t>(S, 1)) *
           (size_t)(kBSymMaxSystem / kBSymRecords) * 4 * sizeof(float);
}

BatWs bat_layout(const nbody_law *law, int64_t n_total, int64_t S)
{
    BatWs w{};
    // records padded per system to 64 (one-sided) or to 256 (symmetric tiles)
    const int64_t npad_max = n_total + kBSymRecords * std::max<int64_t>(S, 1);
    w.max_slots = batch_slot_cap(n_total, S);
    // units = (row blocks of single-part systems) + (slots of split systems); the
    // planner admits up to 2 * max_slots / ipl slots (ipl >= 1); or the symmetric tiles
    const int64_t units_max = std::max(n_total / 64 + std::max<int64_t>(S, 1) + 1 + 2 * w.max_slots,
                                       bsym_units_bound(n_total, S));
    w.max_units = units_max;
    w.max_records = npad_max;
    size_t off = 0;
    w.rec_off = off;
    off = align256(off + (size_t)npad_max * rec_bytes(law->kind, law->precision));
    w.unit_off = off;
    off = align256(off + (size_t)units_max * 4 * sizeof(int32_t));
    w.off_off = off;
    off = align256(off + (size_t)(S + 1) * sizeof(int64_t));
    w.poff_off = off;
    off = align256(off + (size_t)(S + 1) * sizeof(int64_t));
    w.systab_off = off;
    off = align256(off + (size_t)std::max<int64_t>(S, 1) * 3 * sizeof(int64_t));
    w.red_off = off;
    off = align256(off + (size_t)red_capacity(n_total, S) * 2 * sizeof(int32_t));
    w.part_off = off;
    // the one-sided part sums or the symmetric tiles' slot partials (never both in one launch)
    w.part_bytes = std::max((size_t)w.max_slots * 128 * 4 * sizeof(double),
                            law_has_bsym(law) ? bsym_slot_bytes_bound(n_total, S) : (size_t)0);
    off = align256(off + w.part_bytes);
    w.ticket_off = off;
    off = align256(off + 256);
    w.total = off;
    return w;
}

// Batched adjoint: adjoint records padded per system, the unit tables and the
// part sums of split systems (8 doubles per row; half the forward's slot count).
struct AdjBatWs {
    size_t rec_off, unit_off, off_off, poff_off, systab_off, red_off, part_off, ticket_off, type_off, total;
    size_t part_bytes;
    int64_t max_slots, max_units, max_records;
};

// the batched adjoint's symmetric tiles apply to this law and precision
bool law_has_bsym_adj(const nbody_law *law) { return bsym_adj_supported(law->kind, law->precision); }

AdjBatWs adjb_layout(const nbody_law *law, int64_t n_total, int64_t S)
{
    AdjBatWs w{};
    // records padded per system to 64 (one-sided) or to 256 (symmetric tiles)
    const int64_t npad_max = n_total + kBSymRecords * std::max<int64_t>(S, 1);
    w.max_slots = std::max<int64_t>(1, batch_slot_cap(n_total, S) / 2);
    const int64_t units_max = std::max(n_total / 64 + std::max<int64_t>(S, 1) + 1 + 2 * w.max_slots,
                                       bsym_units_bound(n_total, S));
    w.max_units = units_max;
    w.max_records = npad_max;
    size_t off = 0;
    w.rec_off = off;
    off = align256(off + (size_t)npad_max * adj_rec_bytes(law->kind, law->precision));
    w.unit_off = off;
    off = align256(off + (size_t)units_max * 4 * sizeof(int32_t));
    w.off_off = off;
    off = align256(off + (size_t)(S + 1) * sizeof(int64_t));
    w.poff_off = off;
    off = align256(off + (size_t)(S + 1) * sizeof(int64_t));
    w.systab_off = off;
    off = align256(off + (size_t)std::max<int64_t>(S, 1) * 3 * sizeof(int64_t));
    w.red_off = off;
    off = align256(off + (size_t)red_capacity(n_total, S) * 2 * sizeof(int32_t));
    w.part_off = off;
    // the one-sided part sums or the symmetric tiles' slot partials (3 or 6 FP32 sums per slot
    // row, in 128-bit vectors)
    w.part_bytes = std::max((size_t)w.max_slots * 128 * 8 * sizeof(double),
                            law_has_bsym_adj(law) ? bsym_slot_bytes_bound(n_total, S) *
                                                        (size_t)((bsym_adj_sums(law->kind) + 3) / 4)
                                                  : (size_t)0);
    off = align256(off + w.part_bytes);
    w.ticket_off = off;
    off = align256(off + 256);
    w.type_off = off;
    off = align256(off + (size_t)kTypePartDoubles * sizeof(double));
    w.total = off;
    return w;
}

// Charge scaling packed into the records so that qs_i qs_j is the Coulomb prefactor.
double qscale_of(const nbody_law *law)
{
    switch (law->kind) {
    case NBODY_LAW_LJC_LINEAR: return std::sqrt(2.0 * law->coulomb_k / law->dielectric);
    case NBODY_LAW_LJC_CONSTANT: return std::sqrt(law->coulomb_k / law->dielectric);
    case NBODY_LAW_LJC_SIGMOIDAL: return std::sqrt(law->coulomb_k);
    default: return 0.0;
    }
}

Epilogue make_epi(const nbody_law *law, double *out_force, double *out_pot)
{
    Epilogue e{};
    if (law->kind == NBODY_LAW_GRAVITY) {
        e.fscale = law->G;
        e.pscale = -law->G;
    } else {
        e.fscale = 1.0;     // the pair function accumulates -W d = W (r_i - r_j) already
        // LJC(linear) accumulates 2 u_ij, the other dielectrics u_ij
        e.pscale = law->kind == NBODY_LAW_LJC_LINEAR ? 0.5 : 1.0;
    }
    e.out_force = out_force;
    e.out_pot = out_pot;
    e.kick = 0;
    return e;
}

// pack + all-pairs (+ split reduction) for one system already validated
int run_forward(const nbody_law *law, const Cfg &c, const double *pos, const double *params,
                int64_t n, const int64_t *rows, int64_t nrows, const Epilogue &epi, bool pot,
                void *ws, const FwdWs &lay, hipStream_t s, PackLaunch *pk_in,
                const ExclArgs &excl = ExclArgs{}, bool timed = true, int64_t share = 0,
                int64_t n_shares = 1)
{
    // the symmetric tiles (j_stage 2) evaluate whole systems; sanitize admits the
    // configuration only for FP32_KAHAN / FP32_FP64ACC forward laws and gravity's backward
    const bool sym = c.j_stage == kSymStage && rows == nullptr && nrows == n && excl.off == nullptr;
    const int blk = sym ? c.j_tile / 64 : 0;
    const int64_t npad = sym ? sym_npad(n, blk) : round_up(n, 64);
    char *base = (char *)ws;
    PackLaunch pk{};
    if (pk_in) pk = *pk_in;
    pk.law = law->kind;
    pk.prec = law->precision;
    pk.n = n;
    pk.npad = npad;
    if (!pk_in) pk.pos = const_cast<double *>(pos);
    pk.params = params;
    pk.qscale = qscale_of(law);
    pk.rec = base + lay.rec_off;
    hipError_t e = launch_pack(pk, s);
    if (e != hipSuccess) return hip_fail(e, "pack");

    if (sym) {
        SymLaunch a{};
        a.op = sym_op_of(law->kind);
        a.prec = law->precision;
        a.pot = pot ? 1 : 0;
        a.blk = blk;
        a.ich = c.ipl;
        a.split = c.j_split;
        a.nblk = npad / ((int64_t)blk * 64);
        a.npad = npad;
        a.n = n;
        a.eps2 = law->kind == NBODY_LAW_GRAVITY ? law->softening * law->softening : 0.0;
        for (int c = 0; c < 4; ++c) a.zeta[c] = law->kind == NBODY_LAW_LJC_SIGMOIDAL ? law->zeta[c] : 0.0;
        a.rec = base + lay.rec_off;
        a.partial = (float4 *)(base + lay.part_off);
        sym_share_range(a.nblk, share, n_shares, a.t0, a.count);
        a.epi = epi;
        Timer t(s, timed);
        e = launch_sym(a, s);
        t.stop();
        if (e != hipSuccess) return hip_fail(e, "symmetric all-pairs kernel");
        e = launch_sym_reduce(a, s);
        if (e != hipSuccess) return hip_fail(e, "symmetric partial reduction");
        return NBODY_OK;
    }

    FwdLaunch f{};
    f.law = law->kind;
    f.prec = law->precision;
    f.ipl = c.ipl;
    f.pot = pot ? 1 : 0;
    f.block = c.block;
    f.npad = npad;
    f.nrows = nrows;
    f.rows = rows;
    f.j_split = c.j_split;
    f.split_len = round_up((npad + c.j_split - 1) / c.j_split, 64);
    f.j_tile = c.j_tile;
    f.j_stage = c.j_stage;
    f.eps2 = law->kind == NBODY_LAW_GRAVITY ? law->softening * law->softening : 0.0;
    for (int c = 0; c < 4; ++c) f.zeta[c] = law->kind == NBODY_LAW_LJC_SIGMOIDAL ? law->zeta[c] : 0.0;
    f.rec = base + lay.rec_off;
    f.partial = (double *)(base + lay.part_off);
    f.epi = epi;
    f.excl = excl;
    Timer t(s, timed);
    e = launch_forces(f, s);
    t.stop();
    if (e != hipSuccess) return hip_fail(e, "all-pairs kernel");
    e = launch_reduce_split(f, s);
    if (e != hipSuccess) return hip_fail(e, "split reduction");
    return NBODY_OK;
}

int check_ws(void *ws, size_t have, size_t need)
{
    if (!ws && need) return fail(NBODY_EWORKSPACE, "workspace is NULL (need %zu bytes)", need);
    if (have < need) return fail(NBODY_EWORKSPACE, "workspace too small: %zu < %zu bytes", have, need);
    return NBODY_OK;
}

int validate_jerk_law(const nbody_law *law)
{
    int rc = validate_law(law, false);
    if (rc) return rc;
    if (law->kind != NBODY_LAW_GRAVITY) return fail(NBODY_ENOTSUP, "the jerk is provided for gravity only");
    if (law->precision == NBODY_FP32_PLAIN)
        return fail(NBODY_ENOTSUP, "the jerk kernel is provided for FP64, FP32_FP64ACC and FP32_KAHAN");
    return NBODY_OK;
}

// pack (optionally predicted) records + acceleration/jerk kernel (+ split reduction)
int run_jerk(const nbody_law *law, const Cfg &c, const JerkPackLaunch &pk_in, const int64_t *rows,
             int64_t nrows, double *out_acc, double *out_jerk, double *out_pot, void *ws,
             const JerkWs &lay, hipStream_t s)
{
    // the symmetric tiles evaluate every row of the system (the callers pass them no row list)
    const bool sym = c.j_stage == kSymStage;
    if (sym && (rows != nullptr || nrows != pk_in.n || !symjerk_ok(law->kind, law->precision) ||
                pk_in.n > kSymJerkMaxN))
        return fail(NBODY_EINVAL, "the symmetric jerk tiles evaluate whole systems of FP32 gravity only");
    const int64_t npad = sym ? symjerk_npad(pk_in.n) : round_up(pk_in.n, 64);
    char *base = (char *)ws;
    JerkPackLaunch pk = pk_in;
    pk.prec = law->precision;
    pk.npad = npad;
    pk.rec = base + lay.rec_off;
    hipError_t e = launch_pack_jerk(pk, s);
    if (e != hipSuccess) return hip_fail(e, "jerk pack");
    if (sym) {
        SymJerkLaunch a{};
        a.prec = law->precision;
        a.pot = out_pot != nullptr;
        a.split = c.j_split == 2 ? 2 : 1;
        a.nblk = npad / ((int64_t)kSymJerkBlk * 64);
        a.npad = npad;
        a.n = pk_in.n;
        a.eps2 = law->softening * law->softening;
        a.G = law->G;
        a.rec = base + lay.rec_off;
        a.partial = (float4 *)(base + lay.part_off);
        a.out_acc = out_acc;
        a.out_jerk = out_jerk;
        a.out_pot = out_pot;
        Timer t(s);
        e = launch_symjerk(a, s);
        t.stop();
        if (e != hipSuccess) return hip_fail(e, "symmetric jerk tiles");
        e = launch_symjerk_reduce(a, s);
        if (e != hipSuccess) return hip_fail(e, "symmetric jerk slot reduction");
        return NBODY_OK;
    }
    JerkLaunch a{};
    a.prec = law->precision;
    a.ipl = c.ipl;
    a.pot = out_pot != nullptr;
    a.block = c.block;
    a.j_stage = c.j_stage;
    a.npad = npad;
    a.nrows = nrows;
    a.rows = rows;
    a.j_split = std::max(1, std::min(c.j_split, max_split(npad)));
    a.split_len = round_up((npad + a.j_split - 1) / a.j_split, 64);
    a.j_tile = c.j_tile;
    a.eps2 = law->softening * law->softening;
    a.G = law->G;
    a.rec = base + lay.rec_off;
    a.partial = (double *)(base + lay.part_off);
    a.out_acc = out_acc;
    a.out_jerk = out_jerk;
    a.out_pot = out_pot;
    Timer t(s);
    e = launch_jerk(a, s);
    t.stop();
    if (e != hipSuccess) return hip_fail(e, "jerk kernel");
    e = launch_jerk_reduce(a, s);
    if (e != hipSuccess) return hip_fail(e, "jerk split reduction");
    return NBODY_OK;
}

int jerk_impl(const double *pos, const double *vel, const double *mass, int64_t n,
              const int64_t *ilist, int64_t ni, const nbody_law *law, double *out_acc,
              double *out_jerk, double *out_potential, void *ws, size_t ws_bytes, void *stream,
              const Cfg *forced)
{
    int rc = validate_jerk_law(law);
    if (rc) return rc;
    if (n < 0 || ni < 0) return fail(NBODY_EINVAL, "n < 0 or ni < 0");
    if (n > (int64_t(1) << 40)) return fail(NBODY_EINVAL, "n too large");
    if (!ilist && ni != n) return fail(NBODY_EINVAL, "without ilist, ni must equal n");
    if (ni > 0 && n == 0) return fail(NBODY_EINVAL, "rows requested from an empty system");
    if (ni == 0) return NBODY_OK;
    if (!pos || !vel || !mass || !out_acc || !out_jerk)
        return fail(NBODY_EINVAL, "pos, vel, mass, out_acc and out_jerk must be non-NULL");
    const JerkWs lay = jerk_layout(NBODY_API_JERK, law, std::max(n, ni));
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    const int64_t npad = round_up(std::max(n, ni), 64);
    Cfg c = sanitize(forced ? *forced : choose(NBODY_API_JERK, law, ni, 1, out_potential != nullptr, n),
                     NBODY_API_JERK, law->kind, law->precision, npad);
    if (c.j_stage == kSymStage && (ilist || ni != n))   // the tiles take whole systems only
        c = one_sided(c, NBODY_API_JERK, law, ni, n, out_potential != nullptr);
    JerkPackLaunch pk{};
    pk.n = n;
    pk.pos = pos;
    pk.vel = vel;
    pk.mass = mass;
    return run_jerk(law, c, pk, ilist, ni, out_acc, out_jerk, out_potential, ws, lay, (hipStream_t)stream);
}

bool cfg_valid(const nbody_config *c)
{
    return c && c->block >= 64 && c->block <= (c->j_stage == kSymStage ? kSymThreads : 256) &&
           c->block % 64 == 0 && ipl_ok(c->i_per_lane) && c->j_tile >= 64 && c->j_tile % 64 == 0 &&
           c->j_tile <= (1 << 20) && c->j_split >= 1 && c->j_split <= kMaxSplit &&
           (c->j_stage == 0 || c->j_stage == 1 || c->j_stage == kSymStage);
}

Cfg from_abi(const nbody_config *c)
{
    Cfg r;
    r.block = c->block;
    r.ipl = c->i_per_lane;
    r.j_tile = c->j_tile;
    r.j_split = c->j_split;
    r.j_stage = c->j_stage;
    return r;
}

void to_abi(const Cfg &c, nbody_config *o)
{
    o->block = c.block;
    o->i_per_lane = c.ipl;
    o->j_tile = c.j_tile;
    o->j_split = c.j_split;
    o->j_stage = c.j_stage;
}

// ------------------------------------------------------------ batched plan
struct BatchPlan {
    std::vector<int64_t> poff;
    std::vector<int64_t> systab;      // [S][3] parts, records per part, first slot
    std::vector<int32_t> units;       // [n][4]
    std::vector<int32_t> red;         // [n_red][2] (system, row block) of the row blocks with P > 1
    int64_t npad_total = 0;
    int64_t n_slots = 0;
};

// Work units (system, row block, j part).  A system's padded j range of pn
// records is cut into P = ceil(pn / j_unit) parts of equal length (a multiple
// of 64; j_unit = 0: one part), so that large systems yield enough units to
// balance the persistent grid; each row block of a system with P > 1 owns P
// consecutive partial slots.
BatchPlan plan_batched(const int64_t *offsets, int64_t S, int ipl, int64_t j_unit)
{
    BatchPlan p;
    p.poff.assign((size_t)S + 1, 0);
    p.systab.assign((size_t)S * 3, 0);
    struct U {
        int64_t cost;
        int32_t s, rb, part;
    };
    std::vector<U> us;
    const int64_t rows = 64 * ipl;
    int64_t slots = 0;
    for (int64_t s = 0; s < S; ++s) {
        const int64_t ns = offsets[s + 1] - offsets[s];
        const int64_t pn = round_up(ns, 64);
        p.poff[s + 1] = p.poff[s] + pn;
        int64_t parts = (j_unit > 0 && pn > j_unit) ? (pn + j_unit - 1) / j_unit : 1;
        const int64_t plen = std::max<int64_t>(64, round_up((pn + parts - 1) / std::max<int64_t>(parts, 1), 64));
        parts = pn > 0 ? (pn + plen - 1) / plen : 1;
        const int64_t nrb = (ns + rows - 1) / rows;
        p.systab[3 * s] = parts;
        p.systab[3 * s + 1] = plen;
        p.systab[3 * s + 2] = parts > 1 ? slots : 0;
        if (parts > 1) {
            slots += nrb * parts;
            for (int64_t rb = 0; rb < nrb; ++rb) {
                p.red.push_back((int32_t)s);
                p.red.push_back((int32_t)rb);
            }
        }
        for (int64_t rb = 0; rb < nrb; ++rb) {
            const int64_t r = std::min(rows, ns - rb * rows);
            for (int64_t q = 0; q < parts; ++q) {
                const int64_t len = std::min(plen, pn - q * plen);
                us.push_back({r * len, (int32_t)s, (int32_t)rb, (int32_t)q});
            }
        }
    }
    p.npad_total = p.poff[S];
    p.n_slots = slots;
    // longest processing time first; ties keep system order (stable)
    std::stable_sort(us.begin(), us.end(), [](const U &a, const U &b) { return a.cost > b.cost; });
    p.units.resize(us.size() * 4);
    for (size_t k = 0; k < us.size(); ++k) {
        p.units[4 * k] = us[k].s;
        p.units[4 * k + 1] = us[k].rb;
        p.units[4 * k + 2] = us[k].part;
        p.units[4 * k + 3] = 0;
    }
    return p;
}

// The batched symmetric tiles' plan: systems padded to blocks of kBSymRecords; units (s, b1, b2)
// for b1 <= b2 < nb_s, the off-diagonal tiles first (the diagonal ones cost about 10/16 of
// them); per system (nb_s, 0, first float4 of its [nb_s][npad_s] slot partials); and the row
// blocks of 256 rows that the reduction walks.  n_slots counts float4 slot partials.
BatchPlan plan_bsym(const int64_t *offsets, int64_t S)
{
    BatchPlan p;
    p.poff.assign((size_t)S + 1, 0);
    p.systab.assign((size_t)S * 3, 0);
    std::vector<int32_t> diag;
    int64_t slots = 0;
    for (int64_t s = 0; s < S; ++s) {
        const int64_t ns = offsets[s + 1] - offsets[s];
        const int64_t pn = round_up(ns, kBSymRecords);
        const int64_t nb = pn / kBSymRecords;
        p.poff[s + 1] = p.poff[s] + pn;
        p.systab[3 * s] = nb;
        p.systab[3 * s + 2] = slots;
        slots += nb * pn;
        for (int64_t b1 = 0; b1 < nb; ++b1) {
            for (int64_t b2 = b1 + 1; b2 < nb; ++b2)
                for (int32_t v : {(int32_t)s, (int32_t)b1, (int32_t)b2, 0}) p.units.push_back(v);
            for (int32_t v : {(int32_t)s, (int32_t)b1, (int32_t)b1, 0}) diag.push_back(v);
        }
        for (int64_t rb = 0; rb * kBSymRecords < ns; ++rb) {
            p.red.push_back((int32_t)s);
            p.red.push_back((int32_t)rb);
        }
    }
    p.units.insert(p.units.end(), diag.begin(), diag.end());
    p.npad_total = p.poff[S];
    p.n_slots = slots;
    return p;
}

// the plan-cache key of the symmetric tiles (rows per lane -1: not a one-sided plan)
constexpr int kBSymPlanKey = -1;

// Plans depend only on (offsets, ipl, j_unit), and a simulation evaluates the
// same ensemble step after step: the last few plans are kept (exact match of
// the offsets, least recently used first out), so planning (a sort of all
// units) is paid once per ensemble.
struct CachedPlan {
    std::vector<int64_t> offsets;
    int ipl;
    int64_t j_unit;
    std::shared_ptr<const BatchPlan> plan;
};
std::mutex g_plan_mu;
std::vector<CachedPlan> g_plans;     // most recently used last
constexpr size_t kPlanCache = 8;

std::shared_ptr<const BatchPlan> cached_plan(const int64_t *offsets, int64_t S, int ipl, int64_t j_unit)
{
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (size_t k = 0; k < g_plans.size(); ++k) {
            const CachedPlan &c = g_plans[k];
            if (c.ipl == ipl && c.j_unit == j_unit && (int64_t)c.offsets.size() == S + 1 &&
                std::equal(c.offsets.begin(), c.offsets.end(), offsets)) {
                CachedPlan hit = c;
                g_plans.erase(g_plans.begin() + (std::ptrdiff_t)k);
                g_plans.push_back(hit);
                return hit.plan;
            }
        }
    }
    auto plan = std::make_shared<const BatchPlan>(ipl == kBSymPlanKey ? plan_bsym(offsets, S)
                                                                      : plan_batched(offsets, S, ipl, j_unit));
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plans.size() >= kPlanCache) g_plans.erase(g_plans.begin());
    g_plans.push_back({std::vector<int64_t>(offsets, offsets + S + 1), ipl, j_unit, plan});
    return plan;
}

// Device copies of plan tables.  A batched launch reads four tables: the units, the caller's
// offsets, the padded offsets and the per-system table.  They depend only on the plan's key
// (offsets, rows per lane, part length), so each device keeps one copy per key, made at the
// first launch of that key on the device (one allocation and one synchronous upload) and kept
// until the process ends: later launches copy nothing from the host, so they can be captured
// in a graph, and a captured launch may read the tables at any later replay.  At most
// kResidentTableBytes of tables are kept per device; past that, launches copy their tables
// into the workspace (from pageable host memory, on the stream) as every launch once did.
struct DevTables {
    int32_t *units = nullptr;
    int64_t *off = nullptr, *poff = nullptr, *systab = nullptr;
    int32_t *red = nullptr;
};
struct ResidentKey {
    int device;
    int ipl;
    int64_t j_unit;
    std::vector<int64_t> offsets;
    bool operator<(const ResidentKey &o) const
    {
        return std::tie(device, ipl, j_unit, offsets) < std::tie(o.device, o.ipl, o.j_unit, o.offsets);
    }
};
constexpr size_t kResidentTableBytes = size_t(256) << 20;
std::mutex g_resident_mu;
std::map<ResidentKey, DevTables> g_resident;
std::map<int, size_t> g_resident_bytes;      // per device

// The device tables of `plan` (key offsets / ipl / j_unit) on the current device, uploading
// them on first use.  Returns false, with *rc == 0, when the per-device budget is spent (the
// caller then copies the tables into its workspace), and false with *rc set on an error: a
// first launch of a key inside a stream capture (no allocation or upload can be captured).
bool resident_tables(const BatchPlan &plan, const int64_t *offsets, int64_t S, int ipl, int64_t j_unit,
                     hipStream_t s, DevTables *out, int *rc)
{
    *rc = NBODY_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *rc = fail(NBODY_EHIP, "hipGetDevice failed");
        return false;
    }
    ResidentKey key{dev, ipl, j_unit, std::vector<int64_t>(offsets, offsets + S + 1)};
    std::lock_guard<std::mutex> lk(g_resident_mu);
    auto it = g_resident.find(key);
    if (it != g_resident.end()) {
        *out = it->second;
        return true;
    }
    const size_t b_units = align256(plan.units.size() * sizeof(int32_t));
    const size_t b_off = align256((size_t)(S + 1) * sizeof(int64_t));
    const size_t b_sys = align256(std::max<size_t>(plan.systab.size(), 1) * sizeof(int64_t));
    const size_t b_red = align256(std::max<size_t>(plan.red.size(), 1) * sizeof(int32_t));
    const size_t bytes = b_units + 2 * b_off + b_sys + b_red;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
    if (cap != hipStreamCaptureStatusNone) {
        *rc = fail(NBODY_EINVAL, "the first batched launch of an ensemble cannot be captured (it uploads the "
                   "ensemble's plan tables): launch it once before capturing");
        return false;
    }
    if (g_resident_bytes[dev] + bytes > kResidentTableBytes) return false;
    void *buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;                                  // no room: the workspace copy still works
    }
    char *b = (char *)buf;
    DevTables t;
    t.units = (int32_t *)b;
    t.off = (int64_t *)(b + b_units);
    t.poff = (int64_t *)(b + b_units + b_off);
    t.systab = (int64_t *)(b + b_units + 2 * b_off);
    t.red = (int32_t *)(b + b_units + 2 * b_off + b_sys);
    hipError_t e = hipMemcpy(t.units, plan.units.data(), plan.units.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.off, offsets, (size_t)(S + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.poff, plan.poff.data(), (size_t)(S + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !plan.systab.empty())
        e = hipMemcpy(t.systab, plan.systab.data(), plan.systab.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !plan.red.empty())
        e = hipMemcpy(t.red, plan.red.data(), plan.red.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(buf);
        *rc = hip_fail(e, "batched plan tables");
        return false;
    }
    g_resident_bytes[dev] += bytes;
    g_resident.emplace(std::move(key), t);
    *out = t;
    return true;
}

// The tables of a batched launch: the device copies of its plan, or copies in the workspace
// regions given (pageable sources: the runtime stages them before returning).
int batched_tables(const BatchPlan &plan, const int64_t *offsets, int64_t S, int ipl, int64_t j_unit,
                   hipStream_t s, char *base, size_t unit_off, size_t off_off, size_t poff_off, size_t systab_off,
                   size_t red_off, DevTables *t)
{
    int rc = NBODY_OK;
    if (resident_tables(plan, offsets, S, ipl, j_unit, s, t, &rc)) return NBODY_OK;
    if (rc) return rc;
    t->units = (int32_t *)(base + unit_off);
    t->off = (int64_t *)(base + off_off);
    t->poff = (int64_t *)(base + poff_off);
    t->systab = (int64_t *)(base + systab_off);
    t->red = (int32_t *)(base + red_off);
    hipError_t e = hipMemcpyAsync(t->units, plan.units.data(), plan.units.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(t->off, offsets, (size_t)(S + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t->poff, plan.poff.data(), (size_t)(S + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t->systab, plan.systab.data(), plan.systab.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !plan.red.empty())
        e = hipMemcpyAsync(t->red, plan.red.data(), plan.red.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "batched tables");
    return NBODY_OK;
}

// The plan of one batched launch: j parts of about `per_wave` units per resident wave
// (`resident` waves on the whole chip; the configuration's j_split, 8 by the rule: more
// parts balance the persistent grid better, fewer parts leave fewer partial sums to add),
// no part shorter than kMinJUnit records,
// the part length doubled until the partial slots of split systems fit the
// workspace (max_slots slots of 128 rows; a slot holds one row block, 64 x ipl
// rows).
struct PlanChoice {
    std::shared_ptr<const BatchPlan> plan;
    int64_t j_unit;
};

PlanChoice plan_for_launch(const int64_t *offsets, int64_t S, int ipl, int64_t resident, int64_t max_slots,
                           int per_wave = kBatchUnitsPerWave)
{
    double work = 0.0;
    for (int64_t q = 0; q < S; ++q) {
        const int64_t ns = offsets[q + 1] - offsets[q];
        work += (double)ns * (double)round_up(ns, 64);
    }
    resident = std::max<int64_t>(resident, 1);
    per_wave = std::max(1, per_wave);
    int64_t j_unit = round_up((int64_t)(work / ((double)per_wave * (double)resident * 64.0 * ipl)) + 1, 64);
    j_unit = std::max(kMinJUnit, j_unit);
    std::shared_ptr<const BatchPlan> pp = cached_plan(offsets, S, ipl, j_unit);
    while (pp->n_slots * ipl > 2 * max_slots) {
        j_unit *= 2;
        pp = cached_plan(offsets, S, ipl, j_unit);
    }
    return {pp, j_unit};
}

// Whether a plan fits the workspace regions it is copied into and the part
// slots its units address: the unit table (max_units units), the padded
// records (max_records) and max_slots slots of 128 rows.
bool plan_fits(const BatchPlan &p, int ipl, int64_t max_units, int64_t max_records, int64_t max_slots,
               int64_t max_red)
{
    return (int64_t)p.units.size() / 4 <= max_units && p.npad_total <= max_records &&
           p.n_slots * ipl <= 2 * max_slots && (int64_t)p.red.size() / 2 <= max_red;
}

int g_num_cus = 0;

int device_cus()
{
    if (g_num_cus > 0) return g_num_cus;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        g_num_cus = prop.multiProcessorCount;
    if (g_num_cus <= 0) g_num_cus = 256;
    return g_num_cus;
}

// Architecture name of the current device ("gfx950"; feature suffixes dropped),
// or "unknown" without one.
std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// whether the symmetric tiles take this ensemble: law and precision, no exclusion lists, and
// every system within kBSymMaxSystem
bool bsym_takes(const nbody_law *law, const int64_t *offsets, int64_t S, bool excl)
{
    if (excl || !law_has_bsym(law)) return false;
    for (int64_t s = 0; s < S; ++s)
        if (offsets[s + 1] - offsets[s] > kBSymMaxSystem) return false;
    return true;
}

// pack (systems padded to blocks of 256) + symmetric tiles + slot-ordered reduction
int run_bsym(const nbody_law *law, const int64_t *offsets, int64_t S, const double *pos, const double *params,
             double *out_force, double *out_pot, void *ws, const BatWs &lay, hipStream_t s)
{
    std::shared_ptr<const BatchPlan> pp = cached_plan(offsets, S, kBSymPlanKey, 0);
    const BatchPlan &plan = *pp;
    if (plan.units.empty()) return NBODY_OK;
    if ((int64_t)plan.units.size() / 4 > lay.max_units || plan.npad_total > lay.max_records ||
        (size_t)plan.n_slots * 4 * sizeof(float) > lay.part_bytes ||
        (int64_t)plan.red.size() / 2 > red_capacity(offsets[S], S))
        return fail(NBODY_EWORKSPACE, "internal: batched symmetric plan exceeds its workspace regions "
                    "(%lld tiles, %lld slot partials)", (long long)(plan.units.size() / 4), (long long)plan.n_slots);
    char *base = (char *)ws;
    DevTables tab;
    int rc = batched_tables(plan, offsets, S, kBSymPlanKey, 0, s, base, lay.unit_off, lay.off_off, lay.poff_off,
                            lay.systab_off, lay.red_off, &tab);
    if (rc) return rc;
    BatchPackLaunch pk{};
    pk.law = law->kind;
    pk.prec = law->precision;
    pk.n_systems = S;
    pk.npad_total = plan.npad_total;
    pk.off = tab.off;
    pk.poff = tab.poff;
    pk.pos = pos;
    pk.params = params;
    pk.qscale = qscale_of(law);
    pk.rec = base + lay.rec_off;
    hipError_t e = launch_pack_batched(pk, s);
    if (e != hipSuccess) return hip_fail(e, "batched pack");
    BSymLaunch a{};
    a.law = law->kind;
    a.prec = law->precision;
    a.pot = out_pot != nullptr;
    a.n_units = (int64_t)plan.units.size() / 4;
    a.units = tab.units;
    a.off = tab.off;
    a.poff = tab.poff;
    a.systab = tab.systab;
    a.red = tab.red;
    a.n_red = (int64_t)plan.red.size() / 2;
    a.n_systems = S;
    a.eps2 = law->kind == NBODY_LAW_GRAVITY ? law->softening * law->softening : 0.0;
    for (int c = 0; c < 4; ++c) a.zeta[c] = law->kind == NBODY_LAW_LJC_SIGMOIDAL ? law->zeta[c] : 0.0;
    a.rec = base + lay.rec_off;
    a.partial = (float4 *)(base + lay.part_off);
    a.epi = make_epi(law, out_force, out_pot);
    Timer t(s);
    e = launch_bsym(a, s);
    t.stop();
    if (e != hipSuccess) return hip_fail(e, "batched symmetric kernel");
    e = launch_bsym_reduce(a, s);
    if (e != hipSuccess) return hip_fail(e, "batched symmetric reduction");
    return NBODY_OK;
}

int run_batched(const nbody_law *law, const Cfg &c, const int64_t *offsets, int64_t S,
                const double *pos, const double *params, double *out_force, double *out_pot,
                void *ws, const BatWs &lay, hipStream_t s, const ExclArgs &excl = ExclArgs{})
{
    const int per_cu =
        std::max(1, batched_blocks_per_cu_cached(law->kind, law->precision, c.ipl, out_pot != nullptr,
                                                 c.j_stage, c.block, excl.off != nullptr));
    const int64_t resident = (int64_t)device_cus() * per_cu * (c.block / 64);
    const PlanChoice pc = plan_for_launch(offsets, S, c.ipl, resident, lay.max_slots, c.j_split);
    const BatchPlan &plan = *pc.plan;
    if (plan.units.empty()) return NBODY_OK;
    if (!plan_fits(plan, c.ipl, lay.max_units, lay.max_records, lay.max_slots, red_capacity(offsets[S], S)))
        return fail(NBODY_EWORKSPACE, "internal: batched plan exceeds its workspace regions "
                    "(%lld units, %lld slots)", (long long)(plan.units.size() / 4), (long long)plan.n_slots);
    char *base = (char *)ws;
    DevTables tab;
    int rc = batched_tables(plan, offsets, S, c.ipl, pc.j_unit, s, base, lay.unit_off, lay.off_off, lay.poff_off,
                            lay.systab_off, lay.red_off, &tab);
    if (rc) return rc;
    int32_t *d_units = tab.units;
    int64_t *d_off = tab.off;
    int64_t *d_poff = tab.poff;
    int64_t *d_systab = tab.systab;
    hipError_t e;

    BatchPackLaunch pk{};
    pk.law = law->kind;
    pk.prec = law->precision;
    pk.n_systems = S;
    pk.npad_total = plan.npad_total;
    pk.off = d_off;
    pk.poff = d_poff;
    pk.pos = pos;
    pk.params = params;
    pk.qscale = qscale_of(law);
    pk.rec = base + lay.rec_off;
    pk.ticket = (int *)(base + lay.ticket_off);
    e = launch_pack_batched(pk, s);
    if (e != hipSuccess) return hip_fail(e, "batched pack");

    BatchLaunch b{};
    b.law = law->kind;
    b.prec = law->precision;
    b.ipl = c.ipl;
    b.pot = out_pot != nullptr;
    b.block = c.block;
    b.j_stage = c.j_stage;
    const int64_t n_units = (int64_t)plan.units.size() / 4;
    const int64_t waves_needed = n_units;
    const int64_t blocks_needed = (waves_needed + c.block / 64 - 1) / (c.block / 64);
    b.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)device_cus() * per_cu, blocks_needed));
    b.n_units = n_units;
    b.units = d_units;
    b.off = d_off;
    b.poff = d_poff;
    b.systab = d_systab;
    b.partial = (double *)(base + lay.part_off);
    b.any_parts = plan.n_slots > 0;
    b.red = tab.red;
    b.n_red = (int64_t)plan.red.size() / 2;
    b.n_systems = S;
    b.n_total = offsets[S];
    b.npad_total = plan.npad_total;
    b.j_tile = c.j_tile;
    b.eps2 = law->kind == NBODY_LAW_GRAVITY ? law->softening * law->softening : 0.0;
    for (int c = 0; c < 4; ++c) b.zeta[c] = law->kind == NBODY_LAW_LJC_SIGMOIDAL ? law->zeta[c] : 0.0;
    b.rec = base + lay.rec_off;
    b.ticket = (int *)(base + lay.ticket_off);
    b.ticket_zeroed = 1;
    b.epi = make_epi(law, out_force, out_pot);
    b.excl = excl;
    Timer t(s);
    e = launch_batched(b, s);
    t.stop();
    if (e != hipSuccess) return hip_fail(e, "batched kernel");
    return NBODY_OK;
}


int validate_offsets(const int64_t *offsets, int64_t S)
{
    if (S < 0) return fail(NBODY_EINVAL, "n_systems < 0");
    if (!offsets) return fail(NBODY_EINVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(NBODY_EINVAL, "offsets[0] must be 0");
    for (int64_t s = 0; s < S; ++s) {
        if (offsets[s + 1] < offsets[s]) return fail(NBODY_EINVAL, "offsets decrease at %lld", (long long)s);
        if (offsets[s + 1] - offsets[s] > (int64_t(1) << 30))
            return fail(NBODY_EINVAL, "system %lld is larger than 2^30 particles", (long long)s);
    }
    if (S > (int64_t(1) << 30)) return fail(NBODY_EINVAL, "too many systems");
    return NBODY_OK;
}

// Exclusion lists: host struct of device arrays.  The kernels clamp every
// list range to [0, count) and only compare entries, so list content cannot
// cause an out-of-bounds access; `offsets` must hold n + 1 entries.
int validate_excl(const nbody_exclusions *ex, const nbody_law *law, bool backward)
{
    if (!ex) return NBODY_OK;
    if (!ex->offsets) return fail(NBODY_EINVAL, "exclusions.offsets is NULL");
    if (ex->count < 0) return fail(NBODY_EINVAL, "exclusions.count < 0");
    if (ex->count > 0 && !ex->index) return fail(NBODY_EINVAL, "exclusions.index is NULL");
    if (law->kind == NBODY_LAW_GRAVITY) return fail(NBODY_ENOTSUP, "exclusion lists apply to the LJC laws");
    if (backward && law->kind != NBODY_LAW_LJC_LINEAR)
        return fail(NBODY_ENOTSUP, "the adjoint with exclusions is provided for LJC(linear)");
    if (law->precision == NBODY_FP32_PLAIN)
        return fail(NBODY_ENOTSUP, "exclusion lists are provided for FP64, FP32_FP64ACC and FP32_KAHAN");
    return NBODY_OK;
}

ExclArgs excl_args(const nbody_exclusions *ex)
{
    ExclArgs a{};
    if (ex) {
        a.off = ex->offsets;
        a.idx = ex->index;
        a.count = ex->count;
    }
    return a;
}

// the exclusion kernels use LDS staging with up to 2 rows per lane
Cfg with_excl(Cfg c, bool excl)
{
    if (excl) {
        c.j_stage = 1;
        c.ipl = std::min(c.ipl, 2);
    }
    return c;
}

int forces_impl(const double *pos, const double *params, int64_t n, const int64_t *rows,
                int64_t nrows, const nbody_law *law, double *out_force, double *out_potential,
                void *ws, size_t ws_bytes, void *stream, const Cfg *forced,
                const nbody_exclusions *excl = nullptr)
{
    int rc = validate_law(law, false);
    if (rc) return rc;
    rc = validate_excl(excl, law, false);
    if (rc) return rc;
    if (excl && rows) return fail(NBODY_EINVAL, "exclusion lists apply to whole-system evaluations");
    if (n < 0 || nrows < 0) return fail(NBODY_EINVAL, "n < 0");
    if (n > (int64_t(1) << 40)) return fail(NBODY_EINVAL, "n too large");
    if (nrows > 0 && n == 0) return fail(NBODY_EINVAL, "rows requested from an empty system");
    if (nrows == 0) return NBODY_OK;
    if (!pos || !params || !out_force) return fail(NBODY_EINVAL, "pos, params and out_force must be non-NULL");
    if (rows == nullptr && nrows != n) return fail(NBODY_EINVAL, "row count mismatch");
    const FwdWs lay = fwd_layout(NBODY_API_FORCES, law, std::max(n, nrows));
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    const bool pot = out_potential != nullptr;
    Cfg c = sanitize(forced ? *forced : choose(NBODY_API_FORCES, law, nrows, 1, pot, n), NBODY_API_FORCES,
                     law->kind, law->precision, round_up(std::max(n, nrows), 64));
    if (rows || excl) c = one_sided(c, NBODY_API_FORCES, law, nrows, n, pot);
    const Cfg cs = with_excl(sanitize(c, NBODY_API_FORCES, law->kind, law->precision,
                                      round_up(std::max(n, nrows), 64)), excl != nullptr);
    return run_forward(law, cs, pos, params, n, rows, nrows, make_epi(law, out_force, out_potential),
                       pot, ws, lay, (hipStream_t)stream, nullptr, excl_args(excl));
}

// One share of the symmetric pair tiles (gravity or an LJC law, FP32 pair arithmetic): the tiles of order
// range share / n_shares of the triangle, reduced into per-row partial sums of all n rows.
int share_impl(const double *pos, const double *params, int64_t n, const nbody_law *law, int32_t share,
               int32_t n_shares, double *out_force, double *out_potential, void *ws, size_t ws_bytes,
               void *stream)
{
    int rc = validate_law(law, false);
    if (rc) return rc;
    if (!sym_eligible(NBODY_API_FORCES, law->kind, law->precision))
        return fail(NBODY_ENOTSUP, "shares of the symmetric pair tiles are provided for FP32_KAHAN or "
                    "FP32_FP64ACC (FP64 and FP32_PLAIN shard by rows: nbody_forces_subset)");
    if (n < 0) return fail(NBODY_EINVAL, "n < 0");
    if (n > kSymMaxN) return fail(NBODY_ENOTSUP, "the symmetric pair tiles take up to %lld particles",
                                  (long long)kSymMaxN);
    if (n_shares < 1 || share < 0 || share >= n_shares)
        return fail(NBODY_EINVAL, "share %d of %d: need 0 <= share < n_shares", (int)share, (int)n_shares);
    if (n == 0) return NBODY_OK;
    if (!pos || !params || !out_force) return fail(NBODY_EINVAL, "pos, params and out_force must be non-NULL");
    const FwdWs lay = fwd_layout(NBODY_API_FORCES, law, n);
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    const bool pot = out_potential != nullptr;
    const int64_t npad = round_up(n, 64);
    Cfg c = choose(NBODY_API_FORCES, law, n, 1, pot);
    if (c.j_stage != kSymStage) {                      // the rule's symmetric shape for this size
        c = Cfg{};
        c.j_stage = kSymStage;
        c.j_tile = n <= kSymSmallMax ? 1024 : 2048;
    }
    c = sanitize(c, NBODY_API_FORCES, law->kind, law->precision, npad);
    return run_forward(law, c, pos, params, n, nullptr, n, make_epi(law, out_force, out_potential), pot, ws,
                       lay, (hipStream_t)stream, nullptr, ExclArgs{}, true, share, n_shares);
}

int batched_impl(const int64_t *offsets, int64_t S, const double *pos, const double *params,
                 const nbody_law *law, double *out_force, double *out_potential, void *ws,
                 size_t ws_bytes, void *stream, const Cfg *forced,
                 const nbody_exclusions *excl = nullptr)
{
    int rc = validate_law(law, false);
    if (rc) return rc;
    rc = validate_excl(excl, law, false);
    if (rc) return rc;
    rc = validate_offsets(offsets, S);
    if (rc) return rc;
    const int64_t n = offsets[S];
    if (n == 0) return NBODY_OK;
    if (!pos || !params || !out_force) return fail(NBODY_EINVAL, "pos, params and out_force must be non-NULL");
    const BatWs lay = bat_layout(law, n, S);
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    Cfg c = sanitize(forced ? *forced : choose(NBODY_API_BATCHED, law, n, S, out_potential != nullptr),
                     NBODY_API_BATCHED, law->kind, law->precision, 64);
    if (c.j_stage == kSymStage) {
        if (bsym_takes(law, offsets, S, excl != nullptr))
            return run_bsym(law, offsets, S, pos, params, out_force, out_potential, ws, lay, (hipStream_t)stream);
        c = heuristic(NBODY_API_BATCHED, law->kind, law->precision, n, n, S, out_potential != nullptr, false);
    }
    return run_batched(law, with_excl(c, excl != nullptr), offsets, S, pos, params, out_force, out_potential, ws,
                       lay, (hipStream_t)stream, excl_args(excl));
}

// candidate list for the measured search
std::vector<Cfg> candidate_set(int api, int law, int prec, int64_t n, bool pot);

bool same_cfg(const Cfg &a, const Cfg &b)
{
    return a.block == b.block && a.ipl == b.ipl && a.j_tile == b.j_tile && a.j_split == b.j_split &&
           a.j_stage == b.j_stage;
}

// The configurations the autotuners time, the heuristic's own choice first:
// with kTuneMargin, a measured near-tie keeps it, so the choice repeats across
// runs and devices of one kind.
std::vector<Cfg> candidates(int api, int law, int prec, int64_t n, bool pot)
{
    std::vector<Cfg> out{sanitize(heuristic(api, law, prec, n, n, 1, pot), api, law, prec,
                                  round_up(std::max<int64_t>(n, 1), 64))};
    for (const Cfg &c : candidate_set(api, law, prec, n, pot))
        if (!same_cfg(c, out[0])) out.push_back(c);
    return out;
}

// The timing sweep of both autotuners.  run(c) enqueues one evaluation with
// configuration c on s.  One untimed evaluation comes first (the first
// candidate is not timed on an idle device); each candidate is then timed
// twice and its faster run counts; a later candidate replaces the best only if
// faster by more than kTuneMargin.  A winner other than the first candidate
// (the heuristic's) is then timed against it three more times, alternating,
// and kept only if it still wins by the margin, so that one noisy timing does
// not displace the rule.
template <typename Run>
int tune_sweep(const std::vector<Cfg> &cands, hipStream_t s, Run run, Cfg &best, double &best_ms)
{
    best_ms = 1e300;
    if (cands.empty()) return fail(NBODY_EINVAL, "no candidate configurations");
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return fail(NBODY_EHIP, "event creation failed");
    }
    bool saved_timing;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        saved_timing = g_timing;
        g_timing = false;
    }
    auto time_once = [&](const Cfg &c, double &ms_out) -> int {
        (void)hipEventRecord(a, s);
        const int r = run(c);
        (void)hipEventRecord(b, s);
        if (r) return r;
        if (hipEventSynchronize(b) != hipSuccess) return fail(NBODY_EHIP, "autotune synchronisation failed");
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        ms_out = ms;
        return NBODY_OK;
    };
    double t = 0;
    int rc = time_once(cands[0], t);
    best = cands[0];
    for (size_t k = 0; rc == NBODY_OK && k < cands.size(); ++k) {
        double ms_min = 1e300;
        for (int rep = 0; rep < 2 && rc == NBODY_OK; ++rep) {
            rc = time_once(cands[k], t);
            ms_min = std::min(ms_min, t);
        }
        if (rc == NBODY_OK && ms_min < best_ms * (1.0 - kTuneMargin)) {
            best_ms = ms_min;
            best = cands[k];
        }
    }
    if (rc == NBODY_OK && !same_cfg(best, cands[0])) {
        double h = 1e300, w = 1e300;
        for (int rep = 0; rep < 3 && rc == NBODY_OK; ++rep) {
            rc = time_once(cands[0], t);
            h = std::min(h, t);
            if (rc == NBODY_OK) rc = time_once(best, t);
            w = std::min(w, t);
        }
        if (rc == NBODY_OK) {
            if (w < h * (1.0 - kTuneMargin)) {
                best_ms = w;
            } else {
                best = cands[0];
                best_ms = h;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_timing = saved_timing;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

std::vector<Cfg> candidate_set(int api, int law, int prec, int64_t n, bool pot)
{
    std::vector<Cfg> out;
    const int64_t npad = round_up(std::max<int64_t>(n, 1), 64);
    if (api == NBODY_API_BATCHED) {
        if (bsym_supported(law, prec)) {         // the symmetric tiles (taken when every system fits)
            Cfg c;
            c.j_stage = kSymStage;
            out.push_back(sanitize(c, api, law, prec, npad));
        }
        for (int js : {0, 1})
            for (int ipl : {1, 2})
                for (int b : {64, 128, 256})
                    for (int jt : {64, 256})
                        for (int upw : {kBatchUnitsPerWave, 4, 16}) {
                            if (js == 0 && !is_f32(prec) && ipl > 1) continue;
                            (void)law;
                            Cfg c;
                            c.ipl = ipl;
                            c.block = b;
                            c.j_tile = jt;
                            c.j_split = upw;
                            c.j_stage = js;
                            out.push_back(c);
                        }
        return out;
    }
    if (sym_eligible(api, law, prec) && npad <= kSymMaxN)
        for (int jt : {1024, 2048})            // the symmetric tiles, both block edges and shapes,
            for (int ipl : {2, 4})             // whole tiles or tiles in 2 or 4 j parts
                for (int sp : {1, 2, 4}) {
                    if (jt == 1024 && n > kSymSmallMax) continue;
                    Cfg c;
                    c.j_stage = kSymStage;
                    c.j_tile = jt;
                    c.ipl = ipl;
                    c.block = ipl == 4 ? 256 : kSymThreads;
                    c.j_split = sp;
                    c = sanitize(c, api, law, prec, npad);
                    if (c.j_split == sp) out.push_back(c);      // (parts not allowed here: skipped)
                }
    if (api == NBODY_API_JERK && symjerk_ok(law, prec) && npad <= kSymJerkMaxN)
        for (int sp : {1, 2}) {                 // the symmetric tiles, whole or in 2 j parts
            if (sp > symjerk_max_split(npad)) continue;
            Cfg c;
            c.j_stage = kSymStage;
            c.j_split = sp;
            out.push_back(sanitize(c, api, law, prec, npad));
        }
    const bool jerk = api == NBODY_API_JERK;
    for (int js : {0, 1})
        for (int ipl : {1, 2, 4, 8}) {
            if (ipl > max_ipl(api, prec) || (js == 1 && ipl > 4)) continue;
            if (jerk && ipl > 2) continue;
            if (law >= NBODY_LAW_LJC_CONSTANT && ipl > 2) continue;
            const int block = 256;
            std::vector<int> splits = ranked_splits(law, prec, n, n, ipl, pot, js, block, max_split(npad), jerk);
            std::vector<int> pick;
            for (int sp : splits) {
                if ((int)pick.size() >= 3) break;
                pick.push_back(sp);
            }
            if (std::find(pick.begin(), pick.end(), 1) == pick.end()) pick.push_back(1);
            if ((jerk || n <= (int64_t(1) << 18)) && !splits.empty())
                // the jerk kernel, and the forces kernels below a few hundred
                // thousand rows, gain from more, shorter waves than the model
                // predicts (the last round's imbalance shrinks; measured): also
                // try 2x and 4x its best split
                for (int f : {2, 4}) {
                    const int sp = std::min(splits[0] * f, max_split(npad));
                    if (std::find(pick.begin(), pick.end(), sp) == pick.end()) pick.push_back(sp);
                }
            for (int sp : pick) {
                Cfg c;
                c.ipl = ipl;
                c.block = block;
                c.j_tile = is_f32(prec) ? 256 : 1024;
                c.j_split = sp;
                c.j_stage = js;
                out.push_back(c);
            }
        }
    return out;
}

// The j split of the Hermite entry points' jerk evaluations, by the number of
// rows evaluated: entry w is for (w + 1) row waves (64 ipl rows each) against
// all n records.  The split_cost model's best over 1..64 and a geometric
// ladder above (the kernel keeps few registers per wave, so it runs best with
// every wave slot of the chip busy, and a due set of a few rows needs a split
// of hundreds to fill them), held to at least 128 records a j part and to
// what the partial buffer holds (max_split(npad) x npad rows); the entry for
// all n rows is therefore at most max_split(npad).  A forced configuration's
// split instead, held to the same bounds.  Built once per law, size, kernel
// shape and configuration state.
std::shared_ptr<const std::vector<int>> hermite_split_table(const nbody_law *law, int64_t n, const Cfg &c)
{
    using Key = std::tuple<int, int64_t, int, int, int, uint64_t>;
    static std::mutex mu;
    static std::vector<std::pair<Key, std::shared_ptr<const std::vector<int>>>> cache;   // most recent last
    uint64_t ver;
    int forced = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ver = g_cfg_version;
        if (g_override_set[NBODY_API_HERMITE]) forced = g_override[NBODY_API_HERMITE].j_split;
    }
    const Key key(law->precision, n, c.ipl, c.block, c.j_stage, ver);
    {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t k = 0; k < cache.size(); ++k)
            if (cache[k].first == key) {
                auto hit = cache[k];
                cache.erase(cache.begin() + (std::ptrdiff_t)k);
                cache.push_back(hit);
                return hit.second;
            }
    }
    const int64_t npad = round_up(n, 64), rpw = 64 * c.ipl;
    const int64_t cap = (int64_t)max_split(npad) * npad;
    const int64_t smax_all = std::max<int64_t>(1, std::min<int64_t>(npad / 128, 1 << 20));
    int64_t R = resident_waves_jerk(law->precision, c.ipl, false, c.j_stage, c.block);
    if (R <= 0) R = kTargetWaves;
    const double rate = nominal_rate(NBODY_LAW_GRAVITY, law->precision) * 0.5;
    std::vector<int64_t> ladder;
    for (int64_t s = 1; s <= smax_all; s = s < 64 ? s + 1 : (s * 9 + 7) / 8) ladder.push_back(s);
    auto t = std::make_shared<std::vector<int>>((size_t)((n + rpw - 1) / rpw));
    for (size_t w = 0; w < t->size(); ++w) {
        const int64_t rw = (int64_t)w + 1;
        const int64_t rows = std::min<int64_t>(n, rw * rpw);
        const int64_t smax = std::max<int64_t>(1, std::min(smax_all, cap / round_up(rows, 64)));
        int64_t best = 1;
        if (forced > 0) {
            best = std::min<int64_t>(forced, smax);
        } else {
            double best_t = 1e300;
            for (size_t k = 0; k <= ladder.size(); ++k) {
                const int64_t sp = k < ladder.size() ? ladder[k] : smax;   // and smax itself
                if (sp > smax) continue;
                const double tt = split_cost(rows, npad, rw, R, (int)sp, rate);
                if (tt < best_t) {
                    best_t = tt;
                    best = sp;
                }
            }
        }
        (*t)[w] = (int)best;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() >= 4) cache.erase(cache.begin());
    cache.push_back({key, t});
    return t;
}

bool power_of_two(double x)
{
    int e = 0;
    return x > 0.0 && std::isfinite(x) && std::frexp(x, &e) == 0.5;
}

}  // namespace

// ======================================================================== ABI

extern "C" {

const char *nbody_last_error(void) { return g_err.c_str(); }

const char *nbody_version(void) { return "nbody-mi355x 0.1 (gfx950)"; }

// ------------------------------------------------------------- probes ----
constexpr int kProbeIters = 16384;
constexpr int kProbeOutputs = 9;

// eight waves per SIMD: the rate a dense VGPR-only stream sustains depends on the
// waves a SIMD can alternate between (measured: 3.5 cycles per FMA at four waves,
// 2.5 to 2.8 at eight), so the probe runs at the occupancy of the pair kernels
static int probe_blocks() { return std::min(device_cus(), 4096) * 8; }

size_t nbody_probe_workspace_bytes(void) { return (size_t)probe_blocks() * 256 * sizeof(float) + 256; }

int nbody_probe_issue_rates(double *out, int32_t n_out, void *ws, size_t ws_bytes, void *stream)
{
    if (!out) return fail(NBODY_EINVAL, "out is NULL");
    if (n_out < kProbeOutputs) return fail(NBODY_EINVAL, "out holds %d values, %d needed", n_out, kProbeOutputs);
    const int blocks = probe_blocks();
    int rc = check_ws(ws, ws_bytes, nbody_probe_workspace_bytes());
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    float *o = (float *)ws;
    long long *clk = (long long *)((char *)ws + (size_t)blocks * 256 * sizeof(float));
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return fail(NBODY_EHIP, "event creation failed");
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(NBODY_EHIP, "event creation failed");
    }
    int dev = 0, rtc_khz = 0, max_khz = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&rtc_khz, hipDeviceAttributeWallClockRate, dev);
    (void)hipDeviceGetAttribute(&max_khz, hipDeviceAttributeClockRate, dev);
    const double simds = 4.0 * device_cus();
    // Per mode: warm-up launches (clocks settle), then three timed launches, each
    // at its own clock (shader cycles over wall ticks of its timing wave; the
    // device's maximum if unreadable); the median of the three is reported.
    static const int slot[kProbeModes] = {0, 1, 2, 5, 6, 7, 8};
    hipError_t e = hipSuccess;
    double clock0 = 0.0;
    for (int mode = 0; mode < kProbeModes && e == hipSuccess; ++mode) {
        const double instr = (double)blocks * 4.0 / simds * kProbeIters * probe_units_per_iter(mode);
        for (int w = 0; w < 4 && e == hipSuccess; ++w) e = launch_probe(mode, o, clk, blocks, kProbeIters, s);
        double cyc[3] = {0, 0, 0}, fr[3] = {0, 0, 0};
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
            e = hipEventRecord(a, s);
            if (e == hipSuccess) e = launch_probe(mode, o, clk, blocks, kProbeIters, s);
            if (e == hipSuccess) e = hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
            long long h[2] = {0, 0};
            if (e == hipSuccess) e = hipMemcpyAsync(h, clk, sizeof h, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            double f = (rtc_khz > 0 && h[1] > 0) ? (double)h[0] / ((double)h[1] / (rtc_khz * 1e3)) : 0.0;
            if (!(f > 1e8 && f < 1e10)) f = max_khz * 1e3;
            cyc[r] = t * 1e-3 * f / instr;
            fr[r] = f;
        }
        std::sort(cyc, cyc + 3);
        std::sort(fr, fr + 3);
        out[slot[mode]] = cyc[1];
        if (mode == 0) clock0 = fr[1];
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "issue-rate probe");
    out[3] = clock0 / 1e9;
    out[4] = rtc_khz / 1e3;
    return NBODY_OK;
}

size_t nbody_workspace_bytes(int32_t api, int64_t n_total, int64_t n_systems, const nbody_law *law)
{
    if (!law || n_total < 0 || n_systems < 0) return 0;
    if (law->kind < NBODY_LAW_GRAVITY || law->kind > NBODY_LAW_LJC_SIGMOIDAL) return 0;
    if (law->precision < NBODY_FP64 || law->precision > NBODY_FP32_PLAIN) return 0;
    switch (api) {
    case NBODY_API_FORCES: return fwd_layout(NBODY_API_FORCES, law, n_total).total;
    case NBODY_API_LEAPFROG: return fwd_layout(NBODY_API_LEAPFROG, law, n_total).total;
    case NBODY_API_BACKWARD: return adj_layout(law, n_total).total;
    case NBODY_API_BATCHED: return bat_layout(law, n_total, n_systems).total;
    case NBODY_API_BACKWARD_BATCHED: return adjb_layout(law, n_total, n_systems).total;
    case NBODY_API_JERK:
    case NBODY_API_HERMITE:
        if (law->kind != NBODY_LAW_GRAVITY) return 0;
        return jerk_layout(api, law, n_total).total;
    default: return 0;
    }
}

int nbody_forces(const double *pos, const double *params, int64_t n, const nbody_law *law,
                 double *out_force, double *out_potential, void *ws, size_t ws_bytes, void *stream)
{
    return forces_impl(pos, params, n, nullptr, n, law, out_force, out_potential, ws, ws_bytes,
                       stream, nullptr);
}

int nbody_forces_noalloc(const double *pos, const double *params, int64_t n, const nbody_law *law,
                         double *out_force, double *out_potential, void *stream)
{
    int rc = validate_law(law, false);
    if (rc) return rc;
    if (n < 0) return fail(NBODY_EINVAL, "n < 0");
    if (n == 0) return NBODY_OK;
    if (!pos || !params || !out_force) return fail(NBODY_EINVAL, "pos, params and out_force must be non-NULL");
    const int64_t npad = round_up(n, 64);
    const size_t rbytes = rec_bytes(law->kind, law->precision);
    if (n > (int64_t)(kScratchBytes / rbytes) - 64)
        return fail(NBODY_EINVAL,
                    "n = %lld exceeds the allocation-free entry point's limit of %lld particles for this "
                    "law and precision (%zu-byte records in a %zu-byte device scratch area); use "
                    "nbody_forces with a workspace",
                    (long long)n, (long long)(kScratchBytes / rbytes) - 64, rbytes, kScratchBytes);
    void *base = nullptr;
    hipError_t e = scratch_area(&base);
    if (e != hipSuccess) return hip_fail(e, "scratch area");
    const bool pot = out_potential != nullptr;
    Cfg c = sanitize(choose(NBODY_API_FORCES, law, n, 1, pot, n), NBODY_API_FORCES, law->kind,
                     law->precision, npad);
    if (c.j_stage == kSymStage) {
        // the symmetric tiles when their padded records and slot partials fit the area
        // (the chosen block edge, else the larger one, which needs fewer partials)
        // (the chosen block edge and j parts, else whole tiles, else the larger block edge,
        // which needs fewer partials)
        const int blk0 = c.j_tile / 64;
        const std::pair<int, int> tries[] = {{blk0, c.j_split}, {blk0, 1}, {32, 1}};
        for (const auto &bs : tries) {
            const int blk = bs.first;
            const size_t recs = align256((size_t)sym_npad(n, blk) * rbytes);
            if (recs + sym_partial_bytes(n, blk, bs.second) > kScratchBytes) continue;
            FwdWs lay{};
            lay.rec_off = 0;
            lay.part_off = recs;
            lay.scratch_off = lay.total = kScratchBytes;
            Cfg cb = c;
            cb.j_tile = blk * 64;
            cb.j_split = bs.second;
            return run_forward(law, cb, pos, params, n, nullptr, n, make_epi(law, out_force, out_potential),
                               pot, base, lay, (hipStream_t)stream, nullptr, ExclArgs{}, false);
        }
        c = sanitize(one_sided(c, NBODY_API_FORCES, law, n, n, pot), NBODY_API_FORCES, law->kind,
                     law->precision, npad);
    }
    // the records first, then the split partials of the chosen j split, as far as they fit
    FwdWs lay{};
    lay.rec_off = 0;
    lay.part_off = align256((size_t)npad * rbytes);
    lay.scratch_off = lay.total = kScratchBytes;
    const int64_t fit = (int64_t)((kScratchBytes - lay.part_off) / ((size_t)n * 4 * sizeof(double)));
    c.j_split = (int)std::max<int64_t>(1, std::min<int64_t>(c.j_split, fit));
    return run_forward(law, c, pos, params, n, nullptr, n, make_epi(law, out_force, out_potential), pot,
                       base, lay, (hipStream_t)stream, nullptr, ExclArgs{}, false);
}

int nbody_forces_subset(const double *pos, const double *params, int64_t n, const int64_t *ilist,
                        int64_t ni, const nbody_law *law, double *out_force, double *out_potential,
                        void *ws, size_t ws_bytes, void *stream)
{
    if (ni > 0 && !ilist) return fail(NBODY_EINVAL, "ilist is NULL");
    return forces_impl(pos, params, n, ilist, ni, law, out_force, out_potential, ws, ws_bytes,
                       stream, nullptr);
}

int nbody_forces_share(const double *pos, const double *params, int64_t n, const nbody_law *law, int32_t share,
                       int32_t n_shares, double *out_force, double *out_potential, void *ws, size_t ws_bytes,
                       void *stream)
{
    return share_impl(pos, params, n, law, share, n_shares, out_force, out_potential, ws, ws_bytes, stream);
}

int nbody_forces_batched(const int64_t *offsets, int64_t n_systems, const double *pos,
                         const double *params, const nbody_law *law, double *out_force,
                         double *out_potential, void *ws, size_t ws_bytes, void *stream)
{
    return batched_impl(offsets, n_systems, pos, params, law, out_force, out_potential, ws, ws_bytes,
                        stream, nullptr);
}

int backward_impl(const double *pos, const double *params, int64_t n, const nbody_law *law,
                  const double *grad_force, double *grad_pos, double *grad_params,
                  const int32_t *types, int32_t n_types, double *grad_type_params, void *ws,
                  size_t ws_bytes, void *stream, const nbody_exclusions *excl)
{
    int rc = validate_law(law, true);
    if (rc) return rc;
    rc = validate_excl(excl, law, true);
    if (rc) return rc;
    if (n < 0) return fail(NBODY_EINVAL, "n < 0");
    if (law->kind == NBODY_LAW_GRAVITY && (grad_params || types))
        return fail(NBODY_EINVAL, "gravity has no parameter adjoint here: grad_params/types must be NULL");
    if (types && (n_types <= 0 || !grad_type_params))
        return fail(NBODY_EINVAL, "types given without n_types > 0 and grad_type_params");
    if (types && n_types > kTypePartDoubles / 2)
        return fail(NBODY_ENOTSUP, "at most %lld types", (long long)(kTypePartDoubles / 2));
    if (types && !grad_params)
        return fail(NBODY_EINVAL, "the per-type reduction needs grad_params");
    if (n == 0) return NBODY_OK;
    if (!pos || !params || !grad_force) return fail(NBODY_EINVAL, "pos, params and grad_force must be non-NULL");
    if (!grad_pos && !grad_params) return NBODY_OK;
    const AdjWs lay = adj_layout(law, n);
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Cfg c = with_excl(sanitize(choose(NBODY_API_BACKWARD, law, n, 1, false), NBODY_API_BACKWARD, law->kind,
                               law->precision, round_up(n, 64)),
                      excl != nullptr);
    char *base = (char *)ws;
    if (c.j_stage == kSymStage && law->kind == NBODY_LAW_LJC_LINEAR) {
        // LJC(linear)'s adjoint over unordered pairs (the position terms of the two atoms are
        // opposite, the charge, sigma and epsilon terms share one scalar): the batched adjoint's
        // tiles over the one system, then the per-type sums as below
        const int64_t spad = round_up(n, kBSymRecords);
        AdjPackLaunch pk{};
        pk.law = law->kind;
        pk.prec = law->precision;
        pk.n = n;
        pk.npad = spad;
        pk.pos = pos;
        pk.params = params;
        pk.g = grad_force;
        pk.qscale = qscale_of(law);
        pk.rec = base + lay.rec_off;
        hipError_t e = launch_pack_adjoint(pk, s);
        if (e != hipSuccess) return hip_fail(e, "adjoint pack");
        BSymAdjLaunch b{};
        b.law = law->kind;
        b.prec = law->precision;
        b.n_systems = 1;
        b.single_n = n;
        b.single_npad = spad;
        b.G = law->G;
        b.qscale = qscale_of(law);
        b.rec = base + lay.rec_off;
        b.partial = (float4 *)(base + lay.part_off);
        b.params = params;
        b.grad_pos = grad_pos;
        b.grad_params = grad_params;
        Timer t(s);
        e = launch_bsym_adj(b, s);
        t.stop();
        if (e != hipSuccess) return hip_fail(e, "symmetric LJC adjoint tiles");
        e = launch_bsym_adj_reduce(b, s);
        if (e != hipSuccess) return hip_fail(e, "symmetric LJC adjoint reduction");
        if (types) {
            e = launch_type_reduce(grad_params, types, n, n_types, grad_type_params,
                                   (double *)(base + lay.type_off), kTypePartDoubles, s);
            if (e != hipSuccess) return hip_fail(e, "per-type reduction");
        }
        return NBODY_OK;
    }
    if (c.j_stage == kSymStage) {
        // gravity's position adjoint over unordered pairs: the pair's term for k is minus its
        // term for j (swapping the two negates both w and d), so each pair is evaluated once
        const int blk = c.j_tile / 64;
        const int64_t spad = sym_npad(n, blk);
        AdjPackLaunch pk{};
        pk.law = law->kind;
        pk.prec = law->precision;
        pk.n = n;
        pk.npad = spad;
        pk.pos = pos;
        pk.params = params;
        pk.g = grad_force;
        pk.rec = base + lay.rec_off;
        hipError_t e = launch_pack_adjoint(pk, s);
        if (e != hipSuccess) return hip_fail(e, "adjoint pack");
        SymLaunch a{};
        a.op = SYM_HVP;
        a.prec = law->precision;
        a.pot = 0;
        a.blk = blk;
        a.ich = c.ipl;
        a.split = c.j_split;
        a.nblk = spad / ((int64_t)blk * 64);
        a.npad = spad;
        a.n = n;
        a.eps2 = law->softening * law->softening;
        a.rec = base + lay.rec_off;
        a.partial = (float4 *)(base + lay.part_off);
        sym_share_range(a.nblk, 0, 1, a.t0, a.count);
        a.epi.fscale = law->G;
        a.epi.out_force = grad_pos;
        Timer t(s);
        e = launch_sym(a, s);
        t.stop();
        if (e != hipSuccess) return hip_fail(e, "symmetric adjoint kernel");
        e = launch_sym_reduce(a, s);
        if (e != hipSuccess) return hip_fail(e, "symmetric adjoint reduction");
        return NBODY_OK;
    }
    const int64_t npad = round_up(n, 64);

    AdjPackLaunch pk{};
    pk.law = law->kind;
    pk.prec = law->precision;
    pk.n = n;
    pk.npad = npad;
    pk.pos = pos;
    pk.params = params;
    pk.g = grad_force;
    pk.qscale = qscale_of(law);
    pk.rec = base + lay.rec_off;
    hipError_t e = launch_pack_adjoint(pk, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint pack");

    AdjLaunch a{};
    a.law = law->kind;
    a.prec = law->precision;
    a.ipl = std::min(c.ipl, 4);
    a.block = c.block;
    a.j_stage = c.j_stage;
    a.n = n;
    a.npad = npad;
    a.j_split = std::max(1, std::min(c.j_split, max_split(npad)));
    a.split_len = round_up((npad + a.j_split - 1) / a.j_split, 64);
    a.j_tile = c.j_tile;
    a.eps2 = law->kind == NBODY_LAW_GRAVITY ? law->softening * law->softening : 0.0;
    a.G = law->G;
    a.qscale = qscale_of(law);
    a.rec = base + lay.rec_off;
    a.partial = (double *)(base + lay.part_off);
    a.grad_pos = grad_pos;
    a.grad_params = grad_params;
    a.params = params;
    a.excl = excl_args(excl);
    Timer t(s);
    e = launch_adjoint(a, s);
    t.stop();
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel");
    e = launch_adjoint_reduce(a, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint split reduction");
    if (types) {
        e = launch_type_reduce(grad_params, types, n, n_types, grad_type_params,
                               (double *)(base + lay.type_off), kTypePartDoubles, s);
        if (e != hipSuccess) return hip_fail(e, "per-type reduction");
    }
    return NBODY_OK;
}

int nbody_forces_backward(const double *pos, const double *params, int64_t n, const nbody_law *law,
                          const double *grad_force, double *grad_pos, double *grad_params,
                          const int32_t *types, int32_t n_types, double *grad_type_params,
                          void *ws, size_t ws_bytes, void *stream)
{
    return backward_impl(pos, params, n, law, grad_force, grad_pos, grad_params, types, n_types,
                         grad_type_params, ws, ws_bytes, stream, nullptr);
}

int nbody_forces_backward_excl(const double *pos, const double *params, int64_t n,
                               const nbody_exclusions *excl, const nbody_law *law,
                               const double *grad_force, double *grad_pos, double *grad_params,
                               const int32_t *types, int32_t n_types, double *grad_type_params,
                               void *ws, size_t ws_bytes, void *stream)
{
    if (!excl) return fail(NBODY_EINVAL, "excl is NULL");
    return backward_impl(pos, params, n, law, grad_force, grad_pos, grad_params, types, n_types,
                         grad_type_params, ws, ws_bytes, stream, excl);
}

int nbody_forces_excl(const double *pos, const double *params, int64_t n,
                      const nbody_exclusions *excl, const nbody_law *law, double *out_force,
                      double *out_potential, void *ws, size_t ws_bytes, void *stream)
{
    if (!excl) return fail(NBODY_EINVAL, "excl is NULL");
    return forces_impl(pos, params, n, nullptr, n, law, out_force, out_potential, ws, ws_bytes,
                       stream, nullptr, excl);
}

int nbody_forces_batched_excl(const int64_t *offsets, int64_t n_systems, const double *pos,
                              const double *params, const nbody_exclusions *excl,
                              const nbody_law *law, double *out_force, double *out_potential,
                              void *ws, size_t ws_bytes, void *stream)
{
    if (!excl) return fail(NBODY_EINVAL, "excl is NULL");
    return batched_impl(offsets, n_systems, pos, params, law, out_force, out_potential, ws,
                        ws_bytes, stream, nullptr, excl);
}

namespace {

// whether the adjoint's symmetric tiles take this ensemble: law and precision, no exclusion
// lists, and every system within kBSymMaxSystem
bool bsym_adj_takes(const nbody_law *law, const int64_t *offsets, int64_t S, bool excl)
{
    if (excl || !law_has_bsym_adj(law)) return false;
    for (int64_t s = 0; s < S; ++s)
        if (offsets[s + 1] - offsets[s] > kBSymMaxSystem) return false;
    return true;
}

// pack (systems padded to blocks of 256) + symmetric adjoint tiles + slot-ordered reduction
int run_bsym_adj(const nbody_law *law, const int64_t *offsets, int64_t S, const double *pos,
                 const double *params, const double *grad_force, double *grad_pos, double *grad_params,
                 void *ws, const AdjBatWs &lay, hipStream_t s)
{
    std::shared_ptr<const BatchPlan> pp = cached_plan(offsets, S, kBSymPlanKey, 0);
    const BatchPlan &plan = *pp;
    if (plan.units.empty()) return NBODY_OK;
    const int nv = (bsym_adj_sums(law->kind) + 3) / 4;
    if ((int64_t)plan.units.size() / 4 > lay.max_units || plan.npad_total > lay.max_records ||
        (size_t)plan.n_slots * (size_t)nv * 4 * sizeof(float) > lay.part_bytes ||
        (int64_t)plan.red.size() / 2 > red_capacity(offsets[S], S))
        return fail(NBODY_EWORKSPACE, "internal: batched symmetric adjoint plan exceeds its workspace regions "
                    "(%lld tiles, %lld slot rows)", (long long)(plan.units.size() / 4), (long long)plan.n_slots);
    char *base = (char *)ws;
    DevTables tab;
    int rc = batched_tables(plan, offsets, S, kBSymPlanKey, 0, s, base, lay.unit_off, lay.off_off, lay.poff_off,
                            lay.systab_off, lay.red_off, &tab);
    if (rc) return rc;
    AdjBatchLaunch pk{};
    pk.law = law->kind;
    pk.prec = law->precision;
    pk.n_systems = S;
    pk.npad_total = plan.npad_total;
    pk.off = tab.off;
    pk.poff = tab.poff;
    pk.pos = pos;
    pk.params = params;
    pk.g = grad_force;
    pk.qscale = qscale_of(law);
    pk.rec = base + lay.rec_off;
    pk.ticket_zeroed = 0;                      // no work ticket: one wave per listed tile
    hipError_t e = launch_pack_adjoint_batched(pk, s);
    if (e != hipSuccess) return hip_fail(e, "batched adjoint pack");
    BSymAdjLaunch a{};
    a.law = law->kind;
    a.prec = law->precision;
    a.n_units = (int64_t)plan.units.size() / 4;
    a.units = tab.units;
    a.off = tab.off;
    a.poff = tab.poff;
    a.systab = tab.systab;
    a.red = tab.red;
    a.n_red = (int64_t)plan.red.size() / 2;
    a.n_systems = S;
    a.eps2 = law->kind == NBODY_LAW_GRAVITY ? law->softening * law->softening : 0.0;
    a.G = law->G;
    a.qscale = qscale_of(law);
    a.rec = base + lay.rec_off;
    a.partial = (float4 *)(base + lay.part_off);
    a.params = params;
    a.grad_pos = grad_pos;
    a.grad_params = grad_params;
    Timer t(s);
    e = launch_bsym_adj(a, s);
    t.stop();
    if (e != hipSuccess) return hip_fail(e, "batched symmetric adjoint kernel");
    e = launch_bsym_adj_reduce(a, s);
    if (e != hipSuccess) return hip_fail(e, "batched symmetric adjoint reduction");
    return NBODY_OK;
}

}  // namespace

int nbody_forces_backward_batched(const int64_t *offsets, int64_t n_systems, const double *pos,
                                  const double *params, const nbody_exclusions *excl,
                                  const nbody_law *law, const double *grad_force, double *grad_pos,
                                  double *grad_params, const int32_t *types, int32_t n_types,
                                  double *grad_type_params, void *ws, size_t ws_bytes, void *stream)
{
    int rc = validate_law(law, true);
    if (rc) return rc;
    rc = validate_excl(excl, law, true);
    if (rc) return rc;
    rc = validate_offsets(offsets, n_systems);
    if (rc) return rc;
    if (law->kind == NBODY_LAW_GRAVITY && (grad_params || types))
        return fail(NBODY_EINVAL, "gravity has no parameter adjoint here: grad_params/types must be NULL");
    if (types && (n_types <= 0 || !grad_type_params))
        return fail(NBODY_EINVAL, "types given without n_types > 0 and grad_type_params");
    if (types && n_types > kTypePartDoubles / 2)
        return fail(NBODY_ENOTSUP, "at most %lld types", (long long)(kTypePartDoubles / 2));
    if (types && !grad_params) return fail(NBODY_EINVAL, "the per-type reduction needs grad_params");
    const int64_t n = offsets[n_systems];
    if (n == 0) return NBODY_OK;
    if (!pos || !params || !grad_force) return fail(NBODY_EINVAL, "pos, params and grad_force must be non-NULL");
    if (!grad_pos && !grad_params) return NBODY_OK;
    const AdjBatWs lay = adjb_layout(law, n, n_systems);
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Cfg c = choose(NBODY_API_BACKWARD_BATCHED, law, n, n_systems, false);
    if (c.j_stage == kSymStage) {
        if (bsym_adj_takes(law, offsets, n_systems, excl != nullptr)) {
            rc = run_bsym_adj(law, offsets, n_systems, pos, params, grad_force, grad_pos, grad_params, ws, lay, s);
            if (rc) return rc;
            if (types) {
                const hipError_t e = launch_type_reduce(grad_params, types, n, n_types, grad_type_params,
                                                        (double *)((char *)ws + lay.type_off), kTypePartDoubles, s);
                if (e != hipSuccess) return hip_fail(e, "per-type reduction");
            }
            return NBODY_OK;
        }
        // a system above the tiles' size, or exclusion lists: the rule's one-sided configuration
        c = heuristic(NBODY_API_BACKWARD_BATCHED, law->kind, law->precision, n, n, n_systems, false, false);
    }
    c = with_excl(c, excl != nullptr);
    const int ipl = std::min(c.ipl, 2);
    AdjBatchLaunch a{};
    a.law = law->kind;
    a.prec = law->precision;
    a.ipl = ipl;
    a.block = c.block;
    a.j_stage = c.j_stage;
    a.excl = excl_args(excl);
    int per_cu = 0;
    {
        using Key = std::tuple<int, int, int, int, int, int>;
        static std::map<Key, int> cache;
        static std::mutex mu;
        const Key key(a.law, a.prec, a.ipl, a.block, a.j_stage, a.excl.off != nullptr ? 1 : 0);
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        per_cu = it != cache.end() ? it->second : (cache[key] = adjoint_batched_blocks_per_cu(a));
        per_cu = std::max(1, per_cu);
    }
    const int64_t resident = (int64_t)device_cus() * per_cu * (c.block / 64);
    const PlanChoice pc = plan_for_launch(offsets, n_systems, ipl, resident, lay.max_slots, c.j_split);
    const BatchPlan &plan = *pc.plan;
    if (plan.units.empty()) return NBODY_OK;
    if (!plan_fits(plan, ipl, lay.max_units, lay.max_records, lay.max_slots, red_capacity(n, n_systems)))
        return fail(NBODY_EWORKSPACE, "internal: batched adjoint plan exceeds its workspace regions");
    char *base = (char *)ws;
    DevTables tab;
    rc = batched_tables(plan, offsets, n_systems, ipl, pc.j_unit, s, base, lay.unit_off, lay.off_off,
                        lay.poff_off, lay.systab_off, lay.red_off, &tab);
    if (rc) return rc;
    int32_t *d_units = tab.units;
    int64_t *d_off = tab.off;
    int64_t *d_poff = tab.poff;
    int64_t *d_systab = tab.systab;
    hipError_t e;
    a.j_tile = c.j_tile;
    a.n_units = (int64_t)plan.units.size() / 4;
    a.units = d_units;
    a.off = d_off;
    a.poff = d_poff;
    a.n_systems = n_systems;
    a.npad_total = plan.npad_total;
    a.n_total = n;
    a.systab = d_systab;
    a.partial = (double *)(base + lay.part_off);
    a.any_parts = plan.n_slots > 0;
    a.red = tab.red;
    a.n_red = (int64_t)plan.red.size() / 2;
    a.eps2 = law->kind == NBODY_LAW_GRAVITY ? law->softening * law->softening : 0.0;
    a.G = law->G;
    a.qscale = qscale_of(law);
    a.pos = pos;
    a.params = params;
    a.g = grad_force;
    a.rec = base + lay.rec_off;
    a.ticket = (int *)(base + lay.ticket_off);
    a.ticket_zeroed = 1;
    a.grad_pos = grad_pos;
    a.grad_params = grad_params;
    e = launch_pack_adjoint_batched(a, s);
    if (e != hipSuccess) return hip_fail(e, "batched adjoint pack");
    const int64_t blocks_needed = (a.n_units + c.block / 64 - 1) / (c.block / 64);
    a.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)device_cus() * per_cu, blocks_needed));
    Timer t(s);
    e = launch_adjoint_batched(a, s);
    t.stop();
    if (e != hipSuccess) return hip_fail(e, "batched adjoint kernel");
    if (types) {
        e = launch_type_reduce(grad_params, types, n, n_types, grad_type_params,
                               (double *)(base + lay.type_off), kTypePartDoubles, s);
        if (e != hipSuccess) return hip_fail(e, "per-type reduction");
    }
    return NBODY_OK;
}

int leapfrog_step(double *pos, double *vel, double *acc, const double *params,
                  const double *inv_mass, int64_t n, const nbody_law *law, double dt,
                  int32_t nsteps, double *out_potential, void *ws, size_t ws_bytes, void *stream)
{
    int rc = validate_law(law, false);
    if (rc) return rc;
    if (n < 0) return fail(NBODY_EINVAL, "n < 0");
    if (nsteps < 0) return fail(NBODY_EINVAL, "nsteps < 0");
    if (!std::isfinite(dt)) return fail(NBODY_EINVAL, "dt must be finite");
    if (n == 0) return NBODY_OK;
    if (!pos || !vel || !acc || !params) return fail(NBODY_EINVAL, "pos, vel, acc and params must be non-NULL");
    if (nsteps == 0 && !out_potential) return NBODY_OK;
    const FwdWs lay = fwd_layout(NBODY_API_LEAPFROG, law, n);
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    if (nsteps == 0) {
        const Cfg c = choose(NBODY_API_LEAPFROG, law, n, 1, true);
        return run_forward(law, c, pos, params, n, nullptr, n,
                           make_epi(law, (double *)(base + lay.scratch_off), out_potential), true, ws,
                           lay, s, nullptr);
    }
    for (int32_t k = 0; k < nsteps; ++k) {
        const bool last = (k == nsteps - 1);
        const bool pot = last && out_potential;
        const Cfg c = choose(NBODY_API_LEAPFROG, law, n, 1, pot);
        PackLaunch pk{};
        pk.pos = pos;
        pk.kick_drift = 1;
        pk.vel = vel;
        pk.acc = acc;
        pk.half_dt = 0.5 * dt;
        pk.dt = dt;
        Epilogue epi = make_epi(law, acc, pot ? out_potential : nullptr);
        epi.kick = 1;
        epi.half_dt = 0.5 * dt;
        epi.vel = vel;
        epi.inv_mass = inv_mass;
        rc = run_forward(law, c, pos, params, n, nullptr, n, epi, pot, ws, lay, s, &pk);
        if (rc) return rc;
    }
    return NBODY_OK;
}

int nbody_forces_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                      const int64_t *ilist, int64_t ni, const nbody_law *law, double *out_acc,
                      double *out_jerk, double *out_potential, void *ws, size_t ws_bytes,
                      void *stream)
{
    return jerk_impl(pos, vel, mass, n, ilist, ni, law, out_acc, out_jerk, out_potential, ws,
                     ws_bytes, stream, nullptr);
}

int hermite_step(double *pos, double *vel, double *acc, double *jerk, const double *mass,
                 int64_t n, const nbody_law *law, double dt, int32_t nsteps, void *ws,
                 size_t ws_bytes, void *stream)
{
    int rc = validate_jerk_law(law);
    if (rc) return rc;
    if (n < 0 || nsteps < 0) return fail(NBODY_EINVAL, "n < 0 or nsteps < 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NBODY_EINVAL, "dt must be finite and > 0");
    if (n == 0 || nsteps == 0) return NBODY_OK;
    if (!pos || !vel || !acc || !jerk || !mass)
        return fail(NBODY_EINVAL, "pos, vel, acc, jerk and mass must be non-NULL");
    const JerkWs lay = jerk_layout(NBODY_API_HERMITE, law, n);
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    double *a1 = (double *)(base + lay.a1_off), *j1 = (double *)(base + lay.j1_off);
    Cfg c = sanitize(choose(NBODY_API_HERMITE, law, n, 1, false, n), NBODY_API_HERMITE, law->kind,
                     law->precision, round_up(n, 64));
    c.j_split = hermite_split_table(law, n, c)->back();   // the block steps' rule for all n rows
    // a shared step evaluates every row: the symmetric tiles where the acceleration-and-jerk
    // entry point's configuration for the whole system selects them
    const Cfg cj = sanitize(choose(NBODY_API_JERK, law, n, 1, false, n), NBODY_API_JERK, law->kind,
                            law->precision, round_up(n, 64));
    if (cj.j_stage == kSymStage) c = cj;
    for (int32_t k = 0; k < nsteps; ++k) {
        JerkPackLaunch pk{};
        pk.n = n;
        pk.pos = pos;
        pk.vel = vel;
        pk.mass = mass;
        pk.predict = 1;
        pk.acc = acc;
        pk.jerk = jerk;
        pk.tau = dt;
        rc = run_jerk(law, c, pk, nullptr, n, a1, j1, nullptr, ws, lay, s);
        if (rc) return rc;
        HermiteLaunch h{};
        h.nrows = n;
        h.pos = pos;
        h.vel = vel;
        h.acc = acc;
        h.jerk = jerk;
        h.a1 = a1;
        h.j1 = j1;
        h.h = dt;
        hipError_t e = launch_hermite_correct(h, s);
        if (e != hipSuccess) return hip_fail(e, "Hermite corrector");
    }
    return NBODY_OK;
}

int hermite_block_init(const double *acc, const double *jerk, int64_t n, double eta_s, double dt_max,
                       double *t_i, double *dt_i, void *stream)
{
    if (n < 0) return fail(NBODY_EINVAL, "n < 0");
    if (!(eta_s > 0.0) || !std::isfinite(eta_s)) return fail(NBODY_EINVAL, "eta_s must be finite and > 0");
    if (!power_of_two(dt_max)) return fail(NBODY_EINVAL, "dt_max must be a power of two");
    if (n == 0) return NBODY_OK;
    if (!acc || !jerk || !t_i || !dt_i) return fail(NBODY_EINVAL, "acc, jerk, t_i and dt_i must be non-NULL");
    hipError_t e = launch_block_init(acc, jerk, n, eta_s, dt_max, t_i, dt_i, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "block-step initialisation");
    return NBODY_OK;
}

int hermite_block_steps(double *pos, double *vel, double *acc, double *jerk, double *t_i,
                        double *dt_i, const double *mass, int64_t n, const nbody_law *law,
                        double eta, double dt_max, double t_end, int32_t nblocks,
                        int64_t *active_counts, double *t_now, void *ws, size_t ws_bytes, void *stream)
{
    int rc = validate_jerk_law(law);
    if (rc) return rc;
    if (n < 0 || nblocks < 0) return fail(NBODY_EINVAL, "n < 0 or nblocks < 0");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(NBODY_EINVAL, "eta must be finite and > 0");
    if (!power_of_two(dt_max)) return fail(NBODY_EINVAL, "dt_max must be a power of two");
    if (std::isnan(t_end)) return fail(NBODY_EINVAL, "t_end is NaN");
    if (n == 0 || nblocks == 0) return NBODY_OK;
    if (!pos || !vel || !acc || !jerk || !t_i || !dt_i || !mass)
        return fail(NBODY_EINVAL, "pos, vel, acc, jerk, t_i, dt_i and mass must be non-NULL");
    const JerkWs lay = jerk_layout(NBODY_API_HERMITE, law, n);
    rc = check_ws(ws, ws_bytes, lay.total);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    const int64_t npad = round_up(n, 64);
    // one kernel shape for every block step; the split follows the due count
    const Cfg c = sanitize(choose(NBODY_API_HERMITE, law, n, 1, false, n), NBODY_API_HERMITE, law->kind,
                           law->precision, npad);
    const int rpw = 64 * c.ipl;
    const std::shared_ptr<const std::vector<int>> table = hermite_split_table(law, n, c);
    // launch sizes covering every entry: jerk waves (row waves x split) and the
    // corrector's threads (rows x lanes per row of the split sum)
    int64_t grid_waves = 0, corr_threads = n, smax = 1;
    for (size_t w = 0; w < table->size(); ++w) {
        const int64_t sp = (*table)[w], rows = std::min<int64_t>(n, (int64_t)(w + 1) * rpw);
        grid_waves = std::max(grid_waves, (int64_t)(w + 1) * sp);
        if (sp > 1) corr_threads = std::max(corr_threads, rows * split_group(sp));
        smax = std::max(smax, sp);
    }
    const int64_t cap_rows = (int64_t)max_split(npad) * npad;
    int *dtable = (int *)(base + lay.table_off);
    hipError_t e = hipMemcpyAsync(dtable, table->data(), table->size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "split table upload");

    BlockState *st = (BlockState *)(base + lay.out_off);
    int64_t *clog = (int64_t *)(base + lay.log_off);
    double *tlog = (double *)(clog + kBlockLog);
    int64_t *list = (int64_t *)(base + lay.list_off);
    double *a1 = (double *)(base + lay.a1_off), *j1 = (double *)(base + lay.j1_off);

    SchedLaunch sl{};
    sl.n = n;
    sl.nb = (int)std::min<int64_t>(kSchedBlocks, (n + 255) / 256);
    sl.chunk = (n + sl.nb - 1) / sl.nb;
    sl.t_i = t_i;
    sl.dt_i = dt_i;
    sl.part_min = (double *)(base + lay.pmin_off);
    sl.part_cnt = (int64_t *)(base + lay.pcnt_off);
    sl.list = list;
    sl.state = st;
    sl.t_end = t_end;
    sl.split_table = dtable;
    sl.table_len = (int64_t)table->size();
    sl.rows_per_wave = rpw;
    sl.count_log = clog;
    sl.time_log = tlog;
    sl.fuse_pack = 1;

    JerkPackLaunch pk{};
    pk.prec = law->precision;
    pk.n = n;
    pk.npad = npad;
    pk.pos = pos;
    pk.vel = vel;
    pk.mass = mass;
    pk.predict = 1;
    pk.acc = acc;
    pk.jerk = jerk;
    pk.t_i = t_i;
    pk.t_pred_dev = &st->t;
    pk.live_dev = &st->count;
    pk.rec = base + lay.rec_off;
    sl.pack = pk;

    JerkLaunch a{};
    a.prec = law->precision;
    a.ipl = c.ipl;
    a.pot = 0;
    a.block = c.block;
    a.j_stage = c.j_stage;
    a.npad = npad;
    a.nrows = n;
    a.nrows_dev = &st->count;
    a.rows = list;
    a.j_split = (int)smax;
    a.split_dev = &st->split;
    a.grid_waves = grid_waves;
    a.partial_rows = cap_rows;
    a.j_tile = c.j_tile;
    a.eps2 = law->softening * law->softening;
    a.G = law->G;
    a.rec = base + lay.rec_off;
    a.partial = (double *)(base + lay.part_off);
    a.out_acc = a1;
    a.out_jerk = j1;
    a.out_pot = nullptr;

    HermiteLaunch h{};
    h.nrows = n;
    h.nrows_dev = &st->count;
    h.rows = list;
    h.pos = pos;
    h.vel = vel;
    h.acc = acc;
    h.jerk = jerk;
    h.a1 = a1;
    h.j1 = j1;
    h.t_i = t_i;
    h.dt_i = dt_i;
    h.t_next = &st->t;
    h.eta = eta;
    h.dt_max = dt_max;
    h.partial = a.partial;        // the split sum is done by the corrector
    h.split_dev = &st->split;
    h.split_max = smax;
    h.grid_threads = corr_threads;
    h.partial_rows = cap_rows;
    h.Gc = law->G;

    // Enqueue batches of block steps and read their due counts back after each
    // batch; a step that is not taken ends the call.  Batches double from 8 up
    // to kBlockLog; with a finite t_end, once two step times are known, a batch
    // is also held to a quarter more than the steps the rate so far predicts
    // before t_end (steps past t_end cost their launches).
    std::vector<int64_t> cnt;
    std::vector<double> tim;
    int32_t done = 0, taken = 0;
    int64_t batch = 8;
    double t_first = 0.0, t_last = 0.0;
    bool ended = false;
    while (done < nblocks && !ended) {
        const int64_t nb = std::min<int64_t>(batch, (int64_t)nblocks - done);
        for (int64_t k = 0; k < nb; ++k) {
            sl.log_index = k;
            e = launch_schedule(sl, s);      // due list, split and predicted records
            if (e != hipSuccess) return hip_fail(e, "block scheduling");
            Timer tm(s);
            e = launch_jerk(a, s);
            tm.stop();
            if (e != hipSuccess) return hip_fail(e, "jerk kernel");
            e = launch_hermite_correct(h, s);   // split sum + corrector
            if (e != hipSuccess) return hip_fail(e, "Hermite corrector");
        }
        cnt.resize((size_t)nb);
        tim.resize((size_t)nb);
        e = hipMemcpyAsync(cnt.data(), clog, (size_t)nb * sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(tim.data(), tlog, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "block-step read-back");
        for (int64_t k = 0; k < nb; ++k) {
            const int64_t na = cnt[(size_t)k];
            // a step with nothing due must be one past t_end
            if (na < 0 || na > n || (na > 0 && (ended || !std::isfinite(tim[(size_t)k]))) ||
                (na == 0 && tim[(size_t)k] <= t_end))
                return fail(NBODY_EHIP, "block scheduling produced an invalid due set (%lld)", (long long)na);
            if (active_counts) active_counts[done + k] = na;
            if (na == 0) {
                ended = true;
            } else {
                if (taken++ == 0) t_first = tim[(size_t)k];
                t_last = tim[(size_t)k];
                if (t_now) *t_now = t_last;
            }
        }
        done += (int32_t)nb;
        batch = std::min<int64_t>(2 * batch, kBlockLog);
        if (std::isfinite(t_end) && taken >= 2 && t_last > t_first) {
            const double est = (double)(taken - 1) * (t_end - t_last) / (t_last - t_first);
            batch = std::max<int64_t>(1, (int64_t)std::min<double>((double)batch, std::ceil(1.25 * est) + 1.0));
        }
    }
    if (active_counts)
        for (int32_t b = done; b < nblocks; ++b) active_counts[b] = 0;
    return NBODY_OK;
}

int nbody_autotune_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                        const nbody_law *law, double *out_acc, double *out_jerk,
                        double *out_potential, void *ws, size_t ws_bytes, void *stream,
                        nbody_config *out_best, double *out_ms)
{
    int rc = validate_jerk_law(law);
    if (rc) return rc;
    if (n <= 0) return fail(NBODY_EINVAL, "nothing to tune");
    tune_cache_load_once();
    Cfg best;
    double best_ms = 1e300;
    rc = tune_sweep(candidates(NBODY_API_JERK, law->kind, law->precision, n, out_potential != nullptr),
                    (hipStream_t)stream,
                    [&](const Cfg &c) {
                        return jerk_impl(pos, vel, mass, n, nullptr, n, law, out_acc, out_jerk,
                                         out_potential, ws, ws_bytes, stream, &c);
                    },
                    best, best_ms);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[TuneKey(NBODY_API_JERK, law->kind, law->precision, out_potential ? 1 : 0,
                        size_bucket(n), tune_sbucket(NBODY_API_JERK, 1, n))] = {best, best_ms};
        ++g_cfg_version;
    }
    tune_cache_store();
    rc = jerk_impl(pos, vel, mass, n, nullptr, n, law, out_acc, out_jerk, out_potential, ws, ws_bytes,
                   stream, &best);
    if (rc) return rc;
    if (out_best) to_abi(best, out_best);
    if (out_ms) *out_ms = best_ms;
    return NBODY_OK;
}

int nbody_set_config(int32_t api, const nbody_config *cfg)
{
    if (api < 0 || api >= kNumApi) return fail(NBODY_EINVAL, "unknown api %d", api);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!cfg) {
        g_override_set[api] = false;
        ++g_cfg_version;
        return NBODY_OK;
    }
    if (!cfg_valid(cfg)) return fail(NBODY_EINVAL, "configuration outside the documented ranges");
    g_override[api] = from_abi(cfg);
    g_override_set[api] = true;
    ++g_cfg_version;
    return NBODY_OK;
}

int nbody_get_config(int32_t api, int64_t n, int64_t n_systems, const nbody_law *law, nbody_config *out)
{
    if (api < 0 || api >= kNumApi) return fail(NBODY_EINVAL, "unknown api %d", api);
    int rc = validate_law(law, false);
    if (rc) return rc;
    if (!out || n < 0) return fail(NBODY_EINVAL, "bad arguments");
    if (api == NBODY_API_HERMITE && n > 0 && law->kind == NBODY_LAW_GRAVITY &&
        law->precision != NBODY_FP32_PLAIN) {
        // the Hermite steps' kernel shape with their split rule for all n rows
        Cfg c = sanitize(choose(api, law, n, 1, false, n), api, law->kind, law->precision, round_up(n, 64));
        c.j_split = hermite_split_table(law, n, c)->back();
        to_abi(c, out);
        return NBODY_OK;
    }
    to_abi(choose(api, law, n, std::max<int64_t>(n_systems, 1), true), out);
    return NBODY_OK;
}

int nbody_autotune(int32_t api, const int64_t *offsets, int64_t n_systems, const double *pos,
                   const double *params, int64_t n, const nbody_law *law, double *out_force,
                   double *out_potential, void *ws, size_t ws_bytes, void *stream,
                   nbody_config *out_best, double *out_ms)
{
    if (api != NBODY_API_FORCES && api != NBODY_API_BATCHED)
        return fail(NBODY_ENOTSUP, "autotune covers the forces and batched entry points");
    int rc = validate_law(law, false);
    if (rc) return rc;
    int64_t ntot = n, S = 1;
    if (api == NBODY_API_BATCHED) {
        rc = validate_offsets(offsets, n_systems);
        if (rc) return rc;
        ntot = offsets[n_systems];
        S = n_systems;
    }
    if (ntot <= 0) return fail(NBODY_EINVAL, "nothing to tune");
    tune_cache_load_once();
    Cfg best;
    double best_ms = 1e300;
    rc = tune_sweep(candidates(api, law->kind, law->precision, ntot, out_potential != nullptr),
                    (hipStream_t)stream,
                    [&](const Cfg &c) {
                        return api == NBODY_API_FORCES
                                   ? forces_impl(pos, params, n, nullptr, n, law, out_force,
                                                 out_potential, ws, ws_bytes, stream, &c)
                                   : batched_impl(offsets, n_systems, pos, params, law, out_force,
                                                  out_potential, ws, ws_bytes, stream, &c);
                    },
                    best, best_ms);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[TuneKey(api, law->kind, law->precision, out_potential ? 1 : 0, size_bucket(ntot),
                        tune_sbucket(api, S, ntot))] = {best, best_ms};
        ++g_cfg_version;
    }
    tune_cache_store();
    // leave the winner's result in the outputs
    rc = api == NBODY_API_FORCES
             ? forces_impl(pos, params, n, nullptr, n, law, out_force, out_potential, ws, ws_bytes,
                           stream, &best)
             : batched_impl(offsets, n_systems, pos, params, law, out_force, out_potential, ws,
                            ws_bytes, stream, &best);
    if (rc) return rc;
    if (out_best) to_abi(best, out_best);
    if (out_ms) *out_ms = best_ms;
    return NBODY_OK;
}

int nbody_tune_save(const char *path)
{
    if (!path) return fail(NBODY_EINVAL, "path is NULL");
    // written beside the target and renamed over it, so that a reader (another
    // process sharing the file) never sees a partly written file
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return fail(NBODY_EINVAL, "cannot open %s", tmp.c_str());
    const std::string arch = device_arch();
    const int cus = device_cus();
    std::lock_guard<std::mutex> lk(g_mu);
    fprintf(f, "{\"arch\": \"%s\", \"device_cus\": %d, \"entries\": [\n", arch.c_str(), cus);
    size_t k = 0;
    for (const auto &kv : g_tuned) {
        const TuneKey &t = kv.first;
        const Cfg &c = kv.second.first;
        fprintf(f,
                "  {\"api\": %d, \"law\": %d, \"precision\": %d, \"potential\": %d, \"n_bucket\": %d, "
                "\"s_bucket\": %d, \"block\": %d, \"i_per_lane\": %d, \"j_tile\": %d, \"j_split\": %d, "
                "\"j_stage\": %d, \"ms\": %.6f}%s\n",
                std::get<0>(t), std::get<1>(t), std::get<2>(t), std::get<3>(t), std::get<4>(t),
                std::get<5>(t), c.block, c.ipl, c.j_tile, c.j_split, c.j_stage, kv.second.second,
                (++k < g_tuned.size()) ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool written = !ferror(f);
    if (fclose(f) != 0 || !written) {
        remove(tmp.c_str());
        return fail(NBODY_EINVAL, "cannot write %s", tmp.c_str());
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return fail(NBODY_EINVAL, "cannot replace %s", path);
    }
    return NBODY_OK;
}

int nbody_tune_load(const char *path)
{
    if (!path) return fail(NBODY_EINVAL, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(NBODY_EINVAL, "cannot open %s", path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
    fclose(f);
    // the file's device must be this one
    char farch[64] = {0};
    int fcus = 0;
    const size_t pa = txt.find("\"arch\": \""), pc = txt.find("\"device_cus\": ");
    if (pa == std::string::npos || pc == std::string::npos ||
        sscanf(txt.c_str() + pa, "\"arch\": \"%63[^\"]\"", farch) != 1 ||
        sscanf(txt.c_str() + pc, "\"device_cus\": %d", &fcus) != 1)
        return fail(NBODY_EINVAL, "%s does not name the device it was tuned on", path);
    const std::string arch = device_arch();
    if (arch != farch || fcus != device_cus())
        return fail(NBODY_EINVAL, "%s was tuned on %s with %d CUs; this device is %s with %d CUs", path, farch,
                    fcus, arch.c_str(), device_cus());
    int loaded = 0;
    size_t pos = 0;
    while ((pos = txt.find("{\"api\"", pos)) != std::string::npos) {
        int api, law, prec, pot, nb, sb, block, ipl, jt, js, jst;
        double ms;
        if (sscanf(txt.c_str() + pos,
                   "{\"api\": %d, \"law\": %d, \"precision\": %d, \"potential\": %d, \"n_bucket\": %d, "
                   "\"s_bucket\": %d, \"block\": %d, \"i_per_lane\": %d, \"j_tile\": %d, \"j_split\": %d, "
                   "\"j_stage\": %d, \"ms\": %lf}",
                   &api, &law, &prec, &pot, &nb, &sb, &block, &ipl, &jt, &js, &jst, &ms) == 12) {
            nbody_config cc{block, ipl, jt, js, jst};
            if (cfg_valid(&cc) && api >= 0 && api < kNumApi) {
                std::lock_guard<std::mutex> lk(g_mu);
                g_tuned[TuneKey(api, law, prec, pot, nb, sb)] = {from_abi(&cc), ms};
                ++g_cfg_version;
                ++loaded;
            }
        }
        ++pos;
    }
    return loaded > 0 ? NBODY_OK : fail(NBODY_EINVAL, "no entries in %s", path);
}

int nbody_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_timing = on != 0;
    return NBODY_OK;
}

int nbody_timing_read(double *total_ms, int64_t *launches, int32_t reset)
{
    std::vector<TimedLaunch> pending;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        pending.swap(g_timed);
    }
    int rc = NBODY_OK;
    for (auto &t : pending) {
        float ms = 0;
        if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess)
            rc = fail(NBODY_EHIP, "timing events failed");
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
        std::lock_guard<std::mutex> lk(g_mu);
        g_timed_ms += ms;
        ++g_timed_count;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (total_ms) *total_ms = g_timed_ms;
    if (launches) *launches = g_timed_count;
    if (reset) {
        g_timed_ms = 0.0;
        g_timed_count = 0;
    }
    return rc;
}

int32_t nbody_flops_per_pair(int32_t api, int32_t law_kind, int32_t with_potential)
{
    if (api == NBODY_API_BACKWARD || api == NBODY_API_BACKWARD_BATCHED)
        return law_kind == NBODY_LAW_GRAVITY ? 41 : 68;
    if (api == NBODY_API_JERK || api == NBODY_API_HERMITE)
        return law_kind == NBODY_LAW_GRAVITY ? (with_potential ? 42 : 41) : 0;
    switch (law_kind) {
    case NBODY_LAW_GRAVITY: return with_potential ? 20 : 19;
    case NBODY_LAW_LJC_LINEAR: return with_potential ? 35 : 30;
    case NBODY_LAW_LJC_CONSTANT: return with_potential ? 36 : 31;
    case NBODY_LAW_LJC_SIGMOIDAL: return with_potential ? 53 : 48;
    default: return 0;
    }
}

}  // extern "C"
