// Scheme family of the SRJ method (host side).
//
// Level -> M follows Appendix B of Islam & Wang (arXiv 2011.06636).  The
// factors of a length-M scheme are Eq. (17):
//     w_j = (l* + 1) / (2 (l* - x_j)),  x_j = cos((2j+1) pi / (2M)),  j = 0..M-1,
// with l* the real root above 1 of T_M(l*) = 3; since T_M(cosh t) = cosh(M t),
// l* = cosh(arccosh(3) / M).
//
// A cycle applies the factors in Leja order of the amplification-polynomial
// roots rho_j = 1 - 1/w_j (Eq. (15)): the largest factor first, then each
// next root is the unused one with the largest sum of log distances to the
// roots already applied (ties: lowest j).  The paper asks for the factors to
// be cycled so each step reduces the error most, for robustness to round-off
// and overflow (section 2, last paragraph); this ordering reproduces the
// printed orders of Table 2.  The sums are accumulated in pick order, so the
// floating-point scores are fully determined.
#include <math.h>

#include <mutex>

#include "internal.h"

namespace srj {

namespace {

const int kLevelM[SRJ_NUM_LEVELS] = {1,   2,   3,   5,   7,   10,   14,   19,   26,
                                     35,  47,  63,  84,  111, 147,  194,  256,  338,
                                     446, 589, 778, 1027, 1356, 1790, 2362};

constexpr double kPi = 3.14159265358979323846;

std::vector<double> natural_factors(int M)
{
    std::vector<double> w(M);
    const double ls = cosh(acosh(3.0) / static_cast<double>(M));
    for (int j = 0; j < M; ++j) {
        const double xj = cos(static_cast<double>(2 * j + 1) * kPi / (2.0 * M));
        w[j] = (ls + 1.0) / (2.0 * (ls - xj));
    }
    return w;
}

std::vector<double> leja_ordered(const std::vector<double> &w)
{
    const int M = static_cast<int>(w.size());
    std::vector<double> rho(M), logsum(M, 0.0), out;
    std::vector<char> taken(M, 0);
    for (int j = 0; j < M; ++j) rho[j] = 1.0 - 1.0 / w[j];
    out.reserve(M);
    int pick = 0;  // largest factor: j = 0 (x_0 is the root nearest l*)
    for (int step = 0; step < M; ++step) {
        taken[pick] = 1;
        out.push_back(w[pick]);
        if (step + 1 == M) break;
        int next = -1;
        for (int j = 0; j < M; ++j) {
            if (taken[j]) continue;
            logsum[j] = logsum[j] + log(fabs(rho[j] - rho[pick]));
            if (next < 0 || logsum[j] > logsum[next]) next = j;
        }
        pick = next;
    }
    return out;
}

std::once_flag g_once;
std::vector<double> g_factors[SRJ_NUM_LEVELS];

void build_all()
{
    for (int l = 0; l < SRJ_NUM_LEVELS; ++l) g_factors[l] = leja_ordered(natural_factors(kLevelM[l]));
}

}  // namespace

int level_m(int level)
{
    if (level < 0 || level >= SRJ_NUM_LEVELS) return -1;
    return kLevelM[level];
}

const std::vector<double> &level_factors(int level)
{
    std::call_once(g_once, build_all);
    return g_factors[level];
}

void full_table(std::vector<double> &omega, std::vector<int32_t> &offsets)
{
    std::call_once(g_once, build_all);
    omega.clear();
    offsets.assign(SRJ_NUM_LEVELS + 1, 0);
    for (int l = 0; l < SRJ_NUM_LEVELS; ++l) {
        offsets[l] = static_cast<int32_t>(omega.size());
        omega.insert(omega.end(), g_factors[l].begin(), g_factors[l].end());
    }
    offsets[SRJ_NUM_LEVELS] = static_cast<int32_t>(omega.size());
}

}  // namespace srj
