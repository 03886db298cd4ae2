// Host set-up of the preconditioner of the extracellular solve: a two-level
// additive method z = omega D^{-1} r + P A_c^{-1} P^T r, with D the diagonal of
// the elliptic operator A, P the piecewise-constant prolongation from
// aggregates of cells (centroids binned on a box grid) and A_c = P^T A P
// inverted densely.  A and A_c annihilate constants and, the flux form being
// conservative, so do their transposes; A_c is inverted with the rank-one
// term (mean |diag| / n) 1 1^T added, which gives the solution of zero sum
// for a right-hand side of zero sum.
#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "prep.hpp"

namespace ep {

std::string build_coarse(const PrepIn &in, const PrepOut &P, int target, Coarse &out) {
    const int64_t nc = P.n_tets;
    if (P.ebeta.empty()) return "no elliptic operator";
    // ---- aggregates: centroids binned on a grid of about `target` boxes
    std::vector<double> cen(3 * nc);
    double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int64_t i = 0; i < nc; ++i) {
        const int32_t *t = in.tets + 4 * (int64_t)P.perm[i];
        for (int a = 0; a < 3; ++a) {
            double x = 0.0;
            for (int k = 0; k < 4; ++k) x += in.xyz[3 * (int64_t)t[k] + a];
            cen[3 * i + a] = 0.25 * x;
            lo[a] = std::min(lo[a], cen[3 * i + a]);
            hi[a] = std::max(hi[a], cen[3 * i + a]);
        }
    }
    double ext[3], vol = 1.0;
    for (int a = 0; a < 3; ++a) { ext[a] = std::max(hi[a] - lo[a], 1e-12); vol *= ext[a]; }
    const double side = std::cbrt(vol / std::max(1, target));
    int64_t nb[3];
    for (int a = 0; a < 3; ++a) nb[a] = std::max<int64_t>(1, (int64_t)std::llround(ext[a] / side));
    std::vector<int64_t> box(nc);
    for (int64_t i = 0; i < nc; ++i) {
        int64_t k[3];
        for (int a = 0; a < 3; ++a)
            k[a] = std::min<int64_t>(nb[a] - 1, (int64_t)((cen[3 * i + a] - lo[a]) / ext[a] * nb[a]));
        box[i] = (k[0] * nb[1] + k[1]) * nb[2] + k[2];
    }
    std::vector<int64_t> ids(box);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    const int64_t na = (int64_t)ids.size();
    if (na > 8192) return "too many aggregates";
    out.n_agg = (int32_t)na;
    out.agg_of.resize(nc);
    for (int64_t i = 0; i < nc; ++i)
        out.agg_of[i] = (int32_t)(std::lower_bound(ids.begin(), ids.end(), box[i]) - ids.begin());
    out.agg_off.assign(na + 1, 0);
    for (int64_t i = 0; i < nc; ++i) out.agg_off[out.agg_of[i] + 1]++;
    for (int64_t a = 0; a < na; ++a) out.agg_off[a + 1] += out.agg_off[a];
    out.agg_cells.resize(nc);
    {
        std::vector<int32_t> f(out.agg_off.begin(), out.agg_off.end() - 1);
        for (int64_t i = 0; i < nc; ++i) out.agg_cells[f[out.agg_of[i]]++] = (int32_t)i;
    }

    // ---- A's diagonal and A_c = P^T A P from the stencil:
    //   (A x)_c = sum_s beta_s sum_k w_{node_s,k} x_k + sum_f b_f (x_nbr - x_c)
    std::vector<double> Ac((size_t)na * na, 0.0);
    out.dinv.assign(nc, 0.0);
    const int64_t n_slices = (int64_t)P.sell_off.size() - 1;
    (void)n_slices;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t I = out.agg_of[c];
        double diag = 0.0;
        for (int s = 0; s < 8; ++s) {
            const double beta = P.ebeta[(int64_t)s * nc + c];
            const int32_t node = P.cnode[(int64_t)s * nc + c];
            const int64_t sl = node >> 6, lane = node & 63;
            for (int64_t e = P.sell_off[sl] + lane; e < P.sell_off[sl + 1]; e += 64) {
                const double w = P.sell_w[e];
                if (w == 0.0) continue;
                const int32_t k = P.sell_cell[e];
                Ac[(size_t)I * na + out.agg_of[k]] += beta * w;
                if (k == c) diag += beta * w;
            }
        }
        for (int f = 0; f < 4; ++f) {
            const double b = P.eb[(int64_t)f * nc + c];
            const int32_t k = P.cnbr[(int64_t)f * nc + c];
            Ac[(size_t)I * na + out.agg_of[k]] += b;
            Ac[(size_t)I * na + I] -= b;
            if (k != c) diag -= b;
        }
        out.dinv[c] = diag != 0.0 ? 1.0 / diag : 0.0;
    }

    // ---- dense inverse of A_c + (mean |diag| / na) 1 1^T (Gauss-Jordan with
    // partial pivoting; row updates split over host threads)
    double md = 0.0;
    for (int64_t a = 0; a < na; ++a) md += std::fabs(Ac[(size_t)a * na + a]);
    md /= (double)na;
    for (auto &x : Ac) x += md / (double)na;
    std::vector<double> inv((size_t)na * na, 0.0);
    for (int64_t a = 0; a < na; ++a) inv[(size_t)a * na + a] = 1.0;
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (int64_t p = 0; p < na; ++p) {
        int64_t piv = p;
        for (int64_t r = p + 1; r < na; ++r)
            if (std::fabs(Ac[(size_t)r * na + p]) > std::fabs(Ac[(size_t)piv * na + p])) piv = r;
        if (Ac[(size_t)piv * na + p] == 0.0) return "singular coarse operator";
        if (piv != p)
            for (int64_t j = 0; j < na; ++j) {
                std::swap(Ac[(size_t)p * na + j], Ac[(size_t)piv * na + j]);
                std::swap(inv[(size_t)p * na + j], inv[(size_t)piv * na + j]);
            }
        const double d = 1.0 / Ac[(size_t)p * na + p];
        for (int64_t j = 0; j < na; ++j) {
            Ac[(size_t)p * na + j] *= d;
            inv[(size_t)p * na + j] *= d;
        }
        auto eliminate = [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r) {
                if (r == p) continue;
                const double f = Ac[(size_t)r * na + p];
                if (f == 0.0) continue;
                for (int64_t j = 0; j < na; ++j) {
                    Ac[(size_t)r * na + j] -= f * Ac[(size_t)p * na + j];
                    inv[(size_t)r * na + j] -= f * inv[(size_t)p * na + j];
                }
            }
        };
        if (na < 256) {
            eliminate(0, na);
        } else {
            std::vector<std::thread> th;
            for (unsigned t = 0; t < nt; ++t)
                th.emplace_back(eliminate, na * t / nt, na * (t + 1) / nt);
            for (auto &x : th) x.join();
        }
    }
    out.cinv = std::move(inv);
    return "";
}

}  // namespace ep
