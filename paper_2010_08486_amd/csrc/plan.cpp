// Planning of a detector launch: the sigma ladder, kernel radii, fp32
// weights and the threshold in kernel precision.
//
// Ladder (Sec. 4, Eq. 1): geometric, k = floor(ln(smax/smin)/ln(rho)) + 1
// DoG planes over k+1 Gaussian planes sigma_i = smin * rho^i; or the paper's
// arithmetic form, n_bin+1 planes sigma_i = smin + i (smax - smin)/n_bin.
// Kernels (Sec. 4.1): sampled out to radius r = floor(truncate*sigma + 0.5)
// and normalised over that support; computed in FP64 and rounded once to
// fp32, mirrored so the fp32 vector is exactly symmetric.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "runtime.h"

namespace dog {

static constexpr int kMaxRadius = 65536;

bool validate_params(const dog_params& p, std::string* err)
{
    auto bad = [&](const char* m) {
        *err = m;
        return false;
    };
    if (!std::isfinite(p.sigma_min) || !(p.sigma_min > 0.0))
        return bad("sigma_min must be finite and > 0");
    if (!std::isfinite(p.sigma_max) || !(p.sigma_max >= p.sigma_min))
        return bad("sigma_max must be finite and >= sigma_min");
    if (p.ladder != 0 && p.ladder != 1)
        return bad("ladder must be 0 (geometric) or 1 (arithmetic)");
    if (p.ladder == 0 && (!std::isfinite(p.sigma_ratio) || !(p.sigma_ratio > 1.0)))
        return bad("sigma_ratio must be finite and > 1");
    if (p.ladder == 1 && (p.n_bin < 1 || p.n_bin + 1 > DOG_MAX_GAUSS))
        return bad("n_bin must be in 1..63 for the arithmetic ladder");
    if (p.coalesce != 0 && p.coalesce != 1)
        return bad("coalesce must be 0 or 1");
    if (p.reserved != 0)
        return bad("reserved must be 0");
    if (!std::isfinite(p.threshold))
        return bad("threshold must be finite");
    if (!std::isfinite(p.overlap) || p.overlap < 0.0 || p.overlap > 1.0)
        return bad("overlap must be in [0, 1]");
    if (!std::isfinite(p.truncate) || p.truncate < 0.0)
        return bad("truncate must be finite and >= 0 (0 selects 4)");
    return true;
}

int dog_planes_for(double smin, double smax, double ratio)
{
    return (int)std::floor(std::log(smax / smin) / std::log(ratio)) + 1;
}

int build_plan(const dog_params& prm, Plan* plan, std::string* err)
{
    if (!validate_params(prm, err))
        return DOG_EINVAL;
    Plan& P = *plan;
    P.prm = prm;
    if (P.prm.truncate == 0.0)
        P.prm.truncate = 4.0;
    const int k = prm.ladder == 1 ? prm.n_bin
                                  : dog_planes_for(prm.sigma_min, prm.sigma_max, prm.sigma_ratio);
    if (k < 1 || k + 1 > DOG_MAX_GAUSS) {
        *err = "ladder has " + std::to_string(k) + " DoG planes; at most " +
               std::to_string(DOG_MAX_GAUSS - 1) + " are supported";
        return DOG_EINVAL;
    }
    P.k = k;
    P.n_g = k + 1;
    P.sigma.assign(P.n_g, 0.0);
    P.r.assign(P.n_g, 0);
    P.weights.clear();
    P.half64.assign(P.n_g, {});
    std::memset(&P.desc, 0, sizeof(P.desc));
    P.desc.n_g = P.n_g;
    for (int i = 0; i < P.n_g; ++i) {
        // Eq. 1: arithmetic, step (max - min)/n_bin; else geometric
        const double s = prm.ladder == 1
                             ? prm.sigma_min + (double)i * ((prm.sigma_max - prm.sigma_min) /
                                                            (double)prm.n_bin)
                             : prm.sigma_min * std::pow(prm.sigma_ratio, (double)i);
        const double rr = std::floor(P.prm.truncate * s + 0.5);
        if (!(rr <= (double)kMaxRadius)) {
            *err = "kernel radius above " + std::to_string(kMaxRadius);
            return DOG_EINVAL;
        }
        const int r = (int)rr;
        P.sigma[i] = s;
        P.r[i] = r;
        // half-kernel g[j] = exp(-j^2 / (2 s^2)), j = 0..r; total = g0 + 2 sum_{j>0} g[j]
        std::vector<double> g(r + 1);
        for (int j = 0; j <= r; ++j)
            g[j] = std::exp(-((double)j * (double)j) / (2.0 * s * s));
        double tail = 0.0;
        for (int j = r; j >= 1; --j)
            tail += g[j];
        const double total = g[0] + 2.0 * tail;
        const int taps = 2 * r + 1;
        const int padded = ((taps + DOG_WPAD - 1) / DOG_WPAD) * DOG_WPAD + DOG_WPAD;
        const int off = (int)P.weights.size();
        P.weights.resize(off + padded, 0.0f);
        for (int j = -r; j <= r; ++j)
            P.weights[off + (j + r)] = (float)(g[j < 0 ? -j : j] / total);
        P.half64[i].resize(r + 1);
        for (int j = 0; j <= r; ++j)
            P.half64[i][j] = g[j] / total;
        P.desc.r[i] = r;
        P.desc.woff[i] = off;
        P.desc.sigma[i] = (float)s;
    }
    // largest float t with t <= threshold: for finite fp32 D,
    // D > t  <=>  (double)D > threshold.
    float t = (float)prm.threshold;
    if ((double)t > prm.threshold)
        t = std::nextafter(t, -INFINITY);
    P.desc.thr = t;
    return DOG_OK;
}

bool same_params(const dog_params& a, const dog_params& b)
{
    return std::memcmp(&a, &b, sizeof(dog_params)) == 0;
}

}  // namespace dog
