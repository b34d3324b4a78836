// Host post-processing of a frame's candidate list: sort by (y, x, scale)
// and overlap pruning (Sec. 4.1: blobs whose normalised overlap exceeds a
// threshold are pruned; blob radius sqrt(2)*sigma, Sec. 3).
//
// Pruning rule: blobs are visited in (y, x, scale) order; for each surviving
// blob a, every later surviving blob b is compared; when the disk
// intersection exceeds `overlap` times the smaller disk's area, the blob
// with the smaller sigma is removed (b on a tie) and, if a was removed, a's
// scan stops.  Pairs whose disks cannot touch (centre distance >= sum of
// radii) are skipped without evaluation, using the row order to stop each
// scan early; skipping them does not change the outcome because their
// overlap is 0 and overlap >= 0.  In coalescing mode (Sec. 4.1: coalescing
// by averaging the radius) the same visits take place, and the survivor of
// each removal takes the mean of the pair's sigmas.
#include <algorithm>
#include <cmath>

#include "runtime.h"

namespace dog {

namespace {

// Area of the intersection of disks of radii a and b whose centres are dist apart.
double disk_intersection(double dist, double a, double b)
{
    if (dist >= a + b)
        return 0.0;
    const double small = std::min(a, b);
    if (dist <= std::fabs(a - b))
        return M_PI * small * small;
    const double d2 = dist * dist, a2 = a * a, b2 = b * b;
    const double ca = std::clamp((d2 + a2 - b2) / (2.0 * dist * a), -1.0, 1.0);
    const double cb = std::clamp((d2 + b2 - a2) / (2.0 * dist * b), -1.0, 1.0);
    const double kite = std::max(0.0, (-dist + a + b) * (dist + a - b) * (dist - a + b) * (dist + a + b));
    return a2 * std::acos(ca) + b2 * std::acos(cb) - 0.5 * std::sqrt(kite);
}

}  // namespace

double overlap_fraction(int y1, int x1, double s1, int y2, int x2, double s2)
{
    const double ra = std::sqrt(2.0) * s1, rb = std::sqrt(2.0) * s2;
    const double dy = (double)y1 - (double)y2, dx = (double)x1 - (double)x2;
    const double dist = std::sqrt(dy * dy + dx * dx);
    const double small = std::min(ra, rb);
    return disk_intersection(dist, ra, rb) / (M_PI * small * small);
}

void sort_blobs(std::vector<dog_blob>& v)
{
    std::sort(v.begin(), v.end(), [](const dog_blob& a, const dog_blob& b) {
        if (a.y != b.y)
            return a.y < b.y;
        if (a.x != b.x)
            return a.x < b.x;
        return a.scale < b.scale;
    });
}

// sigma64[i] is the FP64 sigma of ladder index i (the fp32 copy in dog_blob
// is for output only).  coalesce: the removed blob of an overlapping pair is
// merged into the survivor, whose sigma becomes the mean of the two (Sec.
// 4.1, averaging the radius); later pairs see the new sigma, and survivors'
// sigma fields carry it.  Sigmas only shrink under this rule (the survivor
// has the larger one), so the row-distance bound taken from the starting
// sigmas stays valid.
void prune_blobs(std::vector<dog_blob>& v, const std::vector<double>& sigma64, double overlap,
                 bool coalesce)
{
    const size_t n = v.size();
    if (overlap >= 1.0 || n < 2)
        return;
    std::vector<double> sg(n);
    double smax = 0.0;
    for (size_t i = 0; i < n; ++i) {
        sg[i] = sigma64[v[i].scale];
        smax = std::max(smax, sg[i]);
    }
    const double rmax = std::sqrt(2.0) * smax;
    std::vector<char> alive(n, 1);
    for (size_t a = 0; a < n; ++a) {
        if (!alive[a])
            continue;
        const double reach = std::sqrt(2.0) * sg[a] + rmax;  // no later blob beyond this row distance can touch a
        for (size_t b = a + 1; b < n; ++b) {
            if ((double)(v[b].y - v[a].y) >= reach)
                break;
            if (!alive[b])
                continue;
            const double sa = sg[a], sb = sg[b];
            // disks that clearly cannot touch have overlap 0 <= `overlap`:
            // skip them without the square root (the margin keeps every pair
            // the exact test could see as touching)
            const double dy = (double)(v[b].y - v[a].y), dx = (double)(v[b].x - v[a].x);
            const double rs = std::sqrt(2.0) * (sa + sb);
            if (dy * dy + dx * dx > rs * rs * (1.0 + 1e-9))
                continue;
            const double f = overlap_fraction(v[a].y, v[a].x, sa, v[b].y, v[b].x, sb);
            if (f > overlap) {
                const double mean = 0.5 * (sa + sb);
                if (sa < sb) {
                    alive[a] = 0;
                    if (coalesce)
                        sg[b] = mean;
                    break;
                }
                alive[b] = 0;
                if (coalesce)
                    sg[a] = mean;
            }
        }
    }
    size_t o = 0;
    for (size_t i = 0; i < n; ++i)
        if (alive[i]) {
            if (coalesce)
                v[i].sigma = (float)sg[i];
            v[o++] = v[i];
        }
    v.resize(o);
}

// Radius histogram (Sec. 4.1: blobs are histogrammed with bin centres at the
// radii sqrt(2) sigma_i of the ladder's k DoG scales): each blob counts in
// the bin of the nearest centre, the lower one on a tie; comparing sigmas
// gives the same bins, since every radius carries the factor sqrt(2).
void radius_histogram(const std::vector<double>& ladder, int k, const dog_blob* v, int64_t n,
                      int64_t* counts)
{
    std::fill(counts, counts + k, (int64_t)0);
    for (int64_t b = 0; b < n; ++b) {
        const double s = (double)v[b].sigma;
        // ladders increase: the first centre past s and the one before it
        const auto it = std::lower_bound(ladder.begin(), ladder.begin() + k, s);
        int i = (int)(it - ladder.begin());
        if (i == k)
            i = k - 1;
        else if (i > 0 && s - ladder[i - 1] <= ladder[i] - s)
            i = i - 1;
        counts[i] += 1;
    }
}

}  // namespace dog
