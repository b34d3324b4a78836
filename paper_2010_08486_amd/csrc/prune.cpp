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
// scan early and column buckets to skip distant columns; skipping them does
// not change the outcome because their overlap is 0 and overlap >= 0.  In
// coalescing mode (Sec. 4.1: coalescing by averaging the radius) the same
// visits take place, and the survivor of each removal takes the mean of the
// pair's sigmas.
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

// Sorts by (y, x, scale), equal triples in their incoming order.  When the
// three ranges and the list index fit in 64 bits (always for a frame's
// candidates), each blob becomes one integer key (y, x, scale, index in
// mixed radix) and the keys are sorted: several times faster than a
// three-field comparison on these short lists.
void sort_blobs(std::vector<dog_blob>& v)
{
    const size_t n = v.size();
    if (n < 2)
        return;
    int64_t lo[3] = {v[0].y, v[0].x, v[0].scale}, hi[3] = {lo[0], lo[1], lo[2]};
    for (const dog_blob& b : v) {
        const int64_t f[3] = {b.y, b.x, b.scale};
        for (int j = 0; j < 3; ++j) {
            lo[j] = std::min(lo[j], f[j]);
            hi[j] = std::max(hi[j], f[j]);
        }
    }
    // key = ((y' * RX + x') * RS + s') * n + index, with y' = y - ymin etc.
    const double span = (double)(hi[0] - lo[0] + 1) * (double)(hi[1] - lo[1] + 1) *
                        (double)(hi[2] - lo[2] + 1) * (double)n;
    if (span < 9.0e18) {
        const uint64_t rx = (uint64_t)(hi[1] - lo[1] + 1), rs = (uint64_t)(hi[2] - lo[2] + 1);
        std::vector<uint64_t> key(n);
        for (size_t i = 0; i < n; ++i) {
            const uint64_t y = (uint64_t)((int64_t)v[i].y - lo[0]);
            const uint64_t x = (uint64_t)((int64_t)v[i].x - lo[1]);
            const uint64_t s = (uint64_t)((int64_t)v[i].scale - lo[2]);
            key[i] = ((y * rx + x) * rs + s) * (uint64_t)n + i;
        }
        std::sort(key.begin(), key.end());
        std::vector<dog_blob> out(n);
        for (size_t i = 0; i < n; ++i)
            out[i] = v[key[i] % n];
        v.swap(out);
        return;
    }
    std::stable_sort(v.begin(), v.end(), [](const dog_blob& a, const dog_blob& b) {
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
    int64_t xmin = v[0].x, xmax = v[0].x;
    for (size_t i = 0; i < n; ++i) {
        sg[i] = sigma64[v[i].scale];
        smax = std::max(smax, sg[i]);
        xmin = std::min<int64_t>(xmin, v[i].x);
        xmax = std::max<int64_t>(xmax, v[i].x);
    }
    const double rmax = std::sqrt(2.0) * smax;
    // Column buckets at least as wide as the largest touching distance
    // 2 rmax: a blob can only touch blobs of its own bucket and the two next
    // to it.  Each bucket lists its blobs in list order (so by row), and a
    // blob's scan merges the three lists by index: it visits every blob it
    // could touch in the same order as a scan over the whole list, so the
    // outcome is the same.  A very sparse spread of columns uses one bucket.
    const int64_t bw = std::max<int64_t>(1, (int64_t)std::ceil(2.0 * rmax));
    int64_t nbk = (xmax - xmin) / bw + 1;
    if (nbk > 4 * (int64_t)n + 16)
        nbk = 1;
    auto bucket_of = [&](size_t i) -> int64_t { return nbk == 1 ? 0 : ((int64_t)v[i].x - xmin) / bw; };
    std::vector<size_t> start((size_t)nbk + 1, 0), members(n);
    for (size_t i = 0; i < n; ++i)
        ++start[(size_t)bucket_of(i) + 1];
    for (int64_t c = 0; c < nbk; ++c)
        start[(size_t)c + 1] += start[(size_t)c];
    {
        std::vector<size_t> fill(start.begin(), start.end() - 1);
        for (size_t i = 0; i < n; ++i)
            members[fill[(size_t)bucket_of(i)]++] = i;
    }
    // cur[c]: the first member of bucket c after the blob being scanned
    // (blobs are scanned in list order, so these only move forward)
    std::vector<size_t> cur(start.begin(), start.end() - 1);
    std::vector<char> alive(n, 1);
    for (size_t a = 0; a < n; ++a) {
        const int64_t ca = bucket_of(a);
        ++cur[(size_t)ca];   // a itself is the next member of its bucket
        if (!alive[a])
            continue;
        const double reach = std::sqrt(2.0) * sg[a] + rmax;  // no later blob beyond this row distance can touch a
        size_t pos[3], end[3];
        int nl = 0;
        for (int64_t c = std::max<int64_t>(0, ca - 1); c <= std::min<int64_t>(nbk - 1, ca + 1); ++c) {
            pos[nl] = cur[(size_t)c];
            end[nl] = start[(size_t)c + 1];
            ++nl;
        }
        for (;;) {
            // the next blob by list index among the three buckets
            int best = -1;
            for (int l = 0; l < nl; ++l)
                if (pos[l] < end[l] && (best < 0 || members[pos[l]] < members[pos[best]]))
                    best = l;
            if (best < 0)
                break;
            const size_t b = members[pos[best]];
            if ((double)v[b].y - (double)v[a].y >= reach) {
                end[best] = pos[best];   // this bucket has nothing closer left
                continue;
            }
            ++pos[best];
            if (!alive[b])
                continue;
            const double sa = sg[a], sb = sg[b];
            // disks that clearly cannot touch have overlap 0 <= `overlap`:
            // skip them without the square root (the margin keeps every pair
            // the exact test could see as touching)
            // differences in double: coordinates far apart would overflow int32
            const double dy = (double)v[b].y - (double)v[a].y, dx = (double)v[b].x - (double)v[a].x;
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
