// Host runtime: contexts, device workspace, launch tables and the launch of
// the three-kernel sequence (pass 1, pass 2, local maxima) over a list of
// frames, then the readback of the candidate records.
#include <chrono>

#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace dog {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

int hip_fail(hipError_t e, const char* what)
{
    g_err = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " +
            what;
    return (e == hipErrorOutOfMemory) ? DOG_ENOMEM : DOG_EDEVICE;
}

uint64_t ctx_total_used(const dog_context* c)
{
    uint64_t u = c->used;
    for (const dog_context* l : c->lanes)
        u += l->used;
    return u;
}

int ctx_alloc(dog_context* c, DevBuf* b, size_t bytes, const char* what)
{
    if (b->bytes >= bytes)
        return DOG_OK;
    // a lane allocates out of its parent's budget
    const dog_context* root = c->parent ? c->parent : c;
    const uint64_t held = ctx_total_used(root);
    // grow geometrically so a sequence of slightly larger requests does not
    // reallocate every time (unless exact allocation is asked for)
    size_t want = c->exact_alloc ? bytes : std::max(bytes, b->bytes + b->bytes / 4);
    want = (want + 4095) & ~(size_t)4095;
    const uint64_t after = held - b->bytes + want;
    if (after > root->budget) {
        want = (bytes + 4095) & ~(size_t)4095;
        if (held - b->bytes + want > root->budget) {
            set_error(std::string("HBM budget exceeded allocating ") + what + ": need " +
                      std::to_string(held - b->bytes + want) + " bytes, budget " +
                      std::to_string(root->budget));
            return DOG_ENOMEM;
        }
    }
    if (b->p) {
        DOG_HIP(hipStreamSynchronize(c->stream));
        DOG_HIP(hipFree(b->p));
        c->used -= b->bytes;
        b->p = nullptr;
        b->bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string("hipMalloc failed for ") + what + " (" + std::to_string(want) +
                  " bytes)");
        return DOG_ENOMEM;
    }
    b->p = p;
    b->bytes = want;
    c->used += want;
    return DOG_OK;
}

int ctx_trim(dog_context* c)
{
    if (c->stream)
        DOG_HIP(hipStreamSynchronize(c->stream));
    drop_graph(c);
    for (DevBuf* b : {&c->planes, &c->input, &c->tables, &c->cand}) {
        if (b->p) {
            DOG_HIP(hipFree(b->p));
            c->used -= b->bytes;
        }
        b->p = nullptr;
        b->bytes = 0;
    }
    c->cap = 0;
    c->seen_key.clear();
    return DOG_OK;
}

static constexpr uint64_t kInitialCap = 65536;   // candidate records of a new context

uint64_t frame_plane_bytes(const Plan& P, int64_t H, int64_t W)
{
    const uint64_t pitch = ((uint64_t)H + 63) / 64 * 64;
    return 2ull * (uint64_t)P.n_g * (uint64_t)W * pitch * sizeof(float) + 256;
}

uint64_t frame_input_bytes(int64_t H, int64_t W)
{
    return (uint64_t)H * (uint64_t)W * sizeof(float) + 256;
}

uint64_t overhead_bound(const Plan& P, int n, const int64_t* heights, const int64_t* widths)
{
    // smallest bands of any variant: blur tiles are 64 columns by at least
    // min_band rows, local-maximum tiles 62 columns by at least min_nms rows
    int min_band = 1 << 30, min_nms = 1 << 30, max_pad_rows = 0;
    for (int v = 0; v < dogk_num_variants(); ++v) {
        int S, NW, BI, BN, NWN;
        dogk_variant_geometry(v, &S, &NW, &BI, &BN, &NWN);
        min_band = std::min(min_band, S * NW * BI);
        min_nms = std::min(min_nms, BN * NWN);
        max_pad_rows = std::max(max_pad_rows, (dogk_variant_ring(v) + 1) * S);
    }
    const int rmax = *std::max_element(P.r.begin(), P.r.end());
    const uint64_t pad = (uint64_t)rmax + (uint64_t)max_pad_rows;
    uint64_t tiles = 0, rows = 0;
    for (int f = 0; f < n; ++f) {
        const uint64_t H = (uint64_t)heights[f], W = (uint64_t)widths[f];
        tiles += (uint64_t)P.n_g * ((W + 63) / 64) * ((H + min_band - 1) / min_band);
        tiles += (uint64_t)P.n_g * ((H + 63) / 64) * ((W + min_band - 1) / min_band);
        tiles += ((H + DOG_NMS_COLS - 1) / DOG_NMS_COLS) * ((W + min_nms - 1) / min_nms);
        rows += (H + 2 * pad + 64) + (W + 2 * pad + 64);
    }
    const uint64_t tables = sizeof(FrameDesc) * (uint64_t)n + sizeof(LadderDesc) +
                            sizeof(float) * P.weights.size() + sizeof(Tile) * tiles +
                            sizeof(int) * rows + 8 * 256;
    const uint64_t cand = sizeof(CandHeader) + sizeof(CandRec) * kInitialCap;
    return ((tables + 4095) & ~(uint64_t)4095) + ((cand + 4095) & ~(uint64_t)4095);
}

int ctx_pin(PinBuf* b, size_t bytes)
{
    if (b->bytes >= bytes)
        return DOG_OK;
    size_t want = std::max(bytes, b->bytes + b->bytes / 4);
    want = (want + 4095) & ~(size_t)4095;
    if (b->p) {
        DOG_HIP(hipHostFree(b->p));
        b->p = nullptr;
        b->bytes = 0;
    }
    DOG_HIP(hipHostMalloc(&b->p, want, hipHostMallocDefault));
    b->bytes = want;
    return DOG_OK;
}

int ctx_plan(dog_context* c, const dog_params* prm, const Plan** out)
{
    if (!prm) {
        set_error("params is NULL");
        return DOG_EINVAL;
    }
    // the plan stores truncate 0 as the 4 it selects: compare in that form,
    // so callers that leave it 0 keep their plan (and captured graph)
    dog_params want = *prm;
    if (want.truncate == 0.0)
        want.truncate = 4.0;
    if (!c->have_plan || !same_params(c->plan.prm, want)) {
        Plan P;
        std::string err;
        const int rc = build_plan(*prm, &P, &err);
        if (rc != DOG_OK) {
            set_error(err);
            return rc;
        }
        c->plan = std::move(P);
        c->have_plan = true;
        c->plan_gen += 1;
    }
    *out = &c->plan;
    return DOG_OK;
}

int ctx_set_variant(dog_context* c, int v)
{
    if (v < 0)
        v = c->variant_auto;
    if (v >= dogk_num_variants()) {
        set_error("no such kernel variant");
        return DOG_EINVAL;
    }
    int o[3];
    DOG_HIP(dogk_occupancy(v, &o[0], &o[1], &o[2]));
    if (v != c->variant)
        drop_graph(c);
    c->variant = v;
    for (int i = 0; i < 3; ++i)
        c->occ[i] = std::max(1, o[i]);
    return DOG_OK;
}

static Variant variant_geometry(int v)
{
    Variant g;
    dogk_variant_geometry(v, &g.S, &g.NW, &g.BI, &g.BN, &g.NWN);
    g.group = dogk_variant_group(v);
    return g;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Half-sample symmetric reflection of index t into [0, n), period 2n: the
// extended sequence is x[0..n-1], x[n-1..0], x[0..n-1], ...
static long long reflect_index(long long t, long long n)
{
    const long long p = 2 * n;
    long long u = t % p;
    if (u < 0)
        u += p;
    return u < n ? u : p - 1 - u;
}

// ---- transform-domain blur: shapes, job sizes, kernel transfer functions

// Frames whose sides are powers of two in [64, 2048] may take the transform
// path.
bool frame_dct_ok(int H, int W)
{
    auto p2 = [](int v) { return v >= 64 && v <= 2048 && (v & (v - 1)) == 0; };
    return p2(H) && p2(W);
}

static int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v)
        ++l;
    return l;
}

// H[k] = w_0 + 2 sum_{j=1..r} w_j cos(pi k j / N), k = 0..N-1, from the FP64
// half kernel (cosines by the three-term recurrence in j).
static std::vector<double> dct_transfer(const std::vector<double>& half, int N)
{
    std::vector<double> H((size_t)N);
    const int r = (int)half.size() - 1;
    for (int k = 0; k < N; ++k) {
        const double c1 = std::cos(M_PI * (double)k / (double)N);
        double cm = 1.0, cj = c1, sum = 0.0;
        for (int j = 1; j <= r; ++j) {
            sum += half[j] * cj;
            const double cn = 2.0 * c1 * cj - cm;
            cm = cj;
            cj = cn;
        }
        H[k] = half[0] + 2.0 * sum;
    }
    return H;
}

// ---- blur tiles: which planes one workgroup takes

std::vector<PlaneRun> plane_runs(const Plan& P, const std::vector<int>& planes, int S, bool group)
{
    // cost of a plane in a tile: its tap chunks, plus one for staging the
    // band's first rows
    auto cost = [&](int p) { return (2 * P.r[p] + S) / S + 1; };
    std::vector<PlaneRun> runs;
    if (!group) {
        for (int p : planes)
            runs.push_back({p, 1, cost(p)});
        return runs;
    }
    // Cut the planes (widest first) into runs of consecutive planes: the
    // fewest runs whose longest chain stays within 15 % of the widest
    // plane's, and among those cuts the one with the shortest longest chain.
    int cmax = 0;
    for (int p : planes)
        cmax = std::max(cmax, cost(p));
    size_t i = 0;
    while (i < planes.size()) {
        // a segment of consecutive plane indices
        size_t j = i + 1;
        while (j < planes.size() && planes[j] == planes[j - 1] - 1)
            ++j;
        const int m = (int)(j - i);
        std::vector<int> c(m), pre(m + 1, 0);
        for (int q = 0; q < m; ++q) {
            c[q] = cost(planes[i + q]);
            pre[q + 1] = pre[q] + c[q];
        }
        // best[g][q]: the smallest longest run over cuts of the first q
        // planes into g runs; cut[g][q]: where the last run starts
        const int INF = 1 << 30;
        std::vector<std::vector<int>> best(m + 1, std::vector<int>(m + 1, INF)),
            cut(m + 1, std::vector<int>(m + 1, 0));
        best[0][0] = 0;
        int g_use = m;
        for (int g = 1; g <= m; ++g) {
            for (int q = g; q <= m; ++q)
                for (int s0 = g - 1; s0 < q; ++s0) {
                    const int v = std::max(best[g - 1][s0], pre[q] - pre[s0]);
                    if (v < best[g][q]) {
                        best[g][q] = v;
                        cut[g][q] = s0;
                    }
                }
            if (best[g][m] * 100 <= cmax * 115) {
                g_use = g;
                break;
            }
        }
        std::vector<PlaneRun> seg;
        for (int g = g_use, q = m; g > 0; --g) {
            const int s0 = cut[g][q];
            seg.push_back({planes[i + s0], q - s0, pre[q] - pre[s0]});
            q = s0;
        }
        runs.insert(runs.end(), seg.rbegin(), seg.rend());
        i = j;
    }
    return runs;
}

// Workgroup order for jobs whose neighbours share cache lines: the list is
// cut into DOG_NXCD contiguous slices and slot b (dispatched to XCD b mod
// DOG_NXCD) takes the next job of slice b mod DOG_NXCD, so neighbouring jobs
// run on one XCD and its L2 fetches each line once (round-robin order would
// have every XCD fetch the lines of all its neighbours' jobs).  An exhausted
// slice's slots take jobs from the longest remaining slice.
template <class T>
static std::vector<T> xcd_order(const std::vector<T>& v)
{
    const size_t n = v.size();
    size_t lo[DOG_NXCD], hi[DOG_NXCD];
    for (int x = 0; x < DOG_NXCD; ++x) {
        lo[x] = n * x / DOG_NXCD;
        hi[x] = n * (x + 1) / DOG_NXCD;
    }
    std::vector<T> out;
    out.reserve(n);
    while (out.size() < n) {
        for (int x = 0; x < DOG_NXCD && out.size() < n; ++x) {
            int src = x;
            if (lo[x] >= hi[x]) {
                size_t best = 0;
                for (int y = 0; y < DOG_NXCD; ++y)
                    if (hi[y] - lo[y] > best) {
                        best = hi[y] - lo[y];
                        src = y;
                    }
            }
            out.push_back(v[lo[src]++]);
        }
    }
    return out;
}

// Transform jobs in launch order when each workgroup takes g consecutive
// jobs: padded with empty jobs to whole groups, the groups in XCD-local order
// (xcd_order), their count padded with empty groups to a multiple of `round`.
static size_t grouped_jobs(size_t n, int g, int round)
{
    size_t groups = (n + (size_t)g - 1) / (size_t)g;
    groups = (groups + (size_t)round - 1) / (size_t)round * (size_t)round;
    return groups * (size_t)g;
}

static std::vector<FftJob> group_jobs(const std::vector<FftJob>& v, int g, int round)
{
    std::vector<size_t> ids((v.size() + (size_t)g - 1) / (size_t)g);
    for (size_t i = 0; i < ids.size(); ++i)
        ids[i] = i;
    ids = xcd_order(ids);
    std::vector<FftJob> out;
    out.reserve(grouped_jobs(v.size(), g, round));
    for (size_t id : ids)
        for (int k = 0; k < g; ++k) {
            const size_t i = id * (size_t)g + (size_t)k;
            out.push_back(i < v.size() ? v[i] : FftJob{});   // no planes: does nothing
        }
    out.resize(grouped_jobs(v.size(), g, round), FftJob{});
    return out;
}

// Marks the groups of kFftWaveJobs wave jobs whose lines a workgroup loads
// together (fft_wave_load_cols): four column jobs of one input plane with
// one pitch, line pairs line0, + 2, + 4, + 6 from a multiple of 8 (16-byte
// aligned row pieces: the plane and its rows start at multiples of 64
// floats).
static void mark_column_groups(std::vector<FftJob>& v)
{
    for (size_t g = 0; g + kFftWaveJobs <= v.size(); g += kFftWaveJobs) {
        const FftJob& f = v[g];
        bool ok = f.n_planes > 0 && !f.in_rows && f.in && f.line0 % 8 == 0 && f.in_pitch % 4 == 0 &&
                  ((uintptr_t)f.in % 16) == 0;
        for (int k = 1; ok && k < kFftWaveJobs; ++k) {
            const FftJob& e = v[g + k];
            ok = e.n_planes > 0 && !e.in_rows && e.in == f.in && e.in_pitch == f.in_pitch &&
                 e.line0 == f.line0 + 2 * k;
        }
        v[g].flags = ok ? kFftGroupCols : 0;
    }
}

static constexpr size_t kRecBytes = sizeof(CandRec);
static constexpr uint32_t kUnpublished = 0xffffffffu;  // host-side count before a launch

// Completion of the sequence just queued on st: an event recorded after it.
static int record_done(dog_context* c, hipStream_t st)
{
    if (!c->ev_done)
        DOG_HIP(hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming));
    DOG_HIP(hipEventRecord(c->ev_done, st));
    return DOG_OK;
}

// Wait for that event: poll it for up to 20 ms (a frame's sequence takes tens
// of microseconds, and a blocking wait adds the wake-up latency of an
// interrupt), then fall back to a blocking wait.
static int wait_done(dog_context* c)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(c->ev_done);
        if (e == hipSuccess)
            return DOG_OK;
        if (e != hipErrorNotReady)
            return hip_fail(e, "hipEventQuery");
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
            DOG_HIP(hipEventSynchronize(c->ev_done));
            return DOG_OK;
        }
    }
}

// Pinned host destinations of the local-maximum kernel: records after the
// header slot of h_cand, and one range end per workgroup in h_ends.
static void host_targets(dog_context* c, LaunchArgs* a)
{
    a->host_recs = reinterpret_cast<CandRec*>(static_cast<CandHeader*>(c->h_cand.p) + 1);
    a->host_ends = static_cast<uint32_t*>(c->h_ends.p);
    a->n_host = c->guess;
}

// The launch sequence of the current tables on stream st: upload of the
// frame table from pinned staging (or, for one frame, its descriptor passed
// inline in the kernel arguments, with no upload), then the three kernels
// (with timing events when profiling).  The local-maximum kernel writes the
// first `guess` records and its range ends straight into pinned host memory,
// so there is no readback copy.  Captured once into a graph, or issued
// directly.
static hipError_t enqueue_sequence(dog_context* c, hipStream_t st, const FrameDesc* inline_f0)
{
    LaunchArgs a = c->args;
    host_targets(c, &a);
    hipError_t e = hipSuccess;
    if (inline_f0) {
        a.frames = nullptr;
        a.f0 = *inline_f0;
    } else {
        e = hipMemcpyAsync(const_cast<FrameDesc*>(a.frames), c->h_tables.p, c->frames_bytes,
                           hipMemcpyHostToDevice, st);
    }
    hipEvent_t* ev = c->profiling ? c->ev : nullptr;
    // each pass: the direct planes' tiles, then the transform-domain planes'
    // jobs (events: pass 1, pass 2, local maxima, transform 1, transform 2)
    for (int pass = 1; pass <= 2 && e == hipSuccess; ++pass) {
        e = dogk_launch_pass(c->variant, &a, pass, pass == 1 ? a.n1 : a.n2,
                             c->fft.merged_logn[pass - 1], c->wide1 ? 1 : 0, st,
                             ev ? ev + 2 * (pass - 1) : nullptr);
        const int i = pass - 1;
        for (int lg = 0; lg < 6 && e == hipSuccess; ++lg)
            if (c->fft.n[i][lg] > 0)
                e = dogk_fft_blur(&a, static_cast<const FftJob*>(c->fft.jobs[i][lg]),
                                  c->fft.n[i][lg], lg + 6, c->fft.vec[i], st,
                                  ev ? ev + 6 + 2 * i : nullptr);
    }
    if (e == hipSuccess)
        e = dogk_launch_nms_ev(c->variant, &a, a.n3, c->debug_planes ? 1 : 0, st,
                               ev ? ev + 4 : nullptr);
    return e;
}

void drop_graph(dog_context* c)
{
    if (c->graph_exec)
        (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph)
        (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_key.clear();
    c->tables_ready = false;
}

// Everything that fixes the launch tables, the buffers they point into and
// the captured sequence, apart from the frames' pixel pointers.
static std::vector<long long> launch_key(const dog_context* c, const Plan& P,
                                         const std::vector<FrameIn>& frames, bool dbg_D)
{
    bool wide = true;
    for (const FrameIn& f : frames)
        wide = wide && f.W % 64 == 0 && f.stride % 4 == 0 && ((uintptr_t)f.d & 15) == 0;
    std::vector<long long> k;
    k.reserve(16 + 3 * frames.size());
    k.push_back(wide ? 1 : 0);  // first entry: 16-byte loads in pass 1
    k.push_back((long long)frames.size());
    k.push_back(c->variant);
    k.push_back((long long)c->plan_gen);
    k.push_back(dbg_D ? 1 : 0);
    k.push_back(c->profiling ? 1 : 0);
    k.push_back(c->dct_forced ? 1 : 0);
    k.push_back((long long)(uintptr_t)c->planes.p);
    k.push_back((long long)(uintptr_t)c->tables.p);
    k.push_back((long long)(uintptr_t)c->cand.p);
    k.push_back((long long)(uintptr_t)c->h_tables.p);
    k.push_back((long long)(uintptr_t)c->h_cand.p);
    k.push_back((long long)(uintptr_t)c->h_ends.p);
    k.push_back((long long)c->cap);
    for (const FrameIn& f : frames) {
        k.push_back(f.H);
        k.push_back(f.W);
        k.push_back(f.stride);
        k.push_back(frame_min_taps(c, f.H, f.W, P));
    }
    return k;
}

int launch_frames(dog_context* c, const Plan& P, const std::vector<FrameIn>& frames, hipStream_t s,
                  bool dbg_D, long long* pitch0, float** L0, float** D0)
{
    const int n = (int)frames.size();
    c->pending = false;
    c->pend_n = n;
    if (n == 0) {
        c->pending = true;
        return DOG_OK;
    }
    if (!c->variant_forced) {
        const int v = choose_variant(c, frames, P);
        if (v != c->variant) {
            const int rc = ctx_set_variant(c, v);
            if (rc != DOG_OK)
                return rc;
        }
    }
    const Variant V = variant_geometry(c->variant);
    const int n_g = P.n_g;

    // ---- planes blurred in the transform domain: those whose kernels have
    // at least dct_min_taps taps, on frames whose sides are powers of two
    std::vector<std::vector<int>> dctp(n);
    for (int f = 0; f < n; ++f) {
        const int mt = frame_min_taps(c, frames[f].H, frames[f].W, P);
        if (!frame_dct_ok(frames[f].H, frames[f].W) || mt <= 0)
            continue;
        for (int p = 0; p < n_g; ++p)
            if (2 * P.r[p] + 1 >= mt)
                dctp[f].push_back(p);
    }

    // ---- workspace: T and L planes (transposed, pitch = H rounded to 64)
    std::vector<long long> pitch(n), off(n);
    size_t total = 0;
    for (int f = 0; f < n; ++f) {
        pitch[f] = ((long long)frames[f].H + 63) / 64 * 64;
        const size_t plane = (size_t)frames[f].W * (size_t)pitch[f];
        off[f] = (long long)total;
        total += 2 * (size_t)n_g * plane + ((dbg_D && f == 0) ? (size_t)P.k * plane : 0);
        total = align_up(total, 64);
    }
    int rc = ctx_alloc(c, &c->planes, total * sizeof(float), "scale-space planes");
    if (rc != DOG_OK)
        return rc;
    if (c->cap == 0) {
        if ((rc = ctx_alloc(c, &c->cand, sizeof(CandHeader) + kRecBytes * kInitialCap,
                            "candidates")) != DOG_OK)
            return rc;
        c->cap = (uint32_t)kInitialCap;
    }
    if ((rc = ctx_pin(&c->h_cand, sizeof(CandHeader) + kRecBytes * (size_t)c->cap)) != DOG_OK)
        return rc;
    float* planes = static_cast<float*>(c->planes.p);

    // ---- frame table (the only part that changes between replays)
    std::vector<FrameDesc> fd(n);
    for (int f = 0; f < n; ++f) {
        const size_t plane = (size_t)frames[f].W * (size_t)pitch[f];
        FrameDesc& d = fd[f];
        std::memset(&d, 0, sizeof(d));
        d.src = frames[f].d;
        d.T = planes + off[f];
        d.L = d.T + (size_t)n_g * plane;
        d.Ddbg = (dbg_D && f == 0) ? d.L + (size_t)n_g * plane : nullptr;
        d.src_stride = frames[f].stride;
        d.pitch = pitch[f];
        d.H = frames[f].H;
        d.W = frames[f].W;
        d.ladder = 0;
        d.frame_id = f;
    }
    if (pitch0)
        *pitch0 = pitch[0];
    if (L0)
        *L0 = fd[0].L;
    if (D0)
        *D0 = fd[0].Ddbg;
    const size_t frames_bytes = sizeof(FrameDesc) * n;

    // events recorded inside a graph cannot be timed, so per-kernel timing
    // issues the same sequence directly.  A layout is captured into a graph
    // the second time in a row it is seen (a stream of ever-changing batch
    // compositions is launched directly instead of re-capturing each time).
    std::vector<long long> key = launch_key(c, P, frames, dbg_D);
    const bool have_graph = c->graph_exec != nullptr && key == c->graph_key;
    // one frame goes inline in the kernel arguments and is launched directly
    // (its pixel pointer would otherwise be baked into a graph)
    const bool inline_one = n == 1;
    const bool use_graph = c->use_graphs && !c->profiling && !inline_one &&
                           (have_graph || key == c->seen_key);
    c->seen_key = key;
    const bool tables_ok = c->tables_ready && key == c->graph_key;
    if (!tables_ok || (use_graph && !have_graph)) {
        drop_graph(c);
        // ---- tile tables.  Each (frame, plane) unit's column blocks are cut
        // into DOG_NXCD contiguous slices and slice s goes to XCD (s + frame) %
        // DOG_NXCD, so one XCD's L2 holds one band of columns of every plane
        // (small frames spread over the XCDs).  The local-maximum tiles are
        // sliced by bands instead: their 62-column windows are not aligned to
        // cache lines, and a line shared by two column blocks on different
        // XCDs was fetched twice (1.32 x the planes' bytes; 1.02 x by bands).  Per XCD, tiles are ordered
        // widest kernel first; the launch table interleaves the XCD lists so
        // workgroup b (dispatched to XCD b % 8) gets a tile of list b % 8, and
        // an exhausted list's slot is filled from the longest remaining list.
        const int band = V.band();
        struct Raw {
            int frame, plane, count, n_cb, n_band, cost;
        };
        std::vector<Raw> r1, r2, r3;
        for (int f = 0; f < n; ++f) {
            const int H = frames[f].H, W = frames[f].W;
            std::vector<int> direct;   // planes blurred directly, widest first
            for (int p = n_g - 1; p >= 0; --p)
                if (std::find(dctp[f].begin(), dctp[f].end(), p) == dctp[f].end())
                    direct.push_back(p);
            for (const PlaneRun& u : plane_runs(P, direct, V.S, V.group != 0)) {
                r1.push_back({f, u.top, u.count, (W + 63) / 64, (H + band - 1) / band, u.cost});
                r2.push_back({f, u.top, u.count, (H + 63) / 64, (W + band - 1) / band, u.cost});
            }
            r3.push_back({f, 0, 1, (H + DOG_NMS_COLS - 1) / DOG_NMS_COLS,
                          (W + V.nms_band() - 1) / V.nms_band(), 0});
        }
        auto by_cost = [](const Raw& a, const Raw& b) {
            if (a.cost != b.cost)
                return a.cost > b.cost;
            return a.frame < b.frame;
        };
        std::stable_sort(r1.begin(), r1.end(), by_cost);
        std::stable_sort(r2.begin(), r2.end(), by_cost);
        // slice_bands: cut the bands (the planes' row direction) into the
        // slices instead, the column blocks of a band side by side, so the
        // cache lines that neighbouring column blocks share stay in one L2
        auto build_table = [](const std::vector<Raw>& raw, std::vector<Tile>* outt,
                              bool slice_bands) {
            std::vector<Tile> per[DOG_NXCD];
            for (const Raw& r : raw) {
                const int n_sl = slice_bands ? r.n_band : r.n_cb;
                for (int sl = 0; sl < DOG_NXCD; ++sl) {
                    const int c0 = (int)((long long)sl * n_sl / DOG_NXCD);
                    const int c1 = (int)((long long)(sl + 1) * n_sl / DOG_NXCD);
                    const int x = (sl + r.frame) % DOG_NXCD;
                    for (int o = c0; o < c1; ++o)
                        for (int i = 0; i < (slice_bands ? r.n_cb : r.n_band); ++i) {
                            Tile t;
                            t.frame = (uint16_t)r.frame;
                            t.plane = (uint8_t)r.plane;
                            t.n_planes = (uint8_t)r.count;
                            t.cb = (uint16_t)(slice_bands ? i : o);
                            t.band = (uint16_t)(slice_bands ? o : i);
                            per[x].push_back(t);
                        }
                }
            }
            size_t tot = 0, pos[DOG_NXCD] = {0};
            for (int x = 0; x < DOG_NXCD; ++x)
                tot += per[x].size();
            outt->clear();
            outt->reserve(tot);
            while (outt->size() < tot) {
                for (int x = 0; x < DOG_NXCD && outt->size() < tot; ++x) {
                    int src = x;
                    if (pos[x] >= per[x].size()) {
                        size_t best = 0;
                        for (int y = 0; y < DOG_NXCD; ++y)
                            if (per[y].size() - pos[y] > best) {
                                best = per[y].size() - pos[y];
                                src = y;
                            }
                    }
                    outt->push_back(per[src][pos[src]++]);
                }
            }
        };
        std::vector<Tile> tb1, tb2, tb3;
        build_table(r1, &tb1, false);
        build_table(r2, &tb2, false);
        build_table(r3, &tb3, true);

        // reflected row offsets (bytes) for both blur passes: row t of the
        // table is refl(t - pad) of the plane; one table per distinct shape
        const int rmax = *std::max_element(P.r.begin(), P.r.end());
        const int pad = rmax + (dogk_variant_ring(c->variant) + 1) * V.S;
        std::vector<int> rowtab;
        std::vector<size_t> rows1_off(n), rows2_off(n);
        {
            std::vector<std::pair<std::pair<long long, long long>, size_t>> seen;
            auto table_for = [&](long long nrows, long long pitch_b) {
                for (auto& e : seen)
                    if (e.first.first == nrows && e.first.second == pitch_b)
                        return e.second;
                const size_t at = rowtab.size();
                for (long long t = -pad; t < nrows + pad; ++t)
                    rowtab.push_back((int)(reflect_index(t, nrows) * pitch_b));
                while (rowtab.size() % 64)
                    rowtab.push_back(0);
                seen.push_back({{nrows, pitch_b}, at});
                return at;
            };
            for (int f = 0; f < n; ++f) {
                rows1_off[f] = table_for(frames[f].H, frames[f].stride * 4);
                rows2_off[f] = table_for(frames[f].W, pitch[f] * 4);
            }
        }
        // transform-domain tables: per line length the twiddles, per (length,
        // plane) the kernel's transfer function over N, and the jobs of the
        // two launches (float offsets into one host array first)
        std::vector<float> dtab;                       // twiddles and H vectors
        std::vector<FftJob> djobs[2][6];               // per pass and log2 N - 6
        struct TabRef {
            int N, p;
            size_t at;
        };
        std::vector<TabRef> tw_at, h_at;
        if (c->fft_cache_gen != c->plan_gen) {
            c->fft_transfer.clear();
            c->fft_cache_gen = c->plan_gen;
        }
        auto twiddles = [&](int N) {
            for (const TabRef& t : tw_at)
                if (t.N == N)
                    return t.at;
            std::vector<float>& v = c->fft_twiddles[N];
            if (v.empty()) {
                for (int t = 0; t < N / 2; ++t) {
                    const double a = -2.0 * M_PI * (double)t / (double)N;
                    v.push_back((float)std::cos(a));
                    v.push_back((float)std::sin(a));
                }
                for (int k = 0; k < N; ++k) {
                    const double a = -M_PI * (double)k / (2.0 * (double)N);
                    v.push_back((float)std::cos(a));
                    v.push_back((float)std::sin(a));
                }
                // wave jobs' per-lane factors: W_N^(l 2^i) for 2^i < E, then
                // W_64^((l mod B) 2^i) for 2^i < A, rows of 64 lanes
                const int lgn = ilog2(N);
                if (fft_wave_len(lgn)) {
                    const int E = N / 64, A = E >= 16 ? 16 : 8, B = 64 / A;
                    auto push = [&](long long t, long long period) {
                        const double a = -2.0 * M_PI * (double)(t % period) / (double)period;
                        v.push_back((float)std::cos(a));
                        v.push_back((float)std::sin(a));
                    };
                    for (int k = 1; k < E; k *= 2)
                        for (int l = 0; l < 64; ++l)
                            push((long long)l * k, N);
                    for (int c = 1; c < A; c *= 2)
                        for (int l = 0; l < 64; ++l)
                            push((long long)(l % B) * c, 64);
                }
            }
            const size_t at = dtab.size();
            dtab.insert(dtab.end(), v.begin(), v.end());
            while (dtab.size() % 64)
                dtab.push_back(0.0f);
            tw_at.push_back({N, 0, at});
            return at;
        };
        auto transfer = [&](int N, int p) {
            for (const TabRef& t : h_at)
                if (t.N == N && t.p == p)
                    return t.at;
            std::vector<float>& v = c->fft_transfer[{N, p}];
            if (v.empty()) {
                const std::vector<double> h = dct_transfer(P.half64[p], N);
                for (int k = 0; k < N; ++k)
                    v.push_back((float)(h[k] / (double)N));
            }
            const size_t at = dtab.size();
            dtab.insert(dtab.end(), v.begin(), v.end());
            while (dtab.size() % 64)
                dtab.push_back(0.0f);
            h_at.push_back({N, p, at});
            return at;
        };
        // table pointers are fixed up once the device table's offset is known
        // jobs name their twiddles and plane set by offset until the device
        // table's layout is known; plane sets name their transfer functions
        struct Fix {
            int pass, lg;
            size_t job, tw, set;
        };
        struct SetFix {
            int n_h;
            size_t h[kFftMaxPlanes];
        };
        std::vector<Fix> fixes;
        std::vector<FftPlaneSet> psets;
        std::vector<SetFix> set_fixes;
        const bool wide_src = key[0] != 0;   // frames' rows allow 16-byte loads
        FftLaunch fl{};
        fl.vec[0] = wide_src ? 1 : 0;
        fl.vec[1] = 1;                       // U planes: row pitch W, a power of two
        for (int f = 0; f < n; ++f) {
            if (dctp[f].empty())
                continue;
            const int H = frames[f].H, W = frames[f].W;
            const long long pt = pitch[f];
            const size_t plane = (size_t)W * (size_t)pt;
            float* T0 = planes + off[f];
            float* L0 = T0 + (size_t)n_g * plane;
            // the transform-domain planes blur along x first: pass 1 takes the
            // frame's rows (N = W) to rows of U_p, U_p[y][x] at row pitch W
            // in the slot of T_p (H W <= W pt floats); pass 2 takes the
            // columns of U_p (N = H) to rows of L_p, the transposed layout of
            // the direct blur.  Every store writes whole rows; only pass 2
            // reads across rows.  Pass 1 shares one forward transform among
            // up to kFftMaxPlanes planes (one for lines that run one job per
            // wavefront: the repeated forward transform costs less than
            // holding the coefficients across the inverse ones).
            // Jobs go row pair by row pair, the plane groups of a pair side
            // by side, so the groups re-reading a pair run on one XCD.
            const int per_job = fft_wave_len(ilog2(W)) ? 1 : kFftMaxPlanes;
            const int lg1 = ilog2(W) - 6;
            const size_t tw1 = twiddles(W);
            std::vector<size_t> sets1;
            std::vector<int> sizes1;
            for (size_t g0 = 0; g0 < dctp[f].size(); g0 += per_job) {
                const int ng = (int)std::min<size_t>(per_job, dctp[f].size() - g0);
                FftPlaneSet ps{};
                SetFix sf{ng, {}};
                for (int q = 0; q < ng; ++q) {
                    const int p = dctp[f][g0 + q];
                    ps.out[q] = T0 + (size_t)p * plane;
                    sf.h[q] = transfer(W, p);
                }
                sets1.push_back(psets.size());
                sizes1.push_back(ng);
                psets.push_back(ps);
                set_fixes.push_back(sf);
            }
            for (int l0 = 0; l0 < H; l0 += kFftLines)
                for (size_t g = 0; g < sets1.size(); ++g) {
                    FftJob j{};
                    j.in = nullptr;
                    j.in_rows = 1;
                    j.N = W;
                    j.line0 = l0;
                    j.frame = f;
                    j.n_planes = sizes1[g];
                    j.out_pitch = W;
                    fixes.push_back({0, lg1, djobs[0][lg1].size(), tw1, sets1[g]});
                    djobs[0][lg1].push_back(j);
                }
            for (int p : dctp[f]) {
                FftPlaneSet ps{};
                ps.out[0] = L0 + (size_t)p * plane;
                SetFix sf{1, {}};
                sf.h[0] = transfer(H, p);
                const size_t set = psets.size();
                psets.push_back(ps);
                set_fixes.push_back(sf);
                const int lg = ilog2(H) - 6;
                const size_t tw = twiddles(H);
                for (int l0 = 0; l0 < W; l0 += kFftLines) {
                    FftJob j{};
                    j.in = T0 + (size_t)p * plane;
                    j.in_pitch = W;
                    j.in_rows = 0;
                    j.N = H;
                    j.line0 = l0;
                    j.frame = f;
                    j.n_planes = 1;
                    j.out_pitch = (int)pt;
                    fixes.push_back({1, lg, djobs[1][lg].size(), tw, set});
                    djobs[1][lg].push_back(j);
                }
            }
        }
        // a pass whose jobs all have one line length the variant's blur
        // kernels take runs them in its own launch, first, XCD-local, padded
        // with empty jobs to whole rounds of the XCDs (so the tiles after
        // them keep their XCD placement)
        std::vector<FftJob> mjobs[2];
        for (int i = 0; i < 2; ++i) {
            int only = -1, kinds = 0;
            for (int lg = 0; lg < 6; ++lg)
                if (!djobs[i][lg].empty()) {
                    only = lg;
                    ++kinds;
                }
            if (kinds == 1 && dogk_variant_merges_fft(c->variant, only + 6))
                fl.merged_logn[i] = only + 6;
            for (int lg = 0; lg < 6; ++lg)
                fl.n[i][lg] = fl.merged_logn[i] == lg + 6 ? 0 : (int)djobs[i][lg].size();
        }

        const long long t1 = (long long)tb1.size(), t2 = (long long)tb2.size(),
                        t3 = (long long)tb3.size();
        if (t1 > INT32_MAX / 2 || t2 > INT32_MAX / 2 || t3 > INT32_MAX / 2 || n > 65535) {
            set_error("batch too large for one launch");
            return DOG_EINVAL;
        }

        const size_t o_frames = 0;
        const size_t o_ladder = align_up(o_frames + frames_bytes, 256);
        const size_t o_weights = align_up(o_ladder + sizeof(LadderDesc), 256);
        const size_t o_t1 = align_up(o_weights + sizeof(float) * P.weights.size(), 256);
        const size_t o_t2 = align_up(o_t1 + sizeof(Tile) * tb1.size(), 256);
        const size_t o_t3 = align_up(o_t2 + sizeof(Tile) * tb2.size(), 256);
        const size_t o_rows = align_up(o_t3 + sizeof(Tile) * tb3.size(), 256);
        const size_t o_dtab = align_up(o_rows + sizeof(int) * rowtab.size(), 256);
        const size_t o_psets = align_up(o_dtab + sizeof(float) * dtab.size(), 256);
        size_t o_djobs[2][6];
        size_t o_end = align_up(o_psets + sizeof(FftPlaneSet) * psets.size(), 256);
        for (int i = 0; i < 2; ++i)
            for (int lg = 0; lg < 6; ++lg) {
                o_djobs[i][lg] = o_end;
                const size_t padded =
                    grouped_jobs(djobs[i][lg].size(), fft_jobs_per_group(lg + 6),
                                 fl.merged_logn[i] == lg + 6 ? DOG_NXCD : 1);
                o_end = align_up(o_end + sizeof(FftJob) * padded, 256);
            }
        const size_t tbytes = o_end;
        if ((rc = ctx_alloc(c, &c->tables, tbytes, "launch tables")) != DOG_OK)
            return rc;
        if ((rc = ctx_pin(&c->h_tables, tbytes)) != DOG_OK)
            return rc;
        if ((rc = ctx_pin(&c->h_ends, sizeof(uint32_t) * tb3.size())) != DOG_OK)
            return rc;
        key = launch_key(c, P, frames, dbg_D);  // buffers may have moved
        c->seen_key = key;
        char* dt = static_cast<char*>(c->tables.p);
        char* h = static_cast<char*>(c->h_tables.p);
        const int* drows = reinterpret_cast<const int*>(dt + o_rows);
        c->frame_rows.assign(2 * (size_t)n, nullptr);
        for (int f = 0; f < n; ++f) {
            c->frame_rows[2 * f] = drows + rows1_off[f];
            c->frame_rows[2 * f + 1] = drows + rows2_off[f];
            fd[f].rows1 = drows + rows1_off[f];
            fd[f].rows2 = drows + rows2_off[f];
            fd[f].pad = pad;
        }
        c->row_pad = pad;
        std::memcpy(h + o_frames, fd.data(), frames_bytes);
        std::memcpy(h + o_ladder, &P.desc, sizeof(LadderDesc));
        std::memcpy(h + o_weights, P.weights.data(), sizeof(float) * P.weights.size());
        std::memcpy(h + o_t1, tb1.data(), sizeof(Tile) * tb1.size());
        std::memcpy(h + o_t2, tb2.data(), sizeof(Tile) * tb2.size());
        std::memcpy(h + o_t3, tb3.data(), sizeof(Tile) * tb3.size());
        std::memcpy(h + o_rows, rowtab.data(), sizeof(int) * rowtab.size());
        std::memcpy(h + o_dtab, dtab.data(), sizeof(float) * dtab.size());
        {
            const float* dt_f = reinterpret_cast<const float*>(dt + o_dtab);
            const FftPlaneSet* d_sets = reinterpret_cast<const FftPlaneSet*>(dt + o_psets);
            for (size_t q = 0; q < psets.size(); ++q)
                for (int i = 0; i < set_fixes[q].n_h; ++i)
                    psets[q].h[i] = dt_f + set_fixes[q].h[i];
            std::memcpy(h + o_psets, psets.data(), sizeof(FftPlaneSet) * psets.size());
            for (const Fix& fx : fixes) {
                FftJob& j = djobs[fx.pass][fx.lg][fx.job];
                j.tw = reinterpret_cast<const float2*>(dt_f + fx.tw);
                j.post = reinterpret_cast<const float2*>(dt_f + fx.tw + (size_t)j.N);
                j.planes = d_sets + fx.set;
            }
            for (int i = 0; i < 2; ++i)
                for (int lg = 0; lg < 6; ++lg) {
                    // merged: whole rounds of the XCDs, so the tiles after
                    // the jobs keep their XCD placement
                    const bool merged = fl.merged_logn[i] == lg + 6;
                    djobs[i][lg] = group_jobs(djobs[i][lg], fft_jobs_per_group(lg + 6),
                                              merged ? DOG_NXCD : 1);
                    if (fft_wave_len(lg + 6))
                        mark_column_groups(djobs[i][lg]);
                    if (merged)
                        mjobs[i] = djobs[i][lg];
                    else
                        fl.n[i][lg] = (int)djobs[i][lg].size();
                    std::memcpy(h + o_djobs[i][lg], djobs[i][lg].data(),
                                sizeof(FftJob) * djobs[i][lg].size());
                    fl.jobs[i][lg] = dt + o_djobs[i][lg];
                }
        }
        c->fft = fl;
        DOG_HIP(hipMemcpyAsync(c->tables.p, h, tbytes, hipMemcpyHostToDevice, c->stream));
        DOG_HIP(hipStreamSynchronize(c->stream));

        LaunchArgs& a = c->args;
        std::memset(&a, 0, sizeof(a));
        a.frames = reinterpret_cast<const FrameDesc*>(dt + o_frames);
        a.ladders = reinterpret_cast<const LadderDesc*>(dt + o_ladder);
        a.weights = reinterpret_cast<const float*>(dt + o_weights);
        a.tiles1 = reinterpret_cast<const Tile*>(dt + o_t1);
        a.tiles2 = reinterpret_cast<const Tile*>(dt + o_t2);
        a.tiles3 = reinterpret_cast<const Tile*>(dt + o_t3);
        a.cand = static_cast<CandHeader*>(c->cand.p);
        a.cap = c->cap;
        a.n1 = (int)t1;
        a.n2 = (int)t2;
        a.n3 = (int)t3;
        for (int i = 0; i < 2; ++i) {
            const int lg = fl.merged_logn[i] - 6;
            a.fft_jobs[i] = lg >= 0 ? static_cast<const FftJob*>(fl.jobs[i][lg]) : nullptr;
            a.n_fft[i] = lg >= 0 ? (int)mjobs[i].size() / fft_jobs_per_group(lg + 6) : 0;
        }
        c->n_gauss = n_g;
        c->debug_planes = dbg_D;
        c->wide1 = key[0] != 0;
        // readback size fixed in the captured sequence: header + a guess of
        // the record count (more is copied afterwards if needed)
        c->guess = std::min<uint32_t>(
            c->cap, std::max<uint32_t>(2048, c->last_count + c->last_count / 2 + 256));

        if (c->profiling) {
            for (int i = 0; i < 2 * DOG_NKERNELS; ++i)
                if (!c->ev[i])
                    DOG_HIP(hipEventCreate(&c->ev[i]));
        }
        c->frames_bytes = frames_bytes;
        if (use_graph) {
            // capture: frame table upload and the three kernels
            DOG_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue_sequence(c, c->stream, nullptr);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
            if (e != hipSuccess) {
                if (g)
                    (void)hipGraphDestroy(g);
                return hip_fail(e, "capture of the launch sequence");
            }
            DOG_HIP(e2);
            c->graph = g;
            DOG_HIP(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
        }
        c->graph_key = key;
        c->tables_ready = true;
    } else {
        for (int f = 0; f < n; ++f) {
            fd[f].rows1 = c->frame_rows[2 * f];
            fd[f].rows2 = c->frame_rows[2 * f + 1];
            fd[f].pad = c->row_pad;
        }
        std::memcpy(c->h_tables.p, fd.data(), frames_bytes);
    }

    // ---- run on the caller's stream (NULL: the null stream), so the
    // sequence is ordered after the work that produced the input without a
    // cross-stream event.  The context takes no other work until the launch
    // is collected, so the workspace is never shared by two streams at once
    const hipStream_t st = s;
    uint32_t* ends = static_cast<uint32_t*>(c->h_ends.p);
    const int n3 = c->args.n3;
    for (int i = 0; i < n3; ++i)
        ends[i] = kUnpublished;
    if (use_graph && c->graph_exec)
        DOG_HIP(hipGraphLaunch(c->graph_exec, st));
    else
        DOG_HIP(enqueue_sequence(c, st, inline_one ? &fd[0] : nullptr));
    if ((rc = record_done(c, st)) != DOG_OK)
        return rc;
    c->pend_inline = inline_one;
    c->pend_f0 = fd[0];
    c->pend_stream = st;
    c->pending = true;
    return DOG_OK;
}

int collect_frames(dog_context* c, const Plan& P, std::vector<std::vector<dog_blob>>* out)
{
    if (!c->pending) {
        set_error("no launch to collect");
        return DOG_EINVAL;
    }
    c->pending = false;
    const int n = c->pend_n;
    out->assign(n, {});
    if (n == 0)
        return DOG_OK;
    const bool inline_one = c->pend_inline;
    const hipStream_t st = c->pend_stream;
    const int n_g = P.n_g;
    int rc = wait_done(c);
    if (rc != DOG_OK)
        return rc;
    uint32_t* ends = static_cast<uint32_t*>(c->h_ends.p);
    const int n3 = c->args.n3;
    LaunchArgs a = c->args;
    host_targets(c, &a);
    const uint32_t guess = c->guess;
    uint32_t count = 0;
    for (int i = 0; i < n3; ++i) {
        if (ends[i] == kUnpublished) {
            set_error("a local-maximum workgroup did not publish its candidate range");
            return DOG_EDEVICE;
        }
        count = std::max(count, ends[i]);
    }
    if (c->profiling) {
        // kernels that were launched: pass 1 and 2 when they had tiles or
        // transform jobs of their own, the local maxima, the transform-domain
        // launches that had jobs
        const bool ran[DOG_NKERNELS] = {c->args.n1 + c->args.n_fft[0] > 0,
                                        c->args.n2 + c->args.n_fft[1] > 0, true,
                                        c->fft.total(0) > 0, c->fft.total(1) > 0};
        for (int i = 0; i < DOG_NKERNELS; ++i) {
            if (!ran[i])
                continue;
            float ms = 0.0f;
            DOG_HIP(hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
            c->kernel_ms[i] += ms;
        }
        c->kernel_launches += 1;
    }
    if (count > c->cap) {
        // overflow: enlarge the record buffer and rerun only the local-maximum
        // kernel; the planes are still in the workspace
        const uint32_t newcap = count + count / 4 + 1024;
        if ((rc = ctx_alloc(c, &c->cand, sizeof(CandHeader) + kRecBytes * (size_t)newcap,
                            "candidates")) != DOG_OK)
            return rc;
        c->cap = newcap;
        if ((rc = ctx_pin(&c->h_cand, sizeof(CandHeader) + kRecBytes * (size_t)newcap)) != DOG_OK)
            return rc;
        drop_graph(c);  // points at the old buffers
        a.cand = static_cast<CandHeader*>(c->cand.p);
        a.cap = c->cap;
        host_targets(c, &a);
        if (inline_one) {
            a.frames = nullptr;
            a.f0 = c->pend_f0;
        }
        DOG_HIP(dogk_fill_u32(&a.cand->count, 1, 0u, st));
        DOG_HIP(dogk_launch_nms(c->variant, &a, a.n3, n_g, c->debug_planes ? 1 : 0, st));
        DOG_HIP(hipMemcpyAsync(c->h_cand.p, c->cand.p, sizeof(CandHeader) + kRecBytes * count,
                               hipMemcpyDeviceToHost, st));
        DOG_HIP(hipStreamSynchronize(st));
        const uint32_t again = static_cast<CandHeader*>(c->h_cand.p)->count;
        if (again != count) {
            set_error("candidate count changed between identical launches");
            return DOG_EDEVICE;
        }
    } else if (count > guess) {
        char* hb = static_cast<char*>(c->h_cand.p) + sizeof(CandHeader) + kRecBytes * guess;
        const char* db = static_cast<const char*>(c->cand.p) + sizeof(CandHeader) + kRecBytes * guess;
        DOG_HIP(hipMemcpyAsync(hb, db, kRecBytes * (count - guess), hipMemcpyDeviceToHost, st));
        DOG_HIP(hipStreamSynchronize(st));
    }
    c->last_count = count;

    const CandRec* recs = reinterpret_cast<const CandRec*>(static_cast<char*>(c->h_cand.p) +
                                                           sizeof(CandHeader));
    for (uint32_t i = 0; i < count; ++i) {
        const CandRec& r = recs[i];
        if (r.frame < 0 || r.frame >= n || r.scale < 0 || r.scale >= P.k) {
            set_error("corrupt candidate record");
            return DOG_EDEVICE;
        }
        dog_blob b;
        b.y = r.y;
        b.x = r.x;
        b.scale = r.scale;
        b.sigma = (float)P.sigma[r.scale];
        b.response = r.response;
        (*out)[r.frame].push_back(b);
    }
    for (auto& v : *out)
        sort_blobs(v);
    return DOG_OK;
}

int run_frames(dog_context* c, const Plan& P, const std::vector<FrameIn>& frames, hipStream_t s,
               std::vector<std::vector<dog_blob>>* out, bool dbg_D, long long* pitch0,
               float** L0, float** D0)
{
    const int rc = launch_frames(c, P, frames, s, dbg_D, pitch0, L0, D0);
    if (rc != DOG_OK)
        return rc;
    return collect_frames(c, P, out);
}

}  // namespace dog
