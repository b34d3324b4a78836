// Host runtime: contexts, device workspace, launch tables and the launch of
// the three-kernel sequence (pass 1, pass 2, local maxima) over a list of
// frames, then the readback of the candidate records.
#include "runtime.h"

#include <algorithm>
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

int ctx_alloc(dog_context* c, DevBuf* b, size_t bytes, const char* what)
{
    if (b->bytes >= bytes)
        return DOG_OK;
    // grow geometrically so a sequence of slightly larger requests does not
    // reallocate every time
    size_t want = std::max(bytes, b->bytes + b->bytes / 4);
    want = (want + 4095) & ~(size_t)4095;
    const uint64_t after = c->used - b->bytes + want;
    if (after > c->budget) {
        want = (bytes + 4095) & ~(size_t)4095;
        if (c->used - b->bytes + want > c->budget) {
            set_error(std::string("HBM budget exceeded allocating ") + what + ": need " +
                      std::to_string(c->used - b->bytes + want) + " bytes, budget " +
                      std::to_string(c->budget));
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
    if (!c->have_plan || !same_params(c->plan.prm, *prm) || prm->truncate == 0.0) {
        Plan P;
        std::string err;
        const int rc = build_plan(*prm, &P, &err);
        if (rc != DOG_OK) {
            set_error(err);
            return rc;
        }
        c->plan = std::move(P);
        c->have_plan = true;
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
    c->variant = v;
    for (int i = 0; i < 3; ++i)
        c->occ[i] = std::max(1, o[i]);
    return DOG_OK;
}

static Variant variant_geometry(int v)
{
    Variant g;
    dogk_variant_geometry(v, &g.S, &g.NW, &g.BI, &g.BN, &g.NWN);
    return g;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static constexpr size_t kRecBytes = sizeof(CandRec);

int run_frames(dog_context* c, const Plan& P, const std::vector<FrameIn>& frames, hipStream_t s,
               std::vector<std::vector<dog_blob>>* out, bool dbg_D, long long* pitch0,
               float** L0, float** D0)
{
    const int n = (int)frames.size();
    out->assign(n, {});
    if (n == 0)
        return DOG_OK;
    const Variant V = variant_geometry(c->variant);
    const int n_g = P.n_g;

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
    float* planes = static_cast<float*>(c->planes.p);

    // ---- launch tables
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

    // ---- per-XCD work lists.  Each (frame, plane) unit's column blocks are
    // cut into DOG_NXCD contiguous slices; slice s goes to XCD (s + frame) %
    // DOG_NXCD so one XCD's L2 holds one band of columns of every plane (and
    // small frames spread over the XCDs).  Within a list, units are ordered
    // widest kernel first so the persistent grid drains evenly.
    const int band = V.band();
    struct Raw {
        int frame, plane, n_cb, n_band, radius;
    };
    std::vector<Raw> r1, r2, r3;
    for (int f = 0; f < n; ++f) {
        const int H = frames[f].H, W = frames[f].W;
        for (int p = 0; p < n_g; ++p) {
            r1.push_back({f, p, (W + 63) / 64, (H + band - 1) / band, P.r[p]});
            r2.push_back({f, p, (H + 63) / 64, (W + band - 1) / band, P.r[p]});
        }
        r3.push_back({f, 0, (H + DOG_NMS_COLS - 1) / DOG_NMS_COLS,
                      (W + V.nms_band() - 1) / V.nms_band(), 0});
    }
    auto by_cost = [](const Raw& a, const Raw& b) {
        if (a.radius != b.radius)
            return a.radius > b.radius;
        return a.frame < b.frame;
    };
    std::stable_sort(r1.begin(), r1.end(), by_cost);
    std::stable_sort(r2.begin(), r2.end(), by_cost);
    struct Lists {
        std::vector<WorkUnit> units;
        Queue q;
    };
    auto slice = [](const std::vector<Raw>& raw, Lists* L) -> bool {
        std::vector<WorkUnit> per[DOG_NXCD];
        long long tot[DOG_NXCD] = {0};
        for (const Raw& r : raw) {
            for (int s = 0; s < DOG_NXCD; ++s) {
                const int c0 = (int)((long long)s * r.n_cb / DOG_NXCD);
                const int c1 = (int)((long long)(s + 1) * r.n_cb / DOG_NXCD);
                if (c1 <= c0)
                    continue;
                const int x = (s + r.frame) % DOG_NXCD;
                WorkUnit w{};
                w.frame = r.frame;
                w.plane = r.plane;
                w.cb0 = c0;
                w.n_cb = c1 - c0;
                w.n_band = r.n_band;
                w.first_tile = (int)tot[x];
                tot[x] += (long long)w.n_cb * w.n_band;
                per[x].push_back(w);
            }
        }
        L->units.clear();
        std::memset(&L->q, 0, sizeof(L->q));
        for (int x = 0; x < DOG_NXCD; ++x) {
            if (tot[x] > INT32_MAX / 2)
                return false;
            L->q.off[x] = (int)L->units.size();
            L->q.n[x] = (int)per[x].size();
            L->q.total[x] = (int)tot[x];
            L->units.insert(L->units.end(), per[x].begin(), per[x].end());
        }
        return true;
    };
    Lists l1, l2, l3;
    if (!slice(r1, &l1) || !slice(r2, &l2) || !slice(r3, &l3)) {
        set_error("batch too large for one launch");
        return DOG_EINVAL;
    }
    long long t1 = 0, t2 = 0, t3 = 0;
    for (int x = 0; x < DOG_NXCD; ++x) {
        t1 += l1.q.total[x];
        t2 += l2.q.total[x];
        t3 += l3.q.total[x];
    }

    const size_t o_frames = 0;
    const size_t o_ladder = align_up(o_frames + sizeof(FrameDesc) * n, 256);
    const size_t o_weights = align_up(o_ladder + sizeof(LadderDesc), 256);
    const size_t o_queues = align_up(o_weights + sizeof(float) * P.weights.size(), 256);
    const size_t o_u1 = align_up(o_queues + sizeof(Queue) * 3, 256);
    const size_t o_u2 = align_up(o_u1 + sizeof(WorkUnit) * l1.units.size(), 256);
    const size_t o_u3 = align_up(o_u2 + sizeof(WorkUnit) * l2.units.size(), 256);
    const size_t tbytes = align_up(o_u3 + sizeof(WorkUnit) * l3.units.size(), 256);
    if ((rc = ctx_alloc(c, &c->tables, tbytes, "launch tables")) != DOG_OK)
        return rc;
    if ((rc = ctx_pin(&c->h_tables, tbytes)) != DOG_OK)
        return rc;
    char* dt = static_cast<char*>(c->tables.p);
    l1.q.units = reinterpret_cast<const WorkUnit*>(dt + o_u1);
    l2.q.units = reinterpret_cast<const WorkUnit*>(dt + o_u2);
    l3.q.units = reinterpret_cast<const WorkUnit*>(dt + o_u3);
    const Queue qs[3] = {l1.q, l2.q, l3.q};
    char* h = static_cast<char*>(c->h_tables.p);
    std::memcpy(h + o_frames, fd.data(), sizeof(FrameDesc) * n);
    std::memcpy(h + o_ladder, &P.desc, sizeof(LadderDesc));
    std::memcpy(h + o_weights, P.weights.data(), sizeof(float) * P.weights.size());
    std::memcpy(h + o_queues, qs, sizeof(qs));
    std::memcpy(h + o_u1, l1.units.data(), sizeof(WorkUnit) * l1.units.size());
    std::memcpy(h + o_u2, l2.units.data(), sizeof(WorkUnit) * l2.units.size());
    std::memcpy(h + o_u3, l3.units.data(), sizeof(WorkUnit) * l3.units.size());
    DOG_HIP(hipMemcpyAsync(c->tables.p, h, tbytes, hipMemcpyHostToDevice, s));

    // ---- candidate buffer
    if (c->cap == 0) {
        if ((rc = ctx_alloc(c, &c->cand, sizeof(CandHeader) + kRecBytes * 65536, "candidates")) !=
            DOG_OK)
            return rc;
        c->cap = 65536;
    }

    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.frames = reinterpret_cast<const FrameDesc*>(dt + o_frames);
    a.ladders = reinterpret_cast<const LadderDesc*>(dt + o_ladder);
    a.weights = reinterpret_cast<const float*>(dt + o_weights);
    a.queues = reinterpret_cast<const Queue*>(dt + o_queues);
    a.counters = static_cast<Counters*>(c->counters.p);
    a.cand = static_cast<CandHeader*>(c->cand.p);
    a.cap = c->cap;

    // persistent grids: resident capacity, a multiple of DOG_NXCD, no more
    // workgroups than tiles (rounded up to DOG_NXCD)
    auto grid = [&](int i, long long tiles) {
        long long g = c->grid_override > 0 ? c->grid_override : (long long)c->occ[i] * c->n_cu;
        const long long t8 = (tiles + DOG_NXCD - 1) / DOG_NXCD * DOG_NXCD;
        g = std::min(g, t8);
        g = g / DOG_NXCD * DOG_NXCD;
        return (int)std::max<long long>(DOG_NXCD, g);
    };
    if (c->profiling) {
        for (int i = 0; i < 4; ++i)
            if (!c->ev[i])
                DOG_HIP(hipEventCreate(&c->ev[i]));
    }
    DOG_HIP(dogk_launch_sequence(c->variant, &a, grid(0, t1), grid(1, t2), grid(2, t3), s,
                                 c->profiling ? c->ev : nullptr));

    // ---- readback: header + a guess of the records in one copy
    uint32_t guess = std::min<uint32_t>(c->cap, std::max<uint32_t>(4096, c->last_count + c->last_count / 4 + 256));
    if ((rc = ctx_pin(&c->h_cand, sizeof(CandHeader) + kRecBytes * (size_t)c->cap)) != DOG_OK)
        return rc;
    DOG_HIP(hipMemcpyAsync(c->h_cand.p, c->cand.p, sizeof(CandHeader) + kRecBytes * guess,
                           hipMemcpyDeviceToHost, s));
    DOG_HIP(hipStreamSynchronize(s));
    uint32_t count = static_cast<CandHeader*>(c->h_cand.p)->count;
    if (c->profiling) {
        for (int i = 0; i < 3; ++i) {
            float ms = 0.0f;
            DOG_HIP(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
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
        a.cand = static_cast<CandHeader*>(c->cand.p);
        a.cap = c->cap;
        DOG_HIP(dogk_fill_u32(a.counters->c[2], DOG_NXCD, 0u, s));
        DOG_HIP(dogk_fill_u32(&a.cand->count, 1, 0u, s));
        DOG_HIP(dogk_launch_nms(c->variant, &a, grid(2, t3), s));
        DOG_HIP(hipMemcpyAsync(c->h_cand.p, c->cand.p, sizeof(CandHeader) + kRecBytes * count,
                               hipMemcpyDeviceToHost, s));
        DOG_HIP(hipStreamSynchronize(s));
        const uint32_t again = static_cast<CandHeader*>(c->h_cand.p)->count;
        if (again != count) {
            set_error("candidate count changed between identical launches");
            return DOG_EDEVICE;
        }
    } else if (count > guess) {
        char* hb = static_cast<char*>(c->h_cand.p) + sizeof(CandHeader) + kRecBytes * guess;
        const char* db = static_cast<const char*>(c->cand.p) + sizeof(CandHeader) + kRecBytes * guess;
        DOG_HIP(hipMemcpyAsync(hb, db, kRecBytes * (count - guess), hipMemcpyDeviceToHost, s));
        DOG_HIP(hipStreamSynchronize(s));
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

}  // namespace dog
