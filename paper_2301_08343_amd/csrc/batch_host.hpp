// Host side of the batched multi-contact API (included at the end of
// tacchi.hip so it shares the single-contact helpers).
//
// A batch owns one single-contact handle per contact, each carved from its own
// range of the batch workspace, so state read-out (depth map, image,
// particles) goes through the ordinary calls. Substeps are advanced by the
// batched kernels of batch_kernels.hpp: contacts that share a tuning choice
// (grid block edge B, workgroup size, material model) form a group, and each
// phase of a substep is one launch per group. Runs of an even number of
// substeps are captured once as a HIP graph and replayed.
#include <fstream>
#include <map>
#include <sstream>

#include "batch_kernels.hpp"

struct tacchi_batch {
    int n = 0, nsteps = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<tacchi_config> cfgs;
    std::vector<tacchi_sim *> sims;
    std::vector<int> tile, wg, log2n;
    std::vector<double> dt;
    std::vector<double> traj;  // [n][nsteps+1][7]
    std::vector<size_t> ws_off, ws_len;
    char *ws = nullptr;
    SimDev<float> *descs[2] = {nullptr, nullptr};
    BatchConsts *consts = nullptr;
    IndenterDev<double> *itab = nullptr;
    int *step = nullptr;
    BatchItem *items = nullptr;
    struct Group {
        int B, WG, model;
        BatchItem *items;
        int count;
    };
    std::vector<Group> groups;
    int parity = 0;
    int64_t done = 0;
    int graph_len = 50;
    hipGraph_t graph_def[2] = {nullptr, nullptr};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    std::vector<double> tune_us;  // measured us/substep of the chosen setting per contact (0 = not tuned)
};

namespace {

struct BatchLayout {
    std::vector<size_t> off, len;
    size_t descs[2], consts, itab, step, items, total;
    int64_t max_items;
};

size_t contact_ws_bytes(const tacchi_config &c0)
{
    tacchi_config c = c0;
    size_t best = 0;
    for (int t : {4, 8}) {
        c.tile = t;
        Derived d;
        if (derive(&c, &d) != TACCHI_OK) return 0;
        best = std::max(best, make_layout(d).total);
    }
    return best;
}

tacchi_status batch_layout(const tacchi_config *cfgs, int n, int nsteps, BatchLayout *L)
{
    size_t o = 0;
    L->max_items = 0;
    for (int i = 0; i < n; ++i) {
        if (cfgs[i].precision != TACCHI_F32)
            return fail(TACCHI_E_ARG, "batched contacts run in FP32 (precision must be TACCHI_F32)");
        const size_t b = contact_ws_bytes(cfgs[i]);
        if (b == 0) return TACCHI_E_ARG;  // message set by derive
        L->off.push_back(o);
        L->len.push_back(b);
        o = align256(o + b);
        tacchi_config c = cfgs[i];
        c.tile = 4;  // the finer tiling has the most blocks
        Derived d;
        derive(&c, &d);
        L->max_items += d.nblk;
    }
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L->descs[0] = take((size_t)n * sizeof(SimDev<float>));
    L->descs[1] = take((size_t)n * sizeof(SimDev<float>));
    L->consts = take((size_t)n * sizeof(BatchConsts));
    L->itab = take((size_t)n * nsteps * sizeof(IndenterDev<double>));
    L->step = take(256);
    L->items = take((size_t)L->max_items * sizeof(BatchItem));
    L->total = o;
    return TACCHI_OK;
}

int ilog2(int64_t v)
{
    int r = 0;
    while ((v >> (r + 1)) > 0) ++r;
    return r;
}

std::string device_arch(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Tuning cache: a JSON object {"entries": [{"arch": ..., "precision": "f32",
// "log2n": L, "tile": B, "wg": W, "us_per_substep": t}, ...]}.
struct TuneEntry {
    std::string arch;
    int log2n, tile, wg;
    double us;
};

std::vector<TuneEntry> read_tune_cache(const char *path)
{
    std::vector<TuneEntry> out;
    if (!path || !*path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    auto field = [](const std::string &e, const char *key) -> std::string {
        const std::string k = std::string("\"") + key + "\"";
        size_t p = e.find(k);
        if (p == std::string::npos) return "";
        p = e.find(':', p);
        if (p == std::string::npos) return "";
        ++p;
        while (p < e.size() && (e[p] == ' ' || e[p] == '"')) ++p;
        size_t q = p;
        while (q < e.size() && e[q] != ',' && e[q] != '}' && e[q] != '"') ++q;
        return e.substr(p, q - p);
    };
    while ((pos = s.find('{', pos + 1)) != std::string::npos) {
        const size_t end = s.find('}', pos);
        if (end == std::string::npos) break;
        const std::string e = s.substr(pos, end - pos + 1);
        if (e.find("\"log2n\"") == std::string::npos) continue;
        TuneEntry t;
        t.arch = field(e, "arch");
        if (field(e, "precision") != "f32") continue;
        t.log2n = std::atoi(field(e, "log2n").c_str());
        t.tile = std::atoi(field(e, "tile").c_str());
        t.wg = std::atoi(field(e, "wg").c_str());
        t.us = std::atof(field(e, "us_per_substep").c_str());
        if ((t.tile == 4 || t.tile == 8) && (t.wg == 128 || t.wg == 256)) out.push_back(t);
    }
    return out;
}

bool write_tune_cache(const char *path, const std::vector<TuneEntry> &entries)
{
    std::ofstream f(path);
    if (!f) return false;
    f << "{\n  \"entries\": [\n";
    for (size_t i = 0; i < entries.size(); ++i) {
        const TuneEntry &t = entries[i];
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "    {\"arch\": \"%s\", \"precision\": \"f32\", \"log2n\": %d, \"tile\": %d, \"wg\": %d, "
                      "\"us_per_substep\": %.3f}%s\n",
                      t.arch.c_str(), t.log2n, t.tile, t.wg, t.us, i + 1 < entries.size() ? "," : "");
        f << buf;
    }
    f << "  ]\n}\n";
    return (bool)f;
}

template <int B, int MODEL, int WG>
void launch_group_phase(tacchi_batch *bt, const tacchi_batch::Group &g, int phase, int parity, int bump)
{
    const dim3 grid(g.count), blk(WG);
    // P2G at B = 8 always runs kP2GWG-thread workgroups, as in the
    // single-contact path: its LDS tile allows few workgroups per CU, so the
    // resident waves come from the workgroup size (the tuned size applies to
    // the grid update and G2P)
    constexpr int P2G_WG = B == 8 ? kP2GWG : WG;
    if (phase == 0)
        hipLaunchKernelGGL((k_p2g_batch<B, MODEL, P2G_WG>), grid, dim3(P2G_WG), 0, bt->stream, g.items,
                           bt->descs[parity], bt->consts, bt->step, bump);
    else if (phase == 1)
        hipLaunchKernelGGL((k_grid_batch<B, WG>), grid, blk, 0, bt->stream, g.items, bt->descs[parity], bt->consts,
                           bt->itab, bt->nsteps, bt->step);
    else
        hipLaunchKernelGGL((k_g2p_batch<B, MODEL, WG>), grid, blk, 0, bt->stream, g.items, bt->descs[parity],
                           bt->consts);
}

void launch_group(tacchi_batch *bt, const tacchi_batch::Group &g, int phase, int parity, int bump)
{
    const int key = (g.B == 4 ? 0 : 4) + (g.model ? 2 : 0) + (g.WG == 128 ? 0 : 1);
    switch (key) {
    case 0: launch_group_phase<4, 0, 128>(bt, g, phase, parity, bump); break;
    case 1: launch_group_phase<4, 0, 256>(bt, g, phase, parity, bump); break;
    case 2: launch_group_phase<4, 1, 128>(bt, g, phase, parity, bump); break;
    case 3: launch_group_phase<4, 1, 256>(bt, g, phase, parity, bump); break;
    case 4: launch_group_phase<8, 0, 128>(bt, g, phase, parity, bump); break;
    case 5: launch_group_phase<8, 0, 256>(bt, g, phase, parity, bump); break;
    case 6: launch_group_phase<8, 1, 128>(bt, g, phase, parity, bump); break;
    default: launch_group_phase<8, 1, 256>(bt, g, phase, parity, bump); break;
    }
}

tacchi_status batch_substep(tacchi_batch *bt, int parity)
{
    for (int phase = 0; phase < 3; ++phase)
        for (size_t gi = 0; gi < bt->groups.size(); ++gi) launch_group(bt, bt->groups[gi], phase, parity, gi == 0);
    TC_LAUNCHED();
    return TACCHI_OK;
}

// Creates contact i's handle on its workspace range with the given tile and
// uploads its two descriptors (one per bin-list parity).
tacchi_status batch_make_contact(tacchi_batch *bt, int i, int tile)
{
    if (bt->sims[i]) {
        tacchi_destroy(bt->sims[i]);
        bt->sims[i] = nullptr;
    }
    tacchi_config c = bt->cfgs[i];
    c.tile = tile;
    tacchi_status st = tacchi_create(&c, bt->ws + bt->ws_off[i], bt->ws_len[i], bt->stream, &bt->sims[i]);
    if (st) return st;
    tacchi_sim *s = bt->sims[i];
    SimDev<float> d[2];
    for (int p = 0; p < 2; ++p) {
        s->parity = p;
        d[p] = make_simdev<float>(s);
    }
    s->parity = 0;
    s->sf = make_simdev<float>(s);
    s->sd = make_simdev<double>(s);
    for (int p = 0; p < 2; ++p)
        TC_HIP(hipMemcpyAsync(bt->descs[p] + i, &d[p], sizeof(SimDev<float>), hipMemcpyHostToDevice, bt->stream));
    return TACCHI_OK;
}

// Work items of one group: every grid block of every contact in it.
tacchi_status batch_build_groups(tacchi_batch *bt)
{
    std::map<int, std::vector<int>> by_key;
    for (int i = 0; i < bt->n; ++i) {
        const int key = bt->tile[i] * 1000 + bt->wg[i] * 10 + bt->cfgs[i].mat.model;
        by_key[key].push_back(i);
    }
    std::vector<BatchItem> all;
    bt->groups.clear();
    std::vector<std::pair<size_t, size_t>> ranges;
    for (auto &kv : by_key) {
        const size_t start = all.size();
        for (int i : kv.second)
            for (int b = 0; b < bt->sims[i]->d.nblk; ++b) all.push_back({i, b});
        const int i0 = kv.second[0];
        bt->groups.push_back({bt->tile[i0], bt->wg[i0], bt->cfgs[i0].mat.model, nullptr, (int)(all.size() - start)});
        ranges.push_back({start, all.size() - start});
    }
    for (size_t g = 0; g < bt->groups.size(); ++g) bt->groups[g].items = bt->items + ranges[g].first;
    TC_HIP(hipMemcpyAsync(bt->items, all.data(), all.size() * sizeof(BatchItem), hipMemcpyHostToDevice, bt->stream));
    TC_HIP(hipStreamSynchronize(bt->stream));
    return TACCHI_OK;
}

tacchi_status batch_reset_step(tacchi_batch *bt)
{
    const int minus_one = -1;
    TC_HIP(hipMemcpyAsync(bt->step, &minus_one, sizeof(int), hipMemcpyHostToDevice, bt->stream));
    TC_HIP(hipStreamSynchronize(bt->stream));
    return TACCHI_OK;
}

// Times `reps` substeps of contact i alone with the given setting (after two
// warmup substeps) and returns microseconds per substep. The contact is
// re-created from its initial state before and after.
tacchi_status batch_time_setting(tacchi_batch *bt, int i, int tile, int wgs, double *us)
{
    tacchi_status st = batch_make_contact(bt, i, tile);
    if (st) return st;
    std::vector<BatchItem> its;
    for (int b = 0; b < bt->sims[i]->d.nblk; ++b) its.push_back({i, b});
    TC_HIP(hipMemcpyAsync(bt->items, its.data(), its.size() * sizeof(BatchItem), hipMemcpyHostToDevice, bt->stream));
    st = batch_reset_step(bt);
    if (st) return st;
    tacchi_batch::Group g{tile, wgs, bt->cfgs[i].mat.model, bt->items, (int)its.size()};
    hipEvent_t e0, e1;
    TC_HIP(hipEventCreate(&e0));
    TC_HIP(hipEventCreate(&e1));
    const int warm = 2, reps = std::min(10, std::max(1, bt->nsteps - warm));
    int parity = 0;
    for (int k = 0; k < warm + reps; ++k) {
        if (k == warm) (void)hipEventRecord(e0, bt->stream);
        for (int phase = 0; phase < 3; ++phase) launch_group(bt, g, phase, parity, 1);
        parity ^= 1;
    }
    (void)hipEventRecord(e1, bt->stream);
    TC_LAUNCHED();
    TC_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    TC_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1e3 * ms / reps;
    return batch_make_contact(bt, i, tile);
}

void batch_free(tacchi_batch *bt)
{
    for (int p = 0; p < 2; ++p) {
        if (bt->graph[p]) (void)hipGraphExecDestroy(bt->graph[p]);
        if (bt->graph_def[p]) (void)hipGraphDestroy(bt->graph_def[p]);
    }
    for (tacchi_sim *s : bt->sims)
        if (s) tacchi_destroy(s);
    delete bt;
}

}  // namespace

extern "C" {

size_t tacchi_batch_workspace_bytes(const tacchi_config *cfgs, int32_t n, int32_t substeps)
{
    if (!cfgs || n < 1 || substeps < 1) {
        fail(TACCHI_E_ARG, "need at least one contact and one substep");
        return 0;
    }
    BatchLayout L;
    if (batch_layout(cfgs, n, substeps, &L) != TACCHI_OK) return 0;
    return L.total;
}

tacchi_status tacchi_batch_create(const tacchi_config *cfgs, int32_t n, const tacchi_pose *traj, const double *dt,
                                  int32_t substeps, const char *tune_cache, int32_t tune, void *dev_ws,
                                  size_t ws_bytes, void *hip_stream, tacchi_batch **out)
{
    if (!out || !cfgs || !traj || !dt || n < 1 || substeps < 1) return fail(TACCHI_E_ARG, "bad batch arguments");
    *out = nullptr;
    BatchLayout L;
    tacchi_status st = batch_layout(cfgs, n, substeps, &L);
    if (st) return st;
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(TACCHI_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < L.total) return fail(TACCHI_E_WORKSPACE, "batch workspace too small");
    tacchi_batch *bt = new (std::nothrow) tacchi_batch();
    if (!bt) return fail(TACCHI_E_ARG, "out of host memory");
    bt->n = n;
    bt->nsteps = substeps;
    bt->stream = (hipStream_t)hip_stream;
    bt->ws = (char *)dev_ws;
    bt->cfgs.assign(cfgs, cfgs + n);
    bt->sims.assign(n, nullptr);
    bt->tile.assign(n, 8);
    bt->wg.assign(n, 256);
    bt->tune_us.assign(n, 0.0);
    bt->dt.assign(dt, dt + n);
    bt->ws_off = L.off;
    bt->ws_len = L.len;
    bt->descs[0] = (SimDev<float> *)(bt->ws + L.descs[0]);
    bt->descs[1] = (SimDev<float> *)(bt->ws + L.descs[1]);
    bt->consts = (BatchConsts *)(bt->ws + L.consts);
    bt->itab = (IndenterDev<double> *)(bt->ws + L.itab);
    bt->step = (int *)(bt->ws + L.step);
    bt->items = (BatchItem *)(bt->ws + L.items);
    auto bail = [&](tacchi_status e) {
        batch_free(bt);
        return e;
    };
    if (hipGetDevice(&bt->device) != hipSuccess) return bail(fail(TACCHI_E_DEVICE, "hipGetDevice failed"));
    // trajectories, constants and the indenter table
    bt->traj.resize((size_t)n * (substeps + 1) * 7);
    std::vector<BatchConsts> cc(n);
    std::vector<IndenterDev<double>> itab((size_t)n * substeps);
    for (int i = 0; i < n; ++i) {
        Derived d;
        derive(&cfgs[i], &d);
        bt->log2n.push_back(ilog2(d.N));
        const double cfl = dt[i] * d.cp / d.dx;
        if (!(dt[i] > 0) || cfl > 1.0) return bail(fail(TACCHI_E_UNSTABLE, "a contact's dt is <= 0 or above the CFL limit"));
        for (int k = 0; k <= substeps; ++k) {
            const tacchi_pose &p = traj[(size_t)i * (substeps + 1) + k];
            double *q = &bt->traj[((size_t)i * (substeps + 1) + k) * 7];
            std::memcpy(q, p.pos, 3 * sizeof(double));
            std::memcpy(q + 3, p.quat, 4 * sizeof(double));
        }
        for (int k = 0; k < substeps; ++k) {
            const double *q0 = &bt->traj[((size_t)i * (substeps + 1) + k) * 7];
            itab[(size_t)i * substeps + k] = make_indenter<double>(cfgs[i], q0, q0 + 7, dt[i]);
        }
        const double one = kFixedUnits;  // see P2GScales
        cc[i] = {(float)dt[i], (float)(dt[i] * d.V0 * 4.0 / (d.dx * d.dx)), (float)(one / d.m),
                 (float)(one * dt[i] / d.m), (float)(d.m / one), (float)(d.m / (one * dt[i]))};
    }
    if (hipMemcpyAsync(bt->consts, cc.data(), n * sizeof(BatchConsts), hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
        hipMemcpyAsync(bt->itab, itab.data(), itab.size() * sizeof(IndenterDev<double>), hipMemcpyHostToDevice,
                       bt->stream) != hipSuccess)
        return bail(fail(TACCHI_E_DEVICE, "upload of the batch tables failed"));
    // tuning: cached choices, else timed sweeps per particle-count class
    const std::string arch = device_arch(bt->device);
    std::vector<TuneEntry> cache = read_tune_cache(tune_cache);
    std::map<int, TuneEntry> chosen;
    for (const TuneEntry &t : cache)
        if (t.arch == arch) chosen[t.log2n] = t;
    bool wrote = false;
    for (int i = 0; i < n; ++i) {
        const int cls = bt->log2n[i];
        if (!chosen.count(cls) && tune) {
            TuneEntry best{arch, cls, 8, 256, 1e30};
            for (int t : {4, 8})
                for (int w : {128, 256}) {
                    double us = 0.0;
                    st = batch_time_setting(bt, i, t, w, &us);
                    if (st) return bail(st);
                    if (us < best.us) best = {arch, cls, t, w, us};
                }
            chosen[cls] = best;
            cache.push_back(best);
            wrote = true;
        }
        if (chosen.count(cls)) {
            bt->tile[i] = chosen[cls].tile;
            bt->wg[i] = chosen[cls].wg;
            bt->tune_us[i] = chosen[cls].us;
        }
    }
    if (wrote && tune_cache && *tune_cache && !write_tune_cache(tune_cache, cache))
        return bail(fail(TACCHI_E_ARG, std::string("cannot write the tuning cache ") + tune_cache));
    for (int i = 0; i < n; ++i) {
        st = batch_make_contact(bt, i, bt->tile[i]);
        if (st) return bail(st);
    }
    st = batch_build_groups(bt);
    if (st) return bail(st);
    st = batch_reset_step(bt);
    if (st) return bail(st);
    *out = bt;
    return TACCHI_OK;
}

tacchi_status tacchi_batch_run(tacchi_batch *bt, int32_t substeps)
{
    if (!bt || substeps < 0) return fail(TACCHI_E_ARG, "bad arguments to tacchi_batch_run");
    int cur = -1;
    TC_HIP(hipGetDevice(&cur));
    if (cur != bt->device) TC_HIP(hipSetDevice(bt->device));
    int left = substeps;
    const bool capturable = bt->stream != nullptr;
    while (left > 0) {
        if (capturable && left >= bt->graph_len) {
            const int p = bt->parity;
            if (!bt->graph[p]) {
                TC_HIP(hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal));
                int q = p;
                tacchi_status st = TACCHI_OK;
                for (int k = 0; k < bt->graph_len && st == TACCHI_OK; ++k) {
                    st = batch_substep(bt, q);
                    q ^= 1;
                }
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(bt->stream, &g);
                if (st) return st;
                if (e != hipSuccess) return fail(TACCHI_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
                bt->graph_def[p] = g;
                TC_HIP(hipGraphInstantiate(&bt->graph[p], g, nullptr, nullptr, 0));
            }
            TC_HIP(hipGraphLaunch(bt->graph[p], bt->stream));
            left -= bt->graph_len;
            bt->done += bt->graph_len;
        } else {
            tacchi_status st = batch_substep(bt, bt->parity);
            if (st) return st;
            bt->parity ^= 1;
            left -= 1;
            bt->done += 1;
        }
    }
    // keep the per-contact handles in step with the batch for read-out
    for (int i = 0; i < bt->n; ++i) {
        tacchi_sim *s = bt->sims[i];
        s->parity = bt->parity;
        s->sf = make_simdev<float>(s);
        s->sd = make_simdev<double>(s);
        const int64_t k = std::min<int64_t>(bt->done, bt->nsteps);
        std::memcpy(s->pose, &bt->traj[((size_t)i * (bt->nsteps + 1) + k) * 7], 7 * sizeof(double));
        s->dtA = bt->dt[i];
        s->phase = 0;
    }
    return TACCHI_OK;
}

tacchi_sim *tacchi_batch_contact(tacchi_batch *bt, int32_t i)
{
    if (!bt || i < 0 || i >= bt->n) {
        fail(TACCHI_E_ARG, "contact index out of range");
        return nullptr;
    }
    return bt->sims[i];
}

tacchi_status tacchi_batch_tuning(const tacchi_batch *bt, int32_t *tile, int32_t *wg, double *us_per_substep)
{
    if (!bt) return fail(TACCHI_E_ARG, "batch is NULL");
    for (int i = 0; i < bt->n; ++i) {
        if (tile) tile[i] = bt->tile[i];
        if (wg) wg[i] = bt->wg[i];
        if (us_per_substep) us_per_substep[i] = bt->tune_us[i];
    }
    return TACCHI_OK;
}

int64_t tacchi_batch_substeps_done(const tacchi_batch *bt) { return bt ? bt->done : 0; }

tacchi_status tacchi_batch_surface_displacement(tacchi_batch *bt, int32_t res, int32_t sub, float *out,
                                                int32_t on_device)
{
    if (!bt || !out) return fail(TACCHI_E_ARG, "NULL argument");
    if (!on_device) {
        for (int i = 0; i < bt->n; ++i) {
            tacchi_status st = tacchi_surface_displacement(bt->sims[i], res, sub, out + (size_t)i * res * res * 3, 0);
            if (st) return st;
        }
        return TACCHI_OK;
    }
    for (int i = 0; i < bt->n; ++i) {
        tacchi_status st = tacchi_surface_displacement(bt->sims[i], res, sub, out + (size_t)i * res * res * 3, 1);
        if (st) return st;
    }
    return tacchi_batch_sync(bt);
}

tacchi_status tacchi_batch_sync(tacchi_batch *bt)
{
    if (!bt) return fail(TACCHI_E_ARG, "batch is NULL");
    for (tacchi_sim *s : bt->sims) {
        tacchi_status st = tacchi_sync(s);
        if (st) return st;
    }
    return TACCHI_OK;
}

void tacchi_batch_destroy(tacchi_batch *bt)
{
    if (bt) batch_free(bt);
}

}  // extern "C"
