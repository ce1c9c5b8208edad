// Host side of the batched multi-contact API (included at the end of
// tacchi.hip so it shares the single-contact helpers).
//
// A batch owns one single-contact handle per contact, each carved from its own
// range of the batch workspace, so state read-out (depth map, image,
// particles) goes through the ordinary calls. Substeps are advanced by the
// batched kernels of batch_kernels.hpp: contacts that share a tuning choice
// (grid block edge B, workgroup size, work items per workgroup, material
// model) form a group, and each phase of a substep is one launch per group. Runs of an even number of
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
    std::vector<int> tile, wg, ipw, log2n;
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
        int B, WG, ipw, model;
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
    double tune_batch_us[2] = {0.0, 0.0};  // whole batch per substep: tuned choices, all default (0: not timed)
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
// "model": M, "log2n": L, "tile": B, "wg": W, "ipw": P, "us_per_substep": t,
// "candidates": [[B, W, P, t], ...]}, ...]}, one entry per (arch, precision,
// material model, log2 of the particle count); "candidates" lists every
// setting the sweep timed.
struct TuneCandidate {
    int tile, wg, ipw;
    double us;
};

struct TuneEntry {
    std::string arch;
    int model, log2n, tile, wg, ipw;
    double us;
    std::vector<TuneCandidate> cands;
};

constexpr int kTuneTiles[] = {4, 8};
constexpr int kTuneWGs[] = {64, 128, 256};
constexpr int kTuneIPWs[] = {1, 2};

bool tune_setting_known(int tile, int wg, int ipw)
{
    return (tile == 4 || tile == 8) && (wg == 64 || wg == 128 || wg == 256) && (ipw == 1 || ipw == 2);
}

std::vector<TuneEntry> read_tune_cache(const char *path)
{
    std::vector<TuneEntry> out;
    if (!path || !*path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
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
    // entries are the objects holding "log2n"; their candidate lists hold no braces
    size_t pos = 0;
    while ((pos = s.find('{', pos + 1)) != std::string::npos) {
        const size_t end = s.find('}', pos);
        if (end == std::string::npos) break;
        const std::string e = s.substr(pos, end - pos + 1);
        if (e.find("\"log2n\"") == std::string::npos) continue;
        if (field(e, "precision") != "f32" || field(e, "model").empty()) continue;
        TuneEntry t;
        t.arch = field(e, "arch");
        t.model = std::atoi(field(e, "model").c_str());
        t.log2n = std::atoi(field(e, "log2n").c_str());
        t.tile = std::atoi(field(e, "tile").c_str());
        t.wg = std::atoi(field(e, "wg").c_str());
        t.ipw = std::atoi(field(e, "ipw").c_str());
        t.us = std::atof(field(e, "us_per_substep").c_str());
        if (tune_setting_known(t.tile, t.wg, t.ipw)) out.push_back(t);
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
                      "    {\"arch\": \"%s\", \"precision\": \"f32\", \"model\": %d, \"log2n\": %d, \"tile\": %d, "
                      "\"wg\": %d, \"ipw\": %d, \"us_per_substep\": %.3f, \"candidates\": [",
                      t.arch.c_str(), t.model, t.log2n, t.tile, t.wg, t.ipw, t.us);
        f << buf;
        for (size_t k = 0; k < t.cands.size(); ++k) {
            std::snprintf(buf, sizeof buf, "%s[%d, %d, %d, %.3f]", k ? ", " : "", t.cands[k].tile, t.cands[k].wg,
                          t.cands[k].ipw, t.cands[k].us);
            f << buf;
        }
        f << (i + 1 < entries.size() ? "]},\n" : "]}\n");
    }
    f << "  ]\n}\n";
    return (bool)f;
}

template <int B, int MODEL, int WG, int IPW>
void launch_group_phase(tacchi_batch *bt, const tacchi_batch::Group &g, int phase, int parity, int bump, bool sort)
{
    const dim3 grid((g.count + IPW - 1) / IPW), blk(WG);
    // P2G at B = 8 always runs kP2GWG-thread workgroups, as in the
    // single-contact path: its LDS tile allows few workgroups per CU, so the
    // resident waves come from the workgroup size (the tuned size applies to
    // the grid update and G2P)
    constexpr int P2G_WG = B == 8 ? kP2GWG : WG;
    if (phase == 0)
        hipLaunchKernelGGL((k_p2g_batch<B, MODEL, P2G_WG, IPW>), grid, dim3(P2G_WG), 0, bt->stream, g.items, g.count,
                           bt->descs[parity], bt->consts, bt->step, bump);
    else if (phase == 1)
        hipLaunchKernelGGL((k_grid_batch<B, WG, IPW>), grid, blk, 0, bt->stream, g.items, g.count, bt->descs[parity],
                           bt->consts, bt->itab, bt->nsteps, bt->step);
    else if (sort)
        hipLaunchKernelGGL((k_g2p_batch<B, MODEL, WG, IPW, true>), grid, blk, 0, bt->stream, g.items, g.count,
                           bt->descs[parity], bt->consts);
    else
        hipLaunchKernelGGL((k_g2p_batch<B, MODEL, WG, IPW, false>), grid, blk, 0, bt->stream, g.items, g.count,
                           bt->descs[parity], bt->consts);
}

template <int B, int MODEL, int WG>
void launch_group_w(tacchi_batch *bt, const tacchi_batch::Group &g, int phase, int parity, int bump, bool sort)
{
    if (g.ipw == 2)
        launch_group_phase<B, MODEL, WG, 2>(bt, g, phase, parity, bump, sort);
    else
        launch_group_phase<B, MODEL, WG, 1>(bt, g, phase, parity, bump, sort);
}

template <int B, int MODEL>
void launch_group_bm(tacchi_batch *bt, const tacchi_batch::Group &g, int phase, int parity, int bump, bool sort)
{
    if (g.WG == 64)
        launch_group_w<B, MODEL, 64>(bt, g, phase, parity, bump, sort);
    else if (g.WG == 128)
        launch_group_w<B, MODEL, 128>(bt, g, phase, parity, bump, sort);
    else
        launch_group_w<B, MODEL, 256>(bt, g, phase, parity, bump, sort);
}

void launch_group(tacchi_batch *bt, const tacchi_batch::Group &g, int phase, int parity, int bump,
                  bool sort = false)
{
    if (g.B == 4)
        g.model ? launch_group_bm<4, 1>(bt, g, phase, parity, bump, sort)
                : launch_group_bm<4, 0>(bt, g, phase, parity, bump, sort);
    else
        g.model ? launch_group_bm<8, 1>(bt, g, phase, parity, bump, sort)
                : launch_group_bm<8, 0>(bt, g, phase, parity, bump, sort);
}

// One substep of every group; `index` counts the batch's substeps (inside a
// captured run: the substep's place in the run), and every kSortEvery-th
// substep's G2P sorts the bin lists.
tacchi_status batch_substep(tacchi_batch *bt, int parity, int64_t index)
{
    const bool sort = index % kSortEvery == kSortEvery - 1;
    for (int phase = 0; phase < 3; ++phase)
        for (size_t gi = 0; gi < bt->groups.size(); ++gi)
            launch_group(bt, bt->groups[gi], phase, parity, gi == 0, sort);
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

// Work items of the contacts `ids`: every grid block of every contact, the
// blocks that hold a contact's particles at rest first (contact by contact),
// then the other blocks of each, so that the workgroups of blocks without
// particles, which exit after reading their count, wait in the launch's tail
// instead of between the live ones.
void batch_push_items(const tacchi_batch *bt, const std::vector<int> &ids, std::vector<BatchItem> &out)
{
    for (int pass = 0; pass < 2; ++pass)
        for (int i : ids) {
            const Derived &d = bt->sims[i]->d;
            int lo[3], n[3];
            rest_block_box(d, lo, n);
            const int nbox = n[0] * n[1] * n[2];
            const int b0 = pass == 0 ? 0 : nbox, b1 = pass == 0 ? nbox : d.nblk;
            for (int k = b0; k < b1; ++k)
                out.push_back({i, box_first_block(k, d.nb[0], d.nb[1], d.nb[2], lo[0], lo[1], lo[2], n[0], n[1], n[2], 1)});
        }
}

// Work items of one group: every grid block of every contact in it.
tacchi_status batch_build_groups(tacchi_batch *bt)
{
    std::map<int, std::vector<int>> by_key;
    for (int i = 0; i < bt->n; ++i) {
        const int key = bt->tile[i] * 100000 + bt->wg[i] * 100 + bt->ipw[i] * 10 + bt->cfgs[i].mat.model;
        by_key[key].push_back(i);
    }
    std::vector<BatchItem> all;
    bt->groups.clear();
    std::vector<std::pair<size_t, size_t>> ranges;
    for (auto &kv : by_key) {
        const size_t start = all.size();
        batch_push_items(bt, kv.second, all);
        const int i0 = kv.second[0];
        bt->groups.push_back({bt->tile[i0], bt->wg[i0], bt->ipw[i0], bt->cfgs[i0].mat.model, nullptr,
                              (int)(all.size() - start)});
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

// Times kTuneReps substeps of the contacts `ids` (up to kTuneContacts of one
// class, launched together as in the batch, so the time is their throughput
// rather than one contact's latency) with the given setting and returns
// microseconds per substep. The contacts start from their initial state and
// are first advanced kTuneAdvance substeps along their own trajectories with
// the default setting (so the timed substeps see indented, moving contacts),
// then two warm-up substeps with the setting; they are re-created from their
// initial state afterwards.
constexpr int kTuneAdvance = 200, kTuneWarm = 2, kTuneReps = 20, kTuneContacts = 8;

tacchi_status batch_time_setting(tacchi_batch *bt, const std::vector<int> &ids, int tile, int wgs, int ipw,
                                 double *us)
{
    std::vector<BatchItem> its;
    for (int i : ids) {
        tacchi_status st = batch_make_contact(bt, i, tile);
        if (st) return st;
    }
    batch_push_items(bt, ids, its);
    TC_HIP(hipMemcpyAsync(bt->items, its.data(), its.size() * sizeof(BatchItem), hipMemcpyHostToDevice, bt->stream));
    tacchi_status st = batch_reset_step(bt);
    if (st) return st;
    const int model = bt->cfgs[ids[0]].mat.model;
    const tacchi_batch::Group base{tile, 256, 1, model, bt->items, (int)its.size()};
    const tacchi_batch::Group g{tile, wgs, ipw, model, bt->items, (int)its.size()};
    const int adv = std::min(kTuneAdvance, std::max(0, bt->nsteps - kTuneWarm - kTuneReps));
    hipEvent_t e0, e1;
    TC_HIP(hipEventCreate(&e0));
    TC_HIP(hipEventCreate(&e1));
    int parity = 0;
    for (int k = 0; k < adv + kTuneWarm + kTuneReps; ++k) {
        if (k == adv + kTuneWarm) (void)hipEventRecord(e0, bt->stream);
        const bool sort = k % kSortEvery == kSortEvery - 1;
        for (int phase = 0; phase < 3; ++phase) launch_group(bt, k < adv ? base : g, phase, parity, 1, sort);
        parity ^= 1;
    }
    (void)hipEventRecord(e1, bt->stream);
    TC_LAUNCHED();
    TC_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    TC_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1e3 * ms / kTuneReps;
    for (int i : ids) {
        st = read_error_word(bt->sims[i]);
        if (st) return st;
        st = batch_make_contact(bt, i, tile);
        if (st) return st;
    }
    return TACCHI_OK;
}

// Microseconds per substep of the whole batch with its current choices (all
// contacts created with their tiles, groups built), over kTuneReps substeps
// after kTuneAdvance + kTuneWarm; leaves the batch at its initial state.
tacchi_status batch_time_all(tacchi_batch *bt, double *us)
{
    for (int i = 0; i < bt->n; ++i) {
        tacchi_status st = batch_make_contact(bt, i, bt->tile[i]);
        if (st) return st;
    }
    tacchi_status st = batch_build_groups(bt);
    if (st) return st;
    st = batch_reset_step(bt);
    if (st) return st;
    const int adv = std::min(kTuneAdvance, std::max(0, bt->nsteps - kTuneWarm - kTuneReps));
    hipEvent_t e0, e1;
    TC_HIP(hipEventCreate(&e0));
    TC_HIP(hipEventCreate(&e1));
    int parity = 0;
    for (int k = 0; k < adv + kTuneWarm + kTuneReps; ++k) {
        if (k == adv + kTuneWarm) (void)hipEventRecord(e0, bt->stream);
        st = batch_substep(bt, parity, k);
        if (st) return st;
        parity ^= 1;
    }
    (void)hipEventRecord(e1, bt->stream);
    TC_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    TC_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1e3 * ms / kTuneReps;
    for (int i = 0; i < bt->n; ++i) {
        st = read_error_word(bt->sims[i]);
        if (st) return st;
        st = batch_make_contact(bt, i, bt->tile[i]);
        if (st) return st;
    }
    return TACCHI_OK;
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
    bt->ipw.assign(n, 1);
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
    // tuning: cached choices, else timed sweeps per (material model,
    // particle-count class) on the class's first contact
    const std::string arch = device_arch(bt->device);
    std::vector<TuneEntry> cache = read_tune_cache(tune_cache);
    std::map<std::pair<int, int>, TuneEntry> chosen;
    for (const TuneEntry &t : cache)
        if (t.arch == arch) chosen[{t.model, t.log2n}] = t;
    bool wrote = false;
    std::map<std::pair<int, int>, std::vector<int>> members;
    for (int i = 0; i < n; ++i) {
        std::vector<int> &m = members[{cfgs[i].mat.model, bt->log2n[i]}];
        if ((int)m.size() < kTuneContacts) m.push_back(i);
    }
    for (int i = 0; i < n; ++i) {
        const std::pair<int, int> cls{cfgs[i].mat.model, bt->log2n[i]};
        if (!chosen.count(cls) && tune) {
            TuneEntry best{arch, cls.first, cls.second, 8, 256, 1, 1e30, {}};
            for (int t : kTuneTiles)
                for (int w : kTuneWGs)
                    for (int q : kTuneIPWs) {
                        double us = 0.0;
                        st = batch_time_setting(bt, members[cls], t, w, q, &us);
                        if (st) return bail(st);
                        best.cands.push_back({t, w, q, us});
                        if (us < best.us) {
                            best.tile = t;
                            best.wg = w;
                            best.ipw = q;
                            best.us = us;
                        }
                    }
            chosen[cls] = best;
            cache.push_back(best);
            wrote = true;
        }
        if (chosen.count(cls)) {
            bt->tile[i] = chosen[cls].tile;
            bt->wg[i] = chosen[cls].wg;
            bt->ipw[i] = chosen[cls].ipw;
            bt->tune_us[i] = chosen[cls].us;
        }
    }
    // the classes share each phase's launches, so the tuned choices are kept
    // only if the whole batch runs faster with them than with the default
    // setting for every contact (different choices make more, smaller
    // launches per phase)
    if (tune) {
        double us_tuned = 0.0, us_default = 0.0;
        st = batch_time_all(bt, &us_tuned);
        if (st) return bail(st);
        const std::vector<int> tile_t = bt->tile, wg_t = bt->wg, ipw_t = bt->ipw;
        bt->tile.assign(n, 8);
        bt->wg.assign(n, 256);
        bt->ipw.assign(n, 1);
        st = batch_time_all(bt, &us_default);
        if (st) return bail(st);
        bt->tune_batch_us[0] = us_tuned;
        bt->tune_batch_us[1] = us_default;
        if (us_tuned <= us_default) {
            bt->tile = tile_t;
            bt->wg = wg_t;
            bt->ipw = ipw_t;
        } else {
            bt->tune_us.assign(n, 0.0);
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
                    st = batch_substep(bt, q, k);
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
            tacchi_status st = batch_substep(bt, bt->parity, bt->done);
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

tacchi_status tacchi_batch_tuning(const tacchi_batch *bt, int32_t *tile, int32_t *wg, int32_t *ipw,
                                  double *us_per_substep)
{
    if (!bt) return fail(TACCHI_E_ARG, "batch is NULL");
    for (int i = 0; i < bt->n; ++i) {
        if (tile) tile[i] = bt->tile[i];
        if (wg) wg[i] = bt->wg[i];
        if (ipw) ipw[i] = bt->ipw[i];
        if (us_per_substep) us_per_substep[i] = bt->tune_us[i];
    }
    return TACCHI_OK;
}

tacchi_status tacchi_batch_tuning_check(const tacchi_batch *bt, double *us_tuned, double *us_default)
{
    if (!bt || !us_tuned || !us_default) return fail(TACCHI_E_ARG, "NULL argument");
    *us_tuned = bt->tune_batch_us[0];
    *us_default = bt->tune_batch_us[1];
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
