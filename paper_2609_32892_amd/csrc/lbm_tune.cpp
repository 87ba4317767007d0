// lbm_tune.cpp -- the autotuner of the launch shapes (binomial tile width,
// z planes per binomial workgroup, cells per thread of the QoI reduction).
//
// A client of the library's own C ABI: each candidate tuning is created in
// the caller's scratch arena, stepped from a small seeded velocity field and
// timed with the host clock around lbm_step + lbm_sync; the search is a
// coordinate descent from the automatic choice (tile width, then z chunk,
// then cells per thread).  Results are kept in a text cache, one line per
// (device, grid, closure shape), so that an ensemble of uneven grids times
// each distinct member shape once.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {
int set_error(int code, const char* msg);
}

namespace {

struct Cand {
    int zc, cpt, btx;
    bool operator==(const Cand& o) const { return zc == o.zc && cpt == o.cpt && btx == o.btx; }
};

lbm_config with(const lbm_config* cfg, const Cand& k)
{
    lbm_config c = *cfg;
    c.tune_zc = k.zc;
    c.tune_cpt = k.cpt;
    c.tune_btx = k.btx;
    return c;
}

// The values each coordinate may take (0: the library's automatic choice).
// Runs without a closure launch none of the tuned kernels.
void axes(const lbm_config* cfg, const lbm_closure* cl, std::vector<int>& btx, std::vector<int>& zc,
          std::vector<int>& cpt)
{
    btx = {0};
    zc = {0};
    cpt = {0};
    if (!cl) return;
    if (cfg->lattice == LBM_D3Q19) {
        btx.push_back(32);
        if (cfg->nx % 64 == 0) btx.push_back(64);
        for (int z : {1, 2, 4, 8, 16})
            if (z <= cfg->nz) zc.push_back(z);
    }
    cpt = {0, 1, 2, 4, 8};
}

std::string key_of(const lbm_config* cfg, const lbm_closure* cl)
{
    char dev[128] = "unknown";
    lbm_device_tag(dev, sizeof dev);
    std::string k = "lbm-tune-v1 dev=" + std::string(dev);
    for (char& ch : k)
        if (ch == '\t' || ch == '\n') ch = ' ';
    char buf[256];
    std::snprintf(buf, sizeof buf, " lat=%d prec=%d grid=%dx%dx%d walls=%d sub=%d", cfg->lattice, cfg->precision,
                  cfg->nx, cfg->ny, cfg->nz, cfg->walls_y, cfg->substrate);
    k += buf;
    if (cl) {
        std::snprintf(buf, sizeof buf, " nq=%d h=%d nb=%d q=", cl->nq, cl->h, cl->nbands);
        k += buf;
        for (int i = 0; i < cl->nq; ++i) {
            const lbm_qoi_spec& q = cl->q[i];
            std::snprintf(buf, sizeof buf, "%s%d.%d.%d.%d.%d", i ? "," : "", q.kind, q.filter, q.band, q.scale, q.kmax);
            k += buf;
        }
    } else {
        k += " plain";
    }
    return k;
}

// The last cache line for key (format: key TAB zc cpt btx us_per_step).
bool cache_find(const char* path, const std::string& key, lbm_tuning* out)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    std::string line;
    char chunk[512];
    while (std::fgets(chunk, sizeof chunk, f)) {
        line += chunk;
        if (line.empty() || line.back() != '\n') continue;   // long line: keep reading
        line.pop_back();
        const size_t tab = line.find('\t');
        if (tab != std::string::npos && line.compare(0, tab, key) == 0 && tab == key.size()) {
            lbm_tuning t{};
            if (std::sscanf(line.c_str() + tab + 1, "%d %d %d %lf", &t.tune_zc, &t.tune_cpt, &t.tune_btx,
                            &t.us_per_step) == 4) {
                *out = t;
                found = true;
            }
        }
        line.clear();
    }
    std::fclose(f);
    return found;
}

int cache_add(const char* path, const std::string& key, const lbm_tuning& t)
{
    FILE* f = std::fopen(path, "a");
    if (!f) return lbm::set_error(LBM_EINVAL, "autotune: cannot append to the cache file");
    std::fprintf(f, "%s\t%d %d %d %.4f\n", key.c_str(), t.tune_zc, t.tune_cpt, t.tune_btx, t.us_per_step);
    std::fclose(f);
    return LBM_OK;
}

// Microseconds per step of one candidate; negative on failure (the error
// is left in lbm_last_error).
double time_candidate(const lbm_config* cfg, const lbm_closure* cl, void* arena, size_t bytes, void* stream,
                      int steps, const std::vector<double>& u0)
{
    lbm_ctx* ctx = nullptr;
    if (lbm_create(cfg, cl, arena, bytes, stream, &ctx) != LBM_OK) return -1;
    double us = -1;
    if (lbm_init_velocity(ctx, nullptr, u0.data()) == LBM_OK && lbm_step(ctx, std::max(steps / 4, 8)) == LBM_OK &&
        lbm_sync(ctx) == LBM_OK) {
        const auto t0 = std::chrono::steady_clock::now();
        if (lbm_step(ctx, steps) == LBM_OK && lbm_sync(ctx) == LBM_OK)
            us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() / steps;
    }
    lbm_destroy(ctx);
    return us;
}

}  // namespace

extern "C" {

int lbm_autotune_key(const lbm_config* cfg, const lbm_closure* closure, char* out, size_t n)
{
    if (!cfg || !out || n == 0) return lbm::set_error(LBM_EINVAL, "autotune_key: NULL argument");
    const std::string k = key_of(cfg, closure);
    if (k.size() + 1 > n) return lbm::set_error(LBM_EINVAL, "autotune_key: buffer too small");
    std::memcpy(out, k.c_str(), k.size() + 1);
    return LBM_OK;
}

size_t lbm_autotune_bytes(const lbm_config* cfg, const lbm_closure* closure)
{
    if (!cfg) return 0;
    std::vector<int> bt, zc, cp;
    axes(cfg, closure, bt, zc, cp);
    size_t most = 0;
    for (int b : bt)
        for (int z : zc)
            for (int c : cp) {
                const lbm_config t = with(cfg, {z, c, b});
                const size_t n = lbm_required_bytes(&t, closure);
                if (n == 0) return 0;
                most = std::max(most, n);
            }
    return most;
}

int lbm_autotune(const lbm_config* cfg, const lbm_closure* closure, void* dev_arena, size_t bytes, void* stream,
                 int steps, const char* cache_path, lbm_tuning* out)
{
    if (!cfg || !out) return lbm::set_error(LBM_EINVAL, "autotune: NULL argument");
    if (steps < 1) return lbm::set_error(LBM_EINVAL, "autotune: steps must be >= 1");
    const size_t need = lbm_autotune_bytes(cfg, closure);
    if (need == 0) return LBM_EINVAL;   // the message of lbm_required_bytes stands
    const std::string key = key_of(cfg, closure);
    if (cache_path && cache_find(cache_path, key, out)) {
        out->from_cache = 1;
        out->candidates = 0;
        return LBM_OK;
    }
    if (!dev_arena || bytes < need) return lbm::set_error(LBM_ENOMEM, "autotune: arena smaller than lbm_autotune_bytes");
    // a small seeded velocity field (an integer hash, the same on every call)
    const int d = cfg->lattice == LBM_D2Q9 ? 2 : 3;
    const size_t N = (size_t)cfg->nx * cfg->ny * cfg->nz;
    std::vector<double> u0((size_t)d * N);
    for (size_t i = 0; i < u0.size(); ++i) {
        unsigned long long x = (i + 1) * 0x9E3779B97F4A7C15ull;
        x ^= x >> 31;
        x *= 0xBF58476D1CE4E5B9ull;
        x ^= x >> 29;
        u0[i] = 1e-3 * ((double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5);
    }
    std::vector<int> bt, zc, cp;
    axes(cfg, closure, bt, zc, cp);
    std::vector<std::pair<Cand, double>> seen;
    auto eval = [&](const Cand& k) -> double {
        for (const auto& s : seen)
            if (s.first == k) return s.second;
        const lbm_config t = with(cfg, k);
        const double us = time_candidate(&t, closure, dev_arena, bytes, stream, steps, u0);
        seen.push_back({k, us});
        return us;
    };
    Cand best{0, 0, 0};
    double tbest = eval(best);
    if (tbest < 0) return LBM_EDEVICE;   // the automatic choice itself failed: its error stands
    for (int axis = 0; axis < 3; ++axis) {
        const std::vector<int>& vals = axis == 0 ? bt : (axis == 1 ? zc : cp);
        Cand cur = best;
        for (int v : vals) {
            Cand k = cur;
            (axis == 0 ? k.btx : (axis == 1 ? k.zc : k.cpt)) = v;
            const double us = eval(k);
            if (us >= 0 && us < tbest) {
                tbest = us;
                best = k;
            }
        }
    }
    lbm_tuning t{};
    t.tune_zc = best.zc;
    t.tune_cpt = best.cpt;
    t.tune_btx = best.btx;
    t.us_per_step = tbest;
    t.from_cache = 0;
    t.candidates = (int)seen.size();
    *out = t;
    if (cache_path) return cache_add(cache_path, key, t);
    return LBM_OK;
}

}  // extern "C"
