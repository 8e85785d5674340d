// Autotuner of the MD step launch: picks the step kernel variant and block
// size for a whole batch of replicas, then the cell-list skin (which sets the
// cell width, the neighbour-list radius and, through the drift bound, the
// rebuild interval) globally and per replica size class, by timing candidate
// configurations on the caller's own initial state.  Built on the public ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "mdlg_internal.h"

namespace {

struct Buffers {
    int64_t* counts = nullptr;
    double* moments = nullptr;
    ~Buffers() {
        if (counts) (void)hipFree(counts);
        if (moments) (void)hipFree(moments);
    }
};

// Microseconds per MD step of one configuration: a handle is created, run
// through `units` cell-list intervals (the first two warm up), and the graph
// times of the later ones are averaged.  Returns < 0 when the configuration
// cannot run (its status is kept in *st).
double time_config(int n_rep, const std::vector<lj_params>& p, const double* pos0, const double* vel0, int s_cg,
                   const mdlg_lattice* lat, int units, hipStream_t stream, mdlg_status* st) {
    lj_md* md = nullptr;
    *st = lj_md_init_batch(&md, n_rep, p.data(), pos0, vel0, stream);
    if (*st != MDLG_OK) return -1.0;
    Buffers b;
    if (lat) {
        if (hipMalloc((void**)&b.counts, sizeof(int64_t) * MDLG_NCOUNTS * n_rep) != hipSuccess ||
            hipMalloc((void**)&b.moments, sizeof(double) * MDLG_NMOMENTS * n_rep) != hipSuccess) {
            lj_md_destroy(md);
            *st = mdlg::fail(MDLG_ENOMEM, "lj_md_autotune: device allocation failed");
            return -1.0;
        }
        *st = lj_md_cg_attach(md, s_cg, lat, b.counts, b.moments, nullptr, stream);
        if (*st != MDLG_OK) {
            lj_md_destroy(md);
            return -1.0;
        }
    }
    double ms[3] = {0, 0, 0};
    int32_t cnt[3] = {0, 0, 0};
    *st = lj_md_step_timed(md, units, 1, ms, cnt, stream);
    lj_md_info_t info{};
    if (*st == MDLG_OK) *st = lj_md_check(md, stream);
    if (*st == MDLG_OK) *st = lj_md_info(md, &info);
    lj_md_destroy(md);
    if (*st != MDLG_OK) return -1.0;
    const int K = info.rebuild_every;
    // per MD step: one ordinary step, a coarse-graining step's extra every
    // s_cg steps and a rebuild every K steps
    double us = ms[0] + ms[2] / K;
    if (lat && s_cg > 0 && cnt[1] > 0) us += (ms[1] - ms[0]) / s_cg;
    return 1e3 * us;
}

std::string cache_path() {
    if (const char* e = std::getenv("MDLG_AUTOTUNE_CACHE")) return e;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/mdlg_autotune.txt";
}

int size_class(const lj_params& q) {
    const double dens = (double)q.n / (q.box_l * q.box_l);
    const int nb = (int)std::floor(std::log2((double)q.n) / 2.0);  // factor-4 bins of N
    const int db = (int)std::lround(dens * 20.0);                    // bins of 0.05 per sigma^2
    return nb * 1000 + db;
}

std::string signature(int n_rep, const lj_params* p, int s_cg) {
    std::map<int, int> classes;
    long long ntot = 0;
    for (int r = 0; r < n_rep; ++r) {
        classes[size_class(p[r])] += 1;
        ntot += p[r].n;
    }
    std::ostringstream os;
    os << "gfx950|bits" << p[0].force_bits << "|R" << n_rep << "|N" << ntot << "|scg" << s_cg;
    for (auto& kv : classes) os << "|c" << kv.first << "x" << kv.second;
    return os.str();
}

// cached line: signature kernel block skin_default {class:skin}...
bool cache_lookup(const std::string& sig, int* kernel, int* block, double* skin, std::map<int, double>* cls) {
    FILE* f = std::fopen(cache_path().c_str(), "r");
    if (!f) return false;
    char buf[65536];
    bool found = false;
    while (std::fgets(buf, sizeof(buf), f)) {
        std::istringstream is(buf);
        std::string s;
        is >> s;
        if (s != sig) continue;
        is >> *kernel >> *block >> *skin;
        cls->clear();
        int c;
        double v;
        while (is >> c >> v) (*cls)[c] = v;
        found = true;
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string& sig, int kernel, int block, double skin, const std::map<int, double>& cls) {
    const std::string path = cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;  // a cache that cannot be written is not an error
    // full precision, so that a cached choice reproduces the tuned values exactly
    std::fprintf(f, "%s %d %d %.17g", sig.c_str(), kernel, block, skin);
    for (auto& kv : cls) std::fprintf(f, " %d %.17g", kv.first, kv.second);
    std::fprintf(f, "\n");
    std::fclose(f);
}

}  // namespace

extern "C" mdlg_status lj_md_autotune(int32_t n_rep, const lj_params* p_in, const double* pos0, const double* vel0,
                                      int32_t s_cg, const mdlg_lattice* lat, int32_t flags, lj_params* p_out,
                                      double* us_per_step, void* stream) {
    if (n_rep < 1 || !p_in || !pos0 || !vel0 || !p_out)
        return mdlg::fail(MDLG_EINVAL, "lj_md_autotune: NULL argument or n_rep < 1");
    if (lat && s_cg < 1) return mdlg::fail(MDLG_EINVAL, "lj_md_autotune: s_cg must be >= 1 with a lattice");
    hipStream_t st = (hipStream_t)stream;
    std::vector<lj_params> base(p_in, p_in + n_rep);
    for (auto& q : base) {
        q.step_kernel = 0;
        q.block_size = 0;
        q.rebuild_every = 0;
    }
    const std::string sig = signature(n_rep, p_in, lat ? s_cg : 0);
    int best_kernel = 3, best_block = 256;
    double best_skin = 0.5;
    std::map<int, double> cls_skin;
    const bool use_cache = !(flags & 1);
    const int units = 5;
    double best = -1.0;
    mdlg_status status = MDLG_OK;
    auto apply = [&](int kernel, int block, double skin, const std::map<int, double>& cs) {
        std::vector<lj_params> q = base;
        for (auto& x : q) {
            x.step_kernel = kernel;
            x.block_size = block;
            auto it = cs.find(size_class(x));
            x.skin = it != cs.end() ? it->second : skin;
        }
        return q;
    };
    if (use_cache && cache_lookup(sig, &best_kernel, &best_block, &best_skin, &cls_skin)) {
        std::vector<lj_params> q = apply(best_kernel, best_block, best_skin, cls_skin);
        std::copy(q.begin(), q.end(), p_out);
        if (us_per_step) *us_per_step = -1.0;
        return MDLG_OK;
    }
    // stage 1: kernel variant x block size at the default skin
    for (int kernel : {3, 1, 2}) {
        for (int block : {128, 256, 512}) {
            mdlg_status s;
            const double t = time_config(n_rep, apply(kernel, block, 0.5, {}), pos0, vel0, s_cg, lat, units, st, &s);
            if (t > 0 && (best < 0 || t < best)) {
                best = t;
                best_kernel = kernel;
                best_block = block;
            }
            if (t < 0) status = s;
        }
    }
    if (best < 0) return status != MDLG_OK ? status : mdlg::fail(MDLG_EINVAL, "lj_md_autotune: nothing ran");
    // stage 2: one skin for all replicas
    for (double skin : {0.35, 0.65, 0.8}) {
        mdlg_status s;
        const double t = time_config(n_rep, apply(best_kernel, best_block, skin, {}), pos0, vel0, s_cg, lat, units, st, &s);
        if (t > 0 && t < best) {
            best = t;
            best_skin = skin;
        }
    }
    // stage 3: per size class, one step up and one down from the global skin
    std::map<int, int> classes;
    for (auto& q : base) classes[size_class(q)] += 1;
    if (classes.size() > 1) {
        for (auto& kv : classes) {
            for (double d : {-0.15, 0.15}) {
                const double sk = best_skin + d;
                if (sk < 0.2) continue;
                std::map<int, double> trial = cls_skin;
                trial[kv.first] = sk;
                mdlg_status s;
                const double t = time_config(n_rep, apply(best_kernel, best_block, best_skin, trial), pos0, vel0, s_cg,
                                             lat, units, st, &s);
                if (t > 0 && t < best) {
                    best = t;
                    cls_skin = trial;
                }
            }
        }
    }
    std::vector<lj_params> q = apply(best_kernel, best_block, best_skin, cls_skin);
    std::copy(q.begin(), q.end(), p_out);
    if (us_per_step) *us_per_step = best;
    if (use_cache) cache_store(sig, best_kernel, best_block, best_skin, cls_skin);
    return MDLG_OK;
}
