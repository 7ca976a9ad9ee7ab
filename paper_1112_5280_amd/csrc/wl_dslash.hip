// wl_dslash.hip -- launch dispatch of the hopping term and the autotuner's
// shape record (the kernels are in wl_hop.h).
#include "wl_hop.h"
#include "wl_host.h"

namespace wl {

namespace {

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;


void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("WL_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        char *bar = std::strrchr(line, '|');
        if (!bar) continue;
        Shape sh;
        if (std::sscanf(bar + 1, " nr=%d chunk=%d tg=%d", &sh.nr, &sh.chunk, &sh.tg) != 3 ||
            sh.nr < 1 || sh.nr > kMaxNr || sh.chunk < 1 || sh.tg < 0)
            continue;
        std::string key(line, bar - line);
        while (!key.empty() && key.back() == ' ') key.pop_back();
        TuneEntry e;
        e.best = sh;
        g_tune[key] = e;
    }
    std::fclose(f);
}

void tune_store_locked(const std::string &key, const TuneEntry &e) {
    g_tune[key] = e;
    const char *path = std::getenv("WL_TUNE_FILE");
    if (!path) return;
    if (FILE *f = std::fopen(path, "a")) {
        std::fprintf(f, "%s | nr=%d chunk=%d tg=%d\n", key.c_str(), e.best.nr, e.best.chunk,
                     e.best.tg);
        std::fclose(f);
    }
}


}  // namespace

std::string tune_key(const Geom &g, int prec, bool link12, bool dag, bool xpay, int red,
                     int nrhs, int npar, bool own_gauges) {
    char k[176];
    std::snprintf(k, sizeof k, "hop prec=%d link=%d dag=%d xpay=%d red=%d nrhs=%d npar=%d "
                               "gauges=%s L=%dx%dx%dx%d",
                  prec, link12 ? 12 : 18, int(dag), int(xpay), red, nrhs, npar,
                  own_gauges ? "per-rhs" : "shared", g.L[0], g.L[1], g.L[2], g.L[3]);
    return k;
}

namespace {
thread_local int t_tuning_suspended = 0;
}

TuningSuspended::TuningSuspended() { ++t_tuning_suspended; }
TuningSuspended::~TuningSuspended() { --t_tuning_suspended; }

bool tuning_enabled() {
    if (t_tuning_suspended > 0) return false;
    const char *v = std::getenv("WL_TUNE");
    return !(v && v[0] == '0');
}

bool tune_find(const std::string &key, Shape *best) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *best = it->second.best;
    return true;
}

void tune_store(const std::string &key, const TuneEntry &e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_store_locked(key, e);
}

std::string tuning_report() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::string out;
    for (const auto &kv : g_tune) {
        char buf[96];
        out += kv.first;
        std::snprintf(buf, sizeof buf, " | nr=%d chunk=%d tg=%d", kv.second.best.nr,
                      std::min(kv.second.best.chunk, 1 << 20), kv.second.best.tg);
        out += buf;
        for (const auto &t : kv.second.tried) {
            std::snprintf(buf, sizeof buf, " [%d,%d,%d]=%.1fus", t.first.nr,
                          std::min(t.first.chunk, 1 << 20), t.first.tg, t.second);
            out += buf;
        }
        out += "\n";
    }
    return out;
}

hipError_t launch_hop(const Geom &g, int prec, bool link12, const Phases &ph,
                      const HopCall &call, hipStream_t s) {
    int red = kRedNone;
    if (call.red) {
        if (!call.red->partials || (!call.red->result && !call.red->sc))
            return hipErrorInvalidValue;
        red = call.red->epilogue == kEpiBiAlpha ? kRedDotAux
            : call.red->epilogue == kEpiBiOmega ? kRedTS : kRedNorm;
        if (red == kRedDotAux && !call.aux[call.first_par]) return hipErrorInvalidValue;
        if (red == kRedTS && !call.xs[call.first_par]) return hipErrorInvalidValue;
        if (call.cg[0]) {
            if (call.red->epilogue != kEpiCgRr || !call.red->sc || !call.cg[1] || !call.cg[2] ||
                call.npar != 1 || !call.dag || !call.xs[call.first_par])
                return hipErrorInvalidValue;
            red = kRedCgXR;
        }
    } else if (call.cg[0]) {
        return hipErrorInvalidValue;
    }
    if (call.npar < 1 || call.npar > 2 || !call.out[call.first_par] ||
        !call.in[1 - call.first_par])
        return hipErrorInvalidValue;
    if (prec == WL_F64) return launch_storage_f64(g, prec, link12, ph, call, red, s);
    if (prec == WL_F32) return launch_storage_f32(g, prec, link12, ph, call, red, s);
    return launch_storage_f16(g, prec, link12, ph, call, red, s);
}

}  // namespace wl
