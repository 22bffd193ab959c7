// Tuning cache of libcoffee: launch choices measured by the autotuner
// (paper_1407_0904_amd/tuner.py), one entry per line of a text file:
//
//   linear <form> <cell> <degree> <field_degree> <precision> <grid_mult> [<variant>]
//   batch  <form> <cell> <degree> <precision> <variant> <task_cells> <ns_per_cell>
//   packed <form> <cell> <degree> <precision> <task_cells> <ns_per_cell>
//
// (batch: coffee_assemble_batch, caller's layout; packed:
// coffee_assemble_batch_packed.)
// '#' starts a comment. The paper weighs a cost model against auto-tuning
// (section 4) and reports the best over every feasible unroll factor next to
// the model's pick (section 5.6); here the search is exhaustive over a small
// space and runs offline, so its cost never lands on the assembly path.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>

#include "../../include/coffee.h"

namespace coffee {

struct BatchTune {
    int variant = 0, task_cells = 0;
    double ns_per_cell = 0.0;
};

static std::mutex g_tmu;
static bool g_loaded = false;
static std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> g_linear;  // -> (grid_mult, variant)
static std::map<std::tuple<int, int, int, int>, BatchTune> g_batch;       // (form, cell, degree, prec)
static std::map<std::tuple<int, int, int, int>, BatchTune> g_packed;      // (form, cell, degree, prec)

static coffee_status parse(const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return COFFEE_E_INVALID_ARG;
    std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> lin;
    std::map<std::tuple<int, int, int, int>, BatchTune> bat, pk;
    char line[512];
    coffee_status st = COFFEE_OK;
    while (std::fgets(line, sizeof line, f)) {
        char* hash = std::strchr(line, '#');
        if (hash) *hash = '\0';
        char kind[32];
        if (std::sscanf(line, "%31s", kind) != 1) continue;
        if (!std::strcmp(kind, "linear")) {
            int form, cell, deg, fd, prec, gm, var = 0;
            const int nf = std::sscanf(line, "%*s %d %d %d %d %d %d %d", &form, &cell, &deg, &fd, &prec, &gm, &var);
            // tile-shape variants 0..3 of the symmetric engine
            if (nf < 6 || gm < 1 || var < 0 || var > 3) {
                st = COFFEE_E_INVALID_ARG;
                break;
            }
            lin[std::make_tuple(form, cell, deg, fd, prec)] = std::make_pair(gm, var);
        } else if (!std::strcmp(kind, "batch")) {
            int form, cell, deg, prec, var, tc;
            double ns;
            if (std::sscanf(line, "%*s %d %d %d %d %d %d %lf", &form, &cell, &deg, &prec, &var, &tc, &ns) != 7 ||
                var < 0 || var > 1 || tc < 64 || tc > 1024 || tc % 64 != 0) {
                st = COFFEE_E_INVALID_ARG;
                break;
            }
            BatchTune t;
            t.variant = var;
            t.task_cells = tc;
            t.ns_per_cell = ns;
            bat[std::make_tuple(form, cell, deg, prec)] = t;
        } else if (!std::strcmp(kind, "packed")) {
            int form, cell, deg, prec, tc;
            double ns;
            if (std::sscanf(line, "%*s %d %d %d %d %d %lf", &form, &cell, &deg, &prec, &tc, &ns) != 6 || tc < 64 ||
                tc > 1024 || tc % 64 != 0) {
                st = COFFEE_E_INVALID_ARG;
                break;
            }
            BatchTune t;
            t.variant = 2;
            t.task_cells = tc;
            t.ns_per_cell = ns;
            pk[std::make_tuple(form, cell, deg, prec)] = t;
        } else {
            st = COFFEE_E_INVALID_ARG;
            break;
        }
    }
    std::fclose(f);
    if (st == COFFEE_OK) {
        g_linear.swap(lin);
        g_batch.swap(bat);
        g_packed.swap(pk);
    }
    return st;
}

static void ensure_loaded() {
    if (g_loaded) return;
    g_loaded = true;
    const char* env = std::getenv("COFFEE_TUNE_CACHE");
    if (env && *env) (void)parse(env);
}

int tuned_linear(int form, int cell, int degree, int fd, int prec, int* variant) {
    std::lock_guard<std::mutex> lk(g_tmu);
    ensure_loaded();
    auto it = g_linear.find(std::make_tuple(form, cell, degree, fd, prec));
    *variant = it == g_linear.end() ? 0 : it->second.second;
    return it == g_linear.end() ? 0 : it->second.first;
}

bool tuned_batch(int form, int cell, int degree, int prec, int* variant, int* task_cells) {
    std::lock_guard<std::mutex> lk(g_tmu);
    ensure_loaded();
    auto it = g_batch.find(std::make_tuple(form, cell, degree, prec));
    if (it == g_batch.end()) return false;
    *variant = it->second.variant;
    *task_cells = it->second.task_cells;
    return true;
}

bool tuned_packed(int form, int cell, int degree, int prec, int* task_cells) {
    std::lock_guard<std::mutex> lk(g_tmu);
    ensure_loaded();
    auto it = g_packed.find(std::make_tuple(form, cell, degree, prec));
    if (it == g_packed.end()) return false;
    *task_cells = it->second.task_cells;
    return true;
}

}  // namespace coffee

extern "C" coffee_status coffee_load_tuning(const char* path) {
    std::lock_guard<std::mutex> lk(coffee::g_tmu);
    coffee::g_loaded = true;
    if (!path) {
        coffee::g_linear.clear();
        coffee::g_batch.clear();
        coffee::g_packed.clear();
        return COFFEE_OK;
    }
    return coffee::parse(path);
}
