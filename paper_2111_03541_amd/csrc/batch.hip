// Batched assembly of many structured problems in one persistent launch, replayed as a
// HIP graph, with a small autotuner for the tile shape and the launch shape.  A tile is a
// 4x2 node column of a problem cut along z into chunks; the tuner chooses the number of
// chunks (the tile height) per class of problems, a class being (form, size bucket of the
// column height), then the work-item order and the workgroup count.  The per-problem offsets play the role of the paper's workpiece offsets
// n_dense / n_sp (Sec. 2.2 B-2): every problem keeps its own CSR and vector, located by
// the pointers in its descriptor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "mf_internal.h"

// tile-shape classes: (form, size bucket of the column height NZ = nz + 1)
constexpr int kBuckets = 3;            // NZ <= 20, NZ <= 34, larger
constexpr int kClasses = 2 * kBuckets; // Poisson / mass, elasticity
constexpr int kMaxChunks = 4;          // tile heights tried: NZ / 1 .. NZ / 4

struct mf_batch_s {
    std::vector<mf::AssembleArgs> probs;
    std::vector<mf_form> forms;
    std::vector<int64_t> units;  // work items (tiles) per problem
    std::vector<int> cls;        // class of each problem
    int chunks[kClasses] = {1, 1, 1, 1, 1, 1};
    int xw[kClasses] = {4, 4, 4, 4, 4, 4};  // cross-section per class: 4 (4x2) or 2 (2x4)
    mf_precision prec = MF_F64;
    bool masked = false;  // some problem has Dirichlet flags
    void* dprobs = nullptr;
    void* dstatus = nullptr;
    int* counter = nullptr;
    int2* items = nullptr;
    int64_t items_cap = 0;
    int n_items = 0;
    int n_first = 0;  // items of the kernel launched first (elasticity unless order 2)
    int n_wg = 0;
    int order = 1;
    int num_cus = 256;
    double tuned_us = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
};

namespace {

using namespace mf;

int class_of(const mf_form& f, const mf_pattern_s* P)
{
    const int NZ = (int)P->gz + 1;
    const int bucket = NZ <= 20 ? 0 : (NZ <= 34 ? 1 : 2);
    return (f.kind == MF_FORM_ELASTICITY ? kBuckets : 0) + bucket;
}

void drop_graph(mf_batch_s* B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_stream = nullptr;
}

// Items in two groups, one per kernel: elasticity and the scalar forms (mass, Poisson).
// order 0: problem-major within each group, elasticity group first; 1: round-robin over
// the group's problems, elasticity first; 2: round-robin, scalar group first.
// *n_first: items of the group launched first.
std::vector<int2> build_items(const mf_batch_s* B, int order, int* n_first)
{
    std::vector<int2> it;
    const int np = (int)B->probs.size();
    std::vector<int> el, sc;
    for (int p = 0; p < np; ++p) (B->forms[p].kind == MF_FORM_ELASTICITY ? el : sc).push_back(p);
    const std::vector<int>* groups[2] = {&el, &sc};
    if (order == 2) std::swap(groups[0], groups[1]);
    for (int g = 0; g < 2; ++g) {
        const std::vector<int>& grp = *groups[g];
        if (order == 0) {
            for (int p : grp)
                for (int64_t b = 0; b < B->units[p]; ++b) it.push_back(make_int2(p, (int)b));
        } else {
            int64_t mx = 0;
            for (int p : grp) mx = std::max(mx, B->units[p]);
            for (int64_t k = 0; k < mx; ++k)
                for (int p : grp)
                    if (k < B->units[p]) it.push_back(make_int2(p, (int)k));
        }
        if (g == 0) *n_first = (int)it.size();
    }
    return it;
}

// descriptors (tile heights) and the item list for the current shapes and `order`
mf_status upload_items(mf_batch_s* B, int order)
{
    std::vector<int> ch(B->probs.size()), xw(B->probs.size());
    for (size_t k = 0; k < B->probs.size(); ++k) {
        ch[k] = B->chunks[B->cls[k]];
        xw[k] = B->xw[B->cls[k]];
        B->units[k] = batch_units_of(B->probs[k].P, ch[k], xw[k]);
    }
    MF_HIP(hipDeviceSynchronize());  // a launch in flight may still read the old lists
    mf_status st = batch_upload(B->probs, ch, xw, &B->dprobs, &B->dstatus);
    if (st != MF_OK) return st;
    int n_first = 0;
    std::vector<int2> it = build_items(B, order, &n_first);
    if (B->items && (int64_t)it.size() > B->items_cap) {
        (void)hipFree(B->items);
        B->items = nullptr;
    }
    if (!B->items) {
        B->items_cap = (int64_t)(it.size() > 0 ? it.size() : 1);
        MF_HIP(hipMalloc(&B->items, sizeof(int2) * B->items_cap));
    }
    MF_HIP(hipMemcpy(B->items, it.data(), sizeof(int2) * it.size(), hipMemcpyHostToDevice));
    B->n_items = (int)it.size();
    B->n_first = n_first;
    B->order = order;
    drop_graph(B);
    return MF_OK;
}

std::string tune_key(const mf_batch_s* B)
{
    int per[kClasses] = {0};
    int64_t cols = 0;
    for (size_t k = 0; k < B->probs.size(); ++k) {
        ++per[B->cls[k]];
        cols += batch_units_of(B->probs[k].P, 1, 4);
    }
    // bucket the column count to two significant digits
    double lg = std::floor(std::log10((double)std::max<int64_t>(1, cols)));
    long bucket = (long)(std::round(cols / std::pow(10.0, lg - 1)) * std::pow(10.0, lg - 1));
    std::ostringstream os;
    os << "gfx950|column-v4|prec=" << (B->prec == MF_F64 ? "f64" : "f32") << "|mask=" << (B->masked ? 1 : 0)
       << "|classes=";
    for (int c = 0; c < kClasses; ++c) os << per[c] << (c + 1 < kClasses ? "," : "");
    os << "|columns~" << bucket;
    return os.str();
}

// cache line: key order mult us chunks[0..kClasses) xw[0..kClasses)
bool cache_lookup(const char* path, const std::string& key, int* order, int* mult, double* us, int* chunks,
                  int* xw)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        int o, m;
        double u;
        if (is >> k >> o >> m >> u && k == key) {
            int c[kClasses], x[kClasses];
            for (int j = 0; j < kClasses; ++j)
                if (!(is >> c[j]) || c[j] < 1 || c[j] > kMaxChunks) return false;
            for (int j = 0; j < kClasses; ++j)
                if (!(is >> x[j]) || (x[j] != 2 && x[j] != 4)) return false;
            if (o < 0 || o > 2 || m < 1 || m > 3) return false;
            *order = o;
            *mult = m;
            *us = u;
            for (int j = 0; j < kClasses; ++j) {
                chunks[j] = c[j];
                xw[j] = x[j];
            }
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, int order, int mult, double us, const int* chunks,
                 const int* xw)
{
    if (!path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line))
            if (line.compare(0, key.size() + 1, key + " ") != 0) keep.push_back(line);
    }
    std::ofstream f(path, std::ios::trunc);
    for (auto& l : keep) f << l << "\n";
    f << key << " " << order << " " << mult << " " << us;
    for (int j = 0; j < kClasses; ++j) f << " " << chunks[j];
    for (int j = 0; j < kClasses; ++j) f << " " << xw[j];
    f << "\n";
}

mf_status launch(mf_batch_s* B, hipStream_t s)
{
    return batch_launch(B->dprobs, B->dstatus, (int)B->probs.size(), B->items, B->n_first, B->n_items,
                        B->order != 2, B->counter, B->n_wg, B->prec, B->masked, s);
}

mf_status time_config(mf_batch_s* B, hipStream_t s, double* us)
{
    hipEvent_t e0, e1;
    MF_HIP(hipEventCreate(&e0));
    MF_HIP(hipEventCreate(&e1));
    for (int w = 0; w < 2; ++w) {
        mf_status st = launch(B, s);
        if (st != MF_OK) return st;
    }
    std::vector<float> t;
    for (int r = 0; r < 5; ++r) {
        MF_HIP(hipEventRecord(e0, s));
        mf_status st = launch(B, s);
        if (st != MF_OK) return st;
        MF_HIP(hipEventRecord(e1, s));
        MF_HIP(hipEventSynchronize(e1));
        float ms = 0;
        MF_HIP(hipEventElapsedTime(&ms, e0, e1));
        t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    *us = t[t.size() / 2] * 1e3;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return MF_OK;
}

void free_batch(mf_batch_s* B)
{
    if (!B) return;
    drop_graph(B);
    (void)hipFree(B->dprobs);
    (void)hipFree(B->dstatus);
    (void)hipFree(B->counter);
    (void)hipFree(B->items);
    delete B;
}

}  // namespace

extern "C" {

mf_status mf_batch_create(const mf_batch_problem* problems, int32_t n, mf_precision prec, mf_batch_t** out)
{
    if (!out) return set_error(MF_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!problems || n <= 0) return set_error(MF_ERR_ARG, "need at least one problem");
    if (prec != MF_F64 && prec != MF_F32) return set_error(MF_ERR_ARG, "unknown precision");
    mf_batch_s* B = new mf_batch_s();
    B->prec = prec;
    B->forms.resize(n);
    for (int k = 0; k < n; ++k) {
        const mf_batch_problem& q = problems[k];
        if (!q.pattern || !q.coords || !q.K || !q.d) {
            free_batch(B);
            return set_error(MF_ERR_ARG, "problem %d: NULL pattern, coords, K or d", k);
        }
        B->forms[k] = q.form;
        const int nf_form = q.form.kind == MF_FORM_ELASTICITY ? 3 : 1;
        if (q.pattern->nf != nf_form) {
            free_batch(B);
            return set_error(MF_ERR_ARG, "problem %d: form needs %d fields, pattern has %d", k, nf_form,
                             q.pattern->nf);
        }
    }
    for (int k = 0; k < n; ++k) {
        const mf_batch_problem& q = problems[k];
        AssembleArgs a{};
        a.P = q.pattern;
        a.form = &B->forms[k];
        a.coords = q.coords;
        a.elem_param = q.fields.elem_param;
        a.nodal_src = q.fields.nodal_src;
        a.lin_state = nullptr;
        a.dirichlet = q.fields.dirichlet;
        if (a.dirichlet) B->masked = true;
        a.prec = prec;
        a.K = q.K;
        a.d = q.d;
        mf_status st = batch_check(a);
        if (st != MF_OK) {
            free_batch(B);
            return st;
        }
        B->probs.push_back(a);
        B->cls.push_back(class_of(B->forms[k], q.pattern));
        B->units.push_back(batch_units_of(q.pattern, 1, 4));
    }
    mf_status st = MF_OK;
    if (hipMalloc(&B->counter, 2 * sizeof(int)) != hipSuccess) st = set_error(MF_ERR_OOM, "counter");
    int dev = 0, cus = 256;
    if (st == MF_OK && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
        B->num_cus = cus;
    B->n_wg = B->num_cus;
    if (st == MF_OK) st = upload_items(B, 1);
    if (st != MF_OK) {
        free_batch(B);
        return st;
    }
    *out = B;
    return MF_OK;
}

mf_status mf_batch_tune(mf_batch_t* B, const char* cache_path, void* stream)
{
    if (!B) return set_error(MF_ERR_ARG, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    const std::string key = tune_key(B);
    int order = 1, mult = 1;
    double us = 0;
    int cached[kClasses], cached_xw[kClasses];
    if (cache_lookup(cache_path, key, &order, &mult, &us, cached, cached_xw)) {
        for (int c = 0; c < kClasses; ++c) {
            B->chunks[c] = cached[c];
            B->xw[c] = cached_xw[c];
        }
        mf_status st = upload_items(B, order);
        if (st != MF_OK) return st;
        B->n_wg = B->num_cus * mult;
        B->tuned_us = us;
        return MF_OK;
    }
    // 1. tile shape per class (cross-section 4x2 or 2x4, tile height NZ / 1..4), by
    //    coordinate descent on the whole batch's time (round-robin order, as many
    //    workgroups per CU as the kernel is built for), classes with the most columns first
    int present[kClasses] = {0};
    for (size_t k = 0; k < B->probs.size(); ++k) present[B->cls[k]] += (int)batch_units_of(B->probs[k].P, 1, 4);
    std::vector<int> byw;
    for (int c = 0; c < kClasses; ++c)
        if (present[c] > 0) byw.push_back(c);
    std::sort(byw.begin(), byw.end(), [&](int a, int b) { return present[a] > present[b]; });
    for (int c = 0; c < kClasses; ++c) {
        B->chunks[c] = 1;
        B->xw[c] = 4;
    }
    const int max_mult = batch_max_wg_per_cu(B->prec);
    B->n_wg = B->num_cus * max_mult;
    double best = 1e300;
    {
        mf_status st = upload_items(B, 1);
        if (st != MF_OK) return st;
        st = time_config(B, s, &best);
        if (st != MF_OK) return st;
    }
    for (int c : byw) {
        int keep = B->chunks[c], keep_xw = B->xw[c];
        for (int x : {4, 2}) {
            for (int ch = 1; ch <= kMaxChunks; ++ch) {
                if (x == 4 && ch == 1) continue;  // the starting shape, timed above
                B->chunks[c] = ch;
                B->xw[c] = x;
                mf_status st = upload_items(B, 1);
                if (st != MF_OK) return st;
                double t = 0;
                st = time_config(B, s, &t);
                if (st != MF_OK) return st;
                if (t < best) {
                    best = t;
                    keep = ch;
                    keep_xw = x;
                }
            }
        }
        B->chunks[c] = keep;
        B->xw[c] = keep_xw;
    }
    // 2. launch shape for those tiles: work-item order x workgroups per CU
    best = 1e300;
    int best_order = 1, best_mult = 1;
    for (int o = 0; o < 3; ++o) {
        mf_status st = upload_items(B, o);
        if (st != MF_OK) return st;
        for (int m = 1; m <= max_mult; ++m) {
            B->n_wg = B->num_cus * m;
            double t = 0;
            st = time_config(B, s, &t);
            if (st != MF_OK) return st;
            if (t < best) {
                best = t;
                best_order = o;
                best_mult = m;
            }
        }
    }
    mf_status st = upload_items(B, best_order);
    if (st != MF_OK) return st;
    B->n_wg = B->num_cus * best_mult;
    B->tuned_us = best;
    cache_store(cache_path, key, best_order, best_mult, best, B->chunks, B->xw);
    return MF_OK;
}

mf_status mf_batch_run(mf_batch_t* B, void* stream)
{
    if (!B) return set_error(MF_ERR_ARG, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    for (auto& a : B->probs) const_cast<mf_pattern_s*>(a.P)->last_stream = s;
    if (!s) return launch(B, s);  // the default stream cannot be captured
    if (!B->exec || B->graph_stream != s) {
        drop_graph(B);
        MF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        mf_status st = launch(B, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != MF_OK) return st;
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
        B->graph = g;
        MF_HIP(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
        B->graph_stream = s;
    }
    MF_HIP(hipGraphLaunch(B->exec, s));
    return MF_OK;
}

mf_status mf_batch_info(const mf_batch_t* B, int64_t* n_items, int32_t* n_workgroups, int32_t* order,
                        int32_t* graphed, double* tuned_us)
{
    if (!B) return set_error(MF_ERR_ARG, "batch is NULL");
    if (n_items) *n_items = B->n_items;
    if (n_workgroups) *n_workgroups = B->n_wg;
    if (order) *order = B->order;
    if (graphed) *graphed = B->exec != nullptr;
    if (tuned_us) *tuned_us = B->tuned_us;
    return MF_OK;
}

mf_status mf_batch_tiles(const mf_batch_t* B, int32_t* n_classes, int32_t* problems, int32_t* chunks,
                         int32_t* cross_x)
{
    if (!B) return set_error(MF_ERR_ARG, "batch is NULL");
    if (n_classes) *n_classes = kClasses;
    for (int c = 0; c < kClasses; ++c) {
        if (problems) {
            problems[c] = 0;
            for (int k : B->cls) problems[c] += k == c;
        }
        if (chunks) chunks[c] = B->chunks[c];
        if (cross_x) cross_x[c] = B->xw[c];
    }
    return MF_OK;
}

void mf_batch_destroy(mf_batch_t* B)
{
    if (!B) return;
    if (B->graph_stream) (void)hipStreamSynchronize(B->graph_stream);
    free_batch(B);
}

}  // extern "C"
