// Tuning of the batched kernel: per size class, the panel width and the form
// of the trailing update, kept in one process-wide table per (TW, TF) pair,
// and the autotuner that measures the candidates on the device and caches
// the winners in a text file.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mpir_internal.h"

using namespace mpir;

namespace {

std::mutex g_tune_mu;
mpir_batch_tuning g_tune[2][3];   // [tw == F32][tf: F32, F16, BF16]
bool g_tune_init = false;

void tune_defaults(mpir_batch_tuning *t) {
    std::memset(t, 0, sizeof(*t));
    const int nm[] = {64, 128, 256, 512, 768, 1024};
    t->nclass = 6;
    for (int k = 0; k < 6; ++k) {
        t->nmax[k] = nm[k];
        t->panel[k] = 32;
        t->update[k] = 0;
    }
}

bool prec_ok(int tw, int tf) {
    return (tw == MPIR_F64 || tw == MPIR_F32) && (tf == MPIR_F32 || tf == MPIR_F16 || tf == MPIR_BF16);
}

mpir_batch_tuning &slot(int tw, int tf) {
    if (!g_tune_init) {
        for (auto &a : g_tune)
            for (auto &b : a) tune_defaults(&b);
        g_tune_init = true;
    }
    return g_tune[tw == MPIR_F32][tf == MPIR_F32 ? 0 : tf == MPIR_F16 ? 1 : 2];
}

bool tuning_valid(const mpir_batch_tuning *t) {
    if (t->nclass < 1 || t->nclass > MPIR_TUNE_CLASSES) return false;
    for (int k = 0; k < t->nclass; ++k) {
        if (t->nmax[k] < 1 || t->nmax[k] > batched_max_n()) return false;
        if (k > 0 && t->nmax[k] <= t->nmax[k - 1]) return false;
        if (t->panel[k] != 16 && t->panel[k] != 32) return false;
        if (t->update[k] < 0 || t->update[k] > 2) return false;
        if (t->update[k] == 2 && t->panel[k] != 32) return false;
    }
    return t->nmax[t->nclass - 1] == batched_max_n();
}

// Synthetic tuning systems: off-diagonal entries uniform in [-1, 1] / n from
// a counter hash of (system, row, column, seed), diagonal 1 + |hash|: well
// conditioned, so every candidate runs the same refinement.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352du;
    x ^= x >> 15; x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <typename T>
__global__ void k_tune_fill(T *A, T *b, int64_t n, int64_t count, uint32_t seed) {
    const int64_t per = n * n, tot = per * count;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sys = e / per, r = e - sys * per, j = r / n, i = r - j * n;   // column-major
        const uint32_t h = mix32(mix32((uint32_t)sys * 0x9e3779b9u ^ seed) + (uint32_t)i * 0x85ebca6bu +
                                 (uint32_t)j * 0xc2b2ae35u);
        const double u = (double)h * (2.0 / 4294967296.0) - 1.0;
        A[e] = (T)(i == j ? 1.0 + fabs(u) : u / (double)n);
        if (i == 0 && j == 0) {
            for (int64_t q = 0; q < n; ++q) b[sys * n + q] = (T)1.0;
        }
    }
}

std::string device_key(int tw, int tf) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s cus=%d tw=%d tf=%d", prop.gcnArchName, prop.multiProcessorCount, tw, tf);
    return buf;
}

bool read_cache(const char *path, const std::string &key, mpir_batch_tuning *t) {
    FILE *fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool ok = false;
    mpir_batch_tuning r;
    std::memset(&r, 0, sizeof r);
    if (std::fgets(line, sizeof line, fp) && std::strncmp(line, "mpir-batch-tuning 1", 19) == 0 &&
        std::fgets(line, sizeof line, fp)) {
        line[std::strcspn(line, "\n")] = 0;
        if (key == line && std::fgets(line, sizeof line, fp) && std::sscanf(line, "%d", &r.nclass) == 1 &&
            r.nclass >= 1 && r.nclass <= MPIR_TUNE_CLASSES) {
            ok = true;
            for (int k = 0; k < r.nclass && ok; ++k)
                ok = std::fgets(line, sizeof line, fp) &&
                     std::sscanf(line, "%d %d %d %lf", &r.nmax[k], &r.panel[k], &r.update[k], &r.ms[k]) == 4;
        }
    }
    std::fclose(fp);
    if (!ok || !tuning_valid(&r)) return false;
    r.from_cache = 1;
    *t = r;
    return true;
}

void write_cache(const char *path, const std::string &key, const mpir_batch_tuning *t) {
    FILE *fp = std::fopen(path, "w");
    if (!fp) return;
    std::fprintf(fp, "mpir-batch-tuning 1\n%s\n%d\n", key.c_str(), t->nclass);
    for (int k = 0; k < t->nclass; ++k)
        std::fprintf(fp, "%d %d %d %.6f\n", t->nmax[k], t->panel[k], t->update[k], t->ms[k]);
    std::fclose(fp);
}

}  // namespace

namespace mpir {

int64_t batch_cfg(int tw, int tf, int64_t n, const mpir_batch_tuning *tab) {
    mpir_batch_tuning t;
    if (tab) {
        t = *tab;
    } else {
        std::lock_guard<std::mutex> g(g_tune_mu);
        t = slot(tw, tf);
    }
    int k = 0;
    while (k + 1 < t.nclass && n > t.nmax[k]) ++k;
    return (int64_t)t.panel[k] | ((int64_t)t.update[k] << 8);
}

}  // namespace mpir

extern "C" {

mpir_status mpir_batch_get_tuning(mpir_prec tw, mpir_prec tf, mpir_batch_tuning *t) {
    if (!t || !prec_ok(tw, tf)) return MPIR_ERR_ARG;
    std::lock_guard<std::mutex> g(g_tune_mu);
    *t = slot(tw, tf);
    return MPIR_OK;
}

mpir_status mpir_batch_set_tuning(mpir_prec tw, mpir_prec tf, const mpir_batch_tuning *t) {
    if (!prec_ok(tw, tf)) return MPIR_ERR_ARG;
    if (t && !tuning_valid(t)) return MPIR_ERR_ARG;
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (t) slot(tw, tf) = *t;
    else tune_defaults(&slot(tw, tf));
    return MPIR_OK;
}

mpir_status mpir_batch_autotune(mpir_prec tw, mpir_prec tf, const char *cache_path, void *hip_stream,
                                mpir_batch_tuning *out) {
    if (!prec_ok(tw, tf)) return MPIR_ERR_ARG;
    const std::string key = device_key(tw, tf);
    if (key.empty()) return MPIR_ERR_HIP;
    mpir_batch_tuning res;
    if (cache_path && read_cache(cache_path, key, &res)) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        slot(tw, tf) = res;
        if (out) *out = res;
        return MPIR_OK;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return MPIR_ERR_HIP;
    tune_defaults(&res);
    const int count = 2 * (cus > 0 ? cus : 64);     // two systems per compute unit
    const size_t esz = tw == MPIR_F64 ? 8 : 4;
    const int cand_panel[] = {16, 32}, cand_upd[] = {0, 1, 2};
    mpir_status st = MPIR_OK;
    for (int k = 0; k < res.nclass && st == MPIR_OK; ++k) {
        const int lo = k ? res.nmax[k - 1] : 0;
        const int64_t n = (lo + res.nmax[k] + 1) / 2;
        void *A = nullptr, *B = nullptr, *X = nullptr;
        if (hipMalloc(&A, esz * n * n * count) != hipSuccess || hipMalloc(&B, esz * n * count) != hipSuccess ||
            hipMalloc(&X, esz * n * count) != hipSuccess) {
            hipFree(A); hipFree(B); hipFree(X);
            return MPIR_ERR_ALLOC;
        }
        if (tw == MPIR_F64) k_tune_fill<double><<<1024, 256, 0, s>>>((double *)A, (double *)B, n, count, 2311u + k);
        else k_tune_fill<float><<<1024, 256, 0, s>>>((float *)A, (float *)B, n, count, 2311u + k);
        std::vector<int64_t> ns(count, n), ldas(count, n);
        std::vector<const void *> pa(count), pb(count);
        std::vector<void *> px(count);
        for (int q = 0; q < count; ++q) {
            pa[q] = (const char *)A + esz * n * n * q;
            pb[q] = (const char *)B + esz * n * q;
            px[q] = (char *)X + esz * n * q;
        }
        double best = -1.0;
        for (int pw : cand_panel)
            for (int up : cand_upd) {
                if (up == 2 && pw != 32) continue;      // panels in pairs: 32-column panels
                mpir_batch_tuning one;
                std::memset(&one, 0, sizeof one);
                one.nclass = 1;
                one.nmax[0] = batched_max_n();
                one.panel[0] = pw;
                one.update[0] = up;
                mpir_batch b = nullptr;
                mpir_term term;
                mpir_term_default(&term);
                st = batch_create_with(count, ns.data(), pa.data(), ldas.data(), pb.data(), px.data(), tw, tf,
                                       MPIR_F64, &term, 0, hip_stream, &one, &b);
                if (st != MPIR_OK) break;
                double tbest = -1.0;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = MPIR_ERR_HIP;
                for (int rep = 0; rep < 3 && st == MPIR_OK; ++rep) {
                    if (hipEventRecord(e0, s) != hipSuccess) { st = MPIR_ERR_HIP; break; }
                    const mpir_status rs = mpir_batch_run(b, nullptr);
                    if (rs != MPIR_OK) { st = rs; break; }
                    float ms = 0.f;
                    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = MPIR_ERR_HIP; break; }
                    if (rep > 0 && (tbest < 0 || ms < tbest)) tbest = ms;     // first run warms up
                }
                if (e0) hipEventDestroy(e0);
                if (e1) hipEventDestroy(e1);
                mpir_batch_destroy(b);
                if (st != MPIR_OK) break;
                if (best < 0 || tbest < best) {
                    best = tbest;
                    res.panel[k] = pw;
                    res.update[k] = up;
                    res.ms[k] = tbest;
                }
            }
        hipFree(A);
        hipFree(B);
        hipFree(X);
    }
    if (st != MPIR_OK) return st;
    res.from_cache = 0;
    if (cache_path) write_cache(cache_path, key, &res);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        slot(tw, tf) = res;
    }
    if (out) *out = res;
    return MPIR_OK;
}

}  // extern "C"
