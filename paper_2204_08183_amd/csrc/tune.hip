// Autotuning of the launch shapes.  The paper leaves the block size and the
// items per thread of its fused scan kernel as tunable constants (Sec. 2.7);
// here the tuned quantities are the positions per thread of the
// single-pass fused kernel (tiles of 256 x {4, 8, 16, 32} positions) and
// the segment shape of the persistent sweep (block x positions per thread).
// A choice is kept per (what is tuned, model, storage of e, 0/1 or valued
// design, size bucket = ceil(log2 n)) in a process-wide table; a launch
// consults the table and falls back to the built-in rule when the table
// has no entry.  The tuning calls time every candidate on the caller's own
// data with HIP events and keep the fastest; the table can be written to
// and read from a text file, each line tagged with the GPU architecture it
// was measured on.
#include <map>
#include <mutex>
#include <stdio.h>
#include <string.h>

#include "ss_internal.h"

namespace ss {
namespace {

struct Key {
    int32_t kind, model, storage, valued, bucket;
    bool operator<(const Key &o) const
    {
        return memcmp(this, &o, sizeof(Key)) < 0;
    }
};

std::mutex g_mu;
std::map<Key, int32_t> g_table;

int32_t bucket_of(int64_t n)
{
    int32_t b = 0;
    while (b < 62 && ((int64_t)1 << b) < n) ++b;
    return b;
}

Key make_key(int32_t kind, int32_t model, int32_t storage, int32_t valued, int64_t n)
{
    Key k;
    memset(&k, 0, sizeof(k));
    k.kind = kind;
    k.model = model;
    k.storage = storage;
    k.valued = valued ? 1 : 0;
    k.bucket = bucket_of(n);
    return k;
}

bool valid_choice(int32_t kind, int32_t model, int32_t storage, int32_t choice)
{
    if (kind == SS_TUNE_GRAD_HESS)
        return choice == 4 || choice == 8 || choice == 16 || choice == 32;
    if (kind == SS_TUNE_SWEEP) {
        if (storage != SS_STORAGE_F64) return false;
        for (int c : {25608, 25616, 51208, 51216})
            if (choice == c) return !(choice == 51216 && model == SS_FINE_GRAY);
        return false;
    }
    return false;
}

bool bad_key(int32_t kind, int32_t model, int32_t storage)
{
    return (kind != SS_TUNE_GRAD_HESS && kind != SS_TUNE_SWEEP) ||
           (model != SS_COX && model != SS_FINE_GRAY) || storage < SS_STORAGE_F64 ||
           storage > SS_STORAGE_F32_SUMS32;
}

int32_t device_arch(char *out, size_t len)
{
    int dev = 0;
    SS_HIP_CHECK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SS_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    snprintf(out, len, "%s", prop.gcnArchName);
    // the architecture name up to the first feature flag (gfx950:sramecc+...)
    char *colon = strchr(out, ':');
    if (colon) *colon = '\0';
    return SS_OK;
}

}  // namespace

TuneForce &tune_force()
{
    static thread_local TuneForce f = {-1, 0};
    return f;
}

int32_t tune_lookup(int32_t kind, int32_t model, int32_t storage, int32_t valued, int64_t n)
{
    const TuneForce &f = tune_force();
    if (f.choice && f.kind == kind) return f.choice;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_table.find(make_key(kind, model, storage, valued, n));
    return it == g_table.end() ? 0 : it->second;
}

}  // namespace ss

using namespace ss;

extern "C" {

int32_t ss_tune_get(int32_t kind, int32_t model, int32_t storage, int32_t valued, int64_t n)
{
    if (bad_key(kind, model, storage) || n < 1) return SS_EINVAL;
    const int32_t t = tune_lookup(kind, model, storage, valued, n);
    if (t) return t;
    return kind == SS_TUNE_GRAD_HESS ? default_ipt(n) : 0;
}

int32_t ss_tune_has(int32_t kind, int32_t model, int32_t storage, int32_t valued, int64_t n)
{
    if (bad_key(kind, model, storage) || n < 1) return SS_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_table.count(make_key(kind, model, storage, valued, n)) ? 1 : 0;
}

int32_t ss_tune_set(int32_t kind, int32_t model, int32_t storage, int32_t valued, int64_t n,
                    int32_t choice)
{
    if (bad_key(kind, model, storage) || n < 1) return SS_EINVAL;
    if (choice != 0 && !valid_choice(kind, model, storage, choice)) return SS_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    const Key k = make_key(kind, model, storage, valued, n);
    if (choice == 0)
        g_table.erase(k);
    else
        g_table[k] = choice;
    return SS_OK;
}

int32_t ss_tune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_table.clear();
    return SS_OK;
}

int32_t ss_tune_save(const char *path)
{
    if (!path) return SS_EINVAL;
    char arch[64];
    const int32_t rc = device_arch(arch, sizeof(arch));
    if (rc != SS_OK) return rc;
    FILE *f = fopen(path, "w");
    if (!f) return SS_EINVAL;
    fprintf(f, "# survscan launch shapes: arch kind model storage valued log2n choice\n");
    {
        std::lock_guard<std::mutex> lock(g_mu);
        for (const auto &kv : g_table)
            fprintf(f, "%s %d %d %d %d %d %d\n", arch, kv.first.kind, kv.first.model,
                    kv.first.storage, kv.first.valued, kv.first.bucket, kv.second);
    }
    return fclose(f) == 0 ? SS_OK : SS_EINVAL;
}

int32_t ss_tune_load(const char *path, int32_t *loaded)
{
    if (!path) return SS_EINVAL;
    char arch[64];
    const int32_t rc = device_arch(arch, sizeof(arch));
    if (rc != SS_OK) return rc;
    FILE *f = fopen(path, "r");
    if (!f) return SS_EINVAL;
    char line[256];
    int32_t count = 0;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        char a[64];
        int kind, model, storage, valued, bucket, choice;
        if (sscanf(line, "%63s %d %d %d %d %d %d", a, &kind, &model, &storage, &valued,
                   &bucket, &choice) != 7)
            continue;
        // entries measured on another architecture are ignored
        if (strcmp(a, arch) != 0) continue;
        if (bad_key(kind, model, storage) || bucket < 0 || bucket > 62) continue;
        if (!valid_choice(kind, model, storage, choice)) continue;
        Key k;
        memset(&k, 0, sizeof(k));
        k.kind = kind;
        k.model = model;
        k.storage = storage;
        k.valued = valued ? 1 : 0;
        k.bucket = bucket;
        std::lock_guard<std::mutex> lock(g_mu);
        g_table[k] = choice;
        ++count;
    }
    fclose(f);
    if (loaded) *loaded = count;
    return SS_OK;
}

}  // extern "C"
