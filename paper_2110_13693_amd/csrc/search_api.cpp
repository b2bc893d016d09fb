// Host side of the genetic-search entry points of include/wo.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <vector>
#include <memory>
#include <new>
#include <utility>

#include "wo_common.h"
#include "wo_internal.h"
#include "wo_search.h"
#include "wo_surrogate.h"

using namespace wo;

struct wo_search {
    wo_wh *wh = nullptr;
    int32_t inst = 0;
    int P = 0, n = 0, C = 0;
    wo_search_params prm{};
    uint8_t *pz = nullptr, *cz = nullptr;
    uint16_t *ps = nullptr, *cs = nullptr;
    int32_t *pd = nullptr, *cd = nullptr;
    uint8_t *cand_zone = nullptr;
    int32_t *cand_parent = nullptr, *kept = nullptr, *worst = nullptr;
    float *pred = nullptr;
    int32_t *best = nullptr;
    uint32_t gen = 0;
    std::atomic<int> busy{0};
};

namespace {

template <typename T>
wo_status alloc(T **p, size_t count)
{
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(16, count * sizeof(T)));
    if (e != hipSuccess) {
        *p = nullptr;
        return wo_fail(WO_E_NOMEM, "hipMalloc(%zu) failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    return WO_OK;
}

struct SearchBusy {
    std::atomic<int> *f;
    bool ok;
    explicit SearchBusy(std::atomic<int> *flag) : f(flag)
    {
        int z = 0;
        ok = f->compare_exchange_strong(z, 1);
    }
    ~SearchBusy()
    {
        if (ok) f->store(0);
    }
};

}  // namespace

extern "C" wo_status wo_search_create(wo_wh *wh, int32_t inst, const wo_search_params *prm,
                                      const uint8_t *d_init_zone_of, const uint16_t *d_init_seq, void *stream,
                                      wo_search **out)
{
    if (!out) return wo_fail(WO_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!wh || !prm) return wo_fail(WO_E_INVAL, "NULL argument");
    if (inst < 0 || inst >= instance_count(wh)) return wo_fail(WO_E_RANGE, "instance %d out of range", inst);
    if (!d_init_zone_of || !d_init_seq) return wo_fail(WO_E_INVAL, "initial population is required");
    const int n = instance_orders(wh, inst);
    if (prm->population < 2 || prm->population > (1 << 24))
        return wo_fail(WO_E_RANGE, "population must be in [2, 2^24]");
    if (prm->tournament < 1 || prm->tournament > 64) return wo_fail(WO_E_RANGE, "tournament size in [1, 64]");
    if (prm->candidates < 0 || prm->candidates > (1 << 24)) return wo_fail(WO_E_RANGE, "candidates in [0, 2^24]");
    if (prm->candidates > 0 &&
        (prm->keep < 1 || prm->keep > prm->candidates || prm->keep > WO_SCREEN_MAX_KEEP ||
         prm->keep >= prm->population))
        return wo_fail(WO_E_RANGE, "keep must be in [1, min(candidates, %d, population - 1)]", WO_SCREEN_MAX_KEEP);
    if (breed_lds_bytes(n) > 160u * 1024u - 256u) return wo_fail(WO_E_RANGE, "%d orders exceed the breeding LDS", n);
    if (wo_fault_injected()) return wo_fail(WO_E_NOMEM, "injected allocation failure");
    wo_search *s = new (std::nothrow) wo_search;
    if (!s) return wo_fail(WO_E_NOMEM, "host allocation failed");
    std::unique_ptr<wo_search, wo_status (*)(wo_search *)> guard(s, wo_search_free);
    s->wh = wh;
    s->inst = inst;
    s->P = prm->population;
    s->n = n;
    s->C = instance_categories(wh, inst);
    s->prm = *prm;
    const size_t P = (size_t)s->P;
    wo_status r;
    if ((r = alloc(&s->pz, P * 64)) || (r = alloc(&s->cz, P * 64)) || (r = alloc(&s->ps, P * n)) ||
        (r = alloc(&s->cs, P * n)) || (r = alloc(&s->pd, P)) || (r = alloc(&s->cd, P)) || (r = alloc(&s->best, 1)))
        return r;
    if (prm->candidates > 0) {
        const size_t K = (size_t)prm->candidates;
        if ((r = alloc(&s->cand_zone, K * 64)) || (r = alloc(&s->cand_parent, K)) || (r = alloc(&s->pred, K)) ||
            (r = alloc(&s->kept, (size_t)prm->keep)) || (r = alloc(&s->worst, (size_t)prm->keep)))
            return r;
    }
    hipStream_t st = (hipStream_t)stream;
    WO_HIP(hipMemcpyAsync(s->pz, d_init_zone_of, P * 64, hipMemcpyDeviceToDevice, st));
    WO_HIP(hipMemcpyAsync(s->ps, d_init_seq, P * n * 2, hipMemcpyDeviceToDevice, st));
    if ((r = eval_instance(wh, inst, s->P, s->pz, s->ps, s->pd, nullptr, st))) return r;
    WO_HIP(launch_argmin(s->pd, s->P, s->best, st));
    WO_HIP(hipStreamSynchronize(st));
    guard.release();
    *out = s;
    return WO_OK;
}

extern "C" wo_status wo_search_free(wo_search *s)
{
    if (!s) return WO_OK;
    (void)hipDeviceSynchronize();
    void *bufs[] = {s->pz, s->cz, s->ps, s->cs, s->pd, s->cd, s->cand_zone, s->cand_parent, s->kept, s->worst,
                    s->pred, s->best};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete s;
    return WO_OK;
}

extern "C" wo_status wo_search_step(wo_wh *wh, wo_search *s, wo_sur *sur, int32_t n_generations, void *stream)
{
    if (!wh || !s) return wo_fail(WO_E_INVAL, "NULL handle");
    if (wh != s->wh) return wo_fail(WO_E_INVAL, "search belongs to another warehouse handle");
    SearchBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "search is in use by another thread");
    if (n_generations < 0) return wo_fail(WO_E_INVAL, "n_generations < 0");
    if (sur && s->prm.candidates == 0)
        return wo_fail(WO_E_STATE, "search was created without screening candidates");
    hipStream_t st = (hipStream_t)stream;
    wo_status r;
    for (int g = 0; g < n_generations; g++) {
        if (!sur) {
            BreedArgs b{};
            b.pz = s->pz;
            b.ps = s->ps;
            b.pd = s->pd;
            b.P = s->P;
            b.n = s->n;
            b.C = s->C;
            b.tsize = s->prm.tournament;
            b.mode = 0;
            b.thr = s->prm.mutation_threshold;
            b.gen = s->gen;
            b.seed = s->prm.seed;
            b.best = s->best;
            b.cz = s->cz;
            b.cs = s->cs;
            WO_HIP(launch_breed(b, s->P, st));
            if ((r = eval_instance(wh, s->inst, s->P, s->cz, s->cs, s->cd, nullptr, st))) return r;
            std::swap(s->pz, s->cz);
            std::swap(s->ps, s->cs);
            std::swap(s->pd, s->cd);
        } else {
            CandArgs c{};
            c.pz = s->pz;
            c.pd = s->pd;
            c.P = s->P;
            c.C = s->C;
            c.K = s->prm.candidates;
            c.tsize = s->prm.tournament;
            c.thr = s->prm.mutation_threshold;
            c.gen = s->gen;
            c.seed = s->prm.seed;
            c.cand_zone = s->cand_zone;
            c.cand_parent = s->cand_parent;
            WO_HIP(launch_candidates(c, st));
            if ((r = wo_screen_plans(wh, s->inst, sur, s->prm.candidates, s->cand_zone, s->pred, s->prm.keep,
                                     s->kept, stream)))
                return r;
            BreedArgs b{};
            b.pz = s->pz;
            b.ps = s->ps;
            b.pd = s->pd;
            b.P = s->P;
            b.n = s->n;
            b.C = s->C;
            b.tsize = s->prm.tournament;
            b.mode = 1;
            b.thr = s->prm.mutation_threshold;
            b.gen = s->gen;
            b.seed = s->prm.seed;
            b.kept = s->kept;
            b.cand_parent = s->cand_parent;
            b.cand_zone = s->cand_zone;
            b.cz = s->cz;
            b.cs = s->cs;
            WO_HIP(launch_breed(b, s->prm.keep, st));
            if ((r = eval_instance(wh, s->inst, s->prm.keep, s->cz, s->cs, s->cd, nullptr, st))) return r;
            WO_HIP(launch_worst(s->pd, s->P, s->prm.keep, s->worst, st));
            ReplaceArgs rp{};
            rp.pz = s->pz;
            rp.ps = s->ps;
            rp.pd = s->pd;
            rp.cz = s->cz;
            rp.cs = s->cs;
            rp.cd = s->cd;
            rp.worst = s->worst;
            rp.n = s->n;
            WO_HIP(launch_replace(rp, s->prm.keep, st));
        }
        WO_HIP(launch_argmin(s->pd, s->P, s->best, st));
        s->gen++;
    }
    return WO_OK;
}

extern "C" wo_status wo_search_best(wo_search *s, uint8_t *h_zone_of, uint16_t *h_seq, int32_t *h_dist,
                                    int32_t *h_generation, void *stream)
{
    if (!s) return wo_fail(WO_E_INVAL, "NULL handle");
    SearchBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "search is in use by another thread");
    hipStream_t st = (hipStream_t)stream;
    int32_t b = 0;
    WO_HIP(hipMemcpyAsync(&b, s->best, 4, hipMemcpyDeviceToHost, st));
    WO_HIP(hipStreamSynchronize(st));
    if (h_zone_of) WO_HIP(hipMemcpyAsync(h_zone_of, s->pz + (size_t)b * 64, 64, hipMemcpyDeviceToHost, st));
    if (h_seq) WO_HIP(hipMemcpyAsync(h_seq, s->ps + (size_t)b * s->n, (size_t)s->n * 2, hipMemcpyDeviceToHost, st));
    if (h_dist) WO_HIP(hipMemcpyAsync(h_dist, s->pd + b, 4, hipMemcpyDeviceToHost, st));
    WO_HIP(hipStreamSynchronize(st));
    if (h_generation) *h_generation = (int32_t)s->gen;
    return WO_OK;
}

extern "C" wo_status wo_search_population(wo_search *s, uint8_t *d_zone_of, uint16_t *d_seq, int32_t *d_dist,
                                          int32_t *d_last_kept, void *stream)
{
    if (!s) return wo_fail(WO_E_INVAL, "NULL handle");
    SearchBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "search is in use by another thread");
    hipStream_t st = (hipStream_t)stream;
    const size_t P = (size_t)s->P;
    if (d_zone_of) WO_HIP(hipMemcpyAsync(d_zone_of, s->pz, P * 64, hipMemcpyDeviceToDevice, st));
    if (d_seq) WO_HIP(hipMemcpyAsync(d_seq, s->ps, P * s->n * 2, hipMemcpyDeviceToDevice, st));
    if (d_dist) WO_HIP(hipMemcpyAsync(d_dist, s->pd, P * 4, hipMemcpyDeviceToDevice, st));
    if (d_last_kept) {
        if (!s->kept) return wo_fail(WO_E_STATE, "search has no screening state");
        WO_HIP(hipMemcpyAsync(d_last_kept, s->kept, (size_t)s->prm.keep * 4, hipMemcpyDeviceToDevice, st));
    }
    return WO_OK;
}

// Checkpoint: a header (magic, order and category counts, the parameters, the
// generation counter), then the population's zone rows, sequences and
// distances.  The random numbers are a function of (seed, generation, child,
// position), so a search resumed from the file continues bit-exactly.
namespace {
struct SearchFileHeader {
    char magic[8];
    int32_t n_orders, n_cat, population, reserved;
    wo_search_params prm;
    uint32_t gen, reserved2;
};
const char kSearchMagic[8] = {'W', 'O', 'S', 'R', 'C', 'H', '0', '1'};
}  // namespace

extern "C" wo_status wo_search_save(wo_search *s, const char *path, void *stream)
{
    if (!s || !path) return wo_fail(WO_E_INVAL, "NULL argument");
    SearchBusy busy(&s->busy);
    if (!busy.ok) return wo_fail(WO_E_STATE, "search is in use by another thread");
    const size_t P = (size_t)s->P, n = (size_t)s->n;
    std::vector<uint8_t> z(P * 64);
    std::vector<uint16_t> q(P * n);
    std::vector<int32_t> d(P);
    hipStream_t st = (hipStream_t)stream;
    WO_HIP(hipMemcpyAsync(z.data(), s->pz, P * 64, hipMemcpyDeviceToHost, st));
    WO_HIP(hipMemcpyAsync(q.data(), s->ps, P * n * 2, hipMemcpyDeviceToHost, st));
    WO_HIP(hipMemcpyAsync(d.data(), s->pd, P * 4, hipMemcpyDeviceToHost, st));
    WO_HIP(hipStreamSynchronize(st));
    SearchFileHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kSearchMagic, 8);
    h.n_orders = s->n;
    h.n_cat = s->C;
    h.population = s->P;
    h.prm = s->prm;
    h.gen = s->gen;
    FILE *f = fopen(path, "wb");
    if (!f) return wo_fail(WO_E_INVAL, "cannot open %s for writing", path);
    bool ok = fwrite(&h, sizeof h, 1, f) == 1 && fwrite(z.data(), 1, z.size(), f) == z.size() &&
              fwrite(q.data(), 2, q.size(), f) == q.size() && fwrite(d.data(), 4, d.size(), f) == d.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? WO_OK : wo_fail(WO_E_INVAL, "write to %s failed", path);
}

extern "C" wo_status wo_search_load(wo_wh *wh, int32_t inst, const char *path, void *stream, wo_search **out)
{
    if (!path || !out) return wo_fail(WO_E_INVAL, "NULL argument");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return wo_fail(WO_E_INVAL, "cannot open %s", path);
    SearchFileHeader h;
    bool ok = fread(&h, sizeof h, 1, f) == 1 && memcmp(h.magic, kSearchMagic, 8) == 0 && h.n_orders >= 1 &&
              h.n_orders <= WO_MAX_ORDERS && h.population >= 2 && h.population <= (1 << 24) && h.n_cat >= 1 &&
              h.n_cat <= WO_MAX_CATEGORIES && h.prm.population == h.population;
    // the file must be exactly as long as its header says before anything
    // is sized from the header
    if (ok) {
        const uint64_t P = (uint64_t)h.population, n = (uint64_t)h.n_orders;
        const uint64_t want = sizeof h + P * 64 + P * n * 2 + P * 4;
        ok = fseek(f, 0, SEEK_END) == 0;
        const long len = ok ? ftell(f) : -1;
        ok = ok && len >= 0 && (uint64_t)len == want && fseek(f, (long)sizeof h, SEEK_SET) == 0;
    }
    std::vector<uint8_t> z;
    std::vector<uint16_t> q;
    std::vector<int32_t> d;
    if (ok) {
        const size_t P = (size_t)h.population, n = (size_t)h.n_orders;
        try {
            z.resize(P * 64);
            q.resize(P * n);
            d.resize(P);
        } catch (const std::bad_alloc &) {
            fclose(f);
            return wo_fail(WO_E_NOMEM, "no host memory for a checkpoint of %zu plans", P);
        }
        ok = fread(z.data(), 1, z.size(), f) == z.size() && fread(q.data(), 2, q.size(), f) == q.size() &&
             fread(d.data(), 4, d.size(), f) == d.size();
    }
    fclose(f);
    if (!ok) return wo_fail(WO_E_INVAL, "%s is not a search checkpoint", path);
    if (!wh) return wo_fail(WO_E_INVAL, "NULL warehouse handle");
    if (inst < 0 || inst >= instance_count(wh)) return wo_fail(WO_E_RANGE, "instance %d out of range", inst);
    if (instance_orders(wh, inst) != h.n_orders || instance_categories(wh, inst) != h.n_cat)
        return wo_fail(WO_E_INVAL, "the checkpoint has %d orders and %d categories, the instance %d and %d",
                       h.n_orders, h.n_cat, instance_orders(wh, inst), instance_categories(wh, inst));
    // the population is re-evaluated on creation; the distances must come
    // out as saved, which also checks that the instance is the same
    uint8_t *dz = nullptr;
    uint16_t *dq = nullptr;
    wo_status r;
    if ((r = alloc(&dz, z.size())) || (r = alloc(&dq, q.size()))) {
        if (dz) (void)hipFree(dz);
        return r;
    }
    hipStream_t st = (hipStream_t)stream;
    wo_search *s = nullptr;
    if (hipMemcpyAsync(dz, z.data(), z.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dq, q.data(), q.size() * 2, hipMemcpyHostToDevice, st) != hipSuccess) {
        r = wo_fail(WO_E_DEVICE, "upload of the checkpoint failed");
    } else {
        r = wo_search_create(wh, inst, &h.prm, dz, dq, stream, &s);
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(dz);
    (void)hipFree(dq);
    if (r) return r;
    std::vector<int32_t> d2(d.size());
    if (hipMemcpy(d2.data(), s->pd, d2.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) {
        wo_search_free(s);
        return wo_fail(WO_E_DEVICE, "read-back of the distances failed");
    }
    if (d2 != d) {
        wo_search_free(s);
        return wo_fail(WO_E_INVAL, "the checkpoint's distances differ on this instance");
    }
    s->gen = h.gen;
    *out = s;
    return WO_OK;
}
