// batch.hip -- many independent problems of uneven size, viscosity and
// forcing, advanced by one launch of the fused kernel per step (block table
// maps each workgroup to its instance, tile and march chunk); the step
// launches of a run can be captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "kernels_general.hpp"
#include "march.hpp"

namespace dugks {
long long batch_resident_slots(int lattice, int dtype, bool uniform, int variant, int n_cu);
hipError_t batch_step_launch(int lattice, int dtype, bool uniform, int variant, const void* insts,
                             const long long* bstart, const BatchGeom* geom, int n, long long nblocks, const void* fin,
                             const void* forces, void* fout, const long long* step0, int step, hipStream_t st);
int fused_tile_variants(int lattice);
void fused_tile_shape(int lattice, int variant, int* bx, int* by);

// batch clock: set (reset != 0: s = add) or advance (s += add) the
// device-side step counter (kernel nodes, so a captured run replays them)
__global__ void k_batch_clock(long long* s, long long add, int reset)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *s = reset ? add : *s + add;
}

// initial state of every instance: rest at rho0 (Sec. III), t = t0
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_batch_init(const Inst<T>* __restrict__ insts,
                                                    const long long* __restrict__ cstart, int ninst, double t0,
                                                    T* __restrict__ f)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cstart[ninst]) return;
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    const Inst<T>& P = insts[lo];
    init_body<LAT, T>(P, c - cstart[lo], nullptr, nullptr, nullptr, tfac(P, t0), f + P.off);
}
}  // namespace dugks

using namespace dugks;

struct dugks_batch {
    int n = 0, lattice = 0, dtype = 0, D = 0, Q = 0, esize = 0;
    int tile = 0, chunk = 0;  // tile-shape variant and march chunk (0 = default) in use
    bool uniform = true;      // every instance on a uniform mesh
    bool any_field = false;   // some instance has a force field
    std::vector<dugks_config> cfgs;
    std::vector<std::vector<double>> faces_own;  // copies of custom face coordinates (cfgs[i].faces point here)
    std::vector<unsigned char> hinst;  // host images of Inst<T>, n of them
    void* insts_dev = nullptr;
    void* met_dev = nullptr;
    long long* bstart_dev = nullptr;
    long long* cstart_dev = nullptr;
    long long* step_dev = nullptr;  // device step counter (batch clock)
    BatchGeom* geom_dev = nullptr;
    long long nblocks = 0, ncells = 0;
    std::string err = "no error";
    // captured run
    hipGraphExec_t gexec = nullptr;
    const void* g_in = nullptr;
    void* g_out = nullptr;
    const void* g_forces = nullptr;
    int g_steps = -1;
    hipStream_t g_stream = nullptr;
};

static thread_local std::string g_batch_err = "no error";

static int bfail(dugks_batch* b, int code, const std::string& m)
{
    if (b) b->err = m;
    else g_batch_err = m;
    return code;
}

static void drop_graph(dugks_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->g_steps = -1;
}

namespace dugks {
template <typename T>
void fill_inst(const dugks_config* c, Inst<T>& P, T* met_dev, std::vector<T>& met_host);
size_t metric_len(const dugks_config* c);
}  // namespace dugks

// Workgroup geometry of every instance for tile-shape variant `tile` and
// march chunk `chunk`: tile counts, chunk and the workgroup prefix sum;
// uploaded synchronously (never inside a capture).  chunk > 0: the same chunk
// for every instance; chunk = 0: a chunk per instance from the chunk model
// (auto_chunk) with the device's resident workgroups shared among the
// instances in proportion to their cells, so that large instances march
// long chunks (fewer recomputed halo planes) and small ones short chunks
// (more workgroups at once).
static int set_geometry(dugks_batch* b, int tile, int chunk)
{
    const int n = b->n, D = b->D, M = D - 1;
    int bx, by;
    fused_tile_shape(b->lattice, tile, &bx, &by);
    long long slots = 0;
    if (chunk == 0) {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 0;
        slots = batch_resident_slots(b->lattice, b->dtype, b->uniform, tile, ncu);
    }
    std::vector<long long> bstart(n + 1, 0);
    std::vector<BatchGeom> geom(n);
    for (int i = 0; i < n; ++i) {
        const int* nn = b->cfgs[i].n;
        BatchGeom g;
        g.tiles0 = (nn[0] + bx - 3) / (bx - 2);
        g.tiles1 = D == 3 ? (nn[1] + by - 3) / (by - 2) : 1;
        if (chunk > 0) {
            g.chunk = std::min(chunk, nn[M]);
        } else {
            long long cells = 1;
            for (int a = 0; a < D; ++a) cells *= nn[a];
            const long long share = std::max(1LL, (long long)((double)slots * (double)cells / (double)b->ncells));
            g.chunk = auto_chunk((long long)g.tiles0 * g.tiles1, nn[M], share);
        }
        g.pad = 0;
        const int chunks = (nn[M] + g.chunk - 1) / g.chunk;
        geom[i] = g;
        bstart[i + 1] = bstart[i] + (long long)g.tiles0 * g.tiles1 * chunks;
    }
    if (bstart[n] > 0x7fffffffLL) return bfail(b, DUGKS_EUNSUPPORTED, "batch too large for one launch");
    if (hipMemcpy(b->bstart_dev, bstart.data(), sizeof(long long) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->geom_dev, geom.data(), sizeof(BatchGeom) * n, hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, DUGKS_EHIP, "batch geometry upload");
    drop_graph(b);
    b->nblocks = bstart[n];
    b->tile = tile;
    b->chunk = chunk;
    return DUGKS_OK;
}

template <typename T>
static int build_tables(dugks_batch* b, const int64_t* offsets, hipStream_t st)
{
    const int n = b->n;
    size_t mtot = 0;
    for (int i = 0; i < n; ++i) mtot += metric_len(&b->cfgs[i]);
    if (hipMalloc(&b->met_dev, mtot * sizeof(T)) != hipSuccess) return bfail(b, DUGKS_ENOMEM, "metric allocation");
    std::vector<T> mall;
    mall.reserve(mtot);
    std::vector<Inst<T>> insts(n);
    std::vector<long long> cstart(n + 1, 0);
    size_t moff = 0;
    for (int i = 0; i < n; ++i) {
        std::vector<T> mh;
        fill_inst<T>(&b->cfgs[i], insts[i], (T*)b->met_dev + moff, mh);
        moff += mh.size();
        mall.insert(mall.end(), mh.begin(), mh.end());
        insts[i].off = offsets[i];
        insts[i].foff = -1;
        cstart[i + 1] = cstart[i] + insts[i].nc;
    }
    b->ncells = cstart[n];
    b->hinst.resize(sizeof(Inst<T>) * n);
    std::memcpy(b->hinst.data(), insts.data(), b->hinst.size());
    if (hipMalloc(&b->insts_dev, b->hinst.size()) != hipSuccess ||
        hipMalloc((void**)&b->bstart_dev, sizeof(long long) * (n + 1)) != hipSuccess ||
        hipMalloc((void**)&b->cstart_dev, sizeof(long long) * (n + 1)) != hipSuccess ||
        hipMalloc((void**)&b->geom_dev, sizeof(BatchGeom) * n) != hipSuccess ||
        hipMalloc((void**)&b->step_dev, sizeof(long long)) != hipSuccess)
        return bfail(b, DUGKS_ENOMEM, "batch table allocation");
    if (hipMemcpy(b->met_dev, mall.data(), mall.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->insts_dev, b->hinst.data(), b->hinst.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->cstart_dev, cstart.data(), sizeof(long long) * (n + 1), hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, DUGKS_EHIP, "batch table upload");
    (void)st;
    return set_geometry(b, 0, 0);
}

extern "C" int dugks_batch_create(const dugks_config* cfgs, int n, const int64_t* offsets, void* stream,
                                  dugks_batch** out)
{
    if (!out) return bfail(nullptr, DUGKS_EINVAL, "null output pointer");
    *out = nullptr;
    if (!cfgs || !offsets || n < 1) return bfail(nullptr, DUGKS_EINVAL, "need at least one instance and offsets");
    for (int i = 0; i < n; ++i) {
        std::string why;
        if (validate(&cfgs[i], why) != DUGKS_OK) return bfail(nullptr, DUGKS_EINVAL, "instance " + std::to_string(i) + ": " + why);
        if (cfgs[i].lattice != cfgs[0].lattice || cfgs[i].dtype != cfgs[0].dtype)
            return bfail(nullptr, DUGKS_EINVAL, "all instances must share lattice and dtype");
        if (offsets[i] < 0) return bfail(nullptr, DUGKS_EINVAL, "negative offset");
        if (cfgs[i].model != DUGKS_MODEL_INCOMPRESSIBLE)
            return bfail(nullptr, DUGKS_EUNSUPPORTED, "batched instances use the incompressible model");
        if (cfgs[i].lattice == DUGKS_D3Q27) return bfail(nullptr, DUGKS_EUNSUPPORTED, "no batched D3Q27");
    }
    dugks_batch* b = new dugks_batch();
    b->n = n;
    b->lattice = cfgs[0].lattice;
    b->dtype = cfgs[0].dtype;
    b->D = b->lattice == DUGKS_D2Q9 ? 2 : 3;
    b->Q = b->lattice;
    b->esize = b->dtype == DUGKS_F64 ? 8 : 4;
    b->cfgs.assign(cfgs, cfgs + n);
    b->faces_own.resize((size_t)3 * n);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            b->cfgs[i].faces[a] = nullptr;
            if (a < b->D && cfgs[i].mesh[a] == DUGKS_CUSTOM) {
                std::vector<double>& own = b->faces_own[(size_t)3 * i + a];
                own.assign(cfgs[i].faces[a], cfgs[i].faces[a] + cfgs[i].n[a] + 1);
                b->cfgs[i].faces[a] = own.data();
            }
        }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < b->D; ++a)
            if (cfgs[i].mesh[a] != DUGKS_UNIFORM) b->uniform = false;
    const int rc = b->dtype == DUGKS_F64 ? build_tables<double>(b, offsets, (hipStream_t)stream)
                                         : build_tables<float>(b, offsets, (hipStream_t)stream);
    if (rc != DUGKS_OK) {
        g_batch_err = b->err;
        dugks_batch_destroy(b);
        return rc;
    }
    *out = b;
    return DUGKS_OK;
}

template <class LAT, typename T>
static int batch_init_t(dugks_batch* b, void* f, hipStream_t st)
{
    hipLaunchKernelGGL((k_batch_init<LAT, T>), dim3((unsigned)((b->ncells + 255) / 256)), dim3(256), 0, st,
                       (const Inst<T>*)b->insts_dev, (const long long*)b->cstart_dev, b->n, 0.0, (T*)f);
    hipLaunchKernelGGL(k_batch_clock, dim3(1), dim3(1), 0, st, b->step_dev, 0LL, 1);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DUGKS_OK : bfail(b, DUGKS_EHIP, hipGetErrorString(e));
}

extern "C" int dugks_batch_init(dugks_batch* b, void* f_out, void* stream)
{
    if (!b) return bfail(nullptr, DUGKS_EINVAL, "null batch");
    if (!f_out) return bfail(b, DUGKS_EINVAL, "null state buffer");
    const hipStream_t st = (hipStream_t)stream;
    if (b->lattice == DUGKS_D2Q9)
        return b->dtype == DUGKS_F64 ? batch_init_t<D2Q9, double>(b, f_out, st) : batch_init_t<D2Q9, float>(b, f_out, st);
    return b->dtype == DUGKS_F64 ? batch_init_t<D3Q19, double>(b, f_out, st) : batch_init_t<D3Q19, float>(b, f_out, st);
}

static int batch_launch_any(dugks_batch* b, const void* fin, void* fout, const void* forces, int step, hipStream_t st)
{
    // without any field the field-free kernels run (as for single instances)
    const void* fz = b->any_field ? forces : nullptr;
    const hipError_t e = batch_step_launch(b->lattice, b->dtype, b->uniform, b->tile, b->insts_dev, b->bstart_dev,
                                           b->geom_dev, b->n, b->nblocks, fin, fz, fout, b->step_dev, step, st);
    return e == hipSuccess ? DUGKS_OK : bfail(b, DUGKS_EHIP, hipGetErrorString(e));
}

static int launch_run(dugks_batch* b, const void* f_in, void* f_out, const void* forces, int nsteps, hipStream_t st)
{
    const void* cur = f_in;
    void* nxt = f_out;
    for (int k = 0; k < nsteps; ++k) {
        const int rc = batch_launch_any(b, cur, nxt, forces, k, st);
        if (rc != DUGKS_OK) return rc;
        void* tmp = const_cast<void*>(cur);
        cur = nxt;
        nxt = tmp;
    }
    hipLaunchKernelGGL(k_batch_clock, dim3(1), dim3(1), 0, st, b->step_dev, (long long)nsteps, 0);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DUGKS_OK : bfail(b, DUGKS_EHIP, hipGetErrorString(e));
}

// per-instance force offsets into the instance table (before any launch)
static int apply_force_offsets(dugks_batch* b, const void* forces, const int64_t* force_offsets, hipStream_t st)
{
    bool changed = false;
    const size_t isz = b->dtype == DUGKS_F64 ? sizeof(Inst<double>) : sizeof(Inst<float>);
    for (int i = 0; i < b->n; ++i) {
        long long fo = (forces && force_offsets) ? (long long)force_offsets[i] : -1;
        long long* slot = (long long*)(b->hinst.data() + i * isz +
                                       (b->dtype == DUGKS_F64 ? offsetof(Inst<double>, foff) : offsetof(Inst<float>, foff)));
        if (*slot != fo) { *slot = fo; changed = true; }
    }
    b->any_field = false;
    for (int i = 0; i < b->n; ++i)
        if (forces && force_offsets && force_offsets[i] >= 0) b->any_field = true;
    if (changed) {
        // earlier launches on the caller's stream may still read the table
        // (and a captured graph refers to it): let them finish first
        if (hipStreamSynchronize(st) != hipSuccess) return bfail(b, DUGKS_EHIP, "stream synchronisation");
        drop_graph(b);
        if (hipMemcpy(b->insts_dev, b->hinst.data(), b->hinst.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bfail(b, DUGKS_EHIP, "instance table update");
    }
    return DUGKS_OK;
}

extern "C" int dugks_batch_run(dugks_batch* b, void* f_in, void* f_out, const void* forces,
                               const int64_t* force_offsets, int nsteps, int use_graph, void* stream, int* which_out)
{
    if (!b) return bfail(nullptr, DUGKS_EINVAL, "null batch");
    if (!f_in || !f_out || f_in == f_out) return bfail(b, DUGKS_EINVAL, "need two distinct state buffers");
    if (nsteps < 0) return bfail(b, DUGKS_EINVAL, "negative step count");
    const hipStream_t st = (hipStream_t)stream;
    const int frc = apply_force_offsets(b, forces, force_offsets, st);
    if (frc != DUGKS_OK) return frc;
    if (use_graph) {
        if (!st) return bfail(b, DUGKS_EINVAL, "graph capture needs a non-default stream");
        if (!b->gexec || b->g_in != f_in || b->g_out != f_out || b->g_forces != forces || b->g_steps != nsteps ||
            b->g_stream != st) {
            drop_graph(b);
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return bfail(b, DUGKS_EHIP, "stream capture begin");
            const int rc = launch_run(b, f_in, f_out, forces, nsteps, st);
            const hipError_t ee = hipStreamEndCapture(st, &graph);
            if (rc != DUGKS_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
            if (ee != hipSuccess) return bfail(b, DUGKS_EHIP, "stream capture end");
            const hipError_t ie = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) { b->gexec = nullptr; return bfail(b, DUGKS_EHIP, "graph instantiate"); }
            b->g_in = f_in; b->g_out = f_out; b->g_forces = forces; b->g_steps = nsteps; b->g_stream = st;
        }
        const hipError_t le = hipGraphLaunch(b->gexec, st);
        if (le != hipSuccess) return bfail(b, DUGKS_EHIP, "graph launch");
    } else {
        const int rc = launch_run(b, f_in, f_out, forces, nsteps, st);
        if (rc != DUGKS_OK) return rc;
    }
    if (which_out) *which_out = nsteps & 1;
    return DUGKS_OK;
}

extern "C" int dugks_batch_step(dugks_batch* b, void* f_in, void* f_out, const void* forces,
                                const int64_t* force_offsets, int nsteps, void* stream, int* which_out)
{
    // graph replay needs a non-default stream
    return dugks_batch_run(b, f_in, f_out, forces, force_offsets, nsteps, stream != nullptr ? 1 : 0, stream,
                           which_out);
}

extern "C" int dugks_batch_tune(dugks_batch* b, void* f_a, void* f_b, const void* forces,
                                const int64_t* force_offsets, int nsteps, void* stream, int* tile_out,
                                int* chunk_out)
{
    if (!b) return bfail(nullptr, DUGKS_EINVAL, "null batch");
    if (!f_a || !f_b || f_a == f_b) return bfail(b, DUGKS_EINVAL, "need two distinct scratch buffers");
    if (nsteps < 1) return bfail(b, DUGKS_EINVAL, "need at least one timed step per candidate");
    const hipStream_t st = (hipStream_t)stream;
    const int frc = apply_force_offsets(b, forces, force_offsets, st);
    if (frc != DUGKS_OK) return frc;
    // the clock is restored afterwards: tuning steps do not advance the batch
    long long clock = 0;
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(&clock, b->step_dev, sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess)
        return bfail(b, DUGKS_EHIP, "clock read");
    int maxm = 1;
    for (const auto& c : b->cfgs) maxm = std::max(maxm, c.n[b->D - 1]);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return bfail(b, DUGKS_EHIP, "event create");
    }
    float best = -1.0f;
    int best_tile = 0, best_chunk = 0, rc = DUGKS_OK;
    // 0: a chunk per instance from the chunk model; else one chunk for all
    static const int chunks[] = {0, 4, 8, 16, 32, 64};
    for (int tile = 0; tile < fused_tile_variants(b->lattice) && rc == DUGKS_OK; ++tile) {
        for (int chunk : chunks) {
            if (chunk > 2 * maxm) continue;
            rc = set_geometry(b, tile, chunk);
            if (rc == DUGKS_OK) rc = launch_run(b, f_a, f_b, forces, 1, st);  // warm-up
            if (rc == DUGKS_OK && hipEventRecord(e0, st) != hipSuccess) rc = bfail(b, DUGKS_EHIP, "event record");
            if (rc == DUGKS_OK) rc = launch_run(b, f_a, f_b, forces, nsteps, st);
            if (rc == DUGKS_OK && hipEventRecord(e1, st) != hipSuccess) rc = bfail(b, DUGKS_EHIP, "event record");
            float ms = 0.0f;
            if (rc == DUGKS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = bfail(b, DUGKS_EHIP, "event timing");
            if (rc != DUGKS_OK) break;
            if (best < 0.0f || ms < best) { best = ms; best_tile = tile; best_chunk = chunk; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DUGKS_OK) return rc;
    rc = set_geometry(b, best_tile, best_chunk);
    if (rc != DUGKS_OK) return rc;
    hipLaunchKernelGGL(k_batch_clock, dim3(1), dim3(1), 0, st, b->step_dev, clock, 1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, DUGKS_EHIP, hipGetErrorString(e));
    if (tile_out) *tile_out = best_tile;
    if (chunk_out) *chunk_out = best_chunk;
    return DUGKS_OK;
}

extern "C" void dugks_batch_destroy(dugks_batch* b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    drop_graph(b);
    if (b->insts_dev) (void)hipFree(b->insts_dev);
    if (b->met_dev) (void)hipFree(b->met_dev);
    if (b->bstart_dev) (void)hipFree(b->bstart_dev);
    if (b->cstart_dev) (void)hipFree(b->cstart_dev);
    if (b->geom_dev) (void)hipFree(b->geom_dev);
    if (b->step_dev) (void)hipFree(b->step_dev);
    delete b;
}

extern "C" const char* dugks_batch_last_error(const dugks_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }
