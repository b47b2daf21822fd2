// C-ABI entry points of libdhtrace (declared in include/dhtrace.h).
//
// Every entry point validates its arguments, converts between the canonical
// interface layout and the internal even/odd layout, and reports failures as
// negative return codes with a thread-local message; no C++ exception leaves
// this file.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>

#include "solver.h"

namespace dht {

static thread_local std::string g_err;

// Scratch of dht_apply_noalloc: the two internal even/odd fields of one chunk
// of right-hand sides, in a device-resident array that exists for the life of
// the process (no allocation at call time).  Every GPU the library runs on
// holds its own copy at its own address; host code uses only the per-device
// address that hipGetSymbolAddress returned, never the array's name.
static __device__ __align__(256) unsigned char scratch[DHT_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;   // per device; null until set up

// once per device, with that device current (called by dht_create)
static int scratch_setup(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (g_scratch_ptr[device]) return DHT_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(DHT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return DHT_OK;
}

static void* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

int set_error(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int ws_get(dht_ctx* c, int slot, size_t bytes, void** out) {
    if (slot < 0 || slot >= WS_NSLOTS) return set_error(DHT_ERR_INVALID_ARG, "bad workspace slot");
    // caller-owned workspace: the planned slots live at fixed offsets of the
    // caller's buffer; inside a planned call nothing else may be allocated
    if (c->arena && slot != WS_HOSTPIN) {
        if (c->plan[slot] > 0 && bytes <= c->plan[slot]) {
            *out = c->arena + c->plan_off[slot];
            return DHT_OK;
        }
        if (c->planned_call > 0)
            return set_error(DHT_ERR_OOM, "caller workspace: slot " + std::to_string(slot) + " needs " +
                                              std::to_string(bytes) + " bytes, the plan holds " +
                                              std::to_string(c->plan[slot]) +
                                              " (size the workspace for this batch and these parameters)");
    }
    Buf& b = c->ws[slot];
    if (b.bytes < bytes) {
        if (b.p) {
            DHT_HIP(hipStreamSynchronize(c->stream));
            if (slot == WS_HOSTPIN) (void)hipHostFree(b.p);
            else (void)hipFree(b.p);
            b.p = nullptr;
            b.bytes = 0;
        }
        size_t nb = std::max<size_t>(bytes, 256);
        hipError_t e = slot == WS_HOSTPIN ? hipHostMalloc(&b.p, nb, hipHostMallocDefault) : hipMalloc(&b.p, nb);
        if (e != hipSuccess) {
            b.p = nullptr;
            (void)hipGetLastError();
            return set_error(DHT_ERR_OOM, "workspace allocation of " + std::to_string(nb) + " bytes failed");
        }
        b.bytes = nb;
    }
    *out = b.p;
    return DHT_OK;
}

static int prof_event(dht_ctx* c, int* idx) {
    if (c->prof_free.empty()) {
        hipEvent_t e;
        DHT_HIP(hipEventCreate(&e));
        c->prof_events.push_back(e);
        c->prof_free.push_back((int)c->prof_events.size() - 1);
    }
    *idx = c->prof_free.back();
    c->prof_free.pop_back();
    return DHT_OK;
}

int prof_begin(dht_ctx* c, int* token) {
    *token = -1;
    if (!c->prof) return DHT_OK;
    DHT_TRY(prof_event(c, token));
    DHT_HIP(hipEventRecord(c->prof_events[*token], c->stream));
    return DHT_OK;
}

int prof_end(dht_ctx* c, int token, int cls, double bytes) {
    if (token < 0 || !c->prof) return DHT_OK;
    int e1;
    DHT_TRY(prof_event(c, &e1));
    DHT_HIP(hipEventRecord(c->prof_events[e1], c->stream));
    ProfPending p;
    p.cls = cls;
    p.ev0 = token;
    p.ev1 = e1;
    p.bytes = bytes;
    c->prof_pending.push_back(p);
    return DHT_OK;
}

// Accumulates every timed launch that has completed; launches still running
// (on the side stream) stay pending with their events held.
int prof_harvest(dht_ctx* c) {
    if (c->prof_pending.empty()) return DHT_OK;
    DHT_HIP(hipStreamSynchronize(c->stream));
    size_t keep = 0;
    for (size_t i = 0; i < c->prof_pending.size(); i++) {
        const ProfPending p = c->prof_pending[i];
        hipError_t q = hipEventQuery(c->prof_events[p.ev1]);
        if (q == hipErrorNotReady) {
            c->prof_pending[keep++] = p;
            continue;
        }
        DHT_HIP(q);
        float ms = 0.f;
        DHT_HIP(hipEventElapsedTime(&ms, c->prof_events[p.ev0], c->prof_events[p.ev1]));
        ProfStat& s = c->prof_stat[p.cls];
        s.count++;
        s.ms += ms;
        s.bytes += p.bytes;
        c->prof_free.push_back(p.ev0);
        c->prof_free.push_back(p.ev1);
    }
    c->prof_pending.resize(keep);
    return DHT_OK;
}

static bool valid_prec(int p) { return p == DHT_FP64 || p == DHT_FP32 || p == DHT_BF16; }

// a call whose workspace the caller's plan covers (see ws_get)
struct PlannedCall {
    dht_ctx* c;
    explicit PlannedCall(dht_ctx* cc) : c(cc) { c->planned_call++; }
    ~PlannedCall() { c->planned_call--; }
};

// workspace of dht_trace_batch for a padded batch bp (see its ws_get calls)
static void ws_plan_trace(const dht_ctx* c, const dht_solver_params* prm, int bp, size_t* plan) {
    const size_t fb = full_elems(c, bp) * 16;
    plan_max(plan, WS_Z, fb);
    plan_max(plan, WS_PACK_OUT, fb);
    const int k = c->defl_ready ? c->k : 0;
    const bool mfma = k > 0 && c->wprec == DHT_BF16 && bp <= 64;
    plan_max(plan, WS_COEF, sizeof(Cx<double>) * (2 * (size_t)k * bp + bp) + 64);
    if (mfma) {
        plan_max(plan, WS_ZCODE, full_elems(c, bp));
        ws_plan_project_codes(c, bp, plan);
        if (c->proj_window > 0) {   // a window of more probes than the batch
            const int wpad = pad_rhs(c->proj_window);
            plan_max(plan, WS_PW_CODE, full_elems(c, wpad));
            plan_max(plan, WS_PW_COEF, sizeof(Cx<double>) * 2 * (size_t)k * wpad);
            ws_plan_project_codes(c, wpad, plan);
        }
    } else if (k > 0) {
        ws_plan_project_field(c, bp, plan);
    }
    ws_plan_dots(c, bp, plan);   // q = z^H x of the methods that do not fuse it
    ws_plan_solve(c, prm, bp, plan);
}

// device coefficients [k][bp] -> host [k][n] (first n columns), after a sync
static int copy_coefs(dht_ctx* c, const Cx<double>* d1, const Cx<double>* d2, int bp, int n, double* c1h, double* c2h) {
    const size_t kb = (size_t)c->k * bp;
    std::vector<Cx<double>> h(2 * kb);
    DHT_HIP(hipMemcpyAsync(h.data(), d1, sizeof(Cx<double>) * kb, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipMemcpyAsync(h.data() + kb, d2, sizeof(Cx<double>) * kb, hipMemcpyDeviceToHost, c->stream));
    DHT_HIP(hipStreamSynchronize(c->stream));
    DHT_TRY(prof_harvest(c));
    for (int i = 0; i < c->k; i++)
        for (int r = 0; r < n; r++) {
            c1h[2 * ((size_t)i * n + r)] = h[(size_t)i * bp + r].re;
            c1h[2 * ((size_t)i * n + r) + 1] = h[(size_t)i * bp + r].im;
            c2h[2 * ((size_t)i * n + r)] = h[kb + (size_t)i * bp + r].re;
            c2h[2 * ((size_t)i * n + r) + 1] = h[kb + (size_t)i * bp + r].im;
        }
    return DHT_OK;
}

static int check_ctx(dht_ctx* c) {
    if (!c) return set_error(DHT_ERR_INVALID_ARG, "null context");
    DHT_HIP(hipSetDevice(c->device));
    return DHT_OK;
}

static int record(dht_ctx* c, int i) {
    DHT_HIP(hipEventRecord(c->ev[i], c->stream));
    return DHT_OK;
}

static double elapsed(dht_ctx* c, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) return 0.0;
    return ms;
}

int side_stream(dht_ctx* c) {
    if (c->side) return DHT_OK;
    DHT_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    for (int i = 0; i < 4; i++) {
        if (hipEventCreate(&c->side_ev[i]) != hipSuccess) {
            for (int j = 0; j < i; j++) (void)hipEventDestroy(c->side_ev[j]);
            (void)hipStreamDestroy(c->side);
            c->side = nullptr;
            return set_error(DHT_ERR_HIP, "hipEventCreate failed");
        }
    }
    return DHT_OK;
}

}  // namespace dht

using namespace dht;

extern "C" {

const char* dht_last_error(void) { return g_err.c_str(); }

const char* dht_version(void) { return "dhtrace 0.1 gfx950"; }

int dht_create(const dht_lattice* lat, int device, void* hip_stream, dht_ctx** out) {
    if (!lat || !out) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    for (int i = 0; i < 4; i++)
        if (lat->L[i] < 2 || (lat->L[i] & 1)) return set_error(DHT_ERR_INVALID_ARG, "every lattice extent must be even and >= 2");
    if (!isfinite(lat->mass) || 4.0 + lat->mass == 0.0) return set_error(DHT_ERR_INVALID_ARG, "mass must be finite and != -4");
    int ndev = 0;
    DHT_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return set_error(DHT_ERR_INVALID_ARG, "no such device");
    DHT_HIP(hipSetDevice(device));
    DHT_TRY(scratch_setup(device));
    dht_ctx* c = new (std::nothrow) dht_ctx;
    if (!c) return set_error(DHT_ERR_OOM, "out of host memory");
    for (int i = 0; i < 4; i++) c->g.L[i] = lat->L[i];
    c->g.Lxh = lat->L[0] / 2;
    c->g.V = (int64_t)lat->L[0] * lat->L[1] * lat->L[2] * lat->L[3];
    c->g.Vh = c->g.V / 2;
    c->g.antiperiodic = lat->t_antiperiodic ? 1 : 0;
    c->mass = lat->mass;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->ws.resize(WS_NSLOTS);
    for (int i = 0; i < 6; i++) {
        if (hipEventCreate(&c->ev[i]) != hipSuccess) {
            delete c;
            return set_error(DHT_ERR_HIP, "hipEventCreate failed");
        }
    }
    c->events = true;
    *out = c;
    return DHT_OK;
}

int dht_destroy(dht_ctx* c) {
    if (!c) return DHT_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < 3; i++)
        if (c->U[i]) (void)hipFree(c->U[i]);
    if (c->W) (void)hipFree(c->W);
    if (c->nn.mem) (void)hipFree(c->nn.mem);
    for (int i = 0; i < (int)c->ws.size(); i++) {
        if (!c->ws[i].p) continue;
        if (i == WS_HOSTPIN) (void)hipHostFree(c->ws[i].p);
        else (void)hipFree(c->ws[i].p);
    }
    if (c->events)
        for (int i = 0; i < 6; i++) (void)hipEventDestroy(c->ev[i]);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        for (int i = 0; i < 4; i++) (void)hipEventDestroy(c->side_ev[i]);
        (void)hipStreamDestroy(c->side);
    }
    for (hipEvent_t e : c->prof_events) (void)hipEventDestroy(e);
    delete c;
    return DHT_OK;
}

int dht_workspace_trim(dht_ctx* c) {
    DHT_TRY(check_ctx(c));
    DHT_HIP(hipStreamSynchronize(c->stream));
    if (c->side) DHT_HIP(hipStreamSynchronize(c->side));
    for (int i = 0; i < (int)c->ws.size(); i++) {
        Buf& b = c->ws[i];
        if (!b.p) continue;
        if (i == WS_HOSTPIN) (void)hipHostFree(b.p);
        else (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    c->pw_valid = false;   // the projection window's codes and coefficients lived there
    return DHT_OK;
}

int dht_workspace_size(dht_ctx* c, int max_nrhs, const dht_solver_params* prm, size_t* bytes) {
    DHT_TRY(check_ctx(c));
    if (!prm || !bytes || max_nrhs <= 0 || max_nrhs > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (c->W && !c->defl_ready) return set_error(DHT_ERR_STATE, "deflation basis set but not finalized");
    std::vector<size_t> plan(WS_NSLOTS, 0);
    for (int bp = 1; bp <= pad_rhs(max_nrhs); bp <<= 1) {   // every padded batch up to max_nrhs
        ws_plan_trace(c, prm, bp, plan.data());
        const size_t fb = full_elems(c, bp) * 16;   // dht_solve's packed fields
        plan_max(plan.data(), WS_PACK_IN, fb);
        plan_max(plan.data(), WS_PACK_OUT, fb);
    }
    plan[WS_HOSTPIN] = 0;   // a small pinned host buffer, not device workspace
    size_t total = 0;
    for (int s = 0; s < WS_NSLOTS; s++) total += (plan[s] + 255) / 256 * 256;
    c->plan_next = plan;
    c->plan_next_total = total;
    *bytes = total;
    return DHT_OK;
}

int dht_set_workspace(dht_ctx* c, void* ptr, size_t bytes) {
    DHT_TRY(check_ctx(c));
    DHT_HIP(hipStreamSynchronize(c->stream));
    if (c->side) DHT_HIP(hipStreamSynchronize(c->side));
    c->pw_valid = false;   // the projection window's codes and coefficients move
    if (!ptr) {            // back to library-owned workspace
        c->arena = nullptr;
        c->arena_bytes = 0;
        c->plan.clear();
        c->plan_off.clear();
        return DHT_OK;
    }
    if (c->plan_next.empty()) return set_error(DHT_ERR_STATE, "call dht_workspace_size first");
    if (((uintptr_t)ptr & 255) != 0) return set_error(DHT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < c->plan_next_total)
        return set_error(DHT_ERR_INVALID_ARG, "workspace of " + std::to_string(bytes) + " bytes is smaller than the " +
                                                  std::to_string(c->plan_next_total) + " bytes planned");
    c->plan = c->plan_next;
    c->plan_off.assign(WS_NSLOTS, 0);
    size_t off = 0;
    for (int s = 0; s < WS_NSLOTS; s++) {
        c->plan_off[s] = off;
        off += (c->plan[s] + 255) / 256 * 256;
    }
    c->arena = (char*)ptr;
    c->arena_bytes = bytes;
    for (int i = 0; i < (int)c->ws.size(); i++) {   // library-owned device slots are no longer needed
        Buf& b = c->ws[i];
        if (!b.p || i == WS_HOSTPIN) continue;
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    return DHT_OK;
}

int dht_set_gauge(dht_ctx* c, const double* U_dev) {
    DHT_TRY(check_ctx(c));
    if (!U_dev) return set_error(DHT_ERR_INVALID_ARG, "null links");
    for (int p = 0; p < 3; p++) {
        if (!c->U[p]) {
            // [4][2][Vh] link matrices of link_vecs(p) 16-byte vectors each
            size_t bytes = (size_t)4 * c->g.V * link_vecs(p) * 16;
            if (hipMalloc(&c->U[p], bytes) != hipSuccess) {
                c->U[p] = nullptr;
                (void)hipGetLastError();
                return set_error(DHT_ERR_OOM, "cannot allocate links");
            }
        }
    }
    DHT_TRY(pack_gauge(c, U_dev));
    DHT_HIP(hipStreamSynchronize(c->stream));
    c->have_gauge = true;
    return DHT_OK;
}

int dht_apply(dht_ctx* c, int op, int prec, const double* X, double* Y, int nrhs) {
    DHT_TRY(check_ctx(c));
    if (!X || !Y || nrhs <= 0 || !valid_prec(prec) || op < DHT_OP_D || op > DHT_OP_Q)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (op != DHT_OP_G5 && !c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    const int64_t N = 12 * c->g.V;
    for (int r0 = 0; r0 < nrhs; r0 += 64) {   // chunks of at most 64 right-hand sides
        const int n = std::min(64, nrhs - r0), bp = pad_rhs(n);
        size_t bytes = full_elems(c, bp) * elem_bytes(prec);
        void *fi, *fo;
        DHT_TRY(ws_get(c, WS_PACK_IN, bytes, &fi));
        DHT_TRY(ws_get(c, WS_PACK_OUT, bytes, &fo));
        DHT_TRY(pack_spinor(c, X + 2 * N * r0, fi, prec, n, bp));
        DHT_TRY(apply_full(c, op, prec, fi, fo, bp));
        DHT_TRY(unpack_spinor(c, fo, prec, Y + 2 * N * r0, n, bp));
    }
    DHT_HIP(hipStreamSynchronize(c->stream));
    DHT_TRY(prof_harvest(c));
    return DHT_OK;
}

int dht_apply_noalloc(dht_ctx* c, int op, int prec, const double* X, double* Y, int nrhs) {
    DHT_TRY(check_ctx(c));
    if (!X || !Y || nrhs <= 0 || !valid_prec(prec) || op < DHT_OP_D || op > DHT_OP_Q)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (op != DHT_OP_G5 && !c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    const int bp0 = pad_rhs(std::min(64, nrhs));
    const size_t need = 2 * full_elems(c, bp0) * elem_bytes(prec);
    if (need > (size_t)DHT_NOALLOC_SCRATCH_BYTES)
        return set_error(DHT_ERR_INVALID_ARG, "dht_apply_noalloc: " + std::to_string(need) +
                                                  " bytes of scratch needed, the limit is " +
                                                  std::to_string((size_t)DHT_NOALLOC_SCRATCH_BYTES));
    char* base = (char*)scratch_ptr(c->device);
    if (!base) return set_error(DHT_ERR_STATE, "no-alloc scratch not set up on this device");
    // the per-launch events of the instrumentation would come from a pool
    // that grows on demand: these launches are not profiled
    const bool prof = c->prof;
    c->prof = false;
    int rc = DHT_OK;
    const int64_t N = 12 * c->g.V;
    for (int r0 = 0; r0 < nrhs && rc == DHT_OK; r0 += 64) {   // chunks of at most 64, in stream order
        const int n = std::min(64, nrhs - r0), bp = pad_rhs(n);
        void* fi = base;
        void* fo = base + full_elems(c, bp) * elem_bytes(prec);
        rc = pack_spinor(c, X + 2 * N * r0, fi, prec, n, bp);
        if (rc == DHT_OK) rc = apply_full(c, op, prec, fi, fo, bp);
        if (rc == DHT_OK) rc = unpack_spinor(c, fo, prec, Y + 2 * N * r0, n, bp);
    }
    c->prof = prof;
    return rc;
}

int dht_make_probes(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int nrhs, double* Z) {
    DHT_TRY(check_ctx(c));
    if (!spec || !Z || nrhs <= 0 || nrhs > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    const int bp = pad_rhs(nrhs);
    void* f;
    DHT_TRY(ws_get(c, WS_Z, full_elems(c, bp) * 16, &f));
    DHT_TRY(probes_gen(c, spec, first, nrhs, bp, f, DHT_FP64, nullptr, nullptr));
    DHT_TRY(unpack_spinor(c, f, DHT_FP64, Z, nrhs, bp));
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int dht_probe_indices(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int nrhs, uint8_t* k_dev,
                      int8_t* sign_dev) {
    DHT_TRY(check_ctx(c));
    if (!spec || !k_dev || !sign_dev || nrhs <= 0 || nrhs > DHT_MAX_BATCH)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    DHT_TRY(probes_gen(c, spec, first, nrhs, pad_rhs(nrhs), nullptr, DHT_FP64, k_dev, sign_dev));
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int dht_solve(dht_ctx* c, const dht_solver_params* prm, const double* Z, double* X, int nrhs, dht_solve_stats* stats) {
    DHT_TRY(check_ctx(c));
    PlannedCall pc(c);
    if (!prm || !Z || !X || nrhs <= 0 || nrhs > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    const int bp = pad_rhs(nrhs);
    size_t bytes = full_elems(c, bp) * 16;
    void *fz, *fx;
    DHT_TRY(ws_get(c, WS_PACK_IN, bytes, &fz));
    DHT_TRY(ws_get(c, WS_PACK_OUT, bytes, &fx));
    DHT_TRY(pack_spinor(c, Z, fz, DHT_FP64, nrhs, bp));
    DHT_TRY(record(c, 0));
    std::vector<dht_solve_stats> st(bp);
    int rc = solve_fields(c, prm, fz, fx, bp, st.data());
    if (rc != DHT_OK && rc != DHT_ERR_NOT_CONVERGED) return rc;
    std::string msg = g_err;
    DHT_TRY(record(c, 1));
    DHT_TRY(unpack_spinor(c, fx, DHT_FP64, X, nrhs, bp));
    DHT_HIP(hipStreamSynchronize(c->stream));
    c->timings[1] = elapsed(c, 0, 1);
    DHT_TRY(prof_harvest(c));
    if (stats)
        for (int i = 0; i < nrhs; i++) stats[i] = st[i];
    if (rc != DHT_OK) g_err = msg;
    return rc;
}

int dht_deflation_begin(dht_ctx* c, int k, int prec) {
    DHT_TRY(check_ctx(c));
    return deflation_begin(c, k, prec);
}

int dht_deflation_set(dht_ctx* c, int first, int count, const double* W_dev) {
    DHT_TRY(check_ctx(c));
    if (!W_dev && count > 0) return set_error(DHT_ERR_INVALID_ARG, "null basis");
    DHT_TRY(deflation_set(c, first, count, W_dev));
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int dht_deflation_eigensolve(dht_ctx* c, const dht_eig_params* prm, double* lambda_host, double* resid_host,
                             dht_eig_stats* stats) {
    DHT_TRY(check_ctx(c));
    if (!prm) return set_error(DHT_ERR_INVALID_ARG, "null parameters");
    int rc = eigensolve(c, prm, lambda_host, resid_host, stats);
    DHT_TRY(prof_harvest(c));
    return rc;
}

int dht_deflation_lobpcg(dht_ctx* c, const dht_lobpcg_params* prm, double* sigma_host, double* resid_host,
                         dht_lobpcg_stats* stats) {
    DHT_TRY(check_ctx(c));
    if (!prm) return set_error(DHT_ERR_INVALID_ARG, "null parameters");
    const int rc = lobpcg(c, prm, sigma_host, resid_host, stats);
    const std::string msg = g_err;
    const int hr = prof_harvest(c);
    if (rc != DHT_OK) return set_error(rc, msg);
    return hr;
}

int dht_deflation_get(dht_ctx* c, int first, int count, double* W_dev) {
    DHT_TRY(check_ctx(c));
    if (!c->W || c->k <= 0) return set_error(DHT_ERR_STATE, "no deflation basis");
    if (first < 0 || count < 0 || first + count > c->k || (count > 0 && !W_dev))
        return set_error(DHT_ERR_INVALID_ARG, "columns out of range");
    for (int j = 0; j < count; j += 64) {
        const int n = std::min(64, count - j);
        const int bp = pad_rhs(n);
        void* buf;
        DHT_TRY(ws_get(c, WS_DEFL_GET, full_elems(c, bp) * sizeof(Cx<double>), &buf));
        DHT_TRY(gather_columns(c, first + j, n, bp, buf));
        DHT_TRY(unpack_spinor(c, buf, DHT_FP64, W_dev + (size_t)2 * 12 * c->g.V * j, n, bp));
    }
    DHT_HIP(hipStreamSynchronize(c->stream));
    return DHT_OK;
}

int dht_deflation_finalize(dht_ctx* c, double* TD) {
    DHT_TRY(check_ctx(c));
    DHT_TRY(deflation_finalize(c, false));
    DHT_TRY(prof_harvest(c));
    if (TD) {
        TD[0] = c->TD[0];
        TD[1] = c->TD[1];
    }
    return DHT_OK;
}

int dht_deflation_finalize_diag(dht_ctx* c, double* TD) {
    DHT_TRY(check_ctx(c));
    DHT_TRY(deflation_finalize(c, true));
    DHT_TRY(prof_harvest(c));
    if (TD) {
        TD[0] = c->TD[0];
        TD[1] = c->TD[1];
    }
    return DHT_OK;
}

int dht_profile_enable(dht_ctx* c, int on) {
    DHT_TRY(check_ctx(c));
    DHT_TRY(prof_harvest(c));
    c->prof = on != 0;
    return DHT_OK;
}

int dht_profile_reset(dht_ctx* c) {
    DHT_TRY(check_ctx(c));
    if (c->side) DHT_HIP(hipStreamSynchronize(c->side));
    DHT_TRY(prof_harvest(c));
    for (int i = 0; i < PROF_NCLASS; i++) c->prof_stat[i] = ProfStat();
    return DHT_OK;
}

int dht_profile_get(dht_ctx* c, int cls, int64_t* count, double* total_ms, double* total_bytes) {
    DHT_TRY(check_ctx(c));
    if (cls < 0 || cls >= PROF_NCLASS || !count || !total_ms || !total_bytes)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (c->side) DHT_HIP(hipStreamSynchronize(c->side));
    DHT_TRY(prof_harvest(c));
    *count = c->prof_stat[cls].count;
    *total_ms = c->prof_stat[cls].ms;
    *total_bytes = c->prof_stat[cls].bytes;
    return DHT_OK;
}

int dht_deflation_get_M(dht_ctx* c, double* M) {
    DHT_TRY(check_ctx(c));
    if (!c->defl_ready) return set_error(DHT_ERR_STATE, "deflation not finalized");
    if (!M) return set_error(DHT_ERR_INVALID_ARG, "null output");
    memcpy(M, c->M.data(), sizeof(double) * c->M.size());
    return DHT_OK;
}

int dht_deflation_clear(dht_ctx* c) {
    DHT_TRY(check_ctx(c));
    DHT_HIP(hipStreamSynchronize(c->stream));
    if (c->W) DHT_HIP(hipFree(c->W));
    c->W = nullptr;
    c->k = 0;
    c->defl_ready = false; c->defl_gen++;
    c->TD[0] = c->TD[1] = 0;
    c->M.clear();
    return DHT_OK;
}

int dht_project(dht_ctx* c, const double* Z, int nrhs, double* c1h, double* c2h) {
    DHT_TRY(check_ctx(c));
    if (!Z || !c1h || !c2h || nrhs <= 0 || nrhs > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (!c->W) return set_error(DHT_ERR_STATE, "no deflation basis");
    const int bp = pad_rhs(nrhs);
    void *fz, *cc;
    DHT_TRY(ws_get(c, WS_PACK_IN, full_elems(c, bp) * 16, &fz));
    DHT_TRY(ws_get(c, WS_SCAL2, sizeof(Cx<double>) * 2 * c->k * bp, &cc));
    DHT_TRY(pack_spinor(c, Z, fz, DHT_FP64, nrhs, bp));
    Cx<double>* d1 = (Cx<double>*)cc;
    Cx<double>* d2 = d1 + (size_t)c->k * bp;
    DHT_TRY(project_field(c, fz, DHT_FP64, bp, d1, d2));
    return copy_coefs(c, d1, d2, bp, nrhs, c1h, c2h);
}

int dht_project_probes(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int nrhs, double* c1h, double* c2h) {
    DHT_TRY(check_ctx(c));
    if (!spec || !c1h || !c2h || nrhs <= 0 || nrhs > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (!c->W) return set_error(DHT_ERR_STATE, "no deflation basis");
    const int bp = pad_rhs(nrhs);
    const bool mfma = c->wprec == DHT_BF16 && bp <= 64;
    void *cc, *buf;
    DHT_TRY(ws_get(c, WS_SCAL2, sizeof(Cx<double>) * 2 * c->k * bp, &cc));
    Cx<double>* d1 = (Cx<double>*)cc;
    Cx<double>* d2 = d1 + (size_t)c->k * bp;
    if (mfma) {
        DHT_TRY(ws_get(c, WS_ZCODE, full_elems(c, bp), &buf));
        DHT_TRY(probes_gen(c, spec, first, nrhs, bp, nullptr, DHT_FP64, nullptr, nullptr, (uint8_t*)buf));
        DHT_TRY(project_codes(c, (const uint8_t*)buf, bp, d1, d2));
    } else {
        DHT_TRY(ws_get(c, WS_Z, full_elems(c, bp) * 16, &buf));
        DHT_TRY(probes_gen(c, spec, first, nrhs, bp, buf, DHT_FP64, nullptr, nullptr));
        DHT_TRY(project_field(c, buf, DHT_FP64, bp, d1, d2));
    }
    return copy_coefs(c, d1, d2, bp, nrhs, c1h, c2h);
}

int dht_set_projection_window(dht_ctx* c, int nprobes) {
    DHT_TRY(check_ctx(c));
    if (nprobes < 0 || nprobes > 64) return set_error(DHT_ERR_INVALID_ARG, "projection window must be 0..64 probes");
    if (c->side) DHT_HIP(hipStreamSynchronize(c->side));
    c->proj_window = nprobes;
    c->pw_valid = false;
    return DHT_OK;
}

int dht_trace_batch(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int nrhs, const dht_solver_params* prm,
                    dht_record* records, double* coef_host) {
    DHT_TRY(check_ctx(c));
    PlannedCall pc(c);
    if (!spec || !prm || nrhs <= 0 || nrhs > DHT_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    if (c->W && !c->defl_ready) return set_error(DHT_ERR_STATE, "deflation basis set but not finalized");
    const int bp = pad_rhs(nrhs);
    const size_t fb = full_elems(c, bp) * 16;
    void *fz, *fx, *cc, *zc = nullptr;
    DHT_TRY(ws_get(c, WS_Z, fb, &fz));
    DHT_TRY(ws_get(c, WS_PACK_OUT, fb, &fx));
    const int k = c->defl_ready ? c->k : 0;
    const bool mfma = k > 0 && c->wprec == DHT_BF16 && bp <= 64;
    // With a projection window the basis pass covers the probes of several
    // batches at once (one read of W for up to 64 probes); later batches of
    // the window take their coefficients from that pass.
    const int win = mfma && c->proj_window > nrhs ? c->proj_window : 0;
    const bool hit = win && c->pw_valid && c->pw_gen == c->defl_gen && c->pw_spec.seed == spec->seed &&
                     c->pw_spec.run == spec->run && (c->pw_spec.hp != 0) == (spec->hp != 0) && first >= c->pw_first &&
                     first + nrhs <= c->pw_first + c->pw_count;
    const bool launch = k > 0 && !hit;
    const int wpad = win ? pad_rhs(win) : bp;
    void* pwc = nullptr;
    if (mfma) DHT_TRY(ws_get(c, win ? WS_PW_CODE : WS_ZCODE, full_elems(c, wpad), &zc));
    if (win) DHT_TRY(ws_get(c, WS_PW_COEF, sizeof(Cx<double>) * 2 * (size_t)k * wpad, &pwc));
    DHT_TRY(ws_get(c, WS_COEF, sizeof(Cx<double>) * (2 * (size_t)k * bp + bp) + 64, &cc));
    Cx<double>* d1 = win ? (Cx<double>*)pwc : (Cx<double>*)cc;
    Cx<double>* d2 = d1 + (size_t)k * wpad;
    Cx<double>* dq = (Cx<double>*)cc + 2 * (size_t)k * bp;

    // the BiCGStab paths sum q = z^H x in the epilogues of their final residual
    const bool fused_q = prm->method == DHT_SOLVER_DC_BICGSTAB || prm->method == DHT_SOLVER_BICGSTAB_FP64;
    // probe values are exact in BF16: the solve reads them from a BF16 field
    // (the FP64 hops widen them exactly) unless a generic projection reads z
    const int zprec = fused_q && (k == 0 || mfma) ? DHT_BF16 : DHT_FP64;
    DHT_TRY(record(c, 0));
    DHT_TRY(probes_gen(c, spec, first, nrhs, bp, fz, zprec, nullptr, nullptr, win ? nullptr : (uint8_t*)zc));
    DHT_TRY(record(c, 1));
    // the projection needs only the probes: a batch's own pass runs on the
    // side stream while the main stream solves (both read fz; neither writes
    // it); a window's pass runs on the main stream before the solve (its
    // workgroups hold most of the LDS of every compute unit, so next to the
    // solve it would only delay the solve's kernels)
    if (launch) {
        if (win) c->pw_valid = false;
        DHT_TRY(side_stream(c));
        hipStream_t main_stream = c->stream;
        hipStream_t ps = main_stream;
        if (!win) {
            DHT_HIP(hipEventRecord(c->side_ev[0], c->stream));
            DHT_HIP(hipStreamWaitEvent(c->side, c->side_ev[0], 0));
            ps = c->side;
        }
        c->stream = ps;
        int prc = hipEventRecord(c->side_ev[1], ps) == hipSuccess ? DHT_OK : set_error(DHT_ERR_HIP, "event");
        if (prc == DHT_OK && win)   // the window's probes as 2-bit codes, generated on the side stream
            prc = probes_gen(c, spec, first, win, wpad, nullptr, DHT_FP64, nullptr, nullptr, (uint8_t*)zc);
        if (prc == DHT_OK) {
            if (mfma) prc = project_codes(c, (const uint8_t*)zc, wpad, d1, d2);
            else prc = project_field(c, fz, DHT_FP64, bp, d1, d2);
        }
        if (prc == DHT_OK && hipEventRecord(c->side_ev[2], ps) != hipSuccess) prc = set_error(DHT_ERR_HIP, "event");
        c->stream = main_stream;
        if (prc != DHT_OK) (void)hipStreamSynchronize(ps);
        DHT_TRY(prc);
        if (win) {
            c->pw_valid = true;
            c->pw_first = first;
            c->pw_count = win;
            c->pw_pad = wpad;
            c->pw_spec = *spec;
            c->pw_gen = c->defl_gen;
        }
    }
    std::vector<dht_solve_stats> st(bp);
    // every component of a Z4 / hierarchical probe has modulus 1: ||z||^2 = N
    // exactly for the nrhs probes, 0 for the padding columns
    std::vector<double> zn2(bp, 0.0);
    for (int r = 0; r < nrhs; r++) zn2[r] = (double)(12 * c->g.V);
    std::vector<Cx<double>> zxq(bp);
    int rc = solve_fields(c, prm, fz, fx, bp, st.data(), zn2.data(), fused_q ? zxq.data() : nullptr, zprec);
    if (launch && rc != DHT_OK && rc != DHT_ERR_NOT_CONVERGED) {
        (void)hipStreamSynchronize(c->side);   // the next batch rewrites the probes
        return rc;
    }
    if (rc != DHT_OK && rc != DHT_ERR_NOT_CONVERGED) return rc;
    std::string msg = g_err;
    DHT_TRY(record(c, 2));
    if (launch) DHT_HIP(hipStreamWaitEvent(c->stream, c->side_ev[2], 0));
    DHT_TRY(record(c, 3));
    if (!fused_q) {
        const void* aa[1] = {fz};
        const void* bb[1] = {fx};
        DHT_TRY(dots(c, DHT_FP64, 1, aa, bb, full_elems(c, bp), bp, dq));
    }
    DHT_TRY(record(c, 4));
    std::vector<Cx<double>> hc((size_t)2 * k * bp + bp);
    if (win && k > 0)   // this batch's columns of the window's [2k][wpad] coefficients, next to q
        DHT_HIP(hipMemcpy2DAsync(cc, sizeof(Cx<double>) * bp, d1 + (first - c->pw_first), sizeof(Cx<double>) * wpad,
                                 sizeof(Cx<double>) * nrhs, 2 * (size_t)k, hipMemcpyDeviceToDevice, c->stream));
    DHT_HIP(hipMemcpyAsync(hc.data(), cc, sizeof(Cx<double>) * hc.size(), hipMemcpyDeviceToHost, c->stream));
    DHT_TRY(record(c, 5));
    DHT_HIP(hipStreamSynchronize(c->stream));
    c->timings[0] = elapsed(c, 0, 1);
    c->timings[1] = elapsed(c, 1, 2);
    c->timings[2] = 0.0;   // the projection's own duration (it overlaps the solve)
    if (launch) {
        float pm = 0.f;
        if (hipEventElapsedTime(&pm, c->side_ev[1], c->side_ev[2]) == hipSuccess) c->timings[2] = pm;
    }
    c->timings[3] = elapsed(c, 3, 4);
    c->timings[4] = elapsed(c, 0, 5);
    DHT_TRY(prof_harvest(c));
    std::vector<double> dre(bp, 0.0), dim(bp, 0.0);
    if (k > 0) deflation_corrections(c, hc.data(), hc.data() + (size_t)k * bp, bp, nrhs, dre.data(), dim.data());
    const Cx<double>* q = fused_q ? zxq.data() : hc.data() + (size_t)2 * k * bp;
    // a padding slot that failed cannot fail the batch: only real probes count
    if (rc == DHT_ERR_NOT_CONVERGED) {
        bool any = false;
        for (int r = 0; r < nrhs; r++) any |= st[r].status == DHT_STATUS_NOT_CONVERGED;
        if (!any) rc = DHT_OK;
    }
    for (int r = 0; r < nrhs; r++) {
        double qre = q[r].re, qim = q[r].im;
        double dqre = qre - dre[r], dqim = qim - dim[r];
        // only a solve that met the tolerance is a sample of the estimator: a
        // probe that missed it is reported but left out of the running
        // estimates, so that a batch retried after DHT_ERR_NOT_CONVERGED is
        // counted once
        if (st[r].status != DHT_STATUS_NOT_CONVERGED) {
            c->est_q.add(qre, qim);
            c->est_qd.add(dqre, dqim);
        }
        if (records) {
            records[r].q_re = qre;
            records[r].q_im = qim;
            records[r].qd_re = dqre;
            records[r].qd_im = dqim;
            records[r].s = st[r];
        }
    }
    if (coef_host && k > 0) {
        for (int part = 0; part < 2; part++)
            for (int i = 0; i < k; i++)
                for (int r = 0; r < nrhs; r++) {
                    const Cx<double>& v = hc[(size_t)part * k * bp + (size_t)i * bp + r];
                    size_t o = 2 * ((size_t)part * k * nrhs + (size_t)i * nrhs + r);
                    coef_host[o] = v.re;
                    coef_host[o + 1] = v.im;
                }
    }
    if (rc != DHT_OK) g_err = msg;
    return rc;
}

int dht_estimate_get(dht_ctx* c, dht_estimate* e) {
    if (!c || !e) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    memset(e, 0, sizeof(*e));
    e->n = c->est_q.n;
    e->mean_re = c->est_q.mre;
    e->mean_im = c->est_q.mim;
    e->TD_re = c->TD[0];
    e->TD_im = c->TD[1];
    e->mean_defl_re = c->est_qd.mre + (c->defl_ready ? c->TD[0] : 0.0);
    e->mean_defl_im = c->est_qd.mim + (c->defl_ready ? c->TD[1] : 0.0);
    if (e->n >= 2) {
        double d = (double)(e->n - 1);
        e->var_re = c->est_q.m2re / d;
        e->var_im = c->est_q.m2im / d;
        e->var = e->var_re + e->var_im;
        e->var_defl_re = c->est_qd.m2re / d;
        e->var_defl_im = c->est_qd.m2im / d;
        e->var_defl = e->var_defl_re + e->var_defl_im;
    } else {
        e->var = e->var_re = e->var_im = NAN;
        e->var_defl = e->var_defl_re = e->var_defl_im = NAN;
    }
    return DHT_OK;
}

int dht_estimate_reset(dht_ctx* c) {
    if (!c) return set_error(DHT_ERR_INVALID_ARG, "null context");
    c->est_q = Welford();
    c->est_qd = Welford();
    return DHT_OK;
}

int dht_state_save(dht_ctx* c, const char* path) {
    if (!c || !path) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    FILE* f = fopen(path, "w");
    if (!f) return set_error(DHT_ERR_INVALID_ARG, std::string("cannot write ") + path);
    fprintf(f, "dhtrace-estimate 1\n");
    fprintf(f, "lattice %d %d %d %d %d\n", c->g.L[0], c->g.L[1], c->g.L[2], c->g.L[3], c->g.antiperiodic);
    fprintf(f, "mass %.17g\n", c->mass);
    fprintf(f, "deflation %d %.17g %.17g\n", c->defl_ready ? c->k : 0, c->TD[0], c->TD[1]);
    const Welford* w[2] = {&c->est_q, &c->est_qd};
    for (int i = 0; i < 2; i++)
        fprintf(f, "moments %lld %.17g %.17g %.17g %.17g\n", (long long)w[i]->n, w[i]->mre, w[i]->mim, w[i]->m2re,
                w[i]->m2im);
    const bool ok = fclose(f) == 0;
    return ok ? DHT_OK : set_error(DHT_ERR_INVALID_ARG, std::string("cannot write ") + path);
}

int dht_state_load(dht_ctx* c, const char* path) {
    if (!c || !path) return set_error(DHT_ERR_INVALID_ARG, "null argument");
    FILE* f = fopen(path, "r");
    if (!f) return set_error(DHT_ERR_INVALID_ARG, std::string("cannot read ") + path);
    int ver = 0, L[4], ap, k;
    double mass, td[2];
    long long n[2];
    double m[2][4];
    bool ok = fscanf(f, "dhtrace-estimate %d", &ver) == 1 && ver == 1 &&
              fscanf(f, " lattice %d %d %d %d %d", &L[0], &L[1], &L[2], &L[3], &ap) == 5 &&
              fscanf(f, " mass %lf", &mass) == 1 && fscanf(f, " deflation %d %lf %lf", &k, &td[0], &td[1]) == 3;
    for (int i = 0; ok && i < 2; i++)
        ok = fscanf(f, " moments %lld %lf %lf %lf %lf", &n[i], &m[i][0], &m[i][1], &m[i][2], &m[i][3]) == 5 &&
             n[i] >= 0;
    fclose(f);
    if (!ok) return set_error(DHT_ERR_INVALID_ARG, std::string("not an estimate file: ") + path);
    for (int d = 0; d < 4; d++)
        if (L[d] != c->g.L[d]) return set_error(DHT_ERR_STATE, "estimate file belongs to another lattice");
    if (ap != c->g.antiperiodic || mass != c->mass) return set_error(DHT_ERR_STATE, "estimate file belongs to another operator");
    const int kc = c->defl_ready ? c->k : 0;
    if (k != kc) return set_error(DHT_ERR_STATE, "estimate file belongs to another deflation space");
    if (kc > 0) {
        const double sc = std::max(std::hypot(c->TD[0], c->TD[1]), 1e-300);
        if (std::hypot(td[0] - c->TD[0], td[1] - c->TD[1]) > 1e-12 * sc)
            return set_error(DHT_ERR_STATE, "estimate file belongs to another deflation space (T_D differs)");
    }
    Welford* w[2] = {&c->est_q, &c->est_qd};
    for (int i = 0; i < 2; i++) {
        w[i]->n = n[i];
        w[i]->mre = m[i][0];
        w[i]->mim = m[i][1];
        w[i]->m2re = m[i][2];
        w[i]->m2im = m[i][3];
    }
    return DHT_OK;
}

int dht_solver_counters(dht_ctx* c, int64_t* out, int n) {
    if (!c || !out || n < SC_NCOUNT) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    for (int i = 0; i < SC_NCOUNT; i++) out[i] = c->solver_count[i];
    return DHT_OK;
}

int dht_last_timings(dht_ctx* c, double* ms, int n) {
    if (!c || !ms || n < 5) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    for (int i = 0; i < 5; i++) ms[i] = c->timings[i];
    return DHT_OK;
}

int64_t dht_nn_num_weights(void) { return nn_num_weights(); }

int dht_nn_init(dht_ctx* c, uint64_t seed) {
    DHT_TRY(check_ctx(c));
    // He-normal: std = sqrt(2 / fan_in), fan_in = 81 Cin; SplitMix64 -> Box-Muller
    static const int ch[4] = {24, 48, 48, 24};
    std::vector<float> w((size_t)nn_num_weights());
    uint64_t st = seed;
    auto next = [&]() {
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);   // (0, 1)
    };
    size_t off = 0;
    for (int l = 0; l < 3; l++) {
        // the last layer starts 10x smaller so that the initial output is small
        const double sd = sqrt(2.0 / (81.0 * ch[l])) * (l == 2 ? 0.1 : 1.0);
        const size_t n = (size_t)81 * ch[l] * ch[l + 1];
        for (size_t i = 0; i < n; i++) {
            double u1 = next(), u2 = next();
            w[off + i] = (float)(sd * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
        }
        off += n;
    }
    return nn_set_weights(c, w.data());
}

int dht_nn_set_skip(dht_ctx* c, double sk) {
    DHT_TRY(check_ctx(c));
    if (!isfinite(sk)) return set_error(DHT_ERR_INVALID_ARG, "skip coefficient must be finite");
    c->nn.skip = (float)sk;
    return DHT_OK;
}

int dht_nn_set_weights(dht_ctx* c, const float* w) {
    DHT_TRY(check_ctx(c));
    if (!w) return set_error(DHT_ERR_INVALID_ARG, "null weights");
    return nn_set_weights(c, w);
}

int dht_nn_get_weights(dht_ctx* c, float* w) {
    DHT_TRY(check_ctx(c));
    if (!w) return set_error(DHT_ERR_INVALID_ARG, "null weights");
    return nn_get_weights(c, w, false);
}

int dht_nn_forward(dht_ctx* c, const double* R, double* E, int n) {
    DHT_TRY(check_ctx(c));
    if (!R || !E || n <= 0) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    return nn_forward_canon(c, R, E, n);
}

int dht_nn_grad(dht_ctx* c, const double* R, const double* E, int n, float* grad, double* loss) {
    DHT_TRY(check_ctx(c));
    if (!R || !E || n <= 0 || n > NN_MAX_BATCH) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    DHT_TRY(nn_grad_canon(c, R, E, n, loss));
    if (grad) DHT_TRY(nn_get_weights(c, grad, true));
    return DHT_OK;
}

int dht_nn_train(dht_ctx* c, const double* R, const double* E, int npairs, int epochs, int batch, float lr,
                 double* final_loss) {
    DHT_TRY(check_ctx(c));
    if (!R || !E || npairs <= 0 || epochs < 0 || !(lr > 0)) return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    return nn_train_canon(c, R, E, npairs, epochs, batch, lr, final_loss);
}

int dht_nn_make_pairs(dht_ctx* c, const dht_probe_spec* spec, int64_t first, int nrhs, int restart, double* R,
                      double* E, int cap, int* count) {
    DHT_TRY(check_ctx(c));
    if (!spec || !R || !E || !count || nrhs <= 0 || nrhs > NN_MAX_BATCH || cap < 0 || restart <= 0)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    const int bp = pad_rhs(nrhs);
    const size_t fb = full_elems(c, bp) * 16;
    void *fz, *fx, *xs;
    DHT_TRY(ws_get(c, WS_Z, fb, &fz));
    DHT_TRY(ws_get(c, WS_PACK_OUT, fb, &fx));
    DHT_TRY(ws_get(c, WS_XSTAR, fb, &xs));
    DHT_TRY(probes_gen(c, spec, first, nrhs, bp, fz, DHT_FP64, nullptr, nullptr));
    dht_solver_params p{};
    p.method = DHT_SOLVER_BICGSTAB_FP64;
    p.tol = 1e-12;
    p.maxiter = 100000;
    std::vector<dht_solve_stats> st(bp);
    int rc = solve_fields(c, &p, fz, xs, bp, st.data());
    if (rc != DHT_OK) return rc;
    PairSink sink;
    sink.xstar = xs;
    sink.R = R;
    sink.E = E;
    sink.cap = cap;
    sink.nreal = nrhs;
    dht_solver_params q{};
    q.method = DHT_SOLVER_DC_FGMRES;
    q.tol = 1e-8;
    q.maxiter = 100000;
    q.restart = restart;
    q.inner_tol = 1e-6;
    rc = solve_fgmres(c, &q, fz, fx, bp, nullptr, false, &sink);
    if (rc != DHT_OK && rc != DHT_ERR_NOT_CONVERGED) return rc;
    DHT_HIP(hipStreamSynchronize(c->stream));
    *count = sink.count;
    return DHT_OK;
}

int dht_bench_hop(dht_ctx* c, int prec, int nrhs, int warmup, int reps, double* ms_per_call) {
    DHT_TRY(check_ctx(c));
    if (!valid_prec(prec) || nrhs <= 0 || nrhs > DHT_MAX_BATCH || (nrhs & (nrhs - 1)) || reps <= 0 || warmup < 0 ||
        !ms_per_call)
        return set_error(DHT_ERR_INVALID_ARG, "bad argument (nrhs must be a power of two)");
    if (!c->have_gauge) return set_error(DHT_ERR_STATE, "gauge field not set");
    size_t bytes = full_elems(c, nrhs) * elem_bytes(prec);
    void *fi, *fo;
    DHT_TRY(ws_get(c, WS_PACK_IN, bytes, &fi));
    DHT_TRY(ws_get(c, WS_PACK_OUT, bytes, &fo));
    dht_probe_spec sp = {12345u, 0u, 0};
    DHT_TRY(probes_gen(c, &sp, 0, nrhs, nrhs, fi, prec, nullptr, nullptr));
    const void* in_odd = (const char*)fi + bytes / 2;
    for (int i = 0; i < warmup; i++) DHT_TRY(hop(c, prec, 0, in_odd, fo, nullptr, 0.0, 1.0, nrhs, false, false));
    DHT_TRY(record(c, 0));
    for (int i = 0; i < reps; i++) DHT_TRY(hop(c, prec, 0, in_odd, fo, nullptr, 0.0, 1.0, nrhs, false, false));
    DHT_TRY(record(c, 1));
    DHT_HIP(hipStreamSynchronize(c->stream));
    *ms_per_call = elapsed(c, 0, 1) / reps;
    DHT_TRY(prof_harvest(c));
    return DHT_OK;
}

}  // extern "C"
