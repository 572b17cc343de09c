// GP-SPCA solve server: continuous batching of independent solves on one GPU.
//
// A client registers host matrices (FP32, kept by the client; stored on the
// device in FP32 or bfloat16) and submits requests (formulation, m, gamma, mu,
// tol, max_iter) against them.  `slots` worker threads, each with its own HIP
// stream, take requests as soon as a slot and device memory are free, so
// solves that arrive while others run are admitted and overlap on the device.
// All device memory is sub-allocated from one caller-provided arena
// (serve_core.h): a matrix is uploaded on its first admission, stays resident
// with its cached column norms for later requests on it, and is evicted (least
// recently used first) only when no admitted request uses it and space is
// needed.  Each request's workspace and device outputs live in the arena for
// the duration of its solve; results are copied to host memory owned by the
// server until the client releases them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gpspca_internal.h"
#include "serve_core.h"

namespace gpspca {

namespace {

constexpr size_t kStageBytes = (size_t)64 << 20;  // per-slot device staging for bfloat16 storage
constexpr size_t kPinnedBytes = (size_t)32 << 20; // per-slot pinned host buffer (two halves)

size_t al(size_t x) { return serve::align_up(x); }

struct SMatrix {
    uint64_t id = 0;
    const float* host = nullptr;
    int64_t p = 0, n = 0, ld = 0;
    int dtype = GPSPCA_F32;
    int64_t lda_dev = 0;
    size_t data_bytes = 0;   // device storage of A
    size_t norms_off = 0;    // cached column norms (n doubles) after the data
    size_t bytes = 0;        // data + norms
    bool ready = false;      // uploaded and norms computed
    bool unregistered = false;
};

struct SRequest {
    uint64_t id = 0, matrix = 0;
    int form = 0, m = 1, max_iter = 1;
    double gamma = 0.0, tol = 0.0;
    std::vector<double> mu;
    size_t solve_ws = 0, ws_bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int uploaded = 0;
    bool done = false;
    int status = 0;
    int n_iter = 0;
    int multistart = 0;                 // single-unit form with m > 1: m starts
    std::vector<int> col_n_iter, col_status;
    std::string error;
    std::vector<float> X, Z;
    std::vector<uint32_t> support;
    std::vector<double> trace;
};

}  // namespace

struct Server {
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work;    // workers: something to admit / stop
    std::condition_variable cv_done;    // clients: a request finished; uploads finished
    serve::Scheduler sched;
    std::unordered_map<uint64_t, SMatrix> mats;
    std::unordered_map<uint64_t, SRequest> reqs;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<size_t> stage_off;
    std::vector<uint8_t*> pinned;       // per slot, kPinnedBytes of page-locked host memory
    uint64_t next_matrix = 1, next_req = 1;
    bool stop = false;
    int running = 0;
    uint64_t completed = 0, uploads = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void worker(int slot);
    int upload(SMatrix& M, size_t off, int slot, hipStream_t st, std::string* err);
    hipError_t download(const void* const* src, void* const* dst, const size_t* bytes, int count,
                        int slot, hipStream_t st);
};

// Copy a registered host matrix into the arena at `off`, then its column
// norms.  Column chunks go through the slot's pinned host buffer (two halves:
// the host copies chunk k+1 while the DMA engine moves chunk k); FP32 storage
// lands in place, bfloat16 storage lands in the slot's device staging area and
// is quantized from there.
int Server::upload(SMatrix& M, size_t off, int slot, hipStream_t st, std::string* err) {
    uint8_t* dst = arena + off;
    auto hip_ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        *err = std::string(what) + ": " + hipGetErrorString(e);
        return false;
    };
    const bool f32 = M.dtype == GPSPCA_F32;
    const size_t half = kPinnedBytes / 2;
    // FP32 chunks are laid out with the device leading dimension, bfloat16
    // chunks densely (leading dimension p) for the quantizer
    const int64_t ldc = f32 ? M.lda_dev : M.p;
    int64_t cols = (int64_t)(half / (sizeof(float) * ldc));
    if (!f32) cols = std::min<int64_t>(cols, (int64_t)(kStageBytes / (sizeof(float) * M.p)));
    if (cols < 1) {
        *err = "a column exceeds the upload staging buffer";
        return GPSPCA_ENOMEM;
    }
    hipEvent_t done[2] = {nullptr, nullptr};
    for (int h = 0; h < 2; ++h)
        if (!hip_ok(hipEventCreateWithFlags(&done[h], hipEventDisableTiming), "upload")) {
            if (done[0]) (void)hipEventDestroy(done[0]);
            return GPSPCA_EDEVICE;
        }
    int rc = GPSPCA_OK;
    int k = 0;
    for (int64_t c0 = 0; c0 < M.n && rc == GPSPCA_OK; c0 += cols, ++k) {
        const int64_t nc = std::min<int64_t>(cols, M.n - c0);
        uint8_t* buf = pinned[slot] + (k & 1) * half;
        // the half is free once the copy issued two chunks ago has finished
        if (k >= 2 && !hip_ok(hipEventSynchronize(done[k & 1]), "upload")) { rc = GPSPCA_EDEVICE; break; }
        float* hb = reinterpret_cast<float*>(buf);
        for (int64_t c = 0; c < nc; ++c)
            std::memcpy(hb + c * ldc, M.host + (c0 + c) * M.ld, sizeof(float) * M.p);
        if (f32) {
            if (!hip_ok(hipMemcpyAsync(dst + sizeof(float) * c0 * M.lda_dev, buf,
                                       sizeof(float) * (size_t)(nc * ldc), hipMemcpyHostToDevice, st),
                        "upload")) { rc = GPSPCA_EDEVICE; break; }
        } else {
            uint8_t* stage = arena + stage_off[slot];
            if (!hip_ok(hipMemcpyAsync(stage, buf, sizeof(float) * (size_t)(nc * ldc),
                                       hipMemcpyHostToDevice, st),
                        "upload") ||
                !hip_ok(launch_quantize(reinterpret_cast<const float*>(stage), M.p, (int)M.p, nc,
                                        GPSPCA_BF16, dst + sizeof(uint16_t) * c0 * M.lda_dev,
                                        M.lda_dev, nullptr, st),
                        "quantize")) { rc = GPSPCA_EDEVICE; break; }
        }
        if (!hip_ok(hipEventRecord(done[k & 1], st), "upload")) { rc = GPSPCA_EDEVICE; break; }
    }
    if (rc == GPSPCA_OK && !hip_ok(hipStreamSynchronize(st), "upload")) rc = GPSPCA_EDEVICE;
    for (int h = 0; h < 2; ++h) (void)hipEventDestroy(done[h]);
    if (rc != GPSPCA_OK) return rc;
    gpspca_matrix A;
    std::memset(&A, 0, sizeof(A));
    A.data = dst;
    A.p = M.p;
    A.n = M.n;
    A.lda = M.lda_dev;
    A.dtype = M.dtype;
    rc = gpspca_column_norms(&A, reinterpret_cast<double*>(arena + off + M.norms_off), st);
    if (rc != GPSPCA_OK) {
        *err = gpspca_last_error();
        return rc;
    }
    if (!hip_ok(hipStreamSynchronize(st), "upload")) return GPSPCA_EDEVICE;
    return GPSPCA_OK;
}

// Device-to-host copies of a request's results through the slot's pinned
// buffer (into pageable memory the runtime would stage each copy itself, at a
// fraction of the bandwidth): as many arrays per round trip as fit, larger
// ones in chunks.
hipError_t Server::download(const void* const* src, void* const* dst, const size_t* bytes,
                            int count, int slot, hipStream_t st) {
    uint8_t* buf = pinned[slot];
    int i = 0;
    size_t done_i = 0;   // bytes of array i already copied
    while (i < count) {
        // fill the buffer with the rest of array i and as many next arrays as fit
        struct Piece { int a; size_t from, nb, at; };
        Piece pc[8];
        int np = 0;
        size_t used = 0;
        while (i < count && np < 8 && used < kPinnedBytes) {
            const size_t nb = std::min(bytes[i] - done_i, kPinnedBytes - used);
            if (nb > 0) {
                const hipError_t e = hipMemcpyAsync(buf + used,
                                                    static_cast<const uint8_t*>(src[i]) + done_i, nb,
                                                    hipMemcpyDeviceToHost, st);
                if (e != hipSuccess) return e;
                pc[np++] = Piece{i, done_i, nb, used};
                used += (nb + 255) & ~(size_t)255;
            }
            done_i += nb;
            if (done_i == bytes[i]) { ++i; done_i = 0; }
            if (used >= kPinnedBytes) break;
        }
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        for (int k = 0; k < np; ++k)
            std::memcpy(static_cast<uint8_t*>(dst[pc[k].a]) + pc[k].from, buf + pc[k].at, pc[k].nb);
    }
    return hipSuccess;
}

void Server::worker(int slot) {
    (void)hipSetDevice(device);
    hipStream_t st = streams[slot];
    for (;;) {
        serve::Admission adm;
        SRequest* R = nullptr;
        SMatrix* M = nullptr;
        bool do_upload = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || (sched.waiting() > 0 && sched.admit(&adm)); });
            if (stop) return;
            R = &reqs[adm.req];
            M = &mats[adm.matrix];
            R->t_admit = now();
            do_upload = adm.upload;
            for (uint64_t e : adm.evicted) {
                auto it = mats.find(e);
                if (it != mats.end()) it->second.ready = false;
            }
            if (do_upload) {
                M->ready = false;
                R->uploaded = 1;
                uploads += 1;
            }
            running += 1;
        }
        int rc = GPSPCA_OK;
        std::string err;
        if (do_upload) {
            rc = upload(*M, adm.matrix_offset, slot, st, &err);
            std::lock_guard<std::mutex> lk(mu);
            if (rc == GPSPCA_OK) M->ready = true;
            else sched.drop_residency(adm.matrix);
            cv_done.notify_all();
        } else {
            // another slot may still be uploading this matrix
            std::unique_lock<std::mutex> lk(mu);
            cv_done.wait(lk, [&] { return M->ready || !sched.matrix(adm.matrix)->resident; });
            if (!M->ready) {
                rc = GPSPCA_EDEVICE;
                err = "matrix upload failed";
            }
        }
        if (rc == GPSPCA_OK) {
            gpspca_matrix A;
            std::memset(&A, 0, sizeof(A));
            A.data = arena + adm.matrix_offset;
            A.p = M->p;
            A.n = M->n;
            A.lda = M->lda_dev;
            A.dtype = M->dtype;
            uint8_t* ws = arena + adm.ws_offset;
            float* Xd = reinterpret_cast<float*>(ws + R->solve_ws);
            float* Zd = reinterpret_cast<float*>(ws + R->solve_ws + al(sizeof(float) * M->p * R->m));
            uint32_t* Sd = reinterpret_cast<uint32_t*>(
                ws + R->solve_ws + al(sizeof(float) * M->p * R->m) + al(sizeof(float) * M->n * R->m));
            int nit = 0;
            const double* norms =
                reinterpret_cast<const double*>(arena + adm.matrix_offset + M->norms_off);
            if (R->multistart) {
                // m single-unit problems from the m columns of largest norm
                const std::vector<double> gam((size_t)R->m, R->gamma);
                std::vector<double> tr((size_t)R->m * R->max_iter, 0.0);
                R->col_n_iter.assign(R->m, 0);
                R->col_status.assign(R->m, 0);
                rc = solve_core(&A, R->form, R->m, 0.0, nullptr, gam.data(), 1, nullptr, nullptr,
                                R->tol, R->max_iter, ws, R->solve_ws, st, Xd, Zd, Sd, tr.data(),
                                R->col_n_iter.data(), R->col_status.data(), norms, 1);
                for (int k = 0; k < R->m; ++k) nit = std::max(nit, R->col_n_iter[k]);
                // problem k's trace at [k * n_iter, k * n_iter + col_n_iter[k])
                R->trace.assign((size_t)R->m * nit, 0.0);
                for (int k = 0; k < R->m; ++k)
                    std::copy(tr.begin() + (size_t)k * R->max_iter,
                              tr.begin() + (size_t)k * R->max_iter + R->col_n_iter[k],
                              R->trace.begin() + (size_t)k * nit);
            } else {
                R->trace.assign(R->max_iter, 0.0);
                rc = solve_core(&A, R->form, R->m, R->gamma,
                                R->mu.empty() ? nullptr : R->mu.data(), nullptr, 0, nullptr,
                                nullptr, R->tol, R->max_iter, ws, R->solve_ws, st, Xd, Zd, Sd,
                                R->trace.data(), &nit, nullptr, norms);
            }
            if (rc >= 0) {
                const size_t words = (size_t)((M->n + 31) / 32);
                R->X.resize((size_t)M->p * R->m);
                R->Z.resize((size_t)M->n * R->m);
                R->support.resize(words * R->m);
                const void* src[3] = {Xd, Zd, Sd};
                void* dst[3] = {R->X.data(), R->Z.data(), R->support.data()};
                const size_t nbytes[3] = {sizeof(float) * R->X.size(), sizeof(float) * R->Z.size(),
                                          sizeof(uint32_t) * R->support.size()};
                hipError_t e = download(src, dst, nbytes, 3, slot, st);
                if (e != hipSuccess) {
                    rc = GPSPCA_EDEVICE;
                    err = hipGetErrorString(e);
                }
                R->n_iter = nit;
                if (!R->multistart) R->trace.resize(std::max(0, nit));
            } else {
                err = gpspca_last_error();
            }
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            sched.finish(adm.matrix, adm.ws_offset);
            R->status = rc;
            R->error = err;
            R->t_done = now();
            R->done = true;
            running -= 1;
            completed += 1;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

}  // namespace gpspca

using gpspca::Server;

struct gpspca_server {
    Server s;
};

extern "C" {

int gpspca_server_create(void* arena, size_t arena_bytes, int slots, gpspca_server** out) {
    using namespace gpspca;
    if (!out) return fail(GPSPCA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!arena) return fail(GPSPCA_EINVAL, "arena is NULL");
    if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0)
        return fail(GPSPCA_EINVAL, "arena must be 256-byte aligned");
    if (slots < 1 || slots > 16) return fail(GPSPCA_EINVAL, "need 1 <= slots <= 16");
    const size_t staging = (size_t)slots * kStageBytes;
    if (arena_bytes < staging + ((size_t)64 << 20))
        return fail(GPSPCA_ENOMEM, "arena too small for the staging areas");
    std::unique_ptr<gpspca_server> S(new gpspca_server());
    Server& s = S->s;
    s.arena = static_cast<uint8_t*>(arena);
    s.arena_bytes = arena_bytes;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GPSPCA_EDEVICE, hipGetErrorString(e));
    s.device = dev;
    // staging areas at the end of the arena; the scheduler manages the rest
    const size_t managed = (arena_bytes - staging) / serve::kAlign * serve::kAlign;
    s.sched = serve::Scheduler(managed);
    for (int i = 0; i < slots; ++i) s.stage_off.push_back(managed + (size_t)i * kStageBytes);
    auto release_all = [&s]() {
        for (auto x : s.streams) (void)hipStreamDestroy(x);
        for (auto h : s.pinned) (void)hipHostFree(h);
    };
    for (int i = 0; i < slots; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            release_all();
            return fail(GPSPCA_EDEVICE, hipGetErrorString(e));
        }
        s.streams.push_back(st);
        void* h = nullptr;
        e = hipHostMalloc(&h, kPinnedBytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            release_all();
            return fail(GPSPCA_EDEVICE, hipGetErrorString(e));
        }
        s.pinned.push_back(static_cast<uint8_t*>(h));
    }
    for (int i = 0; i < slots; ++i) s.workers.emplace_back([&s, i] { s.worker(i); });
    *out = S.release();
    return GPSPCA_OK;
}

int gpspca_server_register(gpspca_server* S, const float* host, int64_t p, int64_t n, int64_t ld,
                           int store_dtype, uint64_t* matrix_id) {
    using namespace gpspca;
    if (!S || !host || !matrix_id) return fail(GPSPCA_EINVAL, "NULL argument");
    if (p < 1 || n < 1 || ld < p) return fail(GPSPCA_EINVAL, "need p, n >= 1 and ld >= p");
    if (n >= ((int64_t)1 << 31) || p > ((int64_t)1 << 30)) return fail(GPSPCA_EINVAL, "matrix too large");
    if (store_dtype != GPSPCA_F32 && store_dtype != GPSPCA_BF16)
        return fail(GPSPCA_EDTYPE, "the server stores FP32 or BF16");
    Server& s = S->s;
    SMatrix M;
    M.host = host;
    M.p = p;
    M.n = n;
    M.ld = ld;
    M.dtype = store_dtype;
    M.lda_dev = store_dtype == GPSPCA_F32 ? (p + 3) / 4 * 4 : (p + 15) / 16 * 16;
    M.data_bytes = (store_dtype == GPSPCA_F32 ? 4 : 2) * (size_t)M.lda_dev * (size_t)n;
    M.norms_off = al(M.data_bytes);
    M.bytes = M.norms_off + al(sizeof(double) * (size_t)n);
    std::lock_guard<std::mutex> lk(s.mu);
    M.id = s.next_matrix++;
    s.sched.add_matrix(M.id, M.bytes);
    s.mats[M.id] = M;
    *matrix_id = M.id;
    return GPSPCA_OK;
}

int gpspca_server_unregister(gpspca_server* S, uint64_t matrix_id) {
    using namespace gpspca;
    if (!S) return fail(GPSPCA_EINVAL, "server is NULL");
    Server& s = S->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.mats.find(matrix_id);
    if (it == s.mats.end()) return fail(GPSPCA_EINVAL, "unknown matrix");
    for (auto& kv : s.reqs)
        if (kv.second.matrix == matrix_id && !kv.second.done)
            return fail(GPSPCA_EINVAL, "the matrix has pending requests");
    if (!s.sched.remove_matrix(matrix_id)) return fail(GPSPCA_EINVAL, "the matrix is in use");
    s.mats.erase(it);
    return GPSPCA_OK;
}

int gpspca_server_submit(gpspca_server* S, uint64_t matrix_id, int form, int m, double gamma,
                         const double* mu, double tol, int max_iter, uint64_t* request_id) {
    using namespace gpspca;
    if (!S || !request_id) return fail(GPSPCA_EINVAL, "NULL argument");
    Server& s = S->s;
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.mats.find(matrix_id);
    if (it == s.mats.end()) return fail(GPSPCA_EINVAL, "unknown matrix");
    const SMatrix& M = it->second;
    gpspca_matrix A;
    std::memset(&A, 0, sizeof(A));
    A.data = s.arena;  // a valid aligned pointer; only the shape is used here
    A.p = M.p;
    A.n = M.n;
    A.lda = M.lda_dev;
    A.dtype = M.dtype;
    // a single-unit form with m > 1 runs m starts (the m columns of largest norm)
    const int multistart = (form == GPSPCA_SL1 || form == GPSPCA_SL0) && m > 1;
    int rc = check_problem(&A, form, multistart ? 1 : m, gamma, mu);
    if (rc) return rc;
    if (m < 1 || m > GPSPCA_MAX_M) return fail(GPSPCA_EINVAL, "need 1 <= m <= GPSPCA_MAX_M");
    if (!std::isfinite(tol) || tol < 0.0) return fail(GPSPCA_EINVAL, "tol must be finite and >= 0");
    if (max_iter < 1) return fail(GPSPCA_EINVAL, "max_iter must be >= 1");
    if (m > M.n) return fail(GPSPCA_EINVAL, "default start needs m <= n");
    const size_t ws = multistart ? gpspca_path_workspace_bytes(&A, m, max_iter)
                                 : gpspca_workspace_bytes(&A, form, m, max_iter);
    if (ws == 0) return GPSPCA_EINVAL;
    SRequest R;
    R.matrix = matrix_id;
    R.form = form;
    R.m = m;
    R.gamma = gamma;
    R.tol = tol;
    R.max_iter = max_iter;
    R.multistart = multistart;
    if (mu && form >= GPSPCA_BL1) R.mu.assign(mu, mu + m);
    R.solve_ws = al(ws);
    R.ws_bytes = R.solve_ws + al(sizeof(float) * M.p * m) + al(sizeof(float) * M.n * m) +
                 al(sizeof(uint32_t) * (size_t)((M.n + 31) / 32) * m);
    if (!s.sched.fits_alone(matrix_id, R.ws_bytes))
        return fail(GPSPCA_ENOMEM, "the request does not fit in the arena");
    R.id = s.next_req++;
    R.t_submit = s.now();
    serve::Waiting w;
    w.req = R.id;
    w.matrix = matrix_id;
    w.ws_bytes = R.ws_bytes;
    s.reqs[R.id] = std::move(R);
    s.sched.enqueue(w);
    *request_id = w.req;
    lk.unlock();
    s.cv_work.notify_one();
    return GPSPCA_OK;
}

static int fill_result(const gpspca::SRequest& R, const gpspca::SMatrix* M, gpspca_result* out) {
    if (!out) return GPSPCA_OK;
    std::memset(out, 0, sizeof(*out));
    out->status = R.status;
    out->n_iter = R.n_iter;
    out->m = R.m;
    out->p = M ? M->p : 0;
    out->n = M ? M->n : 0;
    out->X = R.X.empty() ? nullptr : R.X.data();
    out->Z = R.Z.empty() ? nullptr : R.Z.data();
    out->support = R.support.empty() ? nullptr : R.support.data();
    out->obj_trace = R.trace.empty() ? nullptr : R.trace.data();
    out->col_n_iter = R.col_n_iter.empty() ? nullptr : R.col_n_iter.data();
    out->col_status = R.col_status.empty() ? nullptr : R.col_status.data();
    out->t_submit = R.t_submit;
    out->t_admit = R.t_admit;
    out->t_done = R.t_done;
    out->uploaded = R.uploaded;
    return GPSPCA_OK;
}

int gpspca_server_poll(gpspca_server* S, uint64_t request_id, gpspca_result* out) {
    using namespace gpspca;
    if (!S) return fail(GPSPCA_EINVAL, "server is NULL");
    Server& s = S->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.reqs.find(request_id);
    if (it == s.reqs.end()) return fail(GPSPCA_EINVAL, "unknown request");
    if (!it->second.done) return 1;
    auto mt = s.mats.find(it->second.matrix);
    fill_result(it->second, mt == s.mats.end() ? nullptr : &mt->second, out);
    if (it->second.status < 0) fail(it->second.status, it->second.error);
    return 0;
}

int gpspca_server_wait(gpspca_server* S, uint64_t request_id, gpspca_result* out) {
    using namespace gpspca;
    if (!S) return fail(GPSPCA_EINVAL, "server is NULL");
    Server& s = S->s;
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.reqs.find(request_id);
    if (it == s.reqs.end()) return fail(GPSPCA_EINVAL, "unknown request");
    s.cv_done.wait(lk, [&] { return it->second.done; });
    auto mt = s.mats.find(it->second.matrix);
    fill_result(it->second, mt == s.mats.end() ? nullptr : &mt->second, out);
    if (it->second.status < 0) fail(it->second.status, it->second.error);
    return 0;
}

int gpspca_server_release(gpspca_server* S, uint64_t request_id) {
    using namespace gpspca;
    if (!S) return fail(GPSPCA_EINVAL, "server is NULL");
    Server& s = S->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.reqs.find(request_id);
    if (it == s.reqs.end()) return fail(GPSPCA_EINVAL, "unknown request");
    if (!it->second.done) return fail(GPSPCA_EINVAL, "the request is still pending");
    s.reqs.erase(it);
    return GPSPCA_OK;
}

int gpspca_server_stats(gpspca_server* S, gpspca_stats* out) {
    using namespace gpspca;
    if (!S || !out) return fail(GPSPCA_EINVAL, "NULL argument");
    Server& s = S->s;
    std::lock_guard<std::mutex> lk(s.mu);
    std::memset(out, 0, sizeof(*out));
    out->waiting = (int64_t)s.sched.waiting();
    out->running = s.running;
    out->completed = (int64_t)s.completed;
    out->uploads = (int64_t)s.uploads;
    out->evictions = (int64_t)s.sched.evictions();
    out->resident_bytes = s.sched.resident_bytes();
    out->free_bytes = s.sched.arena().free_bytes();
    out->arena_bytes = s.sched.arena().size();
    return GPSPCA_OK;
}

int gpspca_server_destroy(gpspca_server* S) {
    using namespace gpspca;
    if (!S) return GPSPCA_OK;
    Server& s = S->s;
    {
        // wait for every submitted request, then stop the workers
        std::unique_lock<std::mutex> lk(s.mu);
        s.cv_done.wait(lk, [&] { return s.sched.waiting() == 0 && s.running == 0; });
        s.stop = true;
    }
    s.cv_work.notify_all();
    for (auto& t : s.workers) t.join();
    for (auto st : s.streams) (void)hipStreamDestroy(st);
    for (auto h : s.pinned) (void)hipHostFree(h);
    delete S;
    return GPSPCA_OK;
}

}  // extern "C"
