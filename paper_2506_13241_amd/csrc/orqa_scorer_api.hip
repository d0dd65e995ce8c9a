// Host side of the learned truncation scorer: training handle (C ABI).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/orqa.h"
#include "orqa_scorer.h"

using namespace orqa;

namespace orqa {
int api_fail(int code, const char* fmt, ...);  // orqa_api.hip: sets ps_last_error()

// Device arrays of one network + feature definition.
int scorer_alloc(ScorerDev* d) {
    std::memset(d, 0, sizeof *d);
    if (hipMalloc(reinterpret_cast<void**>(&d->W1), kScH * kScIn * 2) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->W2), kScH * kScH * 2) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->W3), kScH * 2) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->b1), kScH * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->b2), kScH * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->b3), 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->qmask), kScIn * sizeof(ulonglong2)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->letter), kScIn) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&d->fscale), kScIn * 4) != hipSuccess) {
        (void)hipGetLastError();
        return api_fail(PS_ERR_CAPACITY, "hipMalloc failed for the scorer network");
    }
    return PS_OK;
}

void scorer_free(ScorerDev* d) {
    void* ps[] = {d->W1, d->W2, d->W3, d->b1, d->b2, d->b3, d->qmask, d->letter, d->fscale};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    std::memset(d, 0, sizeof *d);
}

int scorer_copy(ScorerDev* dst, const ScorerDev* src, hipStream_t s) {
    struct {
        void* d;
        const void* s;
        size_t b;
    } c[] = {{dst->W1, src->W1, size_t(kScH) * kScIn * 2}, {dst->W2, src->W2, size_t(kScH) * kScH * 2},
             {dst->W3, src->W3, kScH * 2}, {dst->b1, src->b1, kScH * 4}, {dst->b2, src->b2, kScH * 4},
             {dst->b3, src->b3, 4}, {dst->qmask, src->qmask, kScIn * sizeof(ulonglong2)},
             {dst->letter, src->letter, kScIn}, {dst->fscale, src->fscale, kScIn * 4}};
    for (auto& e : c)
        if (hipMemcpyAsync(e.d, e.s, e.b, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return api_fail(PS_ERR_HIP, "copying the scorer network failed");
    return PS_OK;
}
}  // namespace orqa

struct ps_scorer {
    int nq = 0;
    hipStream_t stream = nullptr;
    ScorerDev dev{};
    float* params = nullptr;  // fp32 master, kScParams
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    int adam_t = 0;
    // training set
    uint64_t n = 0;
    ulonglong2* X = nullptr;
    ulonglong2* Z = nullptr;
    float* target = nullptr;
    float* y = nullptr;
    float* z1 = nullptr;
    float* z2 = nullptr;
    float* dy = nullptr;
    float* dz1 = nullptr;
    float* dz2 = nullptr;
    uint16_t* f = nullptr;
    double* loss = nullptr;
    int grid = 512;
};

namespace {

#define SC_TRY(expr)                                                                               \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess) return api_fail(PS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

void free_data(ps_scorer* s) {
    void* ps[] = {s->X, s->Z, s->target, s->y, s->z1, s->z2, s->dy, s->dz1, s->dz2, s->f};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    s->X = s->Z = nullptr;
    s->target = s->y = s->z1 = s->z2 = s->dy = s->dz1 = s->dz2 = nullptr;
    s->f = nullptr;
    s->n = 0;
}

int run_forward(ps_scorer* s, bool keep) {
    ScorerFwdArgs a{};
    a.net = s->dev;
    a.X = s->X;
    a.Z = s->Z;
    a.n = s->n;
    a.cap = s->n;
    a.nq = s->nq;
    a.y_out = s->y;
    a.z1_out = keep ? s->z1 : nullptr;
    a.z2_out = keep ? s->z2 : nullptr;
    a.f_out = keep ? s->f : nullptr;
    SC_TRY(launch_scorer_forward(a, s->stream, s->grid));
    return PS_OK;
}

}  // namespace

extern "C" {

int ps_scorer_create(int n_qubits, const uint64_t* qmask, const uint8_t* letters, const float* scales,
                     void* hip_stream, ps_scorer** out) {
    if (!out || !qmask || !letters || !scales) return api_fail(PS_ERR_INVALID, "NULL argument");
    if (n_qubits < 1 || n_qubits > 128) return api_fail(PS_ERR_INVALID, "n_qubits must be in 1..128");
    for (int i = 0; i < kScIn; ++i)
        if (letters[i] > 3) return api_fail(PS_ERR_INVALID, "feature %d: letter must be 0..3", i);
    ps_scorer* s = new ps_scorer;
    s->nq = n_qubits;
    s->stream = static_cast<hipStream_t>(hip_stream);
    int rc = scorer_alloc(&s->dev);
    if (rc) {
        delete s;
        return rc;
    }
    if (hipMalloc(reinterpret_cast<void**>(&s->params), kScParams * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&s->grad), kScParams * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&s->m), kScParams * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&s->v), kScParams * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&s->loss), 8) != hipSuccess) {
        scorer_free(&s->dev);
        delete s;
        return api_fail(PS_ERR_CAPACITY, "hipMalloc failed for the scorer parameters");
    }
    std::vector<ulonglong2> qm(kScIn);
    for (int i = 0; i < kScIn; ++i) qm[i] = make_ulonglong2(qmask[2 * i], qmask[2 * i + 1]);
    SC_TRY(hipMemcpyAsync(s->dev.qmask, qm.data(), kScIn * sizeof(ulonglong2), hipMemcpyHostToDevice, s->stream));
    SC_TRY(hipMemcpyAsync(s->dev.letter, letters, kScIn, hipMemcpyHostToDevice, s->stream));
    SC_TRY(hipMemcpyAsync(s->dev.fscale, scales, kScIn * 4, hipMemcpyHostToDevice, s->stream));
    SC_TRY(hipMemsetAsync(s->params, 0, kScParams * 4, s->stream));
    SC_TRY(hipMemsetAsync(s->m, 0, kScParams * 4, s->stream));
    SC_TRY(hipMemsetAsync(s->v, 0, kScParams * 4, s->stream));
    SC_TRY(launch_scorer_set(s->params, kScParams, s->dev, s->stream));
    SC_TRY(hipStreamSynchronize(s->stream));
    *out = s;
    return PS_OK;
}

int ps_scorer_destroy(ps_scorer* s) {
    if (!s) return PS_OK;
    (void)hipStreamSynchronize(s->stream);
    free_data(s);
    scorer_free(&s->dev);
    void* ps[] = {s->params, s->grad, s->m, s->v, s->loss};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    delete s;
    return PS_OK;
}

int ps_scorer_set_params(ps_scorer* s, const float* params, size_t n) {
    if (!s || !params) return api_fail(PS_ERR_INVALID, "NULL argument");
    if (n != size_t(kScParams)) return api_fail(PS_ERR_INVALID, "expected %d parameters, got %zu", kScParams, n);
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return api_fail(PS_ERR_NONFINITE, "parameter %zu is not finite", i);
    SC_TRY(hipMemcpyAsync(s->params, params, n * 4, hipMemcpyHostToDevice, s->stream));
    SC_TRY(hipMemsetAsync(s->m, 0, n * 4, s->stream));
    SC_TRY(hipMemsetAsync(s->v, 0, n * 4, s->stream));
    s->adam_t = 0;
    SC_TRY(launch_scorer_set(s->params, kScParams, s->dev, s->stream));
    SC_TRY(hipStreamSynchronize(s->stream));
    return PS_OK;
}

int ps_scorer_get_params(ps_scorer* s, float* params, size_t n) {
    if (!s || !params) return api_fail(PS_ERR_INVALID, "NULL argument");
    if (n != size_t(kScParams)) return api_fail(PS_ERR_INVALID, "expected %d parameters, got %zu", kScParams, n);
    SC_TRY(hipMemcpyAsync(params, s->params, n * 4, hipMemcpyDeviceToHost, s->stream));
    SC_TRY(hipStreamSynchronize(s->stream));
    return PS_OK;
}

int ps_scorer_set_data(ps_scorer* s, const ps_pauli* keys, const float* targets, size_t n) {
    if (!s || (n && (!keys || !targets))) return api_fail(PS_ERR_INVALID, "NULL argument");
    free_data(s);
    if (n == 0) return PS_OK;
    const size_t h = size_t(kScH);
    bool ok = hipMalloc(reinterpret_cast<void**>(&s->X), n * 16) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->Z), n * 16) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->target), n * 4) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->y), n * 4) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->z1), n * h * 4) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->z2), n * h * 4) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->dy), n * 4) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->dz1), n * h * 4) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->dz2), n * h * 4) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->f), n * kScIn * 2) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_data(s);
        return api_fail(PS_ERR_CAPACITY, "hipMalloc failed for %zu training strings", n);
    }
    std::vector<ulonglong2> X(n), Z(n);
    for (size_t i = 0; i < n; ++i) {
        X[i] = make_ulonglong2(keys[i].x[0], keys[i].x[1]);
        Z[i] = make_ulonglong2(keys[i].z[0], keys[i].z[1]);
    }
    SC_TRY(hipMemcpyAsync(s->X, X.data(), n * 16, hipMemcpyHostToDevice, s->stream));
    SC_TRY(hipMemcpyAsync(s->Z, Z.data(), n * 16, hipMemcpyHostToDevice, s->stream));
    SC_TRY(hipMemcpyAsync(s->target, targets, n * 4, hipMemcpyHostToDevice, s->stream));
    SC_TRY(hipStreamSynchronize(s->stream));
    s->n = n;
    return PS_OK;
}

int ps_scorer_forward(ps_scorer* s, float* y, uint16_t* features) {
    if (!s) return api_fail(PS_ERR_INVALID, "NULL argument");
    if (s->n == 0) return PS_OK;
    int rc = run_forward(s, true);
    if (rc) return rc;
    if (y) SC_TRY(hipMemcpyAsync(y, s->y, s->n * 4, hipMemcpyDeviceToHost, s->stream));
    if (features) SC_TRY(hipMemcpyAsync(features, s->f, s->n * kScIn * 2, hipMemcpyDeviceToHost, s->stream));
    SC_TRY(hipStreamSynchronize(s->stream));
    return PS_OK;
}

int ps_scorer_loss_grad(ps_scorer* s, double* loss, float* grad) {
    if (!s) return api_fail(PS_ERR_INVALID, "NULL argument");
    if (s->n == 0) return api_fail(PS_ERR_INVALID, "no training data");
    int rc = run_forward(s, true);
    if (rc) return rc;
    ScorerBwdArgs b{};
    b.net = s->dev;
    b.n = s->n;
    b.y = s->y;
    b.target = s->target;
    b.z1 = s->z1;
    b.z2 = s->z2;
    b.dy = s->dy;
    b.dz1 = s->dz1;
    b.dz2 = s->dz2;
    SC_TRY(launch_scorer_backward(b, s->f, s->grad, s->stream));
    SC_TRY(launch_scorer_loss(s->y, s->target, s->n, s->loss, s->stream));
    if (loss) SC_TRY(hipMemcpyAsync(loss, s->loss, 8, hipMemcpyDeviceToHost, s->stream));
    if (grad) SC_TRY(hipMemcpyAsync(grad, s->grad, kScParams * 4, hipMemcpyDeviceToHost, s->stream));
    SC_TRY(hipStreamSynchronize(s->stream));
    return PS_OK;
}

int ps_scorer_adam_step(ps_scorer* s, float lr) {
    if (!s) return api_fail(PS_ERR_INVALID, "NULL argument");
    s->adam_t += 1;
    SC_TRY(launch_scorer_adam(s->params, s->grad, s->m, s->v, kScParams, lr, s->adam_t, s->dev, s->stream));
    SC_TRY(hipStreamSynchronize(s->stream));
    return PS_OK;
}

}  // extern "C"

// Used by the propagation handle (orqa_api.hip).
namespace orqa {
const ScorerDev* scorer_dev(const ps_scorer* s) { return &s->dev; }
}  // namespace orqa
