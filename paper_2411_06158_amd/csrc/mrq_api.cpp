// Host runtime behind the C ABI of include/mrq.h: argument checking, the build sequence of
// Algorithm 1, the search dispatch (batched and per-query), persistence and instrumentation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "mrq_internal.h"

namespace mrq {

namespace {

thread_local std::string g_err;

struct Fail : std::runtime_error {
    mrq_status code;
    Fail(mrq_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            throw Fail(MRQ_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
        throw Fail(MRQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

mrq_status set_err(mrq_status s, const std::string& m) {
    g_err = m;
    return s;
}

template <class F>
mrq_status guarded(F&& f) {
    try {
        g_err.clear();
        return f();
    } catch (const Fail& e) {
        return set_err(e.code, e.what());
    } catch (const std::bad_alloc&) {
        return set_err(MRQ_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return set_err(MRQ_EDEVICE, e.what());
    }
}

bool is_device_ptr(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.isManaged;
}

struct DevTemp {
    void* p = nullptr;
    size_t bytes = 0;
    DevTemp() = default;
    explicit DevTemp(size_t b) { alloc(b); }
    void alloc(size_t b) {
        release();
        bytes = b ? b : 1;
        hip_check(hipMalloc(&p, bytes), "hipMalloc (build scratch)");
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    template <class T>
    T* as() const { return reinterpret_cast<T*>(p); }
    ~DevTemp() { release(); }
    DevTemp(const DevTemp&) = delete;
    DevTemp& operator=(const DevTemp&) = delete;
};

template <class T>
T* dalloc(Index* ix, int64_t n) {
    void* p = nullptr;
    size_t b = (size_t)(n > 0 ? n : 1) * sizeof(T);
    hip_check(hipMalloc(&p, b), "hipMalloc (index)");
    ix->allocations.push_back(p);
    ix->device_bytes += (int64_t)b;
    return reinterpret_cast<T*>(p);
}

void upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
}
void download(void* dst, const void* src, size_t bytes, hipStream_t s) {
    hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), "download");
    hip_check(hipStreamSynchronize(s), "download sync");
}

// SplitMix64 (Steele, Lea, Flood 2014) for the seeded choices of the build.
uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Haar-random orthogonal d x d matrix (Section 4.2's random rotation P): Householder QR of a seeded
// Gaussian matrix with the signs of diag(R) folded into Q.  Row-major, columns orthonormal.
std::vector<double> haar_rotation(int d, uint64_t seed) {
    std::vector<double> A((size_t)d * d);
    uint64_t s = seed;
    const double two_pi = 6.283185307179586476925286766559;
    for (size_t i = 0; i < A.size(); i += 2) {
        double u1 = 1.0 - (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
        double u2 = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
        double r = std::sqrt(-2.0 * std::log(u1));
        A[i] = r * std::cos(two_pi * u2);
        if (i + 1 < A.size()) A[i + 1] = r * std::sin(two_pi * u2);
    }
    // Householder: A = Q R, reflectors v_k stored separately
    std::vector<std::vector<double>> vs;
    std::vector<double> rdiag(d);
    for (int k = 0; k < d; k++) {
        double nrm = 0.0;
        for (int i = k; i < d; i++) nrm += A[(size_t)i * d + k] * A[(size_t)i * d + k];
        nrm = std::sqrt(nrm);
        const double akk = A[(size_t)k * d + k];
        const double alpha = akk > 0 ? -nrm : nrm;
        std::vector<double> v(d, 0.0);
        for (int i = k; i < d; i++) v[i] = A[(size_t)i * d + k];
        v[k] -= alpha;
        double vn = 0.0;
        for (int i = k; i < d; i++) vn += v[i] * v[i];
        if (vn > 0) {
            for (int j = k; j < d; j++) {
                double dot = 0.0;
                for (int i = k; i < d; i++) dot += v[i] * A[(size_t)i * d + j];
                const double f = 2.0 * dot / vn;
                for (int i = k; i < d; i++) A[(size_t)i * d + j] -= f * v[i];
            }
        }
        rdiag[k] = A[(size_t)k * d + k];
        vs.push_back(std::move(v));
    }
    // Q = H_0 H_1 ... H_{d-1} applied to the identity, then Q diag(sign(r_kk))
    std::vector<double> Q((size_t)d * d, 0.0);
    for (int i = 0; i < d; i++) Q[(size_t)i * d + i] = 1.0;
    for (int k = d - 1; k >= 0; k--) {
        const std::vector<double>& v = vs[k];
        double vn = 0.0;
        for (int i = k; i < d; i++) vn += v[i] * v[i];
        if (vn == 0) continue;
        for (int j = 0; j < d; j++) {
            double dot = 0.0;
            for (int i = k; i < d; i++) dot += v[i] * Q[(size_t)i * d + j];
            const double f = 2.0 * dot / vn;
            for (int i = k; i < d; i++) Q[(size_t)i * d + j] -= f * v[i];
        }
    }
    for (int j = 0; j < d; j++)
        if (rdiag[j] < 0)
            for (int i = 0; i < d; i++) Q[(size_t)i * d + j] = -Q[(size_t)i * d + j];
    return Q;
}

// The split exact stage (||x - q||^2 = dis_o' - 2 <x_r, q_r>, Section 5.2's separate leading and tail
// blocks) is taken when the tail is no wider than the leading block: its exact stage then reads at most half
// of a row, and the query's tail coordinates, now needed in FP32, cost at most as much as the leading ones.
void set_split(Index& ix) {
    ix.Dr = ix.D - ix.d;
    ix.split = ix.Dr <= ix.d;
    ix.Dr4 = ix.split ? (ix.Dr + 3) & ~3 : 0;
}

void check_args_build(const float* X, int64_t N, int32_t D, int32_t d, int32_t B, int32_t nlist) {
    if (!X) throw Fail(MRQ_EINVAL, "X is NULL");
    if (N < 1 || N >= (int64_t)0x7fffffff) throw Fail(MRQ_EINVAL, "N must be in [1, 2^31 - 1)");
    if (D < 2) throw Fail(MRQ_EINVAL, "D must be >= 2");
    if (d != 0 && (d < 2 || d > D)) throw Fail(MRQ_EINVAL, "d_r must be 0 (automatic) or in [2, D]");
    if (d > 1536) throw Fail(MRQ_EINVAL, "d_r above 1536 is not supported");
    if (B < 1 || B > 8) throw Fail(MRQ_EINVAL, "bits must be in [1, 8]");
    if (nlist < 1 || nlist > N) throw Fail(MRQ_EINVAL, "nlist must be in [1, N]");
    if (nlist > 16384) throw Fail(MRQ_EINVAL, "nlist above 16384 is not supported");
    if (N + 64 * (int64_t)nlist >= (int64_t)0x7fffffff)
        throw Fail(MRQ_EINVAL, "N + 64 nlist must be below 2^31 - 1 (rows are addressed with int32)");
}

}  // namespace

// ---- KernelTimer ------------------------------------------------------------------------------

int KernelTimer::slot_of(const char* name) {
    for (size_t i = 0; i < names.size(); i++)
        if (names[i] == name) return (int)i;
    names.emplace_back(name);
    ms.push_back(0.0);
    launches.push_back(0);
    return (int)names.size() - 1;
}
void KernelTimer::begin(hipStream_t s, const char* name, Pending* p) {
    p->slot = slot_of(name);
    for (hipEvent_t* e : {&p->a, &p->b}) {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
        } else if (hipEventCreateWithFlags(e, hipEventDisableSystemFence) != hipSuccess) {
            // timing markers only (read after a synchronisation): no system-scope fence, which would write
            // back the caches between the kernels being timed
            p->slot = -1;
            return;
        }
    }
    (void)hipEventRecord(p->a, s);
}
void KernelTimer::end(hipStream_t s, Pending* p) {
    (void)hipEventRecord(p->b, s);
    pending.push_back(*p);
}
void KernelTimer::collect() {
    for (auto& p : pending) {
        float t = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            ms[p.slot] += t;
            launches[p.slot] += 1;
        }
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}
KernelTimer::~KernelTimer() {
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
}

Index::~Index() {
    if (aux) {
        (void)hipStreamSynchronize(aux);
        (void)hipStreamDestroy(aux);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ws.base) (void)hipFree(ws.base);
    for (void* p : ws.retired) (void)hipFree(p);
    for (void* p : allocations) (void)hipFree(p);
}

// ---- build (Algorithm 1) ----------------------------------------------------------------------

static mrq_index* build_index(const float* X, int64_t N, int32_t D, int32_t d, int32_t B, int32_t nlist,
                              const mrq_build_opts& o, hipStream_t s) {
    std::unique_ptr<mrq_index> ix(new mrq_index());
    hip_check(hipGetDevice(&ix->device), "hipGetDevice");
    ix->N = N; ix->D = D; ix->B = B; ix->nlist = nlist;
    ix->D4 = (D + 3) & ~3;

    // input on the device
    const float* Xd = X;
    DevTemp xcopy;
    if (!is_device_ptr(X)) {
        xcopy.alloc((size_t)N * D * sizeof(float));
        upload(xcopy.p, X, (size_t)N * D * sizeof(float), s);
        Xd = xcopy.as<float>();
    }
    {
        DevTemp bad(sizeof(int32_t));
        hip_check(launch_fill_i32(bad.as<int32_t>(), 0, 1, s), "fill");
        hip_check(launch_check_finite(Xd, N * (int64_t)D, bad.as<int32_t>(), s), "check_finite");
        int32_t h = 0;
        download(&h, bad.p, sizeof(h), s);
        if (h) throw Fail(MRQ_EINVAL, "X contains NaN or Inf");
    }

    // PCA: FP64 mean and covariance on the device, eigendecomposition on the host
    DevTemp mu64(sizeof(double) * D);
    {
        const int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(1024, N / 4096));
        DevTemp part(sizeof(double) * nchunk * D);
        hip_check(launch_colmean(Xd, N, D, part.as<double>(), nchunk, mu64.as<double>(), s), "mean");
    }
    std::vector<double> Sh((size_t)D * D), muh(D);
    {
        const int nsplit = cov_splits(N, D);
        DevTemp part(sizeof(double) * (size_t)nsplit * D * D), S(sizeof(double) * (size_t)D * D);
        hip_check(launch_cov(Xd, N, D, mu64.as<double>(), part.as<double>(), nsplit, S.as<double>(), s), "cov");
        download(Sh.data(), S.p, Sh.size() * sizeof(double), s);
        download(muh.data(), mu64.p, muh.size() * sizeof(double), s);
    }
    std::vector<double> lam(D), V((size_t)D * D);
    eigh_host(Sh.data(), D, lam.data(), V.data());
    for (double& l : lam) l = l > 0.0 ? l : 0.0;  // variances (Eq 6): round-off below zero is 0
    ix->lam64 = lam;
    if (d == 0) d = mrq_choose_dr(lam.data(), D);  // Eq 8
    ix->d = d;
    ix->W = (d + 31) / 32;
    ix->WP = padded_words(d);
    ix->d4 = (d + 3) & ~3;
    set_split(*ix);
    const int d4 = ix->d4;
    {
        std::vector<float> Pp32(V.begin(), V.end()), mu32(muh.begin(), muh.end());
        std::vector<float> lt(std::max(D - d, 1), 0.f);
        for (int i = d; i < D; i++) lt[i - d] = (float)lam[i];
        ix->Pp = dalloc<float>(ix.get(), (int64_t)D * D);
        ix->mu = dalloc<float>(ix.get(), D);
        ix->lamTail = dalloc<float>(ix.get(), std::max(D - d, 1));
        upload(ix->Pp, Pp32.data(), Pp32.size() * 4, s);
        upload(ix->mu, mu32.data(), mu32.size() * 4, s);
        upload(ix->lamTail, lt.data(), lt.size() * 4, s);
        ix->PpLead = ix->Pp;
        ix->PpTail = D > d ? ix->Pp + (size_t)d * D : nullptr;
    }

    // x_d = P_p[:d] (x - mu) by id, and the FP64 norms
    DevTemp xd_id(sizeof(float) * (size_t)N * d4), xt_id(sizeof(float) * (size_t)N * std::max(D - d, 1));
    hip_check(launch_fill_f32(xd_id.as<float>(), 0.f, N * (int64_t)d4, s), "fill");
    hip_check(launch_project(Xd, N, D, ix->mu, ix->Pp, d, xd_id.as<float>(), d4, xt_id.as<float>(), D - d, s),
              "project data");
    DevTemp ax64(sizeof(double) * N), tx64(sizeof(double) * N);
    hip_check(launch_rownorms(Xd, N, D, mu64.as<double>(), xd_id.as<float>(), d4, d, ax64.as<double>(),
                              tx64.as<double>(), s), "row norms");

    // k-means on x_d
    ix->C = dalloc<float>(ix.get(), (int64_t)nlist * d4);
    ix->Cn2 = dalloc<float>(ix.get(), nlist);
    hip_check(launch_fill_f32(ix->C, 0.f, (int64_t)nlist * d4, s), "fill");
    {
        std::unordered_map<int64_t, int64_t> swp;
        std::vector<int32_t> pick(nlist);
        uint64_t st = o.seed ^ 0x4B4D45414E53ULL;
        for (int j = 0; j < nlist; j++) {  // partial Fisher-Yates over [0, N)
            const int64_t r = j + (int64_t)(splitmix(st) % (uint64_t)(N - j));
            auto get = [&](int64_t i) { auto it = swp.find(i); return it == swp.end() ? i : it->second; };
            const int64_t vr = get(r), vj = get(j);
            swp[r] = vj;
            swp[j] = vr;
            pick[j] = (int32_t)vr;
        }
        DevTemp pk(sizeof(int32_t) * nlist);
        upload(pk.p, pick.data(), pick.size() * 4, s);
        hip_check(launch_gather_rows(xd_id.as<float>(), d4, pk.as<int32_t>(), nlist, d, ix->C, d4, s), "init");
        hip_check(launch_sqnorms(ix->C, nlist, d4, d, ix->Cn2, s), "cn2");
    }
    DevTemp asgA(sizeof(int32_t) * N), asgB(sizeof(int32_t) * N), mind(sizeof(float) * N), pn2(sizeof(float) * N);
    DevTemp sums(sizeof(double) * (size_t)nlist * d), cnt(sizeof(int32_t) * nlist), changed(sizeof(int32_t));
    hip_check(launch_sqnorms(xd_id.as<float>(), N, d4, d, pn2.as<float>(), s), "pn2");
    int32_t* prev = nullptr;
    int32_t* fin = nullptr;
    std::vector<int32_t> cnt_h(nlist);
    for (int it = 0; it < std::max(1, o.kmeans_iters); it++) {
        int32_t* cur = (it % 2 == 0) ? asgA.as<int32_t>() : asgB.as<int32_t>();
        hip_check(launch_kmeans_assign(xd_id.as<float>(), N, d4, d, ix->C, d4, ix->Cn2, nlist, pn2.as<float>(), cur,
                                       mind.as<float>(), s), "assign");
        hip_check(launch_fill_i32(sums.as<int32_t>(), 0, (int64_t)nlist * d * 2, s), "fill");
        hip_check(launch_fill_i32(cnt.as<int32_t>(), 0, nlist, s), "fill");
        hip_check(launch_fill_i32(changed.as<int32_t>(), 0, 1, s), "fill");
        hip_check(launch_kmeans_accum(xd_id.as<float>(), N, d4, d, cur, prev, sums.as<double>(), cnt.as<int32_t>(),
                                      changed.as<int32_t>(), s), "accumulate");
        int32_t ch = 0;
        download(&ch, changed.p, sizeof(ch), s);
        if (prev && ch == 0) { fin = cur; break; }
        download(cnt_h.data(), cnt.p, cnt_h.size() * 4, s);
        hip_check(launch_kmeans_centroids(sums.as<double>(), cnt.as<int32_t>(), nlist, d, ix->C, d4, ix->Cn2, s),
                  "centroids");
        bool empty = false;
        for (int j = 0; j < nlist; j++) empty |= cnt_h[j] == 0;
        if (empty) {  // an empty cluster takes the farthest point of the largest cluster
            std::vector<int32_t> a_h(N);
            std::vector<float> m_h(N);
            download(a_h.data(), cur, a_h.size() * 4, s);
            download(m_h.data(), mind.p, m_h.size() * 4, s);
            for (int j = 0; j < nlist; j++) {
                if (cnt_h[j] != 0) continue;
                int big = 0;
                for (int t = 1; t < nlist; t++) if (cnt_h[t] > cnt_h[big]) big = t;
                int64_t far = -1;
                float fd = -1.f;
                for (int64_t i = 0; i < N; i++)
                    if (a_h[i] == big && m_h[i] > fd) { fd = m_h[i]; far = i; }
                if (far < 0) continue;
                a_h[far] = j;
                cnt_h[big]--;
                cnt_h[j] = 1;
                hip_check(hipMemcpyAsync(ix->C + (size_t)j * d4, xd_id.as<float>() + (size_t)far * d4, sizeof(float) * d,
                                         hipMemcpyDeviceToDevice, s), "copy centroid");
            }
            hip_check(launch_sqnorms(ix->C, nlist, d4, d, ix->Cn2, s), "cn2");
        }
        prev = cur;
    }
    if (!fin) {
        fin = (prev == asgA.as<int32_t>()) ? asgB.as<int32_t>() : asgA.as<int32_t>();
        hip_check(launch_kmeans_assign(xd_id.as<float>(), N, d4, d, ix->C, d4, ix->Cn2, nlist, pn2.as<float>(), fin,
                                       mind.as<float>(), s), "final assign");
    }
    std::vector<int32_t> assign(N);
    download(assign.data(), fin, assign.size() * 4, s);
    asgA.release(); asgB.release(); mind.release(); pn2.release(); sums.release();

    // list-major layout: each list padded to a multiple of 64 rows, ids ascending inside a list
    std::vector<int64_t> count(nlist, 0);
    for (int64_t i = 0; i < N; i++) count[assign[i]]++;
    ix->h_off_real.assign(nlist + 1, 0);
    ix->h_list_off.assign(nlist + 1, 0);
    std::vector<int32_t> len(nlist), nb(nlist);
    for (int j = 0; j < nlist; j++) {
        len[j] = (int32_t)count[j];
        nb[j] = (int32_t)((count[j] + 63) / 64);
        ix->h_off_real[j + 1] = ix->h_off_real[j] + count[j];
        ix->h_list_off[j + 1] = ix->h_list_off[j] + (int64_t)nb[j] * 64;
        ix->max_list_len = std::max(ix->max_list_len, len[j]);
    }
    ix->Npad = ix->h_list_off[nlist];
    const int64_t Np = ix->Npad;
    std::vector<int32_t> perm(Np, -1);
    {
        std::vector<int64_t> fill(ix->h_list_off.begin(), ix->h_list_off.end() - 1);
        for (int64_t i = 0; i < N; i++) perm[fill[assign[i]]++] = (int32_t)i;
    }
    ix->list_off = dalloc<int64_t>(ix.get(), nlist + 1);
    ix->list_len = dalloc<int32_t>(ix.get(), nlist);
    ix->list_nb = dalloc<int32_t>(ix.get(), nlist);
    upload(ix->list_off, ix->h_list_off.data(), (nlist + 1) * 8, s);
    upload(ix->list_len, len.data(), nlist * 4, s);
    upload(ix->list_nb, nb.data(), nlist * 4, s);
    DevTemp permd(sizeof(int32_t) * Np);
    upload(permd.p, perm.data(), perm.size() * 4, s);

    const int WP = ix->WP;
    ix->ids = dalloc<int32_t>(ix.get(), Np);
    ix->code = dalloc<uint32_t>(ix.get(), Np * WP);
    ix->ext = dalloc<uint32_t>(ix.get(), B > 1 ? Np * (B - 1) * WP : 1);
    ix->fA = dalloc<float>(ix.get(), Np);
    ix->fF = dalloc<float>(ix.get(), Np);
    ix->fE = dalloc<float>(ix.get(), Np);
    ix->fFB = dalloc<float>(ix.get(), Np);
    ix->fEB = dalloc<float>(ix.get(), Np);
    ix->fSX = dalloc<float>(ix.get(), Np);
    ix->xd = dalloc<float>(ix.get(), Np * d4);
    ix->ax = dalloc<float>(ix.get(), Np);
    ix->X = dalloc<float>(ix.get(), Np * ix->D4);
    if (ix->split && ix->Dr4 > 0) ix->xr = dalloc<float>(ix.get(), Np * ix->Dr4);
    ix->nx = dalloc<float>(ix.get(), Np);
    ix->tx = dalloc<float>(ix.get(), Np);
    ix->xi1 = dalloc<float>(ix.get(), Np);
    ix->xiB = dalloc<float>(ix.get(), Np);
    ix->yn = dalloc<float>(ix.get(), Np);
    DevTemp O(sizeof(float) * Np * d4), Xpp(sizeof(float) * Np * d4), txr(sizeof(double) * Np),
        rowl(sizeof(int32_t) * Np);
    hip_check(launch_gather_layout(*ix, Xd, permd.as<int32_t>(), xd_id.as<float>(), ax64.as<double>(),
                                   tx64.as<double>(), txr.as<double>(), rowl.as<int32_t>(), O.as<float>(),
                                   xt_id.as<float>(), s),
              "layout");

    // random rotation P_r and the codes
    {
        std::vector<double> Pr = haar_rotation(d, o.seed ^ 0x524F54415445ULL);
        std::vector<float> PrT((size_t)d4 * d4, 0.f);
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) PrT[(size_t)j * d4 + i] = (float)Pr[(size_t)i * d + j];
        ix->PrT = dalloc<float>(ix.get(), (int64_t)d4 * d4);
        upload(ix->PrT, PrT.data(), PrT.size() * 4, s);
    }
    hip_check(launch_fill_f32(Xpp.as<float>(), 0.f, Np * d4, s), "fill");
    hip_check(launch_gemm_nt(O.as<float>(), d4, nullptr, ix->PrT, d4, Xpp.as<float>(), d4, Np, d, d, s), "rotate");
    ix->RC = dalloc<float>(ix.get(), (int64_t)nlist * d4);
    hip_check(launch_fill_f32(ix->RC, 0.f, (int64_t)nlist * d4, s), "fill");
    hip_check(launch_gemm_nt(ix->C, d4, nullptr, ix->PrT, d4, ix->RC, d4, nlist, d, d, s), "rotate centroids");
    hip_check(launch_encode(*ix, O.as<float>(), Xpp.as<float>(), txr.as<double>(), s), "encode");
    if (o.sq8) {  // MR-SQ codes of the leading coordinates (Appendix A.2, Exp-5)
        ix->dq = (d + 15) & ~15;
        ix->sq_lo = dalloc<float>(ix.get(), ix->dq);
        ix->sq_delta = dalloc<float>(ix.get(), ix->dq);
        ix->sq_code = dalloc<uint8_t>(ix.get(), Np * ix->dq);
        ix->sq_A = dalloc<float>(ix.get(), Np);
        const int nchunk = 256;
        DevTemp part(sizeof(float) * 2 * nchunk * (size_t)d);
        hip_check(launch_sq8_build(*ix, txr.as<double>(), part.as<float>(), nchunk, s), "MR-SQ codes");
    }
    hip_check(hipStreamSynchronize(s), "build sync");
    hip_check(hipEventCreateWithFlags(&ix->ws_event, hipEventDisableTiming), "event");
    return ix.release();
}

// ---- search (Algorithm 2) ---------------------------------------------------------------------

namespace {

struct Carve2 {
    char* base;
    size_t used = 0;
    template <class T>
    T* take(int64_t n) {
        size_t b = ((size_t)(n > 0 ? n : 1) * sizeof(T) + 255) & ~(size_t)255;
        T* r = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += b;
        return r;
    }
};

void resolve_opts(const mrq_search_opts* in, mrq_search_opts* o) {
    mrq_search_opts_default(o);
    if (!in) return;
    *o = *in;
    if (o->bq == 0) o->bq = 4;
    if (!(o->eps0 > 0.f)) o->eps0 = 1.9f;
    if (!(o->m > 0.f)) o->m = 3.f;
}

mrq_status run_search(const mrq_index* cix, const float* Q, int64_t nq, bool uniform_kq, int32_t k_u, int32_t np_u,
                      const int32_t* k_arr, const int32_t* np_arr, const int64_t* out_off_arr, int64_t* ids,
                      float* dists, const mrq_search_opts* opts_in, hipStream_t s, void* fixed_ws = nullptr,
                      size_t fixed_bytes = 0, const TraceSink* trace = nullptr, int32_t dev_kb = 0, int32_t dev_npb = 0,
                      int32_t* rejected = nullptr) {
    // dev_kb > 0: a mixed batch whose k / nprobe / out_off are device arrays, bounded by dev_kb / dev_npb (checked
    // and prefix-summed on the device: no host synchronisation, so the call may be captured)
    const bool dev_mixed = !uniform_kq && dev_kb > 0;
    mrq_index* ix = const_cast<mrq_index*>(cix);
    const bool fixed = fixed_ws != nullptr;  // the allocation-free search: caller buffers plus a fixed workspace
    if (!ix) throw Fail(MRQ_EINVAL, "index is NULL");
    if (!Q || !ids || !dists) throw Fail(MRQ_EINVAL, "Q, ids and dists must not be NULL");
    if (nq < 1 || nq > (int64_t)1 << 28) throw Fail(MRQ_EINVAL, "nq must be in [1, 2^28]");
    mrq_search_opts o;
    resolve_opts(opts_in, &o);
    if (o.bq < 1 || o.bq > 8) throw Fail(MRQ_EINVAL, "bq must be in [1, 8]");
    if (o.mode != MRQ_BATCHED && o.mode != MRQ_PER_QUERY) throw Fail(MRQ_EINVAL, "unknown mode");
    if (o.group < 0 || o.group > 64) throw Fail(MRQ_EINVAL, "group must be in [0, 64]");
    if (o.exact_cap < 0) throw Fail(MRQ_EINVAL, "exact_cap must be >= 0");
    if (o.method != MRQ_METHOD_MRQ && o.method != MRQ_METHOD_MRSQ) throw Fail(MRQ_EINVAL, "unknown method");
    if (phase_shift_of(o.phase_growth, 1) < 0)
        throw Fail(MRQ_EINVAL, "phase_growth must be 0 or a power of two in [2, 1024]");
    if (o.ncounters != 0 && o.ncounters != 8 && o.ncounters != 16) throw Fail(MRQ_EINVAL, "ncounters must be 0, 8 or 16");
    const int ncnt = o.ncounters == 16 ? 16 : 8;
    const int rerank = o.rerank == 0 ? 500 : o.rerank;
    if (o.method == MRQ_METHOD_MRSQ) {
        if (ix->dq == 0) throw Fail(MRQ_ESTATE, "the index has no MR-SQ codes (build it with sq8 = 1)");
        if (rerank < 1 || rerank > 16384) throw Fail(MRQ_EINVAL, "rerank must be in [k, 16384]");
    }
    const int np_cap = std::min(ix->nlist, kMaxProbe);
    // Stream capture (a HIP graph of the search): only device-side work may be recorded, so a captured
    // search takes device buffers, a uniform k / nprobe, no kernel timing, and the workspace sized by an
    // earlier search of the same shape; it is not ordered against other searches on the index.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(s, &cap), "capture status");
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (capturing) {
        if (!uniform_kq && !dev_mixed)
            throw Fail(MRQ_ESTATE, "a search with per-query k / nprobe on the host cannot be captured");
        if (!is_device_ptr(Q) || !is_device_ptr(ids) || !is_device_ptr(dists) ||
            (o.counters && !is_device_ptr(o.counters)))
            throw Fail(MRQ_ESTATE, "a captured search needs device Q, ids, dists and counters");
        if (ix->timer.on) throw Fail(MRQ_ESTATE, "turn kernel timing off before capturing a search");
    }

    // per-query k / nprobe on the host (mixed batches)
    std::vector<int32_t> kh, nph;
    std::vector<int64_t> offh;
    int32_t k_max = k_u, np_max = np_u;
    int64_t total_slots = 0, total_pairs = 0, out_total = 0;
    if (dev_mixed) {
        if (!k_arr || !np_arr) throw Fail(MRQ_EINVAL, "k and nprobe must not be NULL");
        if (!is_device_ptr(k_arr) || !is_device_ptr(np_arr) || (out_off_arr && !is_device_ptr(out_off_arr)) ||
            (rejected && !is_device_ptr(rejected)))
            throw Fail(MRQ_EINVAL, "k, nprobe, out_off and rejected must be device arrays");
        if (dev_kb < 1 || dev_kb > kMaxK) throw Fail(MRQ_EINVAL, "k_max must be in [1, 1024]");
        if (dev_npb < 1 || dev_npb > np_cap) throw Fail(MRQ_EINVAL, "nprobe_max must be in [1, min(nlist, 1024)]");
        if (o.mode != MRQ_BATCHED || o.method != MRQ_METHOD_MRQ)
            throw Fail(MRQ_EINVAL, "a device-side mixed batch runs the batched MRQ method");
        k_max = dev_kb;
        np_max = dev_npb;
        total_slots = nq * dev_kb;  // upper bounds: the kernels read the actual totals from the device offsets
        total_pairs = nq * dev_npb;
        out_total = 0;
    } else if (uniform_kq) {
        if (k_u < 1 || k_u > kMaxK) throw Fail(MRQ_EINVAL, "k must be in [1, 1024]");
        if (np_u < 1 || np_u > np_cap) throw Fail(MRQ_EINVAL, "nprobe must be in [1, min(nlist, 1024)]");
        if (o.method == MRQ_METHOD_MRSQ && k_u > rerank) throw Fail(MRQ_EINVAL, "rerank must be in [k, 16384]");
        total_slots = nq * k_u;
        total_pairs = nq * np_u;
        out_total = nq * k_u;
    } else {
        if (!k_arr || !np_arr || !out_off_arr) throw Fail(MRQ_EINVAL, "k, nprobe and out_off must not be NULL");
        kh.resize(nq);
        nph.resize(nq);
        offh.resize(nq);
        auto fetch = [&](void* dst, const void* src, size_t b) {
            if (is_device_ptr(src)) download(dst, src, b, s);
            else std::memcpy(dst, src, b);
        };
        fetch(kh.data(), k_arr, nq * 4);
        fetch(nph.data(), np_arr, nq * 4);
        fetch(offh.data(), out_off_arr, nq * 8);
        k_max = 0;
        np_max = 0;
        for (int64_t i = 0; i < nq; i++) {
            if (kh[i] < 1 || kh[i] > kMaxK) throw Fail(MRQ_EINVAL, "k[i] must be in [1, 1024]");
            if (o.method == MRQ_METHOD_MRSQ && kh[i] > rerank) throw Fail(MRQ_EINVAL, "rerank must be in [k, 16384]");
            if (nph[i] < 1 || nph[i] > np_cap) throw Fail(MRQ_EINVAL, "nprobe[i] must be in [1, min(nlist, 1024)]");
            if (offh[i] < 0) throw Fail(MRQ_EINVAL, "out_off[i] must be >= 0");
            k_max = std::max(k_max, kh[i]);
            np_max = std::max(np_max, nph[i]);
            total_slots += kh[i];
            total_pairs += nph[i];
            out_total = std::max<int64_t>(out_total, offh[i] + kh[i]);
        }
    }
    const bool per_query = o.mode == MRQ_PER_QUERY;
    const int64_t nq_run = per_query ? 1 : nq;
    const int64_t slots_run = per_query ? k_max : total_slots;
    const int64_t pairs_run = per_query ? np_max : total_pairs;
    const bool q_dev = is_device_ptr(Q), ids_dev = is_device_ptr(ids), d_dev = is_device_ptr(dists);
    const bool cnt_host = o.counters && !is_device_ptr(o.counters);
    if (dev_mixed && (!q_dev || !ids_dev || !d_dev || cnt_host))
        throw Fail(MRQ_EINVAL, "a device-side mixed batch takes device Q, ids, dists and counters");
    if (fixed && (!uniform_kq || !q_dev || !ids_dev || !d_dev || cnt_host))
        throw Fail(MRQ_EINVAL, "the allocation-free search takes device Q, ids, dists and counters and a uniform k / nprobe");

    // workspace: metadata, staging copies, then the search scratch
    auto layout = [&](char* base, size_t* used, int32_t** kq, int32_t** npq, int64_t** so, int64_t** po, int64_t** oo,
                      float** qs, int64_t** ids_s, float** d_s, int64_t** cnt_s, void** sw) {
        Carve2 c{base};
        *kq = c.take<int32_t>(nq);
        *npq = c.take<int32_t>(nq);
        *so = c.take<int64_t>(nq + 1);
        *po = c.take<int64_t>(nq + 1);
        *oo = c.take<int64_t>(nq);
        *qs = q_dev ? nullptr : c.take<float>(nq * ix->D);
        *ids_s = ids_dev ? nullptr : c.take<int64_t>(out_total);
        *d_s = d_dev ? nullptr : c.take<float>(out_total);
        *cnt_s = cnt_host ? c.take<int64_t>(ncnt) : nullptr;
        *sw = base ? base + c.used : nullptr;
        *used = c.used + search_workspace_bytes(*ix, nq_run, slots_run, pairs_run, o.bq, np_max, o.method, rerank);
    };
    int32_t *kq, *npq;
    int64_t *so, *po, *oo, *ids_s, *cnt_s;
    float *qs, *d_s;
    void* sw;
    size_t need = 0;
    layout(nullptr, &need, &kq, &npq, &so, &po, &oo, &qs, &ids_s, &d_s, &cnt_s, &sw);
    if (fixed) {
        if (need > fixed_bytes)
            throw Fail(MRQ_EINVAL, "this search needs " + std::to_string(need) + " bytes of workspace; the allocation-free "
                       "search has " + std::to_string(fixed_bytes) + " (split the batch, or use mrq_search)");
        layout(reinterpret_cast<char*>(fixed_ws), &need, &kq, &npq, &so, &po, &oo, &qs, &ids_s, &d_s, &cnt_s, &sw);
    }
    std::unique_lock<std::mutex> lock(ix->mu_ws, std::defer_lock);
    if (!fixed) lock.lock();
    if (fixed) {
        // nothing of the index's own workspace is touched: no growth, no ordering event
    } else {
    if (capturing && ix->ws.bytes < need)
        throw Fail(MRQ_ESTATE, "run the same search once before capturing it (its workspace cannot grow during capture)");
    if (ix->ws_event_recorded && !capturing) hip_check(hipStreamWaitEvent(s, ix->ws_event, 0), "order workspace");
    if (ix->ws.bytes < need) {
        if (ix->ws.base) {
            hip_check(hipDeviceSynchronize(), "sync before workspace growth");
            if (ix->ws.captured) ix->ws.retired.push_back(ix->ws.base);  // graphs may still replay on it
            else (void)hipFree(ix->ws.base);
            ix->ws.base = nullptr;
            ix->ws.bytes = 0;
            ix->ws.captured = false;
        }
        size_t grow = need + need / 4;
        hip_check(hipMalloc(&ix->ws.base, grow), "hipMalloc (search workspace)");
        ix->ws.bytes = grow;
    }
    layout(reinterpret_cast<char*>(ix->ws.base), &need, &kq, &npq, &so, &po, &oo, &qs, &ids_s, &d_s, &cnt_s, &sw);
    }
    char* const ws_base = fixed ? reinterpret_cast<char*>(fixed_ws) : reinterpret_cast<char*>(ix->ws.base);
    const size_t ws_total = fixed ? fixed_bytes : ix->ws.bytes;
    const size_t sw_bytes = ws_total - (size_t)(reinterpret_cast<char*>(sw) - ws_base);

    const float* Qd = Q;
    if (!q_dev) {
        hip_check(hipMemcpyAsync(qs, Q, sizeof(float) * nq * ix->D, hipMemcpyHostToDevice, s), "copy Q");
        Qd = qs;
    }
    int64_t* ids_d = ids_dev ? ids : ids_s;
    float* dd = d_dev ? dists : d_s;
    int64_t* cnt_d = o.counters ? (cnt_host ? cnt_s : o.counters) : nullptr;
    if (cnt_host) hip_check(launch_fill_i32(reinterpret_cast<int32_t*>(cnt_s), 0, 2 * ncnt, s), "fill");
    if (dev_mixed) {
        hip_check(launch_mixed_meta(nq, k_arr, np_arr, out_off_arr, dev_kb, dev_npb, kq, npq, so, po, oo, rejected, s),
                  "meta");
    } else if (!uniform_kq) {
        std::vector<int64_t> so_h(nq + 1, 0), po_h(nq + 1, 0);
        for (int64_t i = 0; i < nq; i++) {
            so_h[i + 1] = so_h[i] + kh[i];
            po_h[i + 1] = po_h[i] + nph[i];
        }
        hip_check(hipMemcpyAsync(kq, kh.data(), nq * 4, hipMemcpyHostToDevice, s), "meta");
        hip_check(hipMemcpyAsync(npq, nph.data(), nq * 4, hipMemcpyHostToDevice, s), "meta");
        hip_check(hipMemcpyAsync(so, so_h.data(), (nq + 1) * 8, hipMemcpyHostToDevice, s), "meta");
        hip_check(hipMemcpyAsync(po, po_h.data(), (nq + 1) * 8, hipMemcpyHostToDevice, s), "meta");
        hip_check(hipMemcpyAsync(oo, offh.data(), nq * 8, hipMemcpyHostToDevice, s), "meta");
        hip_check(hipStreamSynchronize(s), "meta sync");
    }

    SearchArgs a;
    a.ix = ix;
    a.bq = o.bq;
    a.eps0 = o.eps0;
    a.m = o.m;
    a.stage2 = o.stage2;
    a.use_ext = o.use_ext;
    a.group = o.group > 0 ? o.group : ix->group_default;
    a.exact_cap = o.exact_cap;
    a.method = o.method;
    a.rerank = rerank;
    a.phase_shift = phase_shift_of(o.phase_growth, ix->phase_shift_default);
    a.counters = cnt_d;
    a.ncounters = ncnt;
    a.trace = trace;
    if (trace && (per_query || o.method != MRQ_METHOD_MRQ))
        throw Fail(MRQ_EINVAL, "a traced search runs the batched MRQ method");
    if (fixed) {
        a.timed = false;      // timing events would be created on demand
        a.fork_seed = false;  // no auxiliary stream or events to create
    }
    if (!per_query) {
        if (uniform_kq) hip_check(launch_uniform_meta(nq, k_u, np_u, kq, npq, so, po, oo, s), "meta");
        a.Q = Qd;
        a.nq = nq;
        a.kq = kq;
        a.npq = npq;
        a.slot_off = so;
        a.pair_off = po;
        a.out_off = oo;
        a.total_slots = total_slots;
        a.total_pairs = total_pairs;
        a.np_max = np_max;
        a.k_max = k_max;
        a.ids = ids_d;
        a.dists = dd;
        hip_check(launch_search(a, sw, sw_bytes, s), "search");
    } else {
        // the plain per-query path: the same pipeline, one query per pass
        for (int64_t i = 0; i < nq; i++) {
            const int32_t ki = uniform_kq ? k_u : kh[i];
            const int32_t npi = uniform_kq ? np_u : nph[i];
            const int64_t oi = uniform_kq ? i * k_u : offh[i];
            hip_check(launch_uniform_meta(1, ki, npi, kq, npq, so, po, oo, s), "meta");
            a.Q = Qd + i * ix->D;
            a.nq = 1;
            a.kq = kq;
            a.npq = npq;
            a.slot_off = so;
            a.pair_off = po;
            a.out_off = oo;
            a.total_slots = ki;
            a.total_pairs = npi;
            a.np_max = npi;
            a.k_max = ki;
            a.ids = ids_d + oi;
            a.dists = dd + oi;
            hip_check(launch_search(a, sw, sw_bytes, s), "search");
        }
    }
    if (fixed) {
        // the fixed buffer is not the index's workspace
    } else if (!capturing) {
        hip_check(hipEventRecord(ix->ws_event, s), "record");
        ix->ws_event_recorded = true;
    } else {
        ix->ws.captured = true;
    }
    if (!ids_dev || !d_dev || cnt_host) {
        if (!ids_dev) hip_check(hipMemcpyAsync(ids, ids_s, out_total * 8, hipMemcpyDeviceToHost, s), "copy ids");
        if (!d_dev) hip_check(hipMemcpyAsync(dists, d_s, out_total * 4, hipMemcpyDeviceToHost, s), "copy dists");
        int64_t ch[16] = {0};
        if (cnt_host)
            hip_check(hipMemcpyAsync(ch, cnt_s, sizeof(int64_t) * ncnt, hipMemcpyDeviceToHost, s), "copy counters");
        hip_check(hipStreamSynchronize(s), "search sync");
        if (cnt_host)
            for (int i = 0; i < ncnt; i++) o.counters[i] += ch[i];
    }
    return MRQ_OK;
}

// ---- persistence ------------------------------------------------------------------------------

struct ArrayRef {
    void** p;
    size_t bytes;
};

std::vector<ArrayRef> device_arrays(Index& ix) {
    const int64_t Np = ix.Npad, d4 = ix.d4, D = ix.D, L = ix.nlist;
    const int B = ix.B, WP = ix.WP;
    return {
        {(void**)&ix.mu, sizeof(float) * D},
        {(void**)&ix.Pp, sizeof(float) * D * D},
        {(void**)&ix.lamTail, sizeof(float) * std::max<int64_t>(D - ix.d, 1)},
        {(void**)&ix.PrT, sizeof(float) * d4 * d4},
        {(void**)&ix.C, sizeof(float) * L * d4},
        {(void**)&ix.Cn2, sizeof(float) * L},
        {(void**)&ix.RC, sizeof(float) * L * d4},
        {(void**)&ix.list_off, sizeof(int64_t) * (L + 1)},
        {(void**)&ix.list_len, sizeof(int32_t) * L},
        {(void**)&ix.list_nb, sizeof(int32_t) * L},
        {(void**)&ix.ids, sizeof(int32_t) * Np},
        {(void**)&ix.code, sizeof(uint32_t) * Np * WP},
        {(void**)&ix.ext, sizeof(uint32_t) * (B > 1 ? Np * (B - 1) * WP : 1)},
        {(void**)&ix.fA, sizeof(float) * Np},
        {(void**)&ix.fF, sizeof(float) * Np},
        {(void**)&ix.fE, sizeof(float) * Np},
        {(void**)&ix.fFB, sizeof(float) * Np},
        {(void**)&ix.fEB, sizeof(float) * Np},
        {(void**)&ix.fSX, sizeof(float) * Np},
        {(void**)&ix.xd, sizeof(float) * Np * d4},
        {(void**)&ix.ax, sizeof(float) * Np},
        {(void**)&ix.X, sizeof(float) * Np * ix.D4},
        {(void**)&ix.xr, ix.split && ix.Dr4 > 0 ? sizeof(float) * Np * ix.Dr4 : 0},
        {(void**)&ix.nx, sizeof(float) * Np},
        {(void**)&ix.tx, sizeof(float) * Np},
        {(void**)&ix.xi1, sizeof(float) * Np},
        {(void**)&ix.xiB, sizeof(float) * Np},
        {(void**)&ix.yn, sizeof(float) * Np},
    };
}

std::vector<ArrayRef> sq8_arrays(Index& ix) {
    if (ix.dq == 0) return {};
    return {
        {(void**)&ix.sq_lo, sizeof(float) * ix.dq},
        {(void**)&ix.sq_delta, sizeof(float) * ix.dq},
        {(void**)&ix.sq_code, (size_t)ix.Npad * ix.dq},
        {(void**)&ix.sq_A, sizeof(float) * ix.Npad},
    };
}

struct File {
    FILE* f;
    explicit File(const char* path, const char* mode) : f(std::fopen(path, mode)) {
        if (!f) throw Fail(MRQ_EIO, std::string("cannot open ") + path);
    }
    ~File() { if (f) std::fclose(f); }
    void w(const void* p, size_t b) { if (b && std::fwrite(p, 1, b, f) != b) throw Fail(MRQ_EIO, "write failed"); }
    void r(void* p, size_t b) { if (b && std::fread(p, 1, b, f) != b) throw Fail(MRQ_EIO, "read failed / truncated file"); }
};

template <class T>
std::vector<T> fetch_dev(const T* p, size_t n) {
    std::vector<T> h(n);
    if (n) hip_check(hipMemcpy(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost), "download");
    return h;
}

}  // namespace

// Export in the oracle-facing layout documented in mrq.h.
static void export_index(const mrq_index* ix, const char* path) {
    const int64_t N = ix->N, Np = ix->Npad;
    const int D = ix->D, d = ix->d, B = ix->B, L = ix->nlist, d4 = ix->d4, WP = ix->WP;
    File f(path, "wb");
    f.w("MRQX0001", 8);
    f.w(&N, 8);
    int32_t hdr[4] = {D, d, B, L};
    f.w(hdr, sizeof(hdr));
    f.w(fetch_dev(ix->mu, D).data(), sizeof(float) * D);
    f.w(fetch_dev(ix->Pp, (size_t)D * D).data(), sizeof(float) * D * D);
    f.w(ix->lam64.data(), sizeof(double) * D);
    {
        auto PrT = fetch_dev(ix->PrT, (size_t)d4 * d4);
        std::vector<float> Pr((size_t)d * d);
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) Pr[(size_t)i * d + j] = PrT[(size_t)j * d4 + i];
        f.w(Pr.data(), Pr.size() * 4);
    }
    {
        auto C = fetch_dev(ix->C, (size_t)L * d4);
        std::vector<float> Cc((size_t)L * d);
        for (int j = 0; j < L; j++) std::memcpy(&Cc[(size_t)j * d], &C[(size_t)j * d4], sizeof(float) * d);
        f.w(Cc.data(), Cc.size() * 4);
    }
    f.w(ix->h_off_real.data(), sizeof(int64_t) * (L + 1));
    auto ids = fetch_dev(ix->ids, Np);
    std::vector<int64_t> rows;
    rows.reserve(N);
    for (int64_t r = 0; r < Np; r++)
        if (ids[r] >= 0) rows.push_back(r);
    std::vector<int64_t> id64(N);
    for (int64_t i = 0; i < N; i++) id64[i] = ids[rows[i]];
    f.w(id64.data(), 8 * N);
    {
        auto code = fetch_dev(ix->code, (size_t)Np * WP);
        std::vector<uint32_t> ext;
        if (B > 1) ext = fetch_dev(ix->ext, (size_t)Np * (B - 1) * WP);
        std::vector<uint8_t> u((size_t)N * d);
        for (int64_t i = 0; i < N; i++) {
            const int64_t r = rows[i];
            for (int t = 0; t < d; t++) {
                const int w = t >> 5, b = t & 31;
                uint32_t v = ((code[r * WP + w] >> b) & 1u) << (B - 1);
                for (int a = 0; a < B - 1; a++) v |= ((ext[(r * (B - 1) + a) * WP + w] >> b) & 1u) << a;
                u[(size_t)i * d + t] = (uint8_t)v;
            }
        }
        f.w(u.data(), u.size());
    }
    {
        auto xd = fetch_dev(ix->xd, (size_t)Np * d4);
        std::vector<float> o((size_t)N * d);
        for (int64_t i = 0; i < N; i++) std::memcpy(&o[(size_t)i * d], &xd[(size_t)rows[i] * d4], sizeof(float) * d);
        f.w(o.data(), o.size() * 4);
    }
    for (const float* arr : {ix->nx, ix->tx, ix->ax, ix->xi1, ix->xiB, ix->yn}) {
        auto v = fetch_dev(arr, Np);
        std::vector<float> o(N);
        for (int64_t i = 0; i < N; i++) o[i] = v[rows[i]];
        f.w(o.data(), o.size() * 4);
    }
    if (ix->dq > 0) {  // MR-SQ: grid and codes in natural dimension order
        const int dq = ix->dq;
        f.w("SQ8G", 4);
        f.w(fetch_dev(ix->sq_lo, d).data(), sizeof(float) * d);
        f.w(fetch_dev(ix->sq_delta, d).data(), sizeof(float) * d);
        auto code = fetch_dev(ix->sq_code, (size_t)Np * dq);
        std::vector<uint8_t> u((size_t)N * d);
        for (int64_t i = 0; i < N; i++)
            for (int t = 0; t < d; t++)
                u[(size_t)i * d + t] = code[(size_t)rows[i] * dq + ((t >> 2) & 3) * (dq >> 2) + 4 * (t >> 4) + (t & 3)];
        f.w(u.data(), u.size());
    }
}

}  // namespace mrq

using namespace mrq;

extern "C" {

void mrq_build_opts_default(mrq_build_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->seed = 4001;
    o->kmeans_iters = 25;
}

int32_t mrq_choose_dr(const double* lambda, int32_t D) {
    if (!lambda || D < 2) return -1;
    double tot = 0.0;
    for (int j = 0; j < D; j++) tot += lambda[j];
    for (int dd = 128;; dd *= 2) {
        if (dd >= D) return D <= 1536 ? D : 1024;
        if (dd > 1536) return 1024;
        double part = 0.0;
        for (int j = 0; j < dd; j++) part += lambda[j];
        if (part >= 0.8 * tot) return dd;
    }
}

void mrq_search_opts_default(mrq_search_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = MRQ_BATCHED;
    o->bq = 4;
    o->eps0 = 1.9f;
    o->m = 3.f;
    o->stage2 = 1;
    o->use_ext = 1;
    o->counters = nullptr;
    o->group = 0;
}

mrq_status mrq_build(const float* X, int64_t N, int32_t D, int32_t d_r, int32_t bits, int32_t nlist,
                     const mrq_build_opts* opts, mrq_stream stream, mrq_index** out) {
    return guarded([&]() -> mrq_status {
        if (!out) throw Fail(MRQ_EINVAL, "out is NULL");
        check_args_build(X, N, D, d_r, bits, nlist);
        mrq_build_opts o;
        mrq_build_opts_default(&o);
        if (opts) o = *opts;
        if (o.sq8 != 0 && o.sq8 != 1) throw Fail(MRQ_EINVAL, "sq8 must be 0 or 1");
        *out = build_index(X, N, D, d_r, bits, nlist, o, (hipStream_t)stream);
        return MRQ_OK;
    });
}

mrq_status mrq_search(const mrq_index* index, const float* Q, int64_t nq, int32_t k, int32_t nprobe, int64_t* ids,
                      float* dists, const mrq_search_opts* opts, mrq_stream stream) {
    return guarded([&]() {
        return run_search(index, Q, nq, true, k, nprobe, nullptr, nullptr, nullptr, ids, dists, opts,
                          (hipStream_t)stream);
    });
}

mrq_status mrq_search_noalloc(const mrq_index* index, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                              int64_t* ids, float* dists, const mrq_search_opts* opts, mrq_stream stream) {
    return guarded([&]() {
        void* buf = nullptr;
        size_t bytes = 0;
        hip_check(noalloc_scratch(&buf, &bytes), "fixed search buffer");
        return run_search(index, Q, nq, true, k, nprobe, nullptr, nullptr, nullptr, ids, dists, opts,
                          (hipStream_t)stream, buf, bytes);
    });
}

mrq_status mrq_stream_copy(void* dst, const void* src, size_t bytes, mrq_stream stream) {
    return guarded([&]() {
        if (!dst || !src) throw Fail(MRQ_EINVAL, "dst and src must not be NULL");
        if (bytes % 16 || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
            throw Fail(MRQ_EINVAL, "bytes and both pointers must be multiples of 16");
        if (!is_device_ptr(dst) || !is_device_ptr(src)) throw Fail(MRQ_EINVAL, "device pointers only");
        hip_check(launch_stream_copy(dst, src, bytes, (hipStream_t)stream), "stream copy");
        return MRQ_OK;
    });
}

mrq_status mrq_search_trace(const mrq_index* index, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                            const mrq_search_opts* opts, const int32_t* traced, int32_t ntraced, int64_t* ids,
                            float* dists, mrq_trace_pair* pairs, float* qprime, uint8_t* levels, int64_t max_pairs,
                            int64_t* npairs, mrq_trace_cand* cands, int64_t max_cands, int64_t* ncands) {
    return guarded([&]() {
        if (!index || !Q || !ids || !dists || !npairs || !ncands) throw Fail(MRQ_EINVAL, "NULL argument");
        if (nq < 1 || ntraced < 0 || (ntraced > 0 && !traced) || max_pairs < 0 || max_cands < 0 ||
            (max_pairs > 0 && (!pairs || !qprime || !levels)) || (max_cands > 0 && !cands))
            throw Fail(MRQ_EINVAL, "bad trace buffers");
        if (is_device_ptr(Q) || is_device_ptr(ids) || is_device_ptr(dists))
            throw Fail(MRQ_EINVAL, "a traced search takes host Q, ids and dists");
        std::vector<uint8_t> flag(nq, 0);
        for (int32_t i = 0; i < ntraced; i++) {
            if (traced[i] < 0 || traced[i] >= nq) throw Fail(MRQ_EINVAL, "traced query index out of range");
            flag[traced[i]] = 1;
        }
        const int d = index->d;
        DevTemp dflag(nq), dpairs(sizeof(mrq_trace_pair) * std::max<int64_t>(max_pairs, 1)),
            dqp(sizeof(float) * d * std::max<int64_t>(max_pairs, 1)), du((size_t)d * std::max<int64_t>(max_pairs, 1)),
            dc(sizeof(mrq_trace_cand) * std::max<int64_t>(max_cands, 1)), dn(2 * sizeof(unsigned long long)),
            dsink(sizeof(TraceSink));
        hipStream_t s = nullptr;
        hip_check(hipMemcpy(dflag.p, flag.data(), nq, hipMemcpyHostToDevice), "trace flags");
        hip_check(hipMemset(dn.p, 0, dn.bytes), "trace counts");
        TraceSink sink;
        sink.qflag = dflag.as<uint8_t>();
        sink.pairs = dpairs.as<mrq_trace_pair>();
        sink.qp = dqp.as<float>();
        sink.u = du.as<uint8_t>();
        sink.cands = dc.as<mrq_trace_cand>();
        sink.n = dn.as<unsigned long long>();
        sink.max_pairs = max_pairs;
        sink.max_cands = max_cands;
        hip_check(hipMemcpy(dsink.p, &sink, sizeof(sink), hipMemcpyHostToDevice), "trace sink");
        const mrq_status st = run_search(index, Q, nq, true, k, nprobe, nullptr, nullptr, nullptr, ids, dists, opts, s,
                                         nullptr, 0, dsink.as<TraceSink>());
        if (st != MRQ_OK) return st;
        hip_check(hipDeviceSynchronize(), "trace sync");
        unsigned long long n[2];
        hip_check(hipMemcpy(n, dn.p, sizeof(n), hipMemcpyDeviceToHost), "trace counts");
        *npairs = (int64_t)n[0];
        *ncands = (int64_t)n[1];
        const int64_t wp = std::min<int64_t>((int64_t)n[0], max_pairs), wc = std::min<int64_t>((int64_t)n[1], max_cands);
        if (wp > 0) {
            hip_check(hipMemcpy(pairs, dpairs.p, sizeof(mrq_trace_pair) * wp, hipMemcpyDeviceToHost), "trace pairs");
            hip_check(hipMemcpy(qprime, dqp.p, sizeof(float) * d * wp, hipMemcpyDeviceToHost), "trace q'");
            hip_check(hipMemcpy(levels, du.p, (size_t)d * wp, hipMemcpyDeviceToHost), "trace levels");
        }
        if (wc > 0) hip_check(hipMemcpy(cands, dc.p, sizeof(mrq_trace_cand) * wc, hipMemcpyDeviceToHost), "trace cands");
        return MRQ_OK;
    });
}

mrq_status mrq_tune(mrq_index* index, const float* Q, int64_t nq, int32_t k, int32_t nprobe, mrq_stream stream,
                    int32_t* group, int32_t* phase_growth) {
    return guarded([&]() {
        if (!index || !Q) throw Fail(MRQ_EINVAL, "index and Q must not be NULL");
        if (nq < 1 || k < 1 || k > kMaxK || nprobe < 1) throw Fail(MRQ_EINVAL, "bad nq, k or nprobe");
        hipStream_t s = (hipStream_t)stream;
        DevTemp ids(sizeof(int64_t) * (size_t)nq * k), dd(sizeof(float) * (size_t)nq * k);
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        const int groups[3] = {16, 32, 64}, growths[3] = {2, 4, 8};
        int best_g = index->group_default, best_p = 1 << index->phase_shift_default;
        float best_ms = -1.f;
        mrq_search_opts o;
        mrq_search_opts_default(&o);
        mrq_status st = MRQ_OK;
        for (int pg : growths) {
            for (int g : groups) {
                o.group = g;
                o.phase_growth = pg;
                for (int rep = 0; rep < 2 && st == MRQ_OK; rep++) {  // the first run warms the workspace
                    if (rep == 1) hip_check(hipEventRecord(e0, s), "event");
                    st = run_search(index, Q, nq, true, k, nprobe, nullptr, nullptr, nullptr, ids.as<int64_t>(),
                                    dd.as<float>(), &o, s);
                    if (rep == 1) hip_check(hipEventRecord(e1, s), "event");
                }
                if (st != MRQ_OK) break;
                hip_check(hipEventSynchronize(e1), "event");
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
                if (best_ms < 0.f || ms < best_ms) {
                    best_ms = ms;
                    best_g = g;
                    best_p = pg;
                }
            }
            if (st != MRQ_OK) break;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != MRQ_OK) return st;
        index->group_default = best_g;
        index->phase_shift_default = phase_shift_of(best_p, index->phase_shift_default);
        if (group) *group = best_g;
        if (phase_growth) *phase_growth = best_p;
        return MRQ_OK;
    });
}

mrq_status mrq_search_mixed(const mrq_index* index, const float* Q, int64_t nq, const int32_t* k,
                            const int32_t* nprobe, const int64_t* out_off, int64_t* ids, float* dists,
                            const mrq_search_opts* opts, mrq_stream stream) {
    return guarded([&]() {
        return run_search(index, Q, nq, false, 0, 0, k, nprobe, out_off, ids, dists, opts, (hipStream_t)stream);
    });
}

mrq_status mrq_search_mixed_dev(const mrq_index* index, const float* Q, int64_t nq, const int32_t* k,
                                const int32_t* nprobe, const int64_t* out_off, int32_t k_max, int32_t nprobe_max,
                                int64_t* ids, float* dists, int32_t* rejected, const mrq_search_opts* opts,
                                mrq_stream stream) {
    return guarded([&]() {
        if (k_max < 1) throw Fail(MRQ_EINVAL, "k_max must be in [1, 1024]");
        return run_search(index, Q, nq, false, 0, 0, k, nprobe, out_off, ids, dists, opts, (hipStream_t)stream,
                          nullptr, 0, nullptr, k_max, nprobe_max, rejected);
    });
}

mrq_status mrq_index_info(const mrq_index* ix, int64_t* N, int32_t* D, int32_t* d_r, int32_t* bits, int32_t* nlist,
                          int64_t* device_bytes) {
    if (!ix) return set_err(MRQ_EINVAL, "index is NULL");
    if (N) *N = ix->N;
    if (D) *D = ix->D;
    if (d_r) *d_r = ix->d;
    if (bits) *bits = ix->B;
    if (nlist) *nlist = ix->nlist;
    if (device_bytes) *device_bytes = ix->device_bytes;
    return MRQ_OK;
}

mrq_status mrq_export(const mrq_index* ix, const char* path) {
    return guarded([&]() {
        if (!ix || !path) throw Fail(MRQ_EINVAL, "index and path must not be NULL");
        hip_check(hipDeviceSynchronize(), "sync");
        export_index(ix, path);
        return MRQ_OK;
    });
}

mrq_status mrq_save(const mrq_index* cix, const char* path) {
    return guarded([&]() {
        if (!cix || !path) throw Fail(MRQ_EINVAL, "index and path must not be NULL");
        mrq_index* ix = const_cast<mrq_index*>(cix);
        hip_check(hipDeviceSynchronize(), "sync");
        File f(path, "wb");
        f.w("MRQS0005", 8);
        int64_t h64[2] = {ix->N, ix->Npad};
        int32_t h32[7] = {ix->D, ix->d, ix->B, ix->nlist, ix->WP, ix->max_list_len, ix->dq};
        f.w(h64, sizeof(h64));
        f.w(h32, sizeof(h32));
        f.w(ix->lam64.data(), sizeof(double) * ix->D);
        f.w(ix->h_off_real.data(), sizeof(int64_t) * (ix->nlist + 1));
        f.w(ix->h_list_off.data(), sizeof(int64_t) * (ix->nlist + 1));
        std::vector<ArrayRef> arrays = device_arrays(*ix), sq = sq8_arrays(*ix);
        arrays.insert(arrays.end(), sq.begin(), sq.end());
        for (auto& a : arrays) {
            if (!a.bytes) continue;  // an array this index does not have
            std::vector<char> h(a.bytes);
            hip_check(hipMemcpy(h.data(), *a.p, a.bytes, hipMemcpyDeviceToHost), "download");
            f.w(h.data(), a.bytes);
        }
        return MRQ_OK;
    });
}

mrq_status mrq_load(const char* path, mrq_index** out) {
    return guarded([&]() {
        if (!path || !out) throw Fail(MRQ_EINVAL, "path and out must not be NULL");
        File f(path, "rb");
        char magic[8];
        f.r(magic, 8);
        if (std::memcmp(magic, "MRQS0005", 8) != 0) throw Fail(MRQ_EIO, "not an MRQS0005 file");
        std::unique_ptr<mrq_index> ix(new mrq_index());
        hip_check(hipGetDevice(&ix->device), "hipGetDevice");
        int64_t h64[2];
        int32_t h32[7];
        f.r(h64, sizeof(h64));
        f.r(h32, sizeof(h32));
        ix->N = h64[0];
        ix->Npad = h64[1];
        ix->D = h32[0];
        ix->d = h32[1];
        ix->B = h32[2];
        ix->nlist = h32[3];
        ix->WP = h32[4];
        ix->max_list_len = h32[5];
        ix->dq = h32[6];
        if (ix->N < 1 || ix->D < 2 || ix->d < 2 || ix->d > ix->D || ix->B < 1 || ix->B > 8 || ix->nlist < 1 ||
            ix->WP != padded_words(ix->d) || ix->Npad < ix->N || (ix->dq != 0 && ix->dq != ((ix->d + 15) & ~15)))
            throw Fail(MRQ_EIO, "corrupt header");
        ix->W = (ix->d + 31) / 32;
        ix->d4 = (ix->d + 3) & ~3;
        ix->D4 = (ix->D + 3) & ~3;
        set_split(*ix);
        ix->lam64.resize(ix->D);
        f.r(ix->lam64.data(), sizeof(double) * ix->D);
        ix->h_off_real.resize(ix->nlist + 1);
        ix->h_list_off.resize(ix->nlist + 1);
        f.r(ix->h_off_real.data(), sizeof(int64_t) * (ix->nlist + 1));
        f.r(ix->h_list_off.data(), sizeof(int64_t) * (ix->nlist + 1));
        std::vector<ArrayRef> arrays = device_arrays(*ix), sq = sq8_arrays(*ix);
        arrays.insert(arrays.end(), sq.begin(), sq.end());
        for (auto& a : arrays) {
            if (!a.bytes) continue;
            std::vector<char> h(a.bytes);
            f.r(h.data(), a.bytes);
            void* p = nullptr;
            hip_check(hipMalloc(&p, a.bytes), "hipMalloc (index)");
            ix->allocations.push_back(p);
            ix->device_bytes += (int64_t)a.bytes;
            hip_check(hipMemcpy(p, h.data(), a.bytes, hipMemcpyHostToDevice), "upload");
            *a.p = p;
        }
        ix->PpLead = ix->Pp;
        ix->PpTail = ix->D > ix->d ? ix->Pp + (size_t)ix->d * ix->D : nullptr;
        hip_check(hipEventCreateWithFlags(&ix->ws_event, hipEventDisableTiming), "event");
        *out = ix.release();
        return MRQ_OK;
    });
}

void mrq_free(mrq_index* ix) {
    if (!ix) return;
    if (ix->ws_event_recorded) (void)hipEventSynchronize(ix->ws_event);
    if (ix->ws_event) (void)hipEventDestroy(ix->ws_event);
    delete ix;
}

const char* mrq_last_error(void) { return g_err.c_str(); }

int mrq_timing(const mrq_index* ix, char* names, size_t cap, double* ms, int64_t* launches, int max) {
    if (!ix) return -1;
    ix->timer.collect();
    std::string all;
    const int n = (int)ix->timer.names.size();
    for (int i = 0; i < n; i++) {
        all += ix->timer.names[i];
        all += '\n';
        if (i < max) {
            if (ms) ms[i] = ix->timer.ms[i];
            if (launches) launches[i] = ix->timer.launches[i];
        }
    }
    if (names && cap) {
        std::strncpy(names, all.c_str(), cap - 1);
        names[cap - 1] = 0;
    }
    return n;
}

mrq_status mrq_timing_enable(mrq_index* ix, int on, int reset) {
    if (!ix) return set_err(MRQ_EINVAL, "index is NULL");
    ix->timer.collect();
    ix->timer.on = on != 0;
    if (reset) {
        std::fill(ix->timer.ms.begin(), ix->timer.ms.end(), 0.0);
        std::fill(ix->timer.launches.begin(), ix->timer.launches.end(), 0);
    }
    return MRQ_OK;
}

}  // extern "C"
