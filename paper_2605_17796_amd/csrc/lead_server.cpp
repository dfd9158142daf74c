// Serving loop with continuous batching (lead_server_* in lead.h).
//
// Requests wait in a FIFO per decoder.  A worker thread repeatedly
//   1. retires launch slots whose completion event has fired, copying each
//      request's share of the results out of the slot's pinned buffers;
//   2. fills every idle slot with waiting shots of its decoder (whole
//      requests or parts of them, in arrival order) and enqueues copy-in,
//      decode and copy-out on the slot's stream.
// A request that arrives while all slots are busy is admitted into the next
// slot that frees, so its decode overlaps the launches already on the
// device.  Device memory is admitted slot by slot against the budget: one
// slot per decoder from the start, more while the budget allows, and an
// idle extra slot of a decoder with nothing waiting is freed when another
// decoder's shots wait and the budget is full.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lead.h"
#include "lead_internal.hpp"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    int dec = 0;
    int64_t shots = 0;
    std::vector<uint64_t> synd;      // shots x synd_words (the decoder's width)
    std::vector<float> prior;        // shots
    std::vector<uint64_t> ehat;      // shots x ehat_words
    std::vector<float> post;         // shots x n (only with return_posteriors)
    std::vector<lead_shot_stats> stats;
    int64_t next_shot = 0;           // shots handed to slots so far
    int64_t done_shots = 0;
    int64_t t_submit = 0, t_done = 0;
    bool done = false;
};

struct Part {
    Request *req;
    int64_t req_off, slot_off, count;
};

struct Slot {
    int dec = 0;
    lead_decoder *decoder = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    uint64_t *d_synd = nullptr, *d_ehat = nullptr;
    float *d_prior = nullptr, *d_post = nullptr;
    lead_shot_stats *d_stats = nullptr;
    uint64_t *h_synd = nullptr, *h_ehat = nullptr;
    float *h_prior = nullptr, *h_post = nullptr;
    lead_shot_stats *h_stats = nullptr;
    bool busy = false;
    bool pinned = false;             // the decoder's first slot: never freed early
    int64_t bytes = 0;               // device bytes (decoder copy + buffers)
    std::vector<Part> parts;
};

struct DecShape {
    int n = 0, m = 0, sw = 0, ew = 0;
};

}  // namespace

struct lead_server {
    lead_server_config cfg{};
    std::vector<DecShape> shapes;
    std::vector<Slot> slots;
    std::vector<std::deque<Request *>> waiting;
    std::unordered_map<int64_t, std::unique_ptr<Request>> requests;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    bool closed = false;             // no more submits (lead_server_close)
    std::string fault;               // sticky device error
    int64_t next_ticket = 1;
    lead_server_stats st{};
    int device = 0;
    int64_t used = 0;                // device bytes of the slots in existence
    std::vector<int> nslots;         // slots per decoder
};

namespace {

void free_slot(Slot &s) {
    if (s.decoder) lead_decoder_destroy(s.decoder);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.event) (void)hipEventDestroy(s.event);
    (void)hipFree(s.d_synd);
    (void)hipFree(s.d_ehat);
    (void)hipFree(s.d_prior);
    (void)hipFree(s.d_post);
    (void)hipFree(s.d_stats);
    if (s.h_synd) (void)hipHostFree(s.h_synd);
    if (s.h_ehat) (void)hipHostFree(s.h_ehat);
    if (s.h_prior) (void)hipHostFree(s.h_prior);
    if (s.h_post) (void)hipHostFree(s.h_post);
    if (s.h_stats) (void)hipHostFree(s.h_stats);
    s = Slot();
}

hipError_t alloc_slot(lead_server *sv, int dec, lead_decoder *tmpl, Slot &s) {
    const DecShape &sh = sv->shapes[dec];
    const int64_t cap = sv->cfg.max_batch_shots;
    s.dec = dec;
    if (lead::clone_decoder(tmpl, cap, &s.decoder) != LEAD_OK) return hipErrorOutOfMemory;
    hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.event, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&s.d_synd, sizeof(uint64_t) * cap * sh.sw);
    if (e == hipSuccess) e = hipMalloc(&s.d_prior, sizeof(float) * cap);
    if (e == hipSuccess) e = hipMalloc(&s.d_ehat, sizeof(uint64_t) * cap * sh.ew);
    if (e == hipSuccess) e = hipMalloc(&s.d_stats, sizeof(lead_shot_stats) * cap);
    if (e == hipSuccess && sv->cfg.return_posteriors) e = hipMalloc(&s.d_post, sizeof(float) * cap * sh.n);
    if (e == hipSuccess) e = hipHostMalloc(&s.h_synd, sizeof(uint64_t) * cap * sh.sw, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s.h_prior, sizeof(float) * cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s.h_ehat, sizeof(uint64_t) * cap * sh.ew, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s.h_stats, sizeof(lead_shot_stats) * cap, hipHostMallocDefault);
    if (e == hipSuccess && sv->cfg.return_posteriors)
        e = hipHostMalloc(&s.h_post, sizeof(float) * cap * sh.n, hipHostMallocDefault);
    if (e == hipSuccess) {
        // the decoder copy's own allocation plus the slot's device buffers
        s.bytes = lead::decoder_device_bytes(s.decoder) +
                  cap * (8 * sh.sw + 4 + 8 * sh.ew + (int64_t)sizeof(lead_shot_stats)) +
                  (sv->cfg.return_posteriors ? cap * 4 * sh.n : 0);
    }
    return e;
}

// Called with the lock held: a new slot of decoder `dec`, cloned from its
// first slot, if the budget allows; false otherwise (or on failure).
bool grow(lead_server *sv, int dec) {
    lead_decoder *tmpl = nullptr;
    int64_t bytes = 0;
    for (const Slot &x : sv->slots)
        if (x.dec == dec && x.pinned) {
            tmpl = x.decoder;
            bytes = x.bytes;
        }
    if (!tmpl || sv->used + bytes > sv->cfg.mem_budget_bytes) return false;
    Slot s;
    if (alloc_slot(sv, dec, tmpl, s) != hipSuccess) {
        free_slot(s);
        return false;
    }
    sv->used += s.bytes;
    sv->nslots[dec]++;
    sv->st.slots_created++;
    sv->slots.push_back(std::move(s));
    return true;
}

// Called with the lock held: frees an idle extra slot of a decoder that has
// nothing waiting, to make room for another decoder's waiting shots.
bool evict(lead_server *sv, int for_dec) {
    for (size_t i = 0; i < sv->slots.size(); ++i) {
        Slot &x = sv->slots[i];
        if (x.busy || x.pinned || x.dec == for_dec || !sv->waiting[x.dec].empty()) continue;
        sv->used -= x.bytes;
        sv->nslots[x.dec]--;
        free_slot(x);
        sv->slots.erase(sv->slots.begin() + (std::ptrdiff_t)i);
        sv->st.evictions++;
        return true;
    }
    return false;
}

// Called with the lock held: copy the results of a finished slot out.
void retire(lead_server *sv, Slot &s) {
    const DecShape &sh = sv->shapes[s.dec];
    const int64_t t = now_ns();
    for (const Part &p : s.parts) {
        Request &r = *p.req;
        std::memcpy(&r.ehat[p.req_off * sh.ew], &s.h_ehat[p.slot_off * sh.ew], sizeof(uint64_t) * p.count * sh.ew);
        std::memcpy(&r.stats[p.req_off], &s.h_stats[p.slot_off], sizeof(lead_shot_stats) * p.count);
        if (sv->cfg.return_posteriors)
            std::memcpy(&r.post[p.req_off * sh.n], &s.h_post[p.slot_off * sh.n], sizeof(float) * p.count * sh.n);
        r.done_shots += p.count;
        if (r.done_shots == r.shots) {
            r.done = true;
            r.t_done = t;
            sv->st.completed++;
            sv->st.shots_completed += r.shots;
        }
    }
    s.parts.clear();
    s.busy = false;
}

// Called with the lock held: fill an idle slot with waiting shots and launch.
hipError_t fill_and_launch(lead_server *sv, Slot &s) {
    std::deque<Request *> &q = sv->waiting[s.dec];
    const DecShape &sh = sv->shapes[s.dec];
    const int64_t cap = sv->cfg.max_batch_shots;
    int64_t used = 0;
    while (!q.empty() && used < cap) {
        Request &r = *q.front();
        const int64_t cnt = std::min(r.shots - r.next_shot, cap - used);
        std::memcpy(&s.h_synd[used * sh.sw], &r.synd[r.next_shot * sh.sw], sizeof(uint64_t) * cnt * sh.sw);
        std::memcpy(&s.h_prior[used], &r.prior[r.next_shot], sizeof(float) * cnt);
        s.parts.push_back(Part{&r, r.next_shot, used, cnt});
        r.next_shot += cnt;
        used += cnt;
        if (r.next_shot == r.shots) q.pop_front();
    }
    if (used == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(s.d_synd, s.h_synd, sizeof(uint64_t) * used * sh.sw, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.d_prior, s.h_prior, sizeof(float) * used, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess) {
        lead_status st = lead_decode(s.decoder, used, s.d_synd, sh.sw, s.d_prior, LEAD_PRIOR_PER_SHOT, s.d_ehat,
                                     sh.ew, s.d_post, nullptr, s.d_stats, s.stream);
        if (st != LEAD_OK) e = hipErrorLaunchFailure;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.h_ehat, s.d_ehat, sizeof(uint64_t) * used * sh.ew, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.h_stats, s.d_stats, sizeof(lead_shot_stats) * used, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess && sv->cfg.return_posteriors)
        e = hipMemcpyAsync(s.h_post, s.d_post, sizeof(float) * used * sh.n, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.event, s.stream);
    if (e == hipSuccess) {
        s.busy = true;
        sv->st.launches++;
    }
    return e;
}

void worker_loop(lead_server *sv) {
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        bool progress = false, any_busy = false;
        for (Slot &s : sv->slots) {
            if (!s.busy) continue;
            hipError_t q = hipEventQuery(s.event);
            if (q == hipSuccess) {
                retire(sv, s);
                progress = true;
            } else if (q != hipErrorNotReady) {
                sv->fault = std::string("device error in a launch: ") + hipGetErrorString(q);
                s.busy = false;
            } else {
                any_busy = true;
            }
        }
        if (progress) sv->cv_done.notify_all();
        if (sv->fault.empty()) {
            // admission: a decoder with waiting shots and every slot busy
            // gets another slot within the budget (freeing an idle slot of
            // a decoder with nothing waiting if needed)
            for (int dec = 0; dec < (int)sv->waiting.size(); ++dec) {
                if (sv->waiting[dec].empty() || sv->nslots[dec] >= sv->cfg.max_slots_per_decoder) continue;
                bool idle = false;
                for (const Slot &x : sv->slots) idle = idle || (x.dec == dec && !x.busy);
                if (idle) continue;
                if (!grow(sv, dec) && evict(sv, dec)) (void)grow(sv, dec);
            }
            for (Slot &s : sv->slots) {
                if (s.busy || sv->waiting[s.dec].empty()) continue;
                hipError_t e = fill_and_launch(sv, s);
                if (e != hipSuccess) {
                    sv->fault = std::string("launch failed: ") + hipGetErrorString(e);
                    break;
                }
                progress = true;
                any_busy = true;
            }
        }
        if (!sv->fault.empty()) sv->cv_done.notify_all();
        if (sv->stop && !any_busy) break;
        if (!progress) {
            if (any_busy) {
                // poll the device again soon without holding the lock
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                sv->cv_work.wait(lk, [sv] {
                    if (sv->stop) return true;
                    for (auto &q : sv->waiting)
                        if (!q.empty()) return true;
                    return false;
                });
            }
        }
    }
}

}  // namespace

extern "C" {

int64_t lead_server_clock_ns(void) { return now_ns(); }

lead_status lead_server_create(lead_decoder *const *decoders, int32_t nd, const lead_server_config *config,
                               lead_server **out) {
    if (!decoders || nd <= 0 || !out) return lead::set_error(LEAD_E_ARG, "bad argument");
    *out = nullptr;
    std::unique_ptr<lead_server> sv(new (std::nothrow) lead_server());
    if (!sv) return lead::set_error(LEAD_E_NOMEM, "out of host memory");
    if (config) sv->cfg = *config;
    if (sv->cfg.mem_budget_bytes <= 0) sv->cfg.mem_budget_bytes = int64_t(1) << 30;
    if (sv->cfg.max_batch_shots <= 0) sv->cfg.max_batch_shots = 4096;
    if (sv->cfg.max_slots_per_decoder <= 0) sv->cfg.max_slots_per_decoder = 4;
    if (sv->cfg.max_pending_shots <= 0) sv->cfg.max_pending_shots = int64_t(1) << 24;
    if (hipGetDevice(&sv->device) != hipSuccess) return lead::set_error(LEAD_E_DEVICE, "hipGetDevice failed");
    sv->shapes.resize(nd);
    for (int i = 0; i < nd; ++i) {
        if (!decoders[i]) return lead::set_error(LEAD_E_ARG, "NULL decoder");
        int n, m;
        lead::decoder_shape(decoders[i], &n, &m);
        sv->shapes[i] = DecShape{n, m, (m + 63) / 64, (n + 63) / 64};
    }
    sv->waiting.resize(nd);
    sv->nslots.assign(nd, 0);
    // one slot per decoder (kept for the server's life), then more,
    // round-robin, while the budget allows
    for (int i = 0; i < nd; ++i) {
        Slot s;
        hipError_t e = alloc_slot(sv.get(), i, decoders[i], s);
        if (e != hipSuccess || sv->used + s.bytes > sv->cfg.mem_budget_bytes) {
            const int64_t need = s.bytes;
            free_slot(s);
            for (Slot &x : sv->slots) free_slot(x);
            if (e != hipSuccess) return lead::set_error(LEAD_E_NOMEM, "slot allocation failed");
            return lead::set_error(LEAD_E_CAPACITY,
                                   ("mem_budget_bytes " + std::to_string(sv->cfg.mem_budget_bytes) +
                                    " cannot hold one launch slot per decoder (decoder " + std::to_string(i) +
                                    " needs " + std::to_string(need) + " bytes beyond " + std::to_string(sv->used) + ")")
                                       .c_str());
        }
        s.pinned = true;
        sv->used += s.bytes;
        sv->nslots[i] = 1;
        sv->slots.push_back(std::move(s));
    }
    sv->st.slots_created = nd;
    for (int round = 1; round < sv->cfg.max_slots_per_decoder; ++round)
        for (int i = 0; i < nd; ++i) (void)grow(sv.get(), i);
    lead_server *raw = sv.get();
    try {
        sv->worker = std::thread(worker_loop, raw);
    } catch (...) {
        for (Slot &x : sv->slots) free_slot(x);
        return lead::set_error(LEAD_E_NOMEM, "cannot start the worker thread");
    }
    *out = sv.release();
    return LEAD_OK;
}

lead_status lead_server_submit(lead_server *sv, int32_t dec, int64_t shots, const uint64_t *h_synd,
                               int64_t synd_words, const float *h_prior, int64_t *ticket) {
    if (!sv || !ticket || shots <= 0 || !h_synd || !h_prior) return lead::set_error(LEAD_E_ARG, "bad argument");
    if (dec < 0 || dec >= (int32_t)sv->shapes.size()) return lead::set_error(LEAD_E_ARG, "decoder index out of range");
    const DecShape &sh = sv->shapes[dec];
    if (synd_words < sh.sw) return lead::set_error(LEAD_E_ARG, "synd_words < ceil(m/64)");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->closed || sv->stop) return lead::set_error(LEAD_E_CLOSED, "the server is closed");
        if (shots > sv->cfg.max_pending_shots) {
            sv->st.refused++;
            return lead::set_error(LEAD_E_CAPACITY, ("oversize request: " + std::to_string(shots) +
                                                     " shots, the server holds at most " +
                                                     std::to_string(sv->cfg.max_pending_shots) + " pending")
                                                        .c_str());
        }
        if (sv->st.pending_shots + shots > sv->cfg.max_pending_shots) {
            sv->st.refused++;
            return lead::set_error(LEAD_E_CAPACITY, ("server busy: " + std::to_string(sv->st.pending_shots) +
                                                     " shots pending of at most " +
                                                     std::to_string(sv->cfg.max_pending_shots) +
                                                     "; collect results and retry")
                                                        .c_str());
        }
        sv->st.pending_shots += shots;   // reserved now; released by lead_server_result
    }
    auto unreserve = [&] {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->st.pending_shots -= shots;
    };
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) {
        unreserve();
        return lead::set_error(LEAD_E_NOMEM, "out of host memory");
    }
    if (!r) return lead::set_error(LEAD_E_NOMEM, "out of host memory");
    try {
        r->dec = dec;
        r->shots = shots;
        r->synd.resize((size_t)shots * sh.sw);
        for (int64_t i = 0; i < shots; ++i)
            std::memcpy(&r->synd[i * sh.sw], h_synd + i * synd_words, sizeof(uint64_t) * sh.sw);
        r->prior.assign(h_prior, h_prior + shots);
        r->ehat.resize((size_t)shots * sh.ew);
        r->stats.resize(shots);
        if (sv->cfg.return_posteriors) r->post.resize((size_t)shots * sh.n);
    } catch (const std::bad_alloc &) {
        unreserve();
        return lead::set_error(LEAD_E_NOMEM, "out of host memory");
    }
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (!sv->fault.empty() || sv->closed || sv->stop) {
            sv->st.pending_shots -= shots;
            if (!sv->fault.empty()) return lead::set_error(LEAD_E_DEVICE, sv->fault.c_str());
            return lead::set_error(LEAD_E_CLOSED, "the server is closed");
        }
        *ticket = sv->next_ticket++;
        sv->waiting[dec].push_back(r.get());
        sv->requests[*ticket] = std::move(r);
        sv->st.submitted++;
    }
    sv->cv_work.notify_one();
    return LEAD_OK;
}

lead_status lead_server_poll(lead_server *sv, int64_t ticket, int32_t *done) {
    if (!sv || !done) return lead::set_error(LEAD_E_ARG, "bad argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return lead::set_error(LEAD_E_ARG, "unknown ticket");
    if (!sv->fault.empty() && !it->second->done) return lead::set_error(LEAD_E_DEVICE, sv->fault.c_str());
    *done = it->second->done ? 1 : 0;
    return LEAD_OK;
}

lead_status lead_server_wait(lead_server *sv, int64_t ticket) {
    if (!sv) return lead::set_error(LEAD_E_ARG, "bad argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return lead::set_error(LEAD_E_ARG, "unknown ticket");
    Request *r = it->second.get();
    sv->cv_done.wait(lk, [&] { return r->done || !sv->fault.empty(); });
    if (!r->done) return lead::set_error(LEAD_E_DEVICE, sv->fault.c_str());
    return LEAD_OK;
}

lead_status lead_server_result(lead_server *sv, int64_t ticket, uint64_t *h_ehat, float *h_post,
                               lead_shot_stats *h_stats, int64_t *submit_ns, int64_t *done_ns) {
    if (!sv) return lead::set_error(LEAD_E_ARG, "bad argument");
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->requests.find(ticket);
        if (it == sv->requests.end()) return lead::set_error(LEAD_E_ARG, "unknown ticket");
        if (!it->second->done) return lead::set_error(LEAD_E_ARG, "request not finished");
        if (h_post && !sv->cfg.return_posteriors)
            return lead::set_error(LEAD_E_ARG, "server was created without return_posteriors");
        r = std::move(it->second);
        sv->requests.erase(it);
        sv->st.pending_shots -= r->shots;
    }
    if (h_ehat) std::memcpy(h_ehat, r->ehat.data(), sizeof(uint64_t) * r->ehat.size());
    if (h_post) std::memcpy(h_post, r->post.data(), sizeof(float) * r->post.size());
    if (h_stats) std::memcpy(h_stats, r->stats.data(), sizeof(lead_shot_stats) * r->stats.size());
    if (submit_ns) *submit_ns = r->t_submit;
    if (done_ns) *done_ns = r->t_done;
    return LEAD_OK;
}

lead_status lead_server_get_stats(lead_server *sv, lead_server_stats *out) {
    if (!sv || !out) return lead::set_error(LEAD_E_ARG, "bad argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    out->slots = (int32_t)sv->slots.size();
    out->slot_bytes = sv->used;
    return LEAD_OK;
}

lead_status lead_server_close(lead_server *sv) {
    if (!sv) return lead::set_error(LEAD_E_ARG, "bad argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->closed = true;
    sv->cv_done.wait(lk, [sv] { return sv->st.completed == sv->st.submitted || !sv->fault.empty(); });
    if (sv->st.completed != sv->st.submitted) return lead::set_error(LEAD_E_DEVICE, sv->fault.c_str());
    return LEAD_OK;
}

void lead_server_destroy(lead_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        for (auto &q : sv->waiting) q.clear();
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (Slot &s : sv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        free_slot(s);
    }
    delete sv;
}

}  // extern "C"
