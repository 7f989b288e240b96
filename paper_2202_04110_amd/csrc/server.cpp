// Serving loop: continuous batching of belief-propagation solves.
//
// Requests (a graph, iteration count, damping, temperature and optionally a
// loss gradient for the reverse sweep) are compiled on the submitting thread
// and queued.  A worker thread admits queued requests first-in first-out
// while a slot is free and the memory arena (one device allocation of the
// HBM budget) has room for the graph, its messages and, for backward
// requests, the checkpoint workspace.  Admitted graphs are uploaded on a copy
// stream and stay resident; every round advances all resident graphs by a
// few iterations in shared multi-graph launches on the compute stream, so
// uploads overlap compute and requests join and leave at round boundaries.
// A finished graph is read out (normalised beliefs, MAP and, if asked, the
// gradient w.r.t. its log-potentials) into pinned host buffers and its memory
// returns to the arena.
//
// The same kernels and per-element arithmetic run whether a graph is alone or
// in the mix, so served results are bitwise equal to lone runs.
#include <hip/hip_runtime.h>
#include <sched.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <functional>
#include <thread>
#include <vector>

#include "arena.h"
#include "runtime.h"

using namespace lbp;

namespace {

using Clock = std::chrono::steady_clock;

struct PanelFree {
    void operator()(char *p) const { panel_free(p); }
};
using PanelPtr = std::unique_ptr<char, PanelFree>;

// Host copy of a graph description (the caller may free its arrays once
// lbp_server_submit returns).  The log-potentials go to a pooled page-locked
// buffer, checked for NaN and infinity on the way; the GPU executor uploads
// them from there as they are (the device writes their panel).
struct DescCopy {
    std::vector<int32_t> nst, kind, evar, ftab, tab_ncfg, tab_arity, tab_states;
    std::vector<float> ev;
    std::vector<int64_t> fe_off, tab_off, lp_off;
    PanelPtr lp;
    int64_t lp_bad = -1;  // index of the first non-finite log-potential, or -1
    lbp_graph_desc d{};

    // `src` must have passed validate_desc with these sizes.
    void take(const lbp_graph_desc *src, const int64_t sz[6]) {
        const int64_t V = sz[0], VS = sz[1], F = sz[2], E = sz[3], Tn = sz[5], NT = src->num_cfg_tables;
        nst.assign(src->var_num_states, src->var_num_states + V);
        if (src->evidence) ev.assign(src->evidence, src->evidence + VS);
        kind.assign(src->factor_kind, src->factor_kind + F);
        fe_off.assign(src->factor_edge_off, src->factor_edge_off + F + 1);
        evar.assign(src->edge_var, src->edge_var + E);
        ftab.assign(src->factor_cfg_table, src->factor_cfg_table + F);
        if (NT > 0) {
            tab_ncfg.assign(src->cfg_table_num_cfgs, src->cfg_table_num_cfgs + NT);
            tab_arity.assign(src->cfg_table_arity, src->cfg_table_arity + NT);
            tab_off.assign(src->cfg_table_off, src->cfg_table_off + NT + 1);
            if (tab_off[NT] > 0) tab_states.assign(src->cfg_table_states, src->cfg_table_states + tab_off[NT]);
        }
        lp_off.assign(src->logpot_off, src->logpot_off + F + 1);
        lp.reset((char *)panel_alloc(sizeof(float) * std::max<int64_t>(1, Tn)));
        if (!lp) throw std::bad_alloc();
        if (Tn > 0) lp_bad = copy_check_finite((float *)lp.get(), src->log_potentials, Tn);
        d.num_vars = (int32_t)V;
        d.var_num_states = nst.data();
        d.evidence = src->evidence ? ev.data() : nullptr;
        d.num_factors = (int32_t)F;
        d.factor_kind = kind.data();
        d.factor_edge_off = fe_off.data();
        d.edge_var = evar.data();
        d.factor_cfg_table = ftab.data();
        d.num_cfg_tables = (int32_t)NT;
        d.cfg_table_num_cfgs = tab_ncfg.data();
        d.cfg_table_arity = tab_arity.data();
        d.cfg_table_off = NT > 0 ? tab_off.data() : nullptr;
        d.cfg_table_states = tab_states.data();
        d.logpot_off = lp_off.data();
        d.log_potentials = (const float *)lp.get();
    }
};

struct Request {
    uint64_t id = 0;
    uint64_t seq = 0;
    int prep = 0;  // 0 compiling, 1 ready, 2 failed (guarded by the server mutex)
    int prep_status = LBP_OK;
    std::unique_ptr<DescCopy> desc;
    int32_t iters = 0, k = 10;
    float d = 0.5f, T = 1.0f;
    bool backward = false;
    // early exit (lbp_server_submit_until): tol >= 0 enables it; the
    // residual is measured when done reaches a multiple of check or iters
    float tol = -1.0f;
    int32_t check = 0;
    bool check_now = false;   // this round ends at one of the request's check points
    int32_t res_slot = 0;     // index of its residual in the round's read-back
    bool settled = false;     // a check found the residual below tol
    float residual = -1.0f;   // last residual measured (0 before the first check)
    size_t conv_bytes = 0;    // previous messages, partial maxima, residual
    char *conv = nullptr;
    uint64_t up_gen = 0;      // upload number (executor's count) while its upload may be in flight
    hipEvent_t up_ev = nullptr;  // recorded on the copy stream after its uploads (while they may be in flight)
    bool uploading = false;   // worker: handed to the executor's uploader, not yet taken back
    int upload_status = LBP_OK;
    bool in_backward = false; // read out; its reverse sweep runs on the executor's finisher thread
    int back_status = LBP_OK;
    std::vector<float> grad_q;
    std::vector<DevGraph> adj_views;  // host staging of the reverse sweep's views (copied at admission)
    HostLayout L;
    size_t bytes = 0, graph_bytes = 0, adj_bytes = 0;
    size_t off = Arena::kNone;
    lbp_graph *g = nullptr;
    int32_t done = 0;
    int32_t status = LBP_OK;
    bool cancel = false;
    double t_arrival = 0, t_ready = -1, t_admit = -1, t_done = -1;
    float *q = nullptr;
    int32_t *map = nullptr;
    float *gphi = nullptr;
    float *gq_dev = nullptr, *gphi_dev = nullptr;
    // device data packed for one upload (built by a prep thread) and the
    // log-potentials as given (copied at submission), freed once the upload
    // has completed or with the request
    PanelPtr image, lp;
};

// What the scheduler asks of the machine.  The GPU executor runs the HIP
// path; the host executor only keeps the books (scheduling tests on a host
// without a GPU).
class Executor {
public:
    virtual ~Executor() {}
    virtual int admit(Request &r) = 0;
    virtual int round(const std::vector<Request *> &active, int32_t steps) = 0;
    virtual int wait() = 0;
    // waits for everything queued for rounds (after a failed launch)
    virtual void quiesce() {}
    // Read-out of finished requests: finish_begin for each (slot: its index
    // in this batch, < max_slots), one finish_wait, then finish_end for each.
    virtual int finish_begin(Request &r, int32_t slot) = 0;
    virtual int finish_wait() = 0;
    virtual int finish_end(Request &r, int32_t slot) = 0;
    // after wait(): the residual of every request with check_now
    virtual void residuals(const std::vector<Request *> &active) = 0;
    virtual void release(Request &r) = 0;
    // after wait(): frees the upload images that are no longer needed
    virtual void images_done(const std::vector<Request *> &) {}
    // Reverse sweeps off the worker thread: after its read-out, a backward
    // request may be handed to a finisher (start_backward returns true; the
    // request stays resident); take_backward returns the finished ones, with
    // back_status set; `wake` is called from the finisher when one is done;
    // drain_backward waits until every handed-over sweep has finished.
    virtual bool start_backward(Request &) { return false; }
    virtual void take_backward(std::vector<Request *> &) {}
    virtual void set_wake(std::function<void()>) {}
    virtual void drain_backward() {}
    // Uploads off the worker thread: admit may hand the request to an
    // uploader (setting r.uploading) and return at once; take_uploaded
    // returns those whose uploads are queued, with upload_status set (wake
    // is called when one is); drain_uploads waits until none is left.
    virtual void take_uploaded(std::vector<Request *> &) {}
    virtual void drain_uploads() {}
    virtual int alloc_outputs(Request &r) = 0;
    virtual void free_outputs(Request &r) = 0;
    // whether prep threads should pack each request's upload image
    virtual bool wants_image() const { return false; }
};

class HostExecutor : public Executor {
public:
    int admit(Request &) override { return LBP_OK; }
    int round(const std::vector<Request *> &, int32_t) override { return LBP_OK; }
    int wait() override { return LBP_OK; }
    int finish_begin(Request &, int32_t) override { return LBP_OK; }
    int finish_wait() override { return LBP_OK; }
    int finish_end(Request &, int32_t) override { return LBP_OK; }
    // the bookkeeping executor's messages stay zero, so they never change
    void residuals(const std::vector<Request *> &active) override {
        for (Request *r : active)
            if (r->check_now) r->residual = 0.0f;
    }
    void release(Request &) override {}
    int alloc_outputs(Request &r) override {
        r.q = (float *)calloc((size_t)std::max<int64_t>(1, r.L.VS), sizeof(float));
        r.map = (int32_t *)calloc((size_t)std::max<int64_t>(1, r.L.V), sizeof(int32_t));
        if (r.backward) r.gphi = (float *)calloc((size_t)std::max<int64_t>(1, r.L.Tn), sizeof(float));
        return (r.q && r.map && (!r.backward || r.gphi)) ? LBP_OK : LBP_E_OOM;
    }
    void free_outputs(Request &r) override {
        free(r.q);
        free(r.map);
        free(r.gphi);
        r.q = nullptr;
        r.map = nullptr;
        r.gphi = nullptr;
    }
};

class GpuExecutor : public Executor {
public:
    ~GpuExecutor() override {
        if (up_th_.joinable()) {
            {
                std::lock_guard<std::mutex> lk(umu_);
                ustop_ = true;
            }
            ucv_.notify_all();
            up_th_.join();
        }
        if (fin_th_.joinable()) {
            {
                std::lock_guard<std::mutex> lk(fmu_);
                fstop_ = true;
            }
            fcv_.notify_all();
            fin_th_.join();
        }
        (void)hipSetDevice(ctx_.device);
        if (back_) (void)hipStreamSynchronize(back_);
        if (back_) (void)hipStreamDestroy(back_);
        if (read_) (void)hipStreamSynchronize(read_);
        if (read_) (void)hipStreamDestroy(read_);
        if (compute_) (void)hipStreamSynchronize(compute_);
        if (copy_) (void)hipStreamSynchronize(copy_);
        if (stage_) (void)hipFree(stage_);
        if (base_) (void)hipFree(base_);
        if (res_host_) (void)hipHostFree(res_host_);
        if (jobs_host_) (void)hipHostFree(jobs_host_);
        if (flags_host_) (void)hipHostFree(flags_host_);
        if (read_host_) (void)hipHostFree(read_host_);
        for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
        if (jobs_dev_) (void)hipFree(jobs_dev_);
        if (ev_) (void)hipEventDestroy(ev_);
        if (compute_) (void)hipStreamDestroy(compute_);
        if (copy_) (void)hipStreamDestroy(copy_);
    }

    int init(int device, size_t budget, int32_t max_slots) {
        ctx_.device = device;
        ctx_.use_graphs = false;
        HIP_TRY(hipSetDevice(device));
        HIP_TRY(hipStreamCreateWithFlags(&compute_, hipStreamNonBlocking));
        HIP_TRY(hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking));
        HIP_TRY(hipStreamCreateWithFlags(&back_, hipStreamNonBlocking));
        HIP_TRY(hipStreamCreateWithFlags(&read_, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
        if (hipHostMalloc((void **)&flags_host_, sizeof(int32_t) * (size_t)max_slots) != hipSuccess ||
            hipHostMalloc((void **)&read_host_, sizeof(ReadJob) * (size_t)max_slots) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(LBP_E_OOM, "pinned read-out buffers");
        }
        // read-outs write the result buffers from the device through their
        // host addresses: page-locked memory must be mapped at the same address
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, flags_host_, 0) != hipSuccess || dp != (void *)flags_host_) {
            (void)hipGetLastError();
            return set_error(LBP_E_UNSUPPORTED, "page-locked host memory is not mapped at its host address");
        }
        // convergence checks: one job and one residual per resident request,
        // staged in pinned memory and read back after each round
        const size_t jb = align256(sizeof(ConvJob) * (size_t)max_slots);
        const size_t rb = align256(sizeof(float) * (size_t)max_slots);
        if (hipHostMalloc((void **)&res_host_, sizeof(float) * (size_t)max_slots) != hipSuccess ||
            hipHostMalloc((void **)&jobs_host_, sizeof(ConvJob) * (size_t)max_slots) != hipSuccess ||
            hipMalloc((void **)&jobs_dev_, jb + rb + sizeof(ReadJob) * (size_t)max_slots) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(LBP_E_OOM, "convergence-check and read-out buffers");
        }
        res_dev_ = (float *)((char *)jobs_dev_ + jb);
        read_dev_ = (ReadJob *)((char *)jobs_dev_ + jb + rb);
        ctx_.stream = compute_;
        hipError_t e = hipMalloc((void **)&base_, std::max<size_t>(budget, 256));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            return set_error(LBP_E_OOM, "server arena of " + std::to_string(budget) + " bytes");
        }
        try {
            fin_th_ = std::thread([this] { finisher(); });
            up_th_ = std::thread([this] { uploader(); });
        } catch (const std::system_error &) {
            return set_error(LBP_E_OOM, "could not start the finisher or uploader thread");
        }
        return LBP_OK;
    }

    // Called on the worker thread before any other call.
    void bind() { (void)hipSetDevice(ctx_.device); }

    bool wants_image() const override { return true; }

    // Admission hands the request to the uploader thread, which queues its
    // uploads on the copy stream and waits for none of them: the graph image
    // and potentials, and for a backward request the reverse sweep's views
    // and its loss vector, all from host memory the request keeps (the image
    // and potentials until a round or read-out has waited for this upload,
    // the rest until the request ends; release waits for an upload still in
    // flight).  Each request's copies end with an event of its own, recorded
    // with its upload number under umu_ (numbers follow the copy stream's
    // order), so a round waits only for the uploads of the requests it runs:
    // those of the latest of them, and with them every earlier one.
    int admit(Request &r) override {
        r.uploading = true;
        {
            std::lock_guard<std::mutex> lk(umu_);
            uq_.push_back(&r);
            ++upending_;
        }
        ucv_.notify_one();
        return LBP_OK;
    }

    void take_uploaded(std::vector<Request *> &out) override {
        std::lock_guard<std::mutex> lk(umu_);
        out.insert(out.end(), udone_.begin(), udone_.end());
        udone_.clear();
    }

    void drain_uploads() override {
        std::unique_lock<std::mutex> lk(umu_);
        udone_cv_.wait(lk, [&] { return upending_ == 0; });
    }

    // Stream st waits for the uploads of requests rs not yet known complete;
    // *gen records how far that reaches (complete once st has been waited for).
    int wait_uploads(hipStream_t st, Request *const *rs, size_t n, uint64_t *gen) {
        const Request *last = nullptr;
        for (size_t i = 0; i < n; ++i)
            if (rs[i]->up_gen > up_done_ && (!last || rs[i]->up_gen > last->up_gen)) last = rs[i];
        if (last) {
            HIP_TRY(hipStreamWaitEvent(st, last->up_ev, 0));
            *gen = std::max(*gen, last->up_gen);
        }
        return LBP_OK;
    }

    // an upload known complete: its event goes back to the pool
    void retire_upload(Request &r) {
        if (!r.up_ev) return;
        std::lock_guard<std::mutex> lk(umu_);
        ev_pool_.push_back(r.up_ev);
        r.up_ev = nullptr;
    }

    int round(const std::vector<Request *> &active, int32_t steps) override {
        int urc = wait_uploads(compute_, active.data(), active.size(), &round_gen_);
        if (urc != LBP_OK) return urc;
        std::vector<uint64_t> ids;
        for (Request *r : active) ids.push_back(r->id);
        if (ids != ids_) {
            int rc = rebuild(active);
            if (rc != LBP_OK) return rc;
            ids_ = ids;
        }
        for (Request *r : active)
            if (r->backward && r->done % r->g->adj.k == 0 && r->done < r->iters) {
                int rc = adjoint_checkpoint(r->g, r->done / r->g->adj.k, compute_);
                if (rc != LBP_OK) return rc;
            }
        // requests at a check point: one job each (all checked in shared
        // launches), slot = position in the active list
        int nj = 0, max_m = 0, max_e = 0;
        for (size_t i = 0; i < active.size(); ++i) {
            Request *r = active[i];
            r->res_slot = (int32_t)i;
            if (!r->check_now) continue;
            ConvJob &J = jobs_host_[nj++];
            J.g = r->g->dgraph;
            J.mprev = (float *)r->conv;
            J.partial = (float *)(r->conv + align256(sizeof(float) * std::max<int64_t>(1, r->g->M)));
            J.E = (int32_t)r->g->E;
            J.M = (int32_t)r->g->M;
            J.slot = (int32_t)i;
            J.pad = 0;
            max_m = std::max(max_m, J.M);
            max_e = std::max(max_e, J.E);
        }
        if (nj > 0)
            HIP_TRY(hipMemcpyAsync(jobs_dev_, jobs_host_, sizeof(ConvJob) * nj, hipMemcpyHostToDevice, compute_));
        // every part's iterations but the last, the copies of the checked
        // requests' messages, then every part's last iteration
        for (int32_t it = 0; it < steps; ++it) {
            if (it == steps - 1) HIP_TRY(launch_save_multi(jobs_dev_, nj, max_m, compute_));
            for (const Part &p : parts_) {
                hipError_t e = launch_iteration(p.dgs, p.vl, p.fl, make_params(p.d, p.T), p.T == 0.0f, compute_);
                if (e != hipSuccess) return hip_error(e, "served iteration launch");
            }
        }
        if (nj > 0) {
            HIP_TRY(launch_residual_multi(jobs_dev_, nj, max_e, res_dev_, compute_));
            HIP_TRY(hipMemcpyAsync(res_host_, res_dev_, sizeof(float) * active.size(), hipMemcpyDeviceToHost,
                                   compute_));
        }
        HIP_TRY(hipEventRecord(ev_, compute_));
        return LBP_OK;
    }

    void quiesce() override { (void)hipStreamSynchronize(compute_); }

    int wait() override {
        HIP_TRY(hipEventSynchronize(ev_));
        up_done_ = std::max(up_done_, round_gen_);
        return LBP_OK;
    }

    // the image of a request whose upload is known to have completed
    void drop_image(Request &r) {
        if (r.image && r.up_gen <= up_done_) {
            r.image.reset();
            r.lp.reset();
            retire_upload(r);
        }
    }

    void residuals(const std::vector<Request *> &active) override {
        for (Request *r : active)
            if (r->check_now) r->residual = res_host_[r->res_slot];
    }

    // A batch of read-outs on the read-out stream, beside the next round
    // (which holds none of these graphs): each graph's beliefs from its
    // messages (its own belief launches), then one launch that writes every
    // request's normalised beliefs and MAP straight into its page-locked
    // result buffers, then one wait.  Backward requests then go to the
    // finisher.  The worker has waited for the round that last ran them.
    int finish_begin(Request &r, int32_t slot) override {
        if (r.up_gen > up_done_) {  // not covered by a round yet (zero iterations)
            Request *rp = &r;
            int urc = wait_uploads(read_, &rp, 1, &read_gen_);
            if (urc != LBP_OK) return urc;
        }
        const TParams P = make_params(0.5f, r.T);
        HIP_TRY(launch_iteration(r.g->dgraph, r.g->vl, r.g->fl, P, r.T == 0.0f, read_, 1));
        flags_host_[slot] = 0;
        ReadJob &J = read_host_[fin_.size()];  // jobs packed in the order they are queued
        J.g = r.g->dgraph;
        J.q = r.q;
        J.map = r.map;
        J.flag = flags_host_ + slot;
        J.P = P;
        J.ntiles = r.g->nvt;
        J.maxp = r.T == 0.0f;
        fin_.push_back(&r);
        return LBP_OK;
    }

    int finish_wait() override {
        const int n = (int)fin_.size();
        int max_tiles = 0;
        for (int i = 0; i < n; ++i) max_tiles = std::max(max_tiles, read_host_[i].ntiles);
        int rc = LBP_OK;
        if (n > 0) {
            hipError_t e = hipMemcpyAsync(read_dev_, read_host_, sizeof(ReadJob) * n, hipMemcpyHostToDevice, read_);
            if (e == hipSuccess) e = launch_readout_multi(read_dev_, n, max_tiles, read_);
            if (e != hipSuccess) rc = hip_error(e, "read-out launch");
        }
        fin_.clear();
        HIP_TRY(hipStreamSynchronize(read_));
        up_done_ = std::max(up_done_, read_gen_);
        return rc;
    }

    int finish_end(Request &r, int32_t slot) override {
        drop_image(r);
        return flags_host_[slot] ? set_error(LBP_E_NONFINITE, "beliefs contain NaN or infinity") : LBP_OK;
    }

    bool start_backward(Request &r) override {
        {
            std::lock_guard<std::mutex> lk(fmu_);
            bq_.push_back(&r);
            ++fpending_;
        }
        fcv_.notify_one();
        return true;
    }

    void take_backward(std::vector<Request *> &out) override {
        std::lock_guard<std::mutex> lk(fmu_);
        out.insert(out.end(), bdone_.begin(), bdone_.end());
        bdone_.clear();
    }

    // Once set_wake returns, no call of the previous function is under way
    // or will start: the server clears it before it goes away.
    void set_wake(std::function<void()> w) override {
        std::lock_guard<std::mutex> lk(wmu_);
        wake_ = std::move(w);
    }

    void drain_backward() override {
        std::unique_lock<std::mutex> lk(fmu_);
        fdone_cv_.wait(lk, [&] { return fpending_ == 0; });
    }

    void release(Request &r) override {
        if (r.image) {
            // an upload that no round or read-out has waited for yet: the
            // arena memory and the image are reused only after it completes
            if (r.up_gen > up_done_) {
                if (r.up_ev) (void)hipEventSynchronize(r.up_ev);
                else (void)hipStreamSynchronize(copy_);
                up_done_ = std::max(up_done_, r.up_gen);
            }
            r.image.reset();
            r.lp.reset();
        }
        retire_upload(r);
        graph_destroy(r.g);  // the arena owns the memory
        r.g = nullptr;
        ids_.clear();        // the resident set changes
    }

    void images_done(const std::vector<Request *> &resident) override {
        for (Request *r : resident)
            if (!r->uploading) drop_image(*r);  // the uploader still owns the others
    }

    int alloc_outputs(Request &r) override {
        r.q = (float *)pinned_get(sizeof(float) * std::max<int64_t>(1, r.L.VS));
        r.map = (int32_t *)pinned_get(sizeof(int32_t) * std::max<int64_t>(1, r.L.V));
        if (r.backward) r.gphi = (float *)pinned_get(sizeof(float) * std::max<int64_t>(1, r.L.Tn));
        if (!r.q || !r.map || (r.backward && !r.gphi)) {
            free_outputs(r);
            return set_error(LBP_E_OOM, "pinned output buffers");
        }
        return LBP_OK;
    }

    // Called from the polling thread: buffers go back to the pool.
    void free_outputs(Request &r) override {
        pinned_put(r.q, sizeof(float) * std::max<int64_t>(1, r.L.VS));
        pinned_put(r.map, sizeof(int32_t) * std::max<int64_t>(1, r.L.V));
        if (r.gphi) pinned_put(r.gphi, sizeof(float) * std::max<int64_t>(1, r.L.Tn));
        r.q = nullptr;
        r.map = nullptr;
        r.gphi = nullptr;
    }

private:
    // Wakes the worker (a sweep or an upload has finished).
    void call_wake() {
        std::lock_guard<std::mutex> lk(wmu_);
        if (wake_) wake_();
    }

    // A request's uploads on the copy stream (see admit).
    int upload(Request &r) {
        char *mem = base_ + r.off;
        int rc = graph_create(&ctx_, r.L, false, mem, copy_, &r.g, r.image.get(), false, (const float *)r.lp.get());
        if (rc == LBP_OK) {
            r.g->last_T = r.T;
            if (r.tol >= 0.0f) r.conv = mem + Arena::round(r.graph_bytes);
            if (r.backward) {
                char *am = mem + Arena::round(r.graph_bytes);
                rc = adjoint_prepare(r.g, r.iters, r.d, r.T, r.k, am, copy_, &r.adj_views);
                if (rc == LBP_OK) {
                    r.gq_dev = (float *)(am + Arena::round(r.adj_bytes));
                    r.gphi_dev = (float *)((char *)r.gq_dev + Arena::round(sizeof(float) * r.L.VS));
                    hipError_t e = hipMemcpyAsync(r.gq_dev, r.grad_q.data(), sizeof(float) * r.L.VS,
                                                  hipMemcpyHostToDevice, copy_);
                    if (e != hipSuccess) rc = hip_error(e, "loss vector upload");
                }
            }
        }
        // from here on release waits for the copy stream (also after a
        // failure part-way: some copies may be queued)
        std::lock_guard<std::mutex> lk(umu_);
        r.up_gen = ++up_gen_;
        hipError_t e = hipSuccess;
        if (!ev_pool_.empty()) {
            r.up_ev = ev_pool_.back();
            ev_pool_.pop_back();
        } else {
            e = hipEventCreateWithFlags(&r.up_ev, hipEventDisableTiming);
            if (e != hipSuccess) r.up_ev = nullptr;  // release then waits for the whole copy stream
        }
        if (e == hipSuccess) e = hipEventRecord(r.up_ev, copy_);
        if (e != hipSuccess && r.up_ev) {  // not recorded: release waits for the whole copy stream
            ev_pool_.push_back(r.up_ev);
            r.up_ev = nullptr;
        }
        if (e != hipSuccess && rc == LBP_OK) rc = hip_error(e, "upload event");
        return rc;
    }

    void uploader() {
        (void)hipSetDevice(ctx_.device);
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(umu_);
                ucv_.wait(lk, [&] { return ustop_ || !uq_.empty(); });
                if (uq_.empty()) return;  // stopping with nothing queued
                r = uq_.front();
                uq_.pop_front();
            }
            const int rc = upload(*r);
            {
                std::lock_guard<std::mutex> lk(umu_);
                r->upload_status = rc;
                udone_.push_back(r);
                --upending_;
            }
            udone_cv_.notify_all();
            call_wake();
        }
    }

    // The finisher: reverse sweeps of read-out backward requests on their own
    // stream, so they overlap the worker's rounds.  A request's graph is not
    // touched by the worker while it is here (it is resident but not active).
    void finisher() {
        (void)hipSetDevice(ctx_.device);
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(fmu_);
                fcv_.wait(lk, [&] { return fstop_ || !bq_.empty(); });
                if (bq_.empty()) return;  // stopping with nothing queued
                r = bq_.front();
                bq_.pop_front();
            }
            adjoint_finish_record(r->g);
            int rc = adjoint_backward(r->g, r->gq_dev, r->gphi_dev, nullptr, back_);
            if (rc == LBP_OK) {
                hipError_t e = hipMemcpyAsync(r->gphi, r->gphi_dev, sizeof(float) * r->L.Tn, hipMemcpyDeviceToHost,
                                              back_);
                if (e == hipSuccess) e = hipStreamSynchronize(back_);
                if (e != hipSuccess) rc = hip_error(e, "gradient read-out");
            }
            r->back_status = rc;
            {
                std::lock_guard<std::mutex> lk(fmu_);
                bdone_.push_back(r);
                --fpending_;
            }
            fdone_cv_.notify_all();
            call_wake();
        }
    }

    // Pinned host buffers for results, per power-of-two size class, shared
    // by every server of the process and reused (page-locking is slow, so a
    // new server starts with the buffers earlier ones returned).  At most
    // kIdleCap bytes wait idle; the pool lives until the process ends.
    static constexpr size_t kIdleCap = size_t(512) << 20;
    struct OutPool {
        std::mutex mu;
        std::map<size_t, std::vector<void *>> free_lists;
        size_t idle = 0;
    };
    static OutPool &out_pool() {
        static OutPool *p = new OutPool;
        return *p;
    }
    static size_t size_class(size_t bytes) {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        return c;
    }
    void *pinned_get(size_t bytes) {
        const size_t c = size_class(bytes);
        OutPool &P = out_pool();
        {
            std::lock_guard<std::mutex> lk(P.mu);
            auto &v = P.free_lists[c];
            if (!v.empty()) {
                void *p = v.back();
                v.pop_back();
                P.idle -= c;
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, c) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void pinned_put(void *p, size_t bytes) {
        if (!p) return;
        const size_t c = size_class(bytes);
        OutPool &P = out_pool();
        {
            std::lock_guard<std::mutex> lk(P.mu);
            if (P.idle + c <= kIdleCap) {
                P.free_lists[c].push_back(p);
                P.idle += c;
                return;
            }
        }
        (void)hipHostFree(p);
    }

    // Active graphs sharing (damping, temperature) launch together.
    struct Part {
        float d, T;
        std::vector<DevGraph> hgs;
        LaunchLists ll;
        DevGraph *dgs = nullptr;
        std::vector<Launch> vl, fl;
    };

    int rebuild(const std::vector<Request *> &active) {
        parts_.clear();
        for (Request *r : active) {
            Part *p = nullptr;
            for (Part &q : parts_)
                if (q.d == r->d && q.T == r->T) p = &q;
            if (!p) {
                parts_.push_back(Part{});
                p = &parts_.back();
                p->d = r->d;
                p->T = r->T;
            }
            p->hgs.push_back(r->g->host);
        }
        size_t total = 0;
        std::vector<std::vector<WorkItem>> mids(parts_.size()), highs(parts_.size()), cols(parts_.size());
        for (size_t i = 0; i < parts_.size(); ++i) {
            int32_t gi = 0;
            for (Request *r : active)
                if (r->d == parts_[i].d && r->T == parts_[i].T)
                    add_to_lists(parts_[i].ll, gi++, r->g->shape, &mids[i], &highs[i], &cols[i]);
            finish_lists(parts_[i].ll, mids[i], highs[i], cols[i], true);
            total += align256(sizeof(DevGraph) * parts_[i].hgs.size()) + lists_bytes(parts_[i].ll);
        }
        if (total > stage_bytes_) {
            if (stage_) (void)hipFree(stage_);
            stage_ = nullptr;
            stage_bytes_ = 0;
            hipError_t e = hipMalloc((void **)&stage_, total * 2);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return set_error(LBP_E_OOM, "launch staging buffer");
            }
            stage_bytes_ = total * 2;
        }
        size_t off = 0;
        for (Part &p : parts_) {
            p.dgs = (DevGraph *)(stage_ + off);
            HIP_TRY(hipMemcpyAsync(p.dgs, p.hgs.data(), sizeof(DevGraph) * p.hgs.size(), hipMemcpyHostToDevice,
                                   compute_));
            off += align256(sizeof(DevGraph) * p.hgs.size());
            HIP_TRY(upload_lists(p.ll, stage_ + off, compute_, &p.vl, &p.fl));
            off += lists_bytes(p.ll);
        }
        // the host staging (parts_) lives until the next rebuild, which only
        // happens after the round that used it has been waited for
        return LBP_OK;
    }

    lbp_ctx ctx_{};
    hipStream_t compute_ = nullptr, copy_ = nullptr;
    hipEvent_t ev_ = nullptr;
    char *base_ = nullptr;
    char *stage_ = nullptr;
    size_t stage_bytes_ = 0;
    std::vector<uint64_t> ids_;
    std::vector<Part> parts_;
    float *res_host_ = nullptr;   // pinned, one residual per active slot
    int32_t *flags_host_ = nullptr;  // pinned, one read-out flag per finishing request
    ReadJob *read_host_ = nullptr;   // pinned staging of a read-out batch
    ReadJob *read_dev_ = nullptr;    // its device copy (after res_dev_)
    std::vector<Request *> fin_;     // the batch being read out
    hipStream_t back_ = nullptr;     // the finisher's stream
    hipStream_t read_ = nullptr;     // read-outs of finished requests
    uint64_t read_gen_ = 0;          // uploads the read-out stream was last made to wait for
    std::thread fin_th_;
    std::mutex fmu_;
    std::condition_variable fcv_, fdone_cv_;
    std::deque<Request *> bq_;       // fmu_: waiting for their reverse sweep
    std::vector<Request *> bdone_;   // fmu_: swept, for the worker to complete
    int fpending_ = 0;               // fmu_: handed over and not yet swept
    bool fstop_ = false;             // fmu_
    std::mutex wmu_;                 // guards wake_ and every call of it
    std::function<void()> wake_;
    std::thread up_th_;              // the uploader
    std::mutex umu_;
    std::condition_variable ucv_, udone_cv_;
    std::deque<Request *> uq_;       // umu_: admitted, waiting for the uploader
    std::vector<Request *> udone_;   // umu_: uploads queued, for the worker to take back
    int upending_ = 0;               // umu_: handed over and not yet taken back by the uploader
    bool ustop_ = false;             // umu_
    std::vector<hipEvent_t> ev_pool_;  // umu_: upload events not in use
    uint64_t up_gen_ = 0;            // umu_: uploads issued
    uint64_t up_done_ = 0;           // uploads known to have completed
    uint64_t round_gen_ = 0;         // uploads the compute stream was last made to wait for
    ConvJob *jobs_host_ = nullptr; // pinned staging of the round's checks
    ConvJob *jobs_dev_ = nullptr;  // device copy, followed by res_dev_
    float *res_dev_ = nullptr;
};

}  // namespace

struct lbp_server {
    std::unique_ptr<Executor> exec;
    GpuExecutor *gpu = nullptr;
    Arena arena;
    int32_t max_slots = 1, steps = 5;
    std::mutex mu;
    std::condition_variable cv;        // wakes the worker
    std::condition_variable done_cv;   // wakes drain()
    std::deque<Request *> incoming;    // mu: accepted, in submission order (compiled or not)
    std::deque<Request *> to_prep;     // mu: waiting for a prep thread
    std::condition_variable prep_cv;
    std::vector<std::thread> preps;
    uint64_t next_seq = 0;             // mu
    std::deque<Request *> completed;   // mu
    std::vector<uint64_t> cancels;     // mu
    std::vector<Request *> handed_out; // caller thread: freed at the next poll
    std::deque<Request *> pending;     // worker only
    std::vector<Request *> resident;   // worker only
    int64_t n_in_backward = 0;         // worker only: resident requests with the finisher
    int64_t n_uploading = 0;           // worker only: resident requests with the uploader
    int back_ready = 0;                // mu: finisher completions not yet taken
    bool stop = false;                 // mu
    std::thread th;
    Clock::time_point t0 = Clock::now();
    // statistics (mu)
    int64_t n_submitted = 0, n_finished = 0, n_completed = 0, n_rejected = 0, n_failed = 0, n_cancelled = 0;
    int64_t n_rounds = 0, max_resident = 0;
    int64_t now_resident = 0, now_pending = 0, arena_used = 0, arena_peak = 0;
    double busy_s = 0.0;   // worker: rounds, admissions, read-outs
    double prep_s = 0.0;   // prep threads: compile and check, summed
    double round_s = 0.0;  // worker: launching rounds and waiting for them
    double admit_s = 0.0;  // worker: admissions (arena, outputs, upload enqueue)
    double launch_s = 0.0; // worker: enqueueing rounds (launch lists, kernels)
    double finish_s = 0.0; // worker: read-outs of finished requests, with their wait

    double clock() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    void complete(Request *r, int status) {
        r->status = status;
        r->t_done = clock();
        std::lock_guard<std::mutex> lk(mu);
        ++n_finished;
        if (status == LBP_OK || status == LBP_E_NONFINITE) ++n_completed;
        else if (status == LBP_E_STATE) ++n_cancelled;
        else if (status != LBP_E_BUDGET) ++n_failed;
        completed.push_back(r);
        done_cv.notify_all();
    }

    // Prep threads: compile and check queued descriptions, size the request.
    void prep_loop() {
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                prep_cv.wait(lk, [&] { return stop || !to_prep.empty(); });
                if (stop) return;
                r = to_prep.front();
                to_prep.pop_front();
            }
            int rc = LBP_OK;
            const double tp = clock();
            try {
                std::string err;
                // validates first; the panels go straight into the upload
                // image below when the executor wants one
                rc = compile_desc(&r->desc->d, &r->L, &err, !exec->wants_image());
                if (rc == LBP_OK) rc = check_layout(r->L, &err);
                if (rc == LBP_OK) {
                    r->graph_bytes = graph_device_bytes(r->L, false);
                    r->bytes = Arena::round(r->graph_bytes);
                    if (r->backward) {
                        r->adj_bytes = adjoint_bytes(r->L.M, r->L.VB, r->L.P, r->iters, r->k);
                        r->bytes += Arena::round(r->adj_bytes) + Arena::round(sizeof(float) * r->L.VS) +
                                    Arena::round(sizeof(float) * r->L.Tn);
                    }
                    if (r->tol >= 0.0f) {
                        r->conv_bytes = align256(sizeof(float) * std::max<int64_t>(1, r->L.M)) +
                                        sizeof(float) * (residual_blocks((int)r->L.E) + 1);
                        r->bytes += Arena::round(r->conv_bytes);
                    }
                    if (r->bytes > arena.capacity()) rc = LBP_E_BUDGET;
                }
                if (rc == LBP_OK && exec->wants_image()) {
                    // pack the upload here, off the worker thread, with the
                    // evidence and potential panels written in place
                    if (r->desc->lp_bad >= 0) {
                        rc = nonfinite_potential(r->desc->lp_bad, &err);
                    } else {
                        r->image.reset((char *)panel_alloc(graph_image_bytes(r->L)));
                        if (!r->image) throw std::bad_alloc();
                        rc = graph_fill_image(r->L, r->image.get(), &r->desc->d);
                        r->lp = std::move(r->desc->lp);
                    }
                    std::vector<int32_t>().swap(r->L.tile_fac);
                    if (rc != LBP_OK) {
                        r->image.reset();
                        r->lp.reset();
                    }
                }
            } catch (const std::bad_alloc &) {
                rc = LBP_E_OOM;
            }
            r->desc.reset();
            const double tn = clock();
            r->t_ready = tn;
            std::lock_guard<std::mutex> lk(mu);
            prep_s += tn - tp;
            r->prep = rc == LBP_OK ? 1 : 2;
            r->prep_status = rc;
            cv.notify_one();
        }
    }

    bool head_ready() const { return !pending.empty() && pending.front()->prep != 0; }

    void drop_resident(Request *r) {
        exec->release(*r);
        arena.release(r->off, r->bytes);
    }

    void admit() {
        const double t0 = clock();
        admit_loop();
        std::lock_guard<std::mutex> lk(mu);
        admit_s += clock() - t0;
    }

    void admit_loop() {
        while (!pending.empty() && (int32_t)resident.size() < max_slots) {
            Request *r = pending.front();
            int prep;
            {
                std::lock_guard<std::mutex> lk(mu);
                prep = r->prep;
            }
            if (prep == 0) break;  // first in, first out: wait for its compile
            if (r->cancel) {
                pending.pop_front();
                complete(r, LBP_E_STATE);
                continue;
            }
            if (prep == 2) {
                pending.pop_front();
                if (r->prep_status == LBP_E_BUDGET) {
                    std::lock_guard<std::mutex> lk(mu);
                    ++n_rejected;
                }
                complete(r, r->prep_status);
                continue;
            }
            const size_t off = arena.alloc(r->bytes);
            if (off == Arena::kNone) {
                if (resident.empty() && arena.used() == 0) {
                    // cannot fit even an empty arena (requests are checked
                    // against the budget at submit, so this is a guard only)
                    pending.pop_front();
                    complete(r, LBP_E_BUDGET);
                    continue;
                }
                break;  // first in, first out: wait for memory
            }
            pending.pop_front();
            r->off = off;
            int rc = exec->alloc_outputs(*r);
            if (rc == LBP_OK) rc = exec->admit(*r);
            if (rc != LBP_OK) {
                if (r->g) exec->release(*r);
                arena.release(off, r->bytes);
                complete(r, rc);
                continue;
            }
            r->t_admit = clock();
            if (r->uploading) ++n_uploading;
            resident.push_back(r);
        }
    }

    // Requests the uploader has handed back; those whose upload failed leave.
    void take_uploaded() {
        std::vector<Request *> up;
        exec->take_uploaded(up);
        for (Request *r : up) {
            r->uploading = false;
            --n_uploading;
            if (r->upload_status != LBP_OK) {
                drop_resident(r);
                resident.erase(std::find(resident.begin(), resident.end(), r));
                complete(r, r->upload_status);
            }
        }
    }

    void update_stats() {
        std::lock_guard<std::mutex> lk(mu);
        now_resident = (int64_t)resident.size();
        now_pending = (int64_t)pending.size();
        max_resident = std::max(max_resident, now_resident);
        arena_used = (int64_t)arena.used();
        arena_peak = (int64_t)arena.peak();
    }

    // The worker keeps at most one round in flight.  After waiting for it,
    // it launches the next round first and then, while that runs, reads out
    // the requests the finished round completed (on their own stream) and
    // admits new ones, so the GPU is idle only between a round's end and the
    // next launch.
    void run() {
        if (gpu) gpu->bind();
        std::vector<Request *> inflight;  // the round in flight
        int32_t inflight_s = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                if (inflight.empty())
                    cv.wait(lk, [&] {
                        return stop || !incoming.empty() || (int64_t)resident.size() > n_in_backward + n_uploading ||
                               !cancels.empty() || back_ready > 0 || (!pending.empty() && pending.front()->prep != 0);
                    });
                if (stop) break;
                back_ready = 0;
                while (!incoming.empty()) {
                    pending.push_back(incoming.front());
                    incoming.pop_front();
                }
                for (uint64_t id : cancels) {
                    for (Request *r : pending)
                        if (r->id == id) r->cancel = true;
                    for (Request *r : resident)
                        if (r->id == id) r->cancel = true;
                }
                cancels.clear();
            }
            const double tl = clock();
            // the round in flight ends
            if (!inflight.empty()) {
                const double tw = clock();
                int rc = exec->wait();
                {
                    std::lock_guard<std::mutex> lk(mu);
                    round_s += clock() - tw;
                }
                if (rc != LBP_OK) {
                    for (Request *r : inflight) {
                        drop_resident(r);
                        resident.erase(std::find(resident.begin(), resident.end(), r));
                        complete(r, rc);
                    }
                } else {
                    exec->residuals(inflight);
                    exec->images_done(resident);
                    for (Request *r : inflight) {
                        r->done += inflight_s;
                        if (r->check_now && r->residual < r->tol) r->settled = true;
                    }
                    std::lock_guard<std::mutex> lk(mu);
                    ++n_rounds;
                }
                inflight.clear();
            }
            take_uploaded();
            // requests whose reverse sweep has finished leave
            {
                std::vector<Request *> swept;
                exec->take_backward(swept);
                for (Request *r : swept) {
                    r->in_backward = false;
                    --n_in_backward;
                    drop_resident(r);
                    resident.erase(std::find(resident.begin(), resident.end(), r));
                    complete(r, r->back_status);
                }
            }
            // cancelled resident requests leave at this round boundary (those
            // with the finisher complete when their sweep does, those with
            // the uploader once it hands them back)
            for (size_t i = 0; i < resident.size();) {
                if (resident[i]->cancel && !resident[i]->in_backward && !resident[i]->uploading) {
                    Request *r = resident[i];
                    drop_resident(r);
                    resident.erase(resident.begin() + i);
                    complete(r, LBP_E_STATE);
                } else {
                    ++i;
                }
            }
            admit();
            update_stats();
            // the next round
            std::vector<Request *> active;
            int32_t s = steps;
            for (Request *r : resident)
                if (r->done < r->iters && !r->settled && !r->uploading) {
                    active.push_back(r);
                    s = std::min(s, r->iters - r->done);
                    if (r->backward) s = std::min(s, r->k - r->done % r->k);
                    if (r->tol >= 0.0f) s = std::min(s, r->check - r->done % r->check);
                }
            for (Request *r : active)
                r->check_now = r->tol >= 0.0f && ((r->done + s) % r->check == 0 || r->done + s == r->iters);
            if (!active.empty()) {
                const double tr = clock();
                int rc = exec->round(active, s);
                {
                    std::lock_guard<std::mutex> lk(mu);
                    launch_s += clock() - tr;
                    round_s += clock() - tr;
                }
                if (rc != LBP_OK) {
                    // whatever of it was queued ends before its memory is reused
                    exec->quiesce();
                    for (Request *r : active) {
                        drop_resident(r);
                        resident.erase(std::find(resident.begin(), resident.end(), r));
                        complete(r, rc);
                    }
                } else {
                    inflight = active;
                    inflight_s = s;
                }
            }
            // finished requests (none is in the round just launched): all
            // read-outs queued, one wait, then each leaves (its memory is
            // reused only after the wait)
            std::vector<Request *> fin;
            for (Request *r : resident)
                if ((r->done >= r->iters || r->settled) && !r->in_backward && !r->uploading) fin.push_back(r);
            if (!fin.empty()) {
                const double tf = clock();
                std::vector<int> rcs(fin.size(), LBP_OK);
                for (size_t i = 0; i < fin.size(); ++i) rcs[i] = exec->finish_begin(*fin[i], (int32_t)i);
                const int wrc = exec->finish_wait();
                for (size_t i = 0; i < fin.size(); ++i) {
                    Request *r = fin[i];
                    int rc = rcs[i] != LBP_OK ? rcs[i] : wrc != LBP_OK ? wrc : exec->finish_end(*r, (int32_t)i);
                    if (rc == LBP_OK && r->backward && exec->start_backward(*r)) {
                        r->in_backward = true;  // stays resident until its sweep is done
                        ++n_in_backward;
                        continue;
                    }
                    drop_resident(r);
                    resident.erase(std::find(resident.begin(), resident.end(), r));
                    complete(r, rc);
                }
                std::lock_guard<std::mutex> lk(mu);
                finish_s += clock() - tf;
            }
            admit();  // slots and memory the read-outs freed
            {
                std::lock_guard<std::mutex> lk(mu);
                busy_s += clock() - tl;
            }
            update_stats();
        }
        // a round still in flight ends first
        if (!inflight.empty()) (void)exec->wait();
        // shutting down: uploads and sweeps under way finish, everything else
        // is cancelled
        exec->drain_uploads();
        take_uploaded();
        exec->drain_backward();
        {
            std::vector<Request *> swept;
            exec->take_backward(swept);
            for (Request *r : swept) {
                r->in_backward = false;
                drop_resident(r);
                resident.erase(std::find(resident.begin(), resident.end(), r));
                complete(r, r->back_status);
            }
        }
        for (Request *r : resident) {
            drop_resident(r);
            complete(r, LBP_E_STATE);
        }
        resident.clear();
        for (Request *r : pending) complete(r, LBP_E_STATE);
        pending.clear();
    }
};

namespace {

int server_create(lbp_ctx *ctx, int64_t budget, int32_t max_slots, int32_t steps, bool on_gpu, lbp_server **out) {
    if (!out) return set_error(LBP_E_INVALID, "out is NULL");
    if (budget <= 0 || max_slots < 1 || steps < 1)
        return set_error(LBP_E_INVALID, "budget, max_slots and steps_per_round must be positive");
    try {
        std::unique_ptr<lbp_server> s(new lbp_server);
        s->arena = Arena((size_t)budget);
        s->max_slots = max_slots;
        s->steps = steps;
        if (on_gpu) {
            if (!ctx) return set_error(LBP_E_INVALID, "ctx is NULL");
            std::unique_ptr<GpuExecutor> g(new GpuExecutor);
            int rc = g->init(ctx->device, (size_t)budget, max_slots);
            if (rc != LBP_OK) return rc;
            s->gpu = g.get();
            s->exec = std::move(g);
        } else {
            s->exec.reset(new HostExecutor);
        }
        lbp_server *raw = s.get();
        s->exec->set_wake([raw] {
            std::lock_guard<std::mutex> lk(raw->mu);
            ++raw->back_ready;
            raw->cv.notify_one();
        });
        s->th = std::thread([raw] { raw->run(); });
        // preparation threads: half the CPUs this process may run on, at
        // most 8 (more contend for host memory bandwidth and run slower);
        // LBP_SERVER_PREP_THREADS (1..64) overrides the count
        unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        cpu_set_t set;
        if (sched_getaffinity(0, sizeof(set), &set) == 0) hw = std::max(1, CPU_COUNT(&set));
        unsigned np = std::min(8u, std::max(1u, hw / 2));
        if (const char *env = getenv("LBP_SERVER_PREP_THREADS")) {
            const long v = strtol(env, nullptr, 10);
            if (v >= 1 && v <= 64) np = (unsigned)v;
        }
        for (unsigned i = 0; i < np; ++i) s->preps.emplace_back([raw] { raw->prep_loop(); });
        *out = s.release();
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        return set_error(LBP_E_OOM, "host allocation failed");
    } catch (const std::system_error &) {
        return set_error(LBP_E_OOM, "could not start the server thread");
    }
}

}  // namespace

extern "C" {

int lbp_server_create(lbp_ctx *ctx, int64_t hbm_budget_bytes, int32_t max_slots, int32_t steps_per_round,
                      lbp_server **out) {
    return server_create(ctx, hbm_budget_bytes, max_slots, steps_per_round, true, out);
}

int lbp_server_create_host_only(int64_t budget_bytes, int32_t max_slots, int32_t steps_per_round, lbp_server **out) {
    return server_create(nullptr, budget_bytes, max_slots, steps_per_round, false, out);
}

double lbp_server_clock(const lbp_server *s) { return s ? s->clock() : 0.0; }

}  // extern "C"

namespace {

int submit(lbp_server *s, const lbp_graph_desc *desc, int32_t iters, float damping, float temperature,
           const float *grad_q, int32_t ckpt_every, float tol, int32_t check_every, double t_arrival,
           uint64_t req_id) {
    if (!s) return set_error(LBP_E_INVALID, "server is NULL");
    std::string why;
    if (!valid_params(iters, damping, temperature, &why)) return set_error(LBP_E_INVALID, why);
    try {
        // sizes only (full validation runs on the prep threads)
        if (!desc) return set_error(LBP_E_INVALID, "graph description is NULL");
        int64_t sz[6] = {desc->num_vars, 0, desc->num_factors, 0, 0, 0};
        if (sz[0] < 0 || sz[2] < 0 || desc->num_cfg_tables < 0)
            return set_error(LBP_E_INVALID, "negative num_vars, num_factors or num_cfg_tables");
        if ((sz[0] > 0 && !desc->var_num_states) || !desc->factor_edge_off || !desc->logpot_off ||
            (sz[2] > 0 && (!desc->factor_kind || !desc->factor_cfg_table)) ||
            (desc->num_cfg_tables > 0 && (!desc->cfg_table_num_cfgs || !desc->cfg_table_arity || !desc->cfg_table_off)))
            return set_error(LBP_E_INVALID, "a required array is NULL");
        for (int64_t v = 0; v < sz[0]; ++v) {
            const int32_t n = desc->var_num_states[v];
            if (n < 2 || n > kMaxStates) return set_error(LBP_E_INVALID, "var_num_states outside [2, 64]");
            sz[1] += n;
        }
        sz[3] = desc->factor_edge_off[sz[2]];
        sz[5] = desc->logpot_off[sz[2]];
        const int64_t nts = desc->num_cfg_tables > 0 ? desc->cfg_table_off[desc->num_cfg_tables] : 0;
        if (desc->factor_edge_off[0] != 0 || sz[3] < 0 || sz[3] > INT32_MAX || desc->logpot_off[0] != 0 ||
            sz[5] < 0 || nts < 0 || (sz[3] > 0 && !desc->edge_var) || (sz[5] > 0 && !desc->log_potentials) ||
            (nts > 0 && !desc->cfg_table_states))
            return set_error(LBP_E_INVALID, "malformed offsets");
        std::unique_ptr<Request> r(new Request);
        r->id = req_id;
        r->iters = iters;
        r->d = damping;
        r->T = temperature;
        r->backward = grad_q != nullptr;
        r->t_arrival = t_arrival >= 0.0 ? t_arrival : s->clock();
        if (tol >= 0.0f) {
            r->tol = tol;
            r->check = check_every;
            r->residual = 0.0f;
        }
        if (r->backward) {
            if (!(temperature > 0.0f)) return set_error(LBP_E_INVALID, "backward requests need temperature > 0");
            if (ckpt_every < 1) return set_error(LBP_E_INVALID, "ckpt_every must be >= 1");
            for (int64_t f = 0; f < sz[2]; ++f)
                if (desc->factor_kind[f] != LBP_FACTOR_ENUM)
                    return set_error(LBP_E_UNSUPPORTED, "the adjoint supports enumeration factors only");
            r->k = ckpt_every;
            r->grad_q.assign(grad_q, grad_q + sz[1]);
        }
        r->desc.reset(new DescCopy);
        r->desc->take(desc, sz);
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return set_error(LBP_E_STATE, "server is shutting down");
        ++s->n_submitted;
        r->seq = s->next_seq++;
        Request *raw = r.release();
        s->incoming.push_back(raw);
        s->to_prep.push_back(raw);
        s->prep_cv.notify_one();
        s->cv.notify_one();
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        return set_error(LBP_E_OOM, "host allocation failed");
    }
}

}  // namespace

extern "C" {

int lbp_server_submit(lbp_server *s, const lbp_graph_desc *desc, int32_t iters, float damping, float temperature,
                      const float *grad_q, int32_t ckpt_every, double t_arrival, uint64_t req_id) {
    return submit(s, desc, iters, damping, temperature, grad_q, ckpt_every, -1.0f, 0, t_arrival, req_id);
}

int lbp_server_submit_until(lbp_server *s, const lbp_graph_desc *desc, int32_t max_iters, float damping,
                            float temperature, float tol, int32_t check_every, double t_arrival, uint64_t req_id) {
    if (!(tol >= 0.0f) || !std::isfinite(tol)) return set_error(LBP_E_INVALID, "tol must be finite and >= 0");
    if (check_every < 1) return set_error(LBP_E_INVALID, "check_every must be >= 1");
    return submit(s, desc, max_iters, damping, temperature, nullptr, 10, tol, check_every, t_arrival, req_id);
}

int lbp_server_cancel(lbp_server *s, uint64_t req_id) {
    if (!s) return set_error(LBP_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->cancels.push_back(req_id);
    s->cv.notify_one();
    return LBP_OK;
}

int lbp_server_poll(lbp_server *s, lbp_completion *out, int32_t max, int32_t *n_out) {
    if (!s || !n_out || (max > 0 && !out)) return set_error(LBP_E_INVALID, "bad poll arguments");
    for (Request *r : s->handed_out) {
        s->exec->free_outputs(*r);
        delete r;
    }
    s->handed_out.clear();
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t n = 0;
    while (n < max && !s->completed.empty()) {
        Request *r = s->completed.front();
        s->completed.pop_front();
        lbp_completion &c = out[n++];
        std::memset(&c, 0, sizeof(c));
        c.req_id = r->id;
        c.status = r->status;
        c.num_vars = r->L.V;
        c.num_var_states = r->L.VS;
        c.num_logpots = r->L.Tn;
        const bool ok = r->status == LBP_OK || r->status == LBP_E_NONFINITE;
        c.beliefs = ok ? r->q : nullptr;
        c.map = ok ? r->map : nullptr;
        c.grad_logpot = ok && r->backward ? r->gphi : nullptr;
        c.t_arrival = r->t_arrival;
        c.t_ready = r->t_ready;
        c.t_admit = r->t_admit;
        c.t_done = r->t_done;
        c.iters_done = r->done;
        c.residual = r->residual;
        s->handed_out.push_back(r);
    }
    *n_out = n;
    return LBP_OK;
}

int lbp_server_drain(lbp_server *s, double timeout_s) {
    if (!s) return set_error(LBP_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->done_cv.wait_for(lk, std::chrono::duration<double>(std::max(0.0, timeout_s)),
                                        [&] { return s->n_finished >= s->n_submitted; });
    return ok ? LBP_OK : set_error(LBP_E_STATE, "drain timed out");
}

int lbp_server_stats(lbp_server *s, int64_t out[18]) {
    if (!s || !out) return set_error(LBP_E_INVALID, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->n_submitted;
    out[1] = s->n_finished;
    out[2] = s->n_completed;
    out[3] = s->n_rejected;
    out[4] = s->n_failed;
    out[5] = s->n_cancelled;
    out[6] = s->n_rounds;
    out[7] = s->now_resident;
    out[8] = s->now_pending;
    out[9] = s->max_resident;
    out[10] = s->arena_peak;
    out[11] = (int64_t)(s->busy_s * 1e6);
    out[12] = (int64_t)(s->round_s * 1e6);
    out[13] = (int64_t)(s->prep_s * 1e6);
    out[14] = (int64_t)s->preps.size();
    out[15] = (int64_t)(s->admit_s * 1e6);
    out[16] = (int64_t)(s->launch_s * 1e6);
    out[17] = (int64_t)(s->finish_s * 1e6);
    return LBP_OK;
}

void lbp_server_destroy(lbp_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->prep_cv.notify_all();
    if (s->th.joinable()) s->th.join();
    for (std::thread &t : s->preps)
        if (t.joinable()) t.join();
    s->exec->set_wake(nullptr);  // the worker is gone; nothing is left to wake
    for (Request *r : s->handed_out) {
        s->exec->free_outputs(*r);
        delete r;
    }
    for (Request *r : s->completed) {
        s->exec->free_outputs(*r);
        delete r;
    }
    for (Request *r : s->incoming) delete r;
    delete s;
}

}  // extern "C"
