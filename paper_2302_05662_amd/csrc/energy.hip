// Energy, average power and efficiency of an SpMV.
//
// The paper measures, beside latency, the energy, the average power and the
// efficiency (MFLOPS per watt) of each kernel run, sampling the board sensors
// while the kernel repeats (Experimental Setup, GPU performance monitoring),
// and finds that the format moves power and efficiency even where it does not
// move latency (Results of the run-time optimisation mode).
//
// On MI355X the board exposes a monotone energy accumulator (amd-smi) that the
// firmware advances about once a second. A measurement keeps the
// stream fed with batches of back-to-back runs, polls the counter until it
// moves, keeps running for at least the asked duration and polls until it moves
// again, so the interval between the two updates lies entirely inside the busy
// period. The interval is taken from the host clock at the two detections (the
// firmware stamp returned with the counter does not advance with every update;
// polling every 0.5 ms bounds the error; an interval implying more than 5 kW
// holds a bad reading and is measured again). Average power is the energy difference
// over that interval; the time of one run comes from HIP events around every
// batch, and the energy of one run is their product.
#include <amd_smi/amdsmi.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"

namespace spmv {
namespace {

constexpr int kMaxDev = 64;

struct Smi {
    std::mutex mu;
    bool initialised = false;
    std::string init_error;
    bool looked_up[kMaxDev] = {};
    amdsmi_processor_handle proc[kMaxDev] = {};
};

Smi &smi() {
    static Smi *s = new Smi();  // lives until process exit
    return *s;
}

// amd-smi's packed PCI id: domain << 32 | bus << 8 | device << 3 | function.
uint64_t pci_id_of_current_device(int dev) {
    char bus[64] = {};
    SPMV_HIP(hipDeviceGetPCIBusId(bus, (int)sizeof bus, dev));
    unsigned dom = 0, b = 0, d = 0, fn = 0;
    if (std::sscanf(bus, "%x:%x:%x.%x", &dom, &b, &d, &fn) != 4)
        fail(SPMV_ERR_HIP, "cannot parse PCI bus id '%s'", bus);
    return ((uint64_t)dom << 32) | ((uint64_t)b << 8) | ((uint64_t)(d & 31) << 3) | (fn & 7);
}

// The amd-smi processor of the current HIP device (matched by PCI id).
amdsmi_processor_handle energy_source() {
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) fail(SPMV_ERR_INVALID_ARG, "device id %d", dev);
    Smi &S = smi();
    std::lock_guard<std::mutex> lk(S.mu);
    if (!S.initialised) {
        const amdsmi_status_t st = amdsmi_init(AMDSMI_INIT_AMD_GPUS);
        S.initialised = true;
        if (st != AMDSMI_STATUS_SUCCESS) S.init_error = "amdsmi_init returned " + std::to_string((int)st);
    }
    if (!S.init_error.empty()) fail(SPMV_ERR_NOT_APPLICABLE, "no energy counter: %s", S.init_error.c_str());
    if (!S.looked_up[dev]) {
        const uint64_t want = pci_id_of_current_device(dev);
        uint32_t ns = 0;
        if (amdsmi_get_socket_handles(&ns, nullptr) != AMDSMI_STATUS_SUCCESS)
            fail(SPMV_ERR_NOT_APPLICABLE, "no energy counter: amd-smi lists no sockets");
        std::vector<amdsmi_socket_handle> socks(ns);
        amdsmi_get_socket_handles(&ns, socks.data());
        for (uint32_t i = 0; i < ns && !S.proc[dev]; ++i) {
            uint32_t np = 0;
            if (amdsmi_get_processor_handles(socks[i], &np, nullptr) != AMDSMI_STATUS_SUCCESS) continue;
            std::vector<amdsmi_processor_handle> p(np);
            amdsmi_get_processor_handles(socks[i], &np, p.data());
            for (auto ph : p) {
                uint64_t id = 0;
                if (amdsmi_get_gpu_bdf_id(ph, &id) == AMDSMI_STATUS_SUCCESS && id == want) {
                    S.proc[dev] = ph;
                    break;
                }
            }
        }
        S.looked_up[dev] = true;
    }
    if (!S.proc[dev])
        fail(SPMV_ERR_NOT_APPLICABLE, "no energy counter: amd-smi has no GPU at the PCI id of device %d", dev);
    return S.proc[dev];
}

using Clock = std::chrono::steady_clock;

// One reading of the accumulator, stamped with the host clock when it was taken
// (the firmware stamp that comes with it does not advance with every update).
struct Reading {
    uint64_t ticks = 0;
    double uj_per_tick = 0;
    Clock::time_point at;
};

Reading read_counter(amdsmi_processor_handle p) {
    Reading r;
    float res = 0.f;
    uint64_t fw_ns = 0;
    const amdsmi_status_t st = amdsmi_get_energy_count(p, &r.ticks, &res, &fw_ns);
    r.at = Clock::now();
    if (st != AMDSMI_STATUS_SUCCESS)
        fail(SPMV_ERR_NOT_APPLICABLE, "amdsmi_get_energy_count returned %d", (int)st);
    r.uj_per_tick = res;
    return r;
}
constexpr double kEdgeTimeoutS = 3.0;  // the counter advances about once a second
constexpr int kPollUs = 500;            // between counter reads
constexpr double kMaxWatts = 5000.0;    // above any board's draw: a reading past it is a glitch
constexpr int kAttempts = 3;

// Keeps `s` fed with batches of `batch` runs while polling the counter.
struct Feeder {
    const spmv_matrix_s *h;
    spmv_format f;
    int32_t variant;
    const void *x;
    void *y;
    hipStream_t s;
    int64_t batch;
    std::deque<hipEvent_t> pending;  // end events of enqueued, unfinished batches
    std::vector<hipEvent_t> all;     // every event, for timing and destruction
    int64_t runs = 0;

    ~Feeder() {
        for (auto e : all) (void)hipEventDestroy(e);
    }
    hipEvent_t record() {
        hipEvent_t e = nullptr;
        SPMV_HIP(hipEventCreate(&e));
        all.push_back(e);
        SPMV_HIP(hipEventRecord(e, s));
        return e;
    }
    // Enqueue until two batches are outstanding.
    void top_up() {
        while (!pending.empty()) {
            const hipError_t q = hipEventQuery(pending.front());
            if (q == hipErrorNotReady) break;
            SPMV_HIP(q);
            pending.pop_front();
        }
        while (pending.size() < 2) {
            for (int64_t i = 0; i < batch; ++i) launch_spmv(h, f, variant, 1.0, x, 0.0, y, s);
            runs += batch;
            pending.push_back(record());
        }
    }
    // Wait (feeding the stream) until the counter moves past `prev`.
    Reading next_update(amdsmi_processor_handle p, uint64_t prev) {
        const auto t0 = Clock::now();
        for (;;) {
            top_up();
            const Reading r = read_counter(p);
            if (r.ticks != prev) return r;
            if (std::chrono::duration<double>(Clock::now() - t0).count() > kEdgeTimeoutS)
                fail(SPMV_ERR_NOT_APPLICABLE, "energy counter did not advance in %.0f s", kEdgeTimeoutS);
            std::this_thread::sleep_for(std::chrono::microseconds(kPollUs));
        }
    }
};

// Waits without work of ours until the counter moves past `prev`.
Reading next_update_idle(amdsmi_processor_handle p, uint64_t prev) {
    const auto t0 = Clock::now();
    for (;;) {
        const Reading r = read_counter(p);
        if (r.ticks != prev) return r;
        if (std::chrono::duration<double>(Clock::now() - t0).count() > kEdgeTimeoutS)
            fail(SPMV_ERR_NOT_APPLICABLE, "energy counter did not advance in %.0f s", kEdgeTimeoutS);
        std::this_thread::sleep_for(std::chrono::microseconds(kPollUs));
    }
}

double seconds_since(Clock::time_point t0) {
    return std::chrono::duration<double>(Clock::now() - t0).count();
}

}  // namespace

void check_runnable(const spmv_matrix_s *h, spmv_format f);  // api.hip
void check_vectors(const spmv_matrix_s *h, const void *x, const void *y);  // api.hip

void measure_energy(spmv_matrix_s *h, spmv_format f, int32_t variant, const void *x, void *y,
                    double seconds, double warm_seconds, spmv_energy_result *out, hipStream_t s) {
    amdsmi_processor_handle p = energy_source();
    // time of one run, to size batches of about 2 ms
    Feeder fd{h, f, variant, x, y, s, 1, {}, {}, 0};
    for (int i = 0; i < 3; ++i) launch_spmv(h, f, variant, 1.0, x, 0.0, y, s);
    hipEvent_t a = fd.record();
    constexpr int kProbe = 16;
    for (int i = 0; i < kProbe; ++i) launch_spmv(h, f, variant, 1.0, x, 0.0, y, s);
    hipEvent_t b = fd.record();
    SPMV_HIP(hipStreamSynchronize(s));
    float probe_ms = 0.f;
    SPMV_HIP(hipEventElapsedTime(&probe_ms, a, b));
    const double run_ms = std::max(1e-4, (double)probe_ms / kProbe);
    fd.batch = std::max<int64_t>(1, std::min<int64_t>(1 << 20, (int64_t)std::ceil(2.0 / run_ms)));

    // warm period: clocks and power settle under the load
    const auto t_warm = Clock::now();
    while (seconds_since(t_warm) < warm_seconds) {
        fd.top_up();
        std::this_thread::sleep_for(std::chrono::microseconds(kPollUs));
    }
    // An interval whose energy implies more than kMaxWatts (or none) holds a bad
    // reading; it is measured again, the stream still busy.
    for (int attempt = 0; attempt < kAttempts; ++attempt) {
        const Reading r_prev = read_counter(p);
        const Reading r0 = fd.next_update(p, r_prev.ticks);
        const int64_t runs0 = fd.runs;
        hipEvent_t e0 = fd.record();  // after every batch enqueued before the first update
        const auto t_meas = Clock::now();
        while (seconds_since(t_meas) < seconds) {
            fd.top_up();
            std::this_thread::sleep_for(std::chrono::microseconds(kPollUs));
        }
        const Reading r_last = read_counter(p);
        const Reading r1 = fd.next_update(p, r_last.ticks);
        hipEvent_t e1 = fd.record();
        const int64_t runs1 = fd.runs;
        const double dt = std::chrono::duration<double>(r1.at - r0.at).count();
        const double joules = r1.ticks > r0.ticks
                                  ? (double)(r1.ticks - r0.ticks) * r0.uj_per_tick * 1e-6 : -1.0;
        if (!(dt > 0) || !(joules > 0) || joules / dt > kMaxWatts) continue;
        SPMV_HIP(hipStreamSynchronize(s));
        float loop_ms = 0.f;
        SPMV_HIP(hipEventElapsedTime(&loop_ms, e0, e1));
        out->seconds = dt;
        out->joules = joules;
        out->watts = joules / dt;
        out->runs = runs1 - runs0;
        out->ms_per_run = out->runs > 0 ? loop_ms / (double)out->runs : 0.0;
        out->joules_per_run = out->watts * out->ms_per_run * 1e-3;
        out->mflops_per_watt =
            out->joules_per_run > 0 ? 2.0 * (double)h->nnz / out->joules_per_run * 1e-6 : 0.0;
        return;
    }
    SPMV_HIP(hipStreamSynchronize(s));
    fail(SPMV_ERR_NOT_APPLICABLE, "energy counter gave no consistent interval in %d attempts",
         kAttempts);
}

// Several formats in one sweep: one warm period and one counter update, then each
// format runs from one update to the next (at least `seconds` apart), the update
// that ends a format's interval starting the next one's, so a sweep of F formats
// takes about F update periods. Batches last about 1 ms, so the runs of one format
// that spill past its closing update are a small share of the next interval. An
// interval that fails the consistency check is measured again on its own.
void measure_energy_sweep(spmv_matrix_s *h, int32_t count, const spmv_format *fmts,
                          const int32_t *variants, const void *x, void *y, double seconds,
                          spmv_energy_result *out, hipStream_t s) {
    amdsmi_processor_handle p = energy_source();
    std::vector<int64_t> batch(count);
    for (int32_t i = 0; i < count; ++i) {
        Feeder probe{h, fmts[i], variants[i], x, y, s, 1, {}, {}, 0};
        for (int k = 0; k < 2; ++k) launch_spmv(h, fmts[i], variants[i], 1.0, x, 0.0, y, s);
        hipEvent_t a = probe.record();
        constexpr int kProbe = 8;
        for (int k = 0; k < kProbe; ++k) launch_spmv(h, fmts[i], variants[i], 1.0, x, 0.0, y, s);
        hipEvent_t b = probe.record();
        SPMV_HIP(hipStreamSynchronize(s));
        float ms = 0.f;
        SPMV_HIP(hipEventElapsedTime(&ms, a, b));
        const double run_ms = std::max(1e-4, (double)ms / kProbe);
        batch[i] = std::max<int64_t>(1, std::min<int64_t>(1 << 20, (int64_t)std::ceil(1.0 / run_ms)));
    }
    Feeder fd{h, fmts[0], variants[0], x, y, s, batch[0], {}, {}, 0};
    const auto t_warm = Clock::now();
    while (seconds_since(t_warm) < 0.1) {
        fd.top_up();
        std::this_thread::sleep_for(std::chrono::microseconds(kPollUs));
    }
    const Reading r_prev = read_counter(p);
    Reading r_start = fd.next_update(p, r_prev.ticks);
    hipEvent_t e_start = fd.record();
    struct Span { hipEvent_t e0, e1; int64_t runs; bool ok; };
    std::vector<Span> spans(count);
    for (int32_t i = 0; i < count; ++i) {
        fd.f = fmts[i];
        fd.variant = variants[i];
        fd.batch = batch[i];
        const int64_t runs0 = fd.runs;
        const auto t_meas = Clock::now();
        while (seconds_since(t_meas) < seconds) {
            fd.top_up();
            std::this_thread::sleep_for(std::chrono::microseconds(kPollUs));
        }
        const Reading r_last = read_counter(p);
        const Reading r_end = fd.next_update(p, r_last.ticks);
        hipEvent_t e_end = fd.record();
        const double dt = std::chrono::duration<double>(r_end.at - r_start.at).count();
        const double joules = r_end.ticks > r_start.ticks
                                  ? (double)(r_end.ticks - r_start.ticks) * r_start.uj_per_tick * 1e-6
                                  : -1.0;
        spans[i] = {e_start, e_end, fd.runs - runs0, dt > 0 && joules > 0 && joules / dt <= kMaxWatts};
        if (spans[i].ok) {
            out[i].seconds = dt;
            out[i].joules = joules;
            out[i].watts = joules / dt;
            out[i].runs = spans[i].runs;
        }
        r_start = r_end;
        e_start = e_end;
    }
    SPMV_HIP(hipStreamSynchronize(s));
    for (int32_t i = 0; i < count; ++i) {
        if (!spans[i].ok) {
            measure_energy(h, fmts[i], variants[i], x, y, seconds, 0.05, &out[i], s);
            continue;
        }
        float loop_ms = 0.f;
        SPMV_HIP(hipEventElapsedTime(&loop_ms, spans[i].e0, spans[i].e1));
        out[i].ms_per_run = out[i].runs > 0 ? loop_ms / (double)out[i].runs : 0.0;
        out[i].joules_per_run = out[i].watts * out[i].ms_per_run * 1e-3;
        out[i].mflops_per_watt =
            out[i].joules_per_run > 0 ? 2.0 * (double)h->nnz / out[i].joules_per_run * 1e-6 : 0.0;
    }
}

void measure_idle_power(double seconds, double *watts) {
    amdsmi_processor_handle p = energy_source();
    SPMV_HIP(hipDeviceSynchronize());
    for (int attempt = 0; attempt < kAttempts; ++attempt) {
        const Reading r_prev = read_counter(p);
        const Reading r0 = next_update_idle(p, r_prev.ticks);
        std::this_thread::sleep_for(std::chrono::duration<double>(seconds));
        const Reading r_last = read_counter(p);
        const Reading r1 = next_update_idle(p, r_last.ticks);
        const double dt = std::chrono::duration<double>(r1.at - r0.at).count();
        const double joules = r1.ticks > r0.ticks
                                  ? (double)(r1.ticks - r0.ticks) * r0.uj_per_tick * 1e-6 : -1.0;
        if (!(dt > 0) || !(joules > 0) || joules / dt > kMaxWatts) continue;
        *watts = joules / dt;
        return;
    }
    fail(SPMV_ERR_NOT_APPLICABLE, "energy counter gave no consistent interval in %d attempts",
         kAttempts);
}

}  // namespace spmv

using namespace spmv;

extern "C" spmv_status spmv_energy(spmv_handle h, spmv_format f, int32_t variant, const void *x,
                                   void *y, double seconds, spmv_energy_result *out, void *stream) {
    return guard([&] {
        check_runnable(h, f);
        if (!out) fail(SPMV_ERR_INVALID_ARG, "NULL result");
        if (!(seconds > 0.0) || seconds > 60.0) fail(SPMV_ERR_INVALID_ARG, "seconds must be in (0, 60]");
        check_vectors(h, x, y);
        const int32_t v = variant < 0 ? h->variant[f] : variant;
        if (v >= variant_count(f, h->dt)) fail(SPMV_ERR_INVALID_ARG, "variant %d out of range", v);
        if (!prepare_variant(h, f, v, (hipStream_t)stream))
            fail(SPMV_ERR_NOT_APPLICABLE, "variant %d does not apply to this matrix", v);
        measure_energy(h, f, v, x, y, seconds, 0.1, out, (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_energy_formats(spmv_handle h, int32_t count, const int32_t *formats,
                                           const int32_t *variants, const void *x, void *y,
                                           double seconds, spmv_energy_result *out, void *stream) {
    return guard([&] {
        if (!h || !formats || !out || count < 1 || count > 64)
            fail(SPMV_ERR_INVALID_ARG, "NULL argument or count outside [1, 64]");
        if (!(seconds > 0.0) || seconds > 60.0) fail(SPMV_ERR_INVALID_ARG, "seconds must be in (0, 60]");
        check_vectors(h, x, y);
        std::vector<spmv_format> fmts(count);
        std::vector<int32_t> vars(count);
        for (int32_t i = 0; i < count; ++i) {
            if (formats[i] < 0 || formats[i] >= SPMV_NUM_FORMATS)
                fail(SPMV_ERR_INVALID_ARG, "format %d", formats[i]);
            fmts[i] = (spmv_format)formats[i];
            check_runnable(h, fmts[i]);
            const int32_t v = (!variants || variants[i] < 0) ? h->variant[fmts[i]] : variants[i];
            if (v >= variant_count(fmts[i], h->dt)) fail(SPMV_ERR_INVALID_ARG, "variant %d out of range", v);
            if (!prepare_variant(h, fmts[i], v, (hipStream_t)stream))
                fail(SPMV_ERR_NOT_APPLICABLE, "variant %d of format %d does not apply", v, formats[i]);
            vars[i] = v;
        }
        measure_energy_sweep(h, count, fmts.data(), vars.data(), x, y, seconds, out,
                             (hipStream_t)stream);
    });
}

extern "C" spmv_status spmv_idle_power(double seconds, double *watts) {
    return guard([&] {
        if (!watts) fail(SPMV_ERR_INVALID_ARG, "NULL result");
        if (!(seconds > 0.0) || seconds > 60.0) fail(SPMV_ERR_INVALID_ARG, "seconds must be in (0, 60]");
        measure_idle_power(seconds, watts);
    });
}
