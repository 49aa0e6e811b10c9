// Trace replay for measuring the server: submits requests at given arrival
// offsets from the calling thread and collects their completions, so that
// latency percentiles are measured with native timing rather than through
// an interpreter loop.
#include <chrono>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/trw.h"
#include "../../include/trw_probe.h"

extern "C" int trw_probe_serve_replay(void *server, uint32_t n, const void *requests, const uint64_t *arrival_ns,
                                      void *completions, uint32_t timeout_ms) {
    auto *s = static_cast<trw_server>(server);
    const auto *reqs = static_cast<const trw_request *>(requests);
    auto *out = static_cast<trw_completion *>(completions);
    if (!s || !reqs || !arrival_ns || !out) return 1;
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    std::unordered_map<uint64_t, uint32_t> index;
    index.reserve(n * 2);
    std::vector<trw_completion> buf(256);
    uint32_t submitted = 0, done = 0;
    while (done < n) {
        const uint64_t now = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - t0).count();
        if (now > (uint64_t)timeout_ms * 1000000ull) return 6;
        while (submitted < n && arrival_ns[submitted] <= now) {
            uint64_t id = 0;
            const trw_status st = trw_server_submit(s, &reqs[submitted], &id);
            if (st != TRW_OK) return 10 + (int)st;
            index[id] = submitted;
            ++submitted;
        }
        uint32_t got = 0;
        const uint64_t wait_ms = (submitted < n && arrival_ns[submitted] > now + 2000000ull) ? 1 : 0;
        const trw_status st = trw_server_poll(s, buf.data(), (uint32_t)buf.size(), &got, (uint32_t)wait_ms);
        if (st != TRW_OK && st != TRW_E_TIMEOUT) return 20 + (int)st;
        for (uint32_t i = 0; i < got; ++i) {
            auto it = index.find(buf[i].request_id);
            if (it == index.end()) continue;
            out[it->second] = buf[i];
            ++done;
        }
        if (!got && submitted < n) {
            const uint64_t t = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - t0).count();
            if (arrival_ns[submitted] > t + 50000) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    return 0;
}
