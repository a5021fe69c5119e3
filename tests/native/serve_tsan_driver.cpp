// Host ThreadSanitizer run of the serving scheduler: the mock executor (host threads in
// place of streams, no device) under concurrent submitters, waiters with time-outs, a
// statistics poller and a failing request, with a memory budget small enough that
// admission binds.  Built together with the library's serving and handle sources; the
// device launch entry points are stubs here because the mock executor never reaches them.
// Exit status 0 and no sanitizer report is the pass condition.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <thread>
#include <vector>

#include "../../paper_2312_04830_amd/csrc/props_internal.hpp"

namespace props {
int launch_pr(const props_mech_s *, int, int, const props_in *, const props_out *, int64_t, uint8_t *,
              hipStream_t)
{
    return PROPS_EINVAL;
}
int launch_pr_strided(const props_mech_s *, int, int, const props_in *, const props_out *, int64_t, int64_t,
                      uint8_t *, hipStream_t)
{
    return PROPS_EINVAL;
}
int launch_pr_indirect(const props_mech_s *, int, int, const props_in *, const props_out *, int64_t, int64_t,
                       const int *, const int *, uint8_t *, uint8_t, hipStream_t)
{
    return PROPS_EINVAL;
}
int dnn_eval(props_dnn_s *, props_mech_s *, const props_in *, const props_out *, int64_t, int64_t, uint8_t *,
             int *, int *, hipStream_t)
{
    return PROPS_EINVAL;
}
int launch_diffusion(const props_mech_s *, int, const double *, const double *, const double *, double *,
                     int64_t, uint8_t *, hipStream_t)
{
    return PROPS_EINVAL;
}
}  // namespace props

namespace {

constexpr int NS = 8;

struct Req {
    int64_t n;
    int mode;
    std::vector<double> a, b, Y, out[10];
    std::vector<uint8_t> st;
};

void fill(Req &r, int64_t n, int mode, unsigned seed, bool poison)
{
    r.n = n;
    r.mode = mode;
    r.a.resize(n), r.b.resize(n), r.Y.assign((size_t)NS * n, 1.0 / NS), r.st.assign(n, 255);
    for (auto &o : r.out) o.assign(n, NAN);
    for (int64_t k = 0; k < n; k++) {
        r.a[k] = 1e6 + (double)((seed * 2654435761u + k) % 1000);
        r.b[k] = 100.0 + (double)(k % 977);
    }
    if (poison) r.a[0] = NAN;
}

props_request as_request(Req &r)
{
    props_request q{};
    q.mode = r.mode;
    q.route = PROPS_ROUTE_PR_MIXED;
    q.n = r.n;
    if (r.mode == PROPS_PTY) q.in.P = r.a.data(), q.in.T = r.b.data();
    else if (r.mode == PROPS_RHOEY) q.in.rho = r.a.data(), q.in.e = r.b.data();
    else q.in.h = r.a.data(), q.in.P = r.b.data();
    q.in.Y = r.Y.data();
    double **o[10] = {&q.out.T, &q.out.P, &q.out.Z, &q.out.rho, &q.out.h, &q.out.e, &q.out.cp, &q.out.c,
                      &q.out.mu, &q.out.lambda};
    for (int f = 0; f < 10; f++) *o[f] = r.out[f].data();
    q.status = r.st.data();
    q.memory = PROPS_MEM_HOST;
    return q;
}

}  // namespace

int main()
{
    props_serve_cfg cfg{};
    cfg.mem_budget = 6 * 2000 * 8 * 24;   // a few slots of 2000 cells: admission binds
    cfg.chunk_cells = 2000;
    cfg.streams = 3;
    cfg.executor = PROPS_EXEC_MOCK;
    cfg.mock_ns_per_cell = 20.0;
    cfg.mock_species = NS;
    props_server_t s = nullptr;
    if (serve_create(&cfg, nullptr, nullptr, &s) != PROPS_OK) {
        std::printf("serve_create failed: %s\n", props_last_error());
        return 1;
    }
    std::atomic<int> bad{0};
    std::atomic<bool> done{false};
    std::thread poller([&] {
        while (!done.load()) {
            props_serve_stats st;
            if (serve_stats(s, &st) != PROPS_OK) bad++;
            std::this_thread::yield();
        }
    });
    std::vector<std::thread> th;
    for (int t = 0; t < 6; t++) {
        th.emplace_back([&, t] {
            for (int i = 0; i < 12; i++) {
                Req r;
                const bool poison = (t == 2 && i == 5);
                fill(r, 1 + (int64_t)((t * 7919 + i * 104729) % 9000), (t + i) % 3, t * 100 + i, poison);
                props_request q = as_request(r);
                uint64_t ticket = 0;
                if (serve_submit(s, &q, &ticket) != PROPS_OK) {
                    bad++;
                    continue;
                }
                props_result res;
                int rc;
                while ((rc = serve_wait(s, ticket, 200, &res)) == PROPS_ETIMEDOUT) {
                }
                if (poison) {
                    if (res.rc == PROPS_OK) bad++;
                    continue;
                }
                if (rc != PROPS_OK || res.rc != PROPS_OK || res.n != r.n) {
                    bad++;
                    continue;
                }
                for (int64_t k = 0; k < r.n; k++)
                    if (r.out[0][k] != r.b[k] || r.out[1][k] != r.a[k] || r.out[9][k] != (double)k || r.st[k] != 0) {
                        bad++;
                        break;
                    }
            }
        });
    }
    for (auto &x : th) x.join();
    done = true;
    poller.join();
    props_serve_stats st;
    serve_stats(s, &st);
    serve_destroy(s);
    std::printf("completed %lld failed %lld bad %d\n", (long long)st.completed, (long long)st.failed, bad.load());
    return (bad.load() == 0 && st.failed == 1 && st.completed == 71) ? 0 : 1;
}
