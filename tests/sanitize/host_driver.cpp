// Host-only calls of libdcp, for a build whose host code carries
// AddressSanitizer and UndefinedBehaviorSanitizer: planners, workspace
// sizes, the binomial schedule, the fusing compiler's front end and code
// generator (hipRTC), and argument errors of the device entry points
// (rejected before any device call; placeholder addresses are never
// dereferenced).  Test infrastructure only: built and run by
// tests/test_sanitize_host.py.
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <vector>
#include "dcp.h"

int main() {
    long calls = 0;
    size_t b = 0;
    int64_t shapes[][3] = {{0, 0, 0}, {1, 1, 1}, {2, 3, 4}, {8, 3, 2}, {64, 64, 64}, {70, 33, 21}, {512, 512, 512},
                           {1024, 1024, 512}, {1030, 17, 9}, {4096, 5, 6}, {65536, 8192, 4}, {1 << 24, 1, 1},
                           {-1, 4, 4}, {4, 4, (int64_t)1 << 40}};
    for (auto &s : shapes)
        for (int dt = 0; dt < 2; ++dt)
            for (int impl = 0; impl < 2; ++impl)
                for (int tb = 0; tb <= 4; ++tb)
                    for (int T : {0, 1, 4, 7, 100}) {
                        for (int op = 0; op < 4; ++op) {
                            dcp_workspace_bytes(op, dt, impl, s[0], s[1], s[2], T, 3, tb, 1, &b);
                            dcp_workspace_bytes(op, dt, impl, s[0], s[1], s[2], T, 1, tb, 0, &b);
                            calls += 2;
                        }
                        dcp_run_info info;
                        dcp_run_plan(dt, impl, s[0], s[1], s[2], T, tb, 1, &info);
                        dcp_revolve_workspace_bytes(dt, s[0], s[1], s[2], T, 4, 1, &b);
                        calls += 2;
                    }
    std::vector<int64_t> ops(5 * 100000);
    for (int64_t T : {1, 2, 3, 10, 100, 1000, 5000})
        for (int32_t slots : {1, 2, 3, 8, 30}) {
            int64_t nops = 0, fw = 0;
            dcp_revolve_schedule(T, slots, nullptr, 0, &nops, &fw);
            if (nops <= (int64_t)ops.size() / 5) dcp_revolve_schedule(T, slots, ops.data(), nops, &nops, &fw);
            dcp_revolve_schedule(T, slots, ops.data(), nops > 1 ? nops - 1 : 0, &nops, &fw);  // too small a cap
            calls += 3;
        }
    for (int dims = 1; dims <= 2; ++dims)
        for (int64_t n : {0, 1, 3, 1300, 24000, 46800})
            for (int tb = 0; tb <= 17; ++tb) {
                int64_t passes = 0;
                int32_t halo = 0;
                dcp_jacobi_plan(dims, n, dims == 2 ? n : 0, 1000, tb, &passes, &halo);
                dcp_jacobi_workspace_bytes(dims, n, dims == 2 ? n : 0, 1000, tb, &b);
                calls += 2;
            }
    const char *progs[] = {
        "dtype f64\ninput u f\nparam a\nt0 = shift u -1 0 0\nt1 = shift u 1 0 0\nt2 = add t0 t1\n"
        "t3 = mul a t2\nt4 = add u t3\nt5 = shift t4 0 1 0\nw = add t5 f\noutput w t4\n",
        "dtype f32\ninput u\nt0 = mul u u\nt1 = div t0 3.0\nt2 = neg t1\nt3 = shift t2 0 0 5\noutput t3\n",
        "dtype f64\ninput u\nt0 = shift u 2000000 0 0\noutput t0\n",   // offset out of range
        "dtype f64\ninput u\nt0 = add u v\noutput t0\n",                 // undefined name
        "dtype f16\ninput u\noutput u\n",                                 // bad dtype
        "", "dtype f64\n", "dtype f64\ninput u\nt0 = add u\noutput t0\n"};
    char err[256];
    for (const char *p : progs)
        for (int fuse = 0; fuse < 2; ++fuse) {
            dcp_fused *prog = nullptr;
            const int rc = dcp_fuse_build(p, fuse, &prog, err, sizeof err);
            if (rc == DCP_OK && prog) {
                int32_t info[6];
                dcp_fuse_info(prog, info, 6);
                size_t need = 0;
                dcp_fuse_source(prog, nullptr, 0, &need);
                std::vector<char> src(need + 1);
                dcp_fuse_source(prog, src.data(), src.size(), &need);
                dcp_fuse_source(prog, src.data(), 8, &need);  // truncated
                dcp_fuse_workspace_bytes(prog, 40, 30, 20, &b);
                dcp_fuse_workspace_bytes(prog, -1, 30, 20, &b);
                dcp_fuse_free(prog);
            }
            calls += 1;
        }
    // argument errors: placeholders never dereferenced
    void *P1 = (void *)0x10000000, *P2 = (void *)0x50000000, *P3 = (void *)0x90000000;
    dcp_coeffs c;
    std::memset(&c, 0, sizeof c);
    c.alpha = 1; c.beta = 0.1; c.gamma = 0.5; c.h = 1; c.dt = 0.1;
    double e[4], r[4];
    for (int dt = -1; dt < 3; ++dt) {
        dcp_step_fused(dt, P1, P2, P1, 8, 8, 8, &c, 0, nullptr, P3, 1 << 20, nullptr);    // u_out overlaps u
        dcp_step_unfused(dt, nullptr, P2, P3, 8, 8, 8, &c, 1, nullptr, P3, 1 << 20, nullptr);
        dcp_run(dt, 0, P1, P2, 8, 8, 8, &c, 1, -1, 3, e, r, nullptr, 0, P3, 1 << 20, nullptr);  // T < 0
        dcp_run(dt, 0, P1, P2, 8, 8, 8, nullptr, 1, 4, 3, e, r, nullptr, 0, P3, 1 << 20, nullptr);
        dcp_run(dt, 0, P1, P2, 8, 8, 8, &c, 1, 4, 9, e, r, nullptr, 0, P3, 1 << 20, nullptr);  // tblock 9
        dcp_adjoint_run(dt, P1, 0, P2, P3, 8, 8, 8, &c, 1, 4, 2, P1, e, nullptr, nullptr, P3, 16, nullptr);
        dcp_jacobi_1d(10, (double *)P1, (double *)P1, 100, 4, P3, 16, nullptr);                 // A aliases B
        dcp_jacobi_2d(10, (double *)P1, (double *)P2, -3, 5, 4, P3, 16, nullptr);
        dcp_revolve_forward(dt, P1, P2, 8, 8, 8, &c, 1, 10, 0, 2, P3, 16, nullptr);
        calls += 9;
    }
    for (int s = -12; s <= 1; ++s) (void)dcp_status_string(s);
    for (int dt = -1; dt < 3; ++dt) (void)dcp_max_tblock(dt);
    std::printf("host driver: %ld calls returned\n", calls);
    return 0;
}
