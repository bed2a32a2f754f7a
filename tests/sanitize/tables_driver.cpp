// Host-sanitizer driver of the library's host table code (test
// infrastructure): builds the Adam, scheduled, SGD-with-momentum and AdamW
// tables for several (max_steps, max_defer) and moves them to the last step,
// under -fsanitize=address,undefined.  Exit status 0 = no finding.
#include <cstdio>
#include <vector>

#include "gsdp_internal.h"

int main()
{
    int checked = 0;
    for (int T : {1, 2, 7, 64, 1000})
        for (int K : {0, 1, 15}) {
            std::vector<double> sched(T + 2);
            for (int t = 0; t < T + 2; ++t) sched[t] = 0.5 + 0.001 * t;
            for (int kind = 0; kind < 4; ++kind) {
                const int nclass = kind == 3 ? 2 : 0;
                const int64_t bytes = gsdp::lut_total_bytes(T, K, nclass);
                std::vector<double> img((bytes + 7) / 8);
                const float rates[2] = {1.6e-4f, 5e-3f};
                int rc = 0;
                if (kind == 0) rc = gsdp::build_lut_host(0.9, 0.999, T, K, nullptr, img.data(), bytes);
                if (kind == 1) rc = gsdp::build_lut_host(0.9, 0.999, T, K, sched.data(), img.data(), bytes);
                if (kind == 2) rc = gsdp::build_lut_sgdm_host(0.9, T, K, sched.data(), img.data(), bytes);
                if (kind == 3)
                    rc = gsdp::build_lut_adamw_host(0.9, 0.999, 0.01, rates, 2, T, K, sched.data(), img.data(), bytes);
                if (rc) return 2;
                if (gsdp::seek_lut_host(img.data(), bytes, T + 1) != 0) return 3;
                // out of range seeks are refused
                if (gsdp::seek_lut_host(img.data(), bytes, T) == 0 && T > 1) return 4;
                if (gsdp::seek_lut_host(img.data(), bytes, T + 2) == 0) return 5;
                // a buffer that is too small is refused
                if (gsdp::build_lut_host(0.9, 0.999, T, K, nullptr, img.data(), gsdp::lut_total_bytes(T, K, 0) - 8) == 0)
                    return 6;
                ++checked;
            }
        }
    std::printf("tables driver: %d table sets built and advanced\n", checked);
    return 0;
}
