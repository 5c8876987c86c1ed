// Prints the per-launch schedule of one work item, as the kernels decode it:
//   schedule_dump T K S [Sa]  ->  one line "phase n j count" per launch s = 0, 1, ...
// until the decoder reports idle (phases: 1 forward, 2 recompute, 3 adjoint);
// S forward-type and Sa (default S) adjoint steps per launch.
#include <cstdio>
#include <cstdlib>

#include "fwi_kernels.hpp"

int main(int argc, char** argv)
{
    if (argc != 4 && argc != 5) return 2;
    const int T = std::atoi(argv[1]), K = std::atoi(argv[2]), S = std::atoi(argv[3]);
    const int Sa = argc == 5 ? std::atoi(argv[4]) : S;
    const int J = (T + K - 1) / K;
    for (int s = 0;; ++s) {
        const fwi::Step st = fwi::decode(T, K, J, s, S, Sa);
        if (st.phase == fwi::kIdle) break;
        std::printf("%d %d %d %d\n", st.phase, st.n, st.j, st.count);
    }
    return 0;
}
