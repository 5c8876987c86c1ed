// Prints the per-launch schedule of one work item, as the kernels decode it:
//   schedule_dump T K S [Sa]  ->  one line "phase n j count" per launch s = 0, 1, ...
// until the decoder reports idle (phases: 1 forward, 2 recompute, 3 adjoint);
// S forward-type and Sa (default S) adjoint steps per launch.  Exits 3 if the
// kernels' decoder (precomputed constants, multiply-shift division) differs
// from the reference decoder at any launch index up to past the end.
//   schedule_dump div  ->  checks the multiply-shift quotient against n / d
// for divisors 1 .. 5000 and scattered larger ones, at every n below 4096,
// scattered n and the largest 31-bit values; exits 4 on a mismatch.
#include <cstdio>
#include <cstdlib>

#include "fwi_kernels.hpp"

static int check_div()
{
    unsigned long long x = 88172645463325252ull;   // xorshift64 state
    auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    auto one = [&](int d) {
        const fwi::Div v = fwi::make_div((uint32_t)d);
        auto ok = [&](int n) { return fwi::quo(n, v) == n / d; };
        for (int n = 0; n < 4096; ++n)
            if (!ok(n)) return false;
        for (int k = 0; k < 2000; ++k)
            if (!ok((int)(rnd() & 0x7fffffffu))) return false;
        for (int n = 0x7fffffff; n > 0x7fffffff - 4096; --n)
            if (!ok(n)) return false;
        for (int q = 1; q < 64; ++q) {                 // around multiples of d
            const long long m = (long long)d * (long long)(rnd() % (0x7fffffffu / (unsigned)d));
            for (long long n = m - 2; n <= m + 2; ++n)
                if (n >= 0 && n <= 0x7fffffff && !ok((int)n)) return false;
        }
        return true;
    };
    for (int d = 1; d <= 5000; ++d)
        if (!one(d)) { std::printf("mismatch d=%d\n", d); return 4; }
    for (int k = 0; k < 3000; ++k) {
        const int d = 1 + (int)(rnd() % 0x7ffffffeu);
        if (!one(d)) { std::printf("mismatch d=%d\n", d); return 4; }
    }
    for (int b = 1; b < 31; ++b)
        for (int e = -1; e <= 1; ++e)
            if (!one((1 << b) + e)) { std::printf("mismatch d=%d\n", (1 << b) + e); return 4; }
    return 0;
}

int main(int argc, char** argv)
{
    if (argc == 2 && argv[1][0] == 'd') return check_div();
    if (argc != 4 && argc != 5) return 2;
    const int T = std::atoi(argv[1]), K = std::atoi(argv[2]), S = std::atoi(argv[3]);
    const int Sa = argc == 5 ? std::atoi(argv[4]) : S;
    const int J = (T + K - 1) / K;
    const fwi::Sched sc = fwi::make_sched(T, K, J, S, Sa);
    for (int s = -2;; ++s) {
        const fwi::Step a = fwi::decode(T, K, J, s, S, Sa), b = fwi::decode_s(sc, s);
        if (a.phase != b.phase || (a.phase != fwi::kIdle && (a.n != b.n || a.j != b.j || a.count != b.count))) return 3;
        if (a.phase == fwi::kIdle && s > 0) {
            for (int k = 1; k < 50; ++k)
                if (fwi::decode_s(sc, s + k).phase != fwi::kIdle) return 3;
            break;
        }
    }
    for (int s = 0;; ++s) {
        const fwi::Step st = fwi::decode(T, K, J, s, S, Sa);
        if (st.phase == fwi::kIdle) break;
        std::printf("%d %d %d %d\n", st.phase, st.n, st.j, st.count);
    }
    return 0;
}
