// Independent Philox4x32-10 reference for the oracle pin: evaluates AMD
// rocRAND's host-callable philox4x32_10 engine on (counter, key) pairs read
// from stdin ("c0 c1 c2 c3 k0 k1" per line, hex) and prints the 4 output
// words.  Host code only; built with hipcc so the rocRAND header resolves.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// The engine's 10-round block function is a protected member; a derived
// type exposes it for arbitrary (counter, key) pairs.
struct Ref : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Ref ref;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = {c0, c1, c2, c3};
        uint2 k = {k0, k1};
        uint4 r = ref.block(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
