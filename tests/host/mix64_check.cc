// Reads 64-bit integers (one per line) and prints pybind11's SplitMix64
// finalizer (pybind11::detail::mix64, an implementation independent of this
// project) of each: the oracle's Squares key derivation is checked against it.
#include <cstdio>
#include <pybind11/detail/internals.h>

int main() {
    unsigned long long x;
    while (std::scanf("%llu", &x) == 1)
        std::printf("%llu\n", (unsigned long long)pybind11::detail::mix64(x));
    return 0;
}
