// Prints the search plan's threshold sample for one call shape, for the host
// tests of the planning logic: argv = m n d k graph precision; output = S r cap kk.
#include <cstdio>
#include <cstdlib>

#include "plan.hpp"

int main(int argc, char **argv) {
    if (argc != 7) return 2;
    knn_options_t o{};
    o.precision = std::atoi(argv[6]);
    const knn::Plan p = knn::make_plan(std::atoll(argv[1]), std::atoll(argv[2]), std::atoi(argv[3]),
                                       std::atoi(argv[4]), std::atoi(argv[5]) != 0, &o, 32768);
    std::printf("%d %d %d %d\n", p.S, p.r, p.cap, p.kk);
    return 0;
}
