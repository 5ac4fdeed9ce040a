// The multi-element tile shapes the library is built with (elements per
// workgroup E and register budget in waves per SIMD), per order.  One list
// drives both the kernel instantiations and the autotuner's search.
#pragma once

// X(P, E, BUDGET): E elements of order P per workgroup of ceil(E (P+2)^2 / 64)
// wavefronts.  E = 1 (one wavefront per element, budget 2) is the default
// gather-fold kernel and is not listed.
#define SIPDG_TILE_SHAPES(X) \
    X(1, 7, 2)               \
    X(1, 7, 4)               \
    X(2, 4, 2)               \
    X(2, 4, 4)               \
    X(3, 2, 2)               \
    X(3, 2, 3)               \
    X(3, 5, 2)               \
    X(4, 3, 2)               \
    X(4, 3, 3)               \
    X(4, 7, 2)               \
    X(5, 5, 2)
