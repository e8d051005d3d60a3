// tiles.h - the chain tiles compiled into the library.
//
// A tile is (G lanes per chain, LPL labels per lane); a chain of K labels fits a tile
// with G*LPL >= K.  Every tile is instantiated in its own compilation unit (the build
// script reads this list), and the host dispatch tables below are generated from it.
#pragma once

#define DM_FOR_EACH_TILE(X) \
    X(4, 1)                 \
    X(4, 2)                 \
    X(8, 4)                 \
    X(16, 4)                \
    X(32, 3)                \
    X(32, 4)                \
    X(32, 6)                \
    X(64, 3)                \
    X(64, 4)
