// Internal interface between the search host code and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wo {

// counter-generator streams
enum { RS_TOURNAMENT = 1, RS_ZONE_COIN = 2, RS_ZONE_PARTNER = 3, RS_INSERT_COIN = 4, RS_INSERT_TARGET = 5 };

struct CandArgs {
    const uint8_t *pz;        // population zones [P][64]
    const int32_t *pd;        // population distances [P]
    int P, C, K, tsize;
    uint32_t thr, gen;
    uint64_t seed;
    uint8_t *cand_zone;       // [K][64]
    int32_t *cand_parent;     // [K]
};

struct BreedArgs {
    const uint8_t *pz;
    const uint16_t *ps;       // population sequences [P][n]
    const int32_t *pd;
    int P, n, C, tsize, mode; // mode 0: plain generation, 1: screened survivors
    uint32_t thr, gen;
    uint64_t seed;
    const int32_t *best;      // mode 0: index of the best individual (the elite child 0)
    const int32_t *kept;      // mode 1: candidate id of each child
    const int32_t *cand_parent;
    const uint8_t *cand_zone;
    uint8_t *cz;              // children [n_children][64]
    uint16_t *cs;             // children [n_children][n]
};

struct ReplaceArgs {
    uint8_t *pz;
    uint16_t *ps;
    int32_t *pd;
    const uint8_t *cz;
    const uint16_t *cs;
    const int32_t *cd;
    const int32_t *worst;     // population slot of each child
    int n;
};

hipError_t launch_argmin(const int32_t *dist, int P, int32_t *out, hipStream_t s);
hipError_t launch_candidates(const CandArgs &a, hipStream_t s);
hipError_t launch_breed(const BreedArgs &a, int n_children, hipStream_t s);
hipError_t launch_replace(const ReplaceArgs &a, int keep, hipStream_t s);
uint32_t breed_lds_bytes(int n);

}  // namespace wo
