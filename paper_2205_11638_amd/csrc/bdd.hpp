// bdd.hpp -- host compiler: one linear constraint row -> quasi-reduced ordered decision diagram.
//
// App. B: each subproblem X_j is a diagram with a root, a 1-terminal and a 0-terminal;
// for every variable of the row there is a set of nodes that every root-to-1 path
// visits exactly once (no level is skipped), each node has a lo arc (x = 0) and a hi
// arc (x = 1), and the root-to-1 paths are exactly the feasible assignments.
#pragma once
#include <cstdint>
#include <vector>

namespace dd {

enum { OK = 0, E_ARG = -1, E_INFEASIBLE = -2, E_FORCED = -3, E_PARAM = -4, E_HIP = -5, E_UNSUPPORTED = -6,
       E_OOM = -7, E_NONFINITE = -8, E_STATE = -9 };

// Largest level width representable by the 16-bit child codes (two codes are terminals).
constexpr int kMaxWidth = 65533;

struct RowBdd {
    int L = 0;                    // levels = variables of the row
    int max_width = 0;
    std::vector<int32_t> width;   // [L] nodes per level
    std::vector<uint32_t> arcs;   // level-major, per node lo | hi << 16 (codes: see dd_compile_row)
};

// Scratch buffers reused across rows on one thread.
struct CompileScratch {
    std::vector<std::vector<int64_t>> states;   // per level: live partial sums, ascending
    std::vector<uint8_t> has_true;              // per level: "every completion feasible" state present
    std::vector<int32_t> index;                 // dense partial-sum -> node id of the level below
    std::vector<uint64_t> table_keys;           // open-addressing unique table
    std::vector<int32_t> table_vals;
    std::vector<int64_t> merge;
};

// var must be strictly ascending (the caller sorts); a holds the matching coefficients.
int compile_row(int L, const int32_t *a, int sense, int64_t rhs, RowBdd &out, CompileScratch &scr);

}  // namespace dd
