// Internal structures shared by the host symbolic phase, the numeric driver and
// the C ABI glue of libmf.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mf.h"

namespace mf {

constexpr uint32_t kSymMagic = 0x4d465359;  // "MFSY"
constexpr uint32_t kNumMagic = 0x4d464e55;  // "MFNU"
constexpr int kSpecVersion = 1;

void set_error(const std::string& msg);

// Result of the specified symbolic analysis plus everything the numeric phase
// derives from it once per pattern.
struct Symbolic {
    int64_t n = 0;
    int64_t nnz = 0;
    int32_t leaf_max = 64;
    std::vector<int64_t> rowptr;     // copy of the CSR pattern
    std::vector<int32_t> colind;
    std::vector<int32_t> root;

    // bit-exact outputs
    std::vector<int32_t> perm;          // new -> old
    std::vector<int32_t> front_ptr;     // nf+1
    std::vector<int32_t> front_parent;  // nf
    std::vector<int64_t> rows_ptr;      // nf+1
    std::vector<int32_t> rows;          // original variables
    std::vector<int32_t> var_etree;     // n

    // derived
    int32_t nf = 0;
    std::vector<int32_t> npiv, mnom;            // per front
    std::vector<int32_t> child_ptr, child_idx;  // children in increasing front order
    std::vector<int32_t> level;                 // height: leaves 0
    int32_t nlevels = 0;
    std::vector<int32_t> level_ptr, level_fronts;  // fronts grouped by level (ascending id)
    // inverse nominal maps: for child c, imap[imap_off[c] + i] = nominal CB index of
    // parent row i (0-based among c's non-pivot rows), or -1.  Length mnom[parent].
    std::vector<int64_t> imap_off;
    std::vector<int32_t> imap;
    // unique original entries, ordered by (level, front, colpos, rowpos)
    std::vector<int32_t> ue_front, ue_row, ue_col;  // nominal positions in the front
    std::vector<int64_t> ue_src_ptr;                // n_ue + 1
    std::vector<int32_t> ue_src;                    // CSR positions (duplicates summed)
    std::vector<int64_t> level_ue_ptr;              // nlevels + 1
    double nominal_flops = 0.0;
    double nominal_nnz_lu = 0.0;
    // systems of a batch (block-diagonal merge); one segment for a single system
    std::vector<int64_t> seg_row0{0}, seg_n{0}, seg_nnz0{0};
    // A light merge keeps the pattern and the unique-entry maps of its systems
    // where they are (their device copies) instead of concatenating them on the
    // host: rowptr, colind and the ue_* arrays stay empty, and each (system,
    // level) block of unique entries is described for a device-side copy.
    struct UeBlock {
        int32_t part;
        int32_t slot_delta;   // batch slot = the system's own slot + slot_delta
        int64_t u0, cnt;      // entries [u0, u0 + cnt) of the system's own maps
        int64_t dst_u;        // their first batch entry
        int64_t s0, scnt;     // their CSR sources [s0, s0 + scnt) in the system's map
        int64_t dst_s;        // first batch source
    };
    bool light = false;
    int64_t n_ue = 0, n_src = 0;
    std::vector<UeBlock> ue_blocks;
};

// Block-diagonal merge of several analyzed patterns (a batch): fronts, rows and
// maps are concatenated with offsets; each front keeps its height in its own
// tree, so a tree level of the batch is the union of the systems' levels.
void merge_symbolic(Symbolic& M, const std::vector<const Symbolic*>& parts, bool light = false);

// Runs the specified analysis; throws std::runtime_error / std::invalid_argument.
void analyze_pattern(Symbolic& S, int64_t n, const int64_t* rowptr, const int32_t* colind,
                     int32_t nroot, const int32_t* root_idx, int32_t leaf_max);

}  // namespace mf
