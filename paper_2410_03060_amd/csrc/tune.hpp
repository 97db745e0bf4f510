// Process-wide table of the fastest block-sparse product variant per
// (unknowns per wire, wires, stored blocks, RHS count, precision), filled by
// chaff_autotune and consulted whenever a caller passes variant -1.  The table
// can be written to and read back from a JSON file (chaff_tune_save /
// chaff_tune_load), so a later process starts from earlier measurements.
#pragma once

#include <cstdint>
#include <string>

namespace chaff {

constexpr int TUNE_VARIANTS = 8;

struct TuneEntry {
    int32_t nb;                 // unknowns per wire
    int64_t n, nnzb, s;
    int32_t prec;
    int32_t best;
    double ms[TUNE_VARIANTS];   // measured time per variant (<= 0: not measured)
};

int tuned_variant(int nb, int64_t n, int64_t nnzb, int64_t s, int prec);   // -1 if none
void record_tuning(const TuneEntry& t);
std::string tune_json();
// Replaces or adds the entries of a JSON text written by tune_json; returns
// the number of entries read, or -1 if the text is not such a table.
int tune_merge_json(const std::string& text);

}  // namespace chaff
