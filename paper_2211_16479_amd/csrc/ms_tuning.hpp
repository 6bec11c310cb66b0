// Per-class shape choice of the segmented sort (written by the autotuner).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/msort.h"

namespace ms {

// Candidate index per small class for a (key type, value width) family;
// returns a pointer to SEG_MAX_CLASSES entries, or nullptr if unsupported.
int* seg_tuning_row(ms_key_type kt, size_t val_bytes);
// Bumped on every change of the table (captured graphs depend on it).
uint64_t seg_tuning_generation();
void seg_tuning_bump();

}  // namespace ms
