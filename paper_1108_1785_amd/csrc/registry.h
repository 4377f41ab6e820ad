// Registry object shared by the host builder (registry.cpp) and the device
// entry points (kernels.hip).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "gnm.h"
#include "gnm_internal.h"

struct gnm_registry {
  uint32_t n_sites = 0;
  uint32_t root_bits = 0;
  uint32_t list_max = 0;
  uint32_t node_bits = 0;  // index bits of first-level wide nodes

  // host copy of the lookup structure (see gnm_internal.h)
  std::vector<uint32_t> root, wide, lines;
  // local set as disjoint inclusive ranges [lo, hi], sorted, and the
  // locality masks of every root cell (high words of the device root entries)
  std::vector<uint32_t> local_lo, local_hi;
  std::vector<uint32_t> root_local;

  gnm_registry_info info{};

  // device copy (one allocation)
  bool host_only = true;
  int device = -1;
  void *d_buf = nullptr;
  const uint64_t *d_root = nullptr;
  const uint32_t *d_wide = nullptr, *d_lines = nullptr;
  uint64_t d_bytes = 0;

  // launch-time LDS plan
  bool lines_in_lds = false;
  bool acc_in_lds = false;
  uint32_t lds_off_acc = 0, lds_off_lines = 0, lds_bytes = 0;
  uint32_t cache_slots = 0;  // LDS cache slots when the accumulator table does not fit

  uint64_t rows() const { return 2ull * (n_sites + 1ull) + 1ull; }
};

namespace gnm {
void set_last_error(const std::string &s);
int classify_prepare(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                     uint32_t n_windows, const gnm_params *p, gnm_acc *acc, uint8_t *flags);
}
