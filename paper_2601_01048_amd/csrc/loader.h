// loader.h — host-side program analysis and lowering (see loader.cpp).
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ckc.h"

namespace ckc {

struct Loaded {
  std::vector<uint8_t> blob;            // dprog header + regions (dformat.h)
  ckc_prog_info info;
  std::vector<ckc_access_info> acc;
  uint32_t load_slots = 0;              // bit s: slot s is read by a LOAD
  std::string err;
};

// Validates, prunes (unless no_prune), classifies and lowers.  CKC_OK or
// CKC_E_IR (out->err).
int analyze_program(const void* ir, size_t ir_bytes, Loaded* out, bool no_prune = false);

}  // namespace ckc
