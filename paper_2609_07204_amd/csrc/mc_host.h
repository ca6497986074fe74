// Host-only part of the library: the thread-local error slot, option
// checks and the exact checks of host CSR inputs. Plain C++ with no HIP
// dependency, so the same file also builds for the CPU alone (sanitizer
// builds of the validation layer).
#pragma once
#include <stdint.h>

#include <string>

#include "mincut.h"

std::string& mc_error_slot();
// Sets the thread-local error message and returns code.
mc_status mc_fail(mc_status code, const std::string& msg);

// MC_OK, or MC_E_INVALID_ARG (with the message set) for an option value
// outside its documented range.
mc_status mc_options_check(const mc_options* o);

// Exact checks of one host CSR, in this order: pointers and n >= 2
// (MC_E_INVALID_ARG); row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing
// (MC_E_BAD_GRAPH); every target in [0, n) and weight >= 0
// (MC_E_BAD_GRAPH); total weight below 2^62 (MC_E_OVERFLOW); with
// `symmetric`, every folded pair (u, v, s) matched by (v, u, s)
// (MC_E_BAD_GRAPH). Reads the arrays only.
mc_status check_host_csr(const mc_csr* g, bool symmetric);
