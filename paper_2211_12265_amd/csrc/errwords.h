// Device-detected conditions that a context reports at its next synchronising
// check (host code only; no HIP types).  The error words live in the context's
// statistics block on the device:
//   word 5  Sign tasks dropped at the per-task iteration limit (their signature
//           rows are left unwritten; unreachable in practice: a correct task
//           needs more than 16384 iterations with probability below 10^-1900)
//   word 8  a decreasing msg_off entry (the message was hashed as empty)
//   word 9  a key index outside its key table (the task used key row 0)
// Every condition that is set is named in the text; the code is that of the
// most severe one, and the caller clears all three words once reported.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/dil.h"

namespace dil {

constexpr int ERR_WORD_DROPPED = 5, ERR_WORD_MSG = 8, ERR_WORD_KEY = 9;

inline int report_error_words(uint32_t dropped, uint32_t msg_flag, uint32_t key_flag, char *text, size_t n) {
  if (!dropped && !msg_flag && !key_flag) {
    if (n) text[0] = 0;
    return DIL_OK;
  }
  size_t used = 0;
  auto add = [&](const char *s) {
    if (used < n) {
      int w = snprintf(text + used, n - used, "%s%s", used ? "; " : "", s);
      if (w > 0) used += (size_t)w;
    }
  };
  if (dropped) add("Sign tasks reached the iteration limit (their signature rows were not written)");
  if (key_flag) add("key index outside the key table (those tasks used key row 0)");
  if (msg_flag) add("decreasing msg_off entry (those messages were treated as empty)");
  if (dropped) return DIL_EHIP;
  if (key_flag) return DIL_EINVAL;
  return DIL_EMSG;
}

}  // namespace dil
