// Error reporting of the C ABI: the status of the last failing call on the
// calling thread (with the call's name), and a stream synchronisation that
// turns an asynchronous device fault into a status.
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace {

thread_local int t_status = TSIM_OK;
thread_local char t_msg[256] = {0};
thread_local const char *t_detail = nullptr;  // reason given by the failing call, if any

}  // namespace

void note_detail(const char *why) { t_detail = why; }

int note_status(const char *fn, int st) {
  if (st != TSIM_OK) {
    t_status = st;
    if (t_detail)
      std::snprintf(t_msg, sizeof(t_msg), "%s: %s (%s)", fn, tsim_status_string(st), t_detail);
    else
      std::snprintf(t_msg, sizeof(t_msg), "%s: %s", fn, tsim_status_string(st));
  }
  t_detail = nullptr;
  return st;
}

extern "C" {

int tsim_last_error(char *msg, size_t msg_len) {
  const int st = t_status;
  if (msg && msg_len > 0) {
    std::strncpy(msg, st == TSIM_OK ? "" : t_msg, msg_len - 1);
    msg[msg_len - 1] = '\0';
  }
  t_status = TSIM_OK;
  t_msg[0] = '\0';
  return st;
}

int tsim_sync(tsim_stream stream) {
  const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e == hipSuccess) return TSIM_OK;
  t_status = TSIM_EDEVICE;
  std::snprintf(t_msg, sizeof(t_msg), "tsim_sync: %s (%s)", tsim_status_string(TSIM_EDEVICE),
                hipGetErrorString(e));
  return TSIM_EDEVICE;
}

}  // extern "C"
