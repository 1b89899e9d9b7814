// Controls of the CPU test backend of the SIP server (fake_backend.cpp).
// Test infrastructure: the backend runs the scheduler's steps with the
// oracle on the host.
#pragma once
#include <cstdint>

namespace fake {

// The server's clock: one tick (1 ms of server time) per SIP iteration run.
uint64_t ticks();
// Closes or opens the gate at the start of every step; with the gate closed
// the scheduler thread waits there (without the scheduler's lock), so that
// requests submitted meanwhile queue up together.  until_quit: the gate also
// opens once the server is shutting down.
void close_gate(bool until_quit = false);
void open_gate();
// Waits until the scheduler thread waits at the closed gate.
void wait_at_gate();
// The next n system (or request) allocations fail.
void fail_system_allocs(int n);
void fail_request_allocs(int n);
// The next step fails as a device failure would (SIP_EDEVICE).
void fail_next_step();
// Steps run, and whether the last one ran in the persistent mode (no
// arrival since the step before).
uint64_t steps();
uint64_t persistent_steps();
// Bytes held by live systems and requests (must return to 0 after destroy).
int64_t live_bytes();

}  // namespace fake
