// Test-side interface of the host emulation (tests/hostemu/emu.cpp).
#pragma once

#include <stddef.h>

#include <string>

namespace emu {

[[noreturn]] void die(const std::string& msg);

// "Device" memory: a mapping with inaccessible pages around it, the buffer
// ending as close to the page after it as 256-byte alignment allows.
void* device_alloc(size_t bytes);
void device_free(void* p);

// Memory the kernels may touch, with the problem (owner >= 0) it belongs to;
// owner -1 marks memory shared by the problems of a batch (descriptors).
void register_region(const void* p, size_t bytes, int owner, const char* what);
void clear_regions();

extern long long g_launches, g_checked_passes, g_checked_tables;

}  // namespace emu
